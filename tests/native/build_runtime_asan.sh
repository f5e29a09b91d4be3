#!/bin/bash
# Builds tests/native/runtime_asan_driver: the host runtime of oasm_gpu and
# the driver with AddressSanitizer and UndefinedBehaviorSanitizer on the host
# side only (device code is compiled as usual).  Test infrastructure.
set -euo pipefail
ROOT="$(cd "$(dirname "$0")/../.." && pwd)"
OUT="${1:-$ROOT/tests/native/runtime_asan_driver}"
TMP="$(mktemp -d)"
trap 'rm -rf "$TMP"' EXIT
HIPCC=/opt/rocm/bin/hipcc
FLAGS=(-O1 -g -std=c++17 --offload-arch=gfx950 -fPIC -Xclang -target-feature -Xclang -packed-fp32-ops
       -Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -Xarch_host -fno-omit-frame-pointer
       -I "$ROOT/include" -I "$ROOT/paper_1712_03560_amd/csrc")
SRC="$ROOT/paper_1712_03560_amd/csrc"
pids=()
for f in oasm_scan oasm_kernels oasm_levcalc oasm_runtime; do
    "$HIPCC" "${FLAGS[@]}" -c "$SRC/$f.hip" -o "$TMP/$f.o" 2> "$TMP/$f.err" & pids+=($!)
done
"$HIPCC" "${FLAGS[@]}" -c "$ROOT/tests/native/runtime_asan_driver.cpp" -o "$TMP/driver.o" 2> "$TMP/driver.err" & pids+=($!)
for p in "${pids[@]}"; do wait "$p"; done
"$HIPCC" --offload-arch=gfx950 -Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined \
    "$TMP"/*.o -L/opt/rocm/lib -lrocprofiler-sdk-roctx -Wl,-rpath,/opt/rocm/lib -o "$OUT"
echo "$OUT"
