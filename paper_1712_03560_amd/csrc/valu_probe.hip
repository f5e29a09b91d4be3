// VALU throughput probe for gfx950 (a measurement tool beside the library,
// run by the benchmark): int32 lane-ops per second of single instructions
// and of the scan's column recurrence, with registers only.
//
// Every kernel runs independent chains per thread (no memory in the loop,
// one store per thread at the end to keep the work live) on 16 blocks of 4
// wavefronts per CU.  Instructions are written with inline asm so that each
// test issues exactly the named instruction.  Output: one JSON object.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>

namespace {

#define ASM2(ins) asm volatile(ins " %0, %1, %2" : "=v"(x) : "v"(x), "v"(y))
#define ASM3(ins) asm volatile(ins " %0, %1, %2, %3" : "=v"(x) : "v"(x), "v"(y), "v"(z))

constexpr int kChains = 16;

template <int KIND>
__global__ void __launch_bounds__(256) k_op(uint32_t *out, int iters, uint32_t seed) {
    uint32_t a[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) a[j] = seed * (threadIdx.x + 1) + j * 0x9E3779B9u + blockIdx.x;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) {
            uint32_t x = a[j];
            const uint32_t y = a[(j + 1) % kChains], z = a[(j + 3) % kChains];
            if (KIND == 0) asm volatile("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(x) : "v"(x), "v"(y), "v"(z));
            if (KIND == 1) ASM2("v_add_u32");
            if (KIND == 2) ASM2("v_and_b32");
            if (KIND == 3) ASM2("v_xor_b32");
            if (KIND == 4) ASM2("v_or_b32");
            if (KIND == 5) ASM3("v_or3_b32");
            if (KIND == 6) asm volatile("v_lshlrev_b32 %0, 1, %1" : "=v"(x) : "v"(x));
            if (KIND == 7) asm volatile("v_lshl_or_b32 %0, %1, 1, %2" : "=v"(x) : "v"(x), "v"(y));
            if (KIND == 8) ASM2("v_bcnt_u32_b32");
            if (KIND == 9) ASM3("v_alignbit_b32");
            if (KIND == 10) asm volatile("v_add_co_u32 %0, vcc, %1, %2" : "=v"(x) : "v"(x), "v"(y) : "vcc");
            a[j] = x;
        }
    }
    uint32_t r = 0;
#pragma unroll
    for (int j = 0; j < kChains; ++j) r ^= a[j];
    out[blockIdx.x * blockDim.x + threadIdx.x] = r;
}

// The scan's one-word column step (ten instructions: and, add, three
// bitop3, two self-adds, bitop3, or, bitop3) on 4 independent columns per
// thread, with match masks taken from registers (the asm is not volatile,
// so the compiler may interleave the columns as it does in the scan).
__global__ void __launch_bounds__(256) k_column(uint32_t *out, int iters, uint32_t seed) {
    constexpr int C = 4;
    uint32_t pv[C], cm[C], eq[8];
#pragma unroll
    for (int j = 0; j < C; ++j) {
        pv[j] = ~0u;
        cm[j] = ~0u;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) eq[j] = (seed + j) * 0x9E3779B9u ^ (threadIdx.x * 0x85EBCA6Bu + blockIdx.x);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int s = 0; s < 8; ++s) {
#pragma unroll
            for (int j = 0; j < C; ++j) {
                const uint32_t e = eq[(s + j) & 7];
                uint32_t x, u, o, ph, mh, ph2, mh2, t, npv, ncm;
                asm("v_and_b32 %0, %1, %2" : "=v"(x) : "v"(e), "v"(pv[j]));
                asm("v_add_u32 %0, %1, %2" : "=v"(u) : "v"(x), "v"(pv[j]));
                asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0xfe" : "=v"(o) : "v"(u), "v"(pv[j]), "v"(e));
                asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x3f" : "=v"(ph) : "v"(cm[j]), "v"(o), "v"(o));
                asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0xd0" : "=v"(mh) : "v"(pv[j]), "v"(e), "v"(u));
                asm("v_add_u32 %0, %1, %1" : "=v"(ph2) : "v"(ph));
                asm("v_add_u32 %0, %1, %1" : "=v"(mh2) : "v"(mh));
                asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x04" : "=v"(t) : "v"(e), "v"(cm[j]), "v"(ph2));
                asm("v_or_b32 %0, %1, %2" : "=v"(npv) : "v"(mh2), "v"(t));
                asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x2f" : "=v"(ncm) : "v"(ph2), "v"(e), "v"(cm[j]));
                pv[j] = npv;
                cm[j] = ncm;
            }
        }
    }
    uint32_t r = 0;
#pragma unroll
    for (int j = 0; j < C; ++j) r ^= pv[j] ^ cm[j];
    out[blockIdx.x * blockDim.x + threadIdx.x] = r;
}

// Two one-word columns as the halves of one 64-bit pair: the carry add and
// both one-row shifts as v_lshl_add_u64 over the pair, the logic per half;
// the high half's bottom row is a wildcard row, which absorbs the carry out
// of the low half, and the bit the shifts move across the halves is masked
// (one v_and for the horizontal +1 deltas; the -1 deltas' mask is folded
// into the bitop3 that forms the new +1 vertical deltas).  Eighteen
// instructions per pair; 2 pairs per thread.
__global__ void __launch_bounds__(256) k_column_pair(uint32_t *out, int iters, uint32_t seed) {
    constexpr int C = 2;
    uint32_t pv[C][2], cm[C][2], eq[8];
#pragma unroll
    for (int j = 0; j < C; ++j)
        for (int h = 0; h < 2; ++h) {
            pv[j][h] = ~0u;
            cm[j][h] = ~0u;
        }
#pragma unroll
    for (int j = 0; j < 8; ++j) eq[j] = (seed + j) * 0x9E3779B9u ^ (threadIdx.x * 0x85EBCA6Bu + blockIdx.x);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int s = 0; s < 8; ++s) {
#pragma unroll
            for (int j = 0; j < C; ++j) {
                const uint32_t e[2] = {eq[(s + j) & 7], eq[(s + j + 3) & 7]};
                uint32_t x[2], o[2], ph[2], mh[2], t[2];
                asm("v_and_b32 %0, %1, %2" : "=v"(x[0]) : "v"(e[0]), "v"(pv[j][0]));
                asm("v_and_b32 %0, %1, %2" : "=v"(x[1]) : "v"(e[1]), "v"(pv[j][1]));
                uint64_t u;
                asm("v_lshl_add_u64 %0, %1, 0, %2" : "=v"(u)
                    : "v"(((uint64_t)x[1] << 32) | x[0]), "v"(((uint64_t)pv[j][1] << 32) | pv[j][0]));
                const uint32_t uu[2] = {(uint32_t)u, (uint32_t)(u >> 32)};
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0xfe" : "=v"(o[h]) : "v"(uu[h]), "v"(pv[j][h]), "v"(e[h]));
                    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x3f" : "=v"(ph[h]) : "v"(cm[j][h]), "v"(o[h]), "v"(o[h]));
                    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0xd0" : "=v"(mh[h]) : "v"(pv[j][h]), "v"(e[h]), "v"(uu[h]));
                }
                uint64_t ph2, mh2;
                asm("v_lshl_add_u64 %0, %1, 1, 0" : "=v"(ph2) : "v"(((uint64_t)ph[1] << 32) | ph[0]));
                asm("v_lshl_add_u64 %0, %1, 1, 0" : "=v"(mh2) : "v"(((uint64_t)mh[1] << 32) | mh[0]));
                uint32_t p2[2] = {(uint32_t)ph2, (uint32_t)(ph2 >> 32)};
                const uint32_t m2[2] = {(uint32_t)mh2, (uint32_t)(mh2 >> 32)};
                asm("v_and_b32 %0, -2, %1" : "=v"(p2[1]) : "v"(p2[1]));
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x04" : "=v"(t[h]) : "v"(e[h]), "v"(cm[j][h]), "v"(p2[h]));
                asm("v_or_b32 %0, %1, %2" : "=v"(pv[j][0]) : "v"(m2[0]), "v"(t[0]));
                // (m2 & -2) | t
                asm("v_bitop3_b32 %0, %1, -2, %2 bitop3:0xea" : "=v"(pv[j][1]) : "v"(m2[1]), "v"(t[1]));
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x2f" : "=v"(cm[j][h]) : "v"(p2[h]), "v"(e[h]), "v"(cm[j][h]));
            }
        }
    }
    uint32_t r = 0;
#pragma unroll
    for (int j = 0; j < C; ++j) r ^= pv[j][0] ^ cm[j][0] ^ pv[j][1] ^ cm[j][1];
    out[blockIdx.x * blockDim.x + threadIdx.x] = r;
}

double seconds(void (*launch)(uint32_t *, int, int), uint32_t *d, int blocks, int iters) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1;
    launch(d, blocks, 4);  // warm-up
    (void)hipEventRecord(e0, 0);
    launch(d, blocks, iters);
    (void)hipEventRecord(e1, 0);
    (void)hipEventSynchronize(e1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms * 1e-3;
}

template <int KIND>
void launch_op(uint32_t *d, int blocks, int iters) {
    hipLaunchKernelGGL(k_op<KIND>, dim3(blocks), dim3(256), 0, 0, d, iters, 1u);
}

void launch_column(uint32_t *d, int blocks, int iters) {
    hipLaunchKernelGGL(k_column, dim3(blocks), dim3(256), 0, 0, d, iters, 1u);
}

void launch_column_pair(uint32_t *d, int blocks, int iters) {
    hipLaunchKernelGGL(k_column_pair, dim3(blocks), dim3(256), 0, 0, d, iters, 1u);
}

// ------------------------------------------------------------------ HBM read calibration
// Read kernels of known size, for scaling the FETCH_SIZE counter
// (`valu_probe --read-calibration`): one reads with scalar loads, as the scan
// reads its text (each wavefront walks its own 64 KiB run one dword at a time
// through the scalar cache), the other with 16-byte vector loads, as a device
// copy does.  Each dispatch reads kReadBytes once and writes one dword per
// wavefront (16 KiB).
constexpr size_t kReadBytes = size_t(256) << 20;
constexpr uint32_t kRunWords = 16384;  // 64 KiB per wavefront
constexpr uint32_t kReadWaves = (uint32_t)(kReadBytes / (kRunWords * 4));

typedef __attribute__((address_space(4))) const uint32_t const_u32;

__global__ void __launch_bounds__(256) k_read_scalar(const uint32_t *p, uint32_t *out) {
    const uint32_t wave = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    const const_u32 *q = (const const_u32 *)(p + (size_t)wave * kRunWords);
    uint32_t acc = 0;
#pragma nounroll
    for (uint32_t i = 0; i < kRunWords; ++i) acc = acc * 31u + q[i];
    if ((threadIdx.x & 63) == 0) out[wave] = acc;
}

__global__ void __launch_bounds__(256) k_read_vector(const uint4 *p, uint32_t *out) {
    const uint32_t wave = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    const uint4 *q = p + (size_t)wave * (kRunWords / 4);
    uint32_t acc = 0;
    for (uint32_t i = lane; i < kRunWords / 4; i += 64) {
        const uint4 v = q[i];
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    for (int off = 32; off > 0; off >>= 1) acc ^= __shfl_xor(acc, off, 64);
    if (lane == 0) out[wave] = acc;
}

int read_calibration() {
    uint32_t *buf = nullptr, *out = nullptr;
    if (hipMalloc(&buf, kReadBytes) != hipSuccess || hipMalloc(&out, kReadWaves * 4) != hipSuccess) return 1;
    if (hipMemset(buf, 1, kReadBytes) != hipSuccess) return 1;
    double ms[2] = {0, 0};
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 1;
    for (int k = 0; k < 2; ++k) {
        for (int r = 0; r < 3; ++r) {
            (void)hipEventRecord(e0, 0);
            if (k == 0)
                hipLaunchKernelGGL(k_read_scalar, dim3(kReadWaves / 4), dim3(256), 0, 0, buf, out);
            else
                hipLaunchKernelGGL(k_read_vector, dim3(kReadWaves / 4), dim3(256), 0, 0,
                                   reinterpret_cast<const uint4 *>(buf), out);
            (void)hipEventRecord(e1, 0);
            if (hipEventSynchronize(e1) != hipSuccess) return 1;
            float t = 0;
            (void)hipEventElapsedTime(&t, e0, e1);
            ms[k] = r ? std::min(ms[k], (double)t) : (double)t;
        }
    }
    std::printf("{\"read_bytes_per_dispatch\": %zu, \"write_bytes_per_dispatch\": %u, \"dispatches_each\": 3, "
                "\"k_read_scalar_ms\": %.3f, \"k_read_vector_ms\": %.3f}\n",
                kReadBytes, kReadWaves * 4, ms[0], ms[1]);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(buf);
    (void)hipFree(out);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

}  // namespace

int main(int argc, char **argv) {
    if (argc > 1 && std::strcmp(argv[1], "--read-calibration") == 0) return read_calibration();
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) {
        std::fprintf(stderr, "no device\n");
        return 1;
    }
    const int blocks = cus * 16;
    uint32_t *d = nullptr;
    if (hipMalloc(&d, (size_t)blocks * 256 * sizeof(uint32_t)) != hipSuccess) return 1;
    struct Op {
        const char *name;
        void (*fn)(uint32_t *, int, int);
    };
    const Op ops[] = {{"v_bitop3_b32", launch_op<0>},  {"v_add_u32", launch_op<1>},      {"v_and_b32", launch_op<2>},
                      {"v_xor_b32", launch_op<3>},     {"v_or_b32", launch_op<4>},       {"v_or3_b32", launch_op<5>},
                      {"v_lshlrev_b32", launch_op<6>}, {"v_lshl_or_b32", launch_op<7>},  {"v_bcnt_u32_b32", launch_op<8>},
                      {"v_alignbit_b32", launch_op<9>}, {"v_add_co_u32", launch_op<10>}};
    const int iters = 8000;
    std::printf("{\"cus\": %d, \"blocks\": %d, \"unit\": \"T int32 lane-ops/s\", \"ops\": {", cus, blocks);
    bool first = true;
    for (const Op &op : ops) {
        const double s = seconds(op.fn, d, blocks, iters);
        const double rate = (double)blocks * 256 * iters * kChains / s / 1e12;
        std::printf("%s\"%s\": %.2f", first ? "" : ", ", op.name, rate);
        first = false;
    }
    const int citers = 2000;
    const double s = seconds(launch_column, d, blocks, citers);
    const double steps = (double)blocks * 256 * citers * 8 * 4;  // word-steps
    const double s2 = seconds(launch_column_pair, d, blocks, citers);
    std::printf("}, \"column_step\": {\"ops_per_word_step\": 10, \"word_steps_per_s\": %.4g, \"lane_ops\": %.2f}, "
                "\"column_step_pair64\": {\"instructions_per_two_word_steps\": 18, \"word_steps_per_s\": %.4g}}\n",
                steps / s, steps * 10 / s / 1e12, steps / s2);
    (void)hipFree(d);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}
