"""oasm_gpu: online approximate string matching (arXiv 1712.03560) on MI355X.

The matching path lives in the HIP library ``liboasm_gpu.so`` (sources under
``csrc/``, C ABI in ``include/oasm_gpu.h``); ``oasm`` is its ctypes binding and
``workloads`` draws seeded synthetic inputs.  Submodules are imported on
demand so that ``workloads`` can be used without the built library.
"""
__all__ = ["oasm", "workloads"]
