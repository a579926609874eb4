"""EVIS event-generation path on AMD Instinct MI355X (gfx950).

libevis.so (HIP kernels + C ABI, declared in include/evis.h) does the work;
``evis`` is its ctypes binding; ``scenes`` makes seeded synthetic inputs.
"""
__all__ = ["evis", "scenes"]
