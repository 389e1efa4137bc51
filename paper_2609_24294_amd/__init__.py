"""zfpx: fixed-rate ZFP coding of spectral-transform transpose buffers on MI355X.

The compute path lives in the HIP library ``libzfpx.so`` built from ``csrc/``;
``zfpx`` is its thin ctypes binding, ``workloads`` the seeded input
generator and ``metrics`` the host-side error and size reporting.  Nothing is
imported eagerly, so the input generator can be used without the library.
"""
__all__ = ["zfpx", "workloads", "metrics"]
