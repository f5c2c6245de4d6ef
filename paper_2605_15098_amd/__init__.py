"""svmi: a state-vector quantum simulator for one AMD MI355X (gfx950).

The hot path (gate application, the paper's state partitioning, readouts)
runs in the HIP library ``libsvmi.so`` behind the C ABI of include/sv.h;
``sv`` is its thin ctypes binding and ``workloads`` the seeded circuit
generators. Importing the package loads nothing; the first call into ``sv``
loads the library and raises if it is missing.
"""
__all__ = ["sv", "workloads"]
