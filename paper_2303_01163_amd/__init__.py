"""MI355X (gfx950) implementation of the Anisotropic Submeshes Domain Splitting Method (ASDSM).

The method runs in ``libasdsm.so`` (HIP kernels behind the C ABI of ``include/asdsm.h``);
``paper_2303_01163_amd.asdsm`` is its ctypes binding and ``paper_2303_01163_amd.workloads`` builds
seeded manufactured-solution problems.  Importing the package loads nothing; the library is loaded
on first use.
"""

__all__ = ["asdsm", "workloads", "build"]
__version__ = "0.1.0"
