"""MI355X-native hot path of the Free-Energy Machine (arXiv 2412.09285).

* ``paper_2412_09285_amd.fem`` -- the Python binding of the HIP library
  ``libfem.so`` (C ABI in ``include/fem.h``).
* ``paper_2412_09285_amd.workloads`` -- seeded synthetic inputs.
* ``paper_2412_09285_amd.build`` -- compiles the HIP sources for gfx950.

Importing the package loads nothing; ``fem.lib()`` loads the library and
raises if it is missing.
"""
__all__ = ["fem", "workloads", "build"]
