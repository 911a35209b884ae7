"""MI355X-native geometric-multigrid Poisson solver.

The solver itself is the HIP library ``libgmg.so`` behind the C ABI declared
in ``include/gmg.h``; ``paper_2607_07687_amd.gmg`` is its thin ctypes binding
and ``paper_2607_07687_amd.problems`` builds seeded synthetic inputs.  Importing
the package loads nothing; the binding loads the library on first use and
raises if it is missing.
"""
