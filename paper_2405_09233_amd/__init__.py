"""MI355X-native tensor Krylov solvers for A*X - X*B = C (T-product).

The solvers live in the C-ABI library ``libtsylv.so`` built from ``csrc/``;
:mod:`paper_2405_09233_amd.tsylv` is its thin ctypes binding.  Importing the
package does not load the library; the binding loads it on first use and
raises if it is missing.
"""
