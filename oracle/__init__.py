"""HWENO-U CPU oracle (FP64) -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct CPU implementation of the HWENO-U stage
operator of Fan, Qiu & Zhao (Section 2), used to check the GPU library.
Only `tests/`, `__graft_entry__.smoke()` and the CPU-baseline leg of
`bench.py` may import, call or link anything in this package.  It shares no
code with the GPU path.

Modules:
  derive  -- exact-rational derivation of the reconstruction operators
  driver  -- ctypes driver of the C stage operator + Runge-Kutta combination
  build   -- compiles hwenou_oracle.c with gcc

Parity status: every function here is pinned by the `-m "not gpu"` tests
(printed Appendix tables, printed smoothness-indicator forms, the printed
linear-scheme matrices A-D and moment modification, the stability bound,
polynomial exactness, conservation, weight special cases, symmetries and
convergence orders).  The scale-invariance demonstration with zeta = 1e-6
of Example 3.5 is "parity unpinned": with an absolute epsilon = 1e-10 the
weights collapse to the linear ones at that scale, and the paper only shows
figures for it.
"""
