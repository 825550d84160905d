"""CPU oracle for the SPH neighbour loops -- TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may import
or run anything in this package.  The product path (paper_1807_01341_amd) never
does, and shares no code with it.

  oracle.sph    FP64 plain definitions of the SPH density loop with the
                smoothing-length solve, the ghost quantities, the hydro force
                loop, Eq. 1 time-steps and Eq. 2 time-bins (torch CPU float64,
                differentiable, so the same code gives the reference gradient).
  oracle.cells  ctypes front of cells.c: bit-exact plain definitions of the
                cell build, the 13-axis per-cell sorts, active masks, cell-pair
                lists and FP32 neighbour counts.

Parity status of every function is listed in its docstring; none is
"parity unpinned" except where stated there.
"""
