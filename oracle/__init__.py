"""Plain CPU FP64 oracle for the long-step Richardson(m) / NAG-Richardson(m) hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its
C-ABI and the Python binding in ``paper_2412_08076_amd``) imports, calls or
links anything from this package.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.

The oracle is written from the paper (Wang, Liu, Cui, Shu, "Momentum-Accelerated
Richardson(m) and Their Multilevel Neural Solvers", arXiv 2412.08076) in plain
NumPy, FP64, with no blocking, fusion or reordering beyond what the paper's
definitions state.  Every function cites the passage it follows.

Modules
-------
problem   -- anisotropic Q1 9-point stencil, 5-point Helmholtz stencil, y = A x
iterate   -- Richardson(m), MOM-, NAG-, NAGex-Richardson(m) (Table 1), residual history
weights   -- Chebyshev weights, semi-iteration, Leja order, amplification diagnostics
spectra   -- closed-form eigenvalues of the stencils (DST-I eigenvectors)
refine    -- FP64 iterative refinement around an inner solve
adjoint   -- reverse-mode derivative of the K-step NAG-Richardson(m) unroll
meta      -- the meta network (MLP) and its output head, forward and backward

Parity status: every function is pinned by a ``-m "not gpu"`` test except where
its docstring says "parity unpinned".
"""
