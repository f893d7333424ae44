"""Plain FP64 CPU oracle of 1-D ADER-DG and ADER-WENO-FV time stepping.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, tables or
constants with the HIP library; the only thing both sides consume is the
seeded synthetic input from ``paper_2409_12483_amd.workloads``, which holds
none of the method's arithmetic.

Source: I.S. Popov, "The effective use of BLAS interface for implementation
of finite-element ADER-DG and finite-volume ADER-WENO methods"
(arXiv 2409.12483).  Every function cites the section, equation, algorithm
or table it follows.  The paper is written for 3-D Cartesian meshes; here
every formula is specialised to one space dimension (the eta and zeta
directions are dropped, the multi-index p=(p0,p1,p2,p3) becomes
(p0,p1) = (time node, space node)).  ``dg2d`` keeps two space dimensions
(the zeta direction dropped) and ``dg3d`` all three, for the Euler gas.

Array conventions (AoS, variable index fastest, as in Sec. 1.1 "Using the
BLAS interface"):
    u[c, k, r]        DG nodal coefficients of cell c, space node k, variable r
    q[c, a, l, r]     space-time predictor coefficients: time node a, space node l
    v[c, r]           finite-volume cell averages

Functions whose result has no pin beyond oracle-vs-GPU parity say
"parity unpinned" in their docstring: the Rusanov/path-conservative
Riemann solver and the WENO constants (the paper defines neither).
"""

from . import basis, pde, predictor, dg, dg2d, dg3d, weno, fv, fv2d, fv3d, brute, pade, norms, limiter, riemann  # noqa: F401
