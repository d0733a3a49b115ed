"""Plain, slow FP64 CPU oracle of the p-multigrid spectral-element Laplace solve.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code with the
library (``paper_2009_00705_amd``): every step is written here again, in
NumPy/SciPy, from the paper's definitions:

* ``refelem``  -- 1D rules, triangle nodes, orthonormal basis, cubature and the
                  reference matrices of the prism (Sec. 3.1).
* ``mesh``     -- numbering of the nodal space V^p, gather maps, colouring,
                  curvilinear node placement (Sec. 3.1, Sec. 6.2).
* ``operator`` -- isoparametric geometry, matrix-free and assembled stiffness
                  operator (Sec. 3.1, eq. laplaceproblemdiscrete).
* ``mg``       -- p-multigrid hierarchy, nested transfers (Sec. 5.1, eq. rest),
                  damped-Jacobi smoother (eq. sec_form), coarse solve and the
                  V-cycle (Alg. 1).
* ``krylov``   -- PCG (Alg. 3), PDC (Alg. 2), flexible PCG and stand-alone MG.
* ``mlp``      -- the small network of the learned warm start: forward,
                  manual backward and Adam in FP64.

Functions whose result is pinned only by the solver itself say so in their
docstring ("parity unpinned").
"""
