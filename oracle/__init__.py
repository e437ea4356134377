"""FP64 CPU oracle for the moving-PML sweeping preconditioner (2D).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this package.
The product path (the HIP library and its Python binding) never calls it and
shares no code with it; the only common input is the ``workloads`` module,
which draws seeded velocity fields and sources and holds none of the method's
arithmetic.

Modules
-------
``helmholtz``  PML profiles (eq. sigma), the symmetric stretched operator and its
               5-point discretisation (eq. helmd), the shifted operator A_alpha
               (eq. helmalpha).  scipy.sparse, complex128.
``sweep``      Moving-PML subproblems H_m (Section 2.2), their banded LU in the
               x2-first ordering via LAPACK zgbtrf/zgbtrs, the approximate
               sweeping factorisation and its application (Algorithms 3 and 4,
               two-front variant at the end of Section 2.3), and the exact-mode
               subproblems used as a pin.
``exact``      The exact dense sweeping factorisation (Algorithms 1 and 2).
``krylov``     Right-preconditioned flexible GMRES(k) and left-preconditioned
               GMRES (the paper's formulation M A u = M f).

Pins (all in ``tests/test_oracle_*.py``): closed-form eigenpairs of the
5-point Laplacian, exact complex symmetry, the exact-mode identity
M_alpha = A_alpha^{-1}, Algorithms 1+2 against a sparse direct solve,
reciprocity, second-order convergence to the Hankel Green's function, and
convergence of the moving-PML T~_m to the exact Schur inverse as the layer
widens.  Conventions the paper leaves open are fixed in ``helmholtz.Params``.
"""
from .helmholtz import Params, assemble, strip_operator, sigma_low, sigma_phys, stretch  # noqa: F401
from .sweep import SweepFactor, factor, apply_sweep, subproblem_specs  # noqa: F401
from .krylov import fgmres, gmres_left  # noqa: F401
