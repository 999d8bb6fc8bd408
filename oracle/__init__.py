"""Plain FP64 CPU oracle for the finite-volume Benamou-Brenier interior-point solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library may import, call or
link this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path: it builds its own meshes, its own operators and solves every Newton
system with a sparse direct factorisation.

Paper: Facca, Todeschi, Natale, Benzi, "Efficient preconditioners for solving
dynamical optimal transport via interior point methods" (arXiv 2209.00315).

Modules
-------
mesh       two-level meshes (Sec. 2.1) for the structured right-triangle grids,
           the Cartesian special case and the 3-D grid of cubes (Sec. 4.1).
operators  sparse discrete operators: M, M', Omega = M J, E, grad, W, R_E, R_T,
           coarse operators for the BB approximation (Sec. 2.1, Sec. 4.4.3).
ipm        residual F (Sec. 2.3), KKT Jacobian (Sec. 3), reduced saddle system
           (Sec. 3.1), interior-point continuation (Sec. 2.4), outputs.
bb         projected saddle operator (Sec. 4.4.2) and the exact-inner BB
           preconditioner application (Sec. 4.4.3); projected solve + recovery.
simple     the SIMPLE preconditioner (Sec. 4.3) on the projected system,
           exact inner solve.
gradient   derivative of the transport cost w.r.t. the marginals (envelope
           theorem + one adjoint saddle solve).

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
(closed forms, invariants, brute force on tiny meshes); see the module
docstrings for the pins.  None is "parity unpinned".
"""

from .mesh import Mesh, structured_mesh, cartesian_mesh, cartesian3d_mesh  # noqa: F401
from .operators import Operators  # noqa: F401
from .ipm import (  # noqa: F401
    Problem, residual, kkt_blocks, solve_ipm, kinetic_energy, dual_value,
    normalize_phi, IPMResult,
)
