"""Plain FP64 CPU oracle of the deferred-compression hierarchical solver.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct
definition that the HIP path is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it; the product path (``paper_1811_11248_amd``) never does, and the two
share no code (only the seeded input generators in ``synth`` serve both).

Contents, each following the paper (Chen, Cambier, Boman, Rajamanickam,
Tuminaro, Darve, "A Robust Hierarchical Solver for Ill-conditioned Systems
with Applications to Ice Sheet Modeling"):

* ``tree``     -- extruded (horizontal-only) recursive bisection cluster tree
                  (section "Extruded Partitioning for Ice Sheets").
* ``cpqr``     -- column-pivoted Householder QR used as the rank-revealing
                  compression (Eq. offdiag_new).
* ``hsolver``  -- one scaled low-rank elimination (operators S, E, G, P of
                  section "Scaled Low-rank Elimination"), the factorization
                  Algorithm 1 and the solve Algorithm 2.
* ``pcg``      -- preconditioned conjugate gradients using the factor.
* ``learned``  -- learned-rank form: Philox4x32-10 sketch, level-start
                  features, the rank MLP (forward and backpropagation in
                  fp64) and the (features, rank) training pairs.

Parity status: every function is pinned by a ``-m "not gpu"`` test except
the compressed factor as a whole at tol > 0, whose values the paper does not
print ("parity unpinned" beyond the invariants the tests check: exactness at
tol = 0, the no-fill strip, Proposition 2 identities and the Corollary).
"""
from .tree import (ClusterTree, build_tree, build_tree_graph, level0_graph, coarsen_square,  # noqa: F401
                   d2_colouring)
from .cpqr import cpqr, householder_nonneg, apply_qt, apply_q  # noqa: F401
from .hsolver import (  # noqa: F401
    NotSPDError,
    scaled_lowrank_elimination,
    factor,
    solve,
    Factor,
)
from .pcg import pcg  # noqa: F401
from . import learned  # noqa: F401
