"""CPU oracle for edge-matrix ("auxiliary topology") AMG preconditioned CG.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 NumPy/SciPy implementation
of the method of Kogler & Schoeberl, "Auxiliary topology AMG" (arXiv 2011.13325).  It is the
reference the GPU library is compared against.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it; the library never does, and it
shares no code with the library (only the seeded input generator ``gen`` serves both).

Modules, each following the passage of the paper it cites:

* ``dense``     small dense primitives: Skew, Q maps (eq. qij_epseps; Def. def:deng remark),
                pseudo-inverse, harmonic mean (Lemma thm:mu2), generalized max eigenvalue.
* ``auxtop``    edge / vertex weight matrices: finest level (Thm thm:deng_elast and the scalar
                M-matrix splitting of section "deng"), coarse level (Thm thm:cemats), the
                auxiliary matrix (Def. def:deng, eq. auxa).
* ``criteria``  coarsening measures mu_D, mu_s, mu_b, mu_g (Thm thm:mu1, Lemma thm:mu2,
                Def. def:muc).
* ``coarsen``   successive matching (Algorithm alg:pwagg).
* ``prolong``   tentative and auxiliary smoothed prolongation (Defs. def:pwp, def:pwp_el,
                def:aux_sp).
* ``hierarchy`` Galerkin coarse operators, pseudo-inverse smoother diagonals, coarsest level
                regularization (section "sing2"), coloring.
* ``solve``     V-cycle (Algorithm alg:tg applied recursively) and preconditioned CG.

Parity pins: every function here is checked by ``tests/test_oracle_*.py`` against closed forms,
identities and special cases fixed by the paper and by mathematics.  The successive matching
output and the free parameters (c^ij, omega, sigma, caps, F^i rule) have no closed form:
parity unpinned as values; only their invariants are pinned.
"""
from .dense import (  # noqa: F401
    skew, qmat, q_transport, q_half, pinv_tau, harmonic, genmax, sym,
)
from .auxtop import (  # noqa: F401
    AuxLevel, finest_aux, coarse_aux, dhat_all, assemble_aux_dense,
)
from .criteria import mu_D, mu_s, mu_b, mu_g  # noqa: F401
from .coarsen import cuthill_mckee, successive_matching  # noqa: F401
from .prolong import BCSR, tentative_prolongation, smoothed_prolongation  # noqa: F401
from .hierarchy import SetupParams, Hierarchy, setup  # noqa: F401
from .solve import vcycle, pcg  # noqa: F401
