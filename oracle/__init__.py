"""Plain FP64 CPU oracle -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import anything from this package.  The product library never
does, and the two share no code: only the seeded input generators
(``paper_2201_09729_amd.synth``) feed both sides.

Pinned by the CPU tests against closed forms (free-field momentum-space
operator and propagator, free Laplacian spectrum, constant abelian flux clover
term), invariants (gamma5-hermiticity, gauge covariance, projector algebra,
exact correlator splits), library routines (dense LU, dense Hermitian
eigensolver) and brute force (full dilution equals the exact trace).
The clover sign convention against the literature and absolute correlator
values have no pin in the paper: parity unpinned for those two points.
"""
from .oracle import *  # noqa: F401,F403
from .oracle import PARTS, GAMMA_NAMES  # noqa: F401
