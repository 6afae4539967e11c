"""Plain FP64 CPU oracle for the EM iteration of Synch-EM (2-D MRA in steerable coefficients).

TEST INFRASTRUCTURE ONLY. This package is the checker, not the product: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may import it. The HIP
library never calls it and shares no code with it; its only common input is the seeded generator
in ``workloads``.

Everything is numpy float64/complex128, written for a reader to check against the paper by eye:
the E-step weights (§II-B eq. (15)), the log-likelihood (§II-B eq. (13)), the coefficient update
with a Gaussian image prior (§II-B eq. (17), derived in App. C), the rotation-distribution update
with and without the KL prior (§II-B eq. (18); App. C eq. (42); Algorithm "Synch-EM"), the reduced
search window (§III-C), the stopping rule (Algorithm "Synch-EM"), the relative error up to rotation
(§II-B eq. (19)) and the histogram that learns the post-synchronisation prior (§III-B, eq. (22) and
Algorithm "learning rotation distribution").  Gradients of the marginal log-likelihood (not in the
paper) follow from eq. (13) by the Fisher identity.  ``sync`` holds the step before the path:
pairwise relative rotations, the projected power method and Synchronize and Match (§II-A,
§III-A), with the aligned observations.

Pins (tests marked ``not gpu``): brute force with explicitly rotated coefficients and with
explicitly rotated polar pixel images; rows of the posterior sum to one; monotone log-likelihood /
MAP objective; window = all L rotations reproduces plain EM; K = 1 gives w = rho; sigma^2 -> inf
gives w -> rho; the noiseless closed-form first step and exact recovery up to a global rotation;
the M-step maximises the Q function written out term by term; the rho-update maximises its
Lagrangian; finite differences of the log-likelihood; the histogram is the categorical MLE;
noiseless relative rotations are the exact differences, the power method recovers noiseless
rotations up to one global rotation, nearest neighbours by brute force.
"""
from .em import *          # noqa: F401,F403
from .pixel import *       # noqa: F401,F403
from .sync import *        # noqa: F401,F403
