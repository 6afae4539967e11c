"""Synch-EM for 2-D multi-reference alignment on AMD MI355X (gfx950).

The EM iteration (plain full search and the windowed, prior-weighted form) runs in the HIP library
``libsynchem.so`` built from ``csrc/``; this package is its thin Python binding:

* ``binding.EM``            one EM problem resident on the GPU (em_init / em_step / queries)
* ``binding.learn_prior``   histogram prior over the window from integer rotation errors
* ``binding.sync_match``    Synchronize and Match (relative rotations, power method, nearest
                            neighbours), ``binding.align`` the aligned observations
* ``autograd.marginal_loglik``  differentiable marginal log-likelihood with a hand-written adjoint
"""
from .binding import (EM, SynchemError, align, aligned_mean, error_bins,  # noqa: F401
                      global_rotation, learn_prior, load, nearest, ppm, relative_rotations,
                      sync_match)

__all__ = ["EM", "SynchemError", "align", "aligned_mean", "error_bins", "global_rotation",
           "learn_prior", "load", "nearest", "ppm", "relative_rotations", "sync_match"]
