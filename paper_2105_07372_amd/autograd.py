"""torch.autograd.Function around the library's marginal log-likelihood and its hand-written
adjoint (em_loglik_fwd / em_loglik_bwd).  The gradients are the Fisher-identity gradients of the
likelihood of Section II-B eq. (13) with the rotation marginalised over the window:

  dLL/da      = (2/sigma^2) (S - N a)            (torch convention: dLL/dRe a + i dLL/dIm a)
  dLL/dsigma2 = -N D / sigma^2 + sum_ji w_ji ||R_i a - v_j||^2 / sigma^4
  dLL/deta    = W - N rho,   rho = softmax(eta)

The backward pass recomputes the posteriors from the forward's per-observation log-likelihood
checkpoint instead of keeping the N x W weights.
"""
from __future__ import annotations

import torch

from .binding import EM


class MarginalLogLik(torch.autograd.Function):
    @staticmethod
    def forward(ctx, em: EM, a: torch.Tensor, sigma2: torch.Tensor, eta=None):
        s2 = float(sigma2.detach().reshape(()).item())
        a_c = a.detach().contiguous()
        eta_c = None if eta is None else eta.detach().contiguous()
        ll = em.loglik_fwd(a_c, s2, eta_c)
        ctx.em = em
        ctx.gen = em._fwd_gen
        ctx.s2 = s2
        ctx.save_for_backward(a_c, sigma2, *( [] if eta_c is None else [eta_c]))
        ctx.has_eta = eta is not None
        return torch.tensor(ll, dtype=torch.float64, device=a.device)

    @staticmethod
    def backward(ctx, g):
        em: EM = ctx.em
        saved = ctx.saved_tensors
        a_c, sigma2 = saved[0], saved[1]
        eta_c = saved[2] if ctx.has_eta else None
        if em._fwd_gen != ctx.gen:          # another forward ran since: rebuild the checkpoint
            em.loglik_fwd(a_c, ctx.s2, eta_c)
        grad_a = torch.empty_like(a_c)
        grad_eta = torch.empty_like(eta_c) if eta_c is not None else None
        gs2 = em.loglik_bwd(float(g.detach().item()), grad_a, grad_eta)
        g_s2 = torch.full_like(sigma2, gs2)
        return None, grad_a, g_s2, grad_eta


def marginal_loglik(em: EM, a: torch.Tensor, sigma2: torch.Tensor, eta=None) -> torch.Tensor:
    """LL(a, sigma2, eta) as a differentiable scalar (float64, on a's device)."""
    return MarginalLogLik.apply(em, a, sigma2, eta)
