"""torch.autograd wrappers: per-element gamma and beta draws with their
implicit-reparameterization backward kernels, and multivariate normal rows
with their backward to mu and L.

    z = sample_gamma(alpha, streams)     # element e draws from substream e
    z = sample_beta(a, b, streams)
    z.backward(g)  ->  alpha.grad = g * dz/dalpha  (a.grad, b.grad for beta)

The forward advances the substreams; the backward is stateless and uses the
saved binary32 draws.  Parameters must be contiguous float32 CUDA tensors.
"""
import torch

from . import rp_beta_elem, rp_beta_grad, rp_gamma_elem, rp_gamma_grad, rp_mvn, rp_mvn_backward


def _check_param(t, name):
    if t.dtype != torch.float32 or not t.is_cuda:
        raise TypeError(f"{name} must be a float32 CUDA tensor")
    return t.contiguous()


class GammaFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, alpha, streams):
        alpha = _check_param(alpha, "alpha")
        z = torch.empty_like(alpha)
        rp_gamma_elem(streams, alpha, z, alpha.numel())
        ctx.save_for_backward(z, alpha)
        return z

    @staticmethod
    def backward(ctx, gz):
        z, alpha = ctx.saved_tensors
        gz = gz.to(torch.float32).contiguous()
        ga = torch.empty_like(alpha)
        rp_gamma_grad(z, alpha, gz, ga, alpha.numel())
        return ga, None


class BetaFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a, b, streams):
        a = _check_param(a, "a")
        b = _check_param(b, "b")
        if a.shape != b.shape:
            raise ValueError("a and b must have the same shape")
        z = torch.empty_like(a)
        rp_beta_elem(streams, a, b, z, a.numel())
        ctx.save_for_backward(z, a, b)
        return z

    @staticmethod
    def backward(ctx, gz):
        z, a, b = ctx.saved_tensors
        gz = gz.to(torch.float32).contiguous()
        ga = torch.empty_like(a)
        gb = torch.empty_like(b)
        rp_beta_grad(z, a, b, gz, ga, gb, a.numel())
        return ga, gb, None


def sample_gamma(alpha, streams):
    return GammaFn.apply(alpha, streams)


def sample_beta(a, b, streams):
    return BetaFn.apply(a, b, streams)


class MvnFn(torch.autograd.Function):
    """X = mu + Z L^T for n rows (row i from substream i).  The forward keeps
    a device copy of the substream states it started from; the backward
    regenerates Z from that copy."""

    @staticmethod
    def forward(ctx, mu, L, streams, n):
        mu = _check_param(mu, "mu")
        L = _check_param(L, "L")
        d = mu.numel()
        if L.shape != (d, d):
            raise ValueError("L must be d x d")
        start = streams.duplicate()
        X = torch.empty((n, d), dtype=torch.float32, device=mu.device)
        rp_mvn(streams, mu, L, d, n, X)
        ctx.start = start
        ctx.dims = (d, n)
        return X

    @staticmethod
    def backward(ctx, G):
        d, n = ctx.dims
        G = G.to(torch.float32).contiguous()
        gmu = torch.empty(d, dtype=torch.float32, device=G.device)
        gL = torch.empty((d, d), dtype=torch.float32, device=G.device)
        rp_mvn_backward(ctx.start, G, d, n, gmu, gL)
        return gmu, gL, None, None


def sample_mvn(mu, L, streams, n):
    return MvnFn.apply(mu, L, streams, n)
