"""Multigrid transfer and Poisson solve between eval_rho and eval_mat, through
the library's gpw_poisson (hipFFT and HIP kernels on the plan's device).

For level l with mesh N_l (weight w_l = Omega / N_l), plane waves G = 2 pi m / L
and mask_l(G) = {|m_d| < N_d / 2, |G|^2 < E_l}:

  rho~(G)  = sum_l mask_l(G) w_l FFT(rho_l)(G)
  v_l(r)   = (1 / Omega) sum_G mask_l(G) 4 pi rho~(G) / |G|^2 exp(i G.r)   (G != 0)
  E_J      = (1 / (2 Omega)) sum_{G != 0} 4 pi |rho~(G)|^2 / |G|^2

(Sec. II: the Hartree potential and the multigrid Fourier interpolation), so
E_J = 1/2 sum_l w_l <v_l, rho_l> and dE_J / d rho_l = w_l v_l.
"""
from __future__ import annotations

from . import _lib


class Poisson:
    """The transfer + Poisson step of one plan (``GPW.poisson()``)."""

    def __init__(self, gpw):
        self.g = gpw

    def weights(self):
        return list(self.g.weights)

    def solve(self, rho, out=None, stream=None):
        """(v_l per level, E_J as a float); synchronises the stream for E_J."""
        v, ej = self.solve_async(rho, out=out, stream=stream)
        return v, float(ej.item())

    def solve_async(self, rho, out=None, stream=None):
        """(v_l per level, E_J as a one-element device tensor), enqueued only."""
        import torch
        v = self.g.new_grids() if out is None else out
        ej = torch.empty(1, dtype=torch.float64, device=v[0].device)
        _lib.gpw_poisson(self.g.plan, [r.contiguous() for r in rho], v, ej, stream)
        return v, ej

    def hxc(self, rho, vxc=None, vxc_grad=None, out=None, stream=None):
        """(v_l per level, E_J device scalar) of the Hartree term plus a
        fine-grid XC potential vxc and GGA vector potential vxc_grad (three
        fine grids); either may be None."""
        import torch
        v = self.g.new_grids() if out is None else out
        ej = torch.empty(1, dtype=torch.float64, device=v[0].device)
        _lib.gpw_hxc_potential(self.g.plan, [r.contiguous() for r in rho], v, vxc=vxc, vxc_grad=vxc_grad, e_j=ej,
                               stream=stream)
        return v, ej

    def fine_density(self, rho, gradient=True, stream=None):
        """(rho, [d_x rho, d_y rho, d_z rho] or None) on the finest mesh."""
        import torch
        shape = tuple(self.g.meshes[0])
        dev = rho[0].device
        rf = torch.empty(shape, dtype=torch.float64, device=dev)
        grad = [torch.empty(shape, dtype=torch.float64, device=dev) for _ in range(3)] if gradient else None
        _lib.gpw_fine_density(self.g.plan, [r.contiguous() for r in rho], rho_fine=rf, grad=grad, stream=stream)
        return rf, grad

    def energy(self, rho):
        """E_J as a differentiable torch scalar: its gradient with respect to
        rho_l is w_l v_l."""
        return _HartreeEnergy.apply(self, *rho)


def _hartree_fn():
    import torch

    class HartreeEnergy(torch.autograd.Function):
        @staticmethod
        def forward(ctx, p, *rho):
            v, ej = p.solve_async([r.detach() for r in rho])
            ctx.save_for_backward(*v)
            ctx.w = p.weights()
            return ej[0]

        @staticmethod
        def backward(ctx, g):
            v = ctx.saved_tensors
            return (None, *[g * w * vl for w, vl in zip(ctx.w, v)])

    return HartreeEnergy


class _Lazy:
    fn = None

    @classmethod
    def apply(cls, *args):
        if cls.fn is None:
            cls.fn = _hartree_fn()
        return cls.fn.apply(*args)


_HartreeEnergy = _Lazy
