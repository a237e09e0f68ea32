"""Multigrid transfer and Poisson solve between eval_rho and eval_mat.

This is the reciprocal-space step that sits between the two kernels of the
Fock build (Sec. II, the multigrid Fourier interpolation and the Hartree
potential): the level densities are brought to one set of plane-wave
coefficients, the Poisson equation is solved there, and the potential is
handed back to every level.  It runs with ``torch.fft`` on whatever device
the grids live on and is not part of the timed hot path.

For level l with mesh N_l, points r_j = j h (h = L / N_l), the plane waves
G = 2 pi m / L (integer m, |m_d| < N_d / 2) and the mask |G|^2 < E_l (E_l the
level cutoff in Ry, |G|^2 in bohr^-2; a strict sphere, the same for both
directions so that the transfer is self-adjoint):

  rho~(G) = sum_l mask_l(G) (Omega / N_l) sum_j rho_l(r_j) exp(-i G r_j)
  v~(G)   = 4 pi rho~(G) / |G|^2   (G != 0; v~(0) = 0, neutralising background)
  v_l(r_j) = (1 / Omega) sum_G mask_l(G) v~(G) exp(i G r_j)
  E_J     = (1 / (2 Omega)) sum_{G != 0} 4 pi |rho~(G)|^2 / |G|^2

so that E_J = 1/2 sum_l w_l <v_l, rho_l> with w_l = Omega / N_l, and
dE_J / d rho_l(r_j) = w_l v_l(r_j).  A level without a cutoff (a mesh given
directly) keeps every non-Nyquist plane wave of its mesh.
"""
from __future__ import annotations

import math

import numpy as np


class MultigridPoisson:
    """Transfer + Poisson for one cell and one set of level meshes.

    cell: (3,) orthorhombic side lengths (bohr); meshes: per level (N0, N1, N2),
    finest first; cutoffs_ry: per level cutoff (Ry) or None for "all plane
    waves of the mesh"."""

    def __init__(self, cell, meshes, cutoffs_ry=None, device="cpu"):
        import torch
        self.L = np.asarray(cell, dtype=np.float64).reshape(3)
        self.meshes = [tuple(int(x) for x in m) for m in meshes]
        self.nlevels = len(self.meshes)
        if cutoffs_ry is not None and len(cutoffs_ry) == 0:
            cutoffs_ry = None
        if cutoffs_ry is None and self.nlevels > 1:
            raise ValueError("several levels need their cutoffs")
        self.cutoffs = None if cutoffs_ry is None else [float(e) for e in cutoffs_ry]
        self.volume = float(np.prod(self.L))
        self.device = torch.device(device)
        fine = self.meshes[0]
        for m in self.meshes[1:]:
            if any(a > b for a, b in zip(m, fine)):
                raise ValueError("level 0 must hold the finest mesh")
        self.fine = fine
        # |G|^2 on the fine coefficient grid
        g2 = np.zeros(fine)
        for d in range(3):
            m = np.fft.fftfreq(fine[d]) * fine[d]
            g = 2.0 * math.pi * m / self.L[d]
            shape = [1, 1, 1]
            shape[d] = fine[d]
            g2 = g2 + (g ** 2).reshape(shape)
        self.g2 = torch.as_tensor(g2, device=self.device)
        coul = np.zeros(fine)
        nz = g2 > 0
        coul[nz] = 4.0 * math.pi / g2[nz]
        self.coulomb = torch.as_tensor(coul, device=self.device)
        # per level: flat indices of its masked plane waves in its own grid and in the fine grid
        self.src, self.dst = [], []
        for l, mesh in enumerate(self.meshes):
            ms = [np.fft.fftfreq(n) * n for n in mesh]
            mx, my, mz = np.meshgrid(*ms, indexing="ij")
            ok = np.ones(mesh, dtype=bool)
            for d, md in enumerate((mx, my, mz)):
                ok &= np.abs(md) < mesh[d] / 2.0          # no Nyquist plane
            if self.cutoffs is not None:
                gg = sum((2.0 * math.pi * md / self.L[d]) ** 2 for d, md in enumerate((mx, my, mz)))
                ok &= gg < self.cutoffs[l]
            src = np.flatnonzero(ok.ravel())
            fx = np.mod(mx.ravel()[src], fine[0]).astype(np.int64)
            fy = np.mod(my.ravel()[src], fine[1]).astype(np.int64)
            fz = np.mod(mz.ravel()[src], fine[2]).astype(np.int64)
            dst = (fx * fine[1] + fy) * fine[2] + fz
            self.src.append(torch.as_tensor(src, device=self.device))
            self.dst.append(torch.as_tensor(dst, device=self.device))

    def weights(self):
        return [self.volume / float(np.prod(m)) for m in self.meshes]

    def coefficients(self, rho):
        """rho~ on the fine coefficient grid from the level densities."""
        import torch
        acc = torch.zeros(self.fine, dtype=torch.complex128, device=self.device).reshape(-1)
        for l, r in enumerate(rho):
            f = torch.fft.fftn(r.to(torch.float64)).reshape(-1) * (self.volume / float(np.prod(self.meshes[l])))
            acc = acc.index_add(0, self.dst[l], f[self.src[l]])
        return acc.reshape(self.fine)

    def solve(self, rho):
        """(v_l per level, E_J) from the level densities."""
        import torch
        rt = self.coefficients(rho)
        vt = (rt * self.coulomb).reshape(-1)
        e_j = float((rt.abs() ** 2 * self.coulomb).sum().item()) / (2.0 * self.volume)
        out = []
        for l, mesh in enumerate(self.meshes):
            buf = torch.zeros(int(np.prod(mesh)), dtype=torch.complex128, device=self.device)
            buf[self.src[l]] = vt[self.dst[l]]
            n = float(np.prod(mesh))
            v = torch.fft.ifftn(buf.reshape(mesh)).real * (n / self.volume)
            out.append(v.contiguous())
        return out, e_j

    def energy(self, rho):
        """E_J as a differentiable torch scalar (gradient w_l v_l per level)."""
        rt = self.coefficients(rho)
        return (rt.abs() ** 2 * self.coulomb).sum() / (2.0 * self.volume)
