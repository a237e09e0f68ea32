"""CPU oracle of the multigrid Fourier transfer and Poisson solve.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may use it; the library never does.

What it computes (Sec. II: the Hartree potential of Eqs. (vH), (vHG) and the
multigrid Fourier interpolation between levels), plainly, with full complex
FFTs of numpy (FP64) and one loop over levels:

  level l: mesh N_l, points r_j = j h_l (h_l = L / N_l), weight w_l = Omega / N_l,
           plane waves G = 2 pi m / L with integer m, |m_d| < N_{l,d} / 2 (no
           Nyquist plane), kept when |G|^2 < E_l (cutoff in Ry, |G|^2 in bohr^-2;
           every such plane wave when the level has no cutoff)
  rho~(G)  = sum_l mask_l(G) w_l sum_j rho_l(r_j) exp(-i G . r_j)
  v~(G)    = 4 pi rho~(G) / |G|^2 for G != 0, v~(0) = 0
  v_l(r_j) = (1 / Omega) sum_G mask_l(G) v~(G) exp(i G . r_j)
  E_J      = (1 / (2 Omega)) sum_{G != 0} 4 pi |rho~(G)|^2 / |G|^2

The coefficients of all levels live on the plane-wave set of the finest mesh
(level 0 holds the finest mesh); a level's masked plane wave m lands on the
fine-grid index m mod N_0.  The cell is given by its side lengths L
(orthorhombic) or its lattice vectors as rows (general cell: G = sum_d m_d b_d
with b_d = 2 pi (A^-1)[:, d]).
"""
from __future__ import annotations

import math

import numpy as np


def _freqs(n):
    """Integer frequencies m of an n-point FFT, in numpy's order: 0, 1, ..., then
    the negative half (integers, not fftfreq(n) * n, whose rounding would put a
    plane wave at the wrong fine-grid index)."""
    return np.concatenate([np.arange(0, (n + 1) // 2), np.arange(-(n // 2), 0)]).astype(np.int64)


def lattice(L):
    """Lattice vectors as rows: diag(L) for side lengths L, or L itself (3 x 3)."""
    L = np.asarray(L, dtype=np.float64)
    return np.diag(L.reshape(3)) if L.size == 3 else L.reshape(3, 3)


def gcart(L, mx, my, mz):
    """Cartesian components of G = sum_d m_d b_d, b_d = 2 pi (A^-1)[:, d] (A: the
    lattice vectors as rows, so that G . r = 2 pi m . u for r = u A)."""
    b = 2 * math.pi * np.linalg.inv(lattice(L))     # column d is b_d
    return [mx * b[c, 0] + my * b[c, 1] + mz * b[c, 2] for c in range(3)]


def volume(L):
    return float(abs(np.linalg.det(lattice(L))))


def level_mask(L, mesh, cutoff_ry):
    """Boolean mask over a level's FFT grid: no Nyquist plane, |G|^2 < E_l."""
    m = [_freqs(n) for n in mesh]
    mx, my, mz = np.meshgrid(*m, indexing="ij")
    ok = (np.abs(mx) < mesh[0] / 2.0) & (np.abs(my) < mesh[1] / 2.0) & (np.abs(mz) < mesh[2] / 2.0)
    if cutoff_ry is not None:
        g = gcart(L, mx, my, mz)
        ok &= g[0] ** 2 + g[1] ** 2 + g[2] ** 2 < cutoff_ry
    return ok, (mx, my, mz)


def poisson(L, meshes, cutoffs_ry, rho):
    """(v_l per level, E_J) from the level densities rho_l (C-ordered grids).
    L: side lengths (3,) or lattice vectors as rows (3 x 3); cutoffs_ry: per
    level cutoff in Ry, or None for every plane wave."""
    vol = volume(L)
    fine = tuple(int(x) for x in meshes[0])
    acc = np.zeros(fine, dtype=np.complex128)
    masks = []
    for l, mesh in enumerate(meshes):
        mesh = tuple(int(x) for x in mesh)
        ok, (mx, my, mz) = level_mask(L, mesh, None if cutoffs_ry is None else cutoffs_ry[l])
        w = vol / float(np.prod(mesh))
        f = np.fft.fftn(np.asarray(rho[l], dtype=np.float64).reshape(mesh)) * w
        ix = np.mod(mx[ok], fine[0])
        iy = np.mod(my[ok], fine[1])
        iz = np.mod(mz[ok], fine[2])
        np.add.at(acc, (ix, iy, iz), f[ok])
        masks.append((ok, ix, iy, iz))
    fx, fy, fz = np.meshgrid(*[_freqs(n) for n in fine], indexing="ij")
    g = gcart(L, fx, fy, fz)
    g2 = g[0] ** 2 + g[1] ** 2 + g[2] ** 2
    coul = np.zeros(fine)
    coul[g2 > 0] = 4 * math.pi / g2[g2 > 0]
    vt = acc * coul
    e_j = float(np.sum(np.abs(acc) ** 2 * coul)) / (2.0 * vol)
    out = []
    for l, mesh in enumerate(meshes):
        mesh = tuple(int(x) for x in mesh)
        ok, ix, iy, iz = masks[l]
        buf = np.zeros(mesh, dtype=np.complex128)
        buf[ok] = vt[ix, iy, iz]
        # (1 / Omega) sum_G c(G) e^{iGr} = (N_l / Omega) ifftn
        out.append(np.real(np.fft.ifftn(buf)) * (float(np.prod(mesh)) / vol))
    return out, e_j


def _fine_coefficients(L, meshes, cutoffs_ry, rho):
    """rho~ on the finest mesh's plane waves and the level masks / fine indices."""
    vol = volume(L)
    fine = tuple(int(x) for x in meshes[0])
    acc = np.zeros(fine, dtype=np.complex128)
    masks = []
    for l, mesh in enumerate(meshes):
        mesh = tuple(int(x) for x in mesh)
        ok, (mx, my, mz) = level_mask(L, mesh, None if cutoffs_ry is None else cutoffs_ry[l])
        w = vol / float(np.prod(mesh))
        ix, iy, iz = np.mod(mx[ok], fine[0]), np.mod(my[ok], fine[1]), np.mod(mz[ok], fine[2])
        if rho is not None:
            np.add.at(acc, (ix, iy, iz), np.fft.fftn(np.asarray(rho[l], dtype=np.float64).reshape(mesh))[ok] * w)
        masks.append((ok, ix, iy, iz))
    return acc, masks, L, vol, fine


def _gvectors(L, fine):
    """The Cartesian components of G on the fine FFT grid (full arrays)."""
    fx, fy, fz = np.meshgrid(*[_freqs(n) for n in fine], indexing="ij")
    return gcart(L, fx, fy, fz)


def fine_density(L, meshes, cutoffs_ry, rho):
    """The total density and its gradient on the finest mesh by Fourier
    interpolation (Sec. II: rho~ = sum of the masked level transforms; the GGA
    density gradient as the inverse transform of i G rho~):
      rho(r)     = (1 / Omega) sum_G rho~(G) exp(i G.r)
      d_d rho(r) = (1 / Omega) sum_G i G_d rho~(G) exp(i G.r)."""
    acc, _, L, vol, fine = _fine_coefficients(L, meshes, cutoffs_ry, rho)
    n0 = float(np.prod(fine))
    g = _gvectors(L, fine)
    rf = np.real(np.fft.ifftn(acc)) * (n0 / vol)
    grad = [np.real(np.fft.ifftn(1j * g[d] * acc)) * (n0 / vol) for d in range(3)]
    return rf, grad


def hxc_potential(L, meshes, cutoffs_ry, rho, vxc=None, vxc_grad=None):
    """Level potentials of the Hartree term plus an exchange-correlation
    potential given on the finest mesh (Sec. II, Eqs. (vH), (vHG)): with
    w_0 = Omega / N_0 and F the transform of a fine-grid function,
      v~(G) = 4 pi rho~(G) / |G|^2 + w_0 F(vxc)(G) - i G . w_0 F(vxc_grad)(G)
    (the last term is the GGA potential after integration by parts: minus the
    divergence of the vector potential, evaluated in Fourier space), and
      v_l(r) = (1 / Omega) sum_G mask_l(G) v~(G) exp(i G.r).
    Returns (v_l per level, E_J) with E_J from the Hartree term alone."""
    acc, masks, L, vol, fine = _fine_coefficients(L, meshes, cutoffs_ry, rho)
    ok0 = masks[0][0]
    n0 = float(np.prod(fine))
    w0 = vol / n0
    g = _gvectors(L, fine)
    g2 = g[0] ** 2 + g[1] ** 2 + g[2] ** 2
    coul = np.zeros(fine)
    coul[g2 > 0] = 4 * math.pi / g2[g2 > 0]
    vt = acc * coul
    e_j = float(np.sum(np.abs(acc) ** 2 * coul)) / (2.0 * vol)
    # the fine-grid potentials enter on level 0's plane waves (every level's mask
    # lies inside it)
    if vxc is not None:
        vt = vt + ok0 * w0 * np.fft.fftn(np.asarray(vxc, dtype=np.float64).reshape(fine))
    if vxc_grad is not None:
        for d in range(3):
            vt = vt - ok0 * 1j * g[d] * w0 * np.fft.fftn(
                np.asarray(vxc_grad[d], dtype=np.float64).reshape(fine))
    out = []
    for l, mesh in enumerate(meshes):
        mesh = tuple(int(x) for x in mesh)
        ok, ix, iy, iz = masks[l]
        buf = np.zeros(mesh, dtype=np.complex128)
        buf[ok] = vt[ix, iy, iz]
        out.append(np.real(np.fft.ifftn(buf)) * (float(np.prod(mesh)) / vol))
    return out, e_j
