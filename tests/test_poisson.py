"""Multigrid transfer + Poisson harness (torch.fft, run here on the CPU),
pinned by closed forms: the potential of a plane-wave density, the cutoff
filtering between levels, and the energy identity and its gradient."""
from __future__ import annotations

import math

import numpy as np
import torch

from paper_2603_24881_amd.poisson import MultigridPoisson


def _grid(L, mesh):
    ax = [np.arange(n) * (L[d] / n) for d, n in enumerate(mesh)]
    return np.meshgrid(*ax, indexing="ij")


def _wave(L, mesh, m, fn):
    x, y, z = _grid(L, mesh)
    g = [2 * math.pi * m[d] / L[d] for d in range(3)]
    return fn(g[0] * x + g[1] * y + g[2] * z), sum(t * t for t in g)


def test_plane_wave_potential_and_energy():
    """rho = cos(G.r) gives v = 4 pi / |G|^2 cos(G.r) and E_J = pi Omega / |G|^2."""
    L, mesh = (7.0, 8.0, 9.0), (16, 18, 20)
    rho, g2 = _wave(L, mesh, (1, 2, -3), np.cos)
    p = MultigridPoisson(L, [mesh])
    v, e = p.solve([torch.as_tensor(rho)])
    np.testing.assert_allclose(v[0].numpy(), 4 * math.pi / g2 * rho, atol=1e-12, rtol=0)
    vol = L[0] * L[1] * L[2]
    assert abs(e - math.pi * vol / g2) < 1e-10 * e


def test_two_levels_filter_and_combine():
    """A density split over two levels: plane waves below both cutoffs reach
    both levels' potentials, one between the cutoffs only the fine level."""
    L = (10.0, 10.0, 10.0)
    fine, coarse = (24, 24, 24), (12, 12, 12)
    E = (40.0, 10.0)
    a0, ga = _wave(L, fine, (1, 0, 2), np.cos)
    c0, gc = _wave(L, fine, (5, 3, 4), np.cos)
    b1, gb = _wave(L, coarse, (0, 2, 1), np.sin)
    assert ga < E[1] and gb < E[1] and E[1] < gc < E[0]
    p = MultigridPoisson(L, [fine, coarse], E)
    v, e = p.solve([torch.as_tensor(a0 + c0), torch.as_tensor(b1)])
    a1, _ = _wave(L, coarse, (1, 0, 2), np.cos)
    b0, _ = _wave(L, fine, (0, 2, 1), np.sin)
    k = 4 * math.pi
    np.testing.assert_allclose(v[0].numpy(), k / ga * a0 + k / gb * b0 + k / gc * c0, atol=1e-12, rtol=0)
    np.testing.assert_allclose(v[1].numpy(), k / ga * a1 + k / gb * b1, atol=1e-12, rtol=0)
    vol = 1000.0
    ref = math.pi * vol * (1 / ga + 1 / gb + 1 / gc)
    assert abs(e - ref) < 1e-10 * ref


def test_energy_identity_and_gradient():
    """E_J = 1/2 sum_l w_l <v_l, rho_l> and dE_J/drho_l = w_l v_l on random
    level data."""
    L = (9.0, 10.0, 11.0)
    meshes = [(20, 22, 24), (12, 12, 15), (6, 8, 8)]
    E = (45.0, 15.0, 4.0)
    rng = np.random.default_rng(5)
    rho = [torch.tensor(rng.standard_normal(m), requires_grad=True) for m in meshes]
    p = MultigridPoisson(L, meshes, E)
    v, e = p.solve([r.detach() for r in rho])
    w = p.weights()
    half = 0.5 * sum(wl * float((vl * r.detach()).sum()) for wl, vl, r in zip(w, v, rho))
    assert abs(e - half) < 1e-11 * abs(e)
    et = p.energy(rho)
    assert abs(float(et) - e) < 1e-12 * abs(e)
    et.backward()
    for wl, vl, r in zip(w, v, rho):
        np.testing.assert_allclose(r.grad.numpy(), wl * vl.numpy(), atol=1e-12 * float(vl.abs().max()) * wl)
