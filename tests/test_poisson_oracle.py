"""Pins of the Poisson / multigrid-transfer oracle (oracle/poisson.py) by closed
forms: the potential and energy of a plane-wave density, the cutoff filter
between two levels, the Nyquist and cutoff exclusions, and the energy
identity with its gradient (central differences)."""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import poisson as op


def _grid(L, mesh):
    ax = [np.arange(n) * (L[d] / n) for d, n in enumerate(mesh)]
    return np.meshgrid(*ax, indexing="ij")


def _wave(L, mesh, m, fn):
    x, y, z = _grid(L, mesh)
    g = [2 * math.pi * m[d] / L[d] for d in range(3)]
    return fn(g[0] * x + g[1] * y + g[2] * z), sum(t * t for t in g)


def test_plane_wave_potential_and_energy():
    """rho = cos(G.r): v = 4 pi / |G|^2 cos(G.r), E_J = pi Omega / |G|^2."""
    L, mesh = (7.0, 8.0, 9.0), (16, 18, 20)
    rho, g2 = _wave(L, mesh, (1, 2, -3), np.cos)
    v, e = op.poisson(L, [mesh], None, [rho])
    np.testing.assert_allclose(v[0], 4 * math.pi / g2 * rho, atol=1e-12, rtol=0)
    vol = L[0] * L[1] * L[2]
    assert abs(e - math.pi * vol / g2) < 1e-10 * e


def test_constant_density_is_neutralised():
    """The G = 0 term is dropped (neutralising background): a constant density
    has zero potential and energy."""
    L, mesh = (6.0, 7.0, 8.0), (10, 12, 14)
    v, e = op.poisson(L, [mesh], None, [np.full(mesh, 3.0)])
    assert np.abs(v[0]).max() < 1e-12 and abs(e) < 1e-20


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
    v, e = op.poisson(L, [fine, coarse], E, [a0 + c0, b1])
    a1, _ = _wave(L, coarse, (1, 0, 2), np.cos)
    b0, _ = _wave(L, fine, (0, 2, 1), np.sin)
    k = 4 * math.pi
    np.testing.assert_allclose(v[0], k / ga * a0 + k / gb * b0 + k / gc * c0, atol=1e-12, rtol=0)
    np.testing.assert_allclose(v[1], k / ga * a1 + k / gb * b1, atol=1e-12, rtol=0)
    ref = math.pi * 1000.0 * (1 / ga + 1 / gb + 1 / gc)
    assert abs(e - ref) < 1e-10 * ref


def test_waves_beyond_the_cutoff_or_on_the_nyquist_plane_are_dropped():
    L = (8.0, 8.0, 8.0)
    mesh = (16, 16, 16)
    hi, g_hi = _wave(L, mesh, (4, 3, 0), np.cos)     # |G|^2 above the cutoff
    nyq, _ = _wave(L, mesh, (8, 0, 0), np.cos)       # the Nyquist plane of axis 0
    assert g_hi > 12.0
    v, e = op.poisson(L, [mesh], [12.0], [hi + nyq])
    assert np.abs(v[0]).max() < 1e-12 and abs(e) < 1e-18


def test_energy_identity_and_gradient():
    """E_J = 1/2 sum_l w_l <v_l, rho_l>; dE_J/drho_l(r_j) = w_l v_l(r_j) by
    central differences on a few grid values."""
    L = (9.0, 10.0, 11.0)
    meshes = [(20, 22, 24), (12, 12, 15), (6, 8, 8)]
    E = (45.0, 15.0, 4.0)
    rng = np.random.default_rng(5)
    rho = [rng.standard_normal(m) for m in meshes]
    v, e = op.poisson(L, meshes, E, rho)
    vol = L[0] * L[1] * L[2]
    w = [vol / float(np.prod(m)) for m in meshes]
    half = 0.5 * sum(wl * float(np.vdot(vl, r)) for wl, vl, r in zip(w, v, rho))
    assert abs(e - half) < 1e-11 * abs(e)
    h = 1e-3
    for l, idx in ((0, (3, 4, 5)), (1, (7, 0, 2)), (2, (5, 7, 1))):
        rp = [r.copy() for r in rho]
        rm = [r.copy() for r in rho]
        rp[l][idx] += h
        rm[l][idx] -= h
        fd = (op.poisson(L, meshes, E, rp)[1] - op.poisson(L, meshes, E, rm)[1]) / (2 * h)
        assert abs(fd - w[l] * v[l][idx]) < 1e-7 * abs(w[l] * v[l][idx]) + 1e-9


def test_nyquist_plane_is_dropped_without_a_cutoff():
    """A level with no cutoff keeps every plane wave of its mesh but the
    Nyquist planes: (-1)^j along one axis gives no potential."""
    L, mesh = (8.0, 9.0, 10.0), (16, 18, 20)
    for m in ((8, 0, 0), (0, 9, 0), (0, 0, 10)):
        nyq, _ = _wave(L, mesh, m, np.cos)
        v, e = op.poisson(L, [mesh], None, [nyq])
        assert np.abs(v[0]).max() < 1e-12 and abs(e) < 1e-18, m


def _brute_poisson(L, meshes, cuts, rho):
    """The same definition by explicit sums over integer plane waves m with
    |m_d| < N_d / 2 for every level (no FFT, no index arithmetic)."""
    L = np.asarray(L, dtype=np.float64)
    vol = float(np.prod(L))
    pts, ms, keep = [], [], []
    for l, mesh in enumerate(meshes):
        ax = [np.arange(n) * (L[d] / n) for d, n in enumerate(mesh)]
        r = np.stack(np.meshgrid(*ax, indexing="ij"), axis=-1).reshape(-1, 3)
        rng_ = [np.arange(-((n - 1) // 2), (n - 1) // 2 + 1) for n in mesh]
        m = np.stack(np.meshgrid(*rng_, indexing="ij"), axis=-1).reshape(-1, 3)
        m = m[np.all(2 * np.abs(m) < np.asarray(mesh), axis=1)]
        g = 2 * math.pi * m / L
        g2 = np.sum(g * g, axis=1)
        if cuts is not None:
            m, g, g2 = m[g2 < cuts[l]], g[g2 < cuts[l]], g2[g2 < cuts[l]]
        pts.append(r)
        ms.append(m)
        keep.append(g)
    allm = np.unique(np.concatenate(ms), axis=0)
    index = {tuple(x): i for i, x in enumerate(allm)}
    rt = np.zeros(len(allm), dtype=np.complex128)
    for l, mesh in enumerate(meshes):
        w = vol / float(np.prod(mesh))
        ph = np.exp(-1j * pts[l] @ keep[l].T)
        coef = w * (rho[l].reshape(-1) @ ph)
        for k, m in enumerate(ms[l]):
            rt[index[tuple(m)]] += coef[k]
    ga = 2 * math.pi * allm / L
    g2a = np.sum(ga * ga, axis=1)
    coul = np.where(g2a > 0, 4 * math.pi / np.where(g2a > 0, g2a, 1.0), 0.0)
    vt = rt * coul
    e = float(np.sum(np.abs(rt) ** 2 * coul)) / (2 * vol)
    v = []
    for l, mesh in enumerate(meshes):
        sel = np.array([index[tuple(m)] for m in ms[l]], dtype=np.int64)
        ph = np.exp(1j * pts[l] @ keep[l].T)
        v.append(np.real(ph @ vt[sel]).reshape(mesh) / vol)
    return v, e


def test_matches_explicit_plane_wave_sums_on_meshes_with_factor_three():
    """Random level data on meshes with factors 3 and 5 and odd sizes, two
    levels with cutoffs: the oracle equals the explicit sums (pins the integer
    plane-wave indices of every level on the fine grid)."""
    L = (7.0, 8.0, 9.0)
    meshes = [(18, 24, 10), (9, 6, 5)]   # 18, 24: fftfreq(n) * n is 6.999... at m = 7
    E = (60.0, 6.0)
    rng = np.random.default_rng(9)
    rho = [rng.standard_normal(m) for m in meshes]
    v, e = op.poisson(L, meshes, E, rho)
    vb, eb = _brute_poisson(L, meshes, E, rho)
    for a, b in zip(v, vb):
        assert float(np.abs(a - b).max()) < 1e-11 * float(np.abs(b).max())
    assert abs(e - eb) < 1e-11 * abs(eb)
    v1, e1 = op.poisson(L, [(18, 15, 9)], None, [rng.standard_normal((18, 15, 9))])
    assert np.isfinite(e1)


# ------------------------------------------- fine-grid density, gradient, Hxc

def test_fine_density_and_gradient_of_a_coarse_plane_wave():
    """A plane wave stored on a coarse level is band limited: its Fourier
    interpolation to the fine mesh is the same plane wave there, and the
    gradient is -G sin(G.r) (closed forms)."""
    L = (9.0, 10.0, 11.0)
    fine, coarse = (24, 24, 30), (12, 12, 15)
    b1, gb = _wave(L, coarse, (1, -2, 3), np.cos)
    rf, grad = op.fine_density(L, [fine, coarse], (60.0, 15.0), [np.zeros(fine), b1])
    b0, _ = _wave(L, fine, (1, -2, 3), np.cos)
    s0, _ = _wave(L, fine, (1, -2, 3), np.sin)
    np.testing.assert_allclose(rf, b0, atol=1e-12)
    g = [2 * math.pi * m / L[d] for d, m in enumerate((1, -2, 3))]
    for d in range(3):
        np.testing.assert_allclose(grad[d], -g[d] * s0, atol=1e-11)


def test_hxc_without_density_passes_a_band_limited_xc_potential_through():
    """rho = 0: level 0 receives the fine-grid vxc itself (a plane wave inside
    its cutoff), a coarse level the same plane wave on its own mesh when it is
    below the coarse cutoff; the GGA term of v = (0, sin(G.r), 0) is minus its
    divergence, -G_y cos(G.r)."""
    L = (9.0, 10.0, 11.0)
    fine, coarse = (24, 24, 30), (12, 12, 15)
    E = (60.0, 15.0)
    c0, g2 = _wave(L, fine, (1, 1, -2), np.cos)
    s0, _ = _wave(L, fine, (1, 1, -2), np.sin)
    c1, _ = _wave(L, coarse, (1, 1, -2), np.cos)
    assert g2 < E[1]
    z = [np.zeros(fine), np.zeros(coarse)]
    v, e = op.hxc_potential(L, [fine, coarse], E, z, vxc=c0)
    np.testing.assert_allclose(v[0], c0, atol=1e-12)
    np.testing.assert_allclose(v[1], c1, atol=1e-12)
    assert e == 0.0
    gy = 2 * math.pi * 1 / L[1]
    v, _ = op.hxc_potential(L, [fine, coarse], E, z, vxc_grad=[np.zeros(fine), s0, np.zeros(fine)])
    np.testing.assert_allclose(v[0], -gy * c0, atol=1e-11)
    np.testing.assert_allclose(v[1], -gy * c1, atol=1e-11)


def test_xc_terms_are_adjoint_to_the_fine_density():
    """The level potentials of vxc and of the GGA vector potential are the
    derivatives of w_0 <vxc, rho_fine> and w_0 sum_d <vxc_grad_d, d_d rho_fine>
    with respect to the level densities: sum_l w_l <v_l, rho_l> equals those
    fine-grid sums for random data (the transfer and its transpose)."""
    L = (9.0, 10.0, 11.0)
    meshes = [(20, 22, 24), (12, 12, 15), (6, 8, 8)]
    E = (45.0, 15.0, 4.0)
    rng = np.random.default_rng(12)
    rho = [rng.standard_normal(m) for m in meshes]
    vxc = rng.standard_normal(meshes[0])
    vg = [rng.standard_normal(meshes[0]) for _ in range(3)]
    vol = 990.0
    w = [vol / float(np.prod(m)) for m in meshes]
    rf, grad = op.fine_density(L, meshes, E, rho)
    zero = [np.zeros(m) for m in meshes]
    v1, _ = op.hxc_potential(L, meshes, E, zero, vxc=vxc)
    lhs = sum(wl * float(np.vdot(a, r)) for wl, a, r in zip(w, v1, rho))
    assert abs(lhs - w[0] * float(np.vdot(vxc, rf))) < 1e-10 * abs(lhs)
    v2, _ = op.hxc_potential(L, meshes, E, zero, vxc_grad=vg)
    lhs = sum(wl * float(np.vdot(a, r)) for wl, a, r in zip(w, v2, rho))
    rhs = w[0] * sum(float(np.vdot(vg[d], grad[d])) for d in range(3))
    assert abs(lhs - rhs) < 1e-10 * abs(rhs)
    # the Hartree part is unchanged by the xc inputs
    v3, e3 = op.hxc_potential(L, meshes, E, rho, vxc=vxc, vxc_grad=vg)
    v4, e4 = op.poisson(L, meshes, E, rho)
    assert e3 == pytest.approx(e4, rel=1e-14)
    for a, b, c, d in zip(v3, v4, v1, v2):
        np.testing.assert_allclose(a, b + c + d, atol=1e-10 * float(np.abs(a).max()))
