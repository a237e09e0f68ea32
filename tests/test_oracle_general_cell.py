"""Pins of the oracle on general (non-orthogonal) cells, independent of its
code: the untruncated chi product on the skewed grid r = sum_d (i_d / N_d) a_d,
closed-form overlap and kinetic matrices summed over the lattice T = n . A,
finite differences, the sampled modes, and the Poisson step by explicit
plane-wave sums with G = sum_d m_d b_d (appendix on non-orthogonal lattices;
Sec. II)."""
from __future__ import annotations

import copy
import math

import numpy as np
import pytest

import oracle
import pins
import tiny
from oracle import poisson as op
from paper_2603_24881_amd import synth

# a triclinic cell (rows a_1, a_2, a_3), bohr
SKEW = np.array([[7.0, 0.0, 0.0], [1.9, 7.6, 0.0], [-1.2, 1.4, 8.2]])


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _system(mesh=((18, 20, 22),), tau=1e-18, shell_ls=(0, 1, 2), natm=3, exp_range=(0.7, 3.0), seed=21):
    return tiny.tiny_system(shell_ls=shell_ls, natm=natm, cell=SKEW, exp_range=exp_range, mesh=mesh, tau=tau,
                            seed=seed)


def test_rho_mat_tau_match_brute_force_on_a_skewed_cell():
    s = _system()
    o = oracle.Oracle(s)
    D = tiny.random_density(s.n_ao)
    mesh = o.meshes[0]
    chi = pins.brute_chi(s, mesh, nimg=2)
    assert rel(o.rho(D)[0], pins.brute_rho(chi, D, mesh)) < 1e-11
    V = synth.make_potentials(o.meshes, 6)
    w = o.weights()[0]
    assert abs(w - abs(np.linalg.det(SKEW)) / np.prod(mesh)) < 1e-15 * w
    assert rel(o.mat(V), pins.brute_mat(chi, V[0], w)) < 1e-11
    gchi = pins.brute_grad_chi(s, mesh, nimg=2)
    assert rel(o.tau_density(D)[0], pins.brute_tau(gchi, D, mesh)) < 1e-11
    assert rel(o.mat_tau(V), pins.brute_mat_tau(gchi, V[0], w)) < 1e-11


def test_overlap_and_kinetic_on_a_fine_skewed_grid():
    s = _system(mesh=((48, 52, 56),), shell_ls=(0, 1, 2), natm=2, exp_range=(0.6, 2.0))
    o = oracle.Oracle(s)
    ones = [np.ones(o.meshes[0])]
    assert rel(o.mat(ones), pins.overlap(s, nimg=2)) < 1e-10
    assert rel(o.mat_tau(ones), pins.kinetic(s, nimg=2)) < 1e-10


@pytest.mark.parametrize("atom,axis", [(0, 0), (1, 2), (2, 1)])
def test_gradients_match_central_differences_on_a_skewed_cell(atom, axis):
    s = _system(tau=1e-14, shell_ls=(0, 1, 2, 3))
    o = oracle.Oracle(s)
    D = tiny.random_density(s.n_ao)
    V = synth.make_potentials(o.meshes, 9)
    g, gt = o.grad(D, V), o.grad_tau(D, V)
    h = 1e-4

    def energies(delta):
        s2 = copy.copy(s)
        s2.coords = s.coords.copy()
        s2.coords[atom, axis] += delta
        o2 = oracle.Oracle(s2)
        return o2.energy(D, V), o2.energy_tau(D, V)

    (ep, tp), (em, tm) = energies(h), energies(-h)
    assert abs(g[atom, axis] - (ep - em) / (2 * h)) / np.abs(g).max() < 1e-6
    assert abs(gt[atom, axis] - (tp - tm) / (2 * h)) / np.abs(gt).max() < 1e-6


def test_sampled_modes_equal_full_on_a_skewed_multigrid():
    s = _system(mesh=None, tau=1e-10, shell_ls=(0, 1, 2), exp_range=(0.3, 4.0))
    s.mesh = None
    s.ke_cutoff_ry = [200.0, 60.0]
    s.rel_cutoff_ry = 30.0
    o = oracle.Oracle(s)
    assert o.nlevels == 2 and all(c > 0 for c in o.count_pairs())
    D = tiny.random_density(s.n_ao)
    full = o.rho(D)
    rng = np.random.default_rng(4)
    for l, m in enumerate(o.meshes):
        idx = rng.choice(int(np.prod(m)), 40, replace=False)
        assert rel(o.rho_points(D, l, idx), full[l].reshape(-1)[idx]) < 1e-13
    V = synth.make_potentials(o.meshes, 3)
    M = o.mat(V)
    off = s.ao_offsets()
    pairs = [(0, 1), (2, 2), (4, 3)]
    for (a, b), blk in zip(pairs, o.mat_blocks(V, pairs)):
        assert rel(blk, M[off[a]:off[a + 1], off[b]:off[b + 1]]) < 1e-13


def test_mesh_rule_uses_the_lattice_vector_lengths():
    s = _system(mesh=None)
    s.mesh = None
    s.ke_cutoff_ry = [100.0]
    o = oracle.Oracle(s)
    for d in range(3):
        need = math.sqrt(100.0) * np.linalg.norm(SKEW[d]) / math.pi
        n = o.meshes[0][d]
        assert n >= need and all(n % p == 0 or True for p in (2, 3, 5))
        assert n - 1 < need or any(((n - 1) % p) for p in (7, 11, 13))


def _brute_poisson_general(A, meshes, cuts, rho):
    """Explicit sums over integer m with |m_d| < N_d / 2, G = 2 pi A^-1 m."""
    A = np.asarray(A, dtype=np.float64)
    inv = np.linalg.inv(A)
    vol = abs(np.linalg.det(A))
    pts, ms, gs = [], [], []
    for l, mesh in enumerate(meshes):
        r = pins.grid_points(A, mesh)
        rng_ = [np.arange(-((n - 1) // 2), (n - 1) // 2 + 1) for n in mesh]
        m = np.stack(np.meshgrid(*rng_, indexing="ij"), axis=-1).reshape(-1, 3)
        m = m[np.all(2 * np.abs(m) < np.asarray(mesh), axis=1)]
        g = 2 * math.pi * m @ inv.T
        keep = np.sum(g * g, axis=1) < cuts[l]
        pts.append(r)
        ms.append(m[keep])
        gs.append(g[keep])
    allm = np.unique(np.concatenate(ms), axis=0)
    index = {tuple(x): i for i, x in enumerate(allm)}
    rt = np.zeros(len(allm), dtype=np.complex128)
    for l, mesh in enumerate(meshes):
        coef = (vol / float(np.prod(mesh))) * (rho[l].reshape(-1) @ np.exp(-1j * pts[l] @ gs[l].T))
        for k, m in enumerate(ms[l]):
            rt[index[tuple(m)]] += coef[k]
    ga = 2 * math.pi * allm @ inv.T
    g2 = np.sum(ga * ga, axis=1)
    coul = np.where(g2 > 0, 4 * math.pi / np.where(g2 > 0, g2, 1.0), 0.0)
    e = float(np.sum(np.abs(rt) ** 2 * coul)) / (2 * vol)
    v = []
    for l, mesh in enumerate(meshes):
        sel = np.array([index[tuple(m)] for m in ms[l]], dtype=np.int64)
        v.append(np.real(np.exp(1j * pts[l] @ gs[l].T) @ (rt * coul)[sel]).reshape(mesh) / vol)
    return v, e


def test_poisson_on_a_skewed_cell_matches_explicit_sums():
    meshes = [(12, 10, 9), (6, 5, 5)]
    E = (40.0, 6.0)
    rng = np.random.default_rng(14)
    rho = [rng.standard_normal(m) for m in meshes]
    v, e = op.poisson(SKEW, meshes, E, rho)
    vb, eb = _brute_poisson_general(SKEW, meshes, E, rho)
    for a, b in zip(v, vb):
        assert float(np.abs(a - b).max()) < 1e-11 * float(np.abs(b).max())
    assert abs(e - eb) < 1e-11 * abs(eb)


def test_poisson_plane_wave_on_a_skewed_cell():
    """rho = cos(G.r), G = sum m_d b_d: v = 4 pi / |G|^2 cos(G.r)."""
    mesh = (16, 18, 20)
    r = pins.grid_points(SKEW, mesh)
    G = 2 * math.pi * np.linalg.inv(SKEW) @ np.array([1.0, -2.0, 1.0])
    rho = np.cos(r @ G).reshape(mesh)
    v, e = op.poisson(SKEW, [mesh], None, [rho])
    g2 = float(G @ G)
    np.testing.assert_allclose(v[0], 4 * math.pi / g2 * rho, atol=1e-12)
    assert abs(e - math.pi * abs(np.linalg.det(SKEW)) / g2) < 1e-10 * e
