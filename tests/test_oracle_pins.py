"""Pins of the CPU oracle against references that are not the oracle itself.

Every pin here is independent of the oracle's code: brute-force periodic
orbitals, closed-form Gaussian integrals, Poisson summation, finite
differences, hand-computed meshes, and exact invariances of the definitions.
"""
from __future__ import annotations

import copy
import math

import numpy as np
import pytest

import oracle
import pins
import tiny
from paper_2603_24881_amd import synth


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


# --------------------------------------------------------------- brute force

def test_rho_mat_match_brute_force_spdf():
    """Oracle vs untruncated chi-product on an anisotropic cell/mesh with
    s, p, d and f shells (tau = 1e-14): pins the lattice sum, the fold, the
    Cartesian order, the D contraction and the weight (Sec. II Eq. (rho),
    Sec. III.A Eqs. (rho_wrap), (J_wrap))."""
    s = tiny.tiny_system()
    o = oracle.Oracle(s)
    D = tiny.random_density(s.n_ao)
    chi = pins.brute_chi(s, o.meshes[0], nimg=2)
    rho = o.rho(D)[0]
    assert rel(rho, pins.brute_rho(chi, D, o.meshes[0])) < 1e-11
    V = synth.make_potentials(o.meshes, 5)
    M = o.mat(V)
    assert rel(M, pins.brute_mat(chi, V[0], o.weights()[0])) < 1e-11


def test_config1_matches_brute_force():
    s = synth.config1(tau=1e-14)
    o = oracle.Oracle(s)
    D = synth.make_density(s)
    chi = pins.brute_chi(s, o.meshes[0], nimg=3)
    assert rel(o.rho(D)[0], pins.brute_rho(chi, D, o.meshes[0])) < 1e-11
    V = synth.make_potentials(o.meshes, s.seed)
    assert rel(o.mat(V), pins.brute_mat(chi, V[0], o.weights()[0])) < 1e-11


def test_nonsymmetric_density_uses_symmetric_part():
    """rho(D) = rho(D^T) = rho((D + D^T)/2): both orders of every pair are summed."""
    s = tiny.tiny_system(shell_ls=(0, 1, 2), natm=2, mesh=((16, 18, 20),))
    o = oracle.Oracle(s)
    D = tiny.random_density(s.n_ao, sym=False)
    r1 = o.rho(D)[0]
    r2 = o.rho(D.T.copy())[0]
    r3 = o.rho(0.5 * (D + D.T))[0]
    assert rel(r1, r2) < 1e-13 and rel(r1, r3) < 1e-13


# --------------------------------------------------------------- closed forms

def test_mat_of_unit_potential_is_periodic_overlap():
    """On a fine grid (aliasing exp(-pi^2/(alpha h^2)) < 1e-18), M(v=1) = S and
    sum_r w rho = Tr(D S), with S from closed-form Gaussian moments."""
    s = tiny.tiny_system(shell_ls=(0, 1, 2), natm=2, exp_range=(0.6, 3.0), mesh=((44, 48, 52),))
    o = oracle.Oracle(s)
    S = pins.overlap(s, nimg=2)
    assert rel(o.mat([np.ones(o.meshes[0])]), S) < 1e-10
    D = tiny.random_density(s.n_ao)
    integral = o.rho(D)[0].sum() * o.weights()[0]
    assert abs(integral - np.sum(D * S)) / abs(np.sum(D * S)) < 1e-11


def test_grad_of_unit_potential_is_overlap_derivative():
    """v = 1 on a fine grid: dE/dR_X = sum D dS/dR_X (closed form), tau = 1e-20."""
    s = tiny.tiny_system(shell_ls=(0, 1, 2), natm=2, exp_range=(0.6, 3.0), mesh=((44, 48, 52),),
                         tau=1e-20)
    o = oracle.Oracle(s)
    D = tiny.random_density(s.n_ao)
    g = o.grad(D, [np.ones(o.meshes[0])])
    assert rel(g, pins.overlap_grad(s, D, nimg=2)) < 1e-10


def test_coarse_grid_sums_match_theta_series():
    """s-only system on a coarse, uneven grid: the grid sum including aliasing
    equals the Poisson-summation closed form (far from the continuum S)."""
    s = tiny.tiny_system(shell_ls=(0, 0), natm=2, exp_range=(0.5, 6.0), mesh=((9, 10, 11),),
                         tau=1e-18)
    o = oracle.Oracle(s)
    M1 = o.mat([np.ones(o.meshes[0])])
    Mt = pins.theta_mat_ones(s, o.meshes[0], nimg=3)
    assert rel(M1, Mt) < 1e-12
    assert rel(M1, pins.overlap(s, nimg=3)) > 1e-2   # the grid is genuinely coarse


def test_multigrid_unit_potential_gives_overlap():
    """With every pair exponent below E_0 / E_rel, the level rule puts each pair
    on a grid that resolves it, so sum over levels of M_l(v=1) = S and
    sum_l w_l sum rho_l = Tr(D S).  A pair placed on a too-coarse level aliases
    and breaks this (Sec. II, multigrid)."""
    s = tiny.tiny_system(shell_ls=(0, 1, 2), natm=2, exp_range=(0.3, 2.0), mesh=None)
    s.mesh = None
    s.ke_cutoff_ry = [240.0, 80.0, 27.0]
    s.rel_cutoff_ry = 60.0
    s.tau = 1e-14
    o = oracle.Oracle(s)
    assert o.nlevels == 3
    counts = o.count_pairs()
    assert (counts > 0).sum() >= 2, counts
    S = pins.overlap(s, nimg=2)
    ones = [np.ones(m) for m in o.meshes]
    assert rel(o.mat(ones), S) < 1e-10
    D = tiny.random_density(s.n_ao)
    rho = o.rho(D)
    integral = sum(w * r.sum() for w, r in zip(o.weights(), rho))
    assert abs(integral - np.sum(D * S)) / abs(np.sum(D * S)) < 1e-10


# ------------------------------------------------------- finite differences

@pytest.mark.parametrize("atom,axis", [(0, 0), (1, 2), (2, 1)])
def test_grad_matches_central_differences(atom, axis):
    s = tiny.tiny_system(tau=1e-14)
    o = oracle.Oracle(s)
    D = tiny.random_density(s.n_ao)
    V = synth.make_potentials(o.meshes, 5)
    g = o.grad(D, V)
    h = 1e-4

    def energy(delta):
        s2 = copy.copy(s)
        s2.coords = s.coords.copy()
        s2.coords[atom, axis] += delta
        return oracle.Oracle(s2).energy(D, V)

    fd = (energy(h) - energy(-h)) / (2 * h)
    assert abs(g[atom, axis] - fd) / np.abs(g).max() < 1e-6


# ------------------------------------------------------------- invariances

def _shifted(s, delta, atoms=None):
    s2 = copy.copy(s)
    s2.coords = s.coords.copy()
    if atoms is None:
        s2.coords += delta
    else:
        s2.coords[atoms] += delta
    return s2


def test_shift_by_grid_steps_rolls_rho():
    s = tiny.tiny_system(shell_ls=(0, 1, 2), natm=3, mesh=((20, 24, 28),))
    o = oracle.Oracle(s)
    D = tiny.random_density(s.n_ao)
    rho = o.rho(D)[0]
    h = s.cell / np.asarray(o.meshes[0])
    s2 = _shifted(s, np.array([3 * h[0], 0.0, -2 * h[2]]))
    rho2 = oracle.Oracle(s2).rho(D)[0]
    assert rel(rho2, np.roll(np.roll(rho, 3, axis=0), -2, axis=2)) < 1e-12


def test_lattice_translation_of_an_atom_changes_nothing():
    s = tiny.tiny_system(shell_ls=(0, 1, 2), natm=3, mesh=((20, 24, 28),))
    o = oracle.Oracle(s)
    D = tiny.random_density(s.n_ao)
    V = synth.make_potentials(o.meshes, 9)
    s2 = _shifted(s, np.array([s.cell[0], -2 * s.cell[1], 0.0]), atoms=[1])
    o2 = oracle.Oracle(s2)
    assert rel(o2.rho(D)[0], o.rho(D)[0]) < 1e-12
    assert rel(o2.mat(V), o.mat(V)) < 1e-12
    assert rel(o2.grad(D, V), o.grad(D, V)) < 1e-10


def test_linearity_in_density():
    s = tiny.tiny_system(shell_ls=(0, 1), natm=3, mesh=((16, 18, 20),))
    o = oracle.Oracle(s)
    D1 = tiny.random_density(s.n_ao, seed=1)
    D2 = tiny.random_density(s.n_ao, seed=2)
    lhs = o.rho(2.5 * D1 - 0.5 * D2)[0]
    rhs = 2.5 * o.rho(D1)[0] - 0.5 * o.rho(D2)[0]
    assert rel(lhs, rhs) < 1e-12


def test_atom_permutation_permutes_matrix():
    s = tiny.tiny_system(shell_ls=(0, 1, 2), natm=3, mesh=((16, 18, 20),))
    o = oracle.Oracle(s)
    V = synth.make_potentials(o.meshes, 4)
    M = o.mat(V)
    perm = [2, 0, 1]                      # new atom i is old atom perm[i]
    shells_by_atom = [[sh for sh in range(s.nshell) if s.shell_atom[sh] == a] for a in range(s.natm)]
    off = s.ao_offsets()
    atom_basis = []
    ao_map = []
    for new, old in enumerate(perm):
        shells = []
        for sh in shells_by_atom[old]:
            p0, n = int(s.shell_prim0[sh]), int(s.shell_nprim[sh])
            shells.append((int(s.shell_l[sh]), s.exps[p0:p0 + n], s.coefs[p0:p0 + n]))
            ao_map.extend(range(off[sh], off[sh + 1]))
        atom_basis.append(shells)
    s2 = synth.assemble("perm", s.cell, s.coords[perm], atom_basis, mesh=s.mesh,
                        ke_cutoff_ry=[], tau=s.tau)
    M2 = oracle.Oracle(s2).mat(V)
    assert rel(M2, M[np.ix_(ao_map, ao_map)]) < 1e-13


def test_adjoint_identity():
    """sum_l w_l <v_l, rho_l(D)> = sum D_{mu nu} M(v)_{mu nu} on a multigrid system."""
    s = synth.config2(tau=1e-6)
    sub = tiny.subset_waters(s, 4)
    o = oracle.Oracle(sub)
    D = synth.make_density(sub)
    V = synth.make_potentials(o.meshes, 3)
    E1 = sum(w * float(np.vdot(v, r)) for w, v, r in zip(o.weights(), V, o.rho(D)))
    E2 = float(np.sum(D * o.mat(V)))
    assert abs(E1 - E2) / abs(E1) < 1e-12


# ------------------------------------------------------ truncation & levels

def _brute_pair_levels(s, tau, cuts, rel_cut, nimg=4):
    """Ordered pair images with max_r |K| r^(L+2) e^(-alpha r^2) >= tau, counted
    per level, by brute force over a wide range of images."""
    counts = np.zeros(max(1, len(cuts)), dtype=np.int64)
    prim = []
    for sh in range(s.nshell):
        for k in range(int(s.shell_nprim[sh])):
            prim.append((sh, s.exps[s.shell_prim0[sh] + k], s.coefs[s.shell_prim0[sh] + k]))
    r = range(-nimg, nimg + 1)
    Ts = np.array([[i, j, k] for i in r for j in r for k in r], dtype=np.float64) * s.cell
    for (sa, ea, ca) in prim:
        A = s.coords[s.shell_atom[sa]]
        for (sb, eb, cb) in prim:
            B = s.coords[s.shell_atom[sb]]
            L = int(s.shell_l[sa] + s.shell_l[sb])
            p = ea + eb
            d2 = np.sum((A - B - Ts) ** 2, axis=1)
            K = np.abs(ca * cb) * np.exp(-ea * eb / p * d2)
            rs = math.sqrt((L + 2) / (2 * p))
            fmax = K * rs ** (L + 2) * math.exp(-p * rs * rs)
            n = int(np.sum(fmax >= tau))
            if not cuts:
                lvl = 0
            else:
                lvl = 0
                for i in range(len(cuts) - 1, -1, -1):
                    if cuts[i] >= p * rel_cut:
                        lvl = i
                        break
            counts[lvl] += n
    return counts


def test_pair_image_enumeration_and_levels_match_brute_force():
    s = synth.config2(tau=1e-6)
    sub = tiny.subset_waters(s, 3)
    o = oracle.Oracle(sub)
    expect = _brute_pair_levels(sub, sub.tau, sub.ke_cutoff_ry, sub.rel_cutoff_ry)
    assert np.array_equal(o.count_pairs(), expect)


def test_truncation_error_shrinks_with_tau():
    s = tiny.tiny_system(shell_ls=(0, 1, 2), natm=3, mesh=((20, 24, 28),))
    D = tiny.random_density(s.n_ao)
    chi = pins.brute_chi(s, (20, 24, 28), nimg=2)
    exact = pins.brute_rho(chi, D, (20, 24, 28))
    errs = [rel(oracle.Oracle(s, tau=t).rho(D)[0], exact) for t in (1e-4, 1e-6, 1e-10)]
    assert errs[0] < 1e-1 and errs[1] < 1e-3 and errs[2] < 1e-7
    assert errs[0] > errs[1] > errs[2]


def test_mesh_rule_hand_values():
    """N = smallest 2,3,5-smooth integer >= sqrt(E) L / pi, e.g. 18.6 bohr at
    400/130/45/15 Ry -> 120/72/40/24 and 29.53 bohr -> 192/108/64/40."""
    for L, expect in [(18.6, [120, 72, 40, 24]), (29.53, [192, 108, 64, 40]), (25.0, [160, 96, 54, 32])]:
        s = synth.water_cluster(1, L, 1, synth.O_BASIS_SMALL)
        o = oracle.Oracle(s)
        assert [m[0] for m in o.meshes] == expect


def test_mask_either_gives_complete_gradient_rows():
    """The sampling filter: with pairs that touch the selected atoms, their
    gradient rows equal those of the full sum."""
    s = tiny.subset_waters(synth.config3(tau=1e-12), 3)
    o = oracle.Oracle(s)
    D = synth.make_density(s)
    V = synth.make_potentials(o.meshes, 5)
    g = o.grad(D, V)
    mask = np.zeros(s.natm, dtype=np.uint8)
    mask[[1, 5]] = 1
    gm = oracle.Oracle(s, atom_mask=mask, mask_either=True).grad(D, V)
    assert np.abs(gm[[1, 5]] - g[[1, 5]]).max() < 1e-12 * np.abs(g).max()
