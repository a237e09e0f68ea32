"""Pins of the oracle on g shells (l = 4), independent of its code: the
untruncated brute-force chi product, the closed-form periodic overlap and
kinetic matrices on a fine grid, and central finite differences of the
energies.  These pin the Cartesian order of the 15 g components, the
polynomial depth of the 1-D tables (degree 4 + 2 for the second derivatives
of the meta-GGA gradient) and the lattice sums for the highest angular
momentum the library accepts."""
from __future__ import annotations

import copy

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


def _g_system(mesh=((18, 20, 22),), tau=1e-14, shell_ls=(0, 2, 4), natm=2, exp_range=(0.7, 3.0)):
    return tiny.tiny_system(shell_ls=shell_ls, natm=natm, exp_range=exp_range, mesh=mesh, tau=tau, seed=11)


def test_g_cartesian_order():
    """15 components, lexicographic with lx descending, then ly descending."""
    c = pins.cart_list(4)
    assert len(c) == 15 and c[0] == (4, 0, 0) and c[1] == (3, 1, 0) and c[2] == (3, 0, 1)
    assert c[-1] == (0, 0, 4) and c[4] == (2, 1, 1)


def test_rho_mat_tau_match_brute_force_with_g_shells():
    # tau = 1e-18: the truncation of Eq. (cut) bounds r^(L+2) about P, while a g
    # pair's polynomial about distant centres is larger, so at 1e-14 the
    # truncated sum differs from the untruncated one by ~4e-11 relative
    s = _g_system(tau=1e-18)
    o = oracle.Oracle(s)
    D = tiny.random_density(s.n_ao)
    mesh = o.meshes[0]
    chi = pins.brute_chi(s, mesh, nimg=2)
    assert rel(o.rho(D)[0], pins.brute_rho(chi, D, mesh)) < 1e-11
    V = synth.make_potentials(o.meshes, 6)
    assert rel(o.mat(V), pins.brute_mat(chi, V[0], o.weights()[0])) < 1e-11
    gchi = pins.brute_grad_chi(s, mesh, nimg=2)
    assert rel(o.tau_density(D)[0], pins.brute_tau(gchi, D, mesh)) < 1e-11
    assert rel(o.mat_tau(V), pins.brute_mat_tau(gchi, V[0], o.weights()[0])) < 1e-11


def test_g_overlap_and_kinetic_on_a_fine_grid():
    """M(v = 1) = S and M_tau(v = 1) = T from closed-form Gaussian moments."""
    # degree-10 integrands (g x g, both differentiated): a finer grid than for
    # d shells keeps the aliasing below the tolerance
    s = _g_system(mesh=((60, 64, 72),), shell_ls=(1, 4), exp_range=(0.6, 2.0), tau=1e-18)
    o = oracle.Oracle(s)
    ones = [np.ones(o.meshes[0])]
    assert rel(o.mat(ones), pins.overlap(s, nimg=2)) < 1e-10
    assert rel(o.mat_tau(ones), pins.kinetic(s, nimg=2)) < 1e-10


@pytest.mark.parametrize("atom,axis", [(0, 0), (1, 2)])
def test_g_gradients_match_central_differences(atom, axis):
    s = _g_system(shell_ls=(2, 4))
    o = oracle.Oracle(s)
    D = tiny.random_density(s.n_ao)
    V = synth.make_potentials(o.meshes, 9)
    g = o.grad(D, V)
    gt = o.grad_tau(D, V)
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
