"""HIP path vs the CPU oracle, element by element, through the C ABI.

Tolerance: FP64 results must match the oracle to 1e-10 relative to the
largest magnitude of the reference array (per level for rho)."""
from __future__ import annotations

import copy

import numpy as np
import pytest

import oracle
import tiny
from gpu_helpers import gpu_all, log, rel_err
from paper_2603_24881_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _oracle_all(s, D, V):
    o = oracle.Oracle(s)
    return o.rho(D), o.mat(V), o.grad(D, V), o


def _compare(s, D, V, tol=TOL, precision="fp64"):
    rho_o, M_o, g_o, o = _oracle_all(s, D, V)
    rho_g, M_g, g_g, info = gpu_all(s, D, V, precision=precision)
    assert [tuple(m) for m in info["mesh"]] == o.meshes
    for l, (a, b) in enumerate(zip(rho_g, rho_o)):
        e = rel_err(a, b)
        log(f"  rho level {l}: rel err {e:.2e}")
        assert e < tol, (l, e)
    e = rel_err(M_g, M_o)
    log(f"  M rel err {e:.2e}")
    assert e < tol
    e = rel_err(g_g, g_o)
    log(f"  grad rel err {e:.2e}")
    assert e < tol
    return info


@pytest.mark.parametrize("tau", [1e-6, 1e-14])
def test_config1(tau):
    log(f"config1 tau={tau}")
    s = synth.config1(tau=tau)
    o = oracle.Oracle(s)
    D = synth.make_density(s)
    V = synth.make_potentials(o.meshes, s.seed)
    _compare(s, D, V)


@pytest.mark.parametrize("mesh", [(20, 24, 28), (18, 21, 23), (7, 9, 5)])
def test_tiny_spdf_all_classes(mesh):
    """All ten (l_a, l_b) classes up to (f|f), anisotropic cell, meshes that
    are not multiples of 4 (partial blocks), several lattice images."""
    log(f"tiny spdf mesh={mesh}")
    s = tiny.tiny_system(mesh=(mesh,), tau=1e-10)
    o = oracle.Oracle(s)
    D = tiny.random_density(s.n_ao)
    V = synth.make_potentials(o.meshes, 21)
    info = _compare(s, D, V)
    assert all(c > 0 for c in info["n_pairs_class"][:10]), info["n_pairs_class"]


@pytest.mark.parametrize("mesh", [(20, 24, 28), (13, 11, 9)])
def test_tiny_spdfg_all_fifteen_classes(mesh):
    """g shells: all fifteen (l_a, l_b) classes up to (g|g) (coefficient
    tensors of degree 8, gradient moments of degree 9)."""
    log(f"tiny spdfg mesh={mesh}")
    s = tiny.tiny_system(shell_ls=(0, 1, 2, 3, 4), mesh=(mesh,), tau=1e-10, seed=17)
    o = oracle.Oracle(s)
    D = tiny.random_density(s.n_ao)
    V = synth.make_potentials(o.meshes, 23)
    info = _compare(s, D, V)
    assert len(info["n_pairs_class"]) == 15 and all(c > 0 for c in info["n_pairs_class"]), info["n_pairs_class"]


def test_nonsymmetric_density_and_atoms_outside_cell():
    log("nonsymmetric D, atoms outside the cell")
    s = tiny.tiny_system(shell_ls=(0, 1, 2), natm=3, mesh=((16, 18, 20),), tau=1e-8)
    s.coords = s.coords + np.array([[-9.0, 3.5, 20.0], [8.5, -17.0, 0.0], [0.0, 0.0, -30.0]])
    o = oracle.Oracle(s)
    D = tiny.random_density(s.n_ao, sym=False)
    V = synth.make_potentials(o.meshes, 4)
    _compare(s, D, V)


def test_single_atom_single_shell():
    log("single atom")
    s = tiny.tiny_system(shell_ls=(2,), natm=1, mesh=((12, 12, 12),), tau=1e-10)
    o = oracle.Oracle(s)
    D = tiny.random_density(s.n_ao)
    V = synth.make_potentials(o.meshes, 2)
    _compare(s, D, V)


def test_config2_multigrid():
    log("config2 (32 waters, 4 levels)")
    s = synth.config2()
    o = oracle.Oracle(s)
    D = synth.make_density(s)
    V = synth.make_potentials(o.meshes, s.seed)
    _compare(s, D, V)


def test_config4_diamond_with_empty_levels():
    log("config4 (216 C, 5 levels, some empty)")
    s = synth.config4()
    o = oracle.Oracle(s)
    D = synth.make_density(s)
    V = synth.make_potentials(o.meshes, s.seed)
    info = _compare(s, D, V)
    log(f"  pairs per level {info['n_pairs']}")


def test_config3_subset_gradient():
    log("config3 subset (16 waters, f shells)")
    s = tiny.subset_waters(synth.config3(), 16)
    o = oracle.Oracle(s)
    D = synth.make_density(s)
    V = synth.make_potentials(o.meshes, 33)
    _compare(s, D, V)


def test_adjoint_identity_on_gpu_alone():
    """sum_l w_l <v_l, rho_l(D)> = Tr(D M(v)) with both sides from the GPU."""
    s = synth.config2()
    o = oracle.Oracle(s)
    D = synth.make_density(s)
    V = synth.make_potentials(o.meshes, 77)
    rho, M, _, info = gpu_all(s, D, V)
    e1 = sum(w * float(np.vdot(v, r)) for w, v, r in zip(info["weight"], V, rho))
    e2 = float(np.sum(D * M))
    log(f"  adjoint {e1} {e2}")
    assert abs(e1 - e2) / abs(e1) < 1e-12


def test_fp32_variant_error_is_bounded():
    """FP32 per-point arithmetic (FP64 screening, accumulation across levels and
    matrix reduction): error against the FP64 oracle stays small."""
    log("fp32 variant on config2")
    s = synth.config2()
    o = oracle.Oracle(s)
    D = synth.make_density(s)
    V = synth.make_potentials(o.meshes, s.seed)
    rho_o, M_o, g_o, _ = _oracle_all(s, D, V)
    rho_g, M_g, g_g, _ = gpu_all(s, D, V, precision="fp32")
    errs = [rel_err(a, b) for a, b in zip(rho_g, rho_o)] + [rel_err(M_g, M_o), rel_err(g_g, g_o)]
    log(f"  fp32 rel errs {['%.1e' % e for e in errs]}")
    assert max(errs) < 1e-4


def test_flop_model_follows_its_definition():
    """The plan's work counts, per (l_a, l_b) class over all ten classes: the
    counting convention (direct evaluation, 64 points per block incidence),
    the kernels' arithmetic (coefficient tensor for the rho d and f classes;
    moments for mat with l_a + l_b >= 2) and the
    in-sphere count below the block count."""
    from math import comb
    from paper_2603_24881_amd.gpw import GPW
    s = tiny.tiny_system(mesh=((20, 24, 28),), tau=1e-10)
    g = GPW(s)
    info = g.info
    g.close()
    conv = exec_rho = exec_mat = 0.0
    for la in range(4):
        for lb in range(la + 1):
            c = la * (la + 1) // 2 + lb
            inc = info["n_incidences_class"][c]
            na, nb, L = (la + 1) * (la + 2) // 2, (lb + 1) * (lb + 2) // 2, la + lb
            f1 = 2 * na * nb + 2 * (na + nb) + 4
            conv += 64.0 * f1 * inc
            tensor_rho = la >= 2
            exec_rho += (8 * comb(L + 2, 3) + 32 * comb(L + 1, 2) + 16 + 64 * (2 * L + 3) if tensor_rho
                         else 64 * f1) * inc
            exec_mat += 64.0 * ((2 * L + 3) if L >= 2 else f1) * inc
    assert all(info["n_incidences_class"][c] > 0 for c in range(10))
    assert info["flops_rho_block"] == pytest.approx(conv, rel=1e-12)
    assert info["flops_mat_block"] == pytest.approx(conv, rel=1e-12)
    assert info["flops_rho_exec"] == pytest.approx(exec_rho, rel=1e-12)
    assert info["flops_mat_exec"] == pytest.approx(exec_mat, rel=1e-12)
    assert 0 < info["flops_rho_sphere"] <= info["flops_rho_block"]
    assert info["flops_rho_exec"] < info["flops_rho_block"]
