"""General (non-orthogonal) cells on the HIP path against the CPU oracle,
element by element, through the C ABI (appendix on non-orthogonal lattices):
rho, the matrix and the gradient, the kinetic-energy-density terms, the FP32
variant, multigrid levels from cutoffs, and the Poisson step with
G = sum_d m_d b_d.  FP64 tolerance: 1e-10 relative to the largest magnitude of
the reference array (per level for rho and tau)."""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
import tiny
from gpu_helpers import gpu_all, log, rel_err, to_dev, to_np
from oracle import poisson as opoisson
from paper_2603_24881_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-10

# a triclinic cell (rows a_1, a_2, a_3), bohr
SKEW = np.array([[7.0, 0.0, 0.0], [1.9, 7.6, 0.0], [-1.2, 1.4, 8.2]])
# a left-handed cell with a strong shear (obtuse angles)
SHEAR = np.array([[6.5, 0.8, -0.4], [-3.1, 6.9, 0.0], [0.0, -2.2, -7.4]])


def _gpu_tau(s, D, V, precision="fp64"):
    import torch
    from paper_2603_24881_amd.gpw import GPW
    g = GPW(s, precision=precision)
    Dd = to_dev(D)
    Vd = [to_dev(v) for v in V]
    t = g.tau(Dd)
    M = g.mat_tau(Vd)
    G = g.grad_tau(Dd, Vd)
    torch.cuda.synchronize()
    out = [to_np(x) for x in t], to_np(M), to_np(G)
    g.close()
    return out


def _compare(s, D, V, tol=TOL, tau_terms=True):
    o = oracle.Oracle(s)
    rho_g, M_g, g_g, info = gpu_all(s, D, V)
    assert [tuple(m) for m in info["mesh"]] == o.meshes
    for l, (a, b) in enumerate(zip(rho_g, o.rho(D))):
        e = rel_err(a, b)
        log(f"  rho level {l} {o.meshes[l]}: rel err {e:.2e}")
        assert e < tol, (l, e)
    e = rel_err(M_g, o.mat(V))
    log(f"  M rel err {e:.2e}")
    assert e < tol
    e = rel_err(g_g, o.grad(D, V))
    log(f"  grad rel err {e:.2e}")
    assert e < tol
    if tau_terms:
        t_g, Mt_g, gt_g = _gpu_tau(s, D, V)
        for l, (a, b) in enumerate(zip(t_g, o.tau_density(D))):
            e = rel_err(a, b)
            log(f"  tau level {l}: rel err {e:.2e}")
            assert e < tol, (l, e)
        e = rel_err(Mt_g, o.mat_tau(V))
        log(f"  M_tau rel err {e:.2e}")
        assert e < tol
        e = rel_err(gt_g, o.grad_tau(D, V))
        log(f"  grad_tau rel err {e:.2e}")
        assert e < tol
    return info


@pytest.mark.parametrize("cell,mesh", [(SKEW, (18, 21, 23)), (SHEAR, (20, 24, 28)), (SKEW, (7, 9, 5))])
def test_spdf_all_operations(cell, mesh):
    """All ten classes up to (f|f), every operation, right- and left-handed
    cells, meshes that are not multiples of 4 (partial blocks), several
    lattice images."""
    log(f"[general cell] spdf mesh={mesh}")
    s = tiny.tiny_system(cell=cell, mesh=(mesh,), tau=1e-10)
    o = oracle.Oracle(s)
    D = tiny.random_density(s.n_ao)
    V = synth.make_potentials(o.meshes, 41)
    info = _compare(s, D, V)
    assert all(c > 0 for c in info["n_pairs_class"][:10]), info["n_pairs_class"]


def test_spdfg_fifteen_classes():
    """g shells on a general cell: coefficient tensors of degree 8 (10 for
    tau) rewritten on the index offset, moments up to degree 11."""
    log("[general cell] spdfg")
    s = tiny.tiny_system(shell_ls=(0, 1, 2, 3, 4), cell=SKEW, mesh=((20, 22, 24),), tau=1e-10, seed=17)
    o = oracle.Oracle(s)
    D = tiny.random_density(s.n_ao)
    V = synth.make_potentials(o.meshes, 43)
    info = _compare(s, D, V)
    assert all(c > 0 for c in info["n_pairs_class"]), info["n_pairs_class"]


def test_sharp_exponents_take_the_direct_envelope():
    """Gaussians sharp on a coarse grid: the per-axis factors of the
    envelope recursion would leave the FP64 range far from the product
    centre, so those lanes evaluate one exp per point."""
    log("[general cell] sharp exponents, coarse mesh")
    s = tiny.tiny_system(shell_ls=(0, 1, 2), natm=3, cell=SKEW, exp_range=(40.0, 120.0), mesh=((12, 13, 14),),
                         tau=1e-12, seed=5)
    o = oracle.Oracle(s)
    D = tiny.random_density(s.n_ao)
    V = synth.make_potentials(o.meshes, 45)
    _compare(s, D, V)


def _skewed_water():
    """The 32-water system (4 levels from cutoffs) in a sheared cell: the same
    fractional coordinates and basis, lattice vectors tilted by 10-15 degrees."""
    s = synth.config2()
    L = float(np.asarray(s.cell).reshape(-1)[0])
    A = np.array([[L, 0.0, 0.0], [0.25 * L, L, 0.0], [-0.15 * L, 0.2 * L, L]])
    basis = [[] for _ in range(s.natm)]
    for sh in range(s.nshell):
        p0, n = int(s.shell_prim0[sh]), int(s.shell_nprim[sh])
        basis[int(s.shell_atom[sh])].append((int(s.shell_l[sh]), s.exps[p0:p0 + n].copy(),
                                             s.coefs[p0:p0 + n].copy()))
    return synth.assemble("water32_skew", A, (s.coords / L) @ A, basis, ke_cutoff_ry=list(s.ke_cutoff_ry),
                          rel_cutoff_ry=s.rel_cutoff_ry, tau=s.tau, n_occ=s.n_occ, seed=s.seed)


def test_multigrid_water_in_a_sheared_cell():
    """Levels and meshes from cutoffs on a general cell: every level of rho,
    the matrix and the gradient."""
    log("[general cell] 32 waters, sheared cell, 4 levels")
    s = _skewed_water()
    o = oracle.Oracle(s)
    D = synth.make_density(s)
    V = synth.make_potentials(o.meshes, 47)
    info = _compare(s, D, V, tau_terms=False)
    log(f"  meshes {info['mesh']} pairs per level {info['n_pairs']}")
    assert sum(1 for n in info["n_pairs"] if n > 0) >= 2


def test_fp32_on_a_general_cell():
    log("[general cell] fp32")
    s = tiny.tiny_system(cell=SKEW, mesh=((18, 21, 23),), tau=1e-10)
    o = oracle.Oracle(s)
    D = tiny.random_density(s.n_ao)
    V = synth.make_potentials(o.meshes, 49)
    rho_g, M_g, g_g, _ = gpu_all(s, D, V, precision="fp32")
    t_g, Mt_g, gt_g = _gpu_tau(s, D, V, precision="fp32")
    errs = [rel_err(rho_g[0], o.rho(D)[0]), rel_err(M_g, o.mat(V)), rel_err(g_g, o.grad(D, V)),
            rel_err(t_g[0], o.tau_density(D)[0]), rel_err(Mt_g, o.mat_tau(V)), rel_err(gt_g, o.grad_tau(D, V))]
    log(f"  fp32 rel errs {['%.1e' % e for e in errs]}")
    assert max(errs) < 1e-4


def test_adjoint_identity_on_gpu_alone():
    """sum_l w_l <v_l, rho_l(D)> = Tr(D M(v)) on a general cell."""
    s = tiny.tiny_system(cell=SHEAR, mesh=((20, 24, 28),), tau=1e-10)
    D = tiny.random_density(s.n_ao)
    o = oracle.Oracle(s)
    V = synth.make_potentials(o.meshes, 51)
    rho, M, _, info = gpu_all(s, D, V)
    e1 = sum(w * float(np.vdot(v, r)) for w, v, r in zip(info["weight"], V, rho))
    e2 = float(np.sum(D * M))
    log(f"  adjoint {e1} {e2}")
    assert abs(e1 - e2) / abs(e1) < 1e-12
    assert abs(info["weight"][0] - abs(np.linalg.det(SHEAR)) / np.prod(o.meshes[0])) < 1e-14


def test_poisson_plane_wave_on_a_general_cell():
    """The potential of cos(G.r) with G = sum_d m_d b_d is 4 pi / |G|^2
    cos(G.r) on the skewed grid r = sum_d (i_d / N_d) a_d."""
    import torch
    from paper_2603_24881_amd.gpw import GPW
    log("[general cell] Poisson plane wave")
    mesh = (16, 18, 20)
    s = tiny.tiny_system(shell_ls=(0,), natm=1, cell=SKEW, mesh=(mesh,))
    u = np.meshgrid(*[np.arange(n) / n for n in mesh], indexing="ij")
    m = (1, -2, 3)
    phase = 2 * math.pi * (m[0] * u[0] + m[1] * u[1] + m[2] * u[2])   # G . r = 2 pi m . u
    rho = np.cos(phase)
    b = 2 * math.pi * np.linalg.inv(SKEW)   # column d is b_d
    G = b @ np.array(m, dtype=np.float64)
    g = GPW(s)
    v, ej = g.poisson().solve_async([to_dev(rho)])
    torch.cuda.synchronize()
    g.close()
    np.testing.assert_allclose(to_np(v[0]), 4 * math.pi / float(G @ G) * rho, atol=1e-11)


def test_poisson_multigrid_on_a_sheared_cell():
    """Random level data on the four levels of the sheared water cell:
    potentials, E_J, the fine-grid density and its gradient, and the Hxc
    potentials with a GGA vector potential, against the oracle."""
    import torch
    from paper_2603_24881_amd.gpw import GPW
    log("[general cell] Poisson multigrid")
    s = _skewed_water()
    g = GPW(s)
    meshes = [tuple(x) for x in g.meshes]
    rng = np.random.default_rng(53)
    rho = [rng.standard_normal(x) for x in meshes]
    vxc = rng.standard_normal(meshes[0])
    vg = [rng.standard_normal(meshes[0]) for _ in range(3)]
    p = g.poisson()
    rd = [to_dev(r) for r in rho]
    v, ej = p.solve_async(rd)
    rf, grad = p.fine_density(rd)
    vh, _ = p.hxc(rd, vxc=to_dev(vxc), vxc_grad=[to_dev(x) for x in vg])
    torch.cuda.synchronize()
    cut = s.ke_cutoff_ry
    v_o, e_o = opoisson.poisson(s.cell, meshes, cut, rho)
    for l, (a, b) in enumerate(zip(v, v_o)):
        e = rel_err(to_np(a), b)
        log(f"  v level {l} {meshes[l]}: rel err {e:.2e}")
        assert e < TOL
    assert abs(float(ej.item()) - e_o) < 1e-12 * abs(e_o)
    rf_o, grad_o = opoisson.fine_density(s.cell, meshes, cut, rho)
    assert rel_err(to_np(rf), rf_o) < TOL
    for d in range(3):
        e = rel_err(to_np(grad[d]), grad_o[d])
        log(f"  grad rho [{d}] rel err {e:.2e}")
        assert e < TOL
    vh_o, _ = opoisson.hxc_potential(s.cell, meshes, cut, rho, vxc=vxc, vxc_grad=vg)
    for l, (a, b) in enumerate(zip(vh, vh_o)):
        e = rel_err(to_np(a), b)
        log(f"  v_Hxc level {l}: rel err {e:.2e}")
        assert e < TOL
    g.close()
