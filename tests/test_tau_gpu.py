"""Meta-GGA kinetic-energy-density terms on the HIP path against the CPU oracle,
element by element, through the C ABI: tau_l = 1/2 sum D grad phi . grad phi on
every level (gpw_eval_tau), the matrix term 1/2 sum w vtau grad phi . grad phi
(gpw_eval_mat_tau) and the nuclear gradient of E_tau = sum w <vtau, tau>
(gpw_eval_grad_tau).  FP64 tolerance: 1e-10 relative to the largest magnitude of
the reference array (per level for tau); the full-size system is checked on
sampled outputs the oracle computes one by one."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import tiny
from gpu_helpers import log, rel_err, to_dev, to_np
from paper_2603_24881_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-10


def gpu_tau_all(system, D, V, precision="fp64"):
    import torch
    from paper_2603_24881_amd.gpw import GPW
    g = GPW(system, precision=precision)
    Dd = to_dev(D)
    Vd = [to_dev(v) for v in V]
    t = g.tau(Dd)
    M = g.mat_tau(Vd)
    G = g.grad_tau(Dd, Vd)
    torch.cuda.synchronize()
    out = ([to_np(x) for x in t], to_np(M), to_np(G), g.info)
    g.close()
    return out


def _compare(s, D, V, tol=TOL):
    o = oracle.Oracle(s)
    t_o, M_o, g_o = o.tau_density(D), o.mat_tau(V), o.grad_tau(D, V)
    t_g, M_g, g_g, info = gpu_tau_all(s, D, V)
    for l, (a, b) in enumerate(zip(t_g, t_o)):
        e = rel_err(a, b)
        log(f"  tau level {l}: rel err {e:.2e} (max |ref| {np.abs(b).max():.2e})")
        assert e < tol, (l, e)
    e = rel_err(M_g, M_o)
    log(f"  M_tau rel err {e:.2e}")
    assert e < tol
    e = rel_err(g_g, g_o)
    log(f"  grad_tau rel err {e:.2e}")
    assert e < tol
    return info


@pytest.mark.parametrize("tau", [1e-6, 1e-14])
def test_config1(tau):
    log(f"[tau] config1 tau={tau}")
    s = synth.config1(tau=tau)
    o = oracle.Oracle(s)
    _compare(s, synth.make_density(s), synth.make_potentials(o.meshes, s.seed))


@pytest.mark.parametrize("mesh", [(20, 24, 28), (18, 21, 23), (7, 9, 5)])
def test_tiny_spdf_all_classes(mesh):
    """All ten classes up to (f|f) (tensors of degree up to 8, moments up to 9),
    an anisotropic cell, meshes that are not multiples of 4, several images."""
    log(f"[tau] tiny spdf mesh={mesh}")
    s = tiny.tiny_system(mesh=(mesh,), tau=1e-10)
    o = oracle.Oracle(s)
    info = _compare(s, tiny.random_density(s.n_ao), synth.make_potentials(o.meshes, 21))
    assert all(c > 0 for c in info["n_pairs_class"][:10]), info["n_pairs_class"]


def test_tiny_spdfg_all_fifteen_classes():
    """g shells: tau tensors up to degree 10, moments up to degree 11."""
    log("[tau] tiny spdfg")
    s = tiny.tiny_system(shell_ls=(0, 1, 2, 3, 4), mesh=((20, 24, 28),), tau=1e-10, seed=17)
    o = oracle.Oracle(s)
    info = _compare(s, tiny.random_density(s.n_ao), synth.make_potentials(o.meshes, 23))
    assert all(c > 0 for c in info["n_pairs_class"]), info["n_pairs_class"]


def test_nonsymmetric_density_and_atoms_outside_cell():
    log("[tau] nonsymmetric D, atoms outside the cell")
    s = tiny.tiny_system(shell_ls=(0, 1, 2), natm=3, mesh=((16, 18, 20),), tau=1e-8)
    s.coords = s.coords + np.array([[-9.0, 3.5, 20.0], [8.5, -17.0, 0.0], [0.0, 0.0, -30.0]])
    o = oracle.Oracle(s)
    _compare(s, tiny.random_density(s.n_ao, sym=False), synth.make_potentials(o.meshes, 4))


def test_config2_multigrid():
    log("[tau] config2 (32 waters, 4 levels)")
    s = synth.config2()
    o = oracle.Oracle(s)
    _compare(s, synth.make_density(s), synth.make_potentials(o.meshes, s.seed))


def test_config3_subset_f_shells():
    log("[tau] config3 subset (8 waters, f shells)")
    s = tiny.subset_waters(synth.config3(), 8)
    o = oracle.Oracle(s)
    _compare(s, synth.make_density(s), synth.make_potentials(o.meshes, 33))


def test_adjoint_identity_and_energy_on_gpu_alone():
    """sum_l w_l <vtau_l, tau_l(D)> = Tr(D M_tau(vtau)) with both sides from the
    GPU, and tau >= 0 pointwise for a positive semidefinite D at tau = 1e-14."""
    log("[tau] adjoint identity, positivity")
    s = synth.config1(tau=1e-14)
    o = oracle.Oracle(s)
    D = synth.make_density(s)
    V = synth.make_potentials(o.meshes, 77)
    t, M, _, info = gpu_tau_all(s, D, V)
    e1 = sum(w * float(np.vdot(v, r)) for w, v, r in zip(info["weight"], V, t))
    e2 = float(np.sum(D * M))
    log(f"  adjoint {e1} {e2}")
    assert abs(e1 - e2) / abs(e1) < 1e-12
    assert min(float(x.min()) for x in t) > -1e-12 * max(float(np.abs(x).max()) for x in t)


def test_gradient_against_finite_differences_on_gpu_alone():
    """dE_tau/dR from gpw_eval_grad_tau against central differences of
    E_tau(R) = sum w <vtau, tau(D; R)> from gpw_eval_tau (h = 1e-4 bohr,
    tau = 1e-14, two atoms, all three directions)."""
    import copy
    import torch
    from paper_2603_24881_amd.gpw import GPW
    log("[tau] finite differences")
    s = synth.config1(tau=1e-14)
    o = oracle.Oracle(s)
    D = synth.make_density(s)
    V = synth.make_potentials(o.meshes, 5)
    Dd = to_dev(D)
    Vd = [to_dev(v) for v in V]

    def energy(sys):
        g = GPW(sys)
        t = g.tau(Dd)
        torch.cuda.synchronize()
        e = sum(w * float(torch.vdot(v.reshape(-1), x.reshape(-1))) for w, v, x in zip(g.weights, Vd, t))
        g.close()
        return e

    g = GPW(s)
    G = to_np(g.grad_tau(Dd, Vd))
    g.close()
    h = 1e-4
    fd = np.zeros((2, 3))
    for a in range(2):
        for d in range(3):
            sp, sm = copy.deepcopy(s), copy.deepcopy(s)
            sp.coords[a, d] += h
            sm.coords[a, d] -= h
            fd[a, d] = (energy(sp) - energy(sm)) / (2 * h)
    e = float(np.abs(fd - G[:2]).max() / np.abs(G[:2]).max())
    log(f"  FD rel err {e:.2e}")
    assert e < 1e-6


def test_fp32_variant_error_is_bounded():
    log("[tau] fp32 variant on config2")
    s = synth.config2()
    o = oracle.Oracle(s)
    D = synth.make_density(s)
    V = synth.make_potentials(o.meshes, s.seed)
    t_o, M_o, g_o = o.tau_density(D), o.mat_tau(V), o.grad_tau(D, V)
    t_g, M_g, g_g, _ = gpu_tau_all(s, D, V, precision="fp32")
    errs = [rel_err(a, b) for a, b in zip(t_g, t_o)] + [rel_err(M_g, M_o), rel_err(g_g, g_o)]
    log(f"  fp32 rel errs {['%.1e' % e for e in errs]}")
    assert max(errs) < 1e-4


def test_batch_matches_single_calls():
    """tau / mat_tau / grad_tau tasks of two plans in one gpw_eval_batch, next
    to density tasks, give the single calls' results."""
    import torch
    from paper_2603_24881_amd import _lib
    from paper_2603_24881_amd.gpw import GPW
    log("[tau] batch")
    s1, s2 = synth.config1(), tiny.tiny_system(mesh=((18, 21, 23),), tau=1e-10)
    tasks, refs = [], []
    plans = []
    for s, seed in ((s1, 3), (s2, 4)):
        g = GPW(s)
        plans.append(g)
        D = to_dev(tiny.random_density(s.n_ao, seed=seed))
        V = [to_dev(v) for v in synth.make_potentials(g.meshes, seed)]
        t_out = g.new_grids()
        r_out = g.new_grids()
        M = torch.empty((g.n_ao, g.n_ao), dtype=torch.float64, device=D.device)
        G = torch.empty((g.natm, 3), dtype=torch.float64, device=D.device)
        tasks += [dict(plan=g.plan, op=_lib.GPW_OP_TAU, D=D, rho=t_out),
                  dict(plan=g.plan, op=_lib.GPW_OP_RHO, D=D, rho=r_out),
                  dict(plan=g.plan, op=_lib.GPW_OP_MAT_TAU, v=V, out=M),
                  dict(plan=g.plan, op=_lib.GPW_OP_GRAD_TAU, D=D, v=V, out=G)]
        refs.append((g.tau(D), g.rho(D), g.mat_tau(V), g.grad_tau(D, V), t_out, r_out, M, G))
    _lib.gpw_eval_batch(tasks)
    torch.cuda.synchronize()
    for (t_ref, r_ref, M_ref, G_ref, t_out, r_out, M, G) in refs:
        for a, b in zip(t_out, t_ref):
            assert torch.equal(a, b)
        for a, b in zip(r_out, r_ref):
            assert torch.equal(a, b)
        assert rel_err(to_np(M), to_np(M_ref)) < 1e-13
        assert rel_err(to_np(G), to_np(G_ref)) < 1e-13
    for g in plans:
        g.close()


def test_water256_sampled_parity():
    """The 256-water system in the benchmark's launch configuration: the whole
    tau on every level, M_tau and grad_tau on the GPU; 64 sampled points per
    level, 8 shell-pair blocks of M_tau and 2 complete gradient rows from the
    oracle."""
    import torch
    from paper_2603_24881_amd.gpw import GPW
    s = synth.water256()
    log(f"[tau] water256: {s.natm} atoms, {s.n_ao} AOs")
    g = GPW(s)
    dev = torch.device("cuda", 0)
    C = torch.as_tensor(synth.draw_orbitals(s), device=dev)
    D = (C @ C.T).contiguous()
    del C
    V_np = synth.make_potentials(g.meshes, s.seed + 1)
    V = [to_dev(v) for v in V_np]
    t = g.tau(D)
    M = g.mat_tau(V)
    G = g.grad_tau(D, V)
    torch.cuda.synchronize()
    Dn = D.cpu().numpy()
    rng = np.random.default_rng(20261)
    o = oracle.Oracle(s)
    for l, m in enumerate(o.meshes):
        idx = rng.choice(m[0] * m[1] * m[2], 64, replace=False)
        ref = o.tau_points(Dn, l, idx)
        got = to_np(t[l]).reshape(-1)[idx]
        scale = float(t[l].abs().max())
        if scale == 0.0:
            assert float(np.abs(ref).max()) == 0.0
            continue
        e = float(np.abs(got - ref).max()) / scale
        log(f"  tau level {l}: 64 points, rel err {e:.2e}")
        assert e < TOL, (l, e)
    ls = np.asarray(s.shell_l)
    f_sh = np.flatnonzero(ls == 3)
    d_sh = np.flatnonzero(ls == 2)
    p_sh = np.flatnonzero(ls == 1)
    pairs = [(int(f_sh[0]), int(f_sh[0])), (int(f_sh[1]), int(d_sh[0])), (int(d_sh[3]), int(p_sh[2])),
             (int(p_sh[5]), int(p_sh[5]))]
    pairs += [tuple(int(x) for x in rng.choice(s.nshell, 2, replace=False)) for _ in range(4)]
    off = s.ao_offsets()
    blocks = o.mat_tau_blocks(V_np, pairs)
    Mn = to_np(M)
    scale = float(np.abs(Mn).max())
    for (a, b), ref in zip(pairs, blocks):
        got = Mn[off[a]:off[a + 1], off[b]:off[b + 1]]
        e = float(np.abs(got - ref).max()) / scale
        assert e < TOL, ((a, b), e)
    log(f"  M_tau: {len(pairs)} blocks within {TOL}")
    atoms = [int(x) for x in rng.choice(s.natm, 2, replace=False)]
    mask = np.zeros(s.natm, dtype=np.uint8)
    mask[atoms] = 1
    og = oracle.Oracle(s, atom_mask=mask, mask_either=True).grad_tau(Dn, V_np)
    Gn = to_np(G)
    e = float(np.abs(Gn[atoms] - og[atoms]).max()) / float(np.abs(Gn).max())
    log(f"  grad_tau rows {atoms}: rel err {e:.2e}")
    assert e < TOL
    g.close()
