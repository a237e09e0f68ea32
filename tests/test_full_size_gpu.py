"""Parity at the full 256-water size, in the launch configuration the
benchmark times (single eval_rho / eval_mat / eval_grad calls of the FP64
plan): the whole outputs on the GPU, sampled outputs from the oracle
(64 random points per level, 24 shell-pair blocks of M: f and d shells,
shells of one water unit and random pairs; the complete gradient rows of 3
atoms).  Tolerance 1e-10 relative
to the largest magnitude of the GPU array (per level for rho)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from gpu_helpers import log, rel_err, to_dev, to_np
from paper_2603_24881_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-10


def test_water256_sampled_parity():
    import torch
    from paper_2603_24881_amd.gpw import GPW
    s = synth.water256()
    log(f"water256: {s.natm} atoms, {s.n_ao} AOs")
    g = GPW(s)
    dev = torch.device("cuda", 0)
    C = torch.as_tensor(synth.draw_orbitals(s), device=dev)
    D = (C @ C.T).contiguous()
    del C
    V_np = synth.make_potentials(g.meshes, s.seed)
    V = [to_dev(v) for v in V_np]
    rho = g.rho(D)
    M = g.mat(V)
    G = g.grad(D, V)
    torch.cuda.synchronize()
    Dn = D.cpu().numpy()
    o = oracle.Oracle(s)
    assert [tuple(m) for m in g.meshes] == o.meshes
    rng = np.random.default_rng(20260)
    for l, m in enumerate(o.meshes):
        idx = rng.choice(m[0] * m[1] * m[2], 64, replace=False)
        ref = o.rho_points(Dn, l, idx)
        got = to_np(rho[l]).reshape(-1)[idx]
        scale = float(rho[l].abs().max())
        if scale == 0.0:   # an empty level (no pair image has its exponent range)
            log(f"  rho level {l}: empty; oracle samples max {np.abs(ref).max():.1e}")
            assert float(np.abs(ref).max()) == 0.0 and g.info["n_pairs"][l] == 0
            continue
        e = float(np.abs(got - ref).max()) / scale
        log(f"  rho level {l}: 64 points, max |ref| {np.abs(ref).max():.3e}, rel err {e:.2e}")
        assert e < TOL, (l, e)
    off = s.ao_offsets()
    ls = np.asarray(s.shell_l)
    f_sh = np.flatnonzero(ls == 3)
    d_sh = np.flatnonzero(ls == 2)
    pairs = [(int(f_sh[0]), int(f_sh[0])), (int(f_sh[1]), int(d_sh[0])), (int(d_sh[3]), int(d_sh[3]))]
    sh_atom = np.asarray(s.shell_atom)
    for k in rng.choice(s.natm // 3, 12, replace=False):   # shells of one water unit
        own = np.flatnonzero((sh_atom >= 3 * k) & (sh_atom < 3 * k + 3))
        a, b = rng.choice(own, 2, replace=True)
        pairs.append((int(a), int(b)))
    pairs += [tuple(int(x) for x in rng.choice(s.nshell, 2, replace=False)) for _ in range(9)]
    blocks = o.mat_blocks(V_np, pairs)
    Mn = to_np(M)
    scale = float(np.abs(Mn).max())
    e = 0.0
    nz = 0
    for (a, b), blk in zip(pairs, blocks):
        got = Mn[off[a]:off[a + 1], off[b]:off[b + 1]]
        e = max(e, float(np.abs(got - blk).max()) / scale)
        nz += int(np.abs(blk).max() > 0)
    log(f"  M: {len(pairs)} shell-pair blocks ({nz} nonzero), rel err {e:.2e}")
    assert e < TOL and nz >= 14
    atoms = [0, 301, 767]
    mask = np.zeros(s.natm, dtype=np.uint8)
    mask[atoms] = 1
    gref = oracle.Oracle(s, atom_mask=mask, mask_either=True).grad(Dn, V_np)[atoms]
    Gn = to_np(G)
    e = float(np.abs(Gn[atoms] - gref).max()) / float(np.abs(Gn).max())
    log(f"  grad rows of atoms {atoms}: rel err {e:.2e}")
    assert e < TOL
    g.close()


def test_everything_screened_out_gives_zeros():
    """Coefficients so small that every pair's maximum is below the threshold:
    no pair image survives, the outputs are exactly zero and the calls still
    succeed."""
    import torch
    from paper_2603_24881_amd.gpw import GPW
    s = synth.config1()
    s.coefs = np.asarray(s.coefs) * 1e-30
    g = GPW(s)
    assert sum(g.info["n_pairs"]) == 0
    assert [tuple(m) for m in g.meshes] == oracle.Oracle(s).meshes
    D = to_dev(synth.make_density(s))
    V = [to_dev(v) for v in synth.make_potentials(g.meshes, s.seed)]
    rho = g.rho(D)
    M = g.mat(V)
    G = g.grad(D, V)
    torch.cuda.synchronize()
    assert float(rho[0].abs().max()) == 0.0 and float(M.abs().max()) == 0.0 and float(G.abs().max()) == 0.0
    g.close()


def _diffuse_system(name, L, mesh, exps, ls, tau):
    n = len(ls)
    return synth.System(name=name, cell=np.array([L, L, L]), coords=np.array([[0.45 * L, 0.5 * L, 0.55 * L]]),
                        shell_atom=np.zeros(n, dtype=np.int32), shell_l=np.array(ls, dtype=np.int32),
                        shell_nprim=np.ones(n, dtype=np.int32), shell_prim0=np.arange(n, dtype=np.int32),
                        exps=np.array(exps), coefs=np.ones(n), ke_cutoff_ry=[],
                        mesh=np.array([mesh], dtype=np.int32), tau=tau, n_occ=1)


@pytest.mark.parametrize("case", ["sliced", "very_wide"])
def test_wide_spheres_are_traversed_in_slices(case):
    """Diffuse functions on fine single meshes: the pair boxes hold more block
    rows than the LDS does, so the pair-major kernels walk them in slices of
    x entries.  rho, the matrix and the gradient against the oracle."""
    import torch
    from paper_2603_24881_amd.gpw import GPW
    if case == "sliced":      # about 38 blocks per axis, 3 slices
        s = _diffuse_system("sliced", 20.0, (128, 128, 128), [0.05, 0.07], [0, 1], 1e-6)
    else:                     # about 112 blocks per axis, 13 slices
        s = _diffuse_system("very_wide", 40.0, (480, 480, 480), [0.02], [0], 1e-6)
    g = GPW(s)
    emax = (g.info["max_box_width"] + 3) // 4
    log(f"  {case}: max box width {g.info['max_box_width']} points")
    assert emax * emax > 1024
    o = oracle.Oracle(s)
    D = synth.make_density(s)
    V = synth.make_potentials(o.meshes, 5)
    rho = g.rho(to_dev(D))
    M = g.mat([to_dev(v) for v in V])
    G = g.grad(to_dev(D), [to_dev(v) for v in V])
    torch.cuda.synchronize()
    e = rel_err(to_np(rho[0]), o.rho(D)[0])
    log(f"  rho rel err {e:.2e}")
    assert e < 1e-10
    e = rel_err(to_np(M), o.mat(V))
    log(f"  M rel err {e:.2e}")
    assert e < 1e-10
    go = o.grad(D, V)
    e = float(np.abs(to_np(G) - go).max() / max(np.abs(go).max(), 1e-300))
    log(f"  grad rel err {e:.2e} (max |ref| {np.abs(go).max():.2e})")
    assert e < 1e-10 or np.abs(to_np(G) - go).max() < 1e-12
    g.close()
