"""gpw_poisson (hipFFT half spectra and the library's transfer kernels) against
the Poisson oracle (numpy full spectra), through the C ABI: every level's
potential to 1e-10 relative to its largest magnitude and E_J to 1e-12
relative; plus the energy identity and repeatability on the GPU alone."""
from __future__ import annotations

import math

import numpy as np
import pytest

import tiny
from gpu_helpers import log, rel_err, to_dev, to_np
from oracle import poisson as opoisson
from paper_2603_24881_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _gpu(s, rho):
    import torch
    from paper_2603_24881_amd.gpw import GPW
    g = GPW(s)
    v, ej = g.poisson().solve_async([to_dev(r) for r in rho])
    torch.cuda.synchronize()
    out = [to_np(x) for x in v], float(ej.item()), g.info
    g.close()
    return out


def _compare(s, rho, cut):
    from paper_2603_24881_amd.gpw import GPW
    v_g, e_g, info = _gpu(s, rho)
    meshes = [tuple(m) for m in info["mesh"]]
    v_o, e_o = opoisson.poisson(s.cell, meshes, cut, rho)
    for l, (a, b) in enumerate(zip(v_g, v_o)):
        e = rel_err(a, b)
        log(f"  v level {l} {meshes[l]}: rel err {e:.2e}")
        assert e < TOL, (l, e)
    log(f"  E_J {e_g:.12e} vs {e_o:.12e}")
    assert abs(e_g - e_o) < 1e-12 * abs(e_o)
    return v_g, e_g, info


def test_plane_wave_single_level_without_cutoff():
    """A mesh-defined single level keeps every non-Nyquist plane wave; the
    potential of cos(G.r) is 4 pi / |G|^2 cos(G.r)."""
    log("[poisson] plane wave, single level")
    s = tiny.tiny_system(shell_ls=(0,), natm=1, mesh=((16, 18, 20),))
    L = s.cell
    ax = [np.arange(n) * (L[d] / n) for d, n in enumerate((16, 18, 20))]
    x, y, z = np.meshgrid(*ax, indexing="ij")
    g = [2 * math.pi * m / L[d] for d, m in enumerate((1, 2, -3))]
    rho = np.cos(g[0] * x + g[1] * y + g[2] * z) + np.cos(2 * math.pi * 8 * x / L[0])   # + a Nyquist wave
    v, e, _ = _compare(s, [rho], None)
    g2 = sum(t * t for t in g)
    np.testing.assert_allclose(v[0], 4 * math.pi / g2 * np.cos(g[0] * x + g[1] * y + g[2] * z), atol=1e-11)


@pytest.mark.parametrize("name", ["config2", "config4"])
def test_multigrid_levels_match_the_oracle(name):
    """Random level data on the 4-level water and 5-level diamond meshes
    (odd and even meshes, levels of every size)."""
    log(f"[poisson] {name}")
    s = getattr(synth, name)()
    rng = np.random.default_rng(31)
    from paper_2603_24881_amd.gpw import GPW
    g = GPW(s)
    meshes = [tuple(m) for m in g.meshes]
    g.close()
    rho = [rng.standard_normal(m) for m in meshes]
    _compare(s, rho, s.ke_cutoff_ry)


def test_collocated_density_and_energy_identity():
    """The Poisson step of a collocated density (config 2): parity with the
    oracle, and E_J = 1/2 sum_l w_l <v_l, rho_l> on the GPU alone."""
    import torch
    from paper_2603_24881_amd.gpw import GPW
    log("[poisson] collocated density")
    s = synth.config2()
    g = GPW(s)
    rho = g.rho(to_dev(synth.make_density(s)))
    v, ej = g.poisson().solve_async(rho)
    torch.cuda.synchronize()
    half = 0.5 * sum(w * float(torch.vdot(a.reshape(-1), b.reshape(-1))) for w, a, b in zip(g.weights, v, rho))
    e = float(ej.item())
    log(f"  E_J {e:.12e}, 1/2 sum w <v, rho> {half:.12e}")
    assert abs(e - half) < 1e-12 * abs(e) and e > 0
    v_o, e_o = opoisson.poisson(s.cell, [tuple(m) for m in g.meshes], s.ke_cutoff_ry, [to_np(r) for r in rho])
    assert abs(e - e_o) < 1e-12 * abs(e_o)
    for a, b in zip(v, v_o):
        assert rel_err(to_np(a), b) < TOL
    # repeated calls give the same bits (deterministic reductions)
    v2, ej2 = g.poisson().solve_async(rho)
    torch.cuda.synchronize()
    assert float(ej2.item()) == e and all(torch.equal(a, b) for a, b in zip(v, v2))
    g.close()


def test_water256_full_size():
    """The 256-water meshes (192^3 finest), random level data."""
    log("[poisson] water256")
    s = synth.water256()
    from paper_2603_24881_amd.gpw import GPW
    g = GPW(s)
    meshes = [tuple(m) for m in g.meshes]
    g.close()
    rng = np.random.default_rng(32)
    rho = [rng.standard_normal(m) for m in meshes]
    _compare(s, rho, s.ke_cutoff_ry)


@pytest.mark.parametrize("name", ["config2", "water256"])
def test_fine_density_gradient_and_hxc_match_the_oracle(name):
    """gpw_fine_density (rho and grad rho on the finest mesh) and
    gpw_hxc_potential with random fine-grid vxc and GGA vector potential,
    against the oracle on random level data."""
    import torch
    from paper_2603_24881_amd.gpw import GPW
    log(f"[poisson] fine density and Hxc, {name}")
    s = synth.water256() if name == "water256" else getattr(synth, name)()
    g = GPW(s)
    meshes = [tuple(m) for m in g.meshes]
    rng = np.random.default_rng(33)
    rho = [rng.standard_normal(m) for m in meshes]
    vxc = rng.standard_normal(meshes[0])
    vg = [rng.standard_normal(meshes[0]) for _ in range(3)]
    p = g.poisson()
    rd = [to_dev(r) for r in rho]
    rf, grad = p.fine_density(rd)
    v, ej = p.hxc(rd, vxc=to_dev(vxc), vxc_grad=[to_dev(x) for x in vg])
    torch.cuda.synchronize()
    rf_o, grad_o = opoisson.fine_density(s.cell, meshes, s.ke_cutoff_ry, rho)
    e = rel_err(to_np(rf), rf_o)
    log(f"  fine rho rel err {e:.2e}")
    assert e < TOL
    for d in range(3):
        e = rel_err(to_np(grad[d]), grad_o[d])
        log(f"  grad rho [{d}] rel err {e:.2e}")
        assert e < TOL
    v_o, e_o = opoisson.hxc_potential(s.cell, meshes, s.ke_cutoff_ry, rho, vxc=vxc, vxc_grad=vg)
    for l, (a, b) in enumerate(zip(v, v_o)):
        e = rel_err(to_np(a), b)
        log(f"  v_Hxc level {l}: rel err {e:.2e}")
        assert e < TOL
    assert abs(float(ej.item()) - e_o) < 1e-12 * abs(e_o)
    g.close()
