"""GPWCollocate (torch.autograd.Function): its backward equals the library's
eval_mat / eval_grad, and the centre gradient matches central finite
differences (h = 1e-4 bohr) and the oracle on 8 random atoms of the 64-water
gradient configuration at tau = 1e-14; the Hartree-energy gradient through
the Poisson harness matches finite differences as well."""
from __future__ import annotations

import copy

import numpy as np
import pytest

import oracle
from gpu_helpers import log, rel_err, to_dev, to_np
from paper_2603_24881_amd import synth

pytestmark = pytest.mark.gpu


def _energy(system, D, V, tau=None):
    """sum_l w_l <v_l, rho_l(D; R)> through eval_rho."""
    import torch
    from paper_2603_24881_amd.gpw import GPW
    g = GPW(system, tau=tau)
    rho = g.rho(D)
    e = sum(w * float(torch.dot(r.reshape(-1), v.reshape(-1))) for w, r, v in zip(g.weights, rho, V))
    g.close()
    return e


def _displaced(system, a, d, h):
    s = copy.deepcopy(system)
    s.coords = np.array(system.coords, dtype=np.float64)
    s.coords[a, d] += h
    return s


def test_backward_equals_library_kernels():
    import torch
    from paper_2603_24881_amd.autograd import collocate
    from paper_2603_24881_amd.gpw import GPW
    s = synth.config2()
    g = GPW(s)
    D = to_dev(synth.make_density(s)).requires_grad_(True)
    R = torch.tensor(s.coords, dtype=torch.float64, requires_grad=True)
    V = [to_dev(v) for v in synth.make_potentials(g.meshes, s.seed)]
    rho = collocate(g, D, R)
    loss = sum(w * (r * v).sum() for w, r, v in zip(g.weights, rho, V))
    loss.backward()
    M = to_np(g.mat(V))
    G = to_np(g.grad(D.detach(), V))
    e_d, e_r = rel_err(to_np(D.grad), M), rel_err(R.grad.numpy(), G)
    log(f"  dL/dD vs eval_mat {e_d:.2e}, dL/dR vs eval_grad {e_r:.2e}")
    assert e_d < 1e-12 and e_r < 1e-12
    with pytest.raises(ValueError):
        collocate(g, D, R.detach() + 0.1)
    g.close()


def test_config3_gradient_fd_and_oracle():
    """dE/dR of E = sum_l w_l <v_l, rho_l(D; R)> at fixed D, v: kernel vs
    central differences and vs the oracle restricted to the 8 atoms."""
    import torch
    from paper_2603_24881_amd.autograd import collocate
    from paper_2603_24881_amd.gpw import GPW
    tau, h = 1e-14, 1e-4
    s = synth.config3(tau=tau)
    atoms = np.random.default_rng(s.seed + 3).choice(s.natm, 8, replace=False)
    log(f"  atoms {atoms.tolist()}")
    g = GPW(s)
    Dn = synth.make_density(s)
    D = to_dev(Dn)
    Vn = synth.make_potentials(g.meshes, s.seed)
    V = [to_dev(v) for v in Vn]
    R = torch.tensor(s.coords, dtype=torch.float64, requires_grad=True)
    rho = collocate(g, D, R)
    E = sum(w * (r * v).sum() for w, r, v in zip(g.weights, rho, V))
    E.backward()
    an = R.grad.numpy()[atoms]
    g.close()
    fd = np.zeros((8, 3))
    for i, a in enumerate(atoms):
        for d in range(3):
            ep = _energy(_displaced(s, a, d, +h), D, V)
            em = _energy(_displaced(s, a, d, -h), D, V)
            fd[i, d] = (ep - em) / (2 * h)
    e_fd = float(np.abs(fd - an).max() / np.abs(an).max())
    log(f"  FD vs kernel: max rel {e_fd:.2e} (max |g| {np.abs(an).max():.3e})")
    assert e_fd < 1e-6
    mask = np.zeros(s.natm, dtype=np.uint8)
    mask[atoms] = 1
    go = oracle.Oracle(s, atom_mask=mask, mask_either=True).grad(Dn, Vn)[atoms]
    e_o = rel_err(an, go)
    log(f"  kernel vs oracle on the 8 atoms: {e_o:.2e}")
    assert e_o < 1e-10


def test_hartree_gradient_through_poisson():
    """E_J(R) = Poisson energy of rho(D; R): the autograd gradient (eval_grad
    with v = v_H) against central differences."""
    import torch
    from paper_2603_24881_amd.autograd import collocate
    from paper_2603_24881_amd.gpw import GPW
    s = synth.config1(tau=1e-14)
    D = to_dev(synth.make_density(s))

    def ej(system):
        g = GPW(system)
        e = float(g.poisson().energy(list(g.rho(D))))
        g.close()
        return e

    g = GPW(s)
    R = torch.tensor(s.coords, dtype=torch.float64, requires_grad=True)
    E = g.poisson().energy(list(collocate(g, D, R)))
    E.backward()
    an = R.grad.numpy()
    h = 1e-4
    fd = np.zeros_like(an)
    for a in range(s.natm):
        for d in range(3):
            fd[a, d] = (ej(_displaced(s, a, d, h)) - ej(_displaced(s, a, d, -h))) / (2 * h)
    e = float(np.abs(fd - an).max() / np.abs(an).max())
    log(f"  E_J = {float(E.detach()):.10f}; dE_J/dR FD vs autograd {e:.2e}")
    assert e < 1e-6
    g.close()
