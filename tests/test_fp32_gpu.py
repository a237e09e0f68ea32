"""FP32 variant on the diamond configuration (216 C, 5 levels): errors of
E_J, the Coulomb matrix J = V_{mu nu}(v_H) and the gradient dE_J/dR against
the FP64 oracle, next to those of the FP64 kernels.  The Hartree potential
of each side comes from the multigrid Poisson step applied to that side's
density (the library's gpw_poisson for the GPU, the Poisson oracle for the
oracle)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from gpu_helpers import log, rel_err, to_dev, to_np
from paper_2603_24881_amd import synth

pytestmark = pytest.mark.gpu


def _gpu_pipeline(s, D, precision):
    import torch
    from paper_2603_24881_amd.gpw import GPW
    g = GPW(s, precision=precision)
    p = g.poisson()
    Dd = to_dev(D)
    v, e = p.solve(g.rho(Dd))
    J = to_np(g.mat(v))
    F = to_np(g.grad(Dd, v))
    torch.cuda.synchronize()
    g.close()
    return e, J, F


def test_fp32_errors_on_diamond():
    from oracle import poisson as opoisson
    s = synth.config4()
    D = synth.make_density(s)
    o = oracle.Oracle(s)
    vn, e_o = opoisson.poisson(s.cell, o.meshes, s.ke_cutoff_ry, o.rho(D))
    J_o, F_o = o.mat(vn), o.grad(D, vn)
    rep = {}
    for prec in ("fp64", "fp32"):
        e, J, F = _gpu_pipeline(s, D, prec)
        rep[prec] = dict(E_J_abs=abs(e - e_o), E_J_rel=abs(e - e_o) / abs(e_o),
                         J_max_abs=float(np.abs(J - J_o).max()), J_rel=rel_err(J, J_o),
                         F_max_abs=float(np.abs(F - F_o).max()), F_rel=rel_err(F, F_o))
        log(f"  {prec} vs oracle: " + ", ".join(f"{k} {val:.2e}" for k, val in rep[prec].items()))
    log(f"  E_J (oracle) = {e_o:.10f}")
    assert rep["fp64"]["E_J_rel"] < 1e-10 and rep["fp64"]["J_rel"] < 1e-10 and rep["fp64"]["F_rel"] < 1e-10
    assert rep["fp32"]["E_J_rel"] < 1e-5 and rep["fp32"]["J_rel"] < 1e-4 and rep["fp32"]["F_rel"] < 1e-4
