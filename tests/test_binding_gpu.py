"""The binding rejects buffers that do not match the plan before any call into
the library (sizes, level counts, device), and the plan reports the scratch
each operation takes (GPU: plans are built on the device)."""
from __future__ import annotations

import numpy as np
import pytest

from gpu_helpers import log, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def plan():
    from paper_2603_24881_amd import synth
    from paper_2603_24881_amd.gpw import GPW
    log("[binding] config 1 plan")
    g = GPW(synth.config1())
    yield g
    g.close()


def test_wrong_buffers_raise_before_the_library(plan):
    import torch
    from paper_2603_24881_amd import _lib
    n = plan.n_ao
    D = to_dev(np.eye(n))
    rho = plan.new_grids()
    M = torch.zeros((n, n), dtype=torch.float64, device=D.device)
    with pytest.raises(ValueError):
        _lib.gpw_eval_rho(plan.plan, to_dev(np.eye(n + 1)), rho)          # D too large
    with pytest.raises(ValueError):
        _lib.gpw_eval_rho(plan.plan, D, rho + rho)                         # too many levels
    with pytest.raises(ValueError):
        _lib.gpw_eval_rho(plan.plan, D, [rho[0][:-1].contiguous()])         # grid too small
    with pytest.raises(ValueError):
        _lib.gpw_eval_mat(plan.plan, rho, M[:-1].contiguous())              # M too small
    with pytest.raises(ValueError):
        _lib.gpw_eval_grad(plan.plan, D, rho, torch.zeros(plan.natm * 3 + 1, dtype=torch.float64,
                                                          device=D.device))
    with pytest.raises(ValueError):
        _lib.gpw_eval_batch([dict(plan=plan.plan, op=_lib.GPW_OP_MAT, v=rho[:0], out=M)])
    with pytest.raises(TypeError):
        _lib.gpw_eval_rho(plan.plan, D.float(), rho)
    # the right buffers still work
    _lib.gpw_eval_rho(plan.plan, D, rho)
    torch.cuda.synchronize()
    assert torch.isfinite(rho[0]).all()


def test_scratch_bytes_reported(plan):
    scr = plan.info["scratch_bytes"]
    assert len(scr) == 6 and all(int(x) > 0 for x in scr)
    # the gradient also holds the symmetrised D next to the block-ordered potential
    assert scr[2] >= scr[1] + 8 * plan.n_ao ** 2
    # the meta-GGA terms: larger coefficient tensors than the density's; the same
    # block-ordered potential (and symmetrised D) as integration and gradient
    assert scr[3] > scr[0] and scr[4] == scr[1] and scr[5] == scr[2]
