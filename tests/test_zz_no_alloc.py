"""The allocation-free integration entry point (gpw_eval_mat_noalloc) through the
C ABI: on two calls in a row, the second on a smaller system, its M equals that
of gpw_eval_mat within the FP64 tolerance of 1e-10 relative (the two run the
same kernels and differ only in the order of their atomic additions); it takes
nothing from the stream-ordered pool the allocating call uses; and a plan whose
scratch exceeds the fixed array is rejected with GPW_EBUDGET before anything
runs."""
from __future__ import annotations

import ctypes as C

import numpy as np
import pytest

from gpu_helpers import log, rel_err, to_dev, to_np

pytestmark = pytest.mark.gpu

TOL = 1e-10
HIP_POOL_USED_CURRENT = 0x7   # hipMemPoolAttrUsedMemCurrent
HIP_POOL_USED_HIGH = 0x8      # hipMemPoolAttrUsedMemHigh


class _Pool:
    """Peak use of device 0's default stream-ordered pool (where the library's
    allocating calls take their scratch), read through the HIP runtime."""

    def __init__(self):
        self.hip = C.CDLL("libamdhip64.so")
        self.pool = C.c_void_p()
        assert self.hip.hipDeviceGetDefaultMemPool(C.byref(self.pool), 0) == 0

    def _get(self, attr):
        v = C.c_uint64(0)
        assert self.hip.hipMemPoolGetAttribute(self.pool, attr, C.byref(v)) == 0
        return int(v.value)

    def reset_peak(self) -> bool:
        v = C.c_uint64(0)
        return self.hip.hipMemPoolSetAttribute(self.pool, HIP_POOL_USED_HIGH, C.byref(v)) == 0

    def peak_above_current(self):
        return self._get(HIP_POOL_USED_HIGH) - self._get(HIP_POOL_USED_CURRENT)


def _systems():
    from paper_2603_24881_amd import synth
    # the first call on a 32-water multigrid system, the second on the 4-atom
    # single-grid one: a smaller input into the same scratch array
    return [("32 waters, 4 levels", synth.config2()), ("4 atoms, 24^3", synth.config1())]


def test_noalloc_matches_the_allocating_call_on_two_calls_in_a_row():
    import torch
    from paper_2603_24881_amd import _lib, synth
    from paper_2603_24881_amd.gpw import GPW
    pool = _Pool()
    prev_scratch = None
    for name, s in _systems():
        log(f"[noalloc] {name}")
        g = GPW(s)
        need = int(g.info["scratch_bytes"][_lib.GPW_OP_MAT])
        assert need <= _lib.GPW_NOALLOC_SCRATCH_BYTES
        if prev_scratch is not None:
            assert need < prev_scratch        # the second input is the smaller one
        prev_scratch = need
        V = [to_dev(v) for v in synth.make_potentials(g.meshes, s.seed)]
        ref = torch.empty((g.n_ao, g.n_ao), dtype=torch.float64, device=V[0].device)
        out = torch.full_like(ref, float("nan"))   # every element must be written
        torch.cuda.synchronize()
        # the allocating call takes its scratch from the pool (the control) ...
        tracked = pool.reset_peak()
        _lib.gpw_eval_mat(g.plan, V, ref)
        torch.cuda.synchronize()
        ctl = pool.peak_above_current() if tracked else None
        # ... the allocation-free call takes nothing
        tracked = tracked and pool.reset_peak()
        _lib.gpw_eval_mat_noalloc(g.plan, V, out)
        torch.cuda.synchronize()
        peak = pool.peak_above_current() if tracked else None
        log(f"  pool peak above current: allocating call {ctl}, allocation-free call {peak}")
        if ctl is not None and ctl >= need:
            assert peak == 0
        e = rel_err(to_np(out), to_np(ref))
        log(f"  M rel err vs gpw_eval_mat {e:.2e}")
        assert np.isfinite(to_np(out)).all()
        assert e < TOL
        g.close()


def test_scratch_beyond_the_fixed_array_is_rejected():
    import torch
    from paper_2603_24881_amd import _lib
    # one tight s function on a fine 256^3 mesh: its block-ordered potential
    # copy (64 x 64 x 84 blocks of 512 bytes) exceeds 128 MiB
    log("[noalloc] oversize plan")
    p = _lib.gpw_plan(np.diag([8.0, 8.0, 8.0]), np.array([[4.0, 4.0, 4.0]]), [0], [0], [1], [0], [4.0],
                      [1.0], mesh=[[256, 256, 256]], tau=1e-6)
    need = int(p.info["scratch_bytes"][_lib.GPW_OP_MAT])
    assert need > _lib.GPW_NOALLOC_SCRATCH_BYTES, need
    v = [torch.zeros(256 ** 3, dtype=torch.float64, device="cuda:0")]
    M = torch.zeros((1, 1), dtype=torch.float64, device="cuda:0")
    with pytest.raises(_lib.GPWError) as ei:
        _lib.gpw_eval_mat_noalloc(p, v, M)
    assert ei.value.status == 5
    assert "scratch" in _lib.gpw_last_error()
    p.close()


def test_noalloc_on_a_general_cell():
    """The same entry point on a triclinic cell (the index-coordinate kernels)."""
    import torch
    import tiny
    from paper_2603_24881_amd import _lib, synth
    from paper_2603_24881_amd.gpw import GPW
    log("[noalloc] triclinic cell")
    cell = np.array([[7.0, 0.0, 0.0], [1.9, 7.6, 0.0], [-1.2, 1.4, 8.2]])
    s = tiny.tiny_system(cell=cell, mesh=((18, 21, 23),), tau=1e-10)
    g = GPW(s)
    V = [to_dev(v) for v in synth.make_potentials(g.meshes, 7)]
    ref = torch.empty((g.n_ao, g.n_ao), dtype=torch.float64, device=V[0].device)
    out = torch.full_like(ref, float("nan"))
    _lib.gpw_eval_mat(g.plan, V, ref)
    _lib.gpw_eval_mat_noalloc(g.plan, V, out)
    torch.cuda.synchronize()
    e = rel_err(to_np(out), to_np(ref))
    log(f"  M rel diff {e:.2e}")
    assert not bool(torch.isnan(out).any()) and e < TOL
    g.close()
