"""gpw_eval_batch: tasks of several plans (sizes, classes, precisions,
orthorhombic and general cells) in one batched set of launches give the same
results as the single calls, and the single calls still match the oracle."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import tiny
from gpu_helpers import log, rel_err, to_dev, to_np
from paper_2603_24881_amd import _lib, synth

pytestmark = pytest.mark.gpu

SKEW = np.array([[7.0, 0.0, 0.0], [1.9, 7.6, 0.0], [-1.2, 1.4, 8.2]])


def _systems():
    return [("config1", synth.config1(), "fp64"),
            ("tiny-spdf", tiny.tiny_system(mesh=((18, 21, 23),), tau=1e-10), "fp64"),
            ("config2", synth.config2(), "fp64"),
            ("tiny-spdf-fp32", tiny.tiny_system(mesh=((20, 24, 28),), tau=1e-10), "fp32"),
            # general cells: their segments take the index-coordinate kernels in the same launches
            ("tiny-skew", tiny.tiny_system(cell=SKEW, mesh=((18, 21, 23),), tau=1e-10), "fp64"),
            ("tiny-skew-fp32", tiny.tiny_system(cell=SKEW, mesh=((16, 18, 20),), tau=1e-10, seed=9), "fp32")]


def test_batch_matches_single_calls():
    import torch
    from paper_2603_24881_amd.gpw import GPW
    items = []
    for name, s, prec in _systems():
        g = GPW(s, precision=prec)
        D = to_dev(synth.make_density(s))
        V = [to_dev(v) for v in synth.make_potentials(g.meshes, s.seed)]
        items.append((name, s, g, D, V))
    # single calls
    single = []
    for name, s, g, D, V in items:
        single.append(([to_np(r) for r in g.rho(D)], to_np(g.mat(V)), to_np(g.grad(D, V))))
    torch.cuda.synchronize()
    # one batch with every task of every plan, in a mixed order
    tasks, outs = [], []
    for name, s, g, D, V in items:
        rho = [torch.full(tuple(m), np.nan, dtype=torch.float64, device=D.device) for m in g.meshes]
        M = torch.full((g.n_ao, g.n_ao), np.nan, dtype=torch.float64, device=D.device)
        G = torch.full((g.natm, 3), np.nan, dtype=torch.float64, device=D.device)
        outs.append((rho, M, G))
        tasks += [dict(plan=g.plan, op=_lib.GPW_OP_GRAD, D=D, v=V, out=G),
                  dict(plan=g.plan, op=_lib.GPW_OP_RHO, D=D, rho=rho),
                  dict(plan=g.plan, op=_lib.GPW_OP_MAT, v=V, out=M)]
    _lib.gpw_eval_batch(tasks[::-1])
    torch.cuda.synchronize()
    for (name, s, g, D, V), (rho1, M1, G1), (rho, M, G) in zip(items, single, outs):
        for l, (a, b) in enumerate(zip(rho, rho1)):
            a = to_np(a)
            log(f"  {name} rho[{l}] batch vs single: max abs diff {np.abs(a - b).max():.2e}")
            assert np.array_equal(a, b), (name, l)
        e_m, e_g = rel_err(to_np(M), M1), rel_err(to_np(G), G1)
        log(f"  {name} M rel diff {e_m:.2e}, grad rel diff {e_g:.2e}")
        assert e_m < 1e-12 and e_g < 1e-12, name
    # the batch result of config1 against the oracle
    name, s, g, D, V = items[0]
    o = oracle.Oracle(s)
    rho, M, G = outs[0]
    assert rel_err(to_np(rho[0]), o.rho(to_np(D))[0]) < 1e-10
    assert rel_err(to_np(M), o.mat([to_np(v) for v in V])) < 1e-10
    assert rel_err(to_np(G), o.grad(to_np(D), [to_np(v) for v in V])) < 1e-10
    for it in items:
        it[2].close()


def test_batch_empty_and_repeated_plan():
    """Zero tasks is a no-op; the same plan may appear in several tasks with
    distinct outputs."""
    import torch
    from paper_2603_24881_amd.gpw import GPW
    _lib.gpw_eval_batch([])
    s = synth.config1()
    g = GPW(s)
    D1 = to_dev(synth.make_density(s))
    D2 = to_dev(2.0 * synth.make_density(s) + np.eye(g.n_ao))
    r1, r2 = g.new_grids(), g.new_grids()
    _lib.gpw_eval_batch([dict(plan=g.plan, op=_lib.GPW_OP_RHO, D=D1, rho=r1),
                         dict(plan=g.plan, op=_lib.GPW_OP_RHO, D=D2, rho=r2)])
    torch.cuda.synchronize()
    assert np.array_equal(to_np(r1[0]), to_np(g.rho(D1)[0]))
    assert np.array_equal(to_np(r2[0]), to_np(g.rho(D2)[0]))
    g.close()


def test_batch_with_more_segments_than_one_launch_holds():
    """Six plans of four levels each: 24 (task, level) segments per class, more
    than one launch's table holds, so the launches are split; every task still
    equals its single call."""
    import torch
    from paper_2603_24881_amd.gpw import GPW
    systems = [synth.config5(8, 0), synth.config5(8, 1), synth.config5(16, 0), synth.config5(16, 1),
               synth.config2(), synth.config5(32, 0)]
    plans = [GPW(s) for s in systems]
    assert all(len(g.meshes) == 4 for g in plans)
    Ds = [to_dev(synth.make_density(s)) for s in systems]
    Vs = [[to_dev(v) for v in synth.make_potentials(g.meshes, s.seed)] for g, s in zip(plans, systems)]
    ref = [([to_np(r) for r in g.rho(D)], to_np(g.mat(V))) for g, D, V in zip(plans, Ds, Vs)]
    outs, tasks = [], []
    for g, D, V in zip(plans, Ds, Vs):
        rho = g.new_grids()
        M = torch.empty((g.n_ao, g.n_ao), dtype=torch.float64, device=D.device)
        outs.append((rho, M))
        tasks += [dict(plan=g.plan, op=_lib.GPW_OP_RHO, D=D, rho=rho), dict(plan=g.plan, op=_lib.GPW_OP_MAT, v=V, out=M)]
    _lib.gpw_eval_batch(tasks)
    torch.cuda.synchronize()
    for (rho_r, M_r), (rho, M) in zip(ref, outs):
        for a, b in zip(rho, rho_r):
            assert np.array_equal(to_np(a), b)
        assert rel_err(to_np(M), M_r) < 1e-12
    for g in plans:
        g.close()


def test_one_plan_on_two_streams():
    """One plan evaluated concurrently on two streams with distinct outputs."""
    import torch
    from paper_2603_24881_amd.gpw import GPW
    s = synth.config2()
    g = GPW(s)
    D1 = to_dev(synth.make_density(s))
    D2 = to_dev(synth.make_density(s, seed=s.seed + 1))
    ref1 = [to_np(r) for r in g.rho(D1)]
    ref2 = [to_np(r) for r in g.rho(D2)]
    torch.cuda.synchronize()
    st1, st2 = torch.cuda.Stream(), torch.cuda.Stream()
    r1, r2 = g.new_grids(), g.new_grids()
    torch.cuda.synchronize()
    for _ in range(3):
        g.rho(D1, out=r1, stream=st1)
        g.rho(D2, out=r2, stream=st2)
    torch.cuda.synchronize()
    for a, b in zip(r1, ref1):
        assert np.array_equal(to_np(a), b)
    for a, b in zip(r2, ref2):
        assert np.array_equal(to_np(a), b)
    g.close()
