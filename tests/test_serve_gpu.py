"""Serving on the device: every request's result is the same when it runs in
a continuous-batching mix with requests of other systems and sizes (batches
on two concurrent lanes) as when it runs alone with the plain calls (FP64
tolerance 1e-10 relative), and a Fock result satisfies E_J = 1/2 Tr(D J)."""
from __future__ import annotations

import numpy as np
import pytest

from gpu_helpers import log, rel_err, to_np
from paper_2603_24881_amd import synth
from paper_2603_24881_amd.serve import FOCK, GRAD, GPUExecutor, Request, Scheduler, system_key, summarize

pytestmark = pytest.mark.gpu

SIZES = [(8, 0), (8, 1), (16, 0), (32, 0)]


def _executor():
    ex = GPUExecutor(keep_results=True)
    for n, geo in SIZES:
        ex.register(system_key(n, geo), synth.config5(n, geo))
    return ex


def _requests():
    kinds = [FOCK, GRAD, GRAD, FOCK, FOCK, GRAD]
    keys = [system_key(*SIZES[i % len(SIZES)]) for i in range(6)]
    return [Request(i, kinds[i], keys[i], 0.0, seed=100 + i) for i in range(6)]


def test_same_result_alone_and_in_the_mix():
    import torch
    ex = _executor()
    mix = _requests()
    sch = Scheduler(ex, 64 << 30)
    sch.run(mix)
    log(f"  rounds (requests per round): {sch.rounds}")
    # batches of several requests on the two lanes, which run at the same time
    assert sum(sch.rounds) == 6 and len(sch.rounds) >= 2 and max(sch.rounds) > 1
    alone = _requests()
    Scheduler(ex, 64 << 30).run_sequential(alone)
    for a, b in zip(mix, alone):
        assert a.error is None and b.error is None
        key = "J" if a.kind == FOCK else "grad"
        e = rel_err(to_np(a.result[key]), to_np(b.result[key]))
        de = abs(a.result["E_J"] - b.result["E_J"]) / abs(b.result["E_J"])
        log(f"  request {a.rid} {a.kind} {a.system}: {key} rel diff {e:.2e}, E_J rel diff {de:.2e}")
        assert e < 1e-10 and de < 1e-10
        if a.kind == FOCK:
            D = ex.density(a.system, a.seed)
            half = 0.5 * float((D * a.result["J"]).sum())
            assert abs(half - a.result["E_J"]) < 1e-10 * abs(a.result["E_J"])
    log(f"  mix: {summarize(mix)}")
    log(f"  alone: {summarize(alone)}")
