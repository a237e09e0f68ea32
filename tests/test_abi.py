"""The C ABI library builds, loads and exports every declared symbol; argument
checking happens on the host before any device work (CPU-only tests)."""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2603_24881_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "gpw.h")).read()
    return sorted(set(re.findall(r"\b(gpw_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    lib = _lib.load()
    names = _declared()
    assert set(names) == set(_lib.EXPORTS), names
    for n in names:
        assert hasattr(lib, n), n


def _basis(l=0, exp=1.0):
    return dict(cell=np.diag([8.0, 8.0, 8.0]), coords=np.zeros((1, 3)), shell_atom=[0], shell_l=[l],
                shell_nprim=[1], shell_prim0=[0], exps=[exp], coefs=[1.0])


@pytest.mark.parametrize("bad,status", [
    (dict(shell_l=[5]), 2),            # h shell: unsupported
    (dict(shell_l=[-1]), 1),
    (dict(exps=[0.0]), 1),
    (dict(exps=[-1.0]), 1),
    (dict(shell_atom=[3]), 1),
    (dict(cell=np.array([[8.0, 0.5, 0], [16.0, 1.0, 0], [0, 0, 8]])), 1),   # linearly dependent vectors
    (dict(cell=np.diag([8.0, 0.0, 8.0])), 1),
])
def test_invalid_arguments_are_rejected_on_the_host(bad, status):
    kw = _basis()
    kw.update(bad)
    with pytest.raises(_lib.GPWError) as ei:
        _lib.gpw_plan(**kw, mesh=[[8, 8, 8]], tau=1e-6)
    assert ei.value.status == status
    assert _lib.gpw_last_error()


@pytest.mark.parametrize("cut,status", [
    (dict(mesh=None, ke_cutoff_ry=None), 1),
    (dict(mesh=None, ke_cutoff_ry=[100.0, 200.0]), 1),      # not descending
    (dict(mesh=[[8, 8, 8]], tau=0.0), 1),
    (dict(mesh=[[8, 8, 8]], tau=2.0), 1),
    (dict(mesh=[[8, 8, 8]], precision=7), 1),
])
def test_invalid_cutoffs_are_rejected(cut, status):
    kw = _basis()
    args = dict(tau=1e-6)
    args.update(cut)
    if args.get("mesh") is None and args.get("ke_cutoff_ry") is None:
        args["ke_cutoff_ry"] = []
        args["mesh"] = None
    with pytest.raises(_lib.GPWError) as ei:
        _lib.gpw_plan(**kw, **args)
    assert ei.value.status == status


def test_null_arguments():
    lib = _lib.load()
    h = C.c_void_p()
    assert lib.gpw_plan(None, None, None, C.byref(h)) == 1
    assert lib.gpw_plan_destroy(None) == 0
    assert lib.gpw_plan_query(None, None) == 1
    assert lib.gpw_eval_rho(None, None, None, None) == 1
    assert lib.gpw_eval_mat(None, None, None, None) == 1
    assert lib.gpw_eval_grad(None, None, None, None, None) == 1
    assert lib.gpw_eval_mat_noalloc(None, None, None, None) == 1
    assert lib.gpw_eval_tau(None, None, None, None) == 1
    assert lib.gpw_eval_mat_tau(None, None, None, None) == 1
    assert lib.gpw_eval_grad_tau(None, None, None, None, None) == 1
    assert lib.gpw_eval_batch(None, -1, None) == 1
    assert lib.gpw_eval_batch(None, 0, None) == 0
    one = (_lib.gpw_task * 1)()
    assert lib.gpw_eval_batch(one, 1, None) == 1          # NULL plan
    assert "NULL plan" in _lib.gpw_last_error()


def test_library_and_torch_share_one_hip_runtime():
    """Loading the library before torch must not bring a second HIP runtime into
    the process (torch then reports no device): the binding binds libgpw.so to
    the runtime torch carries."""
    import subprocess
    import sys
    code = ("import paper_2603_24881_amd._lib as L; L.load(); import torch; "
            "print(sorted({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, check=True)
    libs = eval(out.stdout.strip().splitlines()[-1])
    assert len(libs) == 1, libs
