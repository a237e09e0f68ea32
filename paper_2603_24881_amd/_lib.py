"""ctypes binding of libgpw (include/gpw.h).

Argument marshalling only: every computation happens in the HIP kernels of
libgpw.so.  Device buffers are torch tensors (float64, contiguous, on the plan's
device); streams are torch streams (``torch.cuda.current_stream()`` when not
given).  If the library has not been built, importing the binding raises:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgpw.so")

GPW_MAX_LEVELS = 8
GPW_NCLASS = 15
GPW_FP64, GPW_FP32 = 0, 1
GPW_OP_RHO, GPW_OP_MAT, GPW_OP_GRAD, GPW_OP_TAU, GPW_OP_MAT_TAU, GPW_OP_GRAD_TAU = 0, 1, 2, 3, 4, 5
GRID_OPS = (GPW_OP_RHO, GPW_OP_TAU)
MAT_OPS = (GPW_OP_MAT, GPW_OP_MAT_TAU)
GRAD_OPS = (GPW_OP_GRAD, GPW_OP_GRAD_TAU)
STATUS = {0: "GPW_OK", 1: "GPW_EINVAL", 2: "GPW_EUNSUPPORTED", 3: "GPW_ENOMEM",
          4: "GPW_EDEVICE", 5: "GPW_EBUDGET"}


class GPWError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class gpw_cell(C.Structure):
    _fields_ = [("a", (C.c_double * 3) * 3)]


class gpw_basis(C.Structure):
    _fields_ = [
        ("natm", C.c_int),
        ("coords", C.POINTER(C.c_double)),
        ("nshell", C.c_int),
        ("shell_atom", C.POINTER(C.c_int)),
        ("shell_l", C.POINTER(C.c_int)),
        ("shell_nprim", C.POINTER(C.c_int)),
        ("shell_prim0", C.POINTER(C.c_int)),
        ("exps", C.POINTER(C.c_double)),
        ("coefs", C.POINTER(C.c_double)),
    ]


class gpw_cutoffs(C.Structure):
    _fields_ = [
        ("nlevels", C.c_int),
        ("ke_cutoff_ry", C.POINTER(C.c_double)),
        ("mesh", C.POINTER(C.c_int)),
        ("rel_cutoff_ry", C.c_double),
        ("tau", C.c_double),
        ("precision", C.c_int),
        ("device", C.c_int),
    ]


class gpw_plan_info(C.Structure):
    _fields_ = [
        ("nlevels", C.c_int),
        ("mesh", (C.c_int * 3) * GPW_MAX_LEVELS),
        ("weight", C.c_double * GPW_MAX_LEVELS),
        ("n_grid", C.c_longlong * GPW_MAX_LEVELS),
        ("n_ao", C.c_int),
        ("natm", C.c_int),
        ("precision", C.c_int),
        ("n_pairs", C.c_longlong * GPW_MAX_LEVELS),
        ("n_pairs_class", C.c_longlong * GPW_NCLASS),
        ("n_incidences", C.c_longlong * GPW_MAX_LEVELS),
        ("n_incidences_class", C.c_longlong * GPW_NCLASS),
        ("sphere_points", C.c_double),
        ("flops_rho_block", C.c_double),
        ("flops_rho_sphere", C.c_double),
        ("flops_mat_block", C.c_double),
        ("flops_mat_sphere", C.c_double),
        ("flops_grad_block", C.c_double),
        ("flops_grad_sphere", C.c_double),
        ("flops_rho_exec", C.c_double),
        ("flops_mat_exec", C.c_double),
        ("device_bytes", C.c_longlong),
        ("max_box_width", C.c_int),
        ("scratch_bytes", C.c_longlong * 6),
        ("flops_grad_exec", C.c_double),
        ("flops_tau_exec", C.c_double),
        ("flops_mat_tau_exec", C.c_double),
        ("flops_grad_tau_exec", C.c_double),
        ("poisson_scratch_bytes", C.c_longlong),
    ]


class gpw_task(C.Structure):
    _fields_ = [
        ("plan", C.c_void_p),
        ("op", C.c_int),
        ("D", C.c_void_p),
        ("v", C.c_void_p),
        ("rho", C.c_void_p),
        ("out", C.c_void_p),
    ]


EXPORTS = ("gpw_plan", "gpw_plan_destroy", "gpw_plan_query", "gpw_eval_rho", "gpw_eval_mat",
           "gpw_eval_grad", "gpw_eval_tau", "gpw_eval_mat_tau", "gpw_eval_grad_tau", "gpw_eval_batch",
           "gpw_eval_mat_noalloc", "gpw_poisson", "gpw_hxc_potential", "gpw_fine_density",
           "gpw_last_error")
GPW_NOALLOC_SCRATCH_BYTES = 128 << 20

_lib = None


def load(path: str = LIB_PATH):
    """Load libgpw.so; raises if it is missing (build it with build.py).

    torch is imported first: the ROCm wheel of torch carries its own HIP runtime
    (soname libamdhip64.so.7), and libgpw.so must bind to that same runtime.
    Loaded before torch, libgpw.so would bring in the system copy and torch a
    second one, and torch would then see no device."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libgpw.so not built at {path}; run `python -m paper_2603_24881_amd.build`")
    import torch  # noqa: F401  (see above)
    lib = C.CDLL(path)
    lib.gpw_plan.argtypes = [C.POINTER(gpw_cell), C.POINTER(gpw_basis), C.POINTER(gpw_cutoffs),
                             C.POINTER(C.c_void_p)]
    lib.gpw_plan_destroy.argtypes = [C.c_void_p]
    lib.gpw_plan_query.argtypes = [C.c_void_p, C.POINTER(gpw_plan_info)]
    lib.gpw_eval_rho.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.gpw_eval_mat.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.gpw_eval_grad.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.gpw_eval_tau.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.gpw_eval_mat_tau.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.gpw_eval_grad_tau.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.gpw_eval_batch.argtypes = [C.POINTER(gpw_task), C.c_int, C.c_void_p]
    lib.gpw_eval_mat_noalloc.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.gpw_poisson.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.gpw_hxc_potential.argtypes = [C.c_void_p] * 7
    lib.gpw_fine_density.argtypes = [C.c_void_p] * 5
    lib.gpw_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name != "gpw_last_error":
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        raise GPWError(status, load().gpw_last_error().decode())


def _ptr_array(ptrs):
    arr = (C.c_void_p * max(1, len(ptrs)))()
    for i, p in enumerate(ptrs):
        arr[i] = p
    return arr


def _stream_handle(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dev_ptr(t, what, numel=None, device=None):
    """Device address of a contiguous float64 tensor, after checking its size and
    device against what the library will read or write through it."""
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError(f"{what}: expected a contiguous float64 device tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{what}: {t.numel()} elements, the plan needs {numel}")
    if device is not None and t.device.index != device:
        raise ValueError(f"{what}: on device {t.device.index}, the plan lives on device {device}")
    return t.data_ptr()


def _level_ptrs(plan, arrs, what):
    """Host array of the plan's nlevels level-grid pointers (sizes checked)."""
    if arrs is None or len(arrs) != plan.nlevels:
        raise ValueError(f"{what}: expected one grid per level ({plan.nlevels}), got "
                         f"{None if arrs is None else len(arrs)}")
    return _ptr_array([_dev_ptr(a, f"{what}[{l}]", plan.n_grid[l], plan.device) for l, a in enumerate(arrs)])


def _mat_ptr(plan, t, what):
    return _dev_ptr(t, what, plan.n_ao * plan.n_ao, plan.device)


def _grad_ptr(plan, t, what):
    return _dev_ptr(t, what, plan.natm * 3, plan.device)


class PlanHandle:
    """Owns a gpw_plan_t; the host arrays it was built from are copied by the library."""

    def __init__(self, cell, coords, shell_atom, shell_l, shell_nprim, shell_prim0, exps, coefs,
                 ke_cutoff_ry=None, mesh=None, rel_cutoff_ry=60.0, tau=1e-6,
                 precision=GPW_FP64, device=0):
        lib = load()
        self.handle = None
        cell = np.asarray(cell, dtype=np.float64)
        if cell.shape == (3,):
            cell = np.diag(cell)
        c = gpw_cell()
        for i in range(3):
            for j in range(3):
                c.a[i][j] = float(cell[i, j])
        self._keep = [np.ascontiguousarray(coords, dtype=np.float64),
                      np.ascontiguousarray(shell_atom, dtype=np.int32),
                      np.ascontiguousarray(shell_l, dtype=np.int32),
                      np.ascontiguousarray(shell_nprim, dtype=np.int32),
                      np.ascontiguousarray(shell_prim0, dtype=np.int32),
                      np.ascontiguousarray(exps, dtype=np.float64),
                      np.ascontiguousarray(coefs, dtype=np.float64)]
        k = self._keep
        b = gpw_basis(natm=k[0].shape[0], coords=k[0].ctypes.data_as(C.POINTER(C.c_double)),
                      nshell=k[2].shape[0],
                      shell_atom=k[1].ctypes.data_as(C.POINTER(C.c_int)),
                      shell_l=k[2].ctypes.data_as(C.POINTER(C.c_int)),
                      shell_nprim=k[3].ctypes.data_as(C.POINTER(C.c_int)),
                      shell_prim0=k[4].ctypes.data_as(C.POINTER(C.c_int)),
                      exps=k[5].ctypes.data_as(C.POINTER(C.c_double)),
                      coefs=k[6].ctypes.data_as(C.POINTER(C.c_double)))
        cut = gpw_cutoffs()
        if mesh is not None:
            m = np.ascontiguousarray(mesh, dtype=np.int32).reshape(-1, 3)
            self._keep.append(m)
            cut.mesh = m.ctypes.data_as(C.POINTER(C.c_int))
            nl = m.shape[0]
        else:
            nl = len(ke_cutoff_ry)
        if ke_cutoff_ry is not None and len(ke_cutoff_ry):
            e = np.ascontiguousarray(ke_cutoff_ry, dtype=np.float64)
            self._keep.append(e)
            cut.ke_cutoff_ry = e.ctypes.data_as(C.POINTER(C.c_double))
        cut.nlevels = nl
        cut.rel_cutoff_ry = float(rel_cutoff_ry)
        cut.tau = float(tau)
        cut.precision = int(precision)
        cut.device = int(device)
        h = C.c_void_p()
        _check(lib.gpw_plan(C.byref(c), C.byref(b), C.byref(cut), C.byref(h)))
        self.handle = h.value
        self.device = int(device)
        self.info = self.query()
        self.nlevels = self.info["nlevels"]
        self.n_grid = [int(x) for x in self.info["n_grid"]]
        self.n_ao = int(self.info["n_ao"])
        self.natm = int(self.info["natm"])

    def query(self) -> dict:
        info = gpw_plan_info()
        _check(load().gpw_plan_query(self.handle, C.byref(info)))
        nl = info.nlevels
        return {
            "nlevels": nl,
            "mesh": [tuple(info.mesh[l][d] for d in range(3)) for l in range(nl)],
            "weight": [info.weight[l] for l in range(nl)],
            "n_grid": [info.n_grid[l] for l in range(nl)],
            "n_ao": info.n_ao, "natm": info.natm, "precision": info.precision,
            "n_pairs": [info.n_pairs[l] for l in range(nl)],
            "n_pairs_class": list(info.n_pairs_class),
            "n_incidences": [info.n_incidences[l] for l in range(nl)],
            "n_incidences_class": list(info.n_incidences_class),
            "sphere_points": info.sphere_points,
            "flops_rho_block": info.flops_rho_block, "flops_rho_sphere": info.flops_rho_sphere,
            "flops_mat_block": info.flops_mat_block, "flops_mat_sphere": info.flops_mat_sphere,
            "flops_grad_block": info.flops_grad_block, "flops_grad_sphere": info.flops_grad_sphere,
            "flops_rho_exec": info.flops_rho_exec, "flops_mat_exec": info.flops_mat_exec,
            "device_bytes": info.device_bytes, "max_box_width": info.max_box_width,
            "scratch_bytes": list(info.scratch_bytes),
            "flops_grad_exec": info.flops_grad_exec, "flops_tau_exec": info.flops_tau_exec,
            "flops_mat_tau_exec": info.flops_mat_tau_exec, "flops_grad_tau_exec": info.flops_grad_tau_exec,
            "poisson_scratch_bytes": info.poisson_scratch_bytes,
        }

    def close(self):
        if self.handle is not None:
            load().gpw_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gpw_plan(*args, **kw) -> PlanHandle:
    return PlanHandle(*args, **kw)


def gpw_plan_destroy(plan: PlanHandle):
    plan.close()


def gpw_plan_query(plan: PlanHandle) -> dict:
    return plan.query()


def gpw_eval_rho(plan: PlanHandle, D, rho, stream=None):
    arr = _level_ptrs(plan, rho, "rho")
    _check(load().gpw_eval_rho(plan.handle, _mat_ptr(plan, D, "D"), arr, _stream_handle(stream)))


def gpw_eval_mat(plan: PlanHandle, v, M, stream=None):
    arr = _level_ptrs(plan, v, "v")
    _check(load().gpw_eval_mat(plan.handle, arr, _mat_ptr(plan, M, "M"), _stream_handle(stream)))


def gpw_eval_tau(plan: PlanHandle, D, tau, stream=None):
    arr = _level_ptrs(plan, tau, "tau")
    _check(load().gpw_eval_tau(plan.handle, _mat_ptr(plan, D, "D"), arr, _stream_handle(stream)))


def gpw_eval_mat_tau(plan: PlanHandle, vtau, M, stream=None):
    arr = _level_ptrs(plan, vtau, "vtau")
    _check(load().gpw_eval_mat_tau(plan.handle, arr, _mat_ptr(plan, M, "M"), _stream_handle(stream)))


def gpw_eval_grad_tau(plan: PlanHandle, D, vtau, grad, stream=None):
    arr = _level_ptrs(plan, vtau, "vtau")
    _check(load().gpw_eval_grad_tau(plan.handle, _mat_ptr(plan, D, "D"), arr, _grad_ptr(plan, grad, "grad"),
                                    _stream_handle(stream)))


def gpw_poisson(plan: PlanHandle, rho, v, e_j=None, stream=None):
    """rho, v: one float64 device grid per level; e_j: a one-element float64
    device tensor receiving E_J, or None."""
    ra = _level_ptrs(plan, rho, "rho")
    va = _level_ptrs(plan, v, "v")
    ep = None if e_j is None else _dev_ptr(e_j, "e_j", 1, plan.device)
    _check(load().gpw_poisson(plan.handle, ra, va, ep, _stream_handle(stream)))


def _fine_ptr(plan, t, what):
    return _dev_ptr(t, what, plan.n_grid[0], plan.device)


def gpw_hxc_potential(plan: PlanHandle, rho, v, vxc=None, vxc_grad=None, e_j=None, stream=None):
    """Level potentials of the Hartree term plus a fine-grid XC potential
    (vxc: one level-0 grid) and GGA vector potential (vxc_grad: three level-0
    grids), either may be None."""
    ra = _level_ptrs(plan, rho, "rho")
    va = _level_ptrs(plan, v, "v")
    xp = None if vxc is None else _fine_ptr(plan, vxc, "vxc")
    ga = None
    if vxc_grad is not None:
        if len(vxc_grad) != 3:
            raise ValueError("vxc_grad: expected three components")
        ga = _ptr_array([_fine_ptr(plan, t, f"vxc_grad[{d}]") for d, t in enumerate(vxc_grad)])
    ep = None if e_j is None else _dev_ptr(e_j, "e_j", 1, plan.device)
    _check(load().gpw_hxc_potential(plan.handle, ra, xp, ga, va, ep, _stream_handle(stream)))


def gpw_fine_density(plan: PlanHandle, rho, rho_fine=None, grad=None, stream=None):
    ra = _level_ptrs(plan, rho, "rho")
    rp = None if rho_fine is None else _fine_ptr(plan, rho_fine, "rho_fine")
    ga = None
    if grad is not None:
        if len(grad) != 3:
            raise ValueError("grad: expected three components")
        ga = _ptr_array([_fine_ptr(plan, t, f"grad[{d}]") for d, t in enumerate(grad)])
    _check(load().gpw_fine_density(plan.handle, ra, rp, ga, _stream_handle(stream)))


def gpw_eval_mat_noalloc(plan: PlanHandle, v, M, stream=None):
    arr = _level_ptrs(plan, v, "v")
    _check(load().gpw_eval_mat_noalloc(plan.handle, arr, _mat_ptr(plan, M, "M"), _stream_handle(stream)))


def gpw_eval_grad(plan: PlanHandle, D, v, grad, stream=None):
    arr = _level_ptrs(plan, v, "v")
    _check(load().gpw_eval_grad(plan.handle, _mat_ptr(plan, D, "D"), arr, _grad_ptr(plan, grad, "grad"),
                                _stream_handle(stream)))


def gpw_eval_batch(tasks, stream=None):
    """tasks: list of dicts {plan, op, D, v, rho, out} with torch tensors."""
    n = len(tasks)
    arr = (gpw_task * max(1, n))()
    keep = []
    for i, t in enumerate(tasks):
        plan, op = t["plan"], int(t["op"])
        arr[i].plan = plan.handle
        arr[i].op = op
        if op not in GRID_OPS + MAT_OPS + GRAD_OPS:
            raise ValueError(f"task {i}: unknown op {op}")
        if op in GRID_OPS + GRAD_OPS:
            arr[i].D = _mat_ptr(plan, t.get("D"), f"task {i} D")
        if op in MAT_OPS + GRAD_OPS:
            va = _level_ptrs(plan, t.get("v"), f"task {i} v")
            keep.append(va)
            arr[i].v = C.cast(va, C.c_void_p)
        if op in GRID_OPS:
            ra = _level_ptrs(plan, t.get("rho"), f"task {i} rho")
            keep.append(ra)
            arr[i].rho = C.cast(ra, C.c_void_p)
        elif op in MAT_OPS:
            arr[i].out = _mat_ptr(plan, t.get("out"), f"task {i} M")
        else:
            arr[i].out = _grad_ptr(plan, t.get("out"), f"task {i} grad")
    _check(load().gpw_eval_batch(arr, n, _stream_handle(stream)))


def gpw_last_error() -> str:
    return load().gpw_last_error().decode()
