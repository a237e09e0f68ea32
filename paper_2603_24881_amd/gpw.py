"""Convenience wrapper: a plan bound to one synthetic or user system, with
outputs allocated as torch tensors on the plan's device.  All evaluation goes
through the C ABI (``_lib``)."""
from __future__ import annotations

import numpy as np

from . import _lib


class GPW:
    """``system`` provides cell, coords, shell arrays, exps, coefs,
    ke_cutoff_ry / mesh, rel_cutoff_ry and tau (see ``synth.System``)."""

    def __init__(self, system, precision: str = "fp64", device: int = 0, tau: float | None = None):
        prec = {"fp64": _lib.GPW_FP64, "fp32": _lib.GPW_FP32}[precision]
        cut = list(system.ke_cutoff_ry) if len(system.ke_cutoff_ry) else None
        self.plan = _lib.gpw_plan(system.cell, system.coords, system.shell_atom, system.shell_l,
                                  system.shell_nprim, system.shell_prim0, system.exps, system.coefs,
                                  ke_cutoff_ry=cut, mesh=system.mesh, rel_cutoff_ry=system.rel_cutoff_ry,
                                  tau=system.tau if tau is None else tau, precision=prec, device=device)
        self.info = self.plan.info
        self.meshes = self.info["mesh"]
        self.weights = self.info["weight"]
        self.n_ao = self.info["n_ao"]
        self.natm = self.info["natm"]
        self.device = device
        self.coords = np.array(system.coords, dtype=np.float64)
        self.cell = np.array(system.cell, dtype=np.float64)
        self.cutoffs_ry = list(system.ke_cutoff_ry) if len(system.ke_cutoff_ry) else None

    def _dev(self):
        import torch
        return torch.device("cuda", self.device)

    def new_grids(self):
        import torch
        return [torch.empty(m, dtype=torch.float64, device=self._dev()) for m in self.meshes]

    def rho(self, D, out=None, stream=None):
        out = self.new_grids() if out is None else out
        _lib.gpw_eval_rho(self.plan, D, out, stream)
        return out

    def mat(self, V, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty((self.n_ao, self.n_ao), dtype=torch.float64, device=self._dev())
        _lib.gpw_eval_mat(self.plan, [v.contiguous() for v in V], out, stream)
        return out

    def grad(self, D, V, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty((self.natm, 3), dtype=torch.float64, device=self._dev())
        _lib.gpw_eval_grad(self.plan, D, [v.contiguous() for v in V], out, stream)
        return out

    def tau(self, D, out=None, stream=None):
        """Kinetic energy density 1/2 sum D grad phi . grad phi on every level."""
        out = self.new_grids() if out is None else out
        _lib.gpw_eval_tau(self.plan, D, out, stream)
        return out

    def mat_tau(self, Vtau, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty((self.n_ao, self.n_ao), dtype=torch.float64, device=self._dev())
        _lib.gpw_eval_mat_tau(self.plan, [v.contiguous() for v in Vtau], out, stream)
        return out

    def grad_tau(self, D, Vtau, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty((self.natm, 3), dtype=torch.float64, device=self._dev())
        _lib.gpw_eval_grad_tau(self.plan, D, [v.contiguous() for v in Vtau], out, stream)
        return out

    def poisson(self):
        """Multigrid transfer + Poisson step of this plan (gpw_poisson)."""
        from .poisson import Poisson
        return Poisson(self)

    def close(self):
        self.plan.close()
