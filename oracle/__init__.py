"""CPU oracle for Gaussian-plane-wave collocation / integration / gradient.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product path
(``paper_2603_24881_amd``) never touches it.

The numerics live in ``gpw_oracle.c`` (plain C + OpenMP, FP64).  This module
only compiles it with gcc and marshals arguments through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# points visited per (l_a, l_b) of the ordered pairs, index 5 l_a + l_b (l <= 4)
NCOUNT = 25
_SRC = os.path.join(_HERE, "gpw_oracle.c")
_LIB = os.path.join(_HERE, "libgpw_oracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-std=gnu99", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _OSys(C.Structure):
    _fields_ = [
        ("cell", C.c_double * 3),
        ("natm", C.c_int),
        ("coords", C.POINTER(C.c_double)),
        ("nshell", C.c_int),
        ("shell_atom", C.POINTER(C.c_int)),
        ("shell_l", C.POINTER(C.c_int)),
        ("shell_nprim", C.POINTER(C.c_int)),
        ("shell_prim0", C.POINTER(C.c_int)),
        ("exps", C.POINTER(C.c_double)),
        ("coefs", C.POINTER(C.c_double)),
        ("nlevels", C.c_int),
        ("mesh", C.POINTER(C.c_int)),
        ("level_cut", C.POINTER(C.c_double)),
        ("rel_cut", C.c_double),
        ("tau", C.c_double),
        ("atom_mask", C.POINTER(C.c_ubyte)),
        ("mask_either", C.c_int),
        ("lat", C.POINTER(C.c_double)),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        for name in ("oracle_rho", "oracle_rho_points", "oracle_mat", "oracle_mat_blocks",
                     "oracle_grad", "oracle_count_pairs", "oracle_meshes", "oracle_num_threads",
                     "oracle_tau", "oracle_tau_points", "oracle_mat_tau", "oracle_mat_tau_blocks",
                     "oracle_grad_tau", "oracle_set_threads"):
            getattr(_lib, name).restype = C.c_int
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _lp(a):
    return a.ctypes.data_as(C.POINTER(C.c_long))


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> int:
    """OpenMP threads of the following oracle calls; returns the count in effect."""
    return int(_load().oracle_set_threads(C.c_int(int(n))))


class Oracle:
    """Oracle bound to one system.  ``system`` is a ``synth.System``; ``tau``
    overrides its screening threshold; ``atom_mask`` restricts the sum to pairs
    whose first primitive sits on a selected atom (used for bounded samples), or
    with ``mask_either`` to pairs with either primitive on a selected atom (then
    the gradient rows of the selected atoms are complete)."""

    def __init__(self, system, tau: float | None = None, atom_mask=None, mask_either: bool = False):
        self.s = system
        lib = _load()
        cell = np.asarray(system.cell, dtype=np.float64)
        # a 3 x 3 cell holds the lattice vectors as rows; a diagonal one is orthorhombic
        self.lat = None
        if cell.shape == (3, 3):
            if np.count_nonzero(cell - np.diag(np.diag(cell))) == 0:
                cell = np.diag(cell).copy()
            else:
                self.lat = np.ascontiguousarray(cell)
                cell = np.sqrt((cell ** 2).sum(axis=1))      # |a_d| for the mesh rule
        self.cell = np.ascontiguousarray(cell, dtype=np.float64)
        self.coords = np.ascontiguousarray(system.coords, dtype=np.float64)
        self.shell_atom = np.ascontiguousarray(system.shell_atom, dtype=np.int32)
        self.shell_l = np.ascontiguousarray(system.shell_l, dtype=np.int32)
        self.shell_nprim = np.ascontiguousarray(system.shell_nprim, dtype=np.int32)
        self.shell_prim0 = np.ascontiguousarray(system.shell_prim0, dtype=np.int32)
        self.exps = np.ascontiguousarray(system.exps, dtype=np.float64)
        self.coefs = np.ascontiguousarray(system.coefs, dtype=np.float64)
        if system.mesh is not None:
            self.mesh = np.ascontiguousarray(system.mesh, dtype=np.int32).reshape(-1, 3)
            nl = self.mesh.shape[0]
        else:
            nl = len(system.ke_cutoff_ry)
            self.mesh = np.zeros((nl, 3), dtype=np.int32)
            cut = np.asarray(system.ke_cutoff_ry, dtype=np.float64)
            lib.oracle_meshes(_dp(self.cell), C.c_int(nl), _dp(cut), _ip(self.mesh))
        self.level_cut = np.ascontiguousarray(
            system.ke_cutoff_ry if len(system.ke_cutoff_ry) else [0.0] * nl, dtype=np.float64)
        self.nlevels = nl
        self.n_ao = int(system.n_ao)
        self.tau = float(system.tau if tau is None else tau)
        self.atom_mask = None if atom_mask is None else np.ascontiguousarray(atom_mask, dtype=np.uint8)
        st = _OSys()
        st.cell[:] = list(self.cell)
        st.natm = system.natm
        st.coords = _dp(self.coords)
        st.nshell = system.nshell
        st.shell_atom = _ip(self.shell_atom)
        st.shell_l = _ip(self.shell_l)
        st.shell_nprim = _ip(self.shell_nprim)
        st.shell_prim0 = _ip(self.shell_prim0)
        st.exps = _dp(self.exps)
        st.coefs = _dp(self.coefs)
        st.nlevels = nl
        st.mesh = _ip(self.mesh)
        st.level_cut = _dp(self.level_cut) if len(system.ke_cutoff_ry) else None
        st.rel_cut = float(system.rel_cutoff_ry)
        st.tau = self.tau
        st.atom_mask = (self.atom_mask.ctypes.data_as(C.POINTER(C.c_ubyte))
                        if self.atom_mask is not None else None)
        st.mask_either = 1 if mask_either else 0
        st.lat = _dp(self.lat) if self.lat is not None else None
        self._st = st
        self.counts = np.zeros(NCOUNT, dtype=np.int64)

    # -- layout helpers ---------------------------------------------------
    @property
    def meshes(self):
        return [tuple(int(x) for x in m) for m in self.mesh]

    def volume(self):
        return float(abs(np.linalg.det(self.lat))) if self.lat is not None else float(np.prod(self.cell))

    def weights(self):
        vol = self.volume()
        return [vol / float(np.prod(m)) for m in self.mesh]

    def _concat(self, grids):
        return np.ascontiguousarray(np.concatenate([np.asarray(g, dtype=np.float64).ravel() for g in grids]))

    def _split(self, flat):
        out, o = [], 0
        for m in self.meshes:
            n = m[0] * m[1] * m[2]
            out.append(flat[o:o + n].reshape(m))
            o += n
        return out

    # -- evaluations ------------------------------------------------------
    def rho(self, D):
        D = np.ascontiguousarray(D, dtype=np.float64)
        total = sum(m[0] * m[1] * m[2] for m in self.meshes)
        out = np.zeros(total, dtype=np.float64)
        cnt = np.zeros(NCOUNT, dtype=np.int64)
        if _load().oracle_rho(C.byref(self._st), _dp(D), _dp(out), _lp(cnt)) != 0:
            raise MemoryError("oracle_rho: allocation failed")
        self.counts = cnt
        return self._split(out)

    def rho_points(self, D, level, flat_idx):
        D = np.ascontiguousarray(D, dtype=np.float64)
        idx = np.ascontiguousarray(flat_idx, dtype=np.int64)
        out = np.zeros(len(idx), dtype=np.float64)
        cnt = np.zeros(NCOUNT, dtype=np.int64)
        if _load().oracle_rho_points(C.byref(self._st), _dp(D), C.c_int(level), C.c_long(len(idx)),
                                     _lp(idx), _dp(out), _lp(cnt)) != 0:
            raise MemoryError("oracle_rho_points: allocation failed")
        self.counts = cnt
        return out

    def mat(self, V):
        v = self._concat(V)
        out = np.zeros((self.n_ao, self.n_ao), dtype=np.float64)
        cnt = np.zeros(NCOUNT, dtype=np.int64)
        if _load().oracle_mat(C.byref(self._st), _dp(v), _dp(out), _lp(cnt)) != 0:
            raise MemoryError("oracle_mat: allocation failed")
        self.counts = cnt
        return out

    def mat_blocks(self, V, shell_pairs):
        """Blocks M[a-rows, b-cols] for the listed shell pairs (a, b)."""
        v = self._concat(V)
        ns = self.s.nshell
        off = self.s.ao_offsets()
        slot = -np.ones(ns * ns, dtype=np.int64)
        pos = 0
        sizes = []
        for (a, b) in shell_pairs:
            na = int(off[a + 1] - off[a])
            nb = int(off[b + 1] - off[b])
            slot[a * ns + b] = pos
            sizes.append((pos, na, nb))
            pos += na * nb
        out = np.zeros(max(pos, 1), dtype=np.float64)
        cnt = np.zeros(NCOUNT, dtype=np.int64)
        if _load().oracle_mat_blocks(C.byref(self._st), _dp(v), _lp(slot), C.c_long(max(pos, 1)),
                                     _dp(out), _lp(cnt)) != 0:
            raise MemoryError("oracle_mat_blocks: allocation failed")
        self.counts = cnt
        return [out[p:p + na * nb].reshape(na, nb) for (p, na, nb) in sizes]

    def grad(self, D, V):
        D = np.ascontiguousarray(D, dtype=np.float64)
        v = self._concat(V)
        out = np.zeros((self.s.natm, 3), dtype=np.float64)
        cnt = np.zeros(NCOUNT, dtype=np.int64)
        if _load().oracle_grad(C.byref(self._st), _dp(D), _dp(v), _dp(out), _lp(cnt)) != 0:
            raise MemoryError("oracle_grad: allocation failed")
        self.counts = cnt
        return out

    # -- meta-GGA: kinetic energy density terms -----------------------------
    def tau_density(self, D):
        """tau_l = 1/2 sum D grad(phi) . grad(phi) on every level."""
        D = np.ascontiguousarray(D, dtype=np.float64)
        total = sum(m[0] * m[1] * m[2] for m in self.meshes)
        out = np.zeros(total, dtype=np.float64)
        cnt = np.zeros(NCOUNT, dtype=np.int64)
        if _load().oracle_tau(C.byref(self._st), _dp(D), _dp(out), _lp(cnt)) != 0:
            raise MemoryError("oracle_tau: allocation failed")
        self.counts = cnt
        return self._split(out)

    def tau_points(self, D, level, flat_idx):
        D = np.ascontiguousarray(D, dtype=np.float64)
        idx = np.ascontiguousarray(flat_idx, dtype=np.int64)
        out = np.zeros(len(idx), dtype=np.float64)
        cnt = np.zeros(NCOUNT, dtype=np.int64)
        if _load().oracle_tau_points(C.byref(self._st), _dp(D), C.c_int(level), C.c_long(len(idx)),
                                     _lp(idx), _dp(out), _lp(cnt)) != 0:
            raise MemoryError("oracle_tau_points: allocation failed")
        self.counts = cnt
        return out

    def mat_tau(self, V):
        """The kinetic-energy-density term of the matrix for level potentials vtau."""
        v = self._concat(V)
        out = np.zeros((self.n_ao, self.n_ao), dtype=np.float64)
        cnt = np.zeros(NCOUNT, dtype=np.int64)
        if _load().oracle_mat_tau(C.byref(self._st), _dp(v), _dp(out), _lp(cnt)) != 0:
            raise MemoryError("oracle_mat_tau: allocation failed")
        self.counts = cnt
        return out

    def mat_tau_blocks(self, V, shell_pairs):
        v = self._concat(V)
        ns = self.s.nshell
        off = self.s.ao_offsets()
        slot = -np.ones(ns * ns, dtype=np.int64)
        pos = 0
        sizes = []
        for (a, b) in shell_pairs:
            na = int(off[a + 1] - off[a])
            nb = int(off[b + 1] - off[b])
            slot[a * ns + b] = pos
            sizes.append((pos, na, nb))
            pos += na * nb
        out = np.zeros(max(pos, 1), dtype=np.float64)
        cnt = np.zeros(NCOUNT, dtype=np.int64)
        if _load().oracle_mat_tau_blocks(C.byref(self._st), _dp(v), _lp(slot), C.c_long(max(pos, 1)),
                                         _dp(out), _lp(cnt)) != 0:
            raise MemoryError("oracle_mat_tau_blocks: allocation failed")
        self.counts = cnt
        return [out[p:p + na * nb].reshape(na, nb) for (p, na, nb) in sizes]

    def grad_tau(self, D, V):
        """dE_tau/dR with E_tau = sum_l w_l <vtau_l, tau_l(D)> at fixed D and vtau."""
        D = np.ascontiguousarray(D, dtype=np.float64)
        v = self._concat(V)
        out = np.zeros((self.s.natm, 3), dtype=np.float64)
        cnt = np.zeros(NCOUNT, dtype=np.int64)
        if _load().oracle_grad_tau(C.byref(self._st), _dp(D), _dp(v), _dp(out), _lp(cnt)) != 0:
            raise MemoryError("oracle_grad_tau: allocation failed")
        self.counts = cnt
        return out

    def energy_tau(self, D, V):
        """E_tau = sum_l w_l <vtau_l, tau_l(D)>."""
        t = self.tau_density(D)
        return float(sum(w * float(np.vdot(v, r)) for w, v, r in zip(self.weights(), V, t)))

    def count_pairs(self):
        out = np.zeros(self.nlevels, dtype=np.int64)
        _load().oracle_count_pairs(C.byref(self._st), _lp(out))
        return out

    def energy(self, D, V):
        """E = sum_l w_l <v_l, rho_l(D)>."""
        rho = self.rho(D)
        return float(sum(w * float(np.vdot(v, r)) for w, v, r in zip(self.weights(), V, rho)))
