"""Seeded synthetic inputs: cells, atoms, Gaussian basis sets, density matrices and
grid potentials.

This module only draws inputs.  It holds none of the collocation / integration
arithmetic: no pair screening, no level assignment, no mesh rule, no grid
evaluation.  Both the CPU oracle (tests) and the HIP path (library, bench) take
their inputs from here, so that the two sides see identical numbers.

The systems stand in for the paper's water clusters, diamond supercells and
GTH basis sets (Sec. IV), which are not available: shapes, sizes and exponent
ranges follow the workloads described there, the numbers are random.

Conventions
-----------
* bohr for lengths, bohr^-2 for exponents, Rydberg for plane-wave cutoffs.
* Orthorhombic cells, given by their three side lengths.
* A basis is a list of contracted Cartesian shells.  Each primitive carries a raw
  coefficient that multiplies the *un-normalised* Cartesian primitive
  (x-Ax)^i (y-Ay)^j (z-Az)^k exp(-a |r-A|^2).  The generator folds a radial
  normalisation into the raw coefficient (``radial_norm``).
* Random draws happen in a fixed order: positions, then per-shell primitive
  counts, then exponents, then coefficients, then the orbital matrix C of
  D = C C^T, then grid potentials.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Cartesian component counts per angular momentum.
NCART = (1, 3, 6, 10, 15)

# Water geometry: O-H bond length (bohr) and H-O-H angle (degrees).
OH_BOND = 1.81
HOH_ANGLE = 104.5


@dataclass
class System:
    """A periodic system: cell, atoms, contracted Cartesian basis, multigrid
    cutoffs and screening threshold."""

    name: str
    cell: np.ndarray                  # (3,) orthorhombic side lengths, or (3, 3) lattice vectors as rows
    coords: np.ndarray                # (natm, 3)
    shell_atom: np.ndarray            # (nshell,) int32
    shell_l: np.ndarray               # (nshell,) int32, 0..4
    shell_nprim: np.ndarray           # (nshell,) int32
    shell_prim0: np.ndarray           # (nshell,) int32 offset into exps/coefs
    exps: np.ndarray                  # (nprim_total,) float64
    coefs: np.ndarray                 # (nprim_total,) float64 raw coefficients
    ke_cutoff_ry: list = field(default_factory=list)   # per level, descending
    rel_cutoff_ry: float = 60.0
    mesh: np.ndarray | None = None    # (nlevels, 3) override; None = from cutoffs
    tau: float = 1e-6
    n_occ: int = 1                    # rank of the synthetic density matrix
    seed: int = 0

    @property
    def natm(self) -> int:
        return int(self.coords.shape[0])

    @property
    def nshell(self) -> int:
        return int(self.shell_l.shape[0])

    @property
    def nlevels(self) -> int:
        if self.mesh is not None:
            return int(self.mesh.shape[0])
        return len(self.ke_cutoff_ry)

    @property
    def n_ao(self) -> int:
        return int(sum(NCART[l] for l in self.shell_l))

    def ao_offsets(self) -> np.ndarray:
        off = np.zeros(self.nshell + 1, dtype=np.int64)
        for s, l in enumerate(self.shell_l):
            off[s + 1] = off[s] + NCART[int(l)]
        return off

    def with_tau(self, tau: float) -> "System":
        import copy
        s = copy.copy(self)
        s.tau = float(tau)
        return s


# --------------------------------------------------------------------------
# basic draws
# --------------------------------------------------------------------------

def radial_norm(alpha: float, l: int) -> float:
    """Radial normalisation N(alpha, l): int_0^inf r^(2l+2) N^2 exp(-2 alpha r^2) dr = 1."""
    val = math.gamma(l + 1.5) / (2.0 * (2.0 * alpha) ** (l + 1.5))
    return val ** -0.5


def haar_rotation(rng: np.random.Generator) -> np.ndarray:
    """Haar-random 3x3 rotation: QR of a Gaussian matrix with the sign fix."""
    z = rng.standard_normal((3, 3))
    q, r = np.linalg.qr(z)
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _log_uniform(rng, lo, hi, n):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), n))


def draw_element_basis(rng, shell_ls, exp_range, nprim=None):
    """Draw one element's basis: for each shell a primitive count, then the
    exponents, then the raw coefficients (N(0,1) times the radial norm)."""
    if nprim is None:
        counts = [int(c) for c in rng.integers(1, 4, size=len(shell_ls))]
    else:
        counts = [int(nprim)] * len(shell_ls)
    exps = []
    for c in counts:
        e = np.sort(_log_uniform(rng, exp_range[0], exp_range[1], c))[::-1]
        exps.append(e)
    coefs = []
    for l, e in zip(shell_ls, exps):
        g = rng.standard_normal(len(e))
        coefs.append(np.array([g[i] * radial_norm(e[i], l) for i in range(len(e))]))
    return [(int(l), e, c) for l, e, c in zip(shell_ls, exps, coefs)]


def assemble(name, cell, coords, atom_basis, **kw) -> System:
    """Flatten per-atom shell lists [(l, exps, coefs), ...] into a System."""
    sa, sl, sn, s0, ex, cf = [], [], [], [], [], []
    p0 = 0
    for ia, shells in enumerate(atom_basis):
        for (l, e, c) in shells:
            sa.append(ia)
            sl.append(l)
            sn.append(len(e))
            s0.append(p0)
            ex.extend(float(x) for x in e)
            cf.extend(float(x) for x in c)
            p0 += len(e)
    return System(
        name=name,
        cell=(np.asarray(cell, dtype=np.float64).reshape(3, 3) if np.size(cell) == 9
              else np.asarray(cell, dtype=np.float64).reshape(3)),
        coords=np.asarray(coords, dtype=np.float64).reshape(-1, 3),
        shell_atom=np.asarray(sa, dtype=np.int32),
        shell_l=np.asarray(sl, dtype=np.int32),
        shell_nprim=np.asarray(sn, dtype=np.int32),
        shell_prim0=np.asarray(s0, dtype=np.int32),
        exps=np.asarray(ex, dtype=np.float64),
        coefs=np.asarray(cf, dtype=np.float64),
        **kw,
    )


def water_coords(rng, n_waters, L):
    """n water-like units: O uniform in [0,L)^3, Haar-random orientation,
    O-H 1.81 bohr and H-O-H 104.5 degrees.  Atoms are not wrapped."""
    o = rng.uniform(0.0, L, size=(n_waters, 3))
    half = math.radians(HOH_ANGLE / 2.0)
    local = np.array([[math.sin(half), 0.0, math.cos(half)],
                      [-math.sin(half), 0.0, math.cos(half)]]) * OH_BOND
    coords = []
    for i in range(n_waters):
        q = haar_rotation(rng)
        coords.append(o[i])
        coords.append(o[i] + q @ local[0])
        coords.append(o[i] + q @ local[1])
    return np.array(coords)


DIAMOND_SITES = np.array([
    [0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0],
    [.25, .25, .25], [.25, .75, .75], [.75, .25, .75], [.75, .75, .25]])


# --------------------------------------------------------------------------
# the workloads
# --------------------------------------------------------------------------

WATER_LEVELS = [400.0, 130.0, 45.0, 15.0]
DIAMOND_LEVELS = [600.0, 200.0, 600.0 / 9.0, 600.0 / 27.0, 600.0 / 81.0]
O_BASIS_SMALL = [0, 0, 0, 1, 1, 2]          # 3s2p1d
O_BASIS_F = [0, 0, 0, 1, 1, 2, 2, 3]        # 3s2p2d1f
H_BASIS = [0, 0, 1]                         # 2s1p
C_BASIS = [0, 0, 1, 1, 2]                   # 2s2p1d


def water_cluster(n_waters, L, seed, o_shells, exp_range=(0.1, 30.0),
                  n_occ=None, tau=1e-6, name=None, levels=WATER_LEVELS):
    rng = np.random.default_rng(seed)
    coords = water_coords(rng, n_waters, L)
    o_basis = draw_element_basis(rng, o_shells, exp_range)
    h_basis = draw_element_basis(rng, H_BASIS, exp_range)
    atom_basis = []
    for i in range(n_waters):
        atom_basis += [o_basis, h_basis, h_basis]
    return assemble(name or f"water{n_waters}", [L, L, L], coords, atom_basis,
                    ke_cutoff_ry=list(levels), rel_cutoff_ry=60.0, tau=tau,
                    n_occ=n_occ if n_occ is not None else 5 * n_waters, seed=seed)


def config1(seed=1001, tau=1e-6) -> System:
    """4 atoms in a cubic 8 bohr cell, one s and one p shell of 2 primitives
    each per atom (exponents log-uniform in [0.2, 8]); single 24^3 grid."""
    rng = np.random.default_rng(seed)
    L = 8.0
    coords = rng.uniform(0.0, L, size=(4, 3))
    atom_basis = [draw_element_basis(rng, [0, 1], (0.2, 8.0), nprim=2) for _ in range(4)]
    return assemble("c1", [L, L, L], coords, atom_basis,
                    mesh=np.array([[24, 24, 24]], dtype=np.int32),
                    ke_cutoff_ry=[], tau=tau, n_occ=8, seed=seed)


def config2(seed=1002, tau=1e-6) -> System:
    """32 water-like units in an 18.6 bohr cell; O 3s2p1d, H 2s1p; 4 levels."""
    return water_cluster(32, 18.6, seed, O_BASIS_SMALL, n_occ=160, tau=tau, name="c2")


def config3(seed=1003, tau=1e-6) -> System:
    """64 water-like units in a 25 bohr cell; O 3s2p2d1f, H 2s1p; 4 levels."""
    return water_cluster(64, 25.0, seed, O_BASIS_F, n_occ=320, tau=tau, name="c3")


def config4(seed=1004, tau=1e-6) -> System:
    """Diamond-like 3x3x3 conventional supercell (216 C, a = 6.74 bohr);
    C 2s2p1d, exponents log-uniform in [0.15, 20]; 5 levels from 600 Ry."""
    rng = np.random.default_rng(seed)
    a = 6.74
    coords = []
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for s in DIAMOND_SITES:
                    coords.append((np.array([i, j, k]) + s) * a)
    coords = np.array(coords)
    c_basis = draw_element_basis(rng, C_BASIS, (0.15, 20.0))
    return assemble("c4", [3 * a] * 3, coords, [c_basis] * len(coords),
                    ke_cutoff_ry=list(DIAMOND_LEVELS), rel_cutoff_ry=60.0,
                    tau=tau, n_occ=432, seed=seed)


def config5(n_waters, geometry=0, tau=1e-6) -> System:
    """Serving workload member: n water-like units (config-3 basis) in a cubic
    cell of side n^(1/3) * 4.65 bohr.  Two geometries (seeds) per size."""
    L = n_waters ** (1.0 / 3.0) * 4.65
    seed = 5000 + 10 * n_waters + geometry
    return water_cluster(n_waters, L, seed, O_BASIS_F, n_occ=5 * n_waters,
                         tau=tau, name=f"c5_w{n_waters}_g{geometry}")


def water256(tau=1e-6) -> System:
    """The 256-water-like system: config-5 member with 256 units (768 atoms,
    10496 Cartesian AOs, L = 29.53 bohr)."""
    return config5(256, 0, tau=tau)


CONFIGS = {"c1": config1, "c2": config2, "c3": config3, "c4": config4}


def draw_orbitals(sys: System, seed: int | None = None, n_occ: int | None = None) -> np.ndarray:
    """C (n_ao x n_occ) with N(0,1) entries; the density matrix is D = C C^T."""
    rng = np.random.default_rng((sys.seed if seed is None else seed) + 7)
    k = sys.n_occ if n_occ is None else n_occ
    return rng.standard_normal((sys.n_ao, k))


def make_density(sys: System, seed: int | None = None) -> np.ndarray:
    c = draw_orbitals(sys, seed)
    return c @ c.T


def make_potentials(meshes, seed: int) -> list:
    """One N(0,1) potential per level, C-ordered arrays of the given meshes."""
    rng = np.random.default_rng(seed + 11)
    return [rng.standard_normal(tuple(int(x) for x in m)) for m in meshes]
