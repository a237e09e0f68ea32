"""Small hand-made systems for the oracle pins (test-only)."""
from __future__ import annotations

import copy

import numpy as np

from paper_2603_24881_amd import synth


def tiny_system(shell_ls=(0, 1, 2, 3), natm=3, cell=(7.0, 8.0, 9.0), exp_range=(0.6, 4.0),
                nprim=None, seed=7, tau=1e-14, mesh=((20, 24, 28),), name="tiny"):
    """``natm`` atoms at random positions of an orthorhombic cell, each with its
    own randomly drawn shells of the given angular momenta."""
    rng = np.random.default_rng(seed)
    cell = np.asarray(cell, dtype=np.float64)
    if cell.shape == (3, 3):            # lattice vectors as rows
        coords = rng.uniform(0.0, 1.0, size=(natm, 3)) @ cell
    else:
        coords = rng.uniform(0.0, 1.0, size=(natm, 3)) * cell
    basis = [synth.draw_element_basis(rng, list(shell_ls), exp_range, nprim=nprim)
             for _ in range(natm)]
    return synth.assemble(name, cell, coords, basis,
                          mesh=None if mesh is None else np.asarray(mesh, dtype=np.int32),
                          ke_cutoff_ry=[], tau=tau, n_occ=4, seed=seed)


def subset_atoms(s, atoms, name=None):
    """The same cell, levels and basis restricted to the listed atoms."""
    atoms = list(atoms)
    basis = []
    for a in atoms:
        shells = []
        for sh in range(s.nshell):
            if int(s.shell_atom[sh]) == a:
                p0, n = int(s.shell_prim0[sh]), int(s.shell_nprim[sh])
                shells.append((int(s.shell_l[sh]), s.exps[p0:p0 + n].copy(), s.coefs[p0:p0 + n].copy()))
        basis.append(shells)
    out = synth.assemble(name or (s.name + "_sub"), s.cell, s.coords[atoms], basis,
                         ke_cutoff_ry=list(s.ke_cutoff_ry), rel_cutoff_ry=s.rel_cutoff_ry,
                         mesh=None if s.mesh is None else s.mesh.copy(), tau=s.tau,
                         n_occ=min(s.n_occ, 8), seed=s.seed)
    return out


def subset_waters(s, n):
    """The first n water units (3n atoms) of a water cluster."""
    return subset_atoms(s, range(3 * n), name=f"{s.name}_w{n}")


def random_density(n, seed=3, sym=True):
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((n, max(2, n // 2)))
    d = c @ c.T
    if not sym:
        d = d + 0.3 * rng.standard_normal((n, n))
    return d
