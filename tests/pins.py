"""Independent references used to pin the oracle (test-only, NumPy).

None of these shares code with the oracle or the HIP path:

* ``brute_chi`` / ``brute_rho`` / ``brute_mat``: the periodic orbitals
  chi_mu(r) = sum_T phi_mu(r - T) evaluated on the grid without any truncation,
  then rho = sum D chi chi and M = w chi^T diag(v) chi.  At the Gamma point the
  double lattice sum of Eq. (rho) factorises this way (Sec. II).
* ``overlap`` / ``overlap_grad``: periodic overlap S_{mu nu} = sum_T int phi_mu
  phi_nu(. - T) and its derivative with respect to atom positions, from the
  closed-form Gaussian moments (binomial expansion about the product centre;
  textbook Gaussian integrals).  On a grid fine enough that the quadrature
  error exp(-pi^2 / (alpha h^2)) is negligible, M(v = 1) = S and
  sum_r w rho(r) = Tr(D S).
* ``theta_sum``: the exact grid sum of a 1-D Gaussian by Poisson summation,
  sum_j exp(-a (j h - P)^2) = (1/h) sqrt(pi/a) sum_m exp(-pi^2 m^2 / (a h^2))
  cos(2 pi m P / h), valid on coarse grids where aliasing matters.
"""
from __future__ import annotations

import math

import numpy as np


def cart_list(l):
    """Cartesian exponents of a shell, lexicographic (lx desc, then ly desc)."""
    out = []
    for x in range(l, -1, -1):
        for y in range(l - x, -1, -1):
            out.append((x, y, l - x - y))
    return out


def lattice(cell):
    """Lattice vectors as rows (3 x 3) of a (3,) orthorhombic cell or a 3 x 3 matrix."""
    cell = np.asarray(cell, dtype=np.float64)
    return np.diag(cell) if cell.shape == (3,) else cell


def _images(cell, nimg):
    r = range(-nimg, nimg + 1)
    a = lattice(cell)
    return [np.array([i, j, k], dtype=np.float64) @ a for i in r for j in r for k in r]


def grid_points(cell, mesh):
    """Points of the C-ordered grid: r = sum_d (i_d / N_d) a_d."""
    a = lattice(cell)
    n = np.asarray(mesh)
    ax = [np.arange(n[d]) / n[d] for d in range(3)]
    U = np.stack(np.meshgrid(*ax, indexing="ij"), axis=-1).reshape(-1, 3)
    return U @ a


def brute_chi(sys, mesh, nimg=2):
    """chi[mu, point] on the C-ordered grid of ``mesh`` (no truncation)."""
    cell = np.asarray(sys.cell, dtype=np.float64)
    pts = grid_points(cell, mesh)
    chis = []
    for s in range(sys.nshell):
        l = int(sys.shell_l[s])
        A = sys.coords[sys.shell_atom[s]]
        p0, npr = int(sys.shell_prim0[s]), int(sys.shell_nprim[s])
        comps = cart_list(l)
        acc = np.zeros((len(comps), pts.shape[0]))
        for T in _images(cell, nimg):
            d = pts - (A + T)
            r2 = np.einsum("ij,ij->i", d, d)
            rad = np.zeros(pts.shape[0])
            for k in range(npr):
                rad += sys.coefs[p0 + k] * np.exp(-sys.exps[p0 + k] * r2)
            for c, (ix, iy, iz) in enumerate(comps):
                acc[c] += d[:, 0] ** ix * d[:, 1] ** iy * d[:, 2] ** iz * rad
        chis.append(acc)
    return np.concatenate(chis, axis=0)


def brute_rho(chi, D, mesh):
    return np.einsum("mp,mn,np->p", chi, D, chi).reshape(tuple(mesh))


def brute_mat(chi, v, w):
    return w * (chi * v.ravel()[None, :]) @ chi.T


# ------------------------------------------------------------ closed forms

def _moment(n, p):
    """int t^n exp(-p t^2) dt over the real line."""
    if n % 2:
        return 0.0
    return math.gamma((n + 1) / 2.0) / p ** ((n + 1) / 2.0)


def _int1d(i, j, A, B, a, b):
    """int (x-A)^i (x-B)^j exp(-a (x-A)^2 - b (x-B)^2) dx."""
    p = a + b
    P = (a * A + b * B) / p
    pre = math.exp(-a * b / p * (A - B) ** 2)
    tot = 0.0
    for k in range(i + 1):
        for m in range(j + 1):
            tot += (math.comb(i, k) * (P - A) ** (i - k) * math.comb(j, m) * (P - B) ** (j - m)
                    * _moment(k + m, p))
    return pre * tot


def _prims(sys):
    out = []
    for s in range(sys.nshell):
        p0, npr = int(sys.shell_prim0[s]), int(sys.shell_nprim[s])
        out.append([(sys.exps[p0 + k], sys.coefs[p0 + k]) for k in range(npr)])
    return out


def overlap(sys, nimg=3):
    """Periodic overlap S (n_ao x n_ao) in the contracted Cartesian basis."""
    off = sys.ao_offsets()
    prims = _prims(sys)
    n = sys.n_ao
    S = np.zeros((n, n))
    cell = np.asarray(sys.cell, dtype=np.float64)
    for a in range(sys.nshell):
        A = sys.coords[sys.shell_atom[a]]
        ca = cart_list(int(sys.shell_l[a]))
        for b in range(sys.nshell):
            B0 = sys.coords[sys.shell_atom[b]]
            cb = cart_list(int(sys.shell_l[b]))
            for T in _images(cell, nimg):
                B = B0 + T
                for (ea, wa) in prims[a]:
                    for (eb, wb) in prims[b]:
                        for i, (ix, iy, iz) in enumerate(ca):
                            for j, (jx, jy, jz) in enumerate(cb):
                                S[off[a] + i, off[b] + j] += wa * wb * (
                                    _int1d(ix, jx, A[0], B[0], ea, eb) *
                                    _int1d(iy, jy, A[1], B[1], ea, eb) *
                                    _int1d(iz, jz, A[2], B[2], ea, eb))
    return S


def _dint1d_dA(i, j, A, B, a, b):
    """d/dA of int (x-A)^i (x-B)^j exp(-a (x-A)^2 - b (x-B)^2) dx
    = int [-i (x-A)^(i-1) + 2 a (x-A)^(i+1)] (x-B)^j ... dx."""
    v = 2.0 * a * _int1d(i + 1, j, A, B, a, b)
    if i > 0:
        v -= i * _int1d(i - 1, j, A, B, a, b)
    return v


def overlap_grad(sys, D, nimg=3):
    """g_X = sum_{mu nu} D_{mu nu} dS_{mu nu}/dR_X (natm x 3), both factors."""
    off = sys.ao_offsets()
    prims = _prims(sys)
    g = np.zeros((sys.natm, 3))
    cell = np.asarray(sys.cell, dtype=np.float64)
    for a in range(sys.nshell):
        ia = int(sys.shell_atom[a])
        A = sys.coords[ia]
        ca = cart_list(int(sys.shell_l[a]))
        for b in range(sys.nshell):
            ib = int(sys.shell_atom[b])
            B0 = sys.coords[ib]
            cb = cart_list(int(sys.shell_l[b]))
            for T in _images(cell, nimg):
                B = B0 + T
                for (ea, wa) in prims[a]:
                    for (eb, wb) in prims[b]:
                        for i, pa in enumerate(ca):
                            for j, pb in enumerate(cb):
                                dij = D[off[a] + i, off[b] + j] * wa * wb
                                if dij == 0.0:
                                    continue
                                vals = [_int1d(pa[d], pb[d], A[d], B[d], ea, eb) for d in range(3)]
                                for d in range(3):
                                    dA = _dint1d_dA(pa[d], pb[d], A[d], B[d], ea, eb)
                                    dB = _dint1d_dA(pb[d], pa[d], B[d], A[d], eb, ea)
                                    rest = 1.0
                                    for e in range(3):
                                        if e != d:
                                            rest *= vals[e]
                                    g[ia, d] += dij * dA * rest
                                    g[ib, d] += dij * dB * rest
    return g


def theta_sum(a, h, P, mmax=40):
    """sum over all integers j of exp(-a (j h - P)^2), by Poisson summation."""
    m = np.arange(1, mmax + 1)
    return (1.0 / h) * math.sqrt(math.pi / a) * (
        1.0 + 2.0 * np.sum(np.exp(-math.pi ** 2 * m ** 2 / (a * h * h)) * np.cos(2.0 * math.pi * m * P / h)))


def theta_mat_ones(sys, mesh, nimg=3):
    """M(v = 1) for an s-only system on a (possibly coarse) grid: for each
    pair image, w * c_a c_b exp(-mu |A-B-T|^2) * prod_d theta_sum(alpha_p, h_d, P_d)."""
    assert all(int(l) == 0 for l in sys.shell_l)
    cell = np.asarray(sys.cell, dtype=np.float64)
    h = cell / np.asarray(mesh)
    w = float(np.prod(cell)) / float(np.prod(mesh))
    prims = _prims(sys)
    n = sys.nshell
    M = np.zeros((n, n))
    for a in range(n):
        A = sys.coords[sys.shell_atom[a]]
        for b in range(n):
            B0 = sys.coords[sys.shell_atom[b]]
            for T in _images(cell, nimg):
                B = B0 + T
                for (ea, wa) in prims[a]:
                    for (eb, wb) in prims[b]:
                        p = ea + eb
                        P = (ea * A + eb * B) / p
                        K = wa * wb * math.exp(-ea * eb / p * float(np.sum((A - B) ** 2)))
                        M[a, b] += w * K * np.prod([theta_sum(p, h[d], P[d]) for d in range(3)])
    return M


# ------------------------------------------------ kinetic energy density pins

def brute_grad_chi(sys, mesh, nimg=2):
    """grad chi[d, mu, point] on the C-ordered grid (no truncation): the
    r-derivative of x^i y^j z^k exp(-a r^2) is (i x^(i-1) - 2 a x^(i+1)) y^j z^k
    exp(-a r^2) along x, lattice-summed like ``brute_chi``."""
    cell = np.asarray(sys.cell, dtype=np.float64)
    pts = grid_points(cell, mesh)
    out = []
    for s in range(sys.nshell):
        l = int(sys.shell_l[s])
        A = sys.coords[sys.shell_atom[s]]
        p0, npr = int(sys.shell_prim0[s]), int(sys.shell_nprim[s])
        comps = cart_list(l)
        acc = np.zeros((3, len(comps), pts.shape[0]))
        for T in _images(cell, nimg):
            d = pts - (A + T)
            r2 = np.einsum("ij,ij->i", d, d)
            for k in range(npr):
                a, c = sys.exps[p0 + k], sys.coefs[p0 + k]
                e = c * np.exp(-a * r2)
                for m, pw in enumerate(comps):
                    for ax_ in range(3):
                        term = np.ones(pts.shape[0])
                        for q in range(3):
                            if q == ax_:
                                f = -2.0 * a * d[:, q] ** (pw[q] + 1)
                                if pw[q] > 0:
                                    f = f + pw[q] * d[:, q] ** (pw[q] - 1)
                                term = term * f
                            else:
                                term = term * d[:, q] ** pw[q]
                        acc[ax_, m] += term * e
        out.append(acc)
    return np.concatenate(out, axis=1)


def brute_tau(gchi, D, mesh):
    """tau = 1/2 sum_d sum_{mu nu} D_{mu nu} d_d chi_mu d_d chi_nu."""
    return 0.5 * np.einsum("dmp,mn,dnp->p", gchi, D, gchi).reshape(tuple(mesh))


def brute_mat_tau(gchi, v, w):
    """M_tau = 1/2 w sum_d (d_d chi) diag(v) (d_d chi)^T."""
    vv = v.ravel()[None, :]
    return 0.5 * w * sum((gchi[d] * vv) @ gchi[d].T for d in range(3))


def _dint1d(i, j, A, B, a, b):
    """int d/dx[(x-A)^i e^(-a(x-A)^2)] d/dx[(x-B)^j e^(-b(x-B)^2)] dx, each
    derivative being i (x-A)^(i-1) e - 2a (x-A)^(i+1) e."""
    def terms(k, c):
        t = [(k + 1, -2.0 * c)]
        if k > 0:
            t.append((k - 1, float(k)))
        return t
    return sum(ca * cb * _int1d(p, q, A, B, a, b) for (p, ca) in terms(i, a) for (q, cb) in terms(j, b))


def kinetic(sys, nimg=3):
    """Periodic kinetic matrix T_{mu nu} = 1/2 sum_T int grad phi_mu . grad phi_nu(. - T),
    from closed-form 1-D Gaussian integrals."""
    off = sys.ao_offsets()
    prims = _prims(sys)
    n = sys.n_ao
    T_ = np.zeros((n, n))
    cell = np.asarray(sys.cell, dtype=np.float64)
    for a in range(sys.nshell):
        A = sys.coords[sys.shell_atom[a]]
        ca = cart_list(int(sys.shell_l[a]))
        for b in range(sys.nshell):
            B0 = sys.coords[sys.shell_atom[b]]
            cb = cart_list(int(sys.shell_l[b]))
            for Tv in _images(cell, nimg):
                B = B0 + Tv
                for (ea, wa) in prims[a]:
                    for (eb, wb) in prims[b]:
                        for i, pa in enumerate(ca):
                            for j, pb in enumerate(cb):
                                s1 = [_int1d(pa[d], pb[d], A[d], B[d], ea, eb) for d in range(3)]
                                k1 = [_dint1d(pa[d], pb[d], A[d], B[d], ea, eb) for d in range(3)]
                                T_[off[a] + i, off[b] + j] += 0.5 * wa * wb * (
                                    k1[0] * s1[1] * s1[2] + s1[0] * k1[1] * s1[2] + s1[0] * s1[1] * k1[2])
    return T_


def kinetic_grad(sys, D, nimg=3, h=1e-4):
    """sum_{mu nu} D_{mu nu} dT_{mu nu}/dR_X by central differences of the
    closed-form T (natm x 3); the closed form is smooth, so h = 1e-4 gives ~1e-9."""
    import copy
    g = np.zeros((sys.natm, 3))
    for X in range(sys.natm):
        for d in range(3):
            vals = []
            for sgn in (1.0, -1.0):
                s2 = copy.copy(sys)
                s2.coords = sys.coords.copy()
                s2.coords[X, d] += sgn * h
                vals.append(float(np.sum(D * kinetic(s2, nimg))))
            g[X, d] = (vals[0] - vals[1]) / (2 * h)
    return g
