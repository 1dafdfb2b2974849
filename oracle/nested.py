"""FP64 CPU oracle for the nested-mesh convolution method.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
link this module: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (no kernels, tables, constants or helpers); it takes plain NumPy
arrays and returns plain NumPy arrays.

Paper: Vorobyov, McKevitt, Kulikov, Elbakyan, "Computing the gravitational
potential on nested meshes using the convolution method" (A&A 2023,
arXiv:2301.06763).

What is computed (paper notation: level m = 1..L, coarsest first; here the
array index l = m - 1):

* Sect. 3, Eq. (10): Phi(t) = -G sum_s M(s) Gfun(r_t - r_s), with cell masses
  M = rho h^3 and Gfun the inverse distance between cell centres.
* Sect. 3, Eq. (13): the cell's own contribution, for constant density in a
  cube of side h, is -G rho h^2 beta with beta the integral of 1/r over the
  unit cube centred on the origin.
* Sect. 3 (domain doubling, Fig. 4): the sum of Eq. (10) equals a circular
  convolution on a doubled, zero-padded periodic mesh, evaluated with FFTs
  (Eq. 11 and the text after it).
* Sect. 4 (Fig. 5, Eq. 14): the nested mesh is split into full grids
  Omega^m and grids with a central cavity Omega^m_hole; the potential on
  Omega^n is Phi^n plus the hole potentials of all coarser grids interpolated
  onto it.

Readings where the paper is silent or ambiguous (listed in the design doc too):

* R1 self-cell value: beta = 3 ln(2 + sqrt 3) - pi/2 (closed form of Eq. 13).
* R2 off-diagonal kernel: point-to-point 1/|r_t - r_s| between centres.
* R4 the doubled-mesh Green function at offset N (wrapped index) is 1/N so
  that it is even; it never reaches an output cell.
* R5 padding: P = 2N here (the HIP path may use any P >= 2N - 1).
* R8 restriction: the coarse density under a finer grid is replaced by the
  mean of its 2^3 children, cascaded from the finest grid up (switchable).
* R9 cavity: level m+1 covers level-m cells [N/4, 3N/4) on each axis.
* R10 interpolation of the hole potential onto fine cells: the diagonal
  3/4-1/4 rule of Sect. 2, Eqs. (3)-(6), applied to every fine cell:
  parent c = N/4 + floor(f/2), neighbour offset s = +1 for odd f, -1 for
  even f, per axis; A(f) = 3/4 S(c) + 1/4 S(c + s) (c, s 3-vectors).
* R11 carry: cascaded, A_n = Prolong(A_{n-1} + Phi^{n-1}_hole).
"""
from __future__ import annotations

import math
import os

import numpy as np
import scipy.fft

# ---------------------------------------------------------------------------
# Sect. 3, Eq. (13): integral of 1/r over the unit cube centred on the origin
# (closed form; reading R1).  Pinned in tests against an independent
# quadrature of the same integral.
BETA = 3.0 * math.log(2.0 + math.sqrt(3.0)) - math.pi / 2.0


def _workers() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def cell_centres(N: int, h: float) -> np.ndarray:
    """Centres of the N cells of a level of spacing h, centred on the origin
    (Sect. 2, Fig. 1: concentric nested grids of N cells, side N h)."""
    return (np.arange(N, dtype=np.float64) - N / 2 + 0.5) * h


def level_spacing(h0: float, l: int) -> float:
    """Cell size of level l (0-based): each finer grid halves the spacing
    (Sect. 2: dx_m = (w_R - w_L) / (2^(m-1) N))."""
    return h0 / (2.0 ** l)


# ---------------------------------------------------------------------------
# Green function on the doubled periodic mesh (Sect. 3, Fig. 4; readings R1,
# R2, R4).

def green_periodic(P: int) -> np.ndarray:
    """Inverse distance in cell units between a cell and every cell of a
    P^3 periodic mesh, arranged periodically (offset d and P - d are the
    same distance); the zero offset holds beta (Eq. 13)."""
    i = np.arange(P)
    d = np.minimum(i, P - i).astype(np.float64)
    r2 = d[:, None, None] ** 2 + d[None, :, None] ** 2 + d[None, None, :] ** 2
    with np.errstate(divide="ignore"):
        g = 1.0 / np.sqrt(r2)
    g[0, 0, 0] = BETA
    return g


def kernel_value(dz, dy, dx):
    """Gfun of Eq. (10) in cell units for integer offsets (arrays):
    1/|d| off the diagonal, beta at d = 0."""
    r2 = (np.asarray(dz, dtype=np.float64) ** 2 + np.asarray(dy, dtype=np.float64) ** 2
          + np.asarray(dx, dtype=np.float64) ** 2)
    out = np.empty_like(r2)
    nz = r2 > 0
    out[nz] = 1.0 / np.sqrt(r2[nz])
    out[~nz] = BETA
    return out


# ---------------------------------------------------------------------------
# One regular grid (Sect. 3).

def potential_fft(mass: np.ndarray, h: float, G: float = 1.0, P: int | None = None) -> np.ndarray:
    """Potential of cell masses on one N^3 grid of spacing h, by the
    zero-padded periodic convolution of Sect. 3 (Eq. 11, Fig. 4), FP64.

    Phi = -(G/h) * IFFT( FFT(M padded to P^3) * FFT(g) ) restricted to the
    original N^3 cells.  P defaults to 2N (the paper's doubling)."""
    N = mass.shape[0]
    assert mass.shape == (N, N, N)
    if P is None:
        P = 2 * N
    assert P >= 2 * N - 1
    g = green_periodic(P)
    Mp = np.zeros((P, P, P), dtype=np.float64)
    Mp[:N, :N, :N] = mass
    w = _workers()
    Fm = scipy.fft.rfftn(Mp, workers=w)
    Fg = scipy.fft.rfftn(g, workers=w)
    conv = scipy.fft.irfftn(Fm * Fg, s=(P, P, P), workers=w)
    return -(G / h) * conv[:N, :N, :N]


def potential_direct(mass: np.ndarray, h: float, G: float = 1.0) -> np.ndarray:
    """Brute-force O(N^6) evaluation of Eq. (10) on one grid (no FFT)."""
    N = mass.shape[0]
    idx = np.arange(N)
    zz, yy, xx = np.meshgrid(idx, idx, idx, indexing="ij")
    pts = np.stack([zz.ravel(), yy.ravel(), xx.ravel()], axis=1)
    m = mass.ravel()
    out = np.empty(N ** 3, dtype=np.float64)
    chunk = max(1, 2_000_000 // max(1, N ** 3))
    for a in range(0, N ** 3, chunk):
        t = pts[a:a + chunk]
        d = t[:, None, :] - pts[None, :, :]
        gv = kernel_value(d[..., 0], d[..., 1], d[..., 2])
        out[a:a + chunk] = gv @ m
    return (-(G / h) * out).reshape(N, N, N)


def potential_at(mass: np.ndarray, h: float, pts: np.ndarray, G: float = 1.0) -> np.ndarray:
    """Eq. (10) evaluated by direct summation at selected integer cell
    indices pts[k] = (z, y, x) of the same grid (any N)."""
    N = mass.shape[0]
    idx = np.arange(N, dtype=np.float64)
    out = np.empty(len(pts), dtype=np.float64)
    for k, (z, y, x) in enumerate(np.asarray(pts)):
        dz2 = (z - idx) ** 2
        dy2 = (y - idx) ** 2
        dx2 = (x - idx) ** 2
        r2 = dz2[:, None, None] + dy2[None, :, None] + dx2[None, None, :]
        with np.errstate(divide="ignore"):
            gv = 1.0 / np.sqrt(r2)
        gv[int(z), int(y), int(x)] = BETA
        out[k] = -(G / h) * np.einsum("ijk,ijk->", gv, mass)
    return out


# ---------------------------------------------------------------------------
# Nested coupling (Sect. 4; readings R8-R11).

def child_region(N: int) -> slice:
    """Cells of a level covered by the next finer level (reading R9)."""
    return slice(N // 4, 3 * N // 4)


def restrict_cascade(rho: np.ndarray) -> np.ndarray:
    """Replace, from the finest level up, the density of each level under
    the next finer level by the mean of its 2^3 children (reading R8; mass
    conserving).  rho has shape [L, N, N, N]; returns a new array."""
    out = np.array(rho, dtype=np.float64, copy=True)
    L, N = out.shape[0], out.shape[1]
    c = child_region(N)
    for l in range(L - 1, 0, -1):
        f = out[l]
        coarse = f.reshape(N // 2, 2, N // 2, 2, N // 2, 2).mean(axis=(1, 3, 5))
        out[l - 1][c, c, c] = coarse
    return out


def hole(x: np.ndarray) -> np.ndarray:
    """Omega_hole: the same grid with the density of the cavity zeroed
    (Sect. 4, Fig. 5)."""
    N = x.shape[0]
    c = child_region(N)
    y = np.array(x, copy=True)
    y[c, c, c] = 0.0
    return y


def _prolong_axis(N: int):
    f = np.arange(N)
    c = N // 4 + f // 2
    s = np.where(f % 2 == 1, 1, -1)
    return c, c + s


def prolong(S: np.ndarray) -> np.ndarray:
    """Interpolate a coarse-level field onto the N^3 cells of the next finer
    level with the diagonal 3/4-1/4 rule (Sect. 2, Eqs. 3-6, generalised to
    every fine cell; reading R10).  Reads S on [N/4-1, 3N/4]^3 only."""
    N = S.shape[0]
    c, cs = _prolong_axis(N)
    near = S[c[:, None, None], c[None, :, None], c[None, None, :]]
    far = S[cs[:, None, None], cs[None, :, None], cs[None, None, :]]
    return 0.75 * near + 0.25 * far


def prolong_trilinear(S: np.ndarray) -> np.ndarray:
    """Alternative carry rule: tensor-product linear interpolation with
    weights 3/4 and 1/4 per axis over the 8 surrounding coarse cells."""
    N = S.shape[0]
    c, cs = _prolong_axis(N)
    out = np.zeros((N, N, N), dtype=np.float64)
    for wz, iz in ((0.75, c), (0.25, cs)):
        for wy, iy in ((0.75, c), (0.25, cs)):
            for wx, ix in ((0.75, c), (0.25, cs)):
                out += wz * wy * wx * S[iz[:, None, None], iy[None, :, None], ix[None, None, :]]
    return out


def _single_grid(method: str):
    if method == "fft":
        return potential_fft
    if method == "direct":
        return potential_direct
    raise ValueError(method)


def solve(rho: np.ndarray, h0: float, G: float = 1.0, *, restrict: bool = True,
          trilinear: bool = False, method: str = "fft", return_parts: bool = False):
    """Potential on every level of a nested mesh (Sect. 4, Eq. 14).

    rho: [L, N, N, N] densities, level 0 = coarsest, index order [z][y][x].
    h0:  coarsest cell size; level l has h0 / 2^l.
    Returns phi [L, N, N, N]: phi[n] = Phi(Omega^(n+1)) on all N^3 cells.
    method: "fft" (the convolution method) or "direct" (Eq. 10 by brute force).
    """
    rho = np.asarray(rho, dtype=np.float64)
    L, N = rho.shape[0], rho.shape[1]
    if N % 4:
        raise ValueError("N must be a multiple of 4")
    conv = _single_grid(method)
    rr = restrict_cascade(rho) if restrict else rho.copy()
    full, holes = [], []
    for l in range(L):
        h = level_spacing(h0, l)
        M = rr[l] * h ** 3
        full.append(conv(M, h, G))
        if l < L - 1:
            holes.append(conv(hole(M), h, G))
    pro = prolong_trilinear if trilinear else prolong
    phi = np.empty((L, N, N, N), dtype=np.float64)
    phi[0] = full[0]
    S = holes[0] if L > 1 else None
    carries = [np.zeros((N, N, N))]
    for n in range(1, L):
        A = pro(S)
        carries.append(A)
        phi[n] = full[n] + A
        if n < L - 1:
            S = A + holes[n]
    if return_parts:
        return phi, dict(restricted=rr, full=full, holes=holes, carries=carries)
    return phi


def solve_points(rho: np.ndarray, h0: float, pts, G: float = 1.0, *, restrict: bool = True) -> np.ndarray:
    """Phi(Omega^(l+1)) at selected cells pts[k] = (l, z, y, x), each by
    direct summation of Eq. (10) on every grid involved and the same carry
    rule as solve() (for spot checks at sizes where the full oracle is slow).
    """
    rho = np.asarray(rho, dtype=np.float64)
    L, N = rho.shape[0], rho.shape[1]
    rr = restrict_cascade(rho) if restrict else rho
    masses = {}

    def mass(l, is_hole):
        key = (l, is_hole)
        if key not in masses:
            h = level_spacing(h0, l)
            M = rr[l] * h ** 3
            masses[key] = hole(M) if is_hole else M
        return masses[key]

    def phi_grid(l, is_hole, p):
        return potential_at(mass(l, is_hole), level_spacing(h0, l), np.array([p]), G)[0]

    def carry(n, p):  # A_n at cell p of level n (n >= 1)
        out = 0.0
        for w, off in ((0.75, 0), (0.25, 1)):
            q = []
            for f in p:
                c = N // 4 + f // 2
                s = 1 if f % 2 == 1 else -1
                q.append(c + off * s)
            out += w * S_at(n - 1, tuple(q))
        return out

    def S_at(m, p):  # S_m = A_m + Phi^m_hole, with A_0 = 0
        v = phi_grid(m, True, p)
        if m > 0:
            v += carry(m, p)
        return v

    res = []
    for (l, z, y, x) in pts:
        v = phi_grid(l, False, (z, y, x))
        if l > 0:
            v += carry(l, (z, y, x))
        res.append(v)
    return np.array(res)
