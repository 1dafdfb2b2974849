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

Readings where the paper is silent or ambiguous:

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
* R16 acceleration at the outer faces of the coarsest grid: the paper takes
  boundary potentials there from the analytic solution (Sect. 2, OiCG
  tests); the convolution method has no ghost values, so the second-order
  one-sided difference is used on those faces.
* R18 modified (dipole-preserving) method, Sect. 7 and Appendix B: the
  doubled grid of the pair (n, n+1) is level n+1's (restricted) density
  embedded at the centre of a grid of 2N cells of level n+1's spacing, which
  spans level n; its potential is brought to level n's cells ("tilde",
  fine to coarse) as the mean over the 2^3 fine cells each coarse cell
  covers, the same averaging as the acceleration's method B.
* R20 three-level dipole scheme, Appendix B (the equations for dipoles
  across three neighbouring grids): for a level n with two finer levels,
  the doubled grid holds level n+1's density with its own child region
  zeroed (the "dbl,hole" grid, so that level n+2's mass is not counted
  twice), and the quadrupled grid holds level n+2's (restricted) density
  centred in 4N cells of level n+2's spacing spanning level n, reduced by
  the mean over the 4^3 cells each level-n cell covers.  The second finest
  level keeps the pairwise doubled grid, the finest its own full grid.
* R17 acceleration at covered cells (inside the child region) uses the
  level's own potential; method B applies to coarse cells outside the child
  region whose stencil neighbour lies inside it.
"""
from __future__ import annotations

import functools
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
    w = _workers()
    Fm = scipy.fft.rfftn(np.asarray(mass, dtype=np.float64), s=(P, P, P), workers=w)  # zero-padded to P^3
    Fm *= _green_spectrum(P)
    conv = scipy.fft.irfftn(Fm, s=(P, P, P), workers=w, overwrite_x=True)
    return -(G / h) * conv[:N, :N, :N]


@functools.lru_cache(maxsize=2)
def _green_spectrum(P: int) -> np.ndarray:
    """FFT(g) of green_periodic(P), kept for the next grid of the same
    period (the same array every time; read-only)."""
    Fg = scipy.fft.rfftn(green_periodic(P), workers=_workers())
    Fg.setflags(write=False)
    return Fg


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


def doubled_potential(mass_fine: np.ndarray, h_fine: float, G: float = 1.0, method: str = "fft") -> np.ndarray:
    """Sect. 7 (Fig. 16, Eq. 15) and Appendix B: the potential of a fine
    level's masses on its doubled grid (2N cells of the fine spacing covering
    the next coarser level, the masses in the central N^3, zeros around),
    reduced to the coarser level's N^3 cells by the mean over the 2^3 fine
    cells each covers (reading R18)."""
    N = mass_fine.shape[0]
    Md = np.zeros((2 * N, 2 * N, 2 * N), dtype=np.float64)
    a, b = N // 2, 3 * N // 2
    Md[a:b, a:b, a:b] = mass_fine
    Pd = _single_grid(method)(Md, h_fine, G)
    return Pd.reshape(N, 2, N, 2, N, 2).mean(axis=(1, 3, 5))


def quadrupled_potential(mass_fine: np.ndarray, h_fine: float, G: float = 1.0, method: str = "fft") -> np.ndarray:
    """Reduced potential of the quadrupled grid of Appendix B (three-level
    scheme): the masses of level n+2 (N^3 cells of spacing h_fine) placed at
    cells [3N/2, 5N/2) per axis of a grid of 4N cells of that spacing, which
    spans level n, zeros around; reduced to level n's N^3 cells by the mean
    over the 4^3 fine cells each covers (reading R20)."""
    N = mass_fine.shape[0]
    Mq = np.zeros((4 * N, 4 * N, 4 * N), dtype=np.float64)
    a, b = 3 * N // 2, 5 * N // 2
    Mq[a:b, a:b, a:b] = mass_fine
    Pq = _single_grid(method)(Mq, h_fine, G)
    return Pq.reshape(N, 4, N, 4, N, 4).mean(axis=(1, 3, 5))


def scaled_potential_at(mass_fine: np.ndarray, h_fine: float, S: int, cells, G: float = 1.0) -> np.ndarray:
    """The reduced potential of a scaled grid at selected coarse cells, by
    direct summation (the point form of doubled_potential, S = 2, and
    quadrupled_potential, S = 4; readings R18, R20): the fine masses sit at
    cells [(S-1) N/2, (S+1) N/2) per axis of a grid of S N cells of the fine
    spacing spanning the coarse level, and coarse cell c = (z, y, x) takes
    the mean of Eq. (10) over its S^3 fine cells S c + (0..S-1)^3."""
    N = mass_fine.shape[0]
    off = (S - 1) * N // 2
    nz = np.nonzero(mass_fine)
    m = mass_fine[nz]
    sz, sy, sx = (a.astype(np.float64) + off for a in nz)
    out = np.empty(len(cells), dtype=np.float64)
    for k, (z, y, x) in enumerate(np.asarray(cells)):
        acc = 0.0
        for oz in range(S):
            for oy in range(S):
                for ox in range(S):
                    tz, ty, tx = S * z + oz, S * y + oy, S * x + ox
                    r2 = (sz - tz) ** 2 + (sy - ty) ** 2 + (sx - tx) ** 2
                    with np.errstate(divide="ignore"):
                        gv = 1.0 / np.sqrt(r2)
                    gv[r2 == 0] = BETA
                    acc += float(np.dot(gv, m))
        out[k] = -(G / h_fine) * acc / S ** 3
    return out


def solve_modified(rho: np.ndarray, h0: float, G: float = 1.0, *, restrict: bool = True,
                   method: str = "fft", scheme: str = "pairs", trilinear: bool = False) -> np.ndarray:
    """The modified convolution method that keeps the dipole moments across
    every pair of neighbouring grids (Sect. 7, Appendix B, Eqs. B.1-B.2):
    Phi(Omega^n) = Phi^n_hole + ~Phi^{n+1}_dbl + (hole potentials of the
    coarser grids carried down, as in Eq. 14) for every level but the
    finest, which is Phi^L + the carried hole potentials.  The coarse grid
    thus sees the finer level's masses at the finer resolution instead of
    their restriction, so opposite charges inside one coarse cell no longer
    cancel (Sect. 7, Fig. 15).

    scheme="triples" is Appendix B's scheme for dipoles across three
    neighbouring grids: a level n with two finer levels takes
    Phi^n_hole + ~Phi^{n+1}_{dbl,hole} + ~Phi^{n+2}_{qdp} + the carry
    (reading R20); the other levels are as in "pairs"."""
    if scheme not in ("pairs", "triples"):
        raise ValueError("scheme must be 'pairs' or 'triples'")
    rho = np.asarray(rho, dtype=np.float64)
    L, N = rho.shape[0], rho.shape[1]
    if N % 4:
        raise ValueError("N must be a multiple of 4")
    conv = _single_grid(method)
    rr = restrict_cascade(rho) if restrict else rho.copy()
    phi = np.empty((L, N, N, N), dtype=np.float64)
    S = None
    for n in range(L):
        h = level_spacing(h0, n)
        M = rr[n] * h ** 3
        A = (prolong_trilinear(S) if trilinear else prolong(S)) if n > 0 else 0.0
        if n < L - 1:
            hole_n = conv(hole(M), h, G)
            hf = level_spacing(h0, n + 1)
            if scheme == "triples" and n < L - 2:
                hq = level_spacing(h0, n + 2)
                phi[n] = (hole_n + doubled_potential(hole(rr[n + 1] * hf ** 3), hf, G, method)
                          + quadrupled_potential(rr[n + 2] * hq ** 3, hq, G, method) + A)
            else:
                phi[n] = hole_n + doubled_potential(rr[n + 1] * hf ** 3, hf, G, method) + A
            S = A + hole_n
        else:
            phi[n] = conv(M, h, G) + A
    return phi


def solve_points(rho: np.ndarray, h0: float, pts, G: float = 1.0, *, restrict: bool = True,
                 trilinear: bool = False, scheme: str = "original") -> np.ndarray:
    """Phi(Omega^(l+1)) at selected cells pts[k] = (l, z, y, x), each by
    direct summation of Eq. (10) on every grid involved and the same carry
    rule as solve() (for spot checks at sizes where the full oracle is slow).
    The carry is written out per cell here (parent and neighbour per axis),
    independently of prolong() / prolong_trilinear().

    scheme "pairs" / "triples" gives solve_modified's levels instead: a
    level with a finer one takes its hole potential plus the reduced
    doubled-grid potential of the next level (with that level's child
    region zeroed when a quadrupled grid of the level after it is added,
    "triples"), by scaled_potential_at; the carry is the same."""
    if scheme not in ("original", "pairs", "triples"):
        raise ValueError("scheme must be 'original', 'pairs' or 'triples'")
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
        pc = [(N // 4 + f // 2, 1 if f % 2 == 1 else -1) for f in p]  # parent, direction per axis
        out = 0.0
        if not trilinear:  # along the diagonal: all axes at the parent, or all at the neighbour
            for w, off in ((0.75, 0), (0.25, 1)):
                out += w * S_at(n - 1, tuple(c + off * d for c, d in pc))
            return out
        for oz in (0, 1):  # every corner of the 2^3 block, 3/4 or 1/4 per axis
            for oy in (0, 1):
                for ox in (0, 1):
                    w = 1.0
                    for o in (oz, oy, ox):
                        w *= 0.25 if o else 0.75
                    q = tuple(c + o * d for (c, d), o in zip(pc, (oz, oy, ox)))
                    out += w * S_at(n - 1, q)
        return out

    def S_at(m, p):  # S_m = A_m + Phi^m_hole, with A_0 = 0
        v = phi_grid(m, True, p)
        if m > 0:
            v += carry(m, p)
        return v

    def level_value(l, p):
        if scheme == "original" or l == L - 1:
            return phi_grid(l, False, p)
        hf = level_spacing(h0, l + 1)
        triple = scheme == "triples" and l < L - 2
        fine = rr[l + 1] * hf ** 3
        v = phi_grid(l, True, p) + scaled_potential_at(hole(fine) if triple else fine, hf, 2, [p], G)[0]
        if triple:
            hq = level_spacing(h0, l + 2)
            v += scaled_potential_at(rr[l + 2] * hq ** 3, hq, 4, [p], G)[0]
        return v

    res = []
    for (l, z, y, x) in pts:
        v = level_value(l, (z, y, x))
        if l > 0:
            v += carry(l, (z, y, x))
        res.append(v)
    return np.array(res)


# ---------------------------------------------------------------------------
# Gravitational acceleration (Sect. 2, the six-point central stencil for
# g = -grad Phi, and Appendix A for the cells next to a coarse-fine
# interface).


def _ghost_from_coarse(Pc: np.ndarray, fz, fy, fx) -> np.ndarray:
    """Potential at fine cells (fz, fy, fx) of the next finer level, which may
    lie one cell outside that level, from the coarse level's potential Pc by
    the diagonal 3/4-1/4 rule of Eqs. (3)-(6): per axis the parent
    c = N/4 + floor(f/2) and the neighbour c + s, s = +1 for odd f, -1 for
    even f."""
    N = Pc.shape[0]

    def axis(f):
        f = np.asarray(f)
        c = N // 4 + np.floor_divide(f, 2)
        s = np.where(np.mod(f, 2) == 1, 1, -1)
        return c, c + s

    cz, sz = axis(fz)
    cy, sy = axis(fy)
    cx, sx = axis(fx)
    return 0.75 * Pc[cz, cy, cx] + 0.25 * Pc[sz, sy, sx]


def acceleration(phi: np.ndarray, h0: float) -> np.ndarray:
    """g = -grad Phi on every level of a nested mesh, shape [L, 3, N, N, N]
    with components (g_x, g_y, g_z) and x the fastest array axis.

    Interior cells: g_x = -(Phi[i+1] - Phi[i-1]) / (2 dx) (Sect. 2).
    Appendix A, method A: at a level's outermost cells (level >= 1) the
    missing neighbour is the boundary value interpolated from the next
    coarser level by Eqs. (3)-(6).  Method B: at a coarse cell next to the
    finer grid, a neighbour inside the child region takes the arithmetic
    mean of the finer level's potential over the 2^3 cells it covers.  The
    coarsest level's outer faces use the second-order one-sided difference
    (reading R16); covered cells use the level's own values (reading R17)."""
    phi = np.asarray(phi, dtype=np.float64)
    L, N = phi.shape[0], phi.shape[1]
    lo, hi = N // 4, 3 * N // 4
    out = np.zeros((L, 3, N, N, N), dtype=np.float64)
    idx = np.arange(N)
    Z, Y, X = np.meshgrid(idx, idx, idx, indexing="ij")
    inside = (Z >= lo) & (Z < hi) & (Y >= lo) & (Y < hi) & (X >= lo) & (X < hi)
    for l in range(L):
        h = level_spacing(h0, l)
        P = phi[l]
        mean_fine = None
        if l + 1 < L:
            n2 = N // 2
            mean_fine = phi[l + 1].reshape(n2, 2, n2, 2, n2, 2).mean(axis=(1, 3, 5))
        for comp, ax in ((0, 2), (1, 1), (2, 0)):
            vals = []
            for step in (+1, -1):
                nb = [Z.copy(), Y.copy(), X.copy()]
                nb[ax] = nb[ax] + step
                inrange = (nb[ax] >= 0) & (nb[ax] < N)
                cl = [np.clip(a, 0, N - 1) for a in nb]
                v = P[cl[0], cl[1], cl[2]]
                if l >= 1:  # method A: boundary value from the coarser level
                    ghost = np.zeros_like(v)
                    m = ~inrange
                    ghost[m] = _ghost_from_coarse(phi[l - 1], nb[0][m], nb[1][m], nb[2][m])
                    v = np.where(inrange, v, ghost)
                if mean_fine is not None:  # method B
                    nb_in = inrange & (cl[0] >= lo) & (cl[0] < hi) & (cl[1] >= lo) & (cl[1] < hi) & \
                        (cl[2] >= lo) & (cl[2] < hi)
                    use = nb_in & ~inside
                    mf = mean_fine[np.clip(cl[0] - lo, 0, N // 2 - 1), np.clip(cl[1] - lo, 0, N // 2 - 1),
                                   np.clip(cl[2] - lo, 0, N // 2 - 1)]
                    v = np.where(use, mf, v)
                vals.append(v)
            g = -(vals[0] - vals[1]) / (2.0 * h)
            if l == 0:  # outer faces of the coarsest grid: one-sided (R16)
                sl0 = [slice(None)] * 3
                sl1 = [slice(None)] * 3
                sl2 = [slice(None)] * 3
                sl0[ax], sl1[ax], sl2[ax] = 0, 1, 2
                g[tuple(sl0)] = -(-3.0 * P[tuple(sl0)] + 4.0 * P[tuple(sl1)] - P[tuple(sl2)]) / (2.0 * h)
                sl0[ax], sl1[ax], sl2[ax] = N - 1, N - 2, N - 3
                g[tuple(sl0)] = -(3.0 * P[tuple(sl0)] - 4.0 * P[tuple(sl1)] + P[tuple(sl2)]) / (2.0 * h)
            out[l, comp] = g
    return out
