"""Seeded synthetic inputs for the stray-field operator.

This module only draws and shapes random numbers (NumPy PCG64 generators,
float64 on the host).  It holds none of the operator's arithmetic, so both the
GPU path's tests/benchmarks and the CPU reference implementation may use it.

Layout conventions (shared by every caller):
  * a full-format magnetization is an array ``m[3][nz][ny][nx]`` (x fastest,
    component index first), matching the column-major vec ordering of the
    Kronecker form ``A_z (x) A_y (x) A_x`` (Sec. 3, footnote of Cor. kron_op);
  * grid sizes are given as ``(nx, ny, nz)`` and cell sizes as ``(hx, hy, hz)``;
  * cell i along an axis has its midpoint at ``origin + (i + 1/2) h``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def _normalize(v: np.ndarray) -> np.ndarray:
    nrm = np.sqrt(np.sum(v * v, axis=0, keepdims=True))
    return v / nrm


def cell_centres(n: int, h: float, origin: float) -> np.ndarray:
    """Midpoints of n cells of width h starting at ``origin``."""
    return origin + (np.arange(n, dtype=np.float64) + 0.5) * h


def random_unit_field(n, seed: int = 0) -> np.ndarray:
    """Independent unit vectors per cell: Gaussian 3-vectors normalised.

    ``n`` is an int (cube) or a triple (nx, ny, nz).  Returns m[3][nz][ny][nx].
    """
    nx, ny, nz = (n, n, n) if np.isscalar(n) else tuple(n)
    g = _rng(seed).standard_normal((3, nz, ny, nx))
    return _normalize(g)


def uniform_field(n, axis: int = 2) -> np.ndarray:
    """Uniform magnetization along ``axis`` (0=x, 1=y, 2=z)."""
    nx, ny, nz = (n, n, n) if np.isscalar(n) else tuple(n)
    m = np.zeros((3, nz, ny, nx))
    m[axis] = 1.0
    return m


def vortex_field(n: int = 128, seed: int = 0, noise: float = 0.05) -> np.ndarray:
    """Smooth vortex on [-1/2, 1/2]^3 plus seeded Gaussian noise, renormalised.

    v = (-y, x, 0.2 exp(-r^2/0.05)) with the cylindrical radius r^2 = x^2 + y^2;
    m = normalise(normalise(v) + noise * N(0, 1)).
    """
    h = 1.0 / n
    c = cell_centres(n, h, -0.5)
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    v = np.stack([-y, x, 0.2 * np.exp(-(x * x + y * y) / 0.05)])
    v = _normalize(v)
    g = _rng(seed).standard_normal(v.shape)
    return _normalize(v + noise * g)


def gaussian_bump_field(n: int) -> np.ndarray:
    """m(x) = exp(-|x|^2) (1, 1, 1) sampled at the midpoints of [0, 1]^3."""
    h = 1.0 / n
    c = cell_centres(n, h, 0.0)
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    s = np.exp(-(x * x + y * y + z * z))
    return np.stack([s, s, s])


def staircase_sphere_field(n: int, axis: int = 2) -> np.ndarray:
    """Uniform magnetization inside the ball inscribed in the unit cube."""
    h = 1.0 / n
    c = cell_centres(n, h, -0.5)
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    inside = (x * x + y * y + z * z) <= 0.25
    m = np.zeros((3, n, n, n))
    m[axis][inside] = 1.0
    return m


# ---------------------------------------------------------------- structured
@dataclass
class CPInput:
    """Per magnetization component q: weights lam[q] (r,), factors U[q][d]
    of shape (n_d, r) for d = x, y, z."""
    lam: list
    U: list


@dataclass
class TuckerInput:
    """Per component q: core C[q] of shape (r_x, r_y, r_z) indexed [a][b][c]
    and factors U[q][d] of shape (n_d, r_d)."""
    core: list
    U: list


@dataclass
class TTInput:
    """Per component q: G1[q] (n_x, r1), G2[q] (r1, n_y, r2), G3[q] (r2, n_z)."""
    G1: list
    G2: list
    G3: list


def cp_input(n, rank: int = 10, seed: int = 1, dtype=np.float64) -> CPInput:
    nx, ny, nz = (n, n, n) if np.isscalar(n) else tuple(n)
    rng = _rng(seed)
    lam, U = [], []
    for _q in range(3):
        lam.append(np.ones(rank, dtype=dtype))
        U.append([rng.uniform(-1.0, 1.0, size=(nd, rank)).astype(dtype) for nd in (nx, ny, nz)])
    return CPInput(lam=lam, U=U)


def tucker_input(n, ranks=(8, 8, 8), seed: int = 1, dtype=np.float64) -> TuckerInput:
    nx, ny, nz = (n, n, n) if np.isscalar(n) else tuple(n)
    rng = _rng(seed)
    core, U = [], []
    for _q in range(3):
        core.append(rng.uniform(-1.0, 1.0, size=tuple(ranks)).astype(dtype))
        U.append([rng.uniform(-1.0, 1.0, size=(nd, rd)).astype(dtype)
                  for nd, rd in zip((nx, ny, nz), ranks)])
    return TuckerInput(core=core, U=U)


def tt_input(n, ranks=(8, 8), seed: int = 1, dtype=np.float64) -> TTInput:
    nx, ny, nz = (n, n, n) if np.isscalar(n) else tuple(n)
    r1, r2 = ranks
    rng = _rng(seed)
    G1, G2, G3 = [], [], []
    for _q in range(3):
        G1.append(rng.uniform(-1.0, 1.0, size=(nx, r1)).astype(dtype))
        G2.append(rng.uniform(-1.0, 1.0, size=(r1, ny, r2)).astype(dtype))
        G3.append(rng.uniform(-1.0, 1.0, size=(r2, nz)).astype(dtype))
    return TTInput(G1=G1, G2=G2, G3=G3)


# ---------------------------------------------------------------- batches
@dataclass
class BatchState:
    n: tuple          # (nx, ny, nz)
    h: tuple          # (hx, hy, hz), cubic cells, longest edge of the grid = 1
    seed: int
    m: np.ndarray = field(repr=False, default=None)


def tucker_magnetization(n, kind: str = "uniform", ranks=(2, 3, 2), seed: int = 5):
    """Three magnetization components in Tucker form, each (core [r0][r1][r2],
    [U_x [n_x][r0], U_y [n_y][r1], U_z [n_z][r2]]) in float64:
      uniform  m = (0.3, -0.5, 0.8): rank (1, 1, 1), unit factor columns of ones;
      smooth   cosines cos(pi (l + 1) x) and sines sin(2 x + l) of the cell
               midpoints x in [0, 1] (column l), standard-normal cores;
      random   U[-1, 1] factors and standard-normal cores."""
    rng = _rng(seed)
    out = []
    for q in range(3):
        if kind == "uniform":
            core = np.array([[[(0.3, -0.5, 0.8)[q]]]])
            U = [np.ones((n[p], 1)) for p in range(3)]
        elif kind == "smooth":
            core = rng.standard_normal(ranks)
            U = []
            for p in range(3):
                x = (np.arange(n[p]) + 0.5) / n[p]
                cols = [np.cos(np.pi * (l + 1) * x) if l % 2 == 0 else np.sin(2.0 * x + l) for l in range(ranks[p])]
                U.append(np.stack(cols, axis=1))
        else:
            core = rng.standard_normal(ranks)
            U = [rng.uniform(-1.0, 1.0, (n[p], ranks[p])) for p in range(3)]
        out.append((core, U))
    return out


def tt_cores(n, ranks=(6, 5), decay=(0.3, 0.4), seed: int = 6):
    """A 3D tensor train (G1 [n0][r1], G2 [r1][n1][r2], G3 [r2][n2]) with
    standard-normal entries, the columns of G1 scaled by decay[0]^a and the
    rows of G3 by decay[1]^b (decaying unfolding spectra), float64."""
    rng = _rng(seed)
    r1, r2 = ranks
    G1 = rng.standard_normal((n[0], r1)) * decay[0] ** np.arange(r1)[None, :]
    G2 = rng.standard_normal((r1, n[1], r2))
    G3 = rng.standard_normal((r2, n[2])) * decay[1] ** np.arange(r2)[:, None]
    return G1, G2, G3


def batch_grids(count: int = 256, seed: int = 2, with_fields: bool = True):
    """Uneven batch: state s with s % 8 == 7 is a 256x256xnz film with
    nz = (4, 8, 16)[(s // 8) % 3]; every other state is a cube with edge drawn
    uniformly from {16..96}.  Every grid is scaled so its longest edge is 1 and
    cells are cubic.  Magnetizations are random unit vectors."""
    rng = _rng(seed)
    states = []
    for s in range(count):
        if s % 8 == 7:
            n = (256, 256, (4, 8, 16)[(s // 8) % 3])
        else:
            e = int(rng.integers(16, 97))
            n = (e, e, e)
        hcell = 1.0 / max(n)
        st = BatchState(n=n, h=(hcell, hcell, hcell), seed=seed * 100003 + s)
        if with_fields:
            st.m = random_unit_field(n, seed=st.seed)
        states.append(st)
    return states


# ---------------------------------------------------------------- learned rule
def quad_training_cases(count: int = 20000, seed: int = 3):
    """Features for the node-proposal network: grids 32^3..64^3 with random
    aspect ratios, cell size h = 1/n_max (unit longest edge), log10 tolerance
    uniform in [-9, -4] and a requested node count R' uniform in {16..32}.

    Returns a dict of arrays: n (count, 3) int, h (count,), log10_tol (count,),
    rprime (count,) int.
    """
    rng = _rng(seed)
    n = rng.integers(32, 65, size=(count, 3))
    h = 1.0 / n.max(axis=1)
    log10_tol = rng.uniform(-9.0, -4.0, size=count)
    rprime = rng.integers(16, 33, size=count)
    return {"n": n.astype(np.int64), "h": h, "log10_tol": log10_tol,
            "rprime": rprime.astype(np.int64)}


# ---------------------------------------------------------------- network inputs
MLP_SIZES = (6, 64, 64, 64, 65)


def mlp_param_count(sizes=MLP_SIZES) -> int:
    return sum(o * i + o for i, o in zip(sizes[:-1], sizes[1:]))


def mlp_init(seed: int = 4, sizes=MLP_SIZES, out_scale: float = 0.0) -> np.ndarray:
    """Flat float32 parameter vector [W1 (64x6, row = output), b1, W2, b2, W3,
    b3, W4 (65x64), b4]: hidden weights ~ N(0, 1/fan_in), biases 0, and the
    output layer scaled by ``out_scale`` (0: the untrained network proposes
    the unmodified base rule)."""
    rng = _rng(seed)
    parts = []
    layers = list(zip(sizes[:-1], sizes[1:]))
    for li, (i, o) in enumerate(layers):
        scale = 1.0 / np.sqrt(i)
        if li == len(layers) - 1:
            scale *= out_scale
        parts.append((rng.standard_normal((o, i)) * scale).ravel())
        parts.append(np.zeros(o))
    return np.concatenate(parts).astype(np.float32)


# directions (max-norm 1) of the far samples, taken in a cycle that shifts by
# one per shell group
FIT_DIRECTIONS = ((1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0), (1.0, 1.0, 1.0), (1.0, 1.0, 0.0),
                  (0.0, 1.0, 1.0), (1.0, 0.0, 1.0), (1.0, 0.5, 0.25), (0.5, 1.0, 0.25), (0.25, 0.5, 1.0),
                  (1.0, 0.25, 0.5), (0.5, 0.25, 1.0))


def fit_offsets(n, count: int = 256):
    """Offsets J = (Jx, Jy, Jz), 0 <= J_d < n_d, and weights w_J at which a
    quadrature rule's kernels are compared with the reference's on the grid
    n = (nx, ny, nz), so that sum_J w_J |dK(J)|^2 approximates the sum over
    every offset of the grid of (prod_d (n_d - |J_d|)) |dK(J)|^2, i.e. the
    squared Frobenius norm of the operator's error (each offset J >= 0 stands
    for its 2^(number of nonzero J_d) sign images; kernels are even or odd in
    every J_d).

    * near block: every J with J_d <= 3 (at most 64 offsets), exact weights
      c_x(Jx) c_y(Jy) c_z(Jz), c_d(j) = (n_d - j) (1 if j == 0 else 2);
    * far region, max-norm s = max_d J_d from 4 to s_max = max_d (n_d - 1):
      G = min((count - near) // 8, s_max - 3) groups of consecutive s with
      geometrically growing edges; each group is represented by 8 offsets at
      the max-norm sqrt(s_lo (s_hi - 1)) along 8 of FIT_DIRECTIONS, each
      weighted with 1/8 of the group's total weight.
    Padded to ``count`` rows with J = (0, 0, 0), weight 0.
    Returns (J int32 [count][3], w float64 [count])."""
    nx, ny, nz = (n, n, n) if np.isscalar(n) else tuple(int(v) for v in n)
    nn = (nx, ny, nz)
    c = [[float((nd - j) * (1 if j == 0 else 2)) for j in range(nd)] for nd in nn]
    J, w = [], []
    for z in range(min(4, nz)):
        for y in range(min(4, ny)):
            for x in range(min(4, nx)):
                J.append((x, y, z))
                w.append(c[0][x] * c[1][y] * c[2][z])
    if count < len(J):
        raise ValueError("count too small for the near block")
    cum = []
    for d in range(3):
        acc, row = 0.0, [0.0]
        for v in c[d]:
            acc += v
            row.append(acc)
        cum.append(row)

    def total(s):   # weight of all offsets with max-norm < s
        return cum[0][min(s, nx)] * cum[1][min(s, ny)] * cum[2][min(s, nz)]

    smax = max(nn) - 1
    G = min((count - len(J)) // 8, max(0, smax - 3))
    if G > 0:
        edges = [4]
        for g in range(1, G):
            edges.append(max(edges[-1] + 1, int(round(4.0 * ((smax + 1) / 4.0) ** (g / G)))))
        edges.append(smax + 1)
        uniq = []
        for v in edges:
            v = min(v, smax + 1)
            if not uniq or v != uniq[-1]:
                uniq.append(v)
        for g in range(len(uniq) - 1):
            lo, hi = uniq[g], uniq[g + 1]
            wg = (total(hi) - total(lo)) / 8.0
            sg = int(round(np.sqrt(float(lo * (hi - 1)))))
            for i in range(8):
                u = FIT_DIRECTIONS[(g + i) % len(FIT_DIRECTIONS)]
                J.append(tuple(min(int(np.rint(sg * u[d])), nn[d] - 1) for d in range(3)))
                w.append(wg)
    while len(J) < count:
        J.append((0, 0, 0))
        w.append(0.0)
    return np.array(J, dtype=np.int32), np.array(w, dtype=np.float64)


def quad_features(n, h, log10_tol, rprime) -> np.ndarray:
    """Network input per case (float32, 6 values): the three aspect ratios
    n_d / n_max, the cell size as log2(1/h)/6 - 1, the tolerance as
    (log10 tol + 6.5)/2.5 and the requested node count as (R' - 24)/8.
    Arrays of cases broadcast: n (B, 3), h, log10_tol, rprime (B,)."""
    n = np.atleast_2d(np.asarray(n, dtype=np.float64))
    nmax = n.max(axis=1, keepdims=True)
    h = np.atleast_1d(np.asarray(h, dtype=np.float64))
    x = np.concatenate([n / nmax, (np.log2(1.0 / h) / 6.0 - 1.0)[:, None],
                        ((np.atleast_1d(log10_tol) + 6.5) / 2.5)[:, None],
                        ((np.atleast_1d(rprime).astype(np.float64) - 24.0) / 8.0)[:, None]], axis=1)
    return x.astype(np.float32)


def recompress_test_matrices(n, rmax: int, seed: int = 7):
    """Gaussian test matrices of the randomized range finder of the HOOI
    recompression, K = rmax + 8 candidates: omega = [K][n_p] for p = 0, 1, 2
    one after another, gmat = [K * K][K] (float64)."""
    K = rmax + 8
    rng = _rng(seed)
    omega = np.concatenate([rng.standard_normal((K, int(n[p]))).ravel() for p in range(3)])
    gmat = rng.standard_normal((K * K, K))
    return omega, np.ascontiguousarray(gmat.ravel())
