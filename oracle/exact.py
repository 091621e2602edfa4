"""Exact collocation kernels of Eq. (coll) / (matrix_op) for box cells.

TEST INFRASTRUCTURE ONLY (see the package header).

Reading of the paper (Sec. 3.2, Eqs. (intop2), (coll), (kernel)):
  * Sign.  Integrating Eq. (intop1) by parts gives +1/(4 pi) in front of the
    volume integral, not the -1/(4 pi) printed in Eq. (intop2) and carried
    into Eqs. (coll), (kron_operator) and (conv_pot).  The oracle uses the
    physical sign
        phi(x) = 1/(4 pi) int m(y) . (x - y)/|x - y|^3 dy,   h = -grad phi,
    so that a uniformly magnetized body has h = -N m with N >= 0 (the centre
    of a cube has N_zz = 1/3).
  * Cells.  The collocation points are cell midpoints on a uniform tensor
    grid (Sec. 3.1).  For a target cell i and a source cell j the source box
    seen from the target midpoint is, per axis p, the interval
        s_p in [a_J, b_J] = [(J - 1/2) h_p, (J + 1/2) h_p],   J = i_p - j_p,
    with s = x - y (Sec. 4.2, below Eq. (conv_op)).

Kernels (for a source cell with unit magnetization along q):
  potential   K^q(J)   = 1/(4 pi) int_box s_q / |s|^3 ds
  field       N_pq(J)  = -1/(4 pi) d_p d_q int_box ds / |x - y|      (h_p = -sum_q N_pq m_q)
so that phi_i = sum_q sum_j K^q(i - j) m^q_j and h^p_i = -sum_q sum_j N_pq(i - j) m^q_j.

Route 1 (closed form).  With F any function whose mixed third derivative is
1/|s|, a box integral is the alternating 8-corner sum Delta[F].  The partial
derivatives of F that are needed, each fixed up to terms that cancel in the
corner sum, are (verified symbolically, and pinned numerically by the tests):
  d_1 F      = s2 asinh(s3/rho12) + s3 asinh(s2/rho13) - s1 atan(s2 s3/(s1 r))
  d_1 d_1 F  = -atan(s2 s3 / (s1 r))
  d_1 d_2 F  = asinh(s3 / rho12)
giving K^q = -Delta[d_q F]/(4 pi), N_pp = Delta[atan(.)]/(4 pi), N_pq = -Delta[asinh(.)]/(4 pi).

Route 2 (Eq. (conv_op), Gaussian transform Eq. (gauss_trans)): the same
kernels as one-dimensional tau integrals of products of 1D cell integrals,
evaluated by adaptive quadrature in multiple precision (mpmath).

Route 3 (brute force): integrate the derivative along one axis analytically
(a face difference) and the remaining two axes by adaptive 2D quadrature; the
faces never pass through the collocation point, so the integrand is smooth.
"""
from __future__ import annotations

import numpy as np

FOUR_PI = 4.0 * np.pi


def offset_bounds(n: int, h: float, dtype=np.float64):
    """a_J, b_J for J = -(n-1)..(n-1) (index J + n - 1), per Sec. 4.2."""
    J = np.arange(-(n - 1), n, dtype=dtype)
    h = dtype(h)
    return (J - dtype(0.5)) * h, (J + dtype(0.5)) * h


def _corner_sum(fn, lo, hi):
    """Alternating sum over the 8 corners of the box prod_p [lo_p, hi_p]:
    sum over corners of (-1)^(number of lower bounds) fn(s1, s2, s3)."""
    total = 0.0
    for e1 in (0, 1):
        s1 = hi[0] if e1 else lo[0]
        for e2 in (0, 1):
            s2 = hi[1] if e2 else lo[1]
            for e3 in (0, 1):
                s3 = hi[2] if e3 else lo[2]
                sign = -1.0 if (3 - e1 - e2 - e3) % 2 else 1.0
                total = total + sign * fn(s1, s2, s3)
    return total


def _safe_div(num, den):
    den_ok = den != 0
    return np.where(den_ok, num / np.where(den_ok, den, 1), 0.0)


def _asinh_term(sp, sq, sr):
    """asinh(sr / sqrt(sp^2 + sq^2))."""
    rho = np.sqrt(sp * sp + sq * sq)
    return np.arcsinh(_safe_div(sr, rho))


def _dF(q):
    """d_q F as a function of (s1, s2, s3)."""
    def f(s1, s2, s3):
        s = [s1, s2, s3]
        sq = s[q]
        a, b = [s[i] for i in range(3) if i != q]
        r = np.sqrt(s1 * s1 + s2 * s2 + s3 * s3)
        rho_qa = np.sqrt(sq * sq + a * a)
        rho_qb = np.sqrt(sq * sq + b * b)
        t1 = a * np.arcsinh(_safe_div(b, rho_qa))
        t2 = b * np.arcsinh(_safe_div(a, rho_qb))
        t3 = sq * np.arctan(_safe_div(a * b, sq * r))
        return t1 + t2 - t3
    return f


def _dpdq_F(p, q):
    """d_p d_q F as a function of (s1, s2, s3)."""
    def f(s1, s2, s3):
        s = [s1, s2, s3]
        if p == q:
            a, b = [s[i] for i in range(3) if i != p]
            sp = s[p]
            r = np.sqrt(s1 * s1 + s2 * s2 + s3 * s3)
            return -np.arctan(_safe_div(a * b, sp * r))
        rr = 3 - p - q
        return _asinh_term(s[p], s[q], s[rr])
    return f


def potential_kernel_box(lo, hi, q: int):
    """K^q = 1/(4 pi) int_box s_q/|s|^3 ds for boxes prod_p [lo_p, hi_p]."""
    return -_corner_sum(_dF(q), lo, hi) / FOUR_PI


def demag_tensor_box(lo, hi, p: int, q: int):
    """N_pq = -1/(4 pi) Delta[d_p d_q F] for boxes prod_p [lo_p, hi_p]."""
    return -_corner_sum(_dpdq_F(p, q), lo, hi) / FOUR_PI


def offset_kernels(n, h, dtype=np.float64):
    """All offset kernels of a uniform grid.

    n = (nx, ny, nz), h = (hx, hy, hz).  Returns (K, N) with
      K[q]    shape (2nz-1, 2ny-1, 2nx-1), index [Jz+nz-1][Jy+ny-1][Jx+nx-1]
      N[p][q] same shape.
    """
    nx, ny, nz = n
    ax, bx = offset_bounds(nx, h[0], dtype)
    ay, by = offset_bounds(ny, h[1], dtype)
    az, bz = offset_bounds(nz, h[2], dtype)
    # broadcast to [z][y][x]
    lo = (ax[None, None, :], ay[None, :, None], az[:, None, None])
    hi = (bx[None, None, :], by[None, :, None], bz[:, None, None])
    K = np.stack([potential_kernel_box(lo, hi, q) for q in range(3)]).astype(np.float64)
    N = np.empty((3, 3) + K.shape[1:])
    for p in range(3):
        for q in range(p, 3):
            N[p, q] = demag_tensor_box(lo, hi, p, q)
            N[q, p] = N[p, q]
    return K, N


def box_kernels_at_points(points, box_lo, box_hi):
    """Potential kernels K^q and demag tensor N_pq of ONE box evaluated at
    arbitrary target points (array (..., 3), coordinates x, y, z).  Used for
    the uniformly magnetized whole body, whose cell sum equals this by the
    additivity of the integral."""
    x = np.asarray(points, dtype=np.float64)
    lo = tuple(x[..., p] - box_hi[p] for p in range(3))
    hi = tuple(x[..., p] - box_lo[p] for p in range(3))
    K = np.stack([potential_kernel_box(lo, hi, q) for q in range(3)])
    N = np.empty((3, 3) + K.shape[1:])
    for p in range(3):
        for q in range(3):
            N[p, q] = demag_tensor_box(lo, hi, p, q)
    return K, N


# ------------------------------------------------------------------ route 2
def tau_integral_kernel(J, h, kind, p=None, q=None, dps: int = 30):
    """Kernel from the Gaussian transform, Eq. (gauss_trans) / (conv_op):

        K^q(J)  = pi^(-3/2) int_0^inf tau^2 X_q E E dtau
        N_pp(J) = pi^(-3/2) int_0^inf tau^2 X'_p E E dtau
        N_pq(J) = pi^(-3/2) int_0^inf tau^2 (-2 tau^2 X_p) X_q E_r dtau   (p != q)

    where E = int_a^b exp(-tau^2 x^2) dx, X = int_a^b x exp(-tau^2 x^2) dx and
    X' = d/ds X(s) of the interval [s - h/2, s + h/2] (Sec. 3.3 and the
    derivative of the factor with respect to the target position).
    The tau integral runs over [0, inf) (the integrand is even in tau, which
    turns the 2/sqrt(pi) over R of Eq. (gauss_trans) into 4/sqrt(pi); with the
    1/(4 pi) of the potential this gives pi^(-3/2)).
    kind: 'phi' (uses q) or 'N' (uses p, q).  Multiple precision throughout.
    """
    import mpmath as mp
    mp.mp.dps = dps
    Jv = [int(j) for j in J]
    hv = [mp.mpf(x) for x in h]
    a = [(mp.mpf(Jv[d]) - mp.mpf(1) / 2) * hv[d] for d in range(3)]
    b = [(mp.mpf(Jv[d]) + mp.mpf(1) / 2) * hv[d] for d in range(3)]

    def E(d, t):
        return mp.sqrt(mp.pi) / (2 * t) * (mp.erf(t * b[d]) - mp.erf(t * a[d]))

    def X(d, t):
        return (mp.exp(-(t * a[d]) ** 2) - mp.exp(-(t * b[d]) ** 2)) / (2 * t * t)

    def Xp(d, t):
        return b[d] * mp.exp(-(t * b[d]) ** 2) - a[d] * mp.exp(-(t * a[d]) ** 2)

    def integrand(t):
        if t == 0:
            return mp.mpf(0)
        if kind == "phi":
            f = X(q, t)
            for d in range(3):
                if d != q:
                    f *= E(d, t)
        elif p == q:
            f = Xp(p, t)
            for d in range(3):
                if d != p:
                    f *= E(d, t)
        else:
            r = 3 - p - q
            f = -2 * t * t * X(p, t) * X(q, t) * E(r, t)
        return t * t * f

    hmin = min(hv)
    # break points around the scale where the Gaussians resolve a cell
    pts = [0, 0.25 / hmin, 1 / hmin, 4 / hmin, 16 / hmin, 64 / hmin, mp.inf]
    val = mp.quad(integrand, pts)
    return float(val / mp.pi ** mp.mpf(1.5))


# ------------------------------------------------------------------ route 3
def face_cubature_potential(J, h, q, epsabs=1e-15, epsrel=1e-12):
    """K^q(J) by integrating s_q/|s|^3 along axis q in closed form,
    [-1/|s|] between the two q-faces, and the two other axes by adaptive 2D
    quadrature (scipy dblquad)."""
    from scipy.integrate import dblquad
    a = [(J[d] - 0.5) * h[d] for d in range(3)]
    b = [(J[d] + 0.5) * h[d] for d in range(3)]
    u, v = [d for d in range(3) if d != q]

    def f(sv, su):
        r_a = np.sqrt(a[q] ** 2 + su * su + sv * sv)
        r_b = np.sqrt(b[q] ** 2 + su * su + sv * sv)
        return 1.0 / r_a - 1.0 / r_b

    val, _err = dblquad(f, a[u], b[u], a[v], b[v], epsabs=epsabs, epsrel=epsrel)
    return val / FOUR_PI


def face_cubature_demag(J, h, p, q, epsabs=1e-15, epsrel=1e-12):
    """N_pq(J) = -1/(4 pi) int_box d_p d_q (1/|s|) ds, reduced to the two
    p-faces: -1/(4 pi) int int [d_q(1/|s|)]_{s_p=a_p}^{b_p} over the other
    two axes, with d_q(1/|s|) = -s_q/|s|^3.  The p-faces lie at |s_p| >= h/2,
    so the integrand is smooth for every offset including the self cell."""
    from scipy.integrate import dblquad
    a = [(J[d] - 0.5) * h[d] for d in range(3)]
    b = [(J[d] + 0.5) * h[d] for d in range(3)]
    u, v = [d for d in range(3) if d != p]

    def g(sp, su, sv):
        s = [0.0, 0.0, 0.0]
        s[p], s[u], s[v] = sp, su, sv
        r = np.sqrt(s[0] ** 2 + s[1] ** 2 + s[2] ** 2)
        return -s[q] / r ** 3

    def f(sv, su):
        return g(b[p], su, sv) - g(a[p], su, sv)

    val, _err = dblquad(f, a[u], b[u], a[v], b[v], epsabs=epsabs, epsrel=epsrel)
    return -val / FOUR_PI
