"""The Kronecker operator on non-uniform tensor-product grids.

TEST INFRASTRUCTURE ONLY (see the package header).

Paper: Sec. 3.1 (collocation at the cell centres, Eq. (coll)) and Lemma
sinc_mumag / Cor. kron_op hold for any partition of the axes into intervals;
only the Toeplitz structure of the 1D factors (Sec. 4.2) needs uniform cells.
For target cell i (centre xi_i) and source cell j = [x_j, x_{j+1}] the
interval of u = xi_i - y is [a, b] = [xi_i - x_{j+1}, xi_i - x_j], and
  E = int_a^b exp(-tau^2 u^2) du,   X = int_a^b u exp(-tau^2 u^2) du,
  X' = b exp(-tau^2 b^2) - a exp(-tau^2 a^2)   (d/d xi_i of X),
stored as in oracle.sinc: E~ = w E, X~ = w X, P~ = -w X', Q~ = 2 tau^2 w X.

Edges here are in the scaled domain (longest extent 1) unless noted.
"""
from __future__ import annotations

import numpy as np
from scipy import special

from . import exact, sinc


def centres(edges):
    e = np.asarray(edges, dtype=np.float64)
    return 0.5 * (e[:-1] + e[1:])


def intervals(edges):
    """[a, b] arrays [n][n] (target i, source j)."""
    e = np.asarray(edges, dtype=np.float64)
    xi = centres(e)
    a = xi[:, None] - e[None, 1:]
    b = xi[:, None] - e[None, :-1]
    return a, b


def factor_E(tau, edges):
    a, b = intervals(edges)
    ta, tb = tau * a, tau * b
    diff = np.where(ta > 0.5, special.erfc(ta) - special.erfc(tb),
                    np.where(tb < -0.5, special.erfc(-tb) - special.erfc(-ta), special.erf(tb) - special.erf(ta)))
    return np.sqrt(np.pi) / (2.0 * tau) * diff


def factor_X(tau, edges):
    a, b = intervals(edges)
    t2 = tau * tau
    d2 = (b - a) * (b + a)
    with np.errstate(over="ignore", invalid="ignore"):   # the branch not taken may overflow
        near_a = -np.exp(-t2 * a * a) * np.expm1(-t2 * d2) / (2.0 * t2)
        near_b = np.exp(-t2 * b * b) * np.expm1(t2 * d2) / (2.0 * t2)
    return np.where(d2 >= 0.0, near_a, near_b)


def factor_Xp(tau, edges):
    a, b = intervals(edges)
    t2 = tau * tau
    return b * np.exp(-t2 * b * b) - a * np.exp(-t2 * a * a)


def dense_factors(edges, tau, alpha):
    """[4][M][n][n] stored factors of one axis (node weight W^(1/3) folded in)."""
    tau = np.asarray(tau, dtype=np.float64)
    w = np.cbrt(sinc.node_weights(alpha))
    n = len(edges) - 1
    out = np.empty((4, tau.size, n, n))
    for k in range(tau.size):
        E = factor_E(tau[k], edges)
        X = factor_X(tau[k], edges)
        Xp = factor_Xp(tau[k], edges)
        out[sinc.TYPE_E, k] = w[k] * E
        out[sinc.TYPE_X, k] = w[k] * X
        out[sinc.TYPE_P, k] = -w[k] * Xp
        out[sinc.TYPE_Q, k] = 2.0 * tau[k] ** 2 * w[k] * X
    return out


def _triple(u, Tx, Ty, Tz):
    v = np.einsum("ia,zya->zyi", Tx, u)
    v = np.einsum("ib,zbx->zix", Ty, v)
    return np.einsum("ic,cyx->iyx", Tz, v)


def kron_apply(m, edges, tau, alpha):
    """Kronecker-form apply with the dense factors (same sums as
    oracle.apply.kron_apply_dense).  m [3][nz][ny][nx]; edges = (x, y, z)
    in the scaled domain.  Returns (phi, h[3]) in scaled units."""
    F = [dense_factors(edges[d], tau, alpha) for d in range(3)]
    nz, ny, nx = m.shape[1:]
    phi = np.zeros((nz, ny, nx))
    hf = np.zeros((3, nz, ny, nx))
    for k in range(len(tau)):
        for q in range(3):
            tx, ty, tz = sinc.phi_types(q)
            phi += _triple(m[q], F[0][tx, k], F[1][ty, k], F[2][tz, k])
            for p in range(3):
                tx, ty, tz = sinc.field_types(p, q)
                hf[p] += _triple(m[q], F[0][tx, k], F[1][ty, k], F[2][tz, k])
    return phi, hf


def exact_direct(m, edges):
    """Exact collocation (Eq. (coll)) by direct sums of the closed-form box
    kernels: phi_i = sum_j sum_q K^q(xi_i - box_j) m_j^q, h_i = -sum_j N(xi_i -
    box_j) m_j.  Any units; small grids only (O(N^2) pairs)."""
    e = [np.asarray(x, dtype=np.float64) for x in edges]
    nx, ny, nz = (len(x) - 1 for x in e)
    xi = [centres(x) for x in e]
    # target (z, y, x) x source (z, y, x): offsets lo = xi - x_{j+1}, hi = xi - x_j
    lo, hi = [], []
    for d, shape in ((0, (1, 1, nx, 1, 1, nx)), (1, (1, ny, 1, 1, ny, 1)), (2, (nz, 1, 1, nz, 1, 1))):
        a = xi[d][:, None] - e[d][None, 1:]
        b = xi[d][:, None] - e[d][None, :-1]
        if d == 0:
            lo.append(a.reshape(1, 1, nx, 1, 1, nx)); hi.append(b.reshape(1, 1, nx, 1, 1, nx))
        elif d == 1:
            lo.append(a.reshape(1, ny, 1, 1, ny, 1)); hi.append(b.reshape(1, ny, 1, 1, ny, 1))
        else:
            lo.append(a.reshape(nz, 1, 1, nz, 1, 1)); hi.append(b.reshape(nz, 1, 1, nz, 1, 1))
    lo = np.broadcast_arrays(*lo)
    hi = np.broadcast_arrays(*hi)
    phi = np.zeros((nz, ny, nx))
    hf = np.zeros((3, nz, ny, nx))
    for q in range(3):
        K = exact.potential_kernel_box(tuple(lo), tuple(hi), q)
        phi += np.einsum("zyxcba,cba->zyx", K, m[q])
        for p in range(3):
            N = exact.demag_tensor_box(tuple(lo), tuple(hi), p, q)
            hf[p] -= np.einsum("zyxcba,cba->zyx", N, m[q])
    return phi, hf


def kron_apply_at_cells(m, edges, tau, alpha, cells):
    """The Kronecker-form result of ``kron_apply`` at sampled target cells
    (iz, iy, ix): per node, the rows of the dense factors contracted with m
    one axis at a time (x, then y, then z).  Returns (phi[c], h[c][3])."""
    F = [dense_factors(edges[d], tau, alpha) for d in range(3)]
    res_phi = np.zeros(len(cells))
    res_h = np.zeros((len(cells), 3))
    for c, (iz, iy, ix) in enumerate(cells):
        for k in range(len(tau)):
            rows = [F[0][:, k, ix, :], F[1][:, k, iy, :], F[2][:, k, iz, :]]   # [type][source j]
            for q in range(3):
                mx = m[q] @ rows[0].T                       # [z][y][type_x]
                for out, types in [("phi", sinc.phi_types(q))] + [(p, sinc.field_types(p, q)) for p in range(3)]:
                    tx, ty, tz = types
                    val = rows[2][tz] @ (rows[1][ty] @ mx[:, :, tx].T)
                    if out == "phi":
                        res_phi[c] += val
                    else:
                        res_h[c, out] += val
    return res_phi, res_h
