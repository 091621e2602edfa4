"""Collocated potential and field, exact and in Kronecker form.

TEST INFRASTRUCTURE ONLY (see the package header).

Two results are computed here:

1. The collocation scheme itself, Eq. (coll) with the matrices of Eq.
   (matrix_op): phi_i = sum_q sum_j K^q(i - j) m^q_j and
   h^p_i = -sum_q sum_j N_pq(i - j) m^q_j with the exact cell kernels of
   ``oracle.exact`` (physical sign).  On a uniform grid these are discrete
   linear convolutions (Sec. 4.2), computed here by zero-padded FFTs in
   float64 (convolution theorem, Sec. 4.1), by explicit double loops for tiny
   grids, or for a few sampled target cells by direct sums.

2. The Kronecker-product approximation of Cor. kron_op, Eq. (kron_operator),
   applied with dense Toeplitz factor matrices (no FFT, no reuse between
   terms): for every node k and every (output, input component) pair, the
   triple mode product m_q x_1 T_x x_2 T_y x_3 T_z of Eq. (modemul).  Layout
   is [z][y][x] with x fastest, i.e. the matrix T_z (x) T_y (x) T_x acting on
   vec(m) (footnote of Cor. kron_op with the index typo read as
   I = i1 + (i2 - 1) n1 + (i3 - 1) n1 n2).
   The field uses the derivative factors of ``oracle.sinc`` (exact derivative
   of the separable potential kernel with respect to the target point), not the
   finite differences of the paper's experiments.
"""
from __future__ import annotations

import numpy as np
from scipy import fft as sfft

from . import exact, sinc


# ---------------------------------------------------------------- collocation
def _linear_conv_same(ker: np.ndarray, x: np.ndarray) -> np.ndarray:
    """out[i] = sum_j ker[i - j + n - 1] x[j] for 3D arrays, via rfftn."""
    n = x.shape
    shape = tuple(sfft.next_fast_len(2 * nd - 1 + nd - 1, real=True) for nd in n)
    axes = (0, 1, 2)
    full = sfft.irfftn(sfft.rfftn(ker, shape, axes=axes) * sfft.rfftn(x, shape, axes=axes),
                       shape, axes=axes)
    return full[n[0] - 1:2 * n[0] - 1, n[1] - 1:2 * n[1] - 1, n[2] - 1:2 * n[2] - 1]


def collocated_apply_fft(m: np.ndarray, h, kernels=None):
    """Exact collocation (Eq. (coll)) on a uniform grid by FFT convolution.

    m: [3][nz][ny][nx];  h = (hx, hy, hz).  Returns (phi, hfield[3]).
    ``kernels`` may pass precomputed (K, N) from exact.offset_kernels."""
    nz, ny, nx = m.shape[1:]
    K, N = kernels if kernels is not None else exact.offset_kernels((nx, ny, nz), h)
    phi = sum(_linear_conv_same(K[q], m[q]) for q in range(3))
    hf = np.stack([-sum(_linear_conv_same(N[p, q], m[q]) for q in range(3)) for p in range(3)])
    return phi, hf


def collocated_apply_direct(m: np.ndarray, h):
    """Exact collocation by explicit O(N^2) double loops (tiny grids only)."""
    nz, ny, nx = m.shape[1:]
    K, N = exact.offset_kernels((nx, ny, nz), h)
    phi = np.zeros((nz, ny, nx))
    hf = np.zeros((3, nz, ny, nx))
    for iz in range(nz):
        for iy in range(ny):
            for ix in range(nx):
                for jz in range(nz):
                    for jy in range(ny):
                        for jx in range(nx):
                            o = (iz - jz + nz - 1, iy - jy + ny - 1, ix - jx + nx - 1)
                            mj = m[:, jz, jy, jx]
                            phi[iz, iy, ix] += K[(slice(None),) + o] @ mj
                            hf[:, iz, iy, ix] -= N[(slice(None), slice(None)) + o] @ mj
    return phi, hf


def collocated_at_cells(m: np.ndarray, h, cells):
    """Exact collocation at a few target cells (iz, iy, ix) by direct sums
    over all source cells, with the source boxes' kernels evaluated per pair.
    Returns (phi[ncell], hfield[ncell][3])."""
    nz, ny, nx = m.shape[1:]
    jz, jy, jx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    out_phi, out_h = [], []
    for (iz, iy, ix) in cells:
        J = (ix - jx, iy - jy, iz - jz)
        lo = tuple((J[d] - 0.5) * h[d] for d in range(3))
        hi = tuple((J[d] + 0.5) * h[d] for d in range(3))
        phi = sum(np.sum(exact.potential_kernel_box(lo, hi, q) * m[q]) for q in range(3))
        hv = np.zeros(3)
        for p in range(3):
            for q in range(3):
                hv[p] -= np.sum(exact.demag_tensor_box(lo, hi, p, q) * m[q])
        out_phi.append(phi)
        out_h.append(hv)
    return np.array(out_phi), np.array(out_h)


# ---------------------------------------------------------------- Kronecker form
def axis_factors(n, h, tau, alpha):
    """Stored factors per axis: list over d = x, y, z of arrays [4][M][2n_d-1]."""
    return [sinc.scaled_factors(n[d], h[d], tau, alpha) for d in range(3)]


def _triple_mode_product(u: np.ndarray, Tx, Ty, Tz) -> np.ndarray:
    """u x_x Tx x_y Ty x_z Tz for u[z][y][x] (Eq. (modemul) on each axis)."""
    v = np.einsum("ia,zya->zyi", Tx, u)
    v = np.einsum("ib,zbx->zix", Ty, v)
    return np.einsum("ic,cyx->iyx", Tz, v)


def kron_apply_dense(m: np.ndarray, h, tau, alpha):
    """Kronecker-form apply with dense Toeplitz matrices (Cor. kron_op).

    phi = sum_k sum_q  m_q x (T_x, T_y, T_z) with per-axis types phi_types(q);
    h_p = sum_k sum_q  m_q x (...)            with types field_types(p, q).
    Returns (phi, hfield[3])."""
    nz, ny, nx = m.shape[1:]
    F = axis_factors((nx, ny, nz), h, tau, alpha)
    M = len(tau)
    phi = np.zeros((nz, ny, nx))
    hf = np.zeros((3, nz, ny, nx))
    for k in range(M):
        T = [[sinc.toeplitz(F[d][t, k]) for t in range(4)] for d in range(3)]
        for q in range(3):
            tx, ty, tz = sinc.phi_types(q)
            phi += _triple_mode_product(m[q], T[0][tx], T[1][ty], T[2][tz])
            for p in range(3):
                tx, ty, tz = sinc.field_types(p, q)
                hf[p] += _triple_mode_product(m[q], T[0][tx], T[1][ty], T[2][tz])
    return phi, hf


def kron_apply_at_cells(m: np.ndarray, h, tau, alpha, cells):
    """Kronecker-form result at sampled target cells (iz, iy, ix): each output
    is sum_k sum_q T_z[iz, :] (T_y[iy, :] (T_x[ix, :] . m_q)) -- the rows of
    the dense Toeplitz factors contracted with m one axis at a time."""
    nz, ny, nx = m.shape[1:]
    F = axis_factors((nx, ny, nz), h, tau, alpha)
    M = len(tau)
    res_phi = np.zeros(len(cells))
    res_h = np.zeros((len(cells), 3))
    for c, (iz, iy, ix) in enumerate(cells):
        for k in range(M):
            rows = []
            for d, (i, nd) in enumerate(zip((ix, iy, iz), (nx, ny, nz))):
                j = np.arange(nd)
                rows.append(F[d][:, k, i - j + nd - 1])   # [type][j]
            for q in range(3):
                # contract x first for both x-types needed, then y, then z
                mx = m[q] @ rows[0].T                      # [z][y][type_x]
                for (out, types) in [("phi", sinc.phi_types(q))] + [
                        (p, sinc.field_types(p, q)) for p in range(3)]:
                    tx, ty, tz = types
                    val = rows[2][tz] @ (rows[1][ty] @ mx[:, :, tx].T)
                    if out == "phi":
                        res_phi[c] += val
                    else:
                        res_h[c, out] += val
    return res_phi, res_h


def demag_energy_density(m: np.ndarray, hfield: np.ndarray) -> float:
    """Midpoint-rule demagnetizing energy per volume for a body filling the
    grid: e = -1/2 mean_i (m_i . h_i)  (the uniform cube gives 1/6)."""
    return float(-0.5 * np.mean(np.sum(m * hfield, axis=0)))


def rel_l2(a: np.ndarray, b: np.ndarray) -> float:
    """||a - b||_F / ||b||_F (Frobenius norm, Sec. 2)."""
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(np.asarray(b).ravel()))
