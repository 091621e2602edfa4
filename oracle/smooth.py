"""Potential of a smooth magnetization at one point, by singularity subtraction.

TEST INFRASTRUCTURE ONLY (see the package header).

Reference for Lemma conv_coll and Fig. fig_err: the continuous potential
Eq. (intop2) (physical sign, see oracle.exact) of m(y) = g(y) (1, 1, 1) on the
box Omega at a point xi,
    phi(xi) = g(xi) sum_q K_Omega^q(xi)
            + 1/(4 pi) int_Omega (g(y) - g(xi)) sum_q (xi - y)_q / |xi - y|^3 dy,
where K_Omega^q(xi) is the closed-form potential of the uniformly magnetized
box (oracle.exact.box_kernels_at_points).  The remainder integrand is O(1/r)
at y = xi; Omega is cut at xi into 8 boxes with xi at a corner, each box into 3
pyramids with apex xi, and each pyramid mapped to the unit cube (Duffy map,
Jacobian u^2 L1 L2 L3), after which a tensor Gauss-Legendre rule converges
quickly because the mapped integrand is smooth.
"""
from __future__ import annotations

import numpy as np

from . import exact


def _gl(npts: int):
    x, w = np.polynomial.legendre.leggauss(npts)
    return 0.5 * (x + 1.0), 0.5 * w


def _remainder(g, xi, lo, hi, npts: int) -> float:
    u, wu = _gl(npts)
    U, V, W = np.meshgrid(u, u, u, indexing="ij")
    WW = wu[:, None, None] * wu[None, :, None] * wu[None, None, :]
    total = 0.0
    for sgn in np.ndindex(2, 2, 2):
        L = np.array([(hi[d] - xi[d]) if sgn[d] else (xi[d] - lo[d]) for d in range(3)])
        sig = np.array([1.0 if sgn[d] else -1.0 for d in range(3)])
        if np.any(L <= 0):
            continue
        for p in range(3):
            a, b = [d for d in range(3) if d != p]
            x = [None, None, None]
            x[p] = U * L[p]
            x[a] = U * V * L[a]
            x[b] = U * W * L[b]
            y = [xi[d] + sig[d] * x[d] for d in range(3)]
            s = [xi[d] - y[d] for d in range(3)]
            r3 = (s[0] ** 2 + s[1] ** 2 + s[2] ** 2) ** 1.5
            f = (g(*y) - g(*xi)) * (s[0] + s[1] + s[2]) / r3
            jac = U * U * L[0] * L[1] * L[2]
            total += np.sum(WW * f * jac)
    return total / (4.0 * np.pi)


def potential_smooth_at(g, xi, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), npts: int = 48) -> float:
    """phi(xi) for m = g(x, y, z) (1, 1, 1) on the box [lo, hi]."""
    K, _N = exact.box_kernels_at_points(np.array(xi, dtype=np.float64), lo, hi)
    return float(g(*xi) * np.sum(K)) + _remainder(g, xi, lo, hi, npts)


def collocated_phi_at_cell(mvals, h, cell) -> float:
    """Collocation value phi_i (Eq. (coll)) at one target cell i = (iz, iy, ix)
    by a direct sum over all sources with exact cell kernels."""
    nz, ny, nx = mvals.shape[1:]
    iz, iy, ix = cell
    jz, jy, jx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    J = (ix - jx, iy - jy, iz - jz)
    lo = tuple((J[d] - 0.5) * h[d] for d in range(3))
    hi = tuple((J[d] + 0.5) * h[d] for d in range(3))
    return float(sum(np.sum(exact.potential_kernel_box(lo, hi, q) * mvals[q]) for q in range(3)))
