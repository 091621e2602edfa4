"""Full-format apply of the separable sinc kernel by 3D FFT convolution.

TEST INFRASTRUCTURE ONLY (see the package header).

For unstructured (full-format) tensors Sec. 4.2 recommends evaluating the
discrete convolution with the Kronecker-approximated kernel by FFTs instead
of mode products.  The kernel of each (output, input component) pair is the
separable sum over nodes of Cor. kron_op,

    K[Jz][Jy][Jx] = sum_k f_x[k][Jx] f_y[k][Jy] f_z[k][Jz]     (J_d in [-(n_d-1), n_d-1]),

formed here as a dense 3D array from the same stored 1D factors as
``apply.kron_apply_dense`` (types phi_types / field_types), and applied by a
zero-padded float64 FFT convolution (convolution theorem, Sec. 4.1).  Both
routes compute the same operator, so they agree to rounding.
"""
from __future__ import annotations

import numpy as np

from . import apply, sinc


def kernel_tensor(F, types) -> np.ndarray:
    """Dense separable kernel [2nz-1][2ny-1][2nx-1] for factor types (tx, ty, tz)."""
    tx, ty, tz = types
    return np.einsum("ka,kb,kc->cba", F[0][tx], F[1][ty], F[2][tz])


def fft_apply(m: np.ndarray, h, tau, alpha):
    """phi and h of the separable operator by FFT convolution.  m: [3][nz][ny][nx]."""
    nz, ny, nx = m.shape[1:]
    F = apply.axis_factors((nx, ny, nz), h, tau, alpha)
    phi = sum(apply._linear_conv_same(kernel_tensor(F, sinc.phi_types(q)), m[q]) for q in range(3))
    hf = np.stack([sum(apply._linear_conv_same(kernel_tensor(F, sinc.field_types(p, q)), m[q]) for q in range(3))
                   for p in range(3)])
    return phi, hf
