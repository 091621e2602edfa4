"""The scalar potential of a Tucker magnetization by structured DFTs
(Alg. scpot_fft_tucker, Sec. 4.2), with its tolerance-controlled steps, and
the tensor arithmetic it rests on.

TEST INFRASTRUCTURE ONLY (see the package header).

What each function states, and the passage it follows:
  kernel_cp         Eq. (conv_pot): the potential kernel of magnetization
                    component q as a CP tensor over the offsets
                    J_p = -(n_p - 1)..n_p - 1, one term per sinc node (node
                    weights and constants folded into the factors, as in
                    oracle.sinc).
  hooi              Alg. HOOI (Sec. 2.2) on a dense tensor: truncated HOSVD as
                    the start, then alternating sweeps until the squared core
                    norm stops changing; per mode the rank follows the rule of
                    oracle.recompress.truncation_rank (discarded singular values
                    of norm at most eps / sqrt(3) of all of them).
  dft_tucker        Lemma DFT_tucker: the zero-padded DFT of a Tucker tensor is
                    the Tucker tensor with the same core and the DFTs of its
                    factor columns.
  tucker_hadamard   App. B, Eqs. (t_had), (t_had2): the elementwise product of
                    two Tucker tensors has the Kronecker product of the cores as
                    core and, per mode, the row-wise Kronecker products of the
                    two factor matrices (the transposed Khatri-Rao product of
                    their transposes).
  potential_tucker  Alg. scpot_fft_tucker, step by step: the CP kernels, their
                    compression to Tucker with tol, their DFTs; per component
                    the DFT of the magnetization, the Hadamard product in
                    Fourier space, the inverse DFT, the product
                    recompressed with tol; then the approximate summation with
                    tol.
  tucker_sum        the approximate summation: the exact sum of Tucker tensors
                    (factors side by side, block-diagonal core) recompressed by
                    hooi with tol.
  tt_round          App. C (rounding of the cited TT work): right-to-left
                    orthogonalisation of the cores by QR, then left-to-right
                    truncated SVDs, each discarding singular values of norm at
                    most eps / sqrt(d - 1) times the tensor norm (d = 3), so the
                    result is within eps of the input in relative norm.
  tt_from_tucker    App. C, Eq. (tt_3d_2) read backwards: the middle factor
                    multiplied into the core gives the TT cores.
  tt_from_cp        App. C (CP2TT): a rank-R CP tensor is a TT with ranks (R, R)
                    and a diagonal middle core.
  tucker_from_tt    App. C: the Tucker2 form of Eq. (tt_3d_2) recompressed to
                    Tucker (HOOI with tol).
  potential_at_cells  Eq. (kron_eval_tuck) at single target cells: the
                    uncompressed Kronecker operator's potential of a Tucker
                    magnetization, for sizes where no dense tensor fits.

Readings:
  * DFT length.  The paper pads to 2 n_p - 1 points; every length
    L >= 2 n_p - 1 gives the same window (no wrap-around).  This oracle uses
    2 n_p - 1.
  * Window.  Output i of the Toeplitz product is entry i + n - 1 of the
    convolution of the kernel generator (offset J stored at J + n - 1) with the
    input column.
  * "Hadamard products ... using e.g. the tolerance tol": each product is
    formed exactly (Eq. (t_had2)), then recompressed by HOOI with tol (App. B
    recommends recompressing the product); the summation recompresses again
    with tol.  The errors of the three steps add up: the potential is within
    a small multiple of tol of the uncompressed route.
  * Index order of a product's combined rank index: (l, i) -> l * r + i for
    l a rank index of the second operand (the magnetization) and i one of the
    first (the kernel), in the core and in the factor columns alike (the
    paper's e_(il)(jm)(kn) = c_ijk d_lmn with the Khatri-Rao order of
    Eq. (t_had2)).

Tucker tensors are (core [r1][r2][r3], [U1, U2, U3]) with U_p [n_p][r_p];
dense tensors are indexed [i1][i2][i3] (x, y, z); TT tensors are (G1 [n1][r1],
G2 [r1][n2][r2], G3 [r2][n3]).  Everything is float64 (complex128 in Fourier
space).
"""
from __future__ import annotations

import numpy as np

from . import recompress, sinc


# ---------------------------------------------------------------- dense helpers

def unfold(X, p):
    """Mode-p unfolding: n_p x (product of the other sizes)."""
    return np.moveaxis(X, p, 0).reshape(X.shape[p], -1)


def mode_product(X, A, p):
    """X x_p A for A [J][n_p]: entry (.., j, ..) = sum_i A[j, i] X[.., i, ..]."""
    return np.moveaxis(np.tensordot(A, X, axes=(1, p)), 0, p)


def tucker_dense(core, U):
    """Dense tensor of [[core; U1, U2, U3]] (Eq. (tucker_rep))."""
    X = core
    for p in range(3):
        X = mode_product(X, U[p], p)
    return X


def tt_dense(G1, G2, G3):
    """Dense tensor of a 3D TT (Eq. (tt_3d_1))."""
    return np.einsum("ia,ajb,bk->ijk", G1, G2, G3)


# ------------------------------------------------------------ kernels (Sec. 4.2)

def kernel_cp(n, h, tau, alpha, q):
    """CP kernel of component q: (lam [M], [D1, D2, D3]) with D_p [2 n_p - 1][M],
    row J_p + n_p - 1 holding the factor of offset J_p; lam = 1 (the node
    weight is folded into the factors)."""
    D = []
    for d in range(3):
        F = sinc.scaled_factors(n[d], h[d], tau, alpha)
        D.append(F[sinc.phi_types(q)[d]].T.copy())
    return np.ones(len(tau)), D


def cp_dense(lam, D):
    return np.einsum("t,it,jt,kt->ijk", lam, D[0], D[1], D[2])


# ------------------------------------------------------------------ HOOI (Alg. 1)

def _leading(Y, eps):
    u, sig, _vt = np.linalg.svd(Y, full_matrices=False)
    r = recompress.truncation_rank(sig, eps)
    return u[:, :r]


def hooi(X, eps, max_sweeps=20, fit_tol=1e-13):
    """Alg. HOOI on a dense 3-tensor.  Returns (core, [U1, U2, U3], sweeps)."""
    U = [_leading(unfold(X, p), eps) for p in range(3)]          # truncated HOSVD
    fits = []
    sweeps = 0
    for sweeps in range(1, max_sweeps + 1):
        for p in range(3):
            Y = X
            for s in range(3):
                if s != p:
                    Y = mode_product(Y, U[s].T, s)
            U[p] = _leading(unfold(Y, p), eps)
        core = tucker_dense(X, [u.T for u in U])
        fits.append(float(np.sum(core ** 2)))
        if len(fits) > 1 and abs(fits[-1] - fits[-2]) <= fit_tol * max(fits[-1], 1e-300):
            break
    core = tucker_dense(X, [u.T for u in U])
    return core, U, sweeps


# ----------------------------------------------------- DFT and Hadamard (App. B)

def dft_tucker(core, U, L):
    """Lemma DFT_tucker: factor columns zero-padded to L points and transformed."""
    return core, [np.fft.fft(U[p], n=L[p], axis=0) for p in range(3)]


def rowwise_kron(U, V):
    """W[I, l * r + i] = V[I, l] U[I, i]: the factor ((V^T (.) U^T))^T of Eq. (t_had2)."""
    n, r = U.shape
    return (V[:, :, None] * U[:, None, :]).reshape(n, V.shape[1] * r)


def tucker_hadamard(X, Y):
    """Eq. (t_had2): X . Y for Tucker tensors X = (C, U), Y = (D, V)."""
    C, U = X
    D, V = Y
    return np.kron(D, C), [rowwise_kron(U[p], V[p]) for p in range(3)]


# ------------------------------------------------------------ Alg. scpot_fft_tucker

def kernel_tucker(n, h, tau, alpha, tol):
    """Set-up: the three CP kernels compressed to Tucker with tol (HOOI of
    the dense kernel tensors; small grids only)."""
    out = []
    for q in range(3):
        lam, D = kernel_cp(n, h, tau, alpha, q)
        core, U, _sw = hooi(cp_dense(lam, D), tol)
        out.append((core, U))
    return out


def tucker_sum(terms, tol):
    """Approximate summation of Tucker tensors with tol."""
    X = sum(tucker_dense(c, U) for c, U in terms)
    core, U, _sw = hooi(X, tol)
    return core, U


def hadamard_products(kernels, mag, n):
    """The loop of Alg. scpot_fft_tucker: for each component q, the DFT of
    the magnetization, the Hadamard product with the kernel's DFT and the
    inverse DFT, cut to the convolution window.  Returns the three exact
    products as real Tucker tensors."""
    L = [2 * n[p] - 1 for p in range(3)]
    prods = []
    for q in range(3):
        Kc, KU = dft_tucker(*kernels[q], L)                # set-up step: DFT of the kernel
        Mc, MU = dft_tucker(*mag[q], L)
        E, W = tucker_hadamard((Kc, KU), (Mc, MU))
        Wr = []
        for p in range(3):
            w = np.fft.ifft(W[p], axis=0)
            Wr.append(np.real(w[n[p] - 1:2 * n[p] - 1]))
        prods.append((E, Wr))
    return prods


def potential_tucker(mag, n, h, tau, alpha, tol):
    """Alg. scpot_fft_tucker: mag = three Tucker tensors (core, [U1, U2, U3])
    of the magnetization components.  Returns the potential as a Tucker
    tensor (core, U) (kernel units: the same scale as oracle.apply)."""
    kernels = kernel_tucker(n, h, tau, alpha, tol)
    prods = []
    for E, W in hadamard_products(kernels, mag, n):
        core, U, _sw = hooi(tucker_dense(E, W), tol)
        prods.append((core, U))
    return tucker_sum(prods, tol)


def potential_at_cells(mag, n, h, tau, alpha, cells):
    """The Kronecker operator's potential (Cor. kron_op) of a Tucker
    magnetization at target cells (i1, i2, i3), without any dense tensor:
    Eq. (kron_eval_tuck) evaluated row by row, each Toeplitz factor row
    contracted with the factor matrix of its mode."""
    F = [sinc.scaled_factors(n[d], h[d], tau, alpha) for d in range(3)]
    out = np.zeros(len(cells))
    for c, i in enumerate(cells):
        for q in range(3):
            core, U = mag[q]
            ty = sinc.phi_types(q)
            P = []
            for d in range(3):
                j = np.arange(n[d])
                P.append(F[d][ty[d]][:, i[d] - j + n[d] - 1] @ U[d])     # [M][r_d]
            out[c] += np.einsum("abc,ka,kb,kc->", core, P[0], P[1], P[2])
    return out


# ------------------------------------------------------------------- TT (App. C)

def _tail_rank(sig, delta):
    """Smallest r >= 1 with |sig[r:]| <= delta."""
    tail = np.sqrt(np.cumsum((sig ** 2)[::-1])[::-1])
    for r in range(1, len(sig) + 1):
        if r == len(sig) or tail[r] <= delta:
            return r
    return len(sig)


def tt_round(G1, G2, G3, eps):
    """TT rounding of a 3D TT to relative accuracy eps."""
    G1, G2, G3 = (np.asarray(g, dtype=np.float64) for g in (G1, G2, G3))
    # right-to-left orthogonalisation
    Q, R = np.linalg.qr(G3.T)                   # G3 = R^T Q^T
    G3 = Q.T
    G2 = np.einsum("ajb,cb->ajc", G2, R)
    r1, n2, r2 = G2.shape
    Q, R = np.linalg.qr(G2.reshape(r1, n2 * r2).T)
    G2 = Q.T.reshape(-1, n2, r2)
    G1 = G1 @ R.T
    delta = eps / np.sqrt(2.0) * np.linalg.norm(G1)
    # left-to-right truncation
    U, s, Vt = np.linalg.svd(G1, full_matrices=False)
    r = _tail_rank(s, delta)
    G1 = U[:, :r]
    G2 = np.einsum("ab,bjc->ajc", s[:r, None] * Vt[:r], G2)
    r1, n2, r2 = G2.shape
    U, s, Vt = np.linalg.svd(G2.reshape(r1 * n2, r2), full_matrices=False)
    r = _tail_rank(s, delta)
    G2 = U[:, :r].reshape(r1, n2, r)
    G3 = (s[:r, None] * Vt[:r]) @ G3
    return G1, G2, G3


def tt_from_tucker(core, U):
    """Tucker -> TT: G1 = U1, G2 = core x_2 U2, G3 = U3^T."""
    return U[0].copy(), mode_product(core, U[1], 1), U[2].T.copy()


def tt_from_cp(lam, U):
    """CP -> TT (the conversion the paper cites with TT rounding): ranks
    (R, R), G1 = U1, G2[a, :, b] = delta_ab lam_a U2[:, a], G3 = U3^T."""
    R = len(lam)
    G2 = np.zeros((R, U[1].shape[0], R))
    for a in range(R):
        G2[a, :, a] = lam[a] * U[1][:, a]
    return U[0].copy(), G2, U[2].T.copy()


def tucker_from_tt(G1, G2, G3, tol):
    """TT -> Tucker (Eq. (tt_3d_2) read as a Tucker2 tensor [[G2; G1, id,
    G3^T]], then recompressed): HOOI of the dense tensor with tol."""
    core, U, _sw = hooi(tt_dense(G1, G2, G3), tol)
    return core, U
