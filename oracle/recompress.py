"""Tolerance-controlled recompression of a CP tensor to Tucker form.

TEST INFRASTRUCTURE ONLY (see the package header).

Paper: Sec. 2.2, Eq. (Tucker_fitting3) and Alg. HOOI (higher-order
orthogonal iteration, an alternating least-squares method): initialise the
factor matrices (HOSVD), then for p = 1..3 project the tensor on the other
two factor spaces, take the leading left singular vectors of the mode-p
unfolding of the projection, with the rank chosen by the tolerance, until
the fit stops improving; the core is the projection on all three.  The
remark after the algorithm: for a tensor given as a sum of terms (CP / block
CP) the mode products are formed term by term.

Reading of the rank rule (its printed form is garbled): r_p is the smallest
r for which the discarded singular values carry a Frobenius norm of at most
eps / sqrt(3) times that of all of them, so that the three truncations
together keep the relative error at most eps (HOSVD bound).

A CP tensor here is X[i1, i2, i3] = sum_t lam[t] A[0][t, i1] A[1][t, i2]
A[2][t, i3]: factor columns as rows of A[p] ([T][n_p]), weights lam [T].
Everything is float64 NumPy; SVDs are numpy.linalg.svd.
"""
from __future__ import annotations

import numpy as np


def cp_dense(A, lam):
    """Dense [n1][n2][n3] tensor of a CP tensor (small sizes only)."""
    return np.einsum("t,ta,tb,tc->abc", lam, A[0], A[1], A[2])


def tucker_dense(core, U):
    """Dense tensor of the Tucker tensor [[core; U1, U2, U3]] (U_p [n_p][r_p])."""
    return np.einsum("abc,xa,yb,zc->xyz", core, U[0], U[1], U[2])


def cp_norm2(A, lam):
    """Squared Frobenius norm: lam^T (G1 o G2 o G3) lam with G_p = A_p A_p^T."""
    G = np.ones((len(lam), len(lam)))
    for p in range(3):
        G *= A[p] @ A[p].T
    return float(lam @ G @ lam)


def residual_norm2(A, lam, U):
    """|X - X x_1 P1 x_2 P2 x_3 P3|^2 for the projectors P_p = U_p U_p^T,
    without the cancellation of |X|^2 - |core|^2: the residual splits into
    the mutually orthogonal parts (I - P1) X, P1 (I - P2) X, P1 P2 (I - P3) X,
    each a CP tensor whose squared norm is a weighted product of Gram
    matrices of its columns."""
    total = 0.0
    for p in range(3):
        G = np.ones((len(lam), len(lam)))
        for j in range(3):
            if j < p:
                C = A[j] @ U[j]                          # projected columns, coordinates
            elif j == p:
                C = A[j] - (A[j] @ U[j]) @ U[j].T        # residual columns
            else:
                C = A[j]
            G *= C @ C.T
        total += float(lam @ G @ lam)
    return total


def others(p):
    return [q for q in range(3) if q != p]


def projected_unfolding(A, lam, p, U):
    """Mode-p unfolding of X x_q U_q^T x_s U_s^T (q < s the other modes; a
    None factor leaves its mode unprojected): n_p x (r_q r_s), column index
    a * r_s + b for the (q, s) indices (a, b).  Term by term: the projection
    of term t is a_t^(p) o (U_q^T a_t^(q)) o (U_s^T a_t^(s))."""
    q, s = others(p)
    Wq = A[q] if U[q] is None else A[q] @ U[q]            # [T][r_q]
    Ws = A[s] if U[s] is None else A[s] @ U[s]            # [T][r_s]
    kr = (Wq[:, :, None] * Ws[:, None, :]).reshape(len(lam), -1)   # [T][r_q r_s]
    return A[p].T @ (lam[:, None] * kr)


def truncation_rank(sigma, eps):
    """Smallest r >= 1 whose discarded tail sigma[r:] has norm <= eps/sqrt(3) * |sigma|."""
    total = float(np.sqrt(np.sum(sigma ** 2)))
    if total == 0.0:
        return 1
    tail = np.sqrt(np.cumsum((sigma ** 2)[::-1])[::-1])   # tail[r] = |sigma[r:]|
    bound = eps / np.sqrt(3.0) * total
    for r in range(1, len(sigma) + 1):
        if r == len(sigma) or tail[r] <= bound:
            return r
    return len(sigma)


def leading_vectors(Y, eps, rmax=None):
    """Left singular vectors of Y truncated by the rank rule (and rmax)."""
    u, sig, _vt = np.linalg.svd(Y, full_matrices=False)
    r = truncation_rank(sig, eps)
    if rmax is not None:
        r = min(r, rmax)
    return u[:, :r], sig


def tucker_core(A, lam, U):
    """Core X x_1 U1^T x_2 U2^T x_3 U3^T, term by term."""
    P = [A[p] @ U[p] for p in range(3)]
    return np.einsum("t,ta,tb,tc->abc", lam, P[0], P[1], P[2])


def hosvd(A, lam, eps, rmax=None):
    """Truncated HOSVD: per mode, the leading left singular vectors of the
    full (unprojected) unfolding.  Small sizes only (the unfolding is
    n_p x n_q n_s)."""
    U = []
    for p in range(3):
        u, _sig = leading_vectors(projected_unfolding(A, lam, p, [None, None, None]), eps, rmax)
        U.append(u)
    return U


def hooi(A, lam, eps, rmax=None, max_sweeps=20, fit_tol=1e-13, U0=None):
    """HOOI for a CP tensor (Alg. HOOI).  Returns dict(U, core, ranks,
    rel_err, sweeps, fits): rel_err = |X - [[core; U]]| / |X| (from
    residual_norm2), fits the squared core norm after each sweep."""
    U = list(U0) if U0 is not None else hosvd(A, lam, eps, rmax)
    nx2 = cp_norm2(A, lam)
    fits = []
    sweeps = 0
    for sweeps in range(1, max_sweeps + 1):
        for p in range(3):
            Up = list(U)
            Up[p] = None
            U[p], _sig = leading_vectors(projected_unfolding(A, lam, p, Up), eps, rmax)
        core = tucker_core(A, lam, U)
        fits.append(float(np.sum(core ** 2)))
        if len(fits) > 1 and abs(fits[-1] - fits[-2]) <= fit_tol * max(fits[-1], 1e-300):
            break
    core = tucker_core(A, lam, U)
    err = np.sqrt(max(residual_norm2(A, lam, U), 0.0) / nx2) if nx2 > 0 else 0.0
    return {"U": U, "core": core, "ranks": tuple(u.shape[1] for u in U), "rel_err": float(err),
            "sweeps": sweeps, "fits": fits}


def tucker_as_cp(core, U):
    """A Tucker tensor written as a CP tensor: one term per core entry."""
    r1, r2, r3 = core.shape
    A = [np.empty((r1 * r2 * r3, U[p].shape[0])) for p in range(3)]
    lam = np.empty(r1 * r2 * r3)
    t = 0
    for a in range(r1):
        for b in range(r2):
            for c in range(r3):
                lam[t] = core[a, b, c]
                A[0][t], A[1][t], A[2][t] = U[0][:, a], U[1][:, b], U[2][:, c]
                t += 1
    return A, lam
