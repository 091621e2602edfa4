"""Sinc quadrature nodes and the 1D factors of the Kronecker operator.

TEST INFRASTRUCTURE ONLY (see the package header).

Paper: Sec. 3.3 (sinc quadrature, Eq. (sinc_int), Thm. sinc_theo), Sec. 3.4
(Gaussian transform Eq. (gauss_trans), separable integrands Eq.
(sep_integrands), Lemma sinc_mumag, Cor. kron_op) and Sec. 4.2 (Toeplitz form,
Eq. (conv_op), Eq. (conv_pot)).

Readings adopted here:
  * Weights.  With tau = sinh t the Gaussian-transform integrand is even in t
    and vanishes at t = 0, so the symmetric sinc rule over k = -M..M collapses
    to the M terms k = 1..M with weight 2*theta*cosh(t_k)*sinh(t_k)^2 (the
    alpha_k printed in Cor. kron_op lacks the step theta and the factor 2 of the
    folded +-k pair).  Combined with the 2/sqrt(pi) of Eq. (gauss_trans) and
    the 1/(4 pi) of the potential, the weight of node k in the potential kernel
    is  W_k = alpha_k / (2 pi^(3/2)),  alpha_k = 2 theta cosh t_k sinh^2 t_k.
  * "R" in Cor. kron_op counts the nonzero terms; here it is M (the sinc rule
    has 2M+1 points, e.g. M = 40 <-> 81 points).
  * Step.  theta = c0 ln(M)/M with c0 = 2.15 (Cor. kron_op, Sec. 3.5) by
    default; alternatively the step of Thm. sinc_theo, theta = ln(2 pi a M / b)
    / (a M), with a = 2 and b = rho_min / 4 for rho_min = (h_min/2)^2 (the
    double-exponential decay exp(-rho sinh^2 t) ~ exp(-(rho/4) e^(2|t|))).
  * Sign: physical (see oracle.exact).  The stored factors fold the node
    weight in as W_k^(1/3) per axis and the minus sign of h = -grad phi into
    the derivative factors.

Factor types for one axis with cell size h, offsets J = -(n-1)..n-1, interval
[a_J, b_J] = [(J - 1/2)h, (J + 1/2)h] and tau = tau_k:
  E(J)  = int_a^b exp(-tau^2 x^2) dx                  (axes p != q)
  X(J)  = int_a^b x exp(-tau^2 x^2) dx                (axis p = q)
  X'(J) = d/ds of X over [s - h/2, s + h/2] = b e^(-tau^2 b^2) - a e^(-tau^2 a^2)
  E'(J) = d/ds of E over [s - h/2, s + h/2] = -2 tau^2 X(J)
Stored (scaled) types, index order used everywhere: 0 = E~ = w E, 1 = X~ = w X,
2 = P~ = -w X', 3 = Q~ = -w E' = 2 tau^2 w X, with w = W_k^(1/3).
"""
from __future__ import annotations

import numpy as np
from scipy import special

SQRT_PI = np.sqrt(np.pi)
C_PHI = 1.0 / (2.0 * np.pi ** 1.5)
TYPE_E, TYPE_X, TYPE_P, TYPE_Q = 0, 1, 2, 3


def sinc_nodes(M: int, c0: float = 2.15, step_rule: int = 0, h_min: float | None = None):
    """Nodes t_k = k theta, k = 1..M, tau_k = sinh t_k, and alpha_k.

    step_rule 0: theta = c0 ln M / M          (Cor. kron_op)
    step_rule 1: theta = ln(2 pi a M / b)/(aM) (Thm. sinc_theo), a = 2,
                 b = (h_min/2)^2 / 4 in the unit-scaled domain.
    """
    if step_rule == 0:
        theta = c0 * np.log(M) / M
    else:
        a = 2.0
        b = (0.5 * h_min) ** 2 / 4.0
        theta = np.log(2.0 * np.pi * a * M / b) / (a * M)
    t = theta * np.arange(1, M + 1, dtype=np.float64)
    tau = np.sinh(t)
    alpha = 2.0 * theta * np.cosh(t) * np.sinh(t) ** 2
    return t, tau, alpha


def explicit_nodes(t, alpha):
    """Explicit rule: nodes t_k (tau_k = sinh t_k) with weights alpha_k that
    play the role of 2 theta cosh t_k sinh^2 t_k."""
    t = np.asarray(t, dtype=np.float64)
    return t, np.sinh(t), np.asarray(alpha, dtype=np.float64)


def node_weights(alpha):
    """W_k = alpha_k / (2 pi^(3/2)): weight of node k in the potential kernel."""
    return C_PHI * np.asarray(alpha, dtype=np.float64)


def factor_E(tau: float, n: int, h: float):
    """E(J), J = -(n-1)..n-1, as erf differences; for intervals far on one
    side of 0 the equal difference of erfc is used (same value, no cancellation);
    even in J."""
    J = np.arange(0, n, dtype=np.float64)
    a = (J - 0.5) * h
    b = (J + 0.5) * h
    far = tau * a > 0.5
    diff = np.where(far, special.erfc(tau * a) - special.erfc(tau * b),
                    special.erf(tau * b) - special.erf(tau * a))
    pos = (np.sqrt(np.pi) / (2.0 * tau)) * diff
    pos[0] = (np.sqrt(np.pi) / tau) * special.erf(tau * 0.5 * h)
    return np.concatenate([pos[:0:-1], pos])


def factor_X(tau: float, n: int, h: float):
    """X(J) = (exp(-tau^2 a^2) - exp(-tau^2 b^2)) / (2 tau^2), written as
    -exp(-tau^2 a^2) expm1(-tau^2 (b^2 - a^2)) / (2 tau^2); odd in J."""
    J = np.arange(0, n, dtype=np.float64)
    a = (J - 0.5) * h
    b = (J + 0.5) * h
    t2 = tau * tau
    pos = -np.exp(-t2 * a * a) * np.expm1(-t2 * (b * b - a * a)) / (2.0 * t2)
    pos[0] = 0.0
    return np.concatenate([-pos[:0:-1], pos])


def factor_Xp(tau: float, n: int, h: float):
    """X'(J) = b exp(-tau^2 b^2) - a exp(-tau^2 a^2); even in J."""
    J = np.arange(0, n, dtype=np.float64)
    a = (J - 0.5) * h
    b = (J + 0.5) * h
    t2 = tau * tau
    pos = b * np.exp(-t2 * b * b) - a * np.exp(-t2 * a * a)
    return np.concatenate([pos[:0:-1], pos])


def scaled_factors(n: int, h: float, tau, alpha):
    """Stored factors for one axis: array [4][M][2n-1] of E~, X~, P~, Q~
    (see the module header), node weight W_k^(1/3) folded into each."""
    tau = np.asarray(tau, dtype=np.float64)
    W = node_weights(alpha)
    w = np.cbrt(W)
    M = tau.size
    out = np.empty((4, M, 2 * n - 1))
    for k in range(M):
        E = factor_E(tau[k], n, h)
        X = factor_X(tau[k], n, h)
        Xp = factor_Xp(tau[k], n, h)
        out[TYPE_E, k] = w[k] * E
        out[TYPE_X, k] = w[k] * X
        out[TYPE_P, k] = -w[k] * Xp
        out[TYPE_Q, k] = 2.0 * tau[k] ** 2 * w[k] * X
    return out


def toeplitz(g: np.ndarray) -> np.ndarray:
    """Dense n x n Toeplitz matrix T[i][j] = g[i - j + n - 1] from a generator
    of length 2n - 1 (the offset J = i - j of Sec. 4.2)."""
    n = (g.size + 1) // 2
    i = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    return g[i - j + n - 1]


def kernel_from_factors(fx, fy, fz, J):
    """Sinc approximation of one kernel entry at offset J = (Jx, Jy, Jz) from
    per-node factor vectors fx[k][.], fy[k][.], fz[k][.] (already weighted):
    sum_k fx[k][Jx+nx-1] fy[k][Jy+ny-1] fz[k][Jz+nz-1]."""
    nx = (fx.shape[1] + 1) // 2
    ny = (fy.shape[1] + 1) // 2
    nz = (fz.shape[1] + 1) // 2
    return float(np.sum(fx[:, J[0] + nx - 1] * fy[:, J[1] + ny - 1] * fz[:, J[2] + nz - 1]))


# types per axis d for the potential from component q, and for h_p from m_q
def phi_types(q: int):
    """Factor type per axis (x, y, z) of the potential kernel K^q."""
    return tuple(TYPE_X if d == q else TYPE_E for d in range(3))


def field_types(p: int, q: int):
    """Factor type per axis of the field contribution h_p <- m_q: the
    potential kernel K^q differentiated in the target coordinate p."""
    t = list(phi_types(q))
    t[p] = TYPE_P if t[p] == TYPE_X else TYPE_Q
    return tuple(t)
