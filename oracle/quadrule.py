"""Shortened quadrature rules and their judge (float64 reference).

TEST INFRASTRUCTURE ONLY (see the package header).

The node-proposal network is an addition on top of the paper's method.  Its
outputs modify a base rule, and a judge measures the resulting kernel error:

  base rule   the sinc rule of Cor. kron_op with R' nodes and c0 = 2.15,
              theta = c0 ln(R')/R', t_k = k theta, alpha_k = 2 theta cosh t_k sinh^2 t_k
              (a least-squares fit of R' nodes and weights on the judge's
              residuals lands close to this rule, with end corrections of a
              few percent; the network learns such corrections);
  offsets     t'_k = t_k + 0.45 theta tanh(y_k),
              alpha'_k = alpha_k exp(tanh(y_{32+k})),  k < R' (y: network output);
  reference   the sinc rule with the step of Thm. sinc_theo and 96 nodes;
  fallback    the same with 64 nodes (accurate to ~1e-9 up to 1024 cells);
  judge       at the sentinel offsets J of the grid, the nine kernel values
              (potential K^x, K^y, K^z and field factors of h_p <- m_q for
              p <= q, Cor. kron_op with the derivative factors) of the rule
              are compared with those of a reference rule:
              err = sqrt( mean_J |K'(J) - K_ref(J)|^2 / |K_ref(J)|^2 ).
"""
from __future__ import annotations

import numpy as np

from . import sinc

PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


def base_rule(R: int, h_min: float = None):
    t, _tau, alpha = sinc.sinc_nodes(R, c0=2.15, step_rule=0)
    theta = t[0]
    return t, alpha, theta


def reference_rule(h_min: float, M: int = 96):
    t, _tau, alpha = sinc.sinc_nodes(M, step_rule=1, h_min=h_min)
    return t, alpha


def rule_from_outputs(y, R: int, h_min: float):
    """Learned rule from one network output vector y (65 values)."""
    t, alpha, theta = base_rule(R, h_min)
    y = np.asarray(y, dtype=np.float64)
    tp = t + 0.45 * theta * np.tanh(y[:R])
    ap = alpha * np.exp(np.tanh(y[32:32 + R]))
    return tp, ap


def kernel_values(n, h, t, alpha, J):
    """Nine kernel values per offset (rows of J): [K^x, K^y, K^z, F_xx, F_yy,
    F_zz, F_xy, F_xz, F_yz] with F_pq the factor triple of h_p <- m_q."""
    t = np.asarray(t, dtype=np.float64)
    tau = np.sinh(t)
    F = [sinc.scaled_factors(n[d], h[d], tau, alpha) for d in range(3)]
    out = np.empty((len(J), 9))
    for r, Jv in enumerate(np.asarray(J)):
        vals = [sinc.kernel_from_factors(*[F[d][ty] for d, ty in enumerate(sinc.phi_types(q))], Jv)
                for q in range(3)]
        for p, q in PAIRS:
            ty = sinc.field_types(p, q)
            vals.append(sinc.kernel_from_factors(F[0][ty[0]], F[1][ty[1]], F[2][ty[2]], Jv))
        out[r] = vals
    return out


def judge(n, h, t, alpha, ref, J):
    """err of the rule (t, alpha) against reference kernel values ``ref``."""
    K = kernel_values(n, h, t, alpha, J)
    num = np.sum((K - ref) ** 2, axis=1)
    den = np.sum(ref ** 2, axis=1)
    return float(np.sqrt(np.mean(num / den)))


def judge_grad_fd(n, h, t, alpha, ref, J, rel=1e-6):
    """Central differences of err with respect to t_k and alpha_k."""
    t = np.asarray(t, dtype=np.float64)
    alpha = np.asarray(alpha, dtype=np.float64)
    gt = np.zeros_like(t)
    ga = np.zeros_like(alpha)
    for k in range(t.size):
        dt = rel * max(1.0, abs(t[k]))
        tp, tm = t.copy(), t.copy()
        tp[k] += dt
        tm[k] -= dt
        gt[k] = (judge(n, h, tp, alpha, ref, J) - judge(n, h, tm, alpha, ref, J)) / (2 * dt)
        da = rel * abs(alpha[k])
        ap, am = alpha.copy(), alpha.copy()
        ap[k] += da
        am[k] -= da
        ga[k] = (judge(n, h, t, ap, ref, J) - judge(n, h, t, am, ref, J)) / (2 * da)
    return gt, ga
