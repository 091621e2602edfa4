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
              alpha'_k = 2 theta cosh t'_k sinh^2 t'_k exp(tanh(y_{32+k})),  k < R'
              (y: network output; the weight follows its node, so moving a
              node keeps the trapezoid weight of the substituted integrand);
  reference   the sinc rule with the step of Thm. sinc_theo and 96 nodes;
  fallback    the same with 64 nodes (accurate to ~1e-9 up to 1024 cells);
  judge       at the sentinel offsets J of the grid, the nine kernel values
              (potential K^x, K^y, K^z and field factors of h_p <- m_q for
              p <= q, Cor. kron_op with the derivative factors) of the rule
              are compared with those of a reference rule:
              err = sqrt( mean_J |K'(J) - K_ref(J)|^2 / |K_ref(J)|^2 );
  fit         per grid, damped Gauss-Newton (Levenberg-Marquardt) on the
              residual vector r = (K' - K_ref)(J) / sqrt(S |K_ref(J)|^2)
              (|r| = err) in u_k = 0.45 tanh(y_k), v_k = tanh(y_{32+k})
              (k < R'; t'_k = t_k + theta u_k, alpha' carries exp(v_k)): a step
              solves (A + mu diag A) d = -J^T r with A = J^T J, is projected
              onto |u| <= 0.44, |v| <= 0.99 (the range the outputs reach), and
              is kept when it lowers err (mu / 3), else mu * 4.  The fitted
              outputs y = atanh(u / 0.45), atanh(v) are the network's training
              targets.
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


def rule_from_uv(u, v, R: int):
    """Rule with node offsets u (units of theta) and log-weight factors v."""
    t, _alpha, theta = base_rule(R)
    tp = t + theta * np.asarray(u, dtype=np.float64)[:R]
    ap = 2.0 * theta * np.cosh(tp) * np.sinh(tp) ** 2 * np.exp(np.asarray(v, dtype=np.float64)[:R])
    return tp, ap


def rule_from_outputs(y, R: int, h_min: float = None):
    """Learned rule from one network output vector y (65 values)."""
    y = np.asarray(y, dtype=np.float64)
    return rule_from_uv(0.45 * np.tanh(y[:R]), np.tanh(y[32:32 + R]), R)


def outputs_from_uv(u, v, R: int):
    """Network outputs that reproduce (u, v): atanh(u / 0.45), atanh(v)."""
    y = np.zeros(65)
    y[:R] = np.arctanh(np.asarray(u)[:R] / 0.45)
    y[32:32 + R] = np.arctanh(np.asarray(v)[:R])
    return y


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


def residuals(n, h, t, alpha, ref, J):
    """Residual vector whose 2-norm is the judge's err: rows (J, component)."""
    K = kernel_values(n, h, t, alpha, J)
    den = np.sum(ref ** 2, axis=1)
    return ((K - ref) / np.sqrt(den * len(J))[:, None]).ravel()


U_MAX, V_MAX = 0.44, 0.99


def lm_step(n, h, x, R, ref, J, mu, rel=1e-6):
    """One damped Gauss-Newton step from x = (u_0..u_{R-1}, v_0..v_{R-1}) (the
    Jacobian by central differences), projected onto the output range.
    Returns (x + d, err(x), err(x + d))."""
    x = np.asarray(x, dtype=np.float64)

    def res(z):
        return residuals(n, h, *rule_from_uv(z[:R], z[R:], R), ref, J)

    r0 = res(x)
    Jac = np.empty((r0.size, 2 * R))
    for p in range(2 * R):
        xp, xm = x.copy(), x.copy()
        xp[p] += rel
        xm[p] -= rel
        Jac[:, p] = (res(xp) - res(xm)) / (2 * rel)
    A = Jac.T @ Jac
    g = Jac.T @ r0
    step = np.linalg.solve(A + mu * np.diag(np.diag(A)), -g)
    x1 = x + step
    x1[:R] = np.clip(x1[:R], -U_MAX, U_MAX)
    x1[R:] = np.clip(x1[R:], -V_MAX, V_MAX)
    return x1, float(np.linalg.norm(r0)), float(np.linalg.norm(res(x1)))


def lm_fit(n, h, x0, R, ref, J, iters, mu0=1e-3):
    """Levenberg-Marquardt iterations from x0 (accept when err drops)."""
    x = np.asarray(x0, dtype=np.float64).copy()
    mu = mu0
    err = None
    for _ in range(iters):
        x1, e0, e1 = lm_step(n, h, x, R, ref, J, mu)
        err = e0 if err is None else err
        if e1 < err:
            x, err, mu = x1, e1, max(mu / 3.0, 1e-12)
        else:
            mu = min(mu * 4.0, 1e12)
    return x, err


def distill_loss(y, t64, xfit, H, R: int, lam: float):
    """Training loss of one case: ln(1 + d^T H d) + lam (y_64 - t_64)^2 with
    d = (0.45 tanh y_k, tanh y_{32+k}) - xfit over the active outputs."""
    y = np.asarray(y, dtype=np.float64)
    x = np.r_[0.45 * np.tanh(y[:32]), np.tanh(y[32:64])]
    act = (np.arange(64) % 32) < R
    d = np.where(act, x - np.asarray(xfit, dtype=np.float64), 0.0)
    return float(np.log1p(d @ np.asarray(H, dtype=np.float64) @ d) + lam * (y[64] - t64) ** 2)
