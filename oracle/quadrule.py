"""Shortened quadrature rules and their judge (float64 reference).

TEST INFRASTRUCTURE ONLY (see the package header).

The node-proposal network is an addition on top of the paper's method.  Its
outputs modify a base rule, and a judge measures the resulting operator error:

  base rule   the sinc rule of Cor. kron_op with R' nodes and c0 = 2.15,
              theta = c0 ln(R')/R', t_k = k theta, alpha_k = 2 theta cosh t_k sinh^2 t_k;
  offsets     t'_k = t_k + 0.45 theta tanh(y_k),
              alpha'_k = 2 theta cosh t'_k sinh^2 t'_k exp(tanh(y_{32+k})),  k < R'
              (y: network output; the weight follows its node, so moving a
              node keeps the trapezoid weight of the substituted integrand);
  reference   the sinc rule with the step of Thm. sinc_theo and 96 nodes;
  fallback    the same with the fewest nodes in 33..64 whose certificate meets
              the tolerance (64 when none does);
  kernels     at an offset J, nine values: the potential kernels K^x, K^y,
              K^z (Cor. kron_op) and the field kernels F_pq of h_p <- m_q for
              p <= q (the same with the derivative factors; F_pq = F_qp);
  certificate the relative Frobenius-norm error of the discrete operators,
              separately for the potential P (3N -> N) and the field H
              (3N -> 3N), against the reference rule:
                e_phi^2 = sum_J w(J) sum_q dK^q(J)^2 / sum_J w(J) sum_q K^q_ref(J)^2,
                e_h^2   = sum_J w(J) sum_pq m_pq dF_pq(J)^2 / (same with F_ref),
              over every offset of the grid, w(J) = prod_d (n_d - |J_d|)
              (the number of cell pairs at offset J), m_pq = 1 on the diagonal
              and 2 off it.  Since |A|_F^2 = sum_ij A_ij^2, this is the exact
              relative L2 error of the outputs averaged over inputs with
              independent, equal-variance cell values;
  judge       the same sums over a set of sampled offsets J_s with weights
              w_s (``inputs.fit_offsets``: the near block exactly, shells of
              far offsets by representatives): err = sqrt(e_phi^2 + e_h^2);
  fit         per grid, damped Gauss-Newton (Levenberg-Marquardt) on the
              residual vector r_(s,c) = sqrt(w_s m_c / D_c) dK_c(J_s) (|r| =
              err; D_c the reference's weighted sum of its class) in
              u_k = 0.45 tanh(y_k), v_k = tanh(y_{32+k}) (k < R'; t'_k =
              t_k + theta u_k, alpha' carries exp(v_k)): a step solves
              (A + mu diag A) d = -J^T r with A = J^T J, is projected onto
              |u| <= 0.44, |v| <= 0.99 (the range the outputs reach), and is
              kept when it lowers err (mu / 3), else mu * 4.  The fitted
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


# multiplicity of each of the nine kernel values in the operator's Frobenius
# norm (F_pq = F_qp for p != q counts twice)
MULT = np.array([1, 1, 1, 1, 1, 1, 2, 2, 2], dtype=np.float64)


def judge_parts(n, h, t, alpha, ref, J, w):
    """(e_phi, e_h) of the rule (t, alpha) against reference kernel values
    ``ref`` at offsets J with weights w."""
    K = kernel_values(n, h, t, alpha, J)
    w = np.asarray(w, dtype=np.float64)[:, None]
    d2 = w * (K - ref) ** 2 * MULT
    r2 = w * np.asarray(ref) ** 2 * MULT
    return float(np.sqrt(d2[:, :3].sum() / r2[:, :3].sum())), float(np.sqrt(d2[:, 3:].sum() / r2[:, 3:].sum()))


def judge(n, h, t, alpha, ref, J, w):
    """err = sqrt(e_phi^2 + e_h^2) of the rule (t, alpha) at weighted offsets."""
    ep, eh = judge_parts(n, h, t, alpha, ref, J, w)
    return float(np.hypot(ep, eh))


def judge_grad_fd(n, h, t, alpha, ref, J, w, rel=1e-6):
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
        gt[k] = (judge(n, h, tp, alpha, ref, J, w) - judge(n, h, tm, alpha, ref, J, w)) / (2 * dt)
        da = rel * abs(alpha[k])
        ap, am = alpha.copy(), alpha.copy()
        ap[k] += da
        am[k] -= da
        ga[k] = (judge(n, h, t, ap, ref, J, w) - judge(n, h, t, am, ref, J, w)) / (2 * da)
    return gt, ga


def residuals(n, h, t, alpha, ref, J, w):
    """Residual vector whose 2-norm is the judge's err: rows (J, component)."""
    K = kernel_values(n, h, t, alpha, J)
    w = np.asarray(w, dtype=np.float64)[:, None]
    ref = np.asarray(ref)
    D_phi = (w * ref[:, :3] ** 2).sum()
    D_h = (w * ref[:, 3:] ** 2 * MULT[3:]).sum()
    scale = np.sqrt(w * MULT[None, :] / np.r_[np.full(3, D_phi), np.full(6, D_h)][None, :])
    return ((K - ref) * scale).ravel()


def certify(n, h, t, alpha, t_ref=None, a_ref=None):
    """Exact (e_phi, e_h) of the rule (t, alpha) over every offset of the grid
    n (cell sizes h), against the reference rule (default: reference_rule of
    the smallest cell).  Full kernel tensors: small grids only."""
    if t_ref is None:
        t_ref, a_ref = reference_rule(min(h))
    types = [sinc.phi_types(q) for q in range(3)] + [sinc.field_types(p, q) for p, q in PAIRS]

    def tensors(tt, aa):
        tau = np.sinh(np.asarray(tt, dtype=np.float64))
        F = [sinc.scaled_factors(n[d], h[d], tau, aa)[:, :, n[d] - 1:] for d in range(3)]   # J >= 0
        out = []
        for ty in types:
            A = (F[2][ty[2]][:, :, None] * F[1][ty[1]][:, None, :]).reshape(tau.size, -1)
            out.append(np.tensordot(A, F[0][ty[0]], axes=([0], [0])).reshape(n[2], n[1], n[0]))
        return out

    c = [np.array([(nd - j) * (1.0 if j == 0 else 2.0) for j in range(nd)]) for nd in n]
    W = c[2][:, None, None] * c[1][None, :, None] * c[0][None, None, :]
    K, R = tensors(t, alpha), tensors(t_ref, a_ref)
    num = [m * np.sum(W * (a - b) ** 2) for a, b, m in zip(K, R, MULT)]
    den = [m * np.sum(W * b ** 2) for b, m in zip(R, MULT)]
    return float(np.sqrt(sum(num[:3]) / sum(den[:3]))), float(np.sqrt(sum(num[3:]) / sum(den[3:])))


U_MAX, V_MAX = 0.44, 0.99


def lm_step(n, h, x, R, ref, J, w, mu, rel=1e-6):
    """One damped Gauss-Newton step from x = (u_0..u_{R-1}, v_0..v_{R-1}) (the
    Jacobian by central differences), projected onto the output range.
    Returns (x + d, err(x), err(x + d))."""
    x = np.asarray(x, dtype=np.float64)

    def res(z):
        return residuals(n, h, *rule_from_uv(z[:R], z[R:], R), ref, J, w)

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


def lm_fit(n, h, x0, R, ref, J, w, iters, mu0=1e-3):
    """Levenberg-Marquardt iterations from x0 (accept when err drops)."""
    x = np.asarray(x0, dtype=np.float64).copy()
    mu = mu0
    err = None
    for _ in range(iters):
        x1, e0, e1 = lm_step(n, h, x, R, ref, J, w, mu)
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
