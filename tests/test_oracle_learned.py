"""Pins of the network and judge references (oracle.mlp, oracle.quadrule)."""
import numpy as np
import pytest

from oracle import apply, exact, mlp, quadrule, sinc
from paper_1212_3509_amd import inputs


def test_mlp_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = inputs.mlp_init(seed=5, out_scale=1.0).astype(np.float64)
    X = rng.standard_normal((7, 6))
    C = rng.standard_normal((7, 65))
    loss = lambda q: float(np.sum(C * mlp.forward(q, X)[0]))  # noqa: E731
    Y, cache = mlp.forward(p, X)
    g = mlp.backward(p, cache, C)
    idx = rng.choice(p.size, 60, replace=False)
    for i in idx:
        e = np.zeros_like(p)
        e[i] = 1e-6
        fd = (loss(p + e) - loss(p - e)) / 2e-6
        assert abs(fd - g[i]) <= 1e-6 * (1 + abs(fd))


def test_gelu_is_x_times_normal_cdf():
    x = np.linspace(-6, 6, 101)
    from scipy.stats import norm
    assert np.allclose(mlp.gelu(x), x * norm.cdf(x), rtol=1e-14, atol=1e-15)
    assert np.allclose(mlp.gelu_grad(x), (mlp.gelu(x + 1e-6) - mlp.gelu(x - 1e-6)) / 2e-6, atol=1e-8)


def test_adam_first_step_is_signed_lr():
    p = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -0.1, 0.0])
    p1, m, v = mlp.adam(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(p1, p - 0.01 * np.sign(g) * (np.abs(g) > 0), atol=1e-6)


def test_reference_rule_matches_exact_kernels():
    """The judge's reference reproduces the closed-form cell kernels at the
    fit offsets (to the corner sums' own accuracy)."""
    n = (40, 32, 36)
    h = (1 / 40,) * 3
    J, w = inputs.fit_offsets(n)
    t, a = quadrule.reference_rule(min(h))
    ref = quadrule.kernel_values(n, h, t, a, J)
    ex = []
    for Jv in J:
        lo = tuple(np.array((Jv[d] - 0.5) * h[d]) for d in range(3))
        hi = tuple(np.array((Jv[d] + 0.5) * h[d]) for d in range(3))
        v = [float(exact.potential_kernel_box(lo, hi, q)) for q in range(3)]
        v += [-float(exact.demag_tensor_box(lo, hi, p, q)) for p, q in quadrule.PAIRS]
        ex.append(v)
    assert quadrule.judge(n, h, t, a, np.array(ex), J, w) < 1e-10


def test_zero_outputs_give_the_base_rule():
    t, a = quadrule.rule_from_outputs(np.zeros(65), 20, 1 / 48)
    t0, _tau, a0 = sinc.sinc_nodes(20, c0=2.15)
    assert np.array_equal(t, t0) and np.allclose(a, a0, rtol=1e-14, atol=0)


def test_weights_follow_moved_nodes():
    """Moving node k keeps alpha'_k = 2 theta cosh t' sinh^2 t' (trapezoid weight
    of the substituted integrand at the moved node); the weight output scales it."""
    y = np.zeros(65)
    y[3] = 0.7
    y[32 + 5] = -0.4
    t, a = quadrule.rule_from_outputs(y, 12, 1 / 48)
    t0, _tau, a0 = sinc.sinc_nodes(12, c0=2.15)
    th = t0[0]
    assert np.isclose(t[3], t0[3] + 0.45 * th * np.tanh(0.7), rtol=1e-15)
    assert np.isclose(a[3], 2 * th * np.cosh(t[3]) * np.sinh(t[3]) ** 2, rtol=1e-14)
    assert np.isclose(a[5], a0[5] * np.exp(np.tanh(-0.4)), rtol=1e-14)


def test_residual_norm_is_the_judge_error():
    n = (24, 20, 16)
    h = (1 / 24,) * 3
    J, w = inputs.fit_offsets(n)
    tr, ar = quadrule.reference_rule(min(h))
    ref = quadrule.kernel_values(n, h, tr, ar, J)
    t, a, _ = quadrule.base_rule(17)
    assert np.isclose(np.linalg.norm(quadrule.residuals(n, h, t, a, ref, J, w)),
                      quadrule.judge(n, h, t, a, ref, J, w), rtol=1e-13)


def test_outputs_round_trip_through_uv():
    rng = np.random.default_rng(3)
    R = 10
    u = rng.uniform(-0.4, 0.4, R)
    v = rng.uniform(-0.9, 0.9, R)
    y = quadrule.outputs_from_uv(u, v, R)
    t1, a1 = quadrule.rule_from_outputs(y, R)
    t2, a2 = quadrule.rule_from_uv(u, v, R)
    assert np.allclose(t1, t2, rtol=1e-14) and np.allclose(a1, a2, rtol=1e-13)


def test_lm_step_solves_a_linear_problem_exactly(monkeypatch):
    """With residuals linear in x and mu -> 0 one step lands on the least-squares
    solution (pins the normal equations and the damping form)."""
    rng = np.random.default_rng(9)
    R = 3
    M = rng.standard_normal((20, 2 * R))
    b = 0.01 * rng.standard_normal(20)   # solution inside the projection box
    monkeypatch.setattr(quadrule, "rule_from_uv", lambda u, v, R_: (np.r_[u, v], None))
    monkeypatch.setattr(quadrule, "residuals", lambda n, h, z, a, ref, J, w: M @ z - b)
    x1, e0, e1 = quadrule.lm_step(None, None, np.zeros(2 * R), R, None, None, None, mu=1e-14)
    x = np.linalg.lstsq(M, b, rcond=None)[0]
    assert np.allclose(x1, x, rtol=1e-8, atol=1e-12)
    assert np.isclose(e0, np.linalg.norm(b)) and np.isclose(e1, np.linalg.norm(M @ x - b))
    # damping mu diag(A) shrinks the step: (A + mu D) d = -g
    x2, _, _ = quadrule.lm_step(None, None, np.zeros(2 * R), R, None, None, None, mu=0.5)
    A = M.T @ M
    assert np.allclose(x2, np.linalg.solve(A + 0.5 * np.diag(np.diag(A)), M.T @ b), rtol=1e-8)
    # steps leaving the output range are projected onto it
    monkeypatch.setattr(quadrule, "residuals", lambda n, h, z, a, ref, J, w: M @ z - 100 * b)
    x4, _, _ = quadrule.lm_step(None, None, np.zeros(2 * R), R, None, None, None, mu=1e-14)
    assert np.all(np.abs(x4[:R]) <= quadrule.U_MAX) and np.all(np.abs(x4[R:]) <= quadrule.V_MAX)
    free = np.linalg.lstsq(M, 100 * b, rcond=None)[0]
    assert np.allclose(x4, np.r_[np.clip(free[:R], -0.44, 0.44), np.clip(free[R:], -0.99, 0.99)], rtol=1e-8)


@pytest.mark.slow
def test_lm_fit_lowers_the_judged_error():
    n = (24, 20, 16)
    h = (1 / 24,) * 3
    J, w = inputs.fit_offsets(n)
    tr, ar = quadrule.reference_rule(min(h))
    ref = quadrule.kernel_values(n, h, tr, ar, J)
    R = 8
    x, err = quadrule.lm_fit(n, h, np.zeros(2 * R), R, ref, J, w, iters=6)
    e_base = quadrule.judge(n, h, *quadrule.base_rule(R)[:2], ref, J, w)
    assert err < 0.5 * e_base
    assert np.isclose(err, quadrule.judge(n, h, *quadrule.rule_from_uv(x[:R], x[R:], R), ref, J, w), rtol=1e-12)


def test_judge_error_decreases_with_nodes_and_gradient_is_consistent():
    n = (32, 40, 36)
    h = (1 / 40,) * 3
    J, w = inputs.fit_offsets(n)
    tr, ar = quadrule.reference_rule(min(h))
    ref = quadrule.kernel_values(n, h, tr, ar, J)
    errs = [quadrule.judge(n, h, *quadrule.base_rule(R)[:2], ref, J, w) for R in (16, 24, 32)]
    assert errs[0] > errs[1] > errs[2]
    t, a, _ = quadrule.base_rule(18)
    gt, ga = quadrule.judge_grad_fd(n, h, t, a, ref, J, w)
    # a small step against the gradient lowers the error (first-order check)
    e0 = quadrule.judge(n, h, t, a, ref, J, w)
    s = 1e-3 * e0 / (np.sum(gt ** 2) + np.sum((ga * a) ** 2))
    e1 = quadrule.judge(n, h, t - s * gt, a * np.exp(-s * ga * a), ref, J, w)
    # first-order prediction of the decrease: s * |grad|^2 (in t and log alpha)
    pred = s * (np.sum(gt ** 2) + np.sum((ga * a) ** 2))
    assert 0.5 * pred < e0 - e1 < 1.5 * pred


def test_features_layout():
    x = inputs.quad_features([[32, 64, 48]], [1 / 64], [-6.5], [24])
    assert x.shape == (1, 6) and x.dtype == np.float32
    assert np.allclose(x[0], [0.5, 1.0, 0.75, 0.0, 0.0, 0.0])


def test_distill_loss_special_cases():
    xf = np.zeros(64)
    H = np.eye(64)
    y = np.zeros(65)
    y[64] = 2.0
    assert np.isclose(quadrule.distill_loss(y, -1.0, xf, H, 5, 0.1), 0.1 * 9.0)
    y[2] = np.arctanh(0.3 / 0.45)          # u_2 = 0.3 -> ln(1 + 0.09)
    y[40] = 5.0                            # k = 8 >= R: inactive, ignored
    assert np.isclose(quadrule.distill_loss(y, 2.0, xf, H, 5, 0.1), np.log1p(0.09))


def test_fit_offsets_cover_the_operator_norm():
    """The weights of the sampled offsets add up to the number of cell pairs,
    sum over every offset of prod_d (n_d - |J_d|) = prod_d n_d^2; the near
    block carries its exact weights; offsets stay inside the grid."""
    for n in [(128, 128, 128), (48, 64, 40), (256, 256, 4), (32, 32, 32), (3, 4, 2), (1, 1, 7)]:
        J, w = inputs.fit_offsets(n)
        assert J.shape == (256, 3) and J.dtype == np.int32 and w.shape == (256,)
        assert np.all(J >= 0) and np.all(J <= np.array(n) - 1) and np.all(w >= 0)
        assert np.isclose(w.sum(), np.prod([float(v) ** 2 for v in n]), rtol=1e-14)
        near = int(np.prod([min(4, v) for v in n]))        # the near block comes first
        for Jv, wv in zip(J[:near], w[:near]):
            if True:
                c = [(n[d] - Jv[d]) * (1 if Jv[d] == 0 else 2) for d in range(3)]
                assert wv == c[0] * c[1] * c[2]
    with pytest.raises(ValueError):
        inputs.fit_offsets((8, 8, 8), count=10)


def _dense_operators(n, hs, t, alpha):
    """The potential (N x 3N) and field (3N x 3N) matrices of the Kronecker
    operator, column by column from the dense-Toeplitz apply of unit inputs."""
    N = n[0] * n[1] * n[2]
    _t, tau, al = sinc.explicit_nodes(t, alpha)
    P = np.empty((N, 3 * N))
    H = np.empty((3 * N, 3 * N))
    for col in range(3 * N):
        m = np.zeros(3 * N)
        m[col] = 1.0
        phi, h = apply.kron_apply_dense(m.reshape(3, n[2], n[1], n[0]), hs, tau, al)
        P[:, col] = phi.ravel()
        H[:, col] = h.ravel()
    return P, H


def test_certificate_is_the_operator_frobenius_error():
    """Independent route: on a tiny grid, the certificate equals the relative
    Frobenius distance of the dense operator matrices built by applying the
    Kronecker operator to every unit input."""
    n, hs = (3, 4, 2), (0.25, 0.25, 0.25)
    tr, ar = quadrule.reference_rule(0.25)
    Pr, Hr = _dense_operators(n, hs, tr, ar)
    for R in (6, 10):
        t, a, _ = quadrule.base_rule(R)
        P, H = _dense_operators(n, hs, t, a)
        ep, eh = quadrule.certify(n, hs, t, a)
        assert np.isclose(ep, np.linalg.norm(P - Pr) / np.linalg.norm(Pr), rtol=1e-9)
        assert np.isclose(eh, np.linalg.norm(H - Hr) / np.linalg.norm(Hr), rtol=1e-9)
        assert ep > 1e-8 and eh > 1e-8


def test_judge_equals_certificate_when_offsets_cover_the_grid():
    """With every offset in the near block (n_d <= 4) the sampled judge is the
    exact certificate: err^2 = e_phi^2 + e_h^2."""
    n, hs = (4, 3, 4), (0.25, 0.25, 0.25)
    J, w = inputs.fit_offsets(n)
    tr, ar = quadrule.reference_rule(0.25)
    ref = quadrule.kernel_values(n, hs, tr, ar, J)
    t, a, _ = quadrule.base_rule(9)
    ep, eh = quadrule.certify(n, hs, t, a)
    jp, jh = quadrule.judge_parts(n, hs, t, a, ref, J, w)
    assert np.isclose(jp, ep, rtol=1e-9) and np.isclose(jh, eh, rtol=1e-9)


@pytest.mark.slow
def test_sampled_judge_tracks_the_certificate():
    """On a 48^3 grid the 256 weighted offsets estimate the exact
    certificate of plain rules within 25 % (shell representatives stand for
    the far offsets)."""
    n = (48, 48, 48)
    hs = (1 / 48,) * 3
    J, w = inputs.fit_offsets(n)
    tr, ar = quadrule.reference_rule(hs[0])
    ref = quadrule.kernel_values(n, hs, tr, ar, J)
    for R in (18, 22, 26):
        t, a, _ = quadrule.base_rule(R)
        ep, eh = quadrule.certify(n, hs, t, a)
        jp, jh = quadrule.judge_parts(n, hs, t, a, ref, J, w)
        assert 0.75 < jp / ep < 1.25 and 0.75 < jh / eh < 1.25, (R, jp, ep, jh, eh)
