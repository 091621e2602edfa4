"""Pins of the network and judge references (oracle.mlp, oracle.quadrule)."""
import numpy as np
import pytest

from oracle import exact, mlp, quadrule, sinc
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
    sentinel offsets (to the corner sums' own accuracy)."""
    n = (40, 32, 36)
    h = (1 / 40,) * 3
    J = inputs.sentinel_offsets(n)
    t, a = quadrule.reference_rule(min(h))
    ref = quadrule.kernel_values(n, h, t, a, J)
    ex = []
    for Jv in J:
        lo = tuple(np.array((Jv[d] - 0.5) * h[d]) for d in range(3))
        hi = tuple(np.array((Jv[d] + 0.5) * h[d]) for d in range(3))
        v = [float(exact.potential_kernel_box(lo, hi, q)) for q in range(3)]
        v += [-float(exact.demag_tensor_box(lo, hi, p, q)) for p, q in quadrule.PAIRS]
        ex.append(v)
    assert quadrule.judge(n, h, t, a, np.array(ex), J) < 1e-10


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
    J = inputs.sentinel_offsets(n)
    tr, ar = quadrule.reference_rule(min(h))
    ref = quadrule.kernel_values(n, h, tr, ar, J)
    t, a, _ = quadrule.base_rule(17)
    assert np.isclose(np.linalg.norm(quadrule.residuals(n, h, t, a, ref, J)), quadrule.judge(n, h, t, a, ref, J),
                      rtol=1e-13)


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
    monkeypatch.setattr(quadrule, "residuals", lambda n, h, z, a, ref, J: M @ z - b)
    x1, e0, e1 = quadrule.lm_step(None, None, np.zeros(2 * R), R, None, None, mu=1e-14)
    x = np.linalg.lstsq(M, b, rcond=None)[0]
    assert np.allclose(x1, x, rtol=1e-8, atol=1e-12)
    assert np.isclose(e0, np.linalg.norm(b)) and np.isclose(e1, np.linalg.norm(M @ x - b))
    # damping mu diag(A) shrinks the step: (A + mu D) d = -g
    x2, _, _ = quadrule.lm_step(None, None, np.zeros(2 * R), R, None, None, mu=0.5)
    A = M.T @ M
    assert np.allclose(x2, np.linalg.solve(A + 0.5 * np.diag(np.diag(A)), M.T @ b), rtol=1e-8)
    # steps leaving the output range are projected onto it
    monkeypatch.setattr(quadrule, "residuals", lambda n, h, z, a, ref, J: M @ z - 100 * b)
    x4, _, _ = quadrule.lm_step(None, None, np.zeros(2 * R), R, None, None, mu=1e-14)
    assert np.all(np.abs(x4[:R]) <= quadrule.U_MAX) and np.all(np.abs(x4[R:]) <= quadrule.V_MAX)
    free = np.linalg.lstsq(M, 100 * b, rcond=None)[0]
    assert np.allclose(x4, np.r_[np.clip(free[:R], -0.44, 0.44), np.clip(free[R:], -0.99, 0.99)], rtol=1e-8)


@pytest.mark.slow
def test_lm_fit_lowers_the_judged_error():
    n = (24, 20, 16)
    h = (1 / 24,) * 3
    J = inputs.sentinel_offsets(n)
    tr, ar = quadrule.reference_rule(min(h))
    ref = quadrule.kernel_values(n, h, tr, ar, J)
    R = 8
    x, err = quadrule.lm_fit(n, h, np.zeros(2 * R), R, ref, J, iters=6)
    e_base = quadrule.judge(n, h, *quadrule.base_rule(R)[:2], ref, J)
    assert err < 0.5 * e_base
    assert np.isclose(err, quadrule.judge(n, h, *quadrule.rule_from_uv(x[:R], x[R:], R), ref, J), rtol=1e-12)


def test_judge_error_decreases_with_nodes_and_gradient_is_consistent():
    n = (32, 40, 36)
    h = (1 / 40,) * 3
    J = inputs.sentinel_offsets(n)
    tr, ar = quadrule.reference_rule(min(h))
    ref = quadrule.kernel_values(n, h, tr, ar, J)
    errs = [quadrule.judge(n, h, *quadrule.base_rule(R)[:2], ref, J) for R in (16, 24, 32)]
    assert errs[0] > errs[1] > errs[2]
    t, a, _ = quadrule.base_rule(18)
    gt, ga = quadrule.judge_grad_fd(n, h, t, a, ref, J)
    # a small step against the gradient lowers the error (first-order check)
    s = 1e-5 / np.sqrt(np.sum(gt ** 2) + np.sum((ga * a) ** 2))
    e0 = quadrule.judge(n, h, t, a, ref, J)
    e1 = quadrule.judge(n, h, t - s * gt, a * np.exp(-s * ga * a), ref, J)
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


def test_sentinel_sets_are_in_range_and_disjoint_in_distance():
    for n in [(128, 128, 128), (48, 64, 40), (256, 256, 4), (32, 32, 32)]:
        f = inputs.sentinel_offsets(n, "fit")
        c = inputs.sentinel_offsets(n, "check")
        assert f.shape == c.shape == (256, 3) and f.dtype == np.int32
        for s in (f, c):
            assert np.all(s >= 0) and np.all(s <= np.array(n) - 1)
        assert not np.array_equal(f, c)
    with pytest.raises(ValueError):
        inputs.sentinel_offsets((8, 8, 8), "other")
