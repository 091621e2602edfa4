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
    assert np.array_equal(t, t0) and np.array_equal(a, a0)


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
