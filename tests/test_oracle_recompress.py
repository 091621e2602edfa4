"""Pins of the oracle's HOOI recompression (CPU)."""
import numpy as np
import pytest

from oracle import recompress as rc


def _orth(rng, n, r):
    q, _ = np.linalg.qr(rng.standard_normal((n, r)))
    return q


def _known_tucker(seed=0, n=(20, 18, 16), r=(3, 4, 5)):
    rng = np.random.default_rng(seed)
    U = [_orth(rng, n[p], r[p]) for p in range(3)]
    core = rng.standard_normal(r)
    return core, U


def test_dense_unfolding_matches_structured_unfolding():
    """The term-by-term unfolding equals numpy's reshape of the dense tensor
    (independent route; pins the Khatri-Rao column order)."""
    rng = np.random.default_rng(1)
    n = (7, 6, 5)
    A = [rng.standard_normal((9, n[p])) for p in range(3)]
    lam = rng.standard_normal(9)
    X = rc.cp_dense(A, lam)
    for p in range(3):
        q, s = rc.others(p)
        dense = np.transpose(X, (p, q, s)).reshape(n[p], -1)
        assert np.allclose(rc.projected_unfolding(A, lam, p, [None] * 3), dense, rtol=1e-13, atol=1e-13)


def test_norm_and_error_formula():
    rng = np.random.default_rng(2)
    n = (8, 7, 6)
    A = [rng.standard_normal((5, n[p])) for p in range(3)]
    lam = rng.standard_normal(5)
    X = rc.cp_dense(A, lam)
    assert abs(rc.cp_norm2(A, lam) - np.sum(X ** 2)) < 1e-11 * np.sum(X ** 2)
    for eps in (1e-1, 1e-3):
        res = rc.hooi(A, lam, eps)
        direct = np.linalg.norm(X - rc.tucker_dense(res["core"], res["U"])) / np.linalg.norm(X)
        assert abs(res["rel_err"] - direct) < 1e-10 * max(direct, 1e-3)
        # the error is the norm not kept by the core (orthonormal factors)
        kept = np.sqrt(max(1 - np.sum(res["core"] ** 2) / np.sum(X ** 2), 0))
        assert abs(kept - direct) < 1e-6


def test_recovers_a_known_tucker_tensor():
    core, U = _known_tucker()
    A, lam = rc.tucker_as_cp(core, U)
    res = rc.hooi(A, lam, 1e-10)
    assert res["ranks"] == (3, 4, 5)
    assert res["rel_err"] < 1e-12
    X = rc.tucker_dense(core, U)
    assert np.allclose(rc.tucker_dense(res["core"], res["U"]), X, atol=1e-12 * np.abs(X).max())
    for p in range(3):   # same subspaces
        P1 = res["U"][p] @ res["U"][p].T
        P0 = U[p] @ U[p].T
        assert np.abs(P1 - P0).max() < 1e-12


def test_rank_rule():
    sig = np.array([10.0, 1.0, 0.1, 0.01, 0.001])
    tot = np.sqrt(np.sum(sig ** 2))
    for eps in (0.5, 1e-2, 1e-3, 1e-4, 1e-6):
        r = rc.truncation_rank(sig, eps)
        assert np.sqrt(np.sum(sig[r:] ** 2)) <= eps / np.sqrt(3) * tot
        assert r == 1 or np.sqrt(np.sum(sig[r - 1:] ** 2)) > eps / np.sqrt(3) * tot
    assert rc.truncation_rank(sig, 1e-12) == 5


@pytest.mark.parametrize("eps", [1e-1, 1e-2, 1e-3])
def test_tolerance_is_met_and_hooi_improves_on_hosvd(eps):
    """HOSVD with per-mode tails eps/sqrt(3) has error <= eps; HOOI's fit
    never decreases from there."""
    rng = np.random.default_rng(3)
    n = (14, 12, 10)
    # a smooth-ish CP tensor (decaying spectrum): Gaussian bumps of varying width
    x = [np.linspace(-1, 1, n[p]) for p in range(3)]
    T = 12
    A = [np.stack([np.exp(-(x[p] - rng.uniform(-1, 1)) ** 2 / rng.uniform(0.05, 1.0)) for _ in range(T)])
         for p in range(3)]
    lam = rng.standard_normal(T)
    X = rc.cp_dense(A, lam)
    Uh = rc.hosvd(A, lam, eps)
    Xh = rc.tucker_dense(rc.tucker_core(A, lam, Uh), Uh)
    e_hosvd = np.linalg.norm(X - Xh) / np.linalg.norm(X)
    assert e_hosvd <= eps
    res = rc.hooi(A, lam, eps)
    assert res["rel_err"] <= eps
    assert all(b >= a * (1 - 1e-12) for a, b in zip(res["fits"], res["fits"][1:]))


def test_rmax_caps_the_ranks():
    rng = np.random.default_rng(4)
    n = (10, 9, 8)
    A = [rng.standard_normal((20, n[p])) for p in range(3)]
    lam = np.ones(20)
    res = rc.hooi(A, lam, 1e-12, rmax=3)
    assert res["ranks"] == (3, 3, 3)
    assert 0 < res["rel_err"] < 1
