"""Pins of the oracle's Alg. scpot_fft_tucker route (CPU): Tucker Hadamard
products, the structured DFT, HOOI with a tolerance, the approximate
summation, the whole route against the dense Kronecker apply, and TT
rounding.  Each check compares with something other than the function's own
formula: brute-force dense tensors, numpy's 3D FFT, exact low-rank
constructions, the HOSVD error bound, or the independent dense-Toeplitz apply."""
import numpy as np
import pytest

from oracle import apply, sinc
from oracle import tucker as tk


def _orth(rng, n, r):
    q, _ = np.linalg.qr(rng.standard_normal((n, r)))
    return q


def _rand_tucker(rng, n, r):
    return rng.standard_normal(r), [rng.standard_normal((n[p], r[p])) for p in range(3)]


def test_dense_helpers_against_einsum():
    rng = np.random.default_rng(0)
    core, U = _rand_tucker(rng, (5, 4, 3), (2, 3, 2))
    X = np.einsum("abc,ia,jb,kc->ijk", core, U[0], U[1], U[2])
    assert np.allclose(tk.tucker_dense(core, U), X, rtol=1e-14, atol=1e-14)
    for p in range(3):
        dense = np.transpose(X, [p] + [s for s in range(3) if s != p]).reshape(X.shape[p], -1)
        assert np.array_equal(tk.unfold(X, p), dense)


def test_hadamard_product_equals_elementwise_product():
    """Eq. (t_had2) against the elementwise product of the dense tensors
    (unequal ranks on every mode, so a swapped index order fails)."""
    rng = np.random.default_rng(1)
    n = (6, 5, 4)
    X = _rand_tucker(rng, n, (2, 3, 4))
    Y = _rand_tucker(rng, n, (3, 1, 2))
    E, W = tk.tucker_hadamard(X, Y)
    assert E.shape == (6, 3, 8) and [w.shape[1] for w in W] == [6, 3, 8]
    ref = tk.tucker_dense(*X) * tk.tucker_dense(*Y)
    assert np.allclose(tk.tucker_dense(E, W), ref, rtol=1e-13, atol=1e-13)


def test_dft_tucker_equals_3d_fft():
    """Lemma DFT_tucker: the structured DFT equals numpy's 3D FFT of the
    zero-padded dense tensor."""
    rng = np.random.default_rng(2)
    n = (5, 4, 3)
    L = (9, 7, 5)
    core, U = _rand_tucker(rng, n, (2, 2, 3))
    c, F = tk.dft_tucker(core, U, L)
    ref = np.fft.fftn(tk.tucker_dense(core, U), s=L, axes=(0, 1, 2))
    assert np.allclose(tk.tucker_dense(c, F), ref, rtol=1e-12, atol=1e-12)


def test_kernel_cp_matches_kernel_entries():
    n, h = (6, 5, 4), (0.2, 0.2, 0.2)
    _t, tau, alpha = sinc.sinc_nodes(12)
    F = [sinc.scaled_factors(n[d], h[d], tau, alpha) for d in range(3)]
    for q in range(3):
        P = tk.cp_dense(*tk.kernel_cp(n, h, tau, alpha, q))
        for J in [(0, 0, 0), (3, -2, 1), (-5, 4, -3)]:
            ty = sinc.phi_types(q)
            ref = sinc.kernel_from_factors(F[0][ty[0]], F[1][ty[1]], F[2][ty[2]], J)
            assert P[J[0] + n[0] - 1, J[1] + n[1] - 1, J[2] + n[2] - 1] == pytest.approx(ref, rel=1e-13, abs=1e-16)


def test_hooi_recovers_exact_multilinear_rank():
    rng = np.random.default_rng(3)
    n, r = (14, 12, 10), (3, 4, 2)
    core = rng.standard_normal(r)
    U = [_orth(rng, n[p], r[p]) for p in range(3)]
    X = tk.tucker_dense(core, U)
    c, V, _sw = tk.hooi(X, 1e-10)
    assert c.shape == r
    assert np.linalg.norm(tk.tucker_dense(c, V) - X) < 1e-13 * np.linalg.norm(X)
    for p in range(3):
        assert np.allclose(V[p].T @ V[p], np.eye(r[p]), atol=1e-13)


@pytest.mark.parametrize("eps", [1e-2, 1e-4, 1e-6])
def test_hooi_error_within_tolerance(eps):
    """Decaying multilinear spectra: the relative error stays within eps
    (HOSVD bound) and the ranks drop."""
    rng = np.random.default_rng(4)
    n = (16, 14, 12)
    core = rng.standard_normal(n) * np.einsum("i,j,k->ijk", *[0.3 ** np.arange(m) for m in n])
    X = tk.tucker_dense(core, [_orth(rng, n[p], n[p]) for p in range(3)])
    c, V, sweeps = tk.hooi(X, eps)
    err = np.linalg.norm(tk.tucker_dense(c, V) - X) / np.linalg.norm(X)
    assert err <= eps
    assert max(c.shape) < max(n)                   # it did compress


def test_tucker_sum_of_copies_keeps_ranks():
    rng = np.random.default_rng(5)
    n, r = (12, 11, 10), (3, 2, 4)
    core = rng.standard_normal(r)
    U = [rng.standard_normal((n[p], r[p])) for p in range(3)]
    c, V = tk.tucker_sum([(core, U), (core, U), (-0.5 * core, U)], 1e-12)
    assert c.shape == r
    X = tk.tucker_dense(core, U)
    assert np.linalg.norm(tk.tucker_dense(c, V) - 1.5 * X) < 1e-13 * np.linalg.norm(X)


def test_tucker_sum_error_within_tolerance():
    rng = np.random.default_rng(6)
    n = (14, 13, 12)
    terms = []
    for s in range(3):
        r = (4 + s, 3 + s, 5)
        core = rng.standard_normal(r) * np.einsum("i,j,k->ijk", *[0.2 ** np.arange(m) for m in r])
        terms.append((core, [rng.standard_normal((n[p], r[p])) for p in range(3)]))
    X = sum(tk.tucker_dense(*t) for t in terms)
    for eps in (1e-3, 1e-6, 1e-9):
        c, V = tk.tucker_sum(terms, eps)
        assert np.linalg.norm(tk.tucker_dense(c, V) - X) <= eps * np.linalg.norm(X)


def _mag(kind, n, seed=7):
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return [(np.array([[[v]]]), [np.ones((n[p], 1)) for p in range(3)]) for v in (0.3, -0.5, 0.8)]
    return [_rand_tucker(rng, n, (2, 3, 2)) for _q in range(3)]


@pytest.mark.parametrize("kind", ["uniform", "random"])
def test_route_without_truncation_equals_kronecker_apply(kind):
    """With a vanishing tolerance the route is exact: it equals the dense
    Toeplitz Kronecker apply of Cor. kron_op (pins the convolution window, the
    Hadamard index order and the kernel factors)."""
    n = (9, 7, 6)
    h = tuple(1.0 / max(n) for _ in range(3))
    _t, tau, alpha = sinc.sinc_nodes(20)
    mag = _mag(kind, n)
    m = np.stack([tk.tucker_dense(*mag[q]).transpose(2, 1, 0) for q in range(3)])
    ref, _h = apply.kron_apply_dense(m, h, tau, alpha)
    ref = ref.transpose(2, 1, 0)
    kernels = tk.kernel_tucker(n, h, tau, alpha, 1e-300)
    exact = sum(tk.tucker_dense(*p) for p in tk.hadamard_products(kernels, mag, n))
    assert np.linalg.norm(exact - ref) < 1e-13 * np.linalg.norm(ref)
    c, U = tk.potential_tucker(mag, n, h, tau, alpha, 1e-300)
    assert np.linalg.norm(tk.tucker_dense(c, U) - ref) < 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("tol", [1e-4, 1e-8])
def test_route_with_tolerance(tol):
    """Kernel compression and summation each stay within tol; the potential
    is within a small multiple of tol of the exact apply, with ranks below
    the grid sizes."""
    n = (20, 18, 16)
    h = tuple(1.0 / max(n) for _ in range(3))
    _t, tau, alpha = sinc.sinc_nodes(30)
    for q in range(3):
        P = tk.cp_dense(*tk.kernel_cp(n, h, tau, alpha, q))
        c, U, _sw = tk.hooi(P, tol)
        assert np.linalg.norm(tk.tucker_dense(c, U) - P) <= tol * np.linalg.norm(P)
    mag = _mag("uniform", n)
    m = np.stack([tk.tucker_dense(*mag[q]).transpose(2, 1, 0) for q in range(3)])
    ref = apply.kron_apply_dense(m, h, tau, alpha)[0].transpose(2, 1, 0)
    c, U = tk.potential_tucker(mag, n, h, tau, alpha, tol)
    err = np.linalg.norm(tk.tucker_dense(c, U) - ref) / np.linalg.norm(ref)
    assert err < 30 * tol and all(c.shape[p] < n[p] for p in range(3))


def test_potential_at_cells_matches_dense_apply():
    """Row-by-row evaluation against the dense Kronecker apply."""
    n = (7, 6, 5)
    h = tuple(1.0 / max(n) for _ in range(3))
    _t, tau, alpha = sinc.sinc_nodes(16)
    mag = _mag("random", n, seed=12)
    m = np.stack([tk.tucker_dense(*mag[q]).transpose(2, 1, 0) for q in range(3)])
    ref = apply.kron_apply_dense(m, h, tau, alpha)[0].transpose(2, 1, 0)
    cells = [(0, 0, 0), (6, 5, 4), (3, 1, 2), (5, 4, 0)]
    got = tk.potential_at_cells(mag, n, h, tau, alpha, cells)
    assert np.allclose(got, [ref[c] for c in cells], rtol=1e-12, atol=1e-14 * np.abs(ref).max())


def _rand_tt(rng, n, r):
    return (rng.standard_normal((n[0], r[0])), rng.standard_normal((r[0], n[1], r[1])),
            rng.standard_normal((r[1], n[2])))


def test_tt_round_removes_redundant_ranks():
    """The TT of A + A (cores side by side, block-diagonal middle core)
    rounds back to the ranks of A, equal to 2A."""
    rng = np.random.default_rng(8)
    n, r = (10, 9, 8), (3, 2)
    G1, G2, G3 = _rand_tt(rng, n, r)
    D1 = np.concatenate([G1, G1], axis=1)
    D2 = np.zeros((6, n[1], 4))
    D2[:3, :, :2] = G2
    D2[3:, :, 2:] = G2
    D3 = np.concatenate([G3, G3], axis=0)
    A = tk.tt_dense(G1, G2, G3)
    assert np.allclose(tk.tt_dense(D1, D2, D3), 2 * A)
    H1, H2, H3 = tk.tt_round(D1, D2, D3, 1e-12)
    assert H1.shape[1] == 3 and H3.shape[0] == 2
    assert np.linalg.norm(tk.tt_dense(H1, H2, H3) - 2 * A) < 1e-13 * np.linalg.norm(A)


def test_tt_round_ranks_are_unfolding_ranks():
    """An exact low-rank TT with redundant outer ranks: the rounded ranks are
    the ranks of the unfoldings A_(1) and A_(12) (brute force)."""
    rng = np.random.default_rng(9)
    n = (12, 10, 11)
    G1, G2, G3 = _rand_tt(rng, n, (4, 3))
    G1 = np.concatenate([G1, G1[:, :2] @ rng.standard_normal((2, 3))], axis=1)   # rank 4, stored as 7
    G2 = np.concatenate([G2, np.zeros((3, n[1], 3))], axis=0)
    A = tk.tt_dense(G1, G2, G3)
    ranks = (np.linalg.matrix_rank(A.reshape(n[0], -1)), np.linalg.matrix_rank(A.reshape(n[0] * n[1], -1)))
    H1, H2, H3 = tk.tt_round(G1, G2, G3, 1e-12)
    assert (H1.shape[1], H3.shape[0]) == ranks == (4, 3)
    assert np.linalg.norm(tk.tt_dense(H1, H2, H3) - A) < 1e-13 * np.linalg.norm(A)


@pytest.mark.parametrize("eps", [1e-2, 1e-5])
def test_tt_round_error_within_tolerance(eps):
    rng = np.random.default_rng(10)
    n = (12, 11, 10)
    G1, G2, G3 = _rand_tt(rng, n, (8, 8))
    G1 = G1 * 0.1 ** np.arange(8)[None, :]
    G3 = G3 * 0.15 ** np.arange(8)[:, None]
    A = tk.tt_dense(G1, G2, G3)
    H1, H2, H3 = tk.tt_round(G1, G2, G3, eps)
    assert np.linalg.norm(tk.tt_dense(H1, H2, H3) - A) <= eps * np.linalg.norm(A)
    assert H1.shape[1] < 8 or H3.shape[0] < 8


def test_tt_from_tucker():
    rng = np.random.default_rng(11)
    core, U = _rand_tucker(rng, (6, 5, 4), (2, 3, 2))
    assert np.allclose(tk.tt_dense(*tk.tt_from_tucker(core, U)), tk.tucker_dense(core, U), rtol=1e-13, atol=1e-13)


def test_tt_from_cp_and_tucker_from_tt():
    rng = np.random.default_rng(21)
    n = (7, 6, 5)
    lam = rng.standard_normal(4)
    U = [rng.standard_normal((n[p], 4)) for p in range(3)]
    X = np.einsum("r,ir,jr,kr->ijk", lam, U[0], U[1], U[2])
    T = tk.tt_from_cp(lam, U)
    assert np.allclose(tk.tt_dense(*T), X, rtol=1e-13, atol=1e-13)
    core, V = tk.tucker_from_tt(*T, 1e-12)
    assert max(core.shape) <= 4
    assert np.linalg.norm(tk.tucker_dense(core, V) - X) < 1e-12 * np.linalg.norm(X)
