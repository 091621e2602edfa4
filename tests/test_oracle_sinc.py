"""Pins of the sinc rule and the 1D factors (oracle.sinc) and of the
Kronecker-form apply (oracle.apply.kron_apply_dense)."""
import mpmath as mp
import numpy as np
import pytest

from oracle import apply, exact, sinc, smooth
from paper_1212_3509_amd import inputs


def _pieces(a, b):
    pts = list(mp.linspace(a, b, 17))
    return sorted(set(pts + ([mp.mpf(0)] if a < 0 < b else [])))


def _mp_E(tau, J, h):
    """int_a^b exp(-tau^2 x^2) dx by quadrature; the integrand is scaled by
    its largest value on [a, b] (mpmath's tolerance is absolute)."""
    a, b = (J - 0.5) * h, (J + 0.5) * h
    c = 0 if a < 0 < b else min(abs(a), abs(b))
    s = mp.exp(-(tau * c) ** 2)
    return s * mp.quad(lambda x: mp.exp(-(tau * tau) * (x * x - c * c)), _pieces(a, b))


def _mp_X(tau, J, h):
    a, b = (J - 0.5) * h, (J + 0.5) * h
    c = 0 if a < 0 < b else min(abs(a), abs(b))
    s = mp.exp(-(tau * c) ** 2)
    return s * mp.quad(lambda x: x * mp.exp(-(tau * tau) * (x * x - c * c)), _pieces(a, b))


def _mp_closed(tau, J, h):
    """E, X, X' from the antiderivatives in multiple precision (erfc for
    intervals right of 0, mirror symmetry for those left of 0)."""
    tau = mp.mpf(tau)
    Jm, sgn = abs(J), (1 if J >= 0 else -1)
    a, b = (Jm - mp.mpf(1) / 2) * h, (Jm + mp.mpf(1) / 2) * h
    if Jm == 0:
        E = mp.sqrt(mp.pi) / tau * mp.erf(tau * b)
    else:
        E = mp.sqrt(mp.pi) / (2 * tau) * (mp.erfc(tau * a) - mp.erfc(tau * b))
    X = (mp.exp(-(tau * a) ** 2) - mp.exp(-(tau * b) ** 2)) / (2 * tau * tau)
    Xp = b * mp.exp(-(tau * b) ** 2) - a * mp.exp(-(tau * a) ** 2)
    return E, sgn * X, Xp


@pytest.mark.parametrize("tau", [0.2, 3.0, 57.0, 1391.0])
@pytest.mark.parametrize("h", [1 / 32, 1 / 128])
def test_factors_match_defining_integrals(tau, h):
    """E and X (Eq. (sep_integrands) after the shift of Sec. 4.2) against
    multiple-precision quadrature of their defining integrals wherever that
    quadrature resolves the Gaussian, X' and E' = -2 tau^2 X against numerical
    differentiation of those integrals in the target position, and all of them
    against the antiderivatives in 50-digit arithmetic at every argument."""
    mp.mp.dps = 50
    n = 40
    E = sinc.factor_E(tau, n, h)
    X = sinc.factor_X(tau, n, h)
    Xp = sinc.factor_Xp(tau, n, h)
    for J in (0, 1, 2, 5, -3, n - 1):
        i = J + n - 1
        e_c, x_c, xp_c = (float(v) for v in _mp_closed(tau, J, h))
        assert abs(E[i] - e_c) <= 1e-13 * abs(e_c) + 1e-300
        assert abs(X[i] - x_c) <= 1e-12 * abs(x_c) + 1e-300
        assert abs(Xp[i] - xp_c) <= 1e-12 * abs(xp_c) + 1e-300
        if tau * tau * 2 * abs(J) * h * h <= 30:
            e_q, x_q = float(_mp_E(tau, J, h)), float(_mp_X(tau, J, h))
            assert abs(e_q - e_c) <= 1e-14 * abs(e_c)
            assert abs(x_q - x_c) <= 1e-14 * abs(x_c) + 1e-40
        if tau * tau * 2 * abs(J) * h * h <= 30 and J in (0, 1, -3):
            s = J * h
            xp_d = float(mp.diff(lambda s_: mp.quad(lambda x: x * mp.exp(-(tau * x) ** 2),
                                                     _pieces(s_ - h / 2, s_ + h / 2)), s))
            ep_d = float(mp.diff(lambda s_: mp.quad(lambda x: mp.exp(-(tau * x) ** 2),
                                                     _pieces(s_ - h / 2, s_ + h / 2)), s))
            assert abs(xp_d - xp_c) <= 1e-10 * abs(xp_c) + 1e-20 * h
            assert abs(-2 * tau * tau * x_c - ep_d) <= 1e-10 * abs(ep_d) + 1e-20 * h


def test_factor_symmetries():
    n, h, tau = 17, 1 / 16, 4.0
    E, X, Xp = sinc.factor_E(tau, n, h), sinc.factor_X(tau, n, h), sinc.factor_Xp(tau, n, h)
    assert np.array_equal(E, E[::-1]) and np.array_equal(Xp, Xp[::-1])
    assert np.array_equal(X, -X[::-1]) and X[n - 1] == 0.0


def test_nodes_paper_rule():
    """Cor. kron_op with c0 = 2.15 (Sec. 3.5): theta = c0 ln M / M."""
    t, tau, alpha = sinc.sinc_nodes(40)
    theta = 2.15 * np.log(40) / 40
    assert abs(t[0] - theta) < 1e-16 and abs(t[-1] - 40 * theta) < 1e-14
    assert np.allclose(tau, np.sinh(t), rtol=1e-15)
    assert np.allclose(alpha, 2 * theta * np.cosh(t) * np.sinh(t) ** 2, rtol=1e-15)


def _gauss_transform_rel_err(M, rho, c0=2.15):
    """Sinc rule for rho^(-3/2) = (2/sqrt(pi)) int_R tau^2 exp(-tau^2 rho) dtau
    (Eq. (gauss_trans)), tau = sinh t, folded to k = 1..M."""
    _t, tau, alpha = sinc.sinc_nodes(M, c0)
    approx = (2 / np.sqrt(np.pi)) * np.sum(alpha[:, None] * np.exp(-np.outer(tau * tau, rho)), axis=0)
    return np.abs(approx * rho ** 1.5 - 1.0)


def test_gauss_transform_uniform_error_and_exponential_rate():
    """Sec. 3.5 / Fig. fig1: on rho in [3h^2/4, 3] the relative error is
    uniformly small for h above some h_min, and log(error) decreases affinely
    in the rank (Thm. sinc_theo)."""
    rho = np.geomspace(3 * (1 / 64) ** 2 / 4, 3.0, 2000)
    assert _gauss_transform_rel_err(40, rho).max() < 1e-8
    Ms = np.arange(15, 41, 5)
    errs = np.array([_gauss_transform_rel_err(M, rho).max() for M in Ms])
    assert np.all(np.diff(np.log(errs)) < 0)
    slope, intercept = np.polyfit(Ms, np.log10(errs), 1)
    resid = np.log10(errs) - (slope * Ms + intercept)
    assert slope < -0.15 and np.abs(resid).max() < 0.4


def _kernel_errors(n, M, step_rule=0):
    h = 1.0 / n
    _t, tau, alpha = sinc.sinc_nodes(M, step_rule=step_rule, h_min=h)
    F = sinc.scaled_factors(n, h, tau, alpha)
    errs = []
    for J in [(0, 0, 0), (1, 0, 0), (1, 1, 0), (1, 1, 1), (3, 2, 1), (n - 1, 2, 0)]:
        lo = tuple(np.array((J[d] - 0.5) * h) for d in range(3))
        hi = tuple(np.array((J[d] + 0.5) * h) for d in range(3))
        A = np.array([[-sinc.kernel_from_factors(*[F[t] for t in sinc.field_types(p, q)], J)
                       for q in range(3)] for p in range(3)])
        Ne = np.array([[float(exact.demag_tensor_box(lo, hi, p, q)) for q in range(3)] for p in range(3)])
        errs.append(np.linalg.norm(A - Ne) / np.linalg.norm(Ne))
        a = np.array([sinc.kernel_from_factors(*[F[t] for t in sinc.phi_types(q)], J) for q in range(3)])
        b = np.array([float(exact.potential_kernel_box(lo, hi, q)) for q in range(3)])
        if np.linalg.norm(b) > 1e-12:
            errs.append(np.linalg.norm(a - b) / np.linalg.norm(b))
        else:
            assert np.abs(a).max() < 1e-15
    return max(errs)


def test_cell_kernels_converge_exponentially_in_rank():
    """T-R (ii): the cell-integrated kernels (self cell, faces, edges, corner,
    far) from the separable factors approach the exact collocation kernels
    geometrically in M (Lemma sinc_mumag, Cor. kron_op)."""
    Ms = [10, 20, 30, 40]
    errs = [_kernel_errors(32, M) for M in Ms]
    assert all(e2 < e1 / 10 for e1, e2 in zip(errs, errs[1:]))
    assert errs[-1] < 1e-7


def test_theorem_step_rule_accurate():
    assert _kernel_errors(32, 40, step_rule=1) < 1e-7


def test_rule_not_uniform_in_h():
    """Remark after Lemma sinc_mumag: a fixed rule loses accuracy as h -> 0."""
    assert _kernel_errors(2048, 40) > 100 * _kernel_errors(32, 40)


def test_vec_kronecker_ordering():
    """T-VEC: the [z][y][x] mode products equal (T_z (x) T_y (x) T_x) vec(m)
    with x fastest (footnote of Cor. kron_op)."""
    rng = np.random.default_rng(5)
    u = rng.standard_normal((2, 4, 3))
    Tx, Ty, Tz = (sinc.toeplitz(rng.standard_normal(2 * k - 1)) for k in (3, 4, 2))
    got = apply._triple_mode_product(u, Tx, Ty, Tz).ravel()
    ref = np.kron(Tz, np.kron(Ty, Tx)) @ u.ravel()
    assert np.allclose(got, ref, rtol=1e-14, atol=1e-14)


def test_toeplitz_generator_indexing():
    g = np.arange(7.0)          # J = -3..3
    T = sinc.toeplitz(g)
    assert T[0, 0] == 3 and T[3, 0] == 6 and T[0, 3] == 0 and T[2, 1] == 4


@pytest.mark.parametrize("n", [16, 24])
def test_kronecker_apply_matches_exact_collocation(n):
    """The separable operator (M = 40, c0 = 2.15) reproduces the exact
    collocation of Eq. (coll) for potential and field on a unit cube."""
    h = (1 / n,) * 3
    m = inputs.random_unit_field(n, seed=0)
    _t, tau, alpha = sinc.sinc_nodes(40)
    pk, hk = apply.kron_apply_dense(m, h, tau, alpha)
    pe, he = apply.collocated_apply_fft(m, h)
    assert apply.rel_l2(pk, pe) < 1e-8
    assert apply.rel_l2(hk, he) < 1e-8


def test_kronecker_sampled_cells_match_full():
    n = (10, 9, 8)
    h = (0.1, 0.1, 0.1)
    m = inputs.random_unit_field(n, seed=3)
    _t, tau, alpha = sinc.sinc_nodes(12)
    pk, hk = apply.kron_apply_dense(m, h, tau, alpha)
    cells = [(0, 0, 0), (7, 8, 9), (3, 4, 5)]
    pa, ha = apply.kron_apply_at_cells(m, h, tau, alpha, cells)
    assert np.allclose(pa, [pk[c] for c in cells], rtol=1e-13, atol=1e-16)
    assert np.allclose(ha, [hk[(slice(None),) + c] for c in cells], rtol=1e-13, atol=1e-16)


def test_uniform_cube_kronecker():
    """T-CUBE for the separable operator on an odd grid: centre N_zz = 1/3."""
    n = 33
    m = inputs.uniform_field(n, axis=2)
    _t, tau, alpha = sinc.sinc_nodes(40)
    pk, hk = apply.kron_apply_dense(m, (1 / n,) * 3, tau, alpha)
    assert abs(hk[2, 16, 16, 16] + 1 / 3) < 1e-9
    assert abs(pk[16, 16, 16]) < 1e-15


def test_collocation_converges_quadratically():
    """Lemma conv_coll / Fig. fig_err: the collocated potential of
    m = exp(-|x|^2)(1,1,1) on [0,1]^3 at xi = (h/2)(1,1,1) converges as O(h^2)."""
    g = lambda x, y, z: np.exp(-(x * x + y * y + z * z))  # noqa: E731
    errs = []
    for n in (16, 32, 64):
        h = 1.0 / n
        ref = smooth.potential_smooth_at(g, (h / 2,) * 3)
        col = smooth.collocated_phi_at_cell(inputs.gaussian_bump_field(n), (h, h, h), (0, 0, 0))
        errs.append(abs(col - ref))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert 1.85 < rates[-1] < 2.15
    assert errs[-1] < 1e-5


def test_smooth_reference_quadrature_converged():
    g = lambda x, y, z: np.exp(-(x * x + y * y + z * z))  # noqa: E731
    xi = (1 / 64,) * 3
    a = smooth.potential_smooth_at(g, xi, npts=48)
    b = smooth.potential_smooth_at(g, xi, npts=64)
    assert abs(a - b) < 1e-10


def test_fft_route_equals_kronecker_route():
    """The separable kernel applied by 3D FFT convolution equals the triple
    mode products with dense Toeplitz factors (two independent routes)."""
    from oracle import fftconv
    n = (9, 7, 6)
    h = (0.11, 0.13, 0.09)
    m = inputs.random_unit_field(n, seed=3)
    _t, tau, alpha = sinc.sinc_nodes(10)
    p1, h1 = fftconv.fft_apply(m, h, tau, alpha)
    p2, h2 = apply.kron_apply_dense(m, h, tau, alpha)
    assert apply.rel_l2(p1, p2) < 1e-13 and apply.rel_l2(h1, h2) < 1e-13
