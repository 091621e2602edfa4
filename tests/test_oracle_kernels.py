"""Pins of the exact cell kernels (oracle.exact) and the collocated apply
(oracle.apply) to facts fixed by the mathematics, not by the oracle itself."""
import numpy as np
import pytest

from oracle import apply, exact
from paper_1212_3509_amd import inputs


def _box(J, h):
    lo = tuple(np.array((J[d] - 0.5) * h[d]) for d in range(3))
    hi = tuple(np.array((J[d] + 0.5) * h[d]) for d in range(3))
    return lo, hi


def _K(J, h):
    lo, hi = _box(J, h)
    return np.array([float(exact.potential_kernel_box(lo, hi, q)) for q in range(3)])


def _N(J, h):
    lo, hi = _box(J, h)
    return np.array([[float(exact.demag_tensor_box(lo, hi, p, q)) for q in range(3)] for p in range(3)])


def test_self_cell_cube():
    """T-SELF: a cube's centre has N = I/3 (cubic symmetry + trace 1) and the
    potential kernel vanishes (odd integrand)."""
    h = (0.1, 0.1, 0.1)
    assert np.allclose(_N((0, 0, 0), h), np.eye(3) / 3, atol=1e-15, rtol=0)
    assert np.allclose(_K((0, 0, 0), h), 0.0, atol=1e-17)


def test_self_cell_prism_trace_and_order():
    """Non-cubic self cell: trace 1 (Laplace of the Newton potential is -4 pi
    inside), off-diagonals 0 by mirror symmetry, and the shortest edge gets the
    largest factor."""
    h = (0.1, 0.2, 0.4)
    N = _N((0, 0, 0), h)
    assert abs(np.trace(N) - 1.0) < 1e-14
    assert np.allclose(N - np.diag(np.diag(N)), 0.0, atol=1e-15)
    assert N[0, 0] > N[1, 1] > N[2, 2] > 0


def test_trace_vanishes_off_cell():
    """T-TRACE: outside the source box the Newton potential is harmonic, so
    trace N(J) = 0 for every offset J != 0 (non-cubic cells)."""
    n = (5, 4, 3)
    h = (0.3, 0.2, 0.25)
    _K_all, N = exact.offset_kernels(n, h)
    tr = N[0, 0] + N[1, 1] + N[2, 2]
    centre = (n[2] - 1, n[1] - 1, n[0] - 1)
    assert abs(tr[centre] - 1.0) < 1e-14
    tr[centre] = 0.0
    assert np.abs(tr).max() < 1e-14


OFFSETS = [(1, 0, 0), (0, 1, 1), (2, 1, 3), (-3, 5, 7), (20, -11, 9)]


@pytest.mark.parametrize("J", OFFSETS)
def test_three_routes_agree(J):
    """Closed form (route 1) = face cubature (route 3) = Gaussian-transform tau
    integral in multiple precision (route 2): three independent derivations."""
    h = (1 / 32, 1 / 24, 1 / 40)
    K1, N1 = _K(J, h), _N(J, h)
    K3 = np.array([exact.face_cubature_potential(J, h, q) for q in range(3)])
    N3 = np.array([[exact.face_cubature_demag(J, h, p, q) for q in range(3)] for p in range(3)])
    K2 = np.array([exact.tau_integral_kernel(J, h, "phi", q=q, dps=20) for q in range(3)])
    N2 = np.array([[exact.tau_integral_kernel(J, h, "N", p=p, q=q, dps=20) for q in range(3)]
                   for p in range(3)])
    sK, sN = np.abs(K2).max(), np.abs(N2).max()
    assert np.abs(K1 - K2).max() < 1e-11 * sK
    assert np.abs(K3 - K2).max() < 1e-10 * sK
    assert np.abs(N1 - N2).max() < 1e-11 * sN
    assert np.abs(N3 - N2).max() < 1e-10 * sN


def test_self_cell_tau_integral():
    """Route 2 at the self cell reproduces 1/3: there the tau integral is
    2/sqrt(pi) int_0^inf exp(-u^2) erf(u)^2 du = 1/3 in closed form."""
    h = (0.05, 0.05, 0.05)
    assert abs(exact.tau_integral_kernel((0, 0, 0), h, "N", p=2, q=2) - 1 / 3) < 1e-14


def test_far_field_is_point_dipole():
    """T-DIPOLE: a cell far away acts like a point dipole of moment h^3 m:
    N_pq -> -V/(4 pi) (3 s_p s_q - delta_pq r^2)/r^5 with O((h/r)^2) error."""
    h = (1.0, 1.0, 1.0)
    for J in [(11, 0, 0), (7, 8, -9), (30, 20, 10)]:
        s = np.array(J, dtype=float)
        r = np.linalg.norm(s)
        dip = -(3 * np.outer(s, s) - np.eye(3) * r * r) / (4 * np.pi * r ** 5)
        N = _N(J, h)
        rel = np.abs(N - dip).max() / np.abs(dip).max()
        assert rel < 0.5 / r ** 2
        K = _K(J, h)
        kd = s / (4 * np.pi * r ** 3)
        assert np.abs(K - kd).max() / np.abs(kd).max() < 0.5 / r ** 2


def test_fft_convolution_equals_direct_sum():
    n = (3, 4, 5)
    h = (0.2, 0.25, 0.3)
    m = inputs.random_unit_field(n, seed=4)
    p1, h1 = apply.collocated_apply_fft(m, h)
    p2, h2 = apply.collocated_apply_direct(m, h)
    assert apply.rel_l2(p1, p2) < 1e-14 and apply.rel_l2(h1, h2) < 1e-14
    pc, hc = apply.collocated_at_cells(m, h, [(1, 2, 0), (4, 0, 2)])
    assert np.allclose(pc, [p2[1, 2, 0], p2[4, 0, 2]], atol=1e-15)
    assert np.allclose(hc, [h2[:, 1, 2, 0], h2[:, 4, 0, 2]], atol=1e-15)


def test_uniform_cube_equals_single_box():
    """T-CUBE: for uniform m the cell sum equals the kernel of the whole body
    (additivity of the integral); on an odd grid the centre sees N_zz = 1/3."""
    n = (7, 5, 9)
    h = (1 / 9, 1 / 9, 1 / 9)
    m = inputs.uniform_field(n, axis=2)
    phi, hf = apply.collocated_apply_fft(m, h)
    nx, ny, nz = n
    cz, cy, cx = np.meshgrid(*[(np.arange(k) + 0.5) * h[0] for k in (nz, ny, nx)], indexing="ij")
    pts = np.stack([cx, cy, cz], axis=-1)
    K, N = exact.box_kernels_at_points(pts, (0, 0, 0), (nx * h[0], ny * h[1], nz * h[2]))
    assert np.abs(phi - K[2]).max() < 1e-14
    assert np.abs(hf - (-N[:, 2])).max() < 1e-13
    cube = inputs.uniform_field(9, axis=2)
    _p, hc = apply.collocated_apply_fft(cube, (1 / 9,) * 3)
    assert abs(hc[2, 4, 4, 4] + 1 / 3) < 1e-14
    assert abs(_p[4, 4, 4]) < 1e-15
    assert abs(apply.demag_energy_density(cube, hc) - 1 / 6) < 1e-14


def test_staircase_sphere():
    """T-SPHERE: a uniformly magnetized ball has the uniform field h = -m/3
    inside.  The staircase ball keeps cubic symmetry about its centre, so
    there the value is exact; off the centre it converges as the grid is
    refined."""
    errs = []
    for n in (12, 24, 36):
        m = inputs.staircase_sphere_field(n, axis=2)
        _phi, hf = apply.collocated_apply_fft(m, (1 / n,) * 3)
        c, o = n // 2, n // 6
        assert abs(hf[2, c - 1:c + 1, c - 1:c + 1, c - 1:c + 1].mean() + 1 / 3) < 1e-13
        off = hf[:, c + o - 1:c + o + 1, c - 1:c + 1, c - 1:c + 1].mean(axis=(1, 2, 3))
        assert np.abs(off[:2]).max() < 1e-13
        errs.append(abs(off[2] + 1 / 3))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 7e-4


def test_potential_sign_physical():
    """phi > 0 above a body magnetized along +z, < 0 below (h = -grad phi
    points from the north face outward)."""
    n = 5
    m = inputs.uniform_field(n, axis=2)
    phi, _ = apply.collocated_apply_fft(m, (0.2,) * 3)
    assert phi[-1, 2, 2] > 0 > phi[0, 2, 2]
