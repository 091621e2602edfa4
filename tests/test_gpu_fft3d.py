"""GPU parity of the full-format apply by 3D FFT convolution.

The FFT route computes the same separable operator as the mode products, so
it must agree with the oracle's FFT route and its Kronecker route to FP64
rounding (1e-12 relative L2), on ragged grids (several lines per workgroup,
partial fx tiles, axes of length 1) and at 128^3 against the GPU's own
mode-product apply."""
import numpy as np
import pytest
import torch

from oracle import apply, exact, fftconv, sinc
from paper_1212_3509_amd import api, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    api.library()
    return api.Context(0)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=torch.float64)


@pytest.mark.parametrize("n,h,M", [((9, 7, 6), (0.11, 0.13, 0.09), 10),
                                   ((20, 33, 17), (1 / 33,) * 3, 16),
                                   ((5, 1, 12), (0.2, 0.2, 0.2), 8)])
def test_fft_apply_matches_oracle(ctx, n, h, M):
    m = inputs.random_unit_field(n, seed=5)
    f = ctx.assemble(n, h, M=M)
    _t, tau, alpha = f.nodes()
    # the library works in the domain scaled to a unit longest edge and
    # scales the potential back by the length L
    L = max(n[d] * h[d] for d in range(3))
    hs = [x / L for x in h]
    phi, hf = ctx.apply_fft(f, _dev(m))
    torch.cuda.synchronize()
    p_or, h_or = fftconv.fft_apply(m, hs, tau, alpha)
    p_kr, h_kr = apply.kron_apply_dense(m, hs, tau, alpha)
    phi, hf = phi.cpu().numpy(), hf.cpu().numpy()
    for a, b in ((phi, L * p_or), (hf, h_or), (phi, L * p_kr), (hf, h_kr)):
        assert apply.rel_l2(a, b) < 1e-12, apply.rel_l2(a, b)


@pytest.mark.parametrize("n", [(32, 32, 32), (45, 38, 71)])
def test_fft_apply_equals_mode_products(ctx, n):
    m = _dev(inputs.random_unit_field(n, seed=6))
    f = ctx.assemble(n, (1.0 / max(n),) * 3, M=40)
    p1, h1 = ctx.apply_fft(f, m)
    p2, h2 = ctx.apply_full(f, m, prec="fp64")
    torch.cuda.synchronize()
    rel = lambda a, b: float(torch.linalg.norm((a - b).reshape(-1)) / torch.linalg.norm(b.reshape(-1)))  # noqa: E731
    assert rel(p1, p2) < 1e-12 and rel(h1, h2) < 1e-12, (rel(p1, p2), rel(h1, h2))


@pytest.mark.parametrize("n", [(6, 600, 3), (5, 3, 700), (1100 // 2, 2, 3)])
def test_fft_apply_long_axes(ctx, n):
    """Lines of 2048 points along y or z (multi-wave workgroups, four-line
    column groups of the fused z pass) and real rows of 2048 points along x."""
    m = _dev(inputs.random_unit_field(n, seed=8))
    f = ctx.assemble(n, (1.0 / max(n),) * 3, M=12)
    p1, h1 = ctx.apply_fft(f, m)
    p2, h2 = ctx.apply_full(f, m, prec="fp64")
    torch.cuda.synchronize()
    rel = lambda a, b: float(torch.linalg.norm((a - b).reshape(-1)) / torch.linalg.norm(b.reshape(-1)))  # noqa: E731
    assert rel(p1, p2) < 1e-12 and rel(h1, h2) < 1e-12, (rel(p1, p2), rel(h1, h2))


def test_fft_apply_128_vortex(ctx):
    n = 128
    m = _dev(inputs.vortex_field(n, seed=0))
    f = ctx.assemble((n, n, n), (1.0 / n,) * 3, M=40)
    p1, h1 = ctx.apply_fft(f, m)
    p2, h2 = ctx.apply_full(f, m, prec="fp64")
    torch.cuda.synchronize()
    rel = lambda a, b: float(torch.linalg.norm((a - b).reshape(-1)) / torch.linalg.norm(b.reshape(-1)))  # noqa: E731
    print(f"128^3: FFT route vs mode products: phi {rel(p1, p2):.2e}, h {rel(h1, h2):.2e}")
    assert rel(p1, p2) < 1e-12 and rel(h1, h2) < 1e-12


def test_fft_apply_rejects_large_axes(ctx):
    f = ctx.assemble((2048, 4, 4), (1.0 / 2048,) * 3, M=4)
    m = torch.zeros((3, 4, 4, 2048), dtype=torch.float64, device="cuda")
    with pytest.raises(api.DemagError):
        ctx.apply_fft(f, m)


def test_fft_route_128_uniform_matches_exact_collocation(ctx):
    """The 3D-FFT route at 128^3 (M = 40) for a uniform magnetization: every
    cell against the exact collocated potential and field of the cube
    (closed-form box kernels of the whole cube at the cell centres)."""
    n = 128
    f = ctx.assemble((n, n, n), (1 / n,) * 3, M=40)
    mv = np.array([0.3, -0.5, 0.8])
    m = torch.from_numpy(mv[:, None, None, None] * np.ones((3, n, n, n))).cuda()
    phi, hf = ctx.apply_fft(f, m)
    torch.cuda.synchronize()
    c = (np.arange(n) + 0.5) / n
    pts = np.stack(np.meshgrid(c, c, c, indexing="ij")[::-1], axis=-1)
    K, N = exact.box_kernels_at_points(pts, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    e_phi = apply.rel_l2(phi.cpu().numpy(), np.tensordot(mv, K, axes=1))
    e_h = apply.rel_l2(hf.cpu().numpy(), -np.tensordot(N, mv, axes=([1], [0])))
    print(f"3D-FFT route uniform 128^3 vs exact collocation: phi {e_phi:.2e}, h {e_h:.2e}")
    assert e_phi < 1e-8 and e_h < 1e-8
