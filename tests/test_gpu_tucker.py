"""GPU parity of the Alg. scpot_fft_tucker route (kernel compression,
Fourier-space Hadamard products, approximate summation) and of TT rounding,
against the oracle (oracle.tucker) on the same seeded inputs.

Tucker and TT representations are not unique (bases, signs), so the checks
compare what is: the ranks, and the dense tensors the representations stand
for.  Both sides run the same algorithm in FP64 (HOOI from the truncated
HOSVD, the same rank rule and stopping test), so the dense tensors agree to
rounding amplified by the HOOI iteration; each side is also checked against
the uncompressed tensor within its tolerance bound."""
import numpy as np
import pytest
import torch

from oracle import apply, sinc
from oracle import tucker as tk
from paper_1212_3509_amd import api, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    api.library()
    return api.Context(0)


def _h(n):
    h = 1.0 / max(n)            # longest grid edge 1: the factors' scaled units are physical ones
    return (h, h, h)


def _dev(t):
    core, U = t
    return (torch.from_numpy(np.ascontiguousarray(core)).cuda(),
            [torch.from_numpy(np.ascontiguousarray(U[p].T)).cuda() for p in range(3)])


def _host(core, rows):
    return core.cpu().numpy(), [r.cpu().numpy().T for r in rows]


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("tol", [1e-4, 1e-9])
def test_kernel_compression_matches_oracle(ctx, tol):
    n, M = (20, 18, 16), 30
    h = _h(n)
    kt = ctx.ktucker(ctx.assemble(n, h, M=M), tol)
    _t, tau, alpha = sinc.sinc_nodes(M)
    for q in range(3):
        P = tk.cp_dense(*tk.kernel_cp(n, h, tau, alpha, q))
        c_o, U_o, _sw = tk.hooi(P, tol)
        core, rows = _host(*kt.kernel(q))
        assert core.shape == c_o.shape, (q, core.shape, c_o.shape)
        G, O = tk.tucker_dense(core, rows), tk.tucker_dense(c_o, U_o)
        e_gpu, e_or = _rel(G, P), _rel(O, P)
        print(f"kernel {q} tol {tol:g}: ranks {core.shape}, err {e_gpu:.3e} (oracle {e_or:.3e}), "
              f"vs oracle {_rel(G, O):.2e}")
        assert e_gpu <= tol
        assert _rel(G, O) <= 1e-3 * e_or + 1e-12


def _route_case(ctx, n, M, kind, ranks, tol, seed=5):
    h = _h(n)
    mag = inputs.tucker_magnetization(n, kind, ranks, seed)
    kt = ctx.ktucker(ctx.assemble(n, h, M=M), tol)
    core, rows = ctx.potential_tucker(kt, [_dev(mag[q]) for q in range(3)], tol)
    torch.cuda.synchronize()
    _t, tau, alpha = sinc.sinc_nodes(M)
    c_o, U_o = tk.potential_tucker(mag, n, h, tau, alpha, tol)
    return _host(core, rows), (c_o, U_o), mag, (h, tau, alpha)


@pytest.mark.parametrize("kind,ranks,tol", [("uniform", None, 1e-5), ("uniform", None, 1e-9),
                                            ("random", (2, 3, 2), 1e-6), ("smooth", (2, 2, 3), 1e-10)])
def test_potential_matches_oracle(ctx, kind, ranks, tol):
    n = (20, 18, 16)
    (core, rows), (c_o, U_o), mag, (h, tau, alpha) = _route_case(ctx, n, 30, kind, ranks or (1, 1, 1), tol)
    G, O = tk.tucker_dense(core, rows), tk.tucker_dense(c_o, U_o)
    m = np.stack([tk.tucker_dense(*mag[q]).transpose(2, 1, 0) for q in range(3)])
    exact = apply.kron_apply_dense(m, h, tau, alpha)[0].transpose(2, 1, 0)
    print(f"{kind} tol {tol:g}: ranks {core.shape} (oracle {c_o.shape}), vs oracle {_rel(G, O):.2e}, "
          f"vs uncompressed {_rel(G, exact):.2e} (oracle {_rel(O, exact):.2e})")
    assert core.shape == c_o.shape
    assert _rel(G, exact) < 30 * tol
    assert _rel(G, O) <= 1e-3 * max(_rel(O, exact), 1e-12) + 1e-11


@pytest.mark.parametrize("n", [(1, 5, 33), (65, 2, 9)])
def test_potential_ragged_and_degenerate_sizes(ctx, n):
    (core, rows), (c_o, U_o), mag, (h, tau, alpha) = _route_case(ctx, n, 12, "random", (1, 2, 3), 1e-8, seed=9)
    G, O = tk.tucker_dense(core, rows), tk.tucker_dense(c_o, U_o)
    assert core.shape == c_o.shape
    assert _rel(G, O) < 1e-9


def test_potential_long_axis_8192_point_transforms(ctx):
    """n_x = 4096: the DFTs have 8192 points."""
    n = (4096, 3, 2)
    (core, rows), (c_o, U_o), mag, (h, tau, alpha) = _route_case(ctx, n, 20, "random", (2, 2, 1), 1e-8, seed=11)
    G, O = tk.tucker_dense(core, rows), tk.tucker_dense(c_o, U_o)
    print(f"long axis: ranks {core.shape} (oracle {c_o.shape}), vs oracle {_rel(G, O):.2e}")
    assert core.shape == c_o.shape
    assert _rel(G, O) < 1e-9


@pytest.mark.parametrize("kind", ["uniform", "smooth"])
def test_potential_full_size_sampled(ctx, kind):
    """The paper's Alg. scpot_fft_tucker case of uniform magnetization, and a
    smooth rank-(2,2,2) one, at n = 4096 per axis (M = 40, tol 1e-8): 8
    sampled cells of the compressed potential against the uncompressed
    Kronecker operator, row by row."""
    n, M, tol = (4096, 4096, 4096), 40, 1e-8
    h = _h(n)
    mag = inputs.tucker_magnetization(n, kind, (2, 2, 2))
    kt = ctx.ktucker(ctx.assemble(n, h, M=M), tol)
    core, rows = ctx.potential_tucker(kt, [_dev(mag[q]) for q in range(3)], tol)
    core, rows = _host(core, rows)
    rng = np.random.default_rng(13)
    cells = [tuple(int(v) for v in rng.integers(0, 4096, 3)) for _ in range(6)] + [(0, 0, 0), (4095, 2048, 17)]
    got = np.array([np.einsum("abc,a,b,c->", core, rows[0][i], rows[1][j], rows[2][k]) for i, j, k in cells])
    _t, tau, alpha = sinc.sinc_nodes(M)
    ref = tk.potential_at_cells(mag, n, h, tau, alpha, cells)
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print(f"4096^3 {kind}: ranks {core.shape}, sampled rel err {err:.2e}")
    assert err < 30 * tol
    assert max(core.shape) < 64


def test_potential_full_size_uniform_against_exact_collocation(ctx):
    """Alg. scpot_fft_tucker's uniform-magnetization case at n = 4096 per axis
    with the 64-node theorem-step rule (tol 1e-8): 8 cells of the compressed
    potential against the exact collocated potential of the uniformly
    magnetized cube (closed-form box kernels of the whole cube at the cell
    centres), within 30 tol."""
    from oracle import exact
    n, tol = (4096, 4096, 4096), 1e-8
    h = _h(n)
    mag = inputs.tucker_magnetization(n, "uniform", (2, 2, 2))
    mv = np.array([np.einsum("abc,a,b,c->", mag[q][0], mag[q][1][0][0], mag[q][1][1][0], mag[q][1][2][0])
                   for q in range(3)])
    kt = ctx.ktucker(ctx.assemble(n, h, M=64, step_rule=1), tol)
    core, rows = ctx.potential_tucker(kt, [_dev(mag[q]) for q in range(3)], tol)
    core, rows = _host(core, rows)
    rng = np.random.default_rng(17)
    cells = [tuple(int(v) for v in rng.integers(0, 4096, 3)) for _ in range(6)] + [(0, 0, 0), (4095, 2048, 17)]
    got = np.array([np.einsum("abc,a,b,c->", core, rows[0][i], rows[1][j], rows[2][k]) for i, j, k in cells])
    pts = (np.array(cells, dtype=np.float64) + 0.5) * h[0]
    K, _N = exact.box_kernels_at_points(pts, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    ref = np.tensordot(mv, K, axes=1)
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print(f"4096^3 uniform, 64-node theorem rule: ranks {core.shape}, rel err vs exact collocation {err:.2e}")
    assert err < 30 * tol


@pytest.mark.parametrize("tol", [1e-3, 1e-7, 1e-12])
def test_tucker_sum_matches_oracle(ctx, tol):
    rng = np.random.default_rng(14)
    n = (40, 33, 27)
    terms = []
    for s in range(3):
        r = (4 + s, 3 + s, 5)
        core = rng.standard_normal(r) * np.einsum("i,j,k->ijk", *[0.02 ** np.arange(m) for m in r])
        terms.append((core, [rng.standard_normal((n[p], r[p])) for p in range(3)]))
    core, rows = _host(*ctx.tucker_sum(n, [_dev(t) for t in terms], tol))
    c_o, U_o = tk.tucker_sum(terms, tol)
    X = sum(tk.tucker_dense(*t) for t in terms)
    G, O = tk.tucker_dense(core, rows), tk.tucker_dense(c_o, U_o)
    print(f"sum tol {tol:g}: ranks {core.shape} (oracle {c_o.shape}), err {_rel(G, X):.2e}, vs oracle {_rel(G, O):.2e}")
    assert core.shape == c_o.shape
    assert _rel(G, X) <= tol
    if tol >= 1e-7:
        assert max(core.shape) < 15                # the tolerance truncated
    assert _rel(G, O) <= 1e-3 * max(_rel(O, X), 1e-13) + 1e-12


def _tt_dense_dev(G1, G2, G3):
    return tk.tt_dense(G1.cpu().numpy().T, np.transpose(G2.cpu().numpy(), (0, 2, 1)), G3.cpu().numpy())


def _tt_dev(G1, G2, G3):
    """Oracle layout (G1 [n0][r1], G2 [r1][n1][r2], G3 [r2][n2]) to the library's."""
    return (torch.from_numpy(np.ascontiguousarray(G1.T)).cuda(),
            torch.from_numpy(np.ascontiguousarray(np.transpose(G2, (0, 2, 1)))).cuda(),
            torch.from_numpy(np.ascontiguousarray(G3)).cuda())


@pytest.mark.parametrize("n,ranks,tol", [((30, 25, 20), (6, 5), 1e-3), ((30, 25, 20), (6, 5), 3e-5),
                                         ((50, 4096, 40), (8, 8), 1e-5)])
def test_tt_round_matches_oracle(ctx, n, ranks, tol):
    """Decaying outer cores, so that every tolerance truncates; the last case
    has middle-core rows of 32768 points (chunked Gram-Schmidt)."""
    G1, G2, G3 = inputs.tt_cores(n, ranks, decay=(0.1, 0.08))
    H = ctx.tt_round(*_tt_dev(G1, G2, G3), tol)
    O = tk.tt_round(G1, G2, G3, tol)
    A = tk.tt_dense(G1, G2, G3)
    D, DO = _tt_dense_dev(*H), tk.tt_dense(*O)
    print(f"tt tol {tol:g}: ranks {(H[0].shape[0], H[2].shape[0])} (oracle {(O[0].shape[1], O[2].shape[0])}), "
          f"err {_rel(D, A):.2e}, vs oracle {_rel(D, DO):.2e}")
    assert (H[0].shape[0], H[2].shape[0]) == (O[0].shape[1], O[2].shape[0])
    assert _rel(D, A) <= tol
    assert H[0].shape[0] < ranks[0] or H[2].shape[0] < ranks[1]
    assert _rel(D, DO) <= 1e-3 * max(_rel(DO, A), 1e-13) + 1e-12


def test_tt_round_redundant_ranks(ctx):
    rng = np.random.default_rng(15)
    n = (12, 11, 10)
    G1, G2, G3 = inputs.tt_cores(n, (3, 2), decay=(1.0, 1.0), seed=16)
    D1 = np.concatenate([G1, G1], axis=1)
    D2 = np.zeros((6, n[1], 4))
    D2[:3, :, :2] = G2
    D2[3:, :, 2:] = G2
    D3 = np.concatenate([G3, G3], axis=0)
    H = ctx.tt_round(*_tt_dev(D1, D2, D3), 1e-12)
    assert (H[0].shape[0], H[2].shape[0]) == (3, 2)
    A = tk.tt_dense(G1, G2, G3)
    assert _rel(_tt_dense_dev(*H), 2 * A) < 1e-13


def test_invalid_arguments(ctx):
    n = (8, 8, 8)
    f = ctx.assemble(n, _h(n), M=8)
    with pytest.raises(api.DemagError) as e:
        ctx.ktucker(f, 0.0)
    assert e.value.status == 1
    kt = ctx.ktucker(f, 1e-6)
    mag = [_dev(t) for t in inputs.tucker_magnetization(n, "random", (2, 2, 2))]
    with pytest.raises(api.DemagError) as e:
        ctx.potential_tucker(kt, mag, 1e-6, rmax=1)
    assert e.value.status == 4
    with pytest.raises(api.DemagError) as e:
        ctx.potential_tucker(kt, mag, 2.0)
    assert e.value.status == 1


def test_potential_non_cubic_cells_and_length_scale(ctx):
    """Unequal cell sizes with a longest edge of 2.5: the route works in the
    factors' scaled units (longest edge 1), so potential * L equals the
    oracle's route on the scaled cells times L."""
    n, M, tol = (12, 9, 7), 16, 1e-8
    h = (0.25, 0.2, 0.3)                          # edges 3.0, 1.8, 2.1: L = 3
    f = ctx.assemble(n, h, M=M)
    L = f.length_scale
    assert L == pytest.approx(3.0)
    mag = inputs.tucker_magnetization(n, "random", (2, 1, 2), seed=17)
    kt = ctx.ktucker(f, tol)
    core, rows = _host(*ctx.potential_tucker(kt, [_dev(mag[q]) for q in range(3)], tol))
    hs = tuple(x / L for x in h)
    _t, tau, alpha = sinc.sinc_nodes(M)
    c_o, U_o = tk.potential_tucker(mag, n, hs, tau, alpha, tol)
    assert core.shape == c_o.shape
    assert _rel(L * tk.tucker_dense(core, rows), L * tk.tucker_dense(c_o, U_o)) < 1e-9


def test_tucker_sum_single_cell_modes_and_one_term(ctx):
    rng = np.random.default_rng(18)
    n = (1, 17, 1)
    t = (rng.standard_normal((1, 3, 1)), [rng.standard_normal((n[p], r)) for p, r in enumerate((1, 3, 1))])
    core, rows = _host(*ctx.tucker_sum(n, [_dev(t)], 1e-10))
    X = tk.tucker_dense(*t)
    assert core.shape[0] == 1 and core.shape[2] == 1
    assert _rel(tk.tucker_dense(core, rows), X) < 1e-13


def test_tt_round_rank_one(ctx):
    G1, G2, G3 = inputs.tt_cores((9, 8, 7), (1, 1), seed=19)
    H = ctx.tt_round(*_tt_dev(G1, G2, G3), 1e-10)
    assert (H[0].shape[0], H[2].shape[0]) == (1, 1)
    assert _rel(_tt_dense_dev(*H), tk.tt_dense(G1, G2, G3)) < 1e-13


def test_potential_with_zero_components(ctx):
    """Uniform magnetization along z: the x and y components are zero
    tensors (zero cores), whose products and bases must stay finite."""
    n, M, tol = (14, 12, 10), 16, 1e-8
    h = _h(n)
    mag = [(np.array([[[v]]]), [np.ones((n[p], 1)) for p in range(3)]) for v in (0.0, 0.0, 0.7)]
    kt = ctx.ktucker(ctx.assemble(n, h, M=M), tol)
    core, rows = _host(*ctx.potential_tucker(kt, [_dev(mag[q]) for q in range(3)], tol))
    G = tk.tucker_dense(core, rows)
    assert np.all(np.isfinite(G))
    _t, tau, alpha = sinc.sinc_nodes(M)
    c_o, U_o = tk.potential_tucker(mag, n, h, tau, alpha, tol)
    assert core.shape == c_o.shape
    assert _rel(G, tk.tucker_dense(c_o, U_o)) < 1e-9


def test_tucker_sum_with_zero_term(ctx):
    rng = np.random.default_rng(20)
    n = (10, 9, 8)
    a = (rng.standard_normal((2, 2, 2)), [rng.standard_normal((n[p], 2)) for p in range(3)])
    z = (np.zeros((1, 2, 1)), [np.zeros((n[p], r)) for p, r in enumerate((1, 2, 1))])
    core, rows = _host(*ctx.tucker_sum(n, [_dev(z), _dev(a)], 1e-10))
    G = tk.tucker_dense(core, rows)
    assert np.all(np.isfinite(G)) and core.shape == (2, 2, 2)
    assert _rel(G, tk.tucker_dense(*a)) < 1e-13


def test_format_conversions_match_oracle(ctx):
    """CP -> TT (bit-exact: copies and one product), Tucker -> TT, TT ->
    Tucker (ranks and dense tensor as the oracle's HOOI), and CP -> TT ->
    rounding (the ranks of a rank-3 CP tensor stored as rank 6)."""
    rng = np.random.default_rng(22)
    n = (11, 9, 8)
    lam = rng.standard_normal(6)
    U = [rng.standard_normal((n[p], 6)) for p in range(3)]
    U = [np.concatenate([u[:, :3], u[:, :3] @ rng.standard_normal((3, 3))], axis=1) for u in U[:1]] + U[1:]
    T = ctx.cp_to_tt(torch.from_numpy(lam).cuda(), [torch.from_numpy(np.ascontiguousarray(U[p].T)).cuda()
                                                    for p in range(3)])
    O = tk.tt_from_cp(lam, U)
    assert np.array_equal(T[0].cpu().numpy().T, O[0]) and np.array_equal(T[2].cpu().numpy(), O[2])
    assert np.array_equal(np.transpose(T[1].cpu().numpy(), (0, 2, 1)), O[1])
    core, rows = _host(*ctx.tt_to_tucker(*T, 1e-12))
    c_o, U_o = tk.tucker_from_tt(*O, 1e-12)
    assert core.shape == c_o.shape
    X = tk.tt_dense(*O)
    assert _rel(tk.tucker_dense(core, rows), X) < 1e-12
    assert _rel(tk.tucker_dense(core, rows), tk.tucker_dense(c_o, U_o)) < 1e-12
    t = (rng.standard_normal((2, 3, 4)), [rng.standard_normal((n[p], r)) for p, r in enumerate((2, 3, 4))])
    T2 = ctx.tucker_to_tt(*_dev(t))
    assert _rel(_tt_dense_dev(*T2), tk.tucker_dense(*t)) < 1e-14
