"""GPU parity of the structured (CP / Tucker / TT) apply against the oracle.

Columns are FP32 in and out.  With FP64 transforms each output column is
within FP32 rounding of the oracle's dense-Toeplitz FP64 product; with FP32
transforms (FP64 forward transforms, FP32 spectra and inverse transforms)
within the FP32 roundoff of the inverse transform, relative to the column's
own norm.  The bound for both: 1e-6 of the column norm plus 1e-12 of the
largest column (or, per sampled job, of the largest generator of the job's
factor type times the input column: very narrow kernels give columns that
underflow FP32).  Term and block tables are integer results and must match
exactly."""
import numpy as np
import pytest
import torch

from oracle import apply, exact, sinc, structured
from paper_1212_3509_amd import api, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    api.library()
    return api.Context(0)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _check_cols(got, ref, tol=1e-6):
    """got/ref: lists per axis of arrays [ncols][n]."""
    big = max(np.linalg.norm(r, axis=1).max() for r in ref)
    worst = 0.0
    for g, r in zip(got, ref):
        err = np.linalg.norm(g - r, axis=1)
        nrm = np.linalg.norm(r, axis=1)
        assert np.all(err <= tol * nrm + 1e-12 * big), (err / np.maximum(nrm, 1e-300)).max()
        ok = nrm > 1e-6 * big
        if ok.any():
            worst = max(worst, float((err[ok] / nrm[ok]).max()))
    return worst


def _oracle_rule(n, h, M):
    L = max(n[d] * h[d] for d in range(3))
    hs = [x / L for x in h]
    _t, tau, alpha = sinc.sinc_nodes(M)
    return hs, tau, alpha


N_SMALL = (9, 8, 7)
H_SMALL = (1 / 9,) * 3


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_cp_small(ctx, prec):
    M, r = 6, 3
    f = ctx.assemble(N_SMALL, H_SMALL, M=M)
    cp = inputs.cp_input(N_SMALL, rank=r, seed=1, dtype=np.float32)
    U = [_dev(np.stack([cp.U[q][d].T for q in range(3)])) for d in range(3)]
    out, table = ctx.apply_cp(f, U, prec=prec)
    torch.cuda.synchronize()
    hs, tau, alpha = _oracle_rule(N_SMALL, H_SMALL, M)
    cols, tab_ref = structured.cp_apply(cp, N_SMALL, hs, tau, alpha)
    got = [o.cpu().numpy().reshape(-1, N_SMALL[d]).astype(np.float64) for d, o in enumerate(out)]
    worst = _check_cols(got, cols)
    assert np.array_equal(table, tab_ref)
    # the structured result densifies to the full-format operator applied to the CP tensor
    dense = structured.cp_densify(got, table, cp.lam, M, r, N_SMALL)
    phi, hf = apply.kron_apply_dense(structured.cp_to_full(cp, N_SMALL), hs, tau, alpha)
    assert apply.rel_l2(dense[0], phi) < 1e-6 and apply.rel_l2(dense[1:], hf) < 1e-6
    print(f"cp small: worst column rel err {worst:.2e}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_tucker_small(ctx, prec):
    M, ranks = 5, (2, 3, 2)
    n = (12, 10, 16)
    h = (1 / 16,) * 3
    f = ctx.assemble(n, h, M=M)
    tk = inputs.tucker_input(n, ranks=ranks, seed=1, dtype=np.float32)
    U = [_dev(np.stack([tk.U[q][d].T for q in range(3)])) for d in range(3)]
    out, table = ctx.apply_tucker(f, U, prec=prec)
    torch.cuda.synchronize()
    hs, tau, alpha = _oracle_rule(n, h, M)
    cols, tab_ref = structured.tucker_apply(tk, n, hs, tau, alpha)
    got = [o.cpu().numpy().reshape(-1, n[d]).astype(np.float64) for d, o in enumerate(out)]
    _check_cols(got, cols)
    assert np.array_equal(table, tab_ref)
    dense = structured.tucker_densify(got, table, tk.core, M, n)
    phi, hf = apply.kron_apply_dense(structured.tucker_to_full(tk, n), hs, tau, alpha)
    assert apply.rel_l2(dense[0], phi) < 1e-6 and apply.rel_l2(dense[1:], hf) < 1e-6


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_tt_small(ctx, prec):
    M, r1, r2 = 4, 2, 3
    n = (7, 13, 5)
    h = (0.1, 0.1, 0.1)
    f = ctx.assemble(n, h, M=M)
    tt = inputs.tt_input(n, ranks=(r1, r2), seed=2, dtype=np.float32)
    G1 = _dev(np.stack([tt.G1[q].T for q in range(3)]))                    # [q][a][x]
    G2 = _dev(np.stack([tt.G2[q].transpose(0, 2, 1) for q in range(3)]))   # [q][a][b][y]
    G3 = _dev(np.stack([tt.G3[q] for q in range(3)]))                      # [q][b][z]
    out, table = ctx.apply_tt(f, G1, G2, G3, prec=prec)
    torch.cuda.synchronize()
    hs, tau, alpha = _oracle_rule(n, h, M)
    cols, tab_ref = structured.tt_apply(tt, n, hs, tau, alpha)
    got = [o.cpu().numpy().reshape(-1, n[d]).astype(np.float64) for d, o in enumerate(out)]
    _check_cols(got, cols)
    assert np.array_equal(table, tab_ref)
    dense = structured.tt_densify(got, table, M, n, r1, r2)
    L = max(n[d] * h[d] for d in range(3))
    phi, hf = apply.kron_apply_dense(structured.tt_to_full(tt, n), hs, tau, alpha)
    assert apply.rel_l2(dense[0], phi) < 1e-6 and apply.rel_l2(dense[1:], hf) < 1e-6
    assert L > 1.0   # the potential of the physical grid is L times the scaled one


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_cp_ragged_mid_lengths(ctx, prec):
    """Axes of 200, 700 and 1500 cells (transform lengths 512, 2048, 4096:
    half-length lines of 256, 1024 and 2048 points), CP rank 3, M = 12,
    every column against the oracle's dense-Toeplitz products."""
    n, h, M, r = (200, 700, 1500), (1 / 1500,) * 3, 12, 3
    f = ctx.assemble(n, h, M=M)
    cp = inputs.cp_input(n, rank=r, seed=6, dtype=np.float32)
    U = [_dev(np.stack([cp.U[q][d].T for q in range(3)])) for d in range(3)]
    out, table = ctx.apply_cp(f, U, prec=prec)
    torch.cuda.synchronize()
    hs, tau, alpha = _oracle_rule(n, h, M)
    cols, tab_ref = structured.cp_apply(cp, n, hs, tau, alpha)
    got = [o.cpu().numpy().reshape(-1, n[d]).astype(np.float64) for d, o in enumerate(out)]
    worst = _check_cols(got, cols)
    assert np.array_equal(table, tab_ref)
    print(f"cp ragged {prec}: worst column rel err {worst:.2e}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_cp_4096_rank10_sampled(ctx, prec):
    """n = 4096 per axis, CP rank 10 (seed 1), M = 40: 30 sampled jobs of each
    axis against direct FP64 convolution with the oracle's generators."""
    n, M, r = 4096, 40, 10
    f = ctx.assemble((n, n, n), (1 / n,) * 3, M=M)
    cp = inputs.cp_input(n, rank=r, seed=1, dtype=np.float32)
    U = [_dev(np.stack([cp.U[q][d].T for q in range(3)])) for d in range(3)]
    out, table = ctx.apply_cp(f, U, prec=prec)
    torch.cuda.synchronize()
    assert np.array_equal(table, structured.term_table(M, r))
    _t, tau, alpha = sinc.sinc_nodes(M)
    F = sinc.scaled_factors(n, 1 / n, tau, alpha)
    rng = np.random.default_rng(0)
    got_all = [o.cpu().numpy() for o in out]
    worst = 0.0
    for d in range(3):
        for _ in range(30):
            q, s, k, l = int(rng.integers(3)), int(rng.integers(2)), int(rng.integers(M)), int(rng.integers(r))
            t = structured.type_of(q, d, s)
            u = cp.U[q][d][:, l].astype(np.float64)
            ref = np.convolve(F[t, k], u)[n - 1:2 * n - 1]
            got = got_all[d][q, s, k, l].astype(np.float64)
            nrm = np.linalg.norm(ref)
            err = np.linalg.norm(got - ref)
            floor = 1e-12 * np.abs(F[t]).sum(axis=1).max() * np.linalg.norm(u)
            assert err <= 1e-6 * nrm + floor, (d, q, s, k, l, err / nrm)
            if nrm > 0:
                worst = max(worst, err / nrm)
    print(f"cp 4096 {prec}: worst sampled column rel err {worst:.2e}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_cp_4096_lines_ragged(ctx, prec):
    """Axes of 2049, 3001 and 4096 cells: every axis on 4096-point half-length
    lines (the 512-thread forward and job kernels) with the column shorter
    than the line on two axes; CP rank 2 (seed 4), M = 12, 25 sampled jobs
    per axis against direct FP64 convolution with the oracle's generators."""
    n, M, r = (2049, 3001, 4096), 12, 2
    h = (1 / 4096,) * 3
    f = ctx.assemble(n, h, M=M)
    cp = inputs.cp_input(n, rank=r, seed=4, dtype=np.float32)
    U = [_dev(np.stack([cp.U[q][d].T for q in range(3)])) for d in range(3)]
    out, table = ctx.apply_cp(f, U, prec=prec)
    torch.cuda.synchronize()
    assert np.array_equal(table, structured.term_table(M, r))
    hs, tau, alpha = _oracle_rule(n, h, M)
    rng = np.random.default_rng(3)
    got_all = [o.cpu().numpy() for o in out]
    worst = 0.0
    for d in range(3):
        F = sinc.scaled_factors(n[d], hs[d], tau, alpha)
        for _ in range(25):
            q, s, k, l = int(rng.integers(3)), int(rng.integers(2)), int(rng.integers(M)), int(rng.integers(r))
            t = structured.type_of(q, d, s)
            u = cp.U[q][d][:, l].astype(np.float64)
            ref = np.convolve(F[t, k], u)[n[d] - 1:2 * n[d] - 1]
            got = got_all[d][q, s, k, l].astype(np.float64)
            nrm = np.linalg.norm(ref)
            err = np.linalg.norm(got - ref)
            floor = 1e-12 * np.abs(F[t]).sum(axis=1).max() * np.linalg.norm(u)
            assert err <= 1e-6 * nrm + floor, (d, q, s, k, l, err / nrm)
            if nrm > 0:
                worst = max(worst, err / nrm)
    print(f"cp 4096-point lines ragged {prec}: worst sampled column rel err {worst:.2e}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_cp_mixed_line_lengths(ctx, prec):
    """Axes of 3000, 64 and 200 cells (half-length lines of 4096, 64 and 256
    points): a 4096-point line beside shorter ones takes the 256-thread
    kernels for every axis.  CP rank 3 (seed 8), M = 10, 20 sampled jobs per
    axis against direct FP64 convolution with the oracle's generators."""
    n, M, r = (3000, 64, 200), 10, 3
    h = (1 / 3000,) * 3
    f = ctx.assemble(n, h, M=M)
    cp = inputs.cp_input(n, rank=r, seed=8, dtype=np.float32)
    U = [_dev(np.stack([cp.U[q][d].T for q in range(3)])) for d in range(3)]
    out, table = ctx.apply_cp(f, U, prec=prec)
    torch.cuda.synchronize()
    assert np.array_equal(table, structured.term_table(M, r))
    hs, tau, alpha = _oracle_rule(n, h, M)
    rng = np.random.default_rng(2)
    got_all = [o.cpu().numpy() for o in out]
    worst = 0.0
    for d in range(3):
        F = sinc.scaled_factors(n[d], hs[d], tau, alpha)
        for _ in range(20):
            q, s, k, l = int(rng.integers(3)), int(rng.integers(2)), int(rng.integers(M)), int(rng.integers(r))
            t = structured.type_of(q, d, s)
            u = cp.U[q][d][:, l].astype(np.float64)
            ref = np.convolve(F[t, k], u)[n[d] - 1:2 * n[d] - 1]
            got = got_all[d][q, s, k, l].astype(np.float64)
            nrm = np.linalg.norm(ref)
            err = np.linalg.norm(got - ref)
            floor = 1e-12 * np.abs(F[t]).sum(axis=1).max() * np.linalg.norm(u)
            assert err <= 1e-6 * nrm + floor, (d, q, s, k, l, err / nrm)
            if nrm > 0:
                worst = max(worst, err / nrm)
    print(f"cp mixed line lengths {prec}: worst sampled column rel err {worst:.2e}")


def _check_sampled(got_all, cols_of, R, n, F, M, rng, label, count=40):
    """count sampled (q, s, k, column) jobs per axis against direct FP64
    convolutions of the oracle's generators with the input columns."""
    worst = 0.0
    for d in range(3):
        for _ in range(count):
            q, s, k, l = int(rng.integers(3)), int(rng.integers(2)), int(rng.integers(M)), int(rng.integers(R[d]))
            t = structured.type_of(q, d, s)
            u = cols_of(q, d, l).astype(np.float64)
            ref = np.convolve(F[t, k], u)[n - 1:2 * n - 1]
            got = got_all[d][q, s, k, l].astype(np.float64)
            nrm = np.linalg.norm(ref)
            err = np.linalg.norm(got - ref)
            floor = 1e-12 * np.abs(F[t]).sum(axis=1).max() * np.linalg.norm(u)
            assert err <= 1e-6 * nrm + floor, (label, d, q, s, k, l, err / max(nrm, 1e-300))
            if nrm > 0:
                worst = max(worst, err / nrm)
    print(f"{label} 4096: worst sampled column rel err {worst:.2e}")


@pytest.mark.parametrize("prec,rule", [("fp64", 0), ("fp32", 0), ("fp32", 1)])
def test_tucker_tt_4096_sampled(ctx, prec, rule):
    """n = 4096 per axis: Tucker (8,8,8) and TT (1,8,8,1) inputs (seed 1), 40
    sampled jobs of each axis against direct FP64 convolutions; block tables
    exactly.  Rules: M = 40 (c0 = 2.15) and the theorem-step rule with 64
    nodes (its largest nodes give kernels that underflow FP32)."""
    n = 4096
    M = 40 if rule == 0 else 64
    f = ctx.assemble((n, n, n), (1 / n,) * 3, M=M, step_rule=rule)
    _t, tau, alpha = sinc.sinc_nodes(M, step_rule=rule, h_min=1 / n)
    F = sinc.scaled_factors(n, 1 / n, tau, alpha)
    rng = np.random.default_rng(5)
    tk = inputs.tucker_input(n, ranks=(8, 8, 8), seed=1, dtype=np.float32)
    V = [_dev(np.stack([tk.U[q][d].T for q in range(3)])) for d in range(3)]
    out, table = ctx.apply_tucker(f, V, prec=prec)
    torch.cuda.synchronize()
    assert np.array_equal(table, structured.block_table(M, (8, 8, 8)))
    _check_sampled([o.cpu().numpy() for o in out], lambda q, d, l: tk.U[q][d][:, l], (8, 8, 8), n, F, M, rng,
                   f"tucker (8,8,8) {prec} rule {rule}")
    del out
    tt = inputs.tt_input(n, ranks=(8, 8), seed=1, dtype=np.float32)
    G1 = _dev(np.stack([tt.G1[q].T for q in range(3)]))
    G2 = _dev(np.stack([tt.G2[q].transpose(0, 2, 1) for q in range(3)]))
    G3 = _dev(np.stack([tt.G3[q] for q in range(3)]))
    out, table = ctx.apply_tt(f, G1, G2, G3, prec=prec)
    torch.cuda.synchronize()
    assert np.array_equal(table, structured.block_table(M, (8, 64, 8)))

    def tt_cols(q, d, l):
        if d == 0:
            return tt.G1[q][:, l]                    # column l of G1
        if d == 1:
            return tt.G2[q][l // 8, :, l % 8]        # fibre (a, b) = (l // r2, l % r2)
        return tt.G3[q][l, :]                        # row l of G3
    _check_sampled([o.cpu().numpy() for o in out], tt_cols, (8, 64, 8), n, F, M, rng, f"tt (1,8,8,1) {prec} rule {rule}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_uniform_cube_4096_matches_exact_collocation(ctx, prec):
    """n = 4096 per axis (unit cube), the library's 64-node theorem-step
    rule, a uniform magnetization as a rank-1 CP input (the component folded
    into the x column): the potential and field assembled from the output
    columns at corners, face and edge centres and interior cells equal the
    exact collocated values of the uniformly magnetized cube (closed-form
    box kernels at the cell centres) within 1e-6 relative L2 per cell."""
    n = 4096
    f = ctx.assemble((n, n, n), (1 / n,) * 3, M=64, step_rule=1)
    L = f.length_scale
    m = np.array([0.3, -0.5, 0.8])
    ones = np.ones(n)
    U = [_dev(np.stack([(m[q] * ones)[None, :] for q in range(3)]))] + \
        [_dev(np.stack([ones[None, :] for _q in range(3)])) for _d in range(2)]
    out, table = ctx.apply_cp(f, U, prec=prec)
    torch.cuda.synchronize()
    cols = [o.cpu().numpy().astype(np.float64).reshape(-1, n) for o in out]
    cells = [(0, 0, 0), (4095, 4095, 4095), (0, 2048, 2048), (2048, 0, 4095), (2048, 2048, 2048),
             (1234, 3000, 17), (4095, 2048, 1), (700, 701, 702)]
    worst = 0.0
    for cell in cells:
        got = np.zeros(4)
        for o in range(4):
            tab = table[o]
            got[o] = np.sum(cols[0][tab[:, 0], cell[0]] * cols[1][tab[:, 1], cell[1]] * cols[2][tab[:, 2], cell[2]])
        got[0] *= L
        pt = (np.array(cell) + 0.5) / n
        K, N = exact.box_kernels_at_points(pt, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
        ref = np.concatenate([[K @ m], -N @ m])
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        worst = max(worst, err)
        assert err < 1e-6, (cell, got, ref)
    print(f"uniform cube 4096 {prec}: worst cell rel err vs exact collocation {worst:.2e}")


def test_columns_rejects_bad_arguments(ctx):
    f = ctx.assemble((8, 8, 8), (0.125,) * 3, M=4)
    lib = api.library()
    import ctypes as C
    R = (C.c_int32 * 3)(-1, 1, 1)
    null3 = (C.c_void_p * 3)(None, None, None)
    assert lib.demag_apply_columns(ctx.handle, f.handle, 0, R, null3, null3) == 1
    R1 = (C.c_int32 * 3)(1, 1, 1)
    assert lib.demag_apply_columns(ctx.handle, f.handle, 3, R1, null3, null3) in (1, 4)
