"""GPU checks of the C-ABI contract beyond the arithmetic: the structured
potential's length factor, the caller-owned workspace, the input check, the
stream switch and freeing factors while their work is still queued.

The structured potential with a grid whose longest extent L is not 1 must,
times L, densify to the full-format potential of the same operator (Eqs.
(kron_eval_cp) and (kron_operator): the same sum of Kronecker terms); the
field needs no factor.  Tolerance: FP32 columns, 1e-6 relative L2.
"""
import numpy as np
import pytest
import torch

from oracle import apply, sinc, structured
from paper_1212_3509_amd import api, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    api.library()
    return api.Context(0)


def _dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def test_structured_potential_times_length_scale(ctx):
    n, h, M, r = (12, 10, 8), (0.1, 0.1, 0.1), 10, 3
    f = ctx.assemble(n, h, M=M)
    L = f.length_scale
    assert L == pytest.approx(1.2, rel=1e-15)
    cp = inputs.cp_input(n, rank=r, seed=4, dtype=np.float32)
    U = [_dev(np.stack([cp.U[q][d].T for q in range(3)]), torch.float32) for d in range(3)]
    out, table = ctx.apply_cp(f, U)
    torch.cuda.synchronize()
    got = [o.cpu().numpy().reshape(-1, n[d]).astype(np.float64) for d, o in enumerate(out)]
    dense = structured.cp_densify(got, table, cp.lam, M, r, n)
    m = structured.cp_to_full(cp, n)
    phi, hf = ctx.apply_full(f, _dev(m), prec="fp64")
    torch.cuda.synchronize()
    phi, hf = phi.cpu().numpy(), hf.cpu().numpy()
    assert apply.rel_l2(L * dense[0], phi) < 1e-6
    assert apply.rel_l2(dense[1:], hf) < 1e-6
    # the unscaled sum is off by exactly the factor L
    assert apply.rel_l2(dense[0], phi) > 0.1
    # and both agree with the oracle's scaled-domain operator
    hs = [x / L for x in h]
    _t, tau, alpha = sinc.sinc_nodes(M)
    pref, href = apply.kron_apply_dense(m, hs, tau, alpha)
    assert apply.rel_l2(phi, L * pref) < 1e-12 and apply.rel_l2(hf, href) < 1e-12


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_caller_workspace(ctx, prec):
    """apply_full_ws on a workspace large enough for one chunk is bitwise
    equal to apply_full; on the minimum workspace (one node per chunk) it is
    the same sum in another association order."""
    n, M = (20, 14, 9), 12
    f = ctx.assemble(n, (1 / 20,) * 3, M=M)
    N = n[0] * n[1] * n[2]
    es = 8 if prec == "fp64" else 4
    one, minimum = f.workspace_size(prec)
    assert one == (12 * M + 4) * N * es and minimum == 16 * N * es
    dt = torch.float64 if prec == "fp64" else torch.float32
    m = _dev(inputs.random_unit_field(n, seed=8), dt)
    p0, h0 = ctx.apply_full(f, m, prec=prec)
    ws = torch.empty(one // 4, dtype=torch.float32, device="cuda")
    p1, h1 = ctx.apply_full_ws(f, m, ws, prec=prec)
    ws_min = torch.empty(minimum // 4, dtype=torch.float32, device="cuda")
    p2, h2 = ctx.apply_full_ws(f, m, ws_min, prec=prec)
    torch.cuda.synchronize()
    assert torch.equal(p0, p1) and torch.equal(h0, h1)
    tol = 1e-13 if prec == "fp64" else 1e-6
    assert float((p2 - p0).norm() / p0.norm()) < tol and float((h2 - h0).norm() / h0.norm()) < tol
    small = torch.empty(minimum // 4 - 64, dtype=torch.float32, device="cuda")
    with pytest.raises(api.DemagError) as e:
        ctx.apply_full_ws(f, m, small, prec=prec)
    assert e.value.status == 2


def test_input_check_rejects_nonfinite(ctx):
    n = (8, 6, 5)
    f = ctx.assemble(n, (0.1,) * 3, M=8)
    m = inputs.random_unit_field(n, seed=1)
    ctx.set_input_check(True)
    try:
        for bad in (np.nan, np.inf, -np.inf):
            mm = m.copy()
            mm[1, 2, 3, 4] = bad
            for prec in ("fp64", "fp32"):
                dt = torch.float64 if prec == "fp64" else torch.float32
                with pytest.raises(api.DemagError) as e:
                    ctx.apply_full(f, _dev(mm, dt), prec=prec)
                assert e.value.status == 1 and "NaN" in str(e.value)
            with pytest.raises(api.DemagError):
                ctx.apply_fft(f, _dev(mm))
            cols = [torch.ones((3, 2, n[d]), dtype=torch.float32, device="cuda") for d in range(3)]
            cols[1][0, 1, 2] = float(bad)
            with pytest.raises(api.DemagError):
                ctx.apply_columns(f, cols)
        # finite inputs pass the check and give the unchecked result
        p1, h1 = ctx.apply_full(f, _dev(m), prec="fp64")
    finally:
        ctx.set_input_check(False)
    p0, h0 = ctx.apply_full(f, _dev(m), prec="fp64")
    torch.cuda.synchronize()
    assert torch.equal(p0, p1) and torch.equal(h0, h1)


def test_stream_switch_orders_shared_workspace(ctx):
    """Calls alternating between two streams share the context workspace; the
    switch makes the new stream wait for the old one, so every result equals
    the one computed alone."""
    n, M = (64, 64, 32), 20
    f = ctx.assemble(n, (1 / 64,) * 3, M=M)
    fields = [_dev(inputs.random_unit_field(n, seed=20 + i)) for i in range(4)]
    alone = []
    for m in fields:
        alone.append(ctx.apply_full(f, m, prec="fp64"))
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = []
    for i, m in enumerate(fields):
        with torch.cuda.stream(streams[i % 2]):
            outs.append(ctx.apply_full(f, m, prec="fp64"))
    torch.cuda.synchronize()
    for (p, hh), (pa, ha) in zip(outs, alone):
        assert torch.equal(p, pa) and torch.equal(hh, ha)


def test_free_factors_with_work_queued(ctx):
    """demag_factors_free waits for the queued work that reads the factors:
    freeing right after an asynchronous apply leaves its result intact."""
    n, M = (48, 40, 36), 24
    m = _dev(inputs.random_unit_field(n, seed=2))
    f = ctx.assemble(n, (1 / 48,) * 3, M=M)
    p_ref, h_ref = ctx.apply_full(f, m, prec="fp64")
    torch.cuda.synchronize()
    f2 = ctx.assemble(n, (1 / 48,) * 3, M=M)
    p, hh = ctx.apply_full(f2, m, prec="fp64")
    f2.free()
    torch.cuda.synchronize()
    assert torch.equal(p, p_ref) and torch.equal(hh, h_ref)
