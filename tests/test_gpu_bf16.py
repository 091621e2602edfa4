"""GPU checks of the bfloat16-split precisions.

The split itself is integer work and must match the oracle's bit operations
exactly.  The applies are compared with the FP64 GPU result: three-part
splits carry 24 significant bits like FP32 (same bound as FP32), two-part
splits 16 bits (about 4e-6 on the potential at 128^3)."""
import numpy as np
import pytest
import torch

from oracle import bf16
from paper_1212_3509_amd import api, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    api.library()
    return api.Context(0)


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def test_split_bits_match_oracle(ctx):
    rng = np.random.default_rng(9)
    x = (rng.standard_normal(200000) * np.exp(rng.uniform(-30, 30, 200000))).astype(np.float32)
    x[:4] = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -1 - 2 ** -8], dtype=np.float32)
    parts = ctx.bf16_split(torch.from_numpy(x).cuda(), 3)
    torch.cuda.synchronize()
    got = parts.cpu().numpy().view(np.uint16)
    ref = np.stack(bf16.split(x, 3))
    assert np.array_equal(got, ref)


def _apply(ctx, f, m, prec):
    dt = torch.float64 if prec == "fp64" else torch.float32
    phi, hf = ctx.apply_full(f, torch.from_numpy(m).to(device="cuda", dtype=dt), prec=prec)
    torch.cuda.synchronize()
    return phi.double().cpu().numpy(), hf.double().cpu().numpy()


@pytest.mark.parametrize("n,h", [((32, 32, 32), (1 / 32,) * 3), ((13, 10, 7), (0.1, 0.12, 0.08)),
                                 ((40, 3, 17), (0.05, 0.05, 0.05))])
def test_bf16_split_applies(ctx, n, h):
    f = ctx.assemble(n, h, M=40 if n[0] == 32 else 16)
    m = inputs.random_unit_field(n, seed=0)
    p64, h64 = _apply(ctx, f, m, "fp64")
    p3, h3 = _apply(ctx, f, m, "bf16x3")
    p2, h2 = _apply(ctx, f, m, "bf16x2")
    e3 = (_rel(p3, p64), _rel(h3, h64))
    e2 = (_rel(p2, p64), _rel(h2, h64))
    print(f"{n}: bf16x3 phi {e3[0]:.2e} h {e3[1]:.2e}; bf16x2 phi {e2[0]:.2e} h {e2[1]:.2e}")
    assert max(e3) < 1e-6
    assert max(e2) < 3e-5
    assert e2[1] > e3[1]


def test_bf16x3_128_vortex(ctx):
    n = 128
    f = ctx.assemble((n, n, n), (1 / n,) * 3, M=40)
    m = inputs.vortex_field(n, seed=0)
    p64, h64 = _apply(ctx, f, m, "fp64")
    p3, h3 = _apply(ctx, f, m, "bf16x3")
    e_phi, e_h = _rel(p3, p64), _rel(h3, h64)
    print(f"128^3 bf16x3 vs fp64: phi {e_phi:.3e}  h {e_h:.3e}")
    assert e_h < 1e-6 and e_phi < 1e-6


@pytest.mark.parametrize("prec", ["bf16x3", "bf16x2"])
def test_x_stage_partial_sums(ctx, prec):
    """The x stage's sums over nodes run as four partial-sum jobs when a node
    chunk has at least 3 nodes, as single jobs otherwise (1-node chunks, set
    through the workspace limit, or M = 2); with 3-node chunks the partial
    sums of several chunks accumulate.  All agree with FP64 to the split
    precision, and with each other to FP32 summation order."""
    n = (24, 20, 36)
    h = (1 / 36,) * 3
    m = inputs.random_unit_field(n, seed=5)
    tol = 1e-6 if prec == "bf16x3" else 3e-5
    for M in (2, 12):
        f = ctx.assemble(n, h, M=M)
        p64, h64 = _apply(ctx, f, m, "fp64")
        ps, hs = _apply(ctx, f, m, prec)                 # one chunk of M nodes
        N = n[0] * n[1] * n[2]
        runs = [(ps, hs)]
        # one node per chunk (single jobs), and chunks of 3 nodes (partial
        # sums accumulated over several chunks)
        for kc in (1, 3):
            ctx.set_workspace_limit(4 * N * 4 + 12 * N * 4 * kc)
            try:
                runs.append(_apply(ctx, f, m, prec))
            finally:
                ctx.set_workspace_limit(16 << 30)
        for p, hh in runs:
            assert _rel(p, p64) < tol and _rel(hh, h64) < tol, (M, _rel(p, p64), _rel(hh, h64))
        for p, hh in runs[1:]:
            assert _rel(ps, p) < 1e-6 and _rel(hs, hh) < 1e-6
