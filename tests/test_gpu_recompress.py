"""GPU parity of the HOOI recompression (CP -> Tucker) with the oracle.

The GPU finds singular subspaces with a randomized range finder (K = rmax + 8
candidates), the oracle with full SVDs; both apply the same rank rule.  What
is compared: the ranks, the reported relative error against the directly
computed one, the error bound, and the reconstructed tensors."""
import numpy as np
import pytest
import torch

from oracle import recompress as rc
from oracle import sinc, structured
from paper_1212_3509_amd import api, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    api.library()
    return api.Context(0)


def _upload(A32, lam):
    """One column set per mode (the term's own column), identity table."""
    T = len(lam)
    cols = [torch.from_numpy(np.ascontiguousarray(A32[p])).cuda() for p in range(3)]
    table = torch.from_numpy(np.repeat(np.arange(T, dtype=np.int32)[:, None], 3, axis=1)).cuda()
    return cols, table, torch.from_numpy(np.asarray(lam, dtype=np.float64)).cuda()


def _dense_gpu(res):
    U = [u.cpu().numpy() for u in res["U"]]
    return rc.tucker_dense(res["core"].cpu().numpy(), [u.T for u in U])


def test_recovers_a_known_tucker_tensor(ctx):
    rng = np.random.default_rng(0)
    n = (40, 36, 32)
    r = (3, 4, 5)
    U = [np.linalg.qr(rng.standard_normal((n[p], r[p])))[0] for p in range(3)]
    core = rng.standard_normal(r)
    A, lam = rc.tucker_as_cp(core, U)
    A32 = [a.astype(np.float32) for a in A]
    A64 = [a.astype(np.float64) for a in A32]
    cols, table, lam_d = _upload(A32, lam)
    res = ctx.recompress_cp(n, cols, table, lam_d, 1e-8, rmax=16)
    ref = rc.hooi(A64, lam, 1e-8)
    assert res["ranks"] == ref["ranks"] == r
    X = rc.cp_dense(A64, lam)
    Xg = _dense_gpu(res)
    direct = np.linalg.norm(X - Xg) / np.linalg.norm(X)
    assert direct < 1e-12 and res["rel_err"] < 1e-12, (direct, res["rel_err"])
    for p in range(3):   # same subspaces as the oracle
        Ug = res["U"][p].cpu().numpy().T
        assert np.abs(Ug @ Ug.T - ref["U"][p] @ ref["U"][p].T).max() < 1e-10
        assert np.abs(Ug.T @ Ug - np.eye(r[p])).max() < 1e-12


def _structured_phi(n, M, r, seed):
    """Potential terms of the oracle's structured CP apply for a smooth CP
    input: columns per mode, term table (output phi), weights."""
    rng = np.random.default_rng(seed)
    x = [np.linspace(0, 1, n[d]) for d in range(3)]

    class CP:
        pass
    cp = CP()
    cp.lam = [np.ones(r) for _q in range(3)]
    cp.U = [[np.stack([np.cos(np.pi * (l + 1) * rng.uniform(0.5, 1.5) * x[d] + rng.uniform(0, 3))
                       for l in range(r)], axis=1) for d in range(3)] for _q in range(3)]
    h = (1.0 / max(n),) * 3
    _t, tau, alpha = sinc.sinc_nodes(M)
    cols, table = structured.cp_apply(cp, n, h, tau, alpha)
    tab = table[0]   # output phi
    lam = np.array([cp.lam[t // (M * r)][t % r] for t in range(tab.shape[0])])
    return cols, tab, lam


@pytest.mark.parametrize("eps", [1e-3, 1e-6])
def test_structured_phi_matches_oracle(ctx, eps):
    n = (48, 40, 56)
    M, r = 12, 2
    cols, tab, lam = _structured_phi(n, M, r, seed=3)
    cols32 = [c.astype(np.float32) for c in cols]
    A64 = [cols32[p][tab[:, p]].astype(np.float64) for p in range(3)]
    ref = rc.hooi(A64, lam, eps)
    res = ctx.recompress_cp(n, [torch.from_numpy(c).cuda() for c in cols32], torch.from_numpy(tab).cuda(),
                            torch.from_numpy(lam).cuda(), eps, rmax=48)
    X = rc.cp_dense(A64, lam)
    Xg = _dense_gpu(res)
    direct = np.linalg.norm(X - Xg) / np.linalg.norm(X)
    print(f"eps {eps:g}: ranks gpu {res['ranks']} oracle {ref['ranks']}, err gpu {res['rel_err']:.3e} "
          f"(direct {direct:.3e}) oracle {ref['rel_err']:.3e}, sweeps {res['sweeps']}")
    assert direct <= eps and ref["rel_err"] <= eps
    assert abs(res["rel_err"] - direct) <= 1e-3 * direct + 1e-14
    # ranks within one of the oracle's (a singular value near the threshold
    # may fall either way), and the two approximations within eps of X
    assert all(abs(a - b) <= 1 for a, b in zip(res["ranks"], ref["ranks"]))
    Xo = rc.tucker_dense(ref["core"], ref["U"])
    assert np.linalg.norm(Xg - Xo) / np.linalg.norm(X) <= 2 * eps


def test_rank_cap(ctx):
    rng = np.random.default_rng(5)
    n = (30, 28, 26)
    T = 40
    A32 = [rng.standard_normal((T, n[p])).astype(np.float32) for p in range(3)]
    A64 = [a.astype(np.float64) for a in A32]
    lam = np.ones(T)
    cols, table, lam_d = _upload(A32, lam)
    res = ctx.recompress_cp(n, cols, table, lam_d, 1e-12, rmax=4)
    assert res["ranks"] == (4, 4, 4)
    X = rc.cp_dense(A64, lam)
    direct = np.linalg.norm(X - _dense_gpu(res)) / np.linalg.norm(X)
    assert abs(res["rel_err"] - direct) < 1e-9
    # within a few percent of the oracle's (SVD-based) error at the same ranks
    ref = rc.hooi(A64, lam, 1e-12, rmax=4)
    assert res["rel_err"] <= ref["rel_err"] * 1.05


def test_invalid_arguments(ctx):
    n = (8, 8, 8)
    cols = [torch.zeros((4, 8), dtype=torch.float32, device="cuda") for _ in range(3)]
    lam = torch.ones(4, dtype=torch.float64, device="cuda")
    bad = torch.tensor([[0, 0, 0], [1, 1, 1], [2, 2, 2], [3, 3, 9]], dtype=torch.int32, device="cuda")
    with pytest.raises(api.DemagError):
        ctx.recompress_cp(n, cols, bad, lam, 1e-6, rmax=4)
    good = torch.tensor([[0, 0, 0], [1, 1, 1], [2, 2, 2], [3, 3, 3]], dtype=torch.int32, device="cuda")
    with pytest.raises(api.DemagError):    # zero tensor
        ctx.recompress_cp(n, cols, good, lam, 1e-6, rmax=4)
    with pytest.raises(api.DemagError):
        ctx.recompress_cp(n, cols, good, lam, 1e-6, rmax=65)


@pytest.mark.parametrize("eps", [1e-3, 1e-6])
def test_n4096_potential_sampled(ctx, eps):
    """The benchmarked case: the potential of a CP apply at n = 4096 (1200
    terms of smooth rank-10 columns, M = 40), rmax 64.  The tensor has 2^36
    entries, so the checks hold at any size: orthonormal factor rows, and the
    relative error over 20000 sampled entries (X from the terms, the Tucker
    form from core and factors, both in FP64 on the host) agrees with the
    reported error to within the sampling spread, and the reported error is
    within eps."""
    n = 4096
    f = ctx.assemble((n, n, n), (1.0 / n,) * 3, M=40, c0=2.15)
    x = np.linspace(0.0, 1.0, n)
    rng = np.random.default_rng(9)
    smooth = [np.stack([np.stack([np.cos(np.pi * (l + 1) * rng.uniform(0.5, 1.5) * x + rng.uniform(0, 3))
                                  for l in range(10)]) for _q in range(3)]).astype(np.float32) for _d in range(3)]
    out_cols, table = ctx.apply_cp(f, [torch.from_numpy(c).cuda() for c in smooth])
    tab = np.ascontiguousarray(table[0])
    T = tab.shape[0]
    res = ctx.recompress_cp((n, n, n), out_cols, torch.from_numpy(tab).cuda(),
                            torch.ones(T, dtype=torch.float64, device="cuda"), eps, rmax=64, max_sweeps=10)
    U = [u.cpu().numpy() for u in res["U"]]
    for p in range(3):
        assert np.abs(U[p] @ U[p].T - np.eye(U[p].shape[0])).max() < 1e-10
    core = res["core"].cpu().numpy()
    S = 20000
    idx = np.random.default_rng(4).integers(0, n, (3, S))
    cols = [o.cpu().numpy().reshape(-1, n) for o in out_cols]
    A = [cols[p][tab[:, p]][:, idx[p]].astype(np.float64) for p in range(3)]   # [T][S]
    xs = np.einsum("ts,ts,ts->s", A[0], A[1], A[2])
    ts = np.einsum("abc,as,bs,cs->s", core, U[0][:, idx[0]], U[1][:, idx[1]], U[2][:, idx[2]], optimize=True)
    sampled = np.linalg.norm(xs - ts) / np.linalg.norm(xs)
    print(f"eps {eps:g}: ranks {res['ranks']} reported {res['rel_err']:.3e} sampled {sampled:.3e}")
    assert res["rel_err"] <= eps
    # sampling accuracy: the error is spread over the entries of a smooth
    # tensor, so 20000 samples estimate it within a small factor
    assert 0.2 * res["rel_err"] <= sampled <= 5.0 * res["rel_err"] + 1e-13
