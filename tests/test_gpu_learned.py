"""GPU checks of the shortened-rule network and its judge against the oracle.

Network (FP32 on the GPU, FP64 in the oracle): outputs to 1e-5 relative,
parameter gradients to 1e-4 relative L2.  Judge (FP64 on both sides, own
factor code on each): errors to 1e-6 relative, gradients against central
differences of the oracle judge to 1e-4.  Training must lower the loss and
give lower judged errors than the unmodified base rule at equal R'."""
import numpy as np
import pytest
import torch

from oracle import mlp, quadrule
from paper_1212_3509_amd import api, inputs, learned

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    api.library()
    return api.Context(0)


def test_forward_backward_match_oracle(ctx):
    rng = np.random.default_rng(1)
    p = inputs.mlp_init(seed=6, out_scale=1.0)
    X = rng.standard_normal((37, 6)).astype(np.float32)
    dY = rng.standard_normal((37, 65)).astype(np.float32)
    pd, Xd, dYd = (torch.from_numpy(a).cuda() for a in (p, X, dY))
    y, z, a = ctx.mlp_forward(pd, Xd)
    g = ctx.mlp_backward(pd, Xd, z, a, dYd)
    torch.cuda.synchronize()
    yr, cache = mlp.forward(p, X)
    gr = mlp.backward(p, cache, dY)
    assert np.abs(y.cpu().numpy() - yr).max() <= 1e-5 * np.abs(yr).max()
    assert np.linalg.norm(g.cpu().numpy() - gr) <= 1e-4 * np.linalg.norm(gr)


def test_adam_matches_oracle(ctx):
    rng = np.random.default_rng(2)
    p = rng.standard_normal(1000).astype(np.float32)
    gr = rng.standard_normal(1000).astype(np.float32)
    m = (0.1 * rng.standard_normal(1000)).astype(np.float32)
    v = np.abs(0.1 * rng.standard_normal(1000)).astype(np.float32)
    pd, gd, md, vd = (torch.from_numpy(a.copy()).cuda() for a in (p, gr, m, v))
    ctx.adam_step(pd, gd, md, vd, step=3, lr=1e-2)
    torch.cuda.synchronize()
    pr, mr, vr = mlp.adam(p.astype(np.float64), gr.astype(np.float64), m.astype(np.float64),
                          v.astype(np.float64), 3, lr=1e-2)
    assert np.allclose(pd.cpu().numpy(), pr, rtol=1e-5, atol=1e-6)
    assert np.allclose(md.cpu().numpy(), mr, rtol=1e-5, atol=1e-7)


def _cases():
    grids = np.array([[32, 40, 36], [64, 64, 64], [48, 33, 50], [40, 64, 32]], dtype=np.int32)
    R = np.array([16, 24, 32, 20], dtype=np.int32)
    rng = np.random.default_rng(3)
    Y = (0.3 * rng.standard_normal((4, 65))).astype(np.float32)
    return grids, R, Y


def test_rules_and_judge_match_oracle(ctx):
    grids, R, Y = _cases()
    B = len(R)
    h = 1.0 / grids.max(axis=1)
    Yd = torch.from_numpy(Y).cuda()
    Rd = torch.from_numpy(R).cuda()
    t, a = ctx.quad_rules(Yd, Rd)
    sent = np.stack([inputs.sentinel_offsets(tuple(g)) for g in grids])
    err, dt, da = ctx.quad_judge(torch.from_numpy(grids).cuda(), torch.from_numpy(h).cuda(),
                                 torch.from_numpy(sent).cuda(), t, a, Rd, grad=True)
    torch.cuda.synchronize()
    t, a, err, dt, da = (x.cpu().numpy() for x in (t, a, err, dt, da))
    for b in range(B):
        n = tuple(int(v) for v in grids[b])
        hh = (h[b],) * 3
        tr, ar = quadrule.rule_from_outputs(Y[b].astype(np.float64), int(R[b]), h[b])
        assert np.allclose(t[b, :R[b]], tr, rtol=1e-14, atol=0) and np.allclose(a[b, :R[b]], ar, rtol=1e-13, atol=0)
        assert np.all(t[b, R[b]:] == 0)
        t_ref, a_ref = quadrule.reference_rule(h[b])
        ref = quadrule.kernel_values(n, hh, t_ref, a_ref, sent[b])
        e_or = quadrule.judge(n, hh, tr, ar, ref, sent[b])
        assert abs(err[b] - e_or) <= 1e-6 * e_or
        gt, ga = quadrule.judge_grad_fd(n, hh, tr, ar, ref, sent[b])
        assert np.linalg.norm(dt[b, :R[b]] - gt) <= 1e-4 * np.linalg.norm(gt)
        assert np.linalg.norm(da[b, :R[b]] - ga) <= 1e-4 * np.linalg.norm(ga)


@pytest.fixture(scope="module")
def trained(ctx):
    cases = learned.prepare_cases(4096, seed=3)
    params, loss = learned.train(ctx, cases, steps=400, batch=512)
    torch.cuda.synchronize()
    return params, loss


def test_training_lowers_loss_and_beats_base_rule(ctx, trained):
    params, loss = trained
    assert np.isfinite(loss).all()
    assert loss[-20:].mean() < loss[:5].mean() - 1.0        # ln err drops by > e
    # held-out cases (the recipe's next draws)
    test = learned.prepare_cases(256, seed=11, shuffle_seed=12)
    y, _z, _a = ctx.mlp_forward(params, test["x"])
    t1, a1 = ctx.quad_rules(y, test["R"])
    t0, a0 = ctx.quad_rules(None, test["R"])
    e1 = ctx.quad_judge(test["grids"], test["hmin"], test["sent"], t1, a1, test["R"])
    e0 = ctx.quad_judge(test["grids"], test["hmin"], test["sent"], t0, a0, test["R"])
    torch.cuda.synchronize()
    ratio = (e1 / e0).cpu().numpy()
    gmean = float(np.exp(np.mean(np.log(ratio))))
    print(f"held-out: geometric mean error ratio learned/base {gmean:.3e}, better in {np.mean(ratio < 1):.0%}")
    assert gmean < 0.5 and np.mean(ratio < 1) > 0.8


def test_predict_and_fallback(ctx, trained):
    params, _loss = trained
    r = learned.predict(ctx, params, (48, 64, 40), 1e-6)
    assert 16 <= r["R"] <= 32 or (r["fell_back"] and r["R"] == 64)
    if not r["fell_back"]:
        assert r["judged"] <= 1e-6
    r2 = learned.predict(ctx, params, (48, 64, 40), 1e-13)   # unattainable with R' <= 32
    assert r2["fell_back"] and r2["R"] == 64 and r2["judged"] > 1e-13
