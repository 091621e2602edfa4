"""GPU checks of the shortened-rule network, its judge, its certificate and
the per-grid fit against the oracle, and of what the learned path gains.

Network (FP32 on the GPU, FP64 in the oracle): outputs to 1e-5 relative,
parameter gradients to 1e-4 relative L2.  Judge (FP64 on both sides, own
factor code on each): errors to 1e-6 relative, gradients against central
differences of the oracle judge to 1e-4.  Certificate: the exact operator
Frobenius-norm errors of the oracle to 1e-9 (small grids); on the 128^3 and
256^3 vortex and random fields it bounds the measured relative L2 error of
every rule (vortex: measured <= certified; random inputs: the certificate is
the expected error, measured <= 1.1 x certified).  Fit: one damped
Gauss-Newton step (analytic Jacobian on the GPU, central differences in the
oracle) to 1e-4 of the step; fitted errors equal the oracle's judge of the
returned rule.  Gain: at 128^3 and 1e-6 the learned rule needs at most 0.8x
the nodes the plain sinc rule needs for the same certified tolerance."""
import numpy as np
import pytest
import torch

from oracle import mlp, quadrule, sinc
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
    ow = [inputs.fit_offsets(tuple(int(v) for v in g)) for g in grids]
    sent = np.stack([o[0] for o in ow])
    wts = np.stack([o[1] for o in ow])
    err, parts, dt, da = ctx.quad_judge(torch.from_numpy(grids).cuda(), torch.from_numpy(h).cuda(),
                                        torch.from_numpy(sent).cuda(), torch.from_numpy(wts).cuda(), t, a, Rd,
                                        grad=True, parts=True)
    torch.cuda.synchronize()
    t, a, err, parts, dt, da = (x.cpu().numpy() for x in (t, a, err, parts, dt, da))
    for b in range(B):
        n = tuple(int(v) for v in grids[b])
        hh = (h[b],) * 3
        tr, ar = quadrule.rule_from_outputs(Y[b].astype(np.float64), int(R[b]), h[b])
        assert np.allclose(t[b, :R[b]], tr, rtol=1e-14, atol=0) and np.allclose(a[b, :R[b]], ar, rtol=1e-13, atol=0)
        assert np.all(t[b, R[b]:] == 0)
        t_ref, a_ref = quadrule.reference_rule(h[b])
        ref = quadrule.kernel_values(n, hh, t_ref, a_ref, sent[b])
        e_or = quadrule.judge(n, hh, tr, ar, ref, sent[b], wts[b])
        assert abs(err[b] - e_or) <= 1e-6 * e_or
        ep, eh = quadrule.judge_parts(n, hh, tr, ar, ref, sent[b], wts[b])
        assert abs(parts[b, 0] - ep) <= 1e-6 * ep and abs(parts[b, 1] - eh) <= 1e-6 * eh
        gt, ga = quadrule.judge_grad_fd(n, hh, tr, ar, ref, sent[b], wts[b])
        assert np.linalg.norm(dt[b, :R[b]] - gt) <= 1e-4 * np.linalg.norm(gt)
        assert np.linalg.norm(da[b, :R[b]] - ga) <= 1e-4 * np.linalg.norm(ga)


@pytest.mark.parametrize("n,h", [((24, 20, 16), (1 / 24,) * 3), ((40, 33, 17), (0.025, 0.03, 0.05)),
                                 ((4, 3, 5), (0.2,) * 3)])
def test_certificate_matches_oracle(ctx, n, h):
    """The GPU certificate (weighted sums over every offset) against the
    oracle's exact operator Frobenius-norm errors, plain and theorem-step rules."""
    L = max(n[d] * h[d] for d in range(3))
    hs = tuple(x / L for x in h)
    for t, a in (quadrule.base_rule(12)[:2], quadrule.base_rule(20)[:2],
                 sinc.sinc_nodes(24, step_rule=1, h_min=min(hs))[0::2]):
        got = ctx.quad_certify(n, h, t, a)
        ref = quadrule.certify(n, hs, t, a)
        # both sides form each kernel difference from ~100 FP64 terms of size
        # |K|: an absolute floor of ~1e-15 on the relative error
        assert abs(got[0] - ref[0]) <= 1e-9 * ref[0] + 1e-13, (got, ref)
        assert abs(got[1] - ref[1]) <= 1e-9 * ref[1] + 1e-13, (got, ref)


def test_fit_step_matches_oracle(ctx):
    grids = np.array([[24, 20, 16], [32, 40, 36]], dtype=np.int32)
    R = np.array([16, 21], dtype=np.int32)
    h = 1.0 / grids.max(axis=1)
    rng = np.random.default_rng(4)
    y0 = (0.2 * rng.standard_normal((2, 65))).astype(np.float32)
    ow = [inputs.fit_offsets(tuple(int(v) for v in g)) for g in grids]
    sent = np.stack([o[0] for o in ow])
    wts = np.stack([o[1] for o in ow])
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    y1, t1, a1, e1 = ctx.quad_fit(dev(grids), dev(h), dev(sent), dev(wts), dev(R), dev(y0), iters=1, mu0=1e-2)
    torch.cuda.synchronize()
    y1, t1, a1, e1 = (x.cpu().numpy() for x in (y1, t1, a1, e1))
    for b in range(2):
        n = tuple(int(v) for v in grids[b])
        hh = (h[b],) * 3
        Rb = int(R[b])
        tr, ar = quadrule.reference_rule(h[b])
        ref = quadrule.kernel_values(n, hh, tr, ar, sent[b])
        yb = y0[b].astype(np.float64)
        x0 = np.r_[np.clip(0.45 * np.tanh(yb[:Rb]), -0.44, 0.44), np.clip(np.tanh(yb[32:32 + Rb]), -0.99, 0.99)]
        xo, e_before, e_after = quadrule.lm_step(n, hh, x0, Rb, ref, sent[b], wts[b], 1e-2)
        expect = xo if e_after < e_before else x0
        yg = y1[b].astype(np.float64)
        xg = np.r_[0.45 * np.tanh(yg[:Rb]), np.tanh(yg[32:32 + Rb])]
        assert np.linalg.norm(xg - expect) <= 1e-4 * np.linalg.norm(xo - x0) + 1e-6, b
        # the reported error is the oracle's judge of the returned rule
        e_or = quadrule.judge(n, hh, t1[b, :Rb], a1[b, :Rb], ref, sent[b], wts[b])
        assert abs(e1[b] - e_or) <= 1e-8 * e_or
        assert np.all(t1[b, Rb:] == 0)


def test_fit_lowers_the_error_of_held_out_cases(ctx):
    cases = learned.prepare_cases(64, seed=21, shuffle_seed=22)
    y, t, a, err = ctx.quad_fit(cases["grids"], cases["hmin"], cases["sent"], cases["w"], cases["R"], None, iters=30)
    t0, a0 = ctx.quad_rules(None, cases["R"])
    e0 = ctx.quad_judge(cases["grids"], cases["hmin"], cases["sent"], cases["w"], t0, a0, cases["R"])
    e1 = ctx.quad_judge(cases["grids"], cases["hmin"], cases["sent"], cases["w"], t, a, cases["R"])
    torch.cuda.synchronize()
    err, e0, e1 = (x.cpu().numpy() for x in (err, e0, e1))
    assert np.allclose(err, e1, rtol=1e-9, atol=0)
    assert np.all(err <= e0)
    ratio = err / e0
    gm = float(np.exp(np.mean(np.log(ratio))))
    print(f"fit: geometric mean error ratio fitted/base {gm:.3e}, median {np.median(ratio):.3e}")
    # the fit gains most where the base rule is short of nodes for the grid
    # (the large errors); a quarter of the cases must gain at least 2x
    assert np.quantile(ratio, 0.25) < 0.5
    # one case checked end to end by the oracle
    b = 0
    n = tuple(int(v) for v in cases["n"][b])
    hh = (float(cases["h"][b]),) * 3
    tr, ar = quadrule.reference_rule(hh[0])
    sent = cases["sent"][b].cpu().numpy()
    w = cases["w"][b].cpu().numpy()
    ref = quadrule.kernel_values(n, hh, tr, ar, sent)
    R = int(cases["Rhost"][b])
    tt, aa = t[b, :R].cpu().numpy(), a[b, :R].cpu().numpy()
    assert abs(quadrule.judge(n, hh, tt, aa, ref, sent, w) - err[b]) <= 1e-8 * err[b]
    to, ao = quadrule.rule_from_outputs(y[b].cpu().numpy().astype(np.float64), R, hh[0])
    assert np.allclose(to, tt, rtol=1e-6) and np.allclose(ao, aa, rtol=1e-5)


def test_loss_grad_matches_oracle(ctx):
    rng = np.random.default_rng(8)
    B = 3
    R = np.array([16, 23, 32], dtype=np.int32)
    y = (0.5 * rng.standard_normal((B, 65))).astype(np.float32)
    T = (0.5 * rng.standard_normal((B, 65))).astype(np.float32)
    xf = np.r_[0.4 * np.tanh(rng.standard_normal(32)), 0.9 * np.tanh(rng.standard_normal(32))][None].repeat(B, 0)
    G = rng.standard_normal((B, 64, 64))
    H = (np.einsum("bij,bkj->bik", G, G) * 10.0).astype(np.float32)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    loss, dy = ctx.quad_loss_grad(dev(y), dev(T), dev(xf), dev(H), dev(R), lam=0.1)
    torch.cuda.synchronize()
    loss, dy = loss.cpu().numpy(), dy.cpu().numpy()
    for b in range(B):
        f = lambda v: quadrule.distill_loss(v, float(T[b, 64]), xf[b], H[b], int(R[b]), 0.1)  # noqa: E731
        assert abs(loss[b] - f(y[b])) <= 1e-5 * (1 + abs(f(y[b])))
        fd = np.zeros(65)
        for k in range(65):
            e = np.zeros(65)
            e[k] = 1e-6
            fd[k] = (f(y[b].astype(np.float64) + e) - f(y[b].astype(np.float64) - e)) / 2e-6
        assert np.allclose(dy[b] * B, fd, rtol=1e-4, atol=1e-6 * np.abs(fd).max()), b


@pytest.fixture(scope="module")
def trained(ctx):
    cases = learned.prepare_cases(4096, seed=3)
    learned.fit_targets(ctx, cases, iters=60)
    params, loss = learned.train(ctx, cases, steps=3000, batch=512)
    torch.cuda.synchronize()
    return params, loss


def test_training_learns_the_achievable_error(ctx, trained):
    """The error head predicts, for held-out grids and R', the error a fitted
    R'-node rule reaches: it is what picks R' for a tolerance."""
    params, loss = trained
    assert np.isfinite(loss).all()
    assert loss[-20:].mean() < 0.2 * loss[:5].mean()
    test = learned.prepare_cases(256, seed=11, shuffle_seed=12)
    y, _z, _a = ctx.mlp_forward(params, test["x"])
    _y, _t, _a2, efit = ctx.quad_fit(test["grids"], test["hmin"], test["sent"], test["w"], test["R"], None, 60)
    torch.cuda.synchronize()
    head = y[:, 64].cpu().numpy()
    target = np.log10(efit.cpu().numpy())
    corr = float(np.corrcoef(head, target)[0, 1])
    mae = float(np.mean(np.abs(head - target)))
    print(f"held-out: error head correlation {corr:.3f}, mean abs error {mae:.3f} (log10)")
    assert corr > 0.9 and mae < 0.3


def _apply(ctx, n, m, t=None, a=None, **rule):
    f = ctx.assemble((n, n, n), (1.0 / n,) * 3, t=t, alpha=a, **rule)
    phi, h = ctx.apply_full(f, torch.from_numpy(m).cuda(), prec="fp64")
    torch.cuda.synchronize()
    f.free()
    return phi, h


def _rel(a, b):
    return float((a - b).norm() / b.norm())


@pytest.mark.parametrize("n", [128, 256])
def test_certificate_bounds_the_field_error(ctx, trained, n):
    """Each rule's certified operator errors against the measured relative L2
    errors of its FP64 apply against the reference rule's (the certificate's
    reference, 96 nodes), on the vortex and on a random unit field: the
    vortex errors stay below the certificate and the random-field errors,
    whose expectation the certificate is, within 10 % above it.  The plain
    M = 40 rule is rejected at 256^3 (its near-cell error), accepted at 128^3."""
    params, _loss = trained
    h = 1.0 / n
    fields = {"vortex": inputs.vortex_field(n, seed=0), "random": inputs.random_unit_field(n, seed=1)}
    tr, ar = quadrule.reference_rule(h)
    refs = {k: _apply(ctx, n, m, t=tr, a=ar) for k, m in fields.items()}
    rules = {"c0 M=40": quadrule.base_rule(40)[:2], "c0 M=28": quadrule.base_rule(28)[:2],
             "theorem M=64": sinc.sinc_nodes(64, step_rule=1, h_min=h)[0::2]}
    r = learned.predict(ctx, params, (n, n, n), 1e-6)
    rules["learned"] = (r["t"], r["alpha"])
    certs = {}
    for name, (t, a) in rules.items():
        cp, ch = ctx.quad_certify((n, n, n), (h,) * 3, t, a)
        certs[name] = (cp, ch)
        for fk, m in fields.items():
            phi, hf = _apply(ctx, n, m, t=np.asarray(t), a=np.asarray(a))
            ep, eh = _rel(phi, refs[fk][0]), _rel(hf, refs[fk][1])
            print(f"{n}^3 {name:12s} certified phi {cp:.2e} h {ch:.2e} | {fk} measured phi {ep:.2e} h {eh:.2e}")
            slack = 1.0 if fk == "vortex" else 1.1
            assert ep <= slack * cp and eh <= slack * ch, (name, fk)
    plain = max(certs["c0 M=40"])
    assert (plain > 1e-6) if n == 256 else (plain < 1e-6)


@pytest.fixture(scope="module")
def gain(ctx, trained):
    params, _loss = trained
    n = (128, 128, 128)
    out = {mode: learned.predict(ctx, params, n, 1e-6, mode=mode)
           for mode in ("network", "network_proposal", "search")}
    # plain sinc rules (c0 = 2.15): the fewest nodes certified within 1e-6
    plain = None
    for M in range(24, 41):
        t, a, _ = quadrule.base_rule(M)
        if max(ctx.quad_certify(n, (1 / 128,) * 3, t, a)) <= 1e-6:
            plain = M
            break
    return out, plain


def test_learned_rule_needs_fewer_nodes_than_plain_sinc(ctx, gain):
    """At 128^3 and a certified 1e-6 the learned rule needs at most 0.8x the
    nodes of the plain sinc rule (reading: the node count sets the apply's
    work linearly, so 0.8x is a 1.25x shorter apply)."""
    out, plain = gain
    r = out["network"]
    print("plain sinc nodes for 1e-6 at 128^3:", plain)
    for mode, rr in out.items():
        print(mode, {k: v for k, v in rr.items() if k not in ("t", "alpha")})
    assert plain is not None
    assert not r["fell_back"] and r["accuracy_met"] and r["judged"] <= 1e-6
    assert r["R"] <= 0.8 * plain


def test_mixed_learned_apply_against_exact_collocation(ctx, gain):
    """The mixed form at 128^3: the learned rule (certified within 1e-6) with
    BF16x3 products, for a uniform magnetization, at every cell against the
    exact collocated potential and field of the cube (closed-form box
    kernels of the whole cube at the cell centres).  The FP64 apply with the
    same rule shows the rule's own error, which its certificate bounds for
    the operator; the BF16x3 apply adds its rounding and stays within the
    1e-6 target."""
    from oracle import exact
    r = gain[0]["network"]
    n = 128
    f = ctx.assemble((n, n, n), (1 / n,) * 3, t=r["t"], alpha=r["alpha"])
    mv = np.array([0.3, -0.5, 0.8])
    m = mv[:, None, None, None] * np.ones((3, n, n, n))
    c = (np.arange(n) + 0.5) / n
    pts = np.stack(np.meshgrid(c, c, c, indexing="ij")[::-1], axis=-1)
    K, N = exact.box_kernels_at_points(pts, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    pe, he = np.tensordot(mv, K, axes=1), -np.tensordot(N, mv, axes=([1], [0]))
    errs = {}
    for prec, dt in (("fp64", torch.float64), ("bf16x3", torch.float32)):
        phi, hf = ctx.apply_full(f, torch.from_numpy(m).to(device="cuda", dtype=dt), prec=prec)
        torch.cuda.synchronize()
        p, h = phi.double().cpu().numpy(), hf.double().cpu().numpy()
        errs[prec] = (np.linalg.norm(p - pe) / np.linalg.norm(pe), np.linalg.norm(h - he) / np.linalg.norm(he))
    print(f"learned rule R' = {r['R']} (certified {r['judged']:.2e}) vs exact collocation, uniform 128^3:", errs)
    assert max(errs["fp64"]) <= r["judged"]
    assert max(errs["bf16x3"]) < 1e-6


def test_network_versus_search_without_network(ctx, gain):
    """Ablation.  Without the network, bisection over R' finds the smallest
    fitted rule; the network's error head lands within 2 nodes of it with
    fewer fits.  Both certified within tol."""
    out, _plain = gain
    net, search = out["network"], out["search"]
    assert search["accuracy_met"] and not search["fell_back"]
    assert net["R"] <= search["R"] + 2
    assert net["fits"] < search["fits"]


def test_network_proposal_is_no_better_start(ctx, trained):
    """Ablation of the proposed nodes and weights, on held-out cases: fits
    started from the network's outputs end above fits started from the plain
    rule (geometric mean of the error ratio > 1 at every iteration count
    measured): the proposals are no warm start, so the default mode fits
    from the plain rule and the network contributes its error head."""
    params, _loss = trained
    test = learned.prepare_cases(256, seed=11, shuffle_seed=12)
    y, _z, _a = ctx.mlp_forward(params, test["x"])
    for it in (0, 20, 60):
        _y, _t, _a2, e_net = ctx.quad_fit(test["grids"], test["hmin"], test["sent"], test["w"], test["R"], y, it)
        _y, _t, _a2, e_pl = ctx.quad_fit(test["grids"], test["hmin"], test["sent"], test["w"], test["R"], None, it)
        torch.cuda.synchronize()
        r = (e_net / e_pl).cpu().numpy()
        gm = float(np.exp(np.mean(np.log(r))))
        print(f"{it} LM iterations: error from the proposal / from the plain rule, geometric mean {gm:.2f}, "
              f"better in {np.mean(r < 1):.0%} of the cases")
        assert gm > 1.0


def test_predict_and_fallback(ctx, trained):
    params, _loss = trained
    r = learned.predict(ctx, params, (48, 64, 40), 1e-6)
    print("predict 48x64x40 at 1e-6:", {k: v for k, v in r.items() if k not in ("t", "alpha")})
    assert not r["fell_back"] and 16 <= r["R"] <= 32 and r["judged"] <= 1e-6
    # unattainable with R' <= 32: the theorem-step rule with the fewest nodes
    # in 33..64 that meets it
    r2 = learned.predict(ctx, params, (48, 64, 40), 1e-13)
    R2 = r2["R"]
    assert r2["fell_back"] and 33 <= R2 <= 64 and r2["judged"] <= 1e-13 and r2["accuracy_met"]
    # the returned fallback rule is the oracle's theorem-step rule with R2
    # nodes, its certificate is its own, and one node fewer misses the tolerance
    h = 1.0 / 64
    t, a = sinc.sinc_nodes(R2, step_rule=1, h_min=h)[0::2]
    assert np.allclose(r2["t"][:R2], t, rtol=1e-15) and np.allclose(r2["alpha"][:R2], a, rtol=1e-14)
    cp, ch = ctx.quad_certify((48, 64, 40), (h,) * 3, t, a)
    assert abs(r2["err_phi"] - cp) <= 1e-9 * cp + 1e-13 and abs(r2["err_h"] - ch) <= 1e-9 * ch + 1e-13
    if R2 > 33:
        t1, a1 = sinc.sinc_nodes(R2 - 1, step_rule=1, h_min=h)[0::2]
        assert max(ctx.quad_certify((48, 64, 40), (h,) * 3, t1, a1)) > 1e-13
    print("fallback at 1e-13:", R2, "nodes")
    # below the certificate's FP64 floor nothing qualifies: DEMAG_E_ACCURACY,
    # with the fallback rule returned
    r3 = learned.predict(ctx, params, (48, 64, 40), 1e-17)
    assert r3["fell_back"] and r3["R"] == 64 and not r3["accuracy_met"] and r3["judged"] > 1e-17
    with pytest.raises(api.DemagError):
        ctx.quad_predict(params, (32, 32, 16), (0.1, 0.1, 0.2), 1e-6)   # non-cubic cells
