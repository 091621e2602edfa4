"""Training and use of the shortened-rule network through the C ABI.

Only marshalling: the cases come from ``inputs`` (seeded); every fit,
forward, backward, judge and update step runs in the library's kernels.
"""
from __future__ import annotations

import numpy as np

from . import api, inputs

RPRIME = tuple(range(16, 33))


def prepare_cases(count: int = 20000, seed: int = 3, shuffle_seed: int = 5):
    """Device tensors of the training cases in a seeded shuffled order:
    x [B][6] f32, grids [B][3] i32, hmin [B] f64, R [B] i32, sentinels [B][S][3] i32."""
    import torch
    cases = inputs.quad_training_cases(count, seed=seed)
    order = np.random.default_rng(shuffle_seed).permutation(count)
    n = cases["n"][order]
    h = cases["h"][order]
    tol = cases["log10_tol"][order]
    R = cases["rprime"][order]
    x = inputs.quad_features(n, h, tol, R)
    # the judge's offsets and weights per grid, from the library (the same
    # recipe as inputs.fit_offsets, checked against it by the CPU tests)
    ow = [api.quad_offsets(tuple(int(c) for c in v)) for v in n]
    sent = np.stack([o[0] for o in ow])
    wts = np.stack([o[1] for o in ow])
    dev = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dt)  # noqa: E731
    return {"x": dev(x, torch.float32), "grids": dev(n, torch.int32), "hmin": dev(h, torch.float64),
            "R": dev(R, torch.int32), "sent": dev(sent, torch.int32), "w": dev(wts, torch.float64), "n": n, "h": h,
            "log10_tol": tol, "Rhost": R}


def fit_targets(ctx, cases, iters: int = 60, chunk: int = 4096, with_h: bool = False):
    """Levenberg-Marquardt fits of every case (the training targets), in
    chunks; adds "targets" [count][65] (fitted outputs, slot 64 = log10 of the
    fitted error) and "fit_err" [count], and with_h also "xfit" [count][64]
    and "H" [count][64][64] for the distillation loss."""
    import torch
    count = int(cases["x"].shape[0])
    out = {"targets": [], "fit_err": []}
    if with_h:
        out.update({"xfit": [], "H": []})
    for a in range(0, count, chunk):
        b = min(count, a + chunk)
        r = ctx.quad_fit(cases["grids"][a:b], cases["hmin"][a:b], cases["sent"][a:b], cases["w"][a:b],
                         cases["R"][a:b], None, iters, want_h=with_h)
        out["targets"].append(r[0])
        out["fit_err"].append(r[3])
        if with_h:
            out["xfit"].append(r[4])
            out["H"].append(r[5])
    for k, v in out.items():
        cases[k] = torch.cat(v)
    return cases


def train(ctx, cases, steps: int = 4000, batch: int = 512, lr: float = 1e-3, lam: float = 0.1,
          init_seed: int = 4, distill_steps: int = 0, distill_lr: float = 1e-4):
    """Fresh network trained on the fits of ``cases``: squared errors against
    the fitted outputs and log10 errors, then optionally ``distill_steps``
    on the Gauss-Newton distillation loss.  Returns (params, loss history)."""
    import numpy as np
    import torch
    if "targets" not in cases or (distill_steps and "H" not in cases):
        fit_targets(ctx, cases, with_h=distill_steps > 0)
    p = torch.from_numpy(inputs.mlp_init(seed=init_seed, out_scale=0.0)).cuda()
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    bs = min(batch, int(cases["x"].shape[0]))
    loss = ctx.quad_train(p, m, v, cases["x"], cases["targets"], cases["R"], steps, bs, 0, lr, lam)
    if distill_steps:
        loss2 = ctx.quad_train(p, m, v, cases["x"], cases["targets"], cases["R"], distill_steps, bs, steps,
                               distill_lr, lam, xfit=cases["xfit"], H=cases["H"])
        loss = np.concatenate([loss, loss2])
    return p, loss


def predict(ctx, params, n, tol: float, fit_iters: int = 200, mode: str = "network"):
    """Shortened rule for grid n (unit longest edge, cubic cells) at tol; the
    library computes the network's inputs and the fit's offsets itself."""
    return ctx.quad_predict(params, tuple(int(v) for v in n), 1.0 / max(n), tol, fit_iters, mode)
