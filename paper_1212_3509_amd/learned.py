"""Training and use of the shortened-rule network through the C ABI.

Only marshalling: the cases come from ``inputs`` (seeded), every forward,
backward, judge and update step runs in the library's kernels.
"""
from __future__ import annotations

import numpy as np

from . import inputs

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
    sent = np.stack([inputs.sentinel_offsets(tuple(v)) for v in n])
    dev = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dt)  # noqa: E731
    return {"x": dev(x, torch.float32), "grids": dev(n, torch.int32), "hmin": dev(h, torch.float64),
            "R": dev(R, torch.int32), "sent": dev(sent, torch.int32), "n": n, "h": h, "log10_tol": tol,
            "Rhost": R}


def train(ctx, cases, steps: int = 2000, batch: int = 1024, lr: float = 2e-3, lam: float = 0.1,
          init_seed: int = 4):
    """Fresh network trained on ``cases``; returns (params, loss history)."""
    import torch
    p = torch.from_numpy(inputs.mlp_init(seed=init_seed, out_scale=0.0)).cuda()
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    loss = ctx.quad_train(p, m, v, cases["x"], cases["grids"], cases["hmin"], cases["R"], cases["sent"],
                          steps, min(batch, int(cases["x"].shape[0])), 0, lr, lam)
    return p, loss


def predict(ctx, params, n, tol: float):
    """Shortened rule for grid n (unit longest edge, cubic cells) at tol."""
    import torch
    nmax = max(n)
    h = 1.0 / nmax
    x = inputs.quad_features(np.tile(np.asarray(n)[None], (len(RPRIME), 1)), np.full(len(RPRIME), h),
                             np.full(len(RPRIME), np.log10(tol)), np.array(RPRIME))
    sent = torch.from_numpy(inputs.sentinel_offsets(tuple(n))).to(device="cuda", dtype=torch.int32)
    return ctx.quad_predict(params, torch.from_numpy(x).cuda(), tuple(n), h, sent, tol)
