"""The allocation-free structured apply, called through the C ABI, against
demag_apply_columns on the same inputs: the same kernels on the same data,
so the outputs must be bit-identical (integer comparison of the FP32 words).
Two calls in a row on the shared static scratch, the second with a smaller
input, then the size and preparation checks."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_1212_3509_amd import api, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    api.library()
    return api.Context(0)


def _cols(n, R, seed):
    rng = np.random.default_rng(seed)
    return [torch.from_numpy(rng.uniform(-1, 1, (3, R[d], n[d])).astype(np.float32)).cuda() for d in range(3)]


def _noalloc(ctx, f, cols):
    R = [int(c.shape[1]) for c in cols]
    out = [torch.full((3, 2, f.M, R[d], f.n[d]), float("nan"), dtype=torch.float32, device="cuda") for d in range(3)]
    ctx.use_current_stream()
    st = api.library().demag_apply_columns_noalloc(ctx.handle, f.handle, (C.c_int32 * 3)(*R), ctx._ptr3(cols),
                                                   ctx._ptr3(out))
    return st, out


def test_noalloc_matches_columns_twice(ctx):
    cases = [((4096, 4096, 4096), (10, 10, 10), 40, 1), ((300, 200, 97), (2, 3, 1), 12, 2)]
    for n, R, M, seed in cases:
        print(f"no-alloc case n={n} R={R} M={M}", flush=True)
        f = ctx.assemble(n, tuple(1.0 / max(n) for _ in range(3)), M=M)
        ctx.prepare_structured(f)
        cols = _cols(n, R, seed)
        st, got = _noalloc(ctx, f, cols)
        assert st == 0, api.library().demag_last_error()
        ref = ctx.apply_columns(f, cols)
        torch.cuda.synchronize()
        for g, r in zip(got, ref):
            assert torch.equal(g.view(torch.int32), r.view(torch.int32))
        del got, ref


def test_noalloc_rejects_oversize_and_unprepared(ctx):
    n = (4096, 4096, 4096)
    f = ctx.assemble(n, (1.0 / 4096,) * 3, M=4)
    # spectra not prepared yet: rejected before anything is enqueued
    cols = _cols((8, 8, 8), (1, 1, 1), 3)
    R = (C.c_int32 * 3)(1, 1, 1)
    st = api.library().demag_apply_columns_noalloc(ctx.handle, f.handle, R, ctx._ptr3(cols), ctx._ptr3(cols))
    assert st == 1 and b"demag_prepare_structured" in api.library().demag_last_error()
    ctx.prepare_structured(f)
    # 3 * 400 columns of 4097 complex FP64 points exceed the 64 MiB array
    big = (C.c_int32 * 3)(400, 0, 0)
    st = api.library().demag_apply_columns_noalloc(ctx.handle, f.handle, big, ctx._ptr3(cols), ctx._ptr3(cols))
    assert st == 1 and b"static scratch" in api.library().demag_last_error()
