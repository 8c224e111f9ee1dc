"""GPU test of lrhe_matmul_fast_noalloc, the fast path for callers that cannot
allocate device memory: through the C ABI, its output ciphertexts must equal
lrhe_matmul_fast's (caller workspace) bit for bit, on two calls in a row (the
second with a smaller job, over the scratch contents the first one left), with
no library allocation in the call, and a job above the fixed scratch must be
refused with EINVAL."""
import ctypes
import sys

import numpy as np
import pytest

import workloads as WL
from oracle import oracle as O

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-noalloc]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    return torch


@pytest.fixture(scope="module")
def P(torch):
    import paper_2204_05496_amd as pkg
    pkg.native.lib()
    return pkg


def noalloc(P, ctx, keys, model, xct, rows, y):
    N = P.native
    return N.lib().lrhe_matmul_fast_noalloc(ctx.h, keys.gk, model.handle, N.ptr(xct), rows, N.ptr(y),
                                            P.bfv._stream())


def test_noalloc_equals_workspace_path(P, torch):
    N = P.native
    p = WL.PARAMS["n16k"]
    say("setup n16k")
    ctx = P.Context.from_params(p, device=0)
    keys = ctx.keygen(2024)
    jobs = [WL.single(f=40000),                                              # 16 pairs, 81 MiB of scratch
            WL.make("single_20000x8", "n16k", 1, 20000, 8, 0.01, WL.BASE_SEED + 21)]   # 8 pairs
    for k, wl in enumerate(jobs):
        say("job", wl.name, wl.rows, "x", wl.f, "x", wl.classes)
        model = ctx.model(wl.W, wl.b)
        xct = ctx.encrypt_rows(keys, wl.X, seed=40 + k)
        nout = -(-wl.rows * wl.classes // ctx.n)
        ref = ctx.matmul_fast(keys, model, xct, wl.rows, out=ctx.empty_ct(nout))
        y = ctx.empty_ct(nout)
        y.fill_(0x5A5A5A5A)
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        # the k-th library allocation from now would fail: the call must make none
        prev = N.lib().lrhe_fault_inject(1)
        try:
            rc = noalloc(P, ctx, keys, model, xct, wl.rows, y)
            armed = N.lib().lrhe_fault_inject(-1)
        finally:
            N.lib().lrhe_fault_inject(max(prev, 0))
        assert rc == 0, N.lib().lrhe_last_error()
        assert armed == 1, "the non-allocating call made a library allocation"
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
        assert torch.equal(y, ref), f"{wl.name}: noalloc output differs from the workspace path"
        S, budget = ctx.scores_fast(keys, y, wl.rows, wl.classes)
        assert np.array_equal(S, O.plain_scores(wl.X, wl.W, wl.b, p.t)) and budget > 0


def test_noalloc_refuses_oversize_then_runs(P, torch):
    N = P.native
    p = WL.PARAMS["n16k"]
    ctx = P.Context.from_params(p, device=0)
    keys = ctx.keygen(2024)
    big = WL.make("rows2_40000x16", "n16k", 2, 40000, 16, 0.01, WL.BASE_SEED + 22)   # 32 pairs: 162 MiB
    model = ctx.model(big.W, big.b)
    xct = ctx.encrypt_rows(keys, big.X, seed=50)
    y = ctx.empty_ct(1)
    say("oversize job")
    rc = noalloc(P, ctx, keys, model, xct, big.rows, y)
    assert rc == N.LRHE_EINVAL
    assert b"scratch" in N.lib().lrhe_last_error()
    # one row of the same job fits and matches the workspace path
    ref = ctx.matmul_fast(keys, model, xct, 1, out=ctx.empty_ct(1))
    assert noalloc(P, ctx, keys, model, xct, 1, y) == 0, N.lib().lrhe_last_error()
    torch.cuda.synchronize()
    assert torch.equal(y, ref)


def test_noalloc_small_ring_after_large(P, torch):
    """A context of another ring dimension on the same GPU shares the scratch:
    n = 4096 with 3 data primes after the n = 16384 jobs, two calls in a row."""
    p = WL.PARAMS["tiny3"]
    ctx = P.Context.from_params(p, device=0)
    keys = ctx.keygen(77)
    for k, (rows, f) in enumerate([(40, 5000), (3, 900)]):
        wl = WL.make(f"tiny3_{rows}x{f}", "tiny3", rows, f, 4, 0.02, WL.BASE_SEED + 30 + k)
        model = ctx.model(wl.W, wl.b)
        xct = ctx.encrypt_rows(keys, wl.X, seed=60 + k)
        nout = -(-rows * 4 // ctx.n)
        ref = ctx.matmul_fast(keys, model, xct, rows, out=ctx.empty_ct(nout))
        y = ctx.empty_ct(nout)
        assert noalloc(P, ctx, keys, model, xct, rows, y) == 0, P.native.lib().lrhe_last_error()
        torch.cuda.synchronize()
        assert torch.equal(y, ref), (rows, f)
