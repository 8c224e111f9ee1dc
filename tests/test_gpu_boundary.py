"""GPU tests of the C ABI's failure handling and client calls: allocation
faults forced from the host (LRHE_EDEVICE / LRHE_ENOMEM, then the next call
succeeds), the debug decryption that reports exhausted noise (LRHE_ENOISE),
server submission ordered by a producer stream, and the release of finished
server requests.  No test makes a kernel fail: every fault is injected on the
host before any launch."""
import ctypes
import gc
import sys
import time

import numpy as np
import pytest

import workloads as WL
from oracle import oracle as O

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-boundary]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def P(torch):
    import paper_2204_05496_amd as pkg
    pkg.native.lib()
    return pkg


@pytest.fixture(scope="module")
def tiny3(P):
    p = WL.PARAMS["tiny3"]
    ctx = P.Context.from_params(p, device=0)
    return p, ctx, ctx.keygen(4321)


def test_allocation_fault_then_recovery(tiny3, P, torch):
    p, ctx, keys = tiny3
    lib, N = P.native.lib(), P.native
    wl = WL.tiny(params="tiny3")
    try:
        say("model create under an armed fault")
        lib.lrhe_fault_inject(1)
        with pytest.raises(N.LrheError) as ei:
            ctx.model(wl.W, wl.b)
        assert ei.value.code == N.LRHE_EDEVICE
        assert lib.lrhe_fault_inject(-1) == 0            # spent
        model = ctx.model(wl.W, wl.b)                    # the next call succeeds
        # the third allocation of a model (its bias table) fails: nothing half-built survives
        lib.lrhe_fault_inject(3)
        with pytest.raises(N.LrheError) as ei:
            ctx.model(wl.W, wl.b)
        assert ei.value.code == N.LRHE_EDEVICE
        say("keygen under an armed fault")
        lib.lrhe_fault_inject(1)
        with pytest.raises(N.LrheError) as ei:
            ctx.keygen(99)
        assert ei.value.code == N.LRHE_EDEVICE
        keys2 = ctx.keygen(99)
        say("server and batch under an armed fault")
        lib.lrhe_fault_inject(2)
        with pytest.raises(N.LrheError) as ei:
            P.Server(ctx, keys, hbm_budget=64 << 20)
        assert ei.value.code == N.LRHE_ENOMEM
        srv = P.Server(ctx, keys, hbm_budget=64 << 20)
        xct = ctx.encrypt_rows(keys, wl.X, seed=3)
        y = ctx.empty_ct(1)
        lib.lrhe_fault_inject(1)
        with pytest.raises(N.LrheError) as ei:
            P.Batch(ctx, keys, [(xct, wl.rows, model, y)])
        assert ei.value.code == N.LRHE_EDEVICE
        b = P.Batch(ctx, keys, [(xct, wl.rows, model, y)])
        b.run()
        rid = srv.submit(model, xct, wl.rows, ctx.empty_ct(1))
        srv.drain()
        assert srv.poll(rid)[0]
        S, budget = ctx.scores_fast(keys, y, wl.rows, wl.classes)
        assert np.array_equal(S, O.plain_scores(wl.X, wl.W, wl.b, p.t)) and budget > 0
        srv.close()
        keys2.close()
    finally:
        lib.lrhe_fault_inject(0)


def test_decrypt_check_flags_exhausted_noise(P, torch):
    """On the two-prime tiny parameters the one-hot mask exhausts the noise budget
    (the reading the oracle pins): the debug decryption given the expected
    plaintext returns LRHE_ENOISE.  With three primes the same job decrypts and
    the check passes."""
    for pname, ok in (("tiny3", True), ("tiny", False)):
        p = WL.PARAMS[pname]
        ctx = P.Context.from_params(p, device=0)
        keys = ctx.keygen(1234)
        wl = WL.tiny(params=pname)
        xct = ctx.encrypt_rows(keys, wl.X, seed=99)
        y = ctx.matmul_fast(keys, ctx.model(wl.W, wl.b), xct, wl.rows)
        exp = np.zeros((1, p.n), dtype=np.int64)
        exp[0, :wl.rows * wl.classes] = O.plain_scores(wl.X, wl.W, wl.b, p.t).reshape(-1)
        say(pname, "decrypt_check")
        if ok:
            bud = ctx.decrypt_check(keys, y, exp)
            assert bud[0] > 0
        else:
            with pytest.raises(P.native.LrheError) as ei:
                ctx.decrypt_check(keys, y, exp)
            assert ei.value.code == P.native.LRHE_ENOISE


def test_server_waits_for_producer_stream(tiny3, P, torch):
    """Encryption queued on a side stream, the request submitted right after it
    with that stream current and no synchronisation: the server's tile waits for
    the encryption, and the output equals the request run alone."""
    p, ctx, keys = tiny3
    wl = WL.make("stream", "tiny3", 6, 5000, 16, 0.02, WL.BASE_SEED + 21)
    model = ctx.model(wl.W, wl.b)
    alone = ctx.matmul_fast(keys, model, ctx.encrypt_rows(keys, wl.X, seed=44), wl.rows)
    torch.cuda.synchronize()
    srv = P.Server(ctx, keys, hbm_budget=256 << 20)
    side = torch.cuda.Stream()
    Xd = torch.from_numpy(wl.X).cuda()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        xct = ctx.empty_ct(wl.rows * ctx.K(wl.f))
        xct.fill_(0)
        y = ctx.empty_ct(1)
        ctx.encrypt_rows(keys, Xd, seed=44, out=xct)
        rid = srv.submit(model, xct, wl.rows, y)
    srv.drain()
    assert srv.poll(rid)[0]
    torch.cuda.synchronize()
    assert torch.equal(y, alone)
    srv.close()


def test_server_release_returns_memory(tiny3, P, torch):
    """Finished requests are forgotten on release: the server holds no record and
    the binding no buffer of them, so device memory returns to its level before."""
    p, ctx, keys = tiny3
    wl = WL.tiny(params="tiny3")
    model = ctx.model(wl.W, wl.b)
    srv = P.Server(ctx, keys, hbm_budget=256 << 20)
    gc.collect()                                   # leftovers of earlier tests
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    for round_ in range(3):
        ids = []
        for k in range(20):
            xct = ctx.encrypt_rows(keys, wl.X, seed=100 + k)
            ids.append(srv.submit(model, xct, wl.rows, ctx.empty_ct(1)))
            del xct
        srv.drain()
        assert srv.stats()["held"] == 20
        for rid in ids:
            assert srv.poll(rid)[0]
            srv.release(rid)
        with pytest.raises(P.native.LrheError):
            srv.poll(ids[0])                       # forgotten
        assert srv.stats()["held"] == 0
        gc.collect()
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == base, round_
    srv.close()
