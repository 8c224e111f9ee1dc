"""GPU tests of batched and served execution of Algorithm 1 (many requests).

Each request's output ciphertexts must be bit-identical to the single-request
path and to the oracle, whether the request runs alone, in a planned batch
(eager or replayed from a hipGraph), or in the continuous-batching server mixed
with other requests.  Tolerance: none.
"""
import sys
import time

import numpy as np
import pytest

import workloads as WL
from oracle import oracle as O

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-batch]", *a, flush=True)
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


def coeff(ctx, t):
    from paper_2204_05496_amd import to_numpy_u32
    return to_numpy_u32(ctx.to_coeff(t)).astype(np.uint64)


def make_requests(ctx, keys, specs, seed0, params):
    """specs: (rows, f, classes); each request has its own model and encryption seed."""
    reqs = []
    for k, (rows, f, classes) in enumerate(specs):
        wl = WL.make(f"r{k}", params, rows, f, classes, 0.02, seed0 + 17 * k)
        xct = ctx.encrypt_rows(keys, wl.X, seed=seed0 + k)
        model = ctx.model(wl.W, wl.b)
        reqs.append((wl, xct, model))
    return reqs


@pytest.fixture(scope="module")
def tiny_setup(P):
    p = WL.PARAMS["tiny"]
    ctx = P.Context.from_params(p, device=0)
    ctx.tune_set("tile", 64)   # small tiles: requests straddle tiles and groups split there
    keys = ctx.keygen(1234)
    specs = [(1, 256, 4), (3, 5000, 16), (7, 9000, 4), (2, 100, 16), (5, 4096, 8)]
    reqs = make_requests(ctx, keys, specs, 500, "tiny")
    alone = []
    for wl, xct, model in reqs:
        alone.append(coeff(ctx, ctx.matmul_fast(keys, model, xct, wl.rows)))
    return p, ctx, keys, reqs, alone


def test_batch_matches_alone_and_oracle(tiny_setup, P, torch):
    p, ctx, keys, reqs, alone = tiny_setup
    ys = [ctx.empty_ct(-(-wl.rows * wl.classes // ctx.n)) for wl, _, _ in reqs]
    b = P.Batch(ctx, keys, [(xct, wl.rows, model, y) for (wl, xct, model), y in zip(reqs, ys)])
    say("batch pairs", b.npairs, "tile", b.tile, "groups", b.ngroups)
    b.run()
    torch.cuda.synchronize()
    for k, y in enumerate(ys):
        assert np.array_equal(coeff(ctx, y), alone[k]), f"request {k}"
    # oracle on two of them
    o = O.Oracle(p.n, list(p.q), p.P, p.t)
    ko = o.keygen(1234)
    for k in (1, 3):
        wl = reqs[k][0]
        xo = o.encrypt_rows(ko, wl.X, seed=500 + k)
        ref = o.fast_matmul(ko, xo, o.encode_weights(wl.W), wl.b)
        assert np.array_equal(alone[k], ref), f"request {k} vs oracle"


def test_batch_graph_replays(tiny_setup, P, torch):
    """Replays of the captured graph, with eager library work on the device in
    between, each equal the eager result."""
    p, ctx, keys, reqs, alone = tiny_setup
    ys = [ctx.empty_ct(-(-wl.rows * wl.classes // ctx.n)) for wl, _, _ in reqs]
    b = P.Batch(ctx, keys, [(xct, wl.rows, model, y) for (wl, xct, model), y in zip(reqs, ys)])
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        b.capture(side)
    side.synchronize()
    wl0, xct0, m0 = reqs[0]
    for rep in range(3):
        for y in ys:
            y.fill_(0)
        torch.cuda.synchronize()
        b.run()
        other = ctx.matmul_fast(keys, m0, xct0, wl0.rows)   # eager work between replays
        torch.cuda.synchronize()
        for k, y in enumerate(ys):
            assert np.array_equal(coeff(ctx, y), alone[k]), f"replay {rep} request {k}"
        assert np.array_equal(coeff(ctx, other), alone[0])


def test_server_mix_equals_alone(tiny_setup, P, torch):
    p, ctx, keys, reqs, alone = tiny_setup
    srv = P.Server(ctx, keys, hbm_budget=2 << 30)
    ys = []
    ids = []
    for k, (wl, xct, model) in enumerate(reqs):
        y = ctx.empty_ct(-(-wl.rows * wl.classes // ctx.n))
        ys.append(y)
        rid = srv.submit(model, xct, wl.rows, y)
        assert rid is not None
        ids.append(rid)
        time.sleep(0.001 * k)
    srv.drain()
    for k, rid in enumerate(ids):
        done, lat = srv.poll(rid)
        assert done and lat > 0
        assert np.array_equal(coeff(ctx, ys[k]), alone[k]), f"request {k}"
    st = srv.stats()
    assert st["pairs"] == sum(wl.rows * wl.classes for wl, _, _ in reqs)
    srv.close()


def test_batch_and_server_digit_halves(tiny_setup, P, torch):
    """The small-tile key-switch variant with the digits of each item split over
    two workgroups, in a planned batch and in the server: every output equals
    the request run alone with the default choices."""
    p, ctx, keys, reqs, alone = tiny_setup
    before = ctx.tuning()
    ctx.tune_set("small_below", 1024)   # every tile of 64 pairs in the small class
    ctx.tune_set("small.mac_mode", P.native.MAC_MODE_HALF)
    try:
        ys = [ctx.empty_ct(-(-wl.rows * wl.classes // ctx.n)) for wl, _, _ in reqs]
        b = P.Batch(ctx, keys, [(xct, wl.rows, model, y) for (wl, xct, model), y in zip(reqs, ys)])
        b.run()
        torch.cuda.synchronize()
        for k, y in enumerate(ys):
            assert np.array_equal(coeff(ctx, y), alone[k]), f"batch request {k}"
        srv = P.Server(ctx, keys, hbm_budget=2 << 30)
        ys2, ids = [], []
        for wl, xct, model in reqs:
            y = ctx.empty_ct(-(-wl.rows * wl.classes // ctx.n))
            ys2.append(y)
            ids.append(srv.submit(model, xct, wl.rows, y))
        srv.drain()
        for k, y in enumerate(ys2):
            assert srv.poll(ids[k])[0]
            assert np.array_equal(coeff(ctx, y), alone[k]), f"server request {k}"
        srv.close()
    finally:
        ctx.tune_set("small.mac_mode", before["small"]["mac_mode"])
        ctx.tune_set("small_below", before["small_below"])


def test_server_admission_by_memory(tiny_setup, P, torch):
    p, ctx, keys, reqs, alone = tiny_setup
    ctb = 2 * ctx.L * ctx.n * 4
    wl, xct, model = reqs[4]          # 5 x 8 = 40 pairs
    srv = P.Server(ctx, keys, hbm_budget=ctb * 8)   # room for one such request's partials
    y1, y2 = ctx.empty_ct(1), ctx.empty_ct(1)
    r1 = srv.submit(model, xct, wl.rows, y1)
    assert r1 is not None
    r2 = srv.submit(model, xct, wl.rows, y2)      # arrives while r1 holds the arena
    assert r2 is None
    srv.drain()
    r2 = srv.submit(model, xct, wl.rows, y2)
    assert r2 is not None
    srv.drain()
    assert np.array_equal(coeff(ctx, y1), alone[4]) and np.array_equal(coeff(ctx, y2), alone[4])
    with pytest.raises(P.native.LrheError):        # larger than the whole budget
        srv.submit(reqs[1][2], reqs[1][1], reqs[1][0].rows * 40, ctx.empty_ct(1))
    srv.close()


def test_uneven_requests_n16k_scores(P, torch):
    """Requests shaped like the uneven-batching workload (rows and features vary),
    one launch: bit-identical to each request alone; scores equal X W + b mod t."""
    p = WL.PARAMS["n16k"]
    ctx = P.Context.from_params(p, device=0)
    keys = ctx.keygen(77)
    specs = [(1, 10000, 16), (5, 40000, 16), (33, 23000, 16), (2, 16384, 16), (17, 31000, 16), (64, 12000, 16)]
    reqs = make_requests(ctx, keys, specs, 900, "n16k")
    ys = [ctx.empty_ct(1) for _ in reqs]
    b = P.Batch(ctx, keys, [(xct, wl.rows, model, y) for (wl, xct, model), y in zip(reqs, ys)])
    b.run()
    torch.cuda.synchronize()
    for k, (wl, xct, model) in enumerate(reqs):
        alone = ctx.matmul_fast(keys, model, xct, wl.rows)
        assert torch.equal(alone, ys[k]), f"request {k}"
        S, budget = ctx.scores_fast(keys, ys[k], wl.rows, wl.classes)
        assert np.array_equal(S, O.plain_scores(wl.X, wl.W, wl.b, p.t)) and budget > 50


def test_two_clients_batch_and_server(P, torch):
    """Requests of two clients (two key sets) share tiles in a batch and in the
    server: each output equals that client's request run alone, and decrypts
    under that client's secret key to X W + b mod t."""
    p = WL.PARAMS["tiny3"]
    ctx = P.Context.from_params(p, device=0)
    ctx.tune_set("tile", 64)
    ka, kb = ctx.keygen(2101), ctx.keygen(2102)
    specs = [(2, 3000, 4), (5, 700, 8), (1, 4096, 16), (3, 5000, 4)]
    reqs = []
    for k, (rows, f, classes) in enumerate(specs):
        keys = ka if k % 2 == 0 else kb
        wl = WL.make(f"c{k}", "tiny3", rows, f, classes, 0.02, 700 + 13 * k)
        xct = ctx.encrypt_rows(keys, wl.X, seed=800 + k)
        model = ctx.model(wl.W, wl.b)
        alone = ctx.matmul_fast(keys, model, xct, rows)
        reqs.append((wl, keys, xct, model, alone))
    torch.cuda.synchronize()
    ys = [ctx.empty_ct(-(-wl.rows * wl.classes // ctx.n)) for wl, _, _, _, _ in reqs]
    b = P.Batch(ctx, ka, [(xct, wl.rows, model, y) + (() if keys is ka else (keys,))
                          for (wl, keys, xct, model, _), y in zip(reqs, ys)])
    say("two clients: batch of", b.npairs, "pairs")
    b.run()
    torch.cuda.synchronize()
    for k, ((wl, keys, xct, model, alone), y) in enumerate(zip(reqs, ys)):
        assert torch.equal(y, alone), f"batch request {k}"
    srv = P.Server(ctx, ka, hbm_budget=1 << 30)
    ys2, ids = [], []
    for k, (wl, keys, xct, model, _) in enumerate(reqs):
        y = ctx.empty_ct(-(-wl.rows * wl.classes // ctx.n))
        ys2.append(y)
        rid = srv.submit(model, xct, wl.rows, y, keys=None if keys is ka else keys)
        assert rid is not None
        ids.append(rid)
    srv.drain()
    for k, ((wl, keys, xct, model, alone), y) in enumerate(zip(reqs, ys2)):
        assert srv.poll(ids[k])[0]
        assert torch.equal(y, alone), f"server request {k}"
        S, budget = ctx.scores_fast(keys, y, wl.rows, wl.classes)
        assert np.array_equal(S, O.plain_scores(wl.X, wl.W, wl.b, p.t)) and budget > 0
    srv.close()


# ------------------------------------------------------------------ n = 16384, outputs against the oracle
UNEVEN_FILE = "uneven_small_n16k_outputs.txt"


@pytest.fixture(scope="module")
def uneven16(P, torch):
    """Eight requests shaped like the uneven-batching workload (features ~
    U{10,000..40,000}, 1-4 individuals), encrypted as tests/golden/make_golden.py
    encrypted them for the oracle."""
    import golden_ref
    p = WL.PARAMS["n16k"]
    ctx = P.Context.from_params(p, device=0)
    keys = ctx.keygen(2024)
    specs = WL.uneven_requests(count=8, seed=WL.BASE_SEED + 6, max_rows=4)
    models = {}
    reqs = []
    for r, wl in enumerate(specs):
        if wl.f not in models:
            models[wl.f] = ctx.model(wl.W, wl.b)
        xct = ctx.encrypt_rows(keys, wl.X, seed=600 + r)
        reqs.append((wl, xct, models[wl.f]))
    ref = golden_ref.load(UNEVEN_FILE)
    names = [f"req{r}_{wl.rows}x{wl.f}" for r, wl in enumerate(specs)]
    assert set(names) == set(ref)
    return p, ctx, keys, reqs, [ref[nm] for nm in names]


def _check_golden(ctx, y, ref, what):
    import golden_ref
    bad = golden_ref.mismatches(coeff(ctx, y), ref)
    assert not bad, f"{what}: {len(bad)} limbs differ from the oracle, first {bad[0][:3]}"


def test_uneven_n16k_alone_and_batch_vs_oracle(uneven16, P, torch):
    """Each of the eight requests alone, then all eight in one planned batch
    (tiles shared across requests) and its graph replay: every output ciphertext
    equals the oracle's, bit for bit."""
    p, ctx, keys, reqs, refs = uneven16
    for k, (wl, xct, model) in enumerate(reqs):
        say("alone", k, wl.rows, wl.f)
        _check_golden(ctx, ctx.matmul_fast(keys, model, xct, wl.rows), refs[k], f"alone {k}")
    keep = ctx.tune_get("tile")
    ctx.tune_set("tile", 96)      # 384 pairs in 4 tiles: requests straddle tiles
    try:
        ys = [ctx.empty_ct(1) for _ in reqs]
        b = P.Batch(ctx, keys, [(xct, wl.rows, model, y) for (wl, xct, model), y in zip(reqs, ys)])
        say("batch", b.npairs, "pairs, tile", b.tile)
        b.run()
        torch.cuda.synchronize()
        for k, y in enumerate(ys):
            _check_golden(ctx, y, refs[k], f"batch {k}")
        side = torch.cuda.Stream()
        with torch.cuda.stream(side):
            b.capture(side)
        side.synchronize()
        for rep in range(2):
            for y in ys:
                y.fill_(0)
            torch.cuda.synchronize()
            b.run()
            torch.cuda.synchronize()
            for k, y in enumerate(ys):
                _check_golden(ctx, y, refs[k], f"replay {rep} request {k}")
        del b
    finally:
        ctx.tune_set("tile", keep)


def test_uneven_n16k_server_vs_oracle(uneven16, P, torch):
    """The eight requests through the continuous-batching server, submitted one
    by one while earlier ones are still on the GPU (small tiles, so a request
    spans several ticks): every output equals the oracle's, and scores decrypt
    to X W + b mod t."""
    p, ctx, keys, reqs, refs = uneven16
    keep = ctx.tune_get("tile")
    ctx.tune_set("tile", 32)
    try:
        srv = P.Server(ctx, keys, hbm_budget=1 << 30)
        ys, ids, overlapped = [], [], 0
        for k, (wl, xct, model) in enumerate(reqs):
            y = ctx.empty_ct(1)
            ys.append(y)
            # a request submitted while an earlier one has not finished joins the running mix
            overlapped += any(not srv.poll(i)[0] for i in ids)
            ids.append(srv.submit(model, xct, wl.rows, y))
            assert ids[-1] is not None
            time.sleep(0.003)
        srv.drain()
        say("server ticks", srv.stats()["ticks"], "submitted while others ran:", overlapped)
        assert overlapped >= 1
        for k, (wl, xct, model) in enumerate(reqs):
            assert srv.poll(ids[k])[0]
            _check_golden(ctx, ys[k], refs[k], f"server {k}")
            S, budget = ctx.scores_fast(keys, ys[k], wl.rows, wl.classes)
            assert np.array_equal(S, O.plain_scores(wl.X, wl.W, wl.b, p.t)) and budget > 50
            srv.release(ids[k])
        assert srv.stats()["held"] == 0
        srv.close()
    finally:
        ctx.tune_set("tile", keep)
