"""GPU tests of the one-vs-rest binary models (section "Binary models"): one
model per cancer type with its own features and a single output (|Y| = 1),
run as one planned batch of requests.  Every model's output ciphertext equals
the oracle's (small ring) and the same model run alone (n = 16384, the
paper's 543 patients), bit for bit, and decrypts to X_m W_m + b_m mod t."""
import sys

import numpy as np
import pytest

import workloads as WL
from oracle import oracle as O

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-binary]", *a, flush=True)
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


def run_batch(P, ctx, keys, models, torch):
    reqs = []
    for k, wl in enumerate(models):
        xct = ctx.encrypt_rows(keys, wl.X, seed=500 + k)
        reqs.append((xct, wl.rows, ctx.model(wl.W, wl.b), ctx.empty_ct(-(-wl.rows // ctx.n))))
    b = P.Batch(ctx, keys, reqs)
    b.run()
    torch.cuda.synchronize()
    return reqs, b


def test_binary_models_batch_vs_oracle(P, torch):
    p = WL.PARAMS["tiny3"]
    ctx = P.Context.from_params(p, device=0)
    keys = ctx.keygen(321)
    o = O.Oracle(p.n, list(p.q), p.P, p.t)
    ko = o.keygen(321)
    models = WL.binary_models(rows=3, seed=WL.BASE_SEED + 61, params="tiny3", f_lo=500, f_hi=6000, p=0.05)
    reqs, b = run_batch(P, ctx, keys, models, torch)
    from paper_2204_05496_amd import to_numpy_u32
    for k, (wl, (xct, rows, model, y)) in enumerate(zip(models, reqs)):
        say("model", k, "f", wl.f)
        ref = o.fast_matmul(ko, o.encrypt_rows(ko, wl.X, seed=500 + k), o.encode_weights(wl.W), wl.b)
        assert np.array_equal(to_numpy_u32(ctx.to_coeff(y)).astype(np.uint64), ref), f"model {k}"
        S, budget = ctx.scores_fast(keys, y, rows, 1)
        assert np.array_equal(S, O.plain_scores(wl.X, wl.W, wl.b, p.t)) and budget > 0
    b.close()


def test_binary_models_543_batch_equals_alone(P, torch):
    p = WL.PARAMS["n16k"]
    ctx = P.Context.from_params(p, device=0)
    keys = ctx.keygen(2024)
    models = WL.binary_models()
    say("11 binary models, 543 individuals, f", [wl.f for wl in models])
    reqs, b = run_batch(P, ctx, keys, models, torch)
    for k, (wl, (xct, rows, model, y)) in enumerate(zip(models, reqs)):
        alone = ctx.matmul_fast(keys, model, xct, rows)
        torch.cuda.synchronize()
        assert torch.equal(alone, y), f"model {k}"
        S, budget = ctx.scores_fast(keys, y, rows, 1)
        assert np.array_equal(S, O.plain_scores(wl.X, wl.W, wl.b, p.t)) and budget > 30
    b.close()
