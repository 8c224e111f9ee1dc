"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Every stage of Algorithm 1 is compared bit for bit in canonical coefficient
form (ciphertext residues in [0, q_i)); decrypted scores are compared with the
plain integer matmul X W + b mod t of the private inference protocol, which
holds at any size.  Tolerance: none (exact modular integer arithmetic).
"""
import sys

import numpy as np
import pytest

import workloads as WL
from oracle import oracle as O

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-parity]", *a, flush=True)
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


class Setup:
    def __init__(self, P, pname, key_seed):
        p = WL.PARAMS[pname]
        self.p = p
        self.ctx = P.Context.from_params(p, device=0)
        self.o = O.Oracle(p.n, list(p.q), p.P, p.t)
        self.keys = self.ctx.keygen(key_seed)
        self.ko = self.o.keygen(key_seed)

    def coeff(self, t):
        from paper_2204_05496_amd import to_numpy_u32
        return to_numpy_u32(self.ctx.to_coeff(t)).astype(np.uint64)


@pytest.fixture(scope="module")
def tiny(P):
    say("setup tiny n=4096 L=2")
    return Setup(P, "tiny", 1234)


@pytest.fixture(scope="module")
def tiny3(P):
    say("setup tiny3 n=4096 L=3")
    return Setup(P, "tiny3", 4321)


@pytest.fixture(scope="module")
def n16k(P):
    say("setup n16k n=16384 L=7")
    return Setup(P, "n16k", 2024)


# ------------------------------------------------------------------ tiny (n = 4096, two data primes)
def test_encrypt_rows_parity_tiny(tiny, torch):
    wl = WL.tiny()
    say("encrypt_rows tiny")
    xct = tiny.ctx.encrypt_rows(tiny.keys, wl.X, seed=99)
    torch.cuda.synchronize()
    ref = tiny.o.encrypt_rows(tiny.ko, wl.X, seed=99)
    assert np.array_equal(tiny.coeff(xct), ref.reshape(-1, *ref.shape[2:]))


@pytest.mark.parametrize("stage", [1, 2 + 1, 2 + 6, 2 + 12, 100, 0])
def test_stage_parity_tiny(tiny, torch, stage):
    """Per-pair ciphertext after each stage: chunk products + add_many (1),
    s rotate-and-accumulate steps (2 + s), bias (100), one-hot mask (0)."""
    wl = WL.tiny()
    say("stage", stage)
    xct = tiny.ctx.encrypt_rows(tiny.keys, wl.X, seed=99)
    model = tiny.ctx.model(wl.W, wl.b)
    got = tiny.coeff(tiny.ctx.matmul_fast_pairs(tiny.keys, model, xct, wl.rows, 0, wl.rows * wl.classes, stage))
    xo = tiny.o.encrypt_rows(tiny.ko, wl.X, seed=99)
    wo = tiny.o.encode_weights(wl.W)
    for r in range(wl.rows * wl.classes):
        i, j = divmod(r, wl.classes)
        ref = tiny.o.pair(tiny.ko, xo[i], wo[j], int(wl.b[j]), r % tiny.p.n, stage)
        assert np.array_equal(got[r], ref), f"pair {r} stage {stage}"


def test_fast_output_parity_tiny(tiny, torch):
    wl = WL.tiny()
    xct = tiny.ctx.encrypt_rows(tiny.keys, wl.X, seed=99)
    model = tiny.ctx.model(wl.W, wl.b)
    y = tiny.ctx.matmul_fast(tiny.keys, model, xct, wl.rows)
    xo = tiny.o.encrypt_rows(tiny.ko, wl.X, seed=99)
    ref = tiny.o.fast_matmul(tiny.ko, xo, tiny.o.encode_weights(wl.W), wl.b)
    assert np.array_equal(tiny.coeff(y), ref)
    # determinism: a second run gives the same bits
    y2 = tiny.ctx.matmul_fast(tiny.keys, model, xct, wl.rows)
    assert torch.equal(y, y2)


def test_many_outputs_ragged_tiny(tiny, torch):
    """rows x classes > n (two output ciphertexts, the second partly filled),
    f not a multiple of n, groups that straddle tiles."""
    rows, f, classes = 260, 300, 16
    wl = WL.make("ragged", "tiny", rows, f, classes, 0.02, WL.BASE_SEED + 11)
    say("ragged tiny", rows * classes, "pairs")
    xct = tiny.ctx.encrypt_rows(tiny.keys, wl.X, seed=5)
    model = tiny.ctx.model(wl.W, wl.b)
    y = tiny.ctx.matmul_fast(tiny.keys, model, xct, rows)
    xo = tiny.o.encrypt_rows(tiny.ko, wl.X, seed=5)
    ref = tiny.o.fast_matmul(tiny.ko, xo, tiny.o.encode_weights(wl.W), wl.b)
    assert ref.shape[0] == 2
    assert np.array_equal(tiny.coeff(y), ref)


# ------------------------------------------------------------------ tiny3 (three data primes): decryption end to end
def test_scores_fast_and_standard_tiny3(tiny3, torch):
    wl = WL.tiny(params="tiny3")
    ctx = tiny3.ctx
    xct = ctx.encrypt_rows(tiny3.keys, wl.X, seed=31)
    model = ctx.model(wl.W, wl.b)
    y = ctx.matmul_fast(tiny3.keys, model, xct, wl.rows)
    S, budget = ctx.scores_fast(tiny3.keys, y, wl.rows, wl.classes)
    plain = O.plain_scores(wl.X, wl.W, wl.b, tiny3.p.t)
    assert np.array_equal(S, plain) and budget > 0
    xo = tiny3.o.encrypt_rows(tiny3.ko, wl.X, seed=31)
    ref = tiny3.o.fast_matmul(tiny3.ko, xo, tiny3.o.encode_weights(wl.W), wl.b)
    assert np.array_equal(tiny3.coeff(y), ref)
    # standard baseline: individuals in slots, one ciphertext per feature
    fct = ctx.encrypt_cols(tiny3.keys, wl.X, seed=32)
    fo = tiny3.o.encrypt_cols(tiny3.ko, wl.X, seed=32)
    assert np.array_equal(tiny3.coeff(fct), fo)
    ys = ctx.matmul_standard(model, fct)
    assert np.array_equal(tiny3.coeff(ys), tiny3.o.standard_matmul(fo, wl.W, wl.b))
    S2, budget2 = ctx.scores_standard(tiny3.keys, ys, wl.rows)
    assert np.array_equal(S2, plain) and budget2 > 0
    assert np.array_equal(S.argmax(1), plain.argmax(1))


def test_standard_many_rows_tiny3(tiny3, torch):
    rows, f, classes = 700, 97, 5
    wl = WL.make("std", "tiny3", rows, f, classes, 0.3, WL.BASE_SEED + 12)
    ctx = tiny3.ctx
    fct = ctx.encrypt_cols(tiny3.keys, wl.X, seed=8)
    model = ctx.model(wl.W, wl.b)
    S, budget = ctx.scores_standard(tiny3.keys, ctx.matmul_standard(model, fct), rows)
    assert np.array_equal(S, O.plain_scores(wl.X, wl.W, wl.b, tiny3.p.t)) and budget > 0


def test_invalid_shapes_rejected(tiny, P):
    wl = WL.tiny()
    model = tiny.ctx.model(wl.W, wl.b)
    xct = tiny.ctx.encrypt_rows(tiny.keys, wl.X, seed=1)
    with pytest.raises(P.native.LrheError):
        tiny.ctx.matmul_fast(tiny.keys, model, xct, 0)
    with pytest.raises(P.native.LrheError):   # pair range past rows x classes
        tiny.ctx.matmul_fast_pairs(tiny.keys, model, xct, 1, 2, 3, 0)
    ws = tiny.ctx.workspace(P.native.WS_MATMUL_FAST, 1, wl.f, wl.classes)
    with pytest.raises(P.native.LrheError):   # workspace too small
        tiny.ctx.matmul_fast(tiny.keys, model, xct, 1, ws=ws[:1024])


# ------------------------------------------------------------------ n = 16384, seven data primes
def test_single_40k_parity(n16k, torch):
    """1 individual x 40,000 features, 16 classes: ciphertexts after encryption
    and after Algorithm 1 equal the oracle's; scores equal the plain matmul."""
    wl = WL.single()
    ctx, o = n16k.ctx, n16k.o
    say("single 40k encrypt")
    xct = ctx.encrypt_rows(n16k.keys, wl.X, seed=99)
    xo = o.encrypt_rows(n16k.ko, wl.X, seed=99)
    assert np.array_equal(n16k.coeff(xct), xo.reshape(-1, *xo.shape[2:]))
    model = ctx.model(wl.W, wl.b)
    say("single 40k fast")
    y = ctx.matmul_fast(n16k.keys, model, xct, 1)
    S, budget = ctx.scores_fast(n16k.keys, y, 1, wl.classes)
    plain = O.plain_scores(wl.X, wl.W, wl.b, n16k.p.t)
    assert np.array_equal(S, plain) and budget > 50
    say("single 40k oracle")
    ref = o.fast_matmul(n16k.ko, xo, o.encode_weights(wl.W), wl.b)
    assert np.array_equal(n16k.coeff(y), ref)


def test_single_40k_standard(n16k, torch):
    """Standard baseline on the full 40,000 features (scores), and bit parity of
    its ciphertexts on a 300-feature slice."""
    wl = WL.single()
    ctx, o = n16k.ctx, n16k.o
    say("standard 40k")
    fct = ctx.encrypt_cols(n16k.keys, wl.X, seed=7)
    model = ctx.model(wl.W, wl.b)
    ys = ctx.matmul_standard(model, fct)
    S, budget = ctx.scores_standard(n16k.keys, ys, 1)
    assert np.array_equal(S, O.plain_scores(wl.X, wl.W, wl.b, n16k.p.t)) and budget > 50
    del fct, ys
    torch.cuda.empty_cache()
    Xs, Ws = wl.X[:, :300], wl.W[:300]
    fct = ctx.encrypt_cols(n16k.keys, Xs, seed=7)
    ms = ctx.model(Ws, wl.b)
    fo = o.encrypt_cols(n16k.ko, Xs, seed=7)
    assert np.array_equal(n16k.coeff(fct), fo)
    assert np.array_equal(n16k.coeff(ctx.matmul_standard(ms, fct)), o.standard_matmul(fo, Ws, wl.b))


@pytest.mark.parametrize("cls", ["small", "large", "large_xcd", "large_plain", "large_split64"])
@pytest.mark.parametrize("stage", [1, 2 + 1, 2 + 7, 2 + 14, 100, 0])
def test_stage_parity_n16k(n16k, torch, P, stage, cls):
    """Per-pair ciphertext after each stage at n = 16384, L = 7 (1 x 40,000 x 16):
    chunk products (1), 1, 7 and all 14 rotate-and-accumulate steps, bias (100)
    and mask (0), with the small-tile kernels (digit halves), with the
    large-tile ones (the same 16 pairs run as a large tile: by default the split
    launches, special-prime items with the digits first, then the data-modulus
    items ending with the division by P), with the large-tile variant that
    spreads the target moduli by XCD, with the plain one (k_ks_intt,
    k_ks_mac, k_ks_moddown) and with the split launches whose data-modulus
    items sum unreduced 64-bit products; three pairs each against the oracle."""
    wl = WL.single()
    ctx, o = n16k.ctx, n16k.o
    say("stage", stage, cls)
    keep = ctx.tune_get("small_below")
    keep_mode = ctx.tune_get("large.mac_mode")
    if cls != "small":
        ctx.tune_set("small_below", 1)
    if cls == "large_xcd":
        ctx.tune_set("large.mac_mode", P.native.MAC_MODE_XCD)
    if cls == "large_plain":
        ctx.tune_set("large.mac_mode", 1)
    if cls == "large_split64":
        ctx.tune_set("large.mac_mode", P.native.MAC_MODE_SPLIT64)
    try:
        xct = ctx.encrypt_rows(n16k.keys, wl.X, seed=17)
        model = ctx.model(wl.W, wl.b)
        got = n16k.coeff(ctx.matmul_fast_pairs(n16k.keys, model, xct, wl.rows, 0, wl.rows * wl.classes, stage))
    finally:
        ctx.tune_set("small_below", keep)
        ctx.tune_set("large.mac_mode", keep_mode)
    xo = o.encrypt_rows(n16k.ko, wl.X, seed=17)
    wo = o.encode_weights(wl.W)
    for r in (0, 7, 15):
        ref = o.pair(n16k.ko, xo[0], wo[r], int(wl.b[r]), r % o.n, stage)
        assert np.array_equal(got[r], ref), f"pair {r} stage {stage} ({cls} tiles)"


def test_batch_512x40k_launch_config(n16k, torch):
    """512 individuals x 40,000 features (the throughput workload) in the launch
    configuration the benchmark times: the whole output ciphertext equals the
    oracle's (stored by tests/golden/make_golden.py, compared limb by limb),
    scores equal the plain matmul, and sampled pairs equal the oracle pair by pair."""
    import golden_ref
    wl = WL.batch()
    ctx, o = n16k.ctx, n16k.o
    say("batch encrypt")
    xct = ctx.encrypt_rows(n16k.keys, wl.X, seed=3)
    model = ctx.model(wl.W, wl.b)
    say("batch fast")
    y = ctx.matmul_fast(n16k.keys, model, xct, wl.rows)
    torch.cuda.synchronize()
    ref = golden_ref.load("batch_512x40000x16_fast_output.txt")[wl.name]
    bad = golden_ref.mismatches(n16k.coeff(y), ref)
    assert not bad, f"{len(bad)} limbs differ from the oracle, first {bad[0][:3]}"
    say("batch decrypt")
    S, budget = ctx.scores_fast(n16k.keys, y, wl.rows, wl.classes)
    plain = O.plain_scores(wl.X, wl.W, wl.b, n16k.p.t)
    assert np.array_equal(S, plain) and budget > 30
    say("batch sampled pairs")
    # every pair's masked ciphertext, in the same tiles of 4096 pairs as the
    # compressed run above; sampled pairs (tile edges included) against the oracle
    npairs = wl.rows * wl.classes
    allp = ctx.matmul_fast_pairs(n16k.keys, model, xct, wl.rows, 0, npairs, 0)
    torch.cuda.synchronize()
    sample = [0, 1, 4095, 4096, 5000, 8191]
    wo = o.encode_weights(wl.W)
    rows_needed = sorted({r // wl.classes for r in sample})
    xo = {i: o.encrypt_rows(n16k.ko, wl.X[i:i + 1], seed=3, row0=i)[0] for i in rows_needed}
    for r in sample:
        got = n16k.coeff(allp[r:r + 1])[0]
        i, j = divmod(r, wl.classes)
        ref = o.pair(n16k.ko, xo[i], wo[j], int(wl.b[j]), r % o.n, 0)
        assert np.array_equal(got, ref), f"pair {r}"
    # compression: the masked pairs of the output sum, limb by limb mod q_i, to y
    acc = torch.zeros((2, ctx.L, ctx.n), dtype=torch.int64, device=allp.device)
    for c0 in range(0, npairs, 1024):
        acc += allp[c0:c0 + 1024].to(torch.int64).sum(dim=0)
    q = torch.tensor(list(n16k.p.q), dtype=torch.int64, device=allp.device).view(1, -1, 1)
    assert torch.equal(acc % q, y[0].to(torch.int64))
    del allp, acc
    torch.cuda.empty_cache()


@pytest.mark.parametrize("variant", ["xcd", "plain", "split64"])
def test_batch_512x40k_variants(n16k, torch, P, variant):
    """The throughput workload with the other large-tile key-switch variants
    (the default, the split launches, is the launch configuration test's):
    target moduli spread by XCD per window of pairs (its own workgroup-to-item
    map), the plain sequence k_ks_intt, k_ks_mac, k_ks_moddown, and the split
    launches with unreduced 64-bit inner products.  The whole output ciphertext
    equals the oracle's stored one."""
    import golden_ref
    wl = WL.batch()
    ctx = n16k.ctx
    keep = ctx.tune_get("large.mac_mode")
    ctx.tune_set("large.mac_mode", {"xcd": P.native.MAC_MODE_XCD, "plain": 1,
                                    "split64": P.native.MAC_MODE_SPLIT64}[variant])
    try:
        say("batch encrypt")
        xct = ctx.encrypt_rows(n16k.keys, wl.X, seed=3)
        model = ctx.model(wl.W, wl.b)
        say("batch fast, variant", variant)
        y = ctx.matmul_fast(n16k.keys, model, xct, wl.rows)
        torch.cuda.synchronize()
    finally:
        ctx.tune_set("large.mac_mode", keep)
    ref = golden_ref.load("batch_512x40000x16_fast_output.txt")[wl.name]
    bad = golden_ref.mismatches(n16k.coeff(y), ref)
    assert not bad, f"{len(bad)} limbs differ from the oracle, first {bad[0][:3]}"
    del y
    torch.cuda.empty_cache()
