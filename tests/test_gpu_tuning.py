"""GPU: launch tuning never changes a result bit.

Every residues-per-thread choice of the four transform kernels, every
exchange / prefetch variant of the key-switch inner product, and the tile size
give the same output ciphertexts, equal to the oracle's.  Tolerance: none.
"""
import itertools
import sys

import numpy as np
import pytest

import workloads as WL
from bruteforce import ntt_primes
from oracle import oracle as O

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-tuning]", *a, flush=True)
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


def valid_les(ctx):
    out = []
    for le in (4, 5, 6):
        try:
            ctx.tune_set("le_mac", le)
            out.append(le)
        except Exception:
            pass
    ctx.tune_set("le_mac", 5)
    return out


def ring(n, t):
    """Three data primes and a special prime below 2^30, 1 mod 2n (below the
    128-bit bound only for the larger n: test parameters)."""
    ps = ntt_primes(n, 4)
    return WL.Params(f"ring{n}", n, tuple(ps[:3]), ps[3], t, insecure=True)


# n = 2048 and 8192 have a last transform pass of a single stage at 32 and 64
# residues per thread respectively
# one data prime: the second digit half of the digit-halves variant is empty
@pytest.mark.parametrize("pname,rows,f,classes", [("tiny", 3, 5000, 4), ("n16k", 1, 40000, 16),
                                                  ("ring2048", 2, 2500, 3), ("ring8192", 1, 9000, 2),
                                                  ("oneprime", 2, 3000, 3)])
def test_every_tuning_choice_same_bits(P, torch, pname, rows, f, classes):
    if pname == "oneprime":
        ps = ntt_primes(4096, 2)
        p = WL.Params("oneprime", 4096, (ps[0],), ps[1], 65537, insecure=True)
    elif pname.startswith("ring"):
        n = int(pname[4:])
        p = ring(n, 12289 if n == 2048 else 65537)
    else:
        p = WL.PARAMS[pname]
    ctx = P.Context.from_params(p, device=0)
    keys = ctx.keygen(606)
    wl = WL.Workload("tune", pname, rows, f, classes, 0.02, WL.BASE_SEED + 21,
                     WL.features(rows, f, 0.02, WL.BASE_SEED + 21), WL.weights(f, classes, WL.BASE_SEED + 22),
                     WL.biases(classes, WL.BASE_SEED + 23))
    xct = ctx.encrypt_rows(keys, wl.X, seed=44)
    model = ctx.model(wl.W, wl.b)
    ref = ctx.matmul_fast(keys, model, xct, rows)
    torch.cuda.synchronize()
    if pname != "n16k":
        o = O.Oracle(p.n, list(p.q), p.P, p.t)
        ko = o.keygen(606)
        xo = o.encrypt_rows(ko, wl.X, seed=44)
        exp = o.fast_matmul(ko, xo, o.encode_weights(wl.W), wl.b)
        from paper_2204_05496_amd import to_numpy_u32
        assert np.array_equal(to_numpy_u32(ctx.to_coeff(ref)).astype(np.uint64), exp)
    les = valid_les(ctx)
    say(pname, "valid residues-per-thread", les)
    for le, mode, fuse in itertools.product(les, range(P.native.MAC_MODES), (0, 1)):
        for knob in ("le_intt", "le_mac", "le_moddown", "le_mask"):
            ctx.tune_set(knob, le)
        # the split variant's special-prime launch: a different choice from le_mac
        ctx.tune_set("le_mac_p", les[(les.index(le) + 1) % len(les)])
        ctx.tune_set("small.mac_mode", mode)   # every tile of these jobs is in the small class
        ctx.tune_set("fuse_intt", fuse)
        say(pname, "le", le, "mac_mode", mode, "fuse_intt", fuse)
        y = ctx.matmul_fast(keys, model, xct, rows)
        torch.cuda.synchronize()
        assert torch.equal(y, ref), f"le {le} mac_mode {mode} fuse_intt {fuse}"
    # the large-tile variants on the same job (every tile of it large), among them
    # the split launches (digits made by the special-prime launch, the division
    # by P in the data-modulus launch) with L = 1, 2, 3 or 7 data primes
    keep_sb = ctx.tune_get("small_below")
    ctx.tune_set("small_below", 1)
    try:
        for le, mode in itertools.product(les, range(P.native.MAC_MODES)):
            if mode == P.native.MAC_MODE_HALF:
                continue
            for knob in ("le_intt", "le_mac", "le_moddown", "le_mask"):
                ctx.tune_set("large." + knob, le)
            ctx.tune_set("large.le_mac_p", les[(les.index(le) + 1) % len(les)])
            ctx.tune_set("large.mac_mode", mode)
            for fuse in ((0, 1) if mode == 1 else (0,)):
                ctx.tune_set("large.fuse_intt", fuse)
                say(pname, "large tiles: le", le, "mac_mode", mode, "fuse_intt", fuse)
                y = ctx.matmul_fast(keys, model, xct, rows)
                torch.cuda.synchronize()
                assert torch.equal(y, ref), f"large tiles: le {le} mac_mode {mode} fuse_intt {fuse}"
        ctx.tune_set("large.fuse_intt", 0)
    finally:
        ctx.tune_set("small_below", keep_sb)
    for knob in ("le_intt", "le_mac", "le_moddown", "le_mask"):
        ctx.tune_set(knob, 5)
    ctx.tune_set("mac_mode", 0)
    for tile in (1, 3, 64):
        ctx.tune_set("tile", tile)
        y = ctx.matmul_fast(keys, model, xct, rows)
        torch.cuda.synchronize()
        assert torch.equal(y, ref), f"tile {tile}"
    ctx.tune_set("tile", 4096)


def test_autotuner_keeps_bits(P, torch):
    p = WL.PARAMS["tiny"]
    ctx = P.Context.from_params(p, device=0)
    keys = ctx.keygen(7)
    wl = WL.make("auto", "tiny", 9, 3000, 8, 0.02, WL.BASE_SEED + 22)
    xct = ctx.encrypt_rows(keys, wl.X, seed=45)
    model = ctx.model(wl.W, wl.b)
    ref = ctx.matmul_fast(keys, model, xct, wl.rows)
    tuned = ctx.autotune_fast(keys, model, xct, wl.rows)
    say("autotuned", tuned)
    for cls in ("small", "large"):
        t = tuned[cls]
        assert t["mac_mode"] in range(P.native.MAC_MODES) and all(t[k] in (4, 5, 6)
                                                                  for k in ("le_intt", "le_mac", "le_moddown", "le_mac_p"))
    assert tuned["large"]["mac_mode"] != P.native.MAC_MODE_HALF
    y = ctx.matmul_fast(keys, model, xct, wl.rows)
    torch.cuda.synchronize()
    assert torch.equal(y, ref)


def test_digit_halves_small_class_only(P, torch):
    """The digit-halves key-switch variant is a small-tile choice: setting it for
    the large class is refused; a job whose last tile is small runs that tile
    with it (two accumulator slots per pair inside the job's buffer) and keeps
    every bit."""
    p = WL.PARAMS["tiny3"]   # three data primes: enough noise budget to decrypt
    ctx = P.Context.from_params(p, device=0)
    keys = ctx.keygen(808)
    half = P.native.MAC_MODE_HALF
    for key in ("mac_mode", "large.mac_mode"):
        with pytest.raises(P.native.LrheError):
            ctx.tune_set(key, half)
    wl = WL.make("halves", "tiny3", 3, 5000, 4, 0.02, WL.BASE_SEED + 31)   # 12 pairs
    xct = ctx.encrypt_rows(keys, wl.X, seed=46)
    model = ctx.model(wl.W, wl.b)
    ref = ctx.matmul_fast(keys, model, xct, wl.rows)
    torch.cuda.synchronize()
    # tiles of 8 pairs (large class) then 4 (small class, digit halves)
    ctx.tune_set("tile", 8)
    ctx.tune_set("small_below", 5)
    ctx.tune_set("small.mac_mode", half)
    for le in valid_les(ctx):
        ctx.tune_set("small.le_mac", le)
        ctx.tune_set("small.le_moddown", le)
        say("mixed tiles, small class digit halves, le", le)
        y = ctx.matmul_fast(keys, model, xct, wl.rows)
        torch.cuda.synchronize()
        assert torch.equal(y, ref), f"le {le}"
    S, budget = ctx.scores_fast(keys, y, wl.rows, wl.classes)
    assert np.array_equal(S, O.plain_scores(wl.X, wl.W, wl.b, p.t))
