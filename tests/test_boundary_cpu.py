"""CPU checks of the client-side calls of the C ABI that need no GPU: score
decryption with the result layout of Algorithm 1 (result r = i |Y| + j in
output ciphertext r / n, slot r mod n), the standard layout (score (i, j) in
slot i of ciphertext j), the debug decryption that reports LRHE_ENOISE, the
bounds on the plaintext modulus, and the allocation fault injection switch.
Ciphertexts come from the oracle (moved to the library's evaluation form with
its host transform); contexts are host-only."""
import ctypes
import os
import subprocess
import sys

import numpy as np
import pytest

import bruteforce as bf
import workloads as WL
from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def P():
    import paper_2204_05496_amd as pkg
    pkg.native.lib()
    return pkg


@pytest.fixture(scope="module")
def tiny3(P):
    p = WL.PARAMS["tiny3"]
    ctx = P.Context.from_params(p, device=-1)
    o = O.Oracle(p.n, list(p.q), p.P, p.t)
    return p, ctx, o, ctx.keygen(77, galois=False), o.keygen(77, galois=False)


def encrypt_slots(ctx, o, ko, Z, seed):
    """Oracle encryptions of the slot vectors Z[c], in the library's evaluation form."""
    L = len(o.q)
    out = np.zeros((len(Z), 2, L, o.n), dtype=np.uint32)
    for c, z in enumerate(Z):
        ct = o.encrypt_plain(ko, o.encode(z), seed, c)
        for x in range(2):
            for j in range(L):
                out[c, x, j] = ctx.host_transform(ct[x, j].astype(np.uint32), j)
    return out


def test_decrypt_scores_fast_layout(tiny3, P):
    p, ctx, o, keys, ko = tiny3
    rows, classes = 300, 16                     # 4,800 results: two output ciphertexts, the second partly used
    rng = np.random.default_rng(11)
    Z = rng.integers(0, p.t, (2, p.n))
    y = encrypt_slots(ctx, o, ko, Z, 5)
    S, budget = ctx.scores_fast(keys, y, rows, classes)
    r = np.arange(rows * classes)
    exp = o.centre(Z[r // p.n, r % p.n]).reshape(rows, classes)
    assert np.array_equal(S, exp) and budget > 0
    # the budget reported is the smaller of the two ciphertexts'
    _, bud = ctx.decrypt_slots_host(keys, y)
    assert budget == pytest.approx(bud.min())
    N = P.native
    code = N.lib().lrhe_decrypt_scores(ctx.h, keys.sk, N.ptr(y), 0, classes, N.CT_HOST,
                                       N.ptr(np.zeros(1, np.int64)), None, None)
    assert code == N.LRHE_EINVAL                 # no rows
    code = N.lib().lrhe_decrypt_scores(ctx.h, keys.sk, N.ptr(y), rows, classes, 2, N.ptr(np.zeros(rows * classes,
                                       np.int64)), None, None)
    assert code == N.LRHE_EINVAL                 # unknown flag


def test_decrypt_scores_standard_layout(tiny3, P):
    p, ctx, o, keys, ko = tiny3
    rows, classes = 700, 3
    rng = np.random.default_rng(12)
    Z = rng.integers(0, p.t, (classes, p.n))
    y = encrypt_slots(ctx, o, ko, Z, 6)
    S, budget = ctx.scores_standard(keys, y, rows)
    assert np.array_equal(S, o.centre(Z[:, :rows].T)) and budget > 0


def test_decrypt_check_reports_noise(tiny3, P):
    """LRHE_ENOISE when a slot differs from the expected plaintext; OK (with the
    budgets) when all agree."""
    p, ctx, o, keys, ko = tiny3
    rng = np.random.default_rng(13)
    Z = rng.integers(0, p.t, (2, p.n))
    y = encrypt_slots(ctx, o, ko, Z, 7)
    lib, N = P.native.lib(), P.native
    bud = np.zeros(2)
    bad = ctypes.c_uint64()
    exp = np.ascontiguousarray(o.centre(Z), dtype=np.int64)
    assert lib.lrhe_decrypt_check(ctx.h, keys.sk, N.ptr(y), 2, N.ptr(exp), N.CT_HOST, N.ptr(bud), ctypes.byref(bad),
                                  None) == N.LRHE_OK
    assert bad.value == 0 and np.all(bud > 0)
    exp2 = exp + p.t                                   # the same residues mod t
    assert lib.lrhe_decrypt_check(ctx.h, keys.sk, N.ptr(y), 2, N.ptr(exp2), N.CT_HOST, None, None, None) == 0
    exp[1, 17] += 1
    exp[0, 3] -= 5
    code = lib.lrhe_decrypt_check(ctx.h, keys.sk, N.ptr(y), 2, N.ptr(exp), N.CT_HOST, None, ctypes.byref(bad), None)
    assert code == N.LRHE_ENOISE and bad.value == 2
    assert "slot 3" in lib.lrhe_last_error().decode()
    # a ciphertext whose noise has wrapped (a fresh one with a large error added to c0)
    # decrypts to the wrong slots, which the check reports
    ev = y[:1].copy()
    ct = o.encrypt_plain(ko, o.encode(Z[0]), 7, 0)
    Q = 1
    for q in p.q:
        Q *= q
    big = Q // (2 * p.t)                               # the decryption threshold itself
    for j, q in enumerate(p.q):
        c0 = (ct[0, j].astype(object) + big * 3 // 2) % q
        ev[0, 0, j] = ctx.host_transform(np.array(c0, dtype=np.uint32), j)
    exp = np.ascontiguousarray(o.centre(Z[:1]), dtype=np.int64)
    assert lib.lrhe_decrypt_check(ctx.h, keys.sk, N.ptr(ev), 1, N.ptr(exp), N.CT_HOST, None, None,
                                  None) == N.LRHE_ENOISE


def _create(P, n, q, Pm, t, insecure=0):
    lib = P.native.lib()
    arr = (ctypes.c_uint32 * len(q))(*q)
    prm = P.native.LrheParams(n, len(q), arr, Pm, t, insecure)
    h = ctypes.c_void_p()
    code = lib.lrhe_ctx_create(ctypes.byref(prm), -1, ctypes.byref(h))
    if code == 0:
        lib.lrhe_ctx_destroy(h)
    return code, lib.lrhe_last_error().decode()


def test_plaintext_modulus_bounds(P):
    """t may exceed 2^30 (the paper's t0 = 1073872897 at n = 8192) but must stay
    below 2^31 and below twice every ciphertext prime, so that its centred lift is
    a residue of each prime."""
    qs = bf.ntt_primes(8192, 7)
    assert _create(P, 8192, qs[:6], qs[6], 1073872897)[0] == 0, _create(P, 8192, qs[:6], qs[6], 1073872897)
    # a prime t = 1 mod 16384 between 2 min(q) and 2^31
    lo = 2 * min(qs)
    t_big = next(c for c in range(lo // 16384 * 16384 + 1, 1 << 31, 16384) if c > lo and bf.is_prime(c))
    code, msg = _create(P, 8192, qs[:6], qs[6], t_big)
    assert code == P.native.LRHE_EPARAM and "below 2 q" in msg
    t_over = next(c for c in range((1 << 31) + 1, (1 << 32) - 1, 16384) if bf.is_prime(c))
    assert _create(P, 8192, qs[:6], qs[6], t_over)[0] == P.native.LRHE_EPARAM


def test_fault_injection_switch(P):
    """LRHE_FAULT_ALLOC arms the allocation fault at load; lrhe_fault_inject sets,
    reads and disarms it (no device allocation happens on the CPU)."""
    code = ("import sys; sys.path.insert(0, %r); import paper_2204_05496_amd as P; "
            "L = P.native.lib(); print(L.lrhe_fault_inject(-1)); print(L.lrhe_fault_inject(0)); "
            "print(L.lrhe_fault_inject(-1))" % ROOT)
    env = dict(os.environ, LRHE_FAULT_ALLOC="3")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split() == ["3", "3", "0"]
    lib = P.native.lib()
    prev = lib.lrhe_fault_inject(2)
    assert lib.lrhe_fault_inject(-1) == 2
    assert lib.lrhe_fault_inject(prev) == 2


def test_crt_combine_matches_oracle(P):
    """lrhe_crt_combine against the oracle's recombination over the paper's pair,
    on residues of integers spread over the whole signed range (centred and
    non-negative representatives), and its refusals."""
    t0, t1 = WL.T_PAIR
    half = (t0 * t1) // 2
    r = np.random.Generator(np.random.PCG64(5))
    z = np.concatenate([r.integers(-half + 1, half + 1, size=2000, dtype=np.int64),
                        np.array([0, 1, -1, half, -half + 1, 2 ** 44, -(2 ** 44)], dtype=np.int64)])
    r0 = np.array([int(v) % t0 for v in z], dtype=np.int64)
    r1 = np.array([int(v) % t1 for v in z], dtype=np.int64)
    got = P.crt_combine(r0, r1, t0, t1)
    assert np.array_equal(got, z)
    assert list(got) == [int(v) for v in O.crt_pair(r0.astype(object), r1.astype(object), t0, t1)]
    c0 = np.where(r0 > (t0 - 1) // 2, r0 - t0, r0)
    c1 = np.where(r1 > (t1 - 1) // 2, r1 - t1, r1)
    assert np.array_equal(P.crt_combine(c0, c1, t0, t1), z)
    lib = P.native.lib()
    one = np.zeros(1, dtype=np.int64)
    p = P.native.ptr
    assert lib.lrhe_crt_combine(p(one), p(one), 1, 6, 4, p(one)) == P.native.LRHE_EINVAL       # not coprime
    assert lib.lrhe_crt_combine(p(one), p(one), 1, 2 ** 32 + 15, 2 ** 31 + 11, p(one)) == P.native.LRHE_EINVAL
    assert lib.lrhe_crt_combine(p(one), p(one), 1, 1, 7, p(one)) == P.native.LRHE_EINVAL


def test_fixed_point_matches_oracle(P):
    """lrhe_fixed_point against the oracle's conversion on the paper-point
    workload's inputs, weights and biases, ties, signs, and the refusals."""
    wl = WL.paper_single(f=4096)
    for a, bits in ((wl.X, WL.S_X), (wl.W, WL.S_W), (wl.b, WL.S_X + WL.S_W)):
        assert np.array_equal(P.fixed_point(a, bits), O.fixed_point(a, bits))
    ties = np.array([0.5, 1.5, 2.5, -0.5, -1.5, -2.5, 3.0, -7.25])
    assert np.array_equal(P.fixed_point(ties, 0), O.fixed_point(ties, 0))
    with pytest.raises(P.native.LrheError):
        P.fixed_point(np.array([np.inf]), 6)
    with pytest.raises(P.native.LrheError):
        P.fixed_point(np.array([2.0 ** 60]), 6)
    with pytest.raises(P.native.LrheError):
        P.fixed_point(np.array([1.0]), 63)
