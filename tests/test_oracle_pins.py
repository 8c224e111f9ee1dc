"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: published
test vectors, schoolbook products, closed forms, brute force with Python
integers on tiny rings, decryption invariants (Dec(Enc(m)) = m, the trace
invariant "all slots contain the result" of Algorithm 1), and the plain
integer matmul X W + b mod t of the private inference protocol.
"""
import math
import os

import numpy as np
import pytest

import bruteforce as bf
import workloads as WL
from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# tiny rings for brute force: primes = 1 mod 32 below 2^30, t = 257 (= 1 mod 32)
N16 = dict(n=16, q=[1073741441, 1073740609, 1073739937], P=1073739649, t=257)


@pytest.fixture(scope="module")
def o16():
    return O.Oracle(N16["n"], N16["q"], N16["P"], N16["t"])


@pytest.fixture(scope="module")
def k16(o16):
    return o16.keygen(4242)


@pytest.fixture(scope="module")
def o_tiny3():
    p = WL.PARAMS["tiny3"]
    return O.Oracle(p.n, list(p.q), p.P, p.t)


@pytest.fixture(scope="module")
def k_tiny3(o_tiny3):
    return o_tiny3.keygen(1234)


def rng(seed=0):
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------- ChaCha20
def test_chacha20_rfc8439_vectors():
    n = 0
    for line in open(os.path.join(GOLDEN, "chacha20_rfc8439.txt")):
        if line.startswith("#") or not line.strip():
            continue
        k, c, nn, w = [x.strip() for x in line.split("|")]
        key = np.frombuffer(bytes.fromhex(k), dtype="<u4").copy()
        non = np.frombuffer(bytes.fromhex(nn), dtype="<u4").copy()
        out = np.zeros(16, dtype=np.uint32)
        O.lib().ora_chacha20_block(O.P(key), int(c), O.P(non), O.P(out))
        assert [f"{x:08x}" for x in out] == w.split()
        n += 1
    assert n == 2


def _block(seed, kind, ident, counter):
    key = np.zeros(8, dtype=np.uint32)
    key[0], key[1] = seed & 0xFFFFFFFF, seed >> 32
    non = np.array([kind, ident & 0xFFFFFFFF, ident >> 32], dtype=np.uint32)
    out = np.zeros(16, dtype=np.uint32)
    O.lib().ora_chacha20_block(O.P(key), counter, O.P(non), O.P(out))
    return [int(x) for x in out]


def test_sampler_stream_convention():
    """Coefficient k of a 2-word sampler reads stream words 2k (low), 2k+1 (high);
    stream word w is word w % 16 of block w // 16; key = seed words, nonce = (kind, id)."""
    seed, kind, ident, n, q = 0x1234_5678_9ABC_DEF0, 4, (7 << 32) | 3, 64, 1073643521
    words = sum((_block(seed, kind, ident, b) for b in range(8)), [])
    u = np.zeros(n, dtype=np.uint64)
    O.lib().ora_sample_uniform(seed, kind, ident, q, n, O.P(u))
    assert [int(x) for x in u] == [((words[2 * k + 1] << 32) | words[2 * k]) % q for k in range(n)]
    t = np.zeros(n, dtype=np.int64)
    O.lib().ora_sample_ternary(seed, kind, ident, n, O.P(t))
    assert [int(x) for x in t] == [[0, 1, -1][words[k] % 3] for k in range(n)]
    c = np.zeros(n, dtype=np.int64)
    O.lib().ora_sample_cbd(seed, kind, ident, n, O.P(c))
    exp = []
    for k in range(n):
        v = (words[2 * k + 1] << 32) | words[2 * k]
        exp.append(bin(v & (2**21 - 1)).count("1") - bin((v >> 21) & (2**21 - 1)).count("1"))
    assert [int(x) for x in c] == exp


def test_sampler_distributions():
    n = 1 << 16
    t = np.zeros(n, dtype=np.int64)
    O.lib().ora_sample_ternary(99, 1, 0, n, O.P(t))
    for v in (-1, 0, 1):
        assert abs(np.mean(t == v) - 1 / 3) < 0.01
    c = np.zeros(n, dtype=np.int64)
    O.lib().ora_sample_cbd(99, 3, 0, n, O.P(c))
    assert abs(c.mean()) < 0.05 and abs(c.var() - 10.5) < 0.3 and np.abs(c).max() <= 21
    q = 1073643521
    u = np.zeros(n, dtype=np.uint64)
    O.lib().ora_sample_uniform(99, 2, 0, q, n, O.P(u))
    assert u.max() < q and abs(u.astype(np.float64).mean() / q - 0.5) < 0.01
    u2 = np.zeros(n, dtype=np.uint64)
    O.lib().ora_sample_uniform(99, 2, 1, q, n, O.P(u2))   # different id -> different stream
    assert not np.array_equal(u, u2)


# ---------------------------------------------------------------- transform and ring
@pytest.mark.parametrize("n", [16, 64, 256])
def test_ring_mul_matches_schoolbook(n):
    r = rng(n)
    for m in [WL.PARAMS["n16k"].q[0], WL.PARAMS["n16k"].P, 786433, 65537]:
        o = O.Oracle(n, [m], m, 65537 if m != 65537 else 786433)
        for mi in (0, 1, -1):
            mod = [m, m, o.t][mi if mi >= 0 else 2]
            a = O.u64(r.integers(0, mod, n))
            b = O.u64(r.integers(0, mod, n))
            out = np.zeros(n, dtype=np.uint64)
            O.lib().ora_ring_mul(o.ctx, mi, O.P(a), O.P(b), O.P(out))
            assert [int(x) for x in out] == bf.negacyclic(a, b, mod)
            sb = np.zeros(n, dtype=np.uint64)
            O.lib().ora_ring_mul_schoolbook(mod, n, O.P(a), O.P(b), O.P(sb))
            assert np.array_equal(out, sb)


def test_ring_mul_schoolbook_pairs_n4096():
    p = WL.PARAMS["tiny"]
    o = O.Oracle(p.n, list(p.q), p.P, p.t)
    r = rng(7)
    for mi in (0, 2):
        m = (list(p.q) + [p.P])[mi]
        a = O.u64(r.integers(0, m, p.n))
        b = O.u64(r.integers(0, m, p.n))
        x = np.zeros(p.n, dtype=np.uint64)
        y = np.zeros(p.n, dtype=np.uint64)
        O.lib().ora_ring_mul(o.ctx, mi, O.P(a), O.P(b), O.P(x))
        O.lib().ora_ring_mul_schoolbook(m, p.n, O.P(a), O.P(b), O.P(y))
        assert np.array_equal(x, y)


def test_eval_is_evaluation_at_roots(o16):
    """ntt_eval(a)[k] = a(r_k), r_k = r_0^(2k+1), r_0 a primitive 2n-th root (r_k^n = -1)."""
    n = 16
    r = rng(3)
    for mi, m in enumerate(N16["q"] + [N16["P"]]):
        X = np.zeros(n, dtype=np.uint64)
        X[1] = 1
        roots = np.zeros(n, dtype=np.uint64)
        O.lib().ora_ntt_eval(o16.ctx, mi, O.P(X), O.P(roots))
        r0 = int(roots[0])
        assert pow(r0, n, m) == m - 1
        assert [int(v) for v in roots] == [pow(r0, 2 * k + 1, m) for k in range(n)]
        a = O.u64(r.integers(0, m, n))
        A = np.zeros(n, dtype=np.uint64)
        O.lib().ora_ntt_eval(o16.ctx, mi, O.P(a), O.P(A))
        assert [int(v) for v in A] == [sum(int(a[i]) * pow(int(roots[k]), i, m) for i in range(n)) % m for k in range(n)]
        back = np.zeros(n, dtype=np.uint64)
        O.lib().ora_ntt_interp(o16.ctx, mi, O.P(A), O.P(back))
        assert np.array_equal(back, a)


# ---------------------------------------------------------------- batch encoding
def test_psi_t_and_galois_list(o16):
    n, t = 16, N16["t"]
    g = bf.smallest_generator(t)
    assert o16.psi_t == pow(g, (t - 1) // (2 * n), t)
    assert pow(o16.psi_t, n, t) == t - 1
    assert o16.gal == [pow(3, n // 4, 2 * n), pow(3, n // 8, 2 * n), 3, 2 * n - 1]   # s = 4, 2, 1, then the row swap
    for pn in ("tiny", "n16k"):
        p = WL.PARAMS[pn]
        o = O.Oracle(p.n, list(p.q), p.P, p.t)
        assert o.ngal == int(math.log2(p.n))
        assert o.gal[-1] == 2 * p.n - 1 and o.gal[-2] == 3 and o.gal[0] == pow(3, p.n // 4, 2 * p.n)


def test_decode_is_slot_evaluation(o16):
    """slot j = m(psi_t^(e_j)) with the 2 x n/2 hypercube exponents."""
    n, t = 16, N16["t"]
    e = bf.slot_exponents(n)
    m = O.u64(rng(5).integers(0, t, n))
    z = o16.decode(m)
    assert [int(v) for v in z] == [sum(int(m[k]) * pow(o16.psi_t, e[j] * k, t) for k in range(n)) % t for j in range(n)]
    assert np.array_equal(o16.decode(o16.encode(z)), z)


def test_encode_closed_forms(o16, o_tiny3):
    for o in (o16, o_tiny3):
        n, t = o.n, o.t
        e = bf.slot_exponents(n)
        # constant slots -> constant polynomial
        m = o.encode(np.full(n, 42))
        assert m[0] == 42 and not m[1:].any()
        # one-hot slot l -> n^-1 psi_t^(-e_l k)
        ninv = pow(n, -1, t)
        for l in (0, 1, n // 2 - 1, n // 2, n - 1):
            z = np.zeros(n, dtype=np.int64)
            z[l] = 1
            mu = o.encode(z)
            inv = pow(o.psi_t, -1, t)
            ks = range(n) if n <= 64 else [0, 1, 2, 3, n - 1, 777]
            for k in ks:
                assert int(mu[k]) == ninv * pow(inv, e[l] * k, t) % t
            oh = np.zeros(n, dtype=np.uint64)
            O.lib().ora_onehot_plain(o.ctx, l, O.P(oh))
            assert np.array_equal(oh, mu)
        z = rng(1).integers(0, t, n)
        assert np.array_equal(o.decode(o.encode(z)), z.astype(np.uint64))


def test_slot_product_is_negacyclic_product(o16, o_tiny3):
    for o in (o16, o_tiny3):
        n, t = o.n, o.t
        r = rng(11)
        a, b = r.integers(0, t, n), r.integers(0, t, n)
        ma, mb = o.encode(a), o.encode(b)
        prod = np.zeros(n, dtype=np.uint64)
        O.lib().ora_ring_mul(o.ctx, -1, O.P(ma), O.P(mb), O.P(prod))
        if n <= 64:
            assert [int(v) for v in prod] == bf.negacyclic(ma, mb, t)
        assert np.array_equal(o.decode(prod), ((a * b) % t).astype(np.uint64))


def test_automorphisms_rotate_rows(o16):
    n, t = 16, N16["t"]
    h = n // 2
    z = rng(2).integers(0, t, n)
    m = o16.encode(z)
    for r in (1, 2, 3, 5):
        out = np.zeros(n, dtype=np.uint64)
        O.lib().ora_automorph(o16.ctx, -1, pow(3, r, 2 * n), O.P(m), O.P(out))
        assert [int(v) for v in out] == [v % t for v in bf.automorph(m, pow(3, r, 2 * n))]
        dz = o16.decode(out)
        assert np.array_equal(dz[:h], np.roll(z[:h], -r)) and np.array_equal(dz[h:], np.roll(z[h:], -r))
    out = np.zeros(n, dtype=np.uint64)
    O.lib().ora_automorph(o16.ctx, -1, 2 * n - 1, O.P(m), O.P(out))
    dz = o16.decode(out)
    assert np.array_equal(dz[:h], z[h:]) and np.array_equal(dz[h:], z[:h])
    # sigma_g o sigma_h = sigma_{g h}
    g1, g2 = 9, 2 * n - 1
    a = np.zeros(n, dtype=np.uint64)
    b = np.zeros(n, dtype=np.uint64)
    c = np.zeros(n, dtype=np.uint64)
    O.lib().ora_automorph(o16.ctx, -1, g2, O.P(m), O.P(a))
    O.lib().ora_automorph(o16.ctx, -1, g1, O.P(a), O.P(b))
    O.lib().ora_automorph(o16.ctx, -1, (g1 * g2) % (2 * n), O.P(m), O.P(c))
    assert np.array_equal(b, c)


# ---------------------------------------------------------------- BFV constants and keys
@pytest.mark.parametrize("pname", ["tiny", "tiny3", "n16k", "paper_t0", "paper_t1"])
def test_delta_constants(pname):
    p = WL.PARAMS[pname]
    o = O.Oracle(p.n, list(p.q), p.P, p.t)
    Q = o.Q
    assert O.lib().ora_qmod_t(o.ctx) == Q % p.t
    for i, q in enumerate(p.q):
        assert O.lib().ora_qdivt_mod(o.ctx, i) == (Q // p.t) % q
        for v in (0, 1, 2, p.t // 2, p.t // 2 + 1, p.t - 1, 12345 % p.t):
            exact = (Q * v + p.t // 2) // p.t   # round(Q v / t), t odd: no ties
            assert O.lib().ora_delta_mod(o.ctx, i, v) == exact % q


def test_keygen_bruteforce(o16, k16):
    """pk and Galois keys recomputed from the sampled polynomials with schoolbook
    products over the integers."""
    n, q, P, L = 16, N16["q"], N16["P"], 3
    seed = 4242
    s = [int(v) for v in k16.s]
    tern = np.zeros(n, dtype=np.int64)
    O.lib().ora_sample_ternary(seed, 1, 0, n, O.P(tern))
    assert s == [int(v) for v in tern]
    e = np.zeros(n, dtype=np.int64)
    O.lib().ora_sample_cbd(seed, 3, 0, n, O.P(e))
    for j in range(L):
        a = np.zeros(n, dtype=np.uint64)
        O.lib().ora_sample_uniform(seed, 2, j, q[j], n, O.P(a))
        as_ = bf.negacyclic(a, s)
        assert [int(v) for v in k16.pk[1, j]] == [int(v) for v in a]
        assert [int(v) for v in k16.pk[0, j]] == [(-(as_[k] + int(e[k]))) % q[j] for k in range(n)]
    mods = q + [P]
    for gi, g in enumerate(o16.gal):
        sg = bf.automorph(s, g)
        for i in range(L):
            O.lib().ora_sample_cbd(seed, 5, gi * L + i, n, O.P(e))
            for r, m in enumerate(mods):
                a = np.zeros(n, dtype=np.uint64)
                O.lib().ora_sample_uniform(seed, 4, (gi * L + i) * (L + 1) + r, m, n, O.P(a))
                as_ = bf.negacyclic(a, s)
                b = [(-(as_[k] + int(e[k])) + (P * sg[k] if r == i else 0)) % m for k in range(n)]
                assert [int(v) for v in k16.gk[gi, i, 0, r]] == b
                assert np.array_equal(k16.gk[gi, i, 1, r], a)


def test_encrypt_bruteforce(o16, k16):
    n, q, t = 16, N16["q"], N16["t"]
    Q = q[0] * q[1] * q[2]
    seed, cid = 77, 5
    m = O.u64(rng(4).integers(0, t, n))
    ct = o16.encrypt_plain(k16, m, seed, cid)
    u = np.zeros(n, dtype=np.int64)
    e0 = np.zeros(n, dtype=np.int64)
    e1 = np.zeros(n, dtype=np.int64)
    O.lib().ora_sample_ternary(seed, 6, cid, n, O.P(u))
    O.lib().ora_sample_cbd(seed, 7, cid, n, O.P(e0))
    O.lib().ora_sample_cbd(seed, 8, cid, n, O.P(e1))
    for j in range(3):
        p0 = bf.negacyclic(k16.pk[0, j], u)
        p1 = bf.negacyclic(k16.pk[1, j], u)
        assert [int(v) for v in ct[0, j]] == [(p0[k] + int(e0[k]) + (Q * int(m[k]) + t // 2) // t) % q[j] for k in range(n)]
        assert [int(v) for v in ct[1, j]] == [(p1[k] + int(e1[k])) % q[j] for k in range(n)]


def test_key_switch_rounding_bruteforce(o16, k16):
    """out = round(sum_i [d]_{q_i} ksk_i / P) mod q_j, computed with CRT over Q P."""
    n, q, P, L = 16, N16["q"], N16["P"], 3
    mods = q + [P]
    d = np.stack([rng(10 + j).integers(0, q[j], n) for j in range(L)]).astype(np.uint64)
    gi = 2
    ob = np.zeros((L, n), dtype=np.uint64)
    oa = np.zeros((L, n), dtype=np.uint64)
    key = np.ascontiguousarray(k16.gk[gi])
    O.lib().ora_key_switch(o16.ctx, O.P(d), O.P(key), None, O.P(ob), O.P(oa))
    kev = np.ascontiguousarray(k16.gk_ev[gi])
    ob2 = np.zeros_like(ob)
    oa2 = np.zeros_like(oa)
    O.lib().ora_key_switch(o16.ctx, O.P(d), O.P(key), O.P(kev), O.P(ob2), O.P(oa2))
    assert np.array_equal(ob, ob2) and np.array_equal(oa, oa2)
    for x, out in ((0, ob), (1, oa)):
        res = []
        for r, m in enumerate(mods):
            acc = [0] * n
            for i in range(L):
                pr = bf.negacyclic(d[i], key[i, x, r])
                acc = [acc[k] + pr[k] for k in range(n)]
            res.append([v % m for v in acc])
        for k in range(n):
            X, M = bf.crt([res[r][k] for r in range(L + 1)], mods)
            y = (X + (P - 1) // 2) // P      # round(X / P), P odd
            for j in range(L):
                assert int(out[j, k]) == y % q[j]


# ---------------------------------------------------------------- BFV behaviour
def test_dec_enc_many_seeds(o16, k16):
    t = N16["t"]
    for seed in range(40):
        z = rng(seed).integers(0, t, 16)
        ct = o16.encrypt_plain(k16, o16.encode(z), seed, seed)
        m, budget = o16.decrypt_plain(k16, ct)
        assert np.array_equal(o16.decode(m), z.astype(np.uint64)) and budget > 0


def test_dec_enc_tiny3(o_tiny3, k_tiny3):
    o = o_tiny3
    for seed in range(4):
        z = rng(seed).integers(0, o.t, o.n)
        ct = o.encrypt_plain(k_tiny3, o.encode(z), 100 + seed, seed)
        m, budget = o.decrypt_plain(k_tiny3, ct)
        assert np.array_equal(o.decode(m), z.astype(np.uint64))
        # fresh noise: |e0 + e1 s + u e| <= (2n + 1) 21, so >= log2(Q/2t) - log2(that) bits remain
        assert budget > math.log2(o.Q / 2) - math.log2(o.t * (2 * o.n + 1) * 21)


def test_rotation_step_decrypts(o_tiny3, k_tiny3):
    o, k = o_tiny3, k_tiny3
    h = o.n // 2
    z = rng(21).integers(0, o.t, o.n)
    ct0 = o.encrypt_plain(k, o.encode(z), 5, 0)
    for gi in (0, o.ngal - 2, o.ngal - 1):
        ct = ct0.copy()
        O.lib().ora_rotate_add(o.ctx, O.P(k.gk), O.P(k.gk_ev), gi, O.P(ct))
        got, budget = o.decrypt_plain(k, ct)
        got = o.decode(got)
        if gi == o.ngal - 1:
            rot = np.concatenate([z[h:], z[:h]])
        else:
            s = o.n // 4 >> gi
            rot = np.concatenate([np.roll(z[:h], -s), np.roll(z[h:], -s)])
        assert np.array_equal(got, ((z + rot) % o.t).astype(np.uint64)) and budget > 0


def test_trace_invariant_and_mask(o_tiny3, k_tiny3):
    """After the rotate-and-sum every slot holds the sum of all slots; after the
    bias and the one-hot mask only slot l holds it."""
    o, k = o_tiny3, k_tiny3
    x = np.zeros(o.n, dtype=np.int64)
    x[:300] = rng(8).integers(0, 2, 300)
    w = rng(9).integers(-127, 128, o.n)
    xct = o.encrypt_plain(k, o.encode(x), 6, 0)[None]
    wpt = o.encode(w)[None]
    dot = int(np.dot(x, w))
    c = o.pair(k, xct, wpt, 0, 0, stage=100)
    z, budget = o.decrypt_slots(k, c)
    assert np.all(z == o.centre(dot % o.t)) and budget > 0
    l = 1234
    c = o.pair(k, xct, wpt, 17, l, stage=0)
    z, budget = o.decrypt_slots(k, c)
    exp = np.zeros(o.n, dtype=np.int64)
    exp[l] = o.centre((dot + 17) % o.t)
    assert np.array_equal(z, exp) and budget > 0


def test_end_to_end_tiny3_fast_standard_plain(o_tiny3, k_tiny3):
    o, k = o_tiny3, k_tiny3
    wl = WL.tiny(params="tiny3")
    xct = o.encrypt_rows(k, wl.X, seed=31)
    out = o.fast_matmul(k, xct, o.encode_weights(wl.W), wl.b)
    S, budget = o.scores_fast(k, out, wl.rows, wl.classes)
    plain = O.plain_scores(wl.X, wl.W, wl.b, o.t)
    assert np.array_equal(S, plain) and budget > 0
    fct = o.encrypt_cols(k, wl.X, seed=32)
    S2, budget2 = o.scores_standard(k, o.standard_matmul(fct, wl.W, wl.b), wl.rows)
    assert np.array_equal(S2, plain) and budget2 > 0
    assert np.array_equal(O.argmax_lowest(S), O.argmax_lowest(plain))


def test_compression_layout_many_outputs(o16, k16):
    """rows x classes > n: result r = i |Y| + j in output ciphertext r // n, slot r % n."""
    o = o16
    rows, classes, f = 5, 4, 40     # 20 results > 16 slots -> 2 output ciphertexts, K = 3 chunks
    X = rng(12).integers(0, 2, (rows, f))
    W = rng(13).integers(-3, 4, (f, classes))
    b = rng(14).integers(-3, 4, classes)
    xct = o.encrypt_rows(k16, X, seed=3)
    out = o.fast_matmul(k16, xct, o.encode_weights(W), b)
    assert out.shape[0] == 2
    S, budget = o.scores_fast(k16, out, rows, classes)
    assert np.array_equal(S, O.plain_scores(X, W, b, o.t)) and budget > 0
    fct = o.encrypt_cols(k16, X, seed=4)
    S2, _ = o.scores_standard(k16, o.standard_matmul(fct, W, b), rows)
    assert np.array_equal(S2, S)


def test_argmax_ties_lowest():
    S = np.array([[3, 5, 5, 1], [-2, -2, -7, -9]])
    assert list(O.argmax_lowest(S)) == [1, 0]


def test_tiny_two_primes_noise_reading(k_tiny3):
    """With only two 30-bit data primes at n = 4096, t = 65537 the budget is still
    positive through the trace and the bias but the one-hot mask exhausts it:
    the tiny workload checks ciphertext bits at every stage and decrypts only
    through the bias (the three-prime variant carries the end-to-end check)."""
    p = WL.PARAMS["tiny"]
    o = O.Oracle(p.n, list(p.q), p.P, p.t)
    k = o.keygen(1234)
    wl = WL.tiny()
    xct = o.encrypt_rows(k, wl.X, seed=99)
    wpt = o.encode_weights(wl.W)
    c = o.pair(k, xct[0], wpt[0], wl.b[0], 0, stage=100)
    z, budget = o.decrypt_slots(k, c)
    assert budget > 0 and np.all(z == O.plain_scores(wl.X, wl.W, wl.b, o.t)[0, 0])
    c = o.pair(k, xct[0], wpt[0], wl.b[0], 0, stage=0)
    z, budget = o.decrypt_slots(k, c)
    # the noise has wrapped: [t x]_Q is spread over the whole range, so under one
    # bit is left and the one-hot result does not decrypt
    exp = np.zeros(o.n, dtype=np.int64)
    exp[0] = O.plain_scores(wl.X, wl.W, wl.b, o.t)[0, 0]
    assert budget < 1 and not np.array_equal(z, exp)


def test_parameter_sets_are_largest_ntt_primes():
    """The data primes and special prime of every parameter set are the largest
    primes below 2^30 that are 1 mod 2n, in decreasing order; t is prime and 1 mod 2n."""
    from bruteforce import is_prime, ntt_primes
    for p in WL.PARAMS.values():
        L = len(p.q)
        assert list(p.q) + [p.P] == ntt_primes(p.n, L + 1)
        assert is_prime(p.t) and p.t % (2 * p.n) == 1


def _lift(v, t, centred):
    v = int(v) % t
    return v - t if centred and v > (t - 1) // 2 else v


def test_mul_plain_centred_lift_bruteforce(o16):
    """ct x pt lifts each plaintext coefficient (a residue mod t) to its centred
    representative in (-t/2, t/2] before the negacyclic product mod q_j; the
    product is recomputed with Python integers by schoolbook.  The residues are
    chosen so that the [0, t) lift gives a different ciphertext."""
    n, q, t = 16, N16["q"], N16["t"]
    g = rng(31)
    ct = np.stack([np.stack([g.integers(0, qj, n) for qj in q]) for _ in range(2)]).astype(np.uint64)
    w_t = O.u64(g.integers(0, t, n))
    w_t[:4] = [t - 1, (t + 1) // 2, (t - 1) // 2, 0]   # both sides of t/2
    out = np.zeros_like(ct)
    O.lib().ora_mul_plain(o16.ctx, O.P(np.ascontiguousarray(ct)), O.P(w_t), O.P(out))
    for centred in (True, False):
        w = [_lift(v, t, centred) for v in w_t]
        ref = np.array([[bf.negacyclic(ct[x, j], w, q[j]) for j in range(3)] for x in range(2)], dtype=np.uint64)
        assert np.array_equal(out, ref) == centred


def test_standard_scalar_centred_lift_bruteforce(o16):
    """Standard baseline: Y_j = sum_k fct_k w_kj + Delta(b_j) with each scalar weight
    lifted to its centred representative; recomputed with Python integers.  A
    [0, t) lift of the negative weights gives a different ciphertext."""
    n, q, t = 16, N16["q"], N16["t"]
    Q = q[0] * q[1] * q[2]
    g = rng(32)
    f, classes = 5, 3
    fct = np.stack([np.stack([np.stack([g.integers(0, qj, n) for qj in q]) for _ in range(2)])
                    for _ in range(f)]).astype(np.uint64)
    W = g.integers(-127, 128, (f, classes))
    W[0, 0], W[1, 0] = -1, -127
    b = g.integers(-127, 128, classes)
    out = o16.standard_matmul(fct, W, b)
    for centred in (True, False):
        ok = True
        for j in range(classes):
            for x in range(2):
                for li, qj in enumerate(q):
                    acc = [sum(int(fct[k, x, li, e]) * _lift(W[k, j], t, centred) for k in range(f)) for e in range(n)]
                    if x == 0:
                        bt = int(b[j]) % t
                        acc[0] += (Q * bt + t // 2) // t      # Delta(b_j) = round(Q b / t) on coefficient 0
                    ok &= [v % qj for v in acc] == [int(v) for v in out[j, x, li]]
        assert ok == centred


# ---------------------------------------------------------------- the paper's precision point
def test_paper_precision_arithmetic():
    """Section "Private inference protocol": t0 = 1073872897 (30 bits) and t1 =
    114689 (16 bits) are primes that batch at n = 8192 (both 1 mod 2n); t1 does
    not at n = 16384.  Outputs need 8 + s_x + s_w + ceil(log2 f) = 44 bits at
    f = 40,960, within the signed range of t0 t1 (about 2^45.8)."""
    from bruteforce import is_prime
    t0, t1 = WL.T_PAIR
    assert (t0, t1) == (1073872897, 114689) and is_prime(t0) and is_prime(t1)
    assert t0 % 16384 == 1 and t1 % 16384 == 1 and t1 % 32768 != 1
    assert 29 < math.log2(t0) < 30.01 and 16 < math.log2(t1) < 17
    need = 8 + WL.S_X + WL.S_W + math.ceil(math.log2(40960))
    assert need == 44 and 2 ** need < (t0 * t1) // 2


def test_crt_pair_bruteforce():
    """crt_pair returns the unique integer of (-t0 t1 / 2, t0 t1 / 2] with the
    given residues: checked on integers drawn over the whole range and at its
    edges, with residues given in [0, t) and centred."""
    t0, t1 = WL.T_PAIR
    M = t0 * t1
    half = M // 2
    r = rng(11)
    zs = [0, 1, -1, half, -half + 1, half - 1, -half + 2, t0, -t0, t1, -t1, t0 * 7, 2 ** 44, -(2 ** 44)]
    zs += [int(v) for v in r.integers(-half + 1, half + 1, size=200, dtype=np.int64)]
    r0 = np.array([z % t0 for z in zs], dtype=object)
    r1 = np.array([z % t1 for z in zs], dtype=object)
    assert list(O.crt_pair(r0, r1, t0, t1)) == zs
    c0 = np.array([v - t0 if v > (t0 - 1) // 2 else v for v in r0], dtype=object)
    c1 = np.array([v - t1 if v > (t1 - 1) // 2 else v for v in r1], dtype=object)
    assert list(O.crt_pair(c0, c1, t0, t1)) == zs
    # brute force on small coprime moduli: every residue pair, against a search
    for a, b in ((5, 7), (7, 12), (9, 4)):
        for x in range(a):
            for y in range(b):
                z = int(O.crt_pair(np.array([x], dtype=object), np.array([y], dtype=object), a, b)[0])
                cands = [v for v in range(-(a * b) // 2, (a * b) // 2 + 1) if v % a == x and v % b == y
                         and -(a * b) / 2 < v <= (a * b) / 2]
                assert [z] == cands


def test_fixed_point_closed_forms():
    """Values that are exact multiples of 2^-s map to the integer itself; halves
    go to the even neighbour; signs are kept."""
    for s in (WL.S_X, WL.S_W, WL.S_X + WL.S_W):
        k = np.array([0, 1, -1, 5, -77, 2 ** 13, -(2 ** 13)], dtype=np.int64)
        assert np.array_equal(O.fixed_point(k / 2.0 ** s, s), k)
        assert list(O.fixed_point(np.array([0.5, 1.5, 2.5, -0.5, -1.5]) / 2.0 ** s, s)) == [0, 2, 2, 0, -2]
        assert list(O.fixed_point(np.array([0.49, 0.51, -0.51]) / 2.0 ** s, s)) == [0, 1, -1]


def test_paper_point_oracle_end_to_end():
    """n = 8192 with the CRT pair: Algorithm 1 run once per plaintext modulus (each
    under its own keys) decrypts, after recombination, to exactly X_s W_s + b_s,
    the scaled integer result, which exceeds t0 (so neither modulus alone holds it)."""
    t0, t1 = WL.T_PAIR
    wl = WL.real_workload("paper_1x300x11", 1, 300, 11, 0.2, WL.BASE_SEED + 50)
    Xs, Ws = O.fixed_point(wl.X, WL.S_X), O.fixed_point(wl.W, WL.S_W)
    bs = O.fixed_point(wl.b, WL.S_X + WL.S_W)
    plain = O.plain_fixed_scores(Xs, Ws, bs)
    assert max(abs(int(v)) for v in plain.flat) > t0 // 2
    res = []
    for k, pname in enumerate(("paper_t0", "paper_t1")):
        p = WL.PARAMS[pname]
        o = O.Oracle(p.n, list(p.q), p.P, p.t)
        # encoding round trip and the constant closed form at this ring and t
        z = rng(k).integers(0, p.t, p.n)
        assert np.array_equal(o.decode(o.encode(z)), z.astype(np.uint64))
        m = o.encode(np.full(p.n, 5))
        assert m[0] == 5 and not m[1:].any()
        keys = o.keygen(900 + k)
        y = o.fast_matmul(keys, o.encrypt_rows(keys, Xs, seed=31), o.encode_weights(Ws), bs)
        S, budget = o.scores_fast(keys, y, wl.rows, wl.classes)
        assert budget > 20
        assert np.array_equal(S, O.plain_scores(Xs, Ws, bs, p.t))
        res.append(S)
    assert np.array_equal(O.crt_pair(res[0], res[1], t0, t1), plain)
