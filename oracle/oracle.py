"""Python side of the CPU oracle for the encrypted LR matrix multiplication (BFV).

Test infrastructure only: tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg are the only users.  It shares no code with the HIP path.

Paper: arXiv 2204.05496, section "Private inference protocol" (scale, encode,
encrypt, server product, decrypt, decode), Algorithm 1 (fast matrix
multiplication), section "Comparison to standard LR" (baseline), section
"Approximation of non-linear function in private inference" (argmax).

Heavy ring arithmetic runs in ``bfv_oracle.c`` (plain C, '%' arithmetic,
textbook transform).  Decryption, the noise budget and every big-integer
constant are computed here with Python integers, which makes them exact by
construction.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bfv_oracle.c")
_LIB = os.path.join(_HERE, "libbfv_oracle.so")
# a prebuilt oracle library in its place (the sanitizer build of the CPU tests)
_LIB_OVERRIDE = os.environ.get("LRHE_ORACLE_LIB")

u64p = ctypes.POINTER(ctypes.c_uint64)
i64p = ctypes.POINTER(ctypes.c_int64)
u32p = ctypes.POINTER(ctypes.c_uint32)


def build(force: bool = False) -> str:
    """Compile the C oracle (gcc, -O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(_LIB_OVERRIDE or build())
        vp = ctypes.c_void_p
        L.ora_ctx_new.restype = vp
        L.ora_ctx_new.argtypes = [ctypes.c_int, ctypes.c_int, u64p, ctypes.c_uint64]
        L.ora_ctx_free.argtypes = [vp]
        for name, res in [("ora_ngal", ctypes.c_int), ("ora_psi_t", ctypes.c_uint64), ("ora_qmod_t", ctypes.c_uint64)]:
            getattr(L, name).restype = res
            getattr(L, name).argtypes = [vp]
        L.ora_gal.restype = ctypes.c_uint32
        L.ora_gal.argtypes = [vp, ctypes.c_int]
        L.ora_qdivt_mod.restype = ctypes.c_uint64
        L.ora_qdivt_mod.argtypes = [vp, ctypes.c_int]
        L.ora_slot_pos.restype = ctypes.c_uint32
        L.ora_slot_pos.argtypes = [vp, ctypes.c_int]
        L.ora_delta_mod.restype = ctypes.c_uint64
        L.ora_delta_mod.argtypes = [vp, ctypes.c_int, ctypes.c_uint64]
        L.ora_gk_words.restype = ctypes.c_size_t
        L.ora_gk_words.argtypes = [vp]
        L.ora_chacha20_block.argtypes = [u32p, ctypes.c_uint32, u32p, u32p]
        L.ora_sample_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, u64p]
        L.ora_sample_ternary.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, i64p]
        L.ora_sample_cbd.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, i64p]
        L.ora_ring_mul_schoolbook.argtypes = [ctypes.c_uint64, ctypes.c_int, u64p, u64p, u64p]
        L.ora_ring_mul.argtypes = [vp, ctypes.c_int, u64p, u64p, u64p]
        L.ora_ntt_eval.argtypes = [vp, ctypes.c_int, u64p, u64p]
        L.ora_ntt_interp.argtypes = [vp, ctypes.c_int, u64p, u64p]
        L.ora_automorph.argtypes = [vp, ctypes.c_int, ctypes.c_uint32, u64p, u64p]
        L.ora_encode.argtypes = [vp, u64p, u64p]
        L.ora_decode.argtypes = [vp, u64p, u64p]
        L.ora_keygen.argtypes = [vp, ctypes.c_uint64, i64p, u64p, u64p]
        L.ora_encrypt.argtypes = [vp, u64p, u64p, ctypes.c_uint64, ctypes.c_uint64, u64p]
        L.ora_mul_plain.argtypes = [vp, u64p, u64p, u64p]
        L.ora_add.argtypes = [vp, u64p, u64p, u64p]
        L.ora_add_const.argtypes = [vp, ctypes.c_uint64, u64p]
        L.ora_key_switch.argtypes = [vp, u64p, u64p, u64p, u64p, u64p]
        L.ora_gk_transform.argtypes = [vp, u64p, u64p]
        L.ora_rotate_add.argtypes = [vp, u64p, u64p, ctypes.c_int, u64p]
        L.ora_onehot_plain.argtypes = [vp, ctypes.c_int, u64p]
        L.ora_pair.argtypes = [vp, u64p, u64p, u64p, u64p, ctypes.c_int, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, u64p]
        L.ora_fast_matmul.argtypes = [vp, u64p, u64p, u64p, u64p, u64p, ctypes.c_int, ctypes.c_int, ctypes.c_int, u64p]
        L.ora_standard_matmul.argtypes = [vp, u64p, u64p, u64p, ctypes.c_int, ctypes.c_int, u64p]
        _lib = L
    return _lib


def P(a: np.ndarray):
    """ctypes pointer into a C-contiguous numpy array."""
    assert a.flags["C_CONTIGUOUS"]
    if a.dtype == np.uint64:
        return a.ctypes.data_as(u64p)
    if a.dtype == np.int64:
        return a.ctypes.data_as(i64p)
    if a.dtype == np.uint32:
        return a.ctypes.data_as(u32p)
    raise TypeError(a.dtype)


def u64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint64)


@dataclass
class Keys:
    s: np.ndarray      # int64 [n], ternary secret
    pk: np.ndarray     # uint64 [2][L][n]
    gk: np.ndarray     # uint64 [ngal][L][2][L+1][n] (coefficient form)
    gk_ev: np.ndarray  # same key, transform form per modulus


class Oracle:
    """BFV over R = Z[X]/(X^n + 1) with data primes q (L of them), special prime P
    and plaintext modulus t.  Ciphertexts: uint64 [2][L][n], coefficient form."""

    def __init__(self, n: int, q: list[int], P: int, t: int):
        self.n, self.q, self.P, self.t = n, list(q), P, t
        self.L = len(q)
        self.Q = 1
        for x in q:
            self.Q *= x
        self._qp = u64(self.q + [P])
        self.ctx = lib().ora_ctx_new(n, self.L, P_(self._qp), t)
        if not self.ctx:
            raise ValueError("oracle: invalid parameters")
        self.ngal = lib().ora_ngal(self.ctx)
        self.gal = [lib().ora_gal(self.ctx, i) for i in range(self.ngal)]
        self.psi_t = lib().ora_psi_t(self.ctx)

    def __del__(self):
        if getattr(self, "ctx", None):
            lib().ora_ctx_free(self.ctx)
            self.ctx = None

    # sizes
    @property
    def ct_shape(self):
        return (2, self.L, self.n)

    def zeros_ct(self, count: int = 1) -> np.ndarray:
        return np.zeros((count, 2, self.L, self.n), dtype=np.uint64)

    # --- encoding (section "Private inference protocol": n values per polynomial) ---
    def encode(self, slots) -> np.ndarray:
        z = u64(np.asarray(slots, dtype=np.int64) % self.t)
        m = np.zeros(self.n, dtype=np.uint64)
        lib().ora_encode(self.ctx, P(z), P(m))
        return m

    def decode(self, m) -> np.ndarray:
        m = u64(m)
        z = np.zeros(self.n, dtype=np.uint64)
        lib().ora_decode(self.ctx, P(m), P(z))
        return z

    def centre(self, v):
        v = np.asarray(v, dtype=np.int64)
        return np.where(v > (self.t - 1) // 2, v - self.t, v)

    # --- keys and encryption ---
    def keygen(self, seed: int, galois: bool = True) -> Keys:
        s = np.zeros(self.n, dtype=np.int64)
        pk = np.zeros((2, self.L, self.n), dtype=np.uint64)
        gk = np.zeros(lib().ora_gk_words(self.ctx), dtype=np.uint64) if galois else np.zeros(1, dtype=np.uint64)
        lib().ora_keygen(self.ctx, seed, P(s), P(pk), P(gk) if galois else None)
        gk_ev = np.zeros_like(gk)
        if galois:
            lib().ora_gk_transform(self.ctx, P(gk), P(gk_ev))
            shape = (self.ngal, self.L, 2, self.L + 1, self.n)
            gk, gk_ev = gk.reshape(shape), gk_ev.reshape(shape)
        return Keys(s, pk, gk, gk_ev)

    def encrypt_plain(self, keys: Keys, m, seed: int, ct_id: int) -> np.ndarray:
        ct = np.zeros((2, self.L, self.n), dtype=np.uint64)
        lib().ora_encrypt(self.ctx, P(keys.pk), P(u64(m)), seed, ct_id, P(ct))
        return ct

    def encrypt_rows(self, keys: Keys, X: np.ndarray, seed: int, row0: int = 0) -> np.ndarray:
        """Fast layout: row i, chunk k holds X[i, k n : (k+1) n] in its slots
        (zero past f); ciphertext id = (row0 + i) K + k.  Returns [rows][K][2][L][n]."""
        rows, f = X.shape
        K = -(-f // self.n)
        out = np.zeros((rows, K, 2, self.L, self.n), dtype=np.uint64)
        for i in range(rows):
            for k in range(K):
                z = np.zeros(self.n, dtype=np.int64)
                chunk = X[i, k * self.n:(k + 1) * self.n]
                z[:len(chunk)] = chunk
                out[i, k] = self.encrypt_plain(keys, self.encode(z), seed, (row0 + i) * K + k)
        return out

    def encrypt_cols(self, keys: Keys, X: np.ndarray, seed: int, features=None) -> np.ndarray:
        """Standard layout: one ciphertext per feature k with X[:, k] in the slots
        (individuals in slots); ciphertext id = k.  Returns [f][2][L][n]."""
        rows, f = X.shape
        assert rows <= self.n
        feats = range(f) if features is None else features
        out = np.zeros((len(feats), 2, self.L, self.n), dtype=np.uint64)
        for o, k in enumerate(feats):
            z = np.zeros(self.n, dtype=np.int64)
            z[:rows] = X[:, k]
            out[o] = self.encrypt_plain(keys, self.encode(z), seed, k)
        return out

    def encode_weights(self, W: np.ndarray) -> np.ndarray:
        """W^T packed per chunk: plaintext (class j, chunk k) holds W[k n + s, j] in slot s.
        Returns values mod t, [classes][K][n]."""
        f, classes = W.shape
        K = -(-f // self.n)
        out = np.zeros((classes, K, self.n), dtype=np.uint64)
        for j in range(classes):
            for k in range(K):
                z = np.zeros(self.n, dtype=np.int64)
                col = W[k * self.n:(k + 1) * self.n, j]
                z[:len(col)] = col
                out[j, k] = self.encode(z)
        return out

    # --- Algorithm 1 pieces ---
    def pair(self, keys: Keys, xct, wpt, bias_t: int, slot: int, stage: int = 0) -> np.ndarray:
        xct, wpt = u64(xct), u64(wpt)
        K = wpt.shape[0]
        out = np.zeros((2, self.L, self.n), dtype=np.uint64)
        lib().ora_pair(self.ctx, P(keys.gk), P(keys.gk_ev), P(xct), P(wpt), K, int(bias_t) % self.t, slot, stage, P(out))
        return out

    def fast_matmul(self, keys: Keys, xct, wpt, bias) -> np.ndarray:
        xct, wpt = u64(xct), u64(wpt)
        rows, K = xct.shape[0], xct.shape[1]
        classes = wpt.shape[0]
        bias_t = u64(np.asarray(bias, dtype=np.int64) % self.t)
        nout = -(-rows * classes // self.n)
        out = np.zeros((nout, 2, self.L, self.n), dtype=np.uint64)
        lib().ora_fast_matmul(self.ctx, P(keys.gk), P(keys.gk_ev), P(xct), P(wpt), P(bias_t), rows, classes, K, P(out))
        return out

    def standard_matmul(self, fct, W: np.ndarray, bias) -> np.ndarray:
        fct = u64(fct)
        f, classes = W.shape
        W_t = u64(np.asarray(W, dtype=np.int64) % self.t)
        bias_t = u64(np.asarray(bias, dtype=np.int64) % self.t)
        out = np.zeros((classes, 2, self.L, self.n), dtype=np.uint64)
        lib().ora_standard_matmul(self.ctx, P(fct), P(W_t), P(bias_t), f, classes, P(out))
        return out

    # --- decryption (exact, Python integers) ---
    def _phase(self, keys: Keys, ct) -> list[int]:
        """x = [c0 + c1 s]_Q as integers in [0, Q), via CRT."""
        ct = u64(ct)
        n, L = self.n, self.L
        limbs = []
        for j in range(L):
            qj = self.q[j]
            sj = u64(np.asarray(keys.s, dtype=np.int64) % qj)
            prod = np.zeros(n, dtype=np.uint64)
            lib().ora_ring_mul(self.ctx, j, P(u64(ct[1, j])), P(sj), P(prod))
            limbs.append(((ct[0, j].astype(object) + prod.astype(object)) % qj))
        x = [0] * n
        for j in range(L):
            qj = self.q[j]
            Mj = self.Q // qj
            cj = Mj * pow(Mj, -1, qj)
            lj = limbs[j]
            for k in range(n):
                x[k] += int(lj[k]) * cj
        return [v % self.Q for v in x]

    def decrypt_plain(self, keys: Keys, ct) -> tuple[np.ndarray, float]:
        """m = round(t x / Q) mod t; also the remaining noise budget in bits,
        log2(Q/2) - log2(max |[t x]_Q|) (decryption is correct while it is > 0)."""
        x = self._phase(keys, ct)
        Q, t = self.Q, self.t
        m = np.array([((t * v + Q // 2) // Q) % t for v in x], dtype=np.uint64)
        worst = 0
        for v in x:
            w = (t * v) % Q
            if w > Q // 2:
                w = Q - w
            worst = max(worst, w)
        import math
        budget = math.log2(Q / 2) - (math.log2(worst) if worst > 0 else 0.0)
        return m, budget

    def decrypt_slots(self, keys: Keys, ct) -> tuple[np.ndarray, float]:
        m, budget = self.decrypt_plain(keys, ct)
        return self.centre(self.decode(m)), budget

    def scores_fast(self, keys: Keys, out_cts, rows: int, classes: int):
        """Result r = i classes + j sits in output ciphertext r // n, slot r % n."""
        dec = [self.decrypt_slots(keys, c) for c in out_cts]
        S = np.zeros((rows, classes), dtype=np.int64)
        for r in range(rows * classes):
            S[r // classes, r % classes] = dec[r // self.n][0][r % self.n]
        return S, min(b for _, b in dec)

    def scores_standard(self, keys: Keys, out_cts, rows: int):
        dec = [self.decrypt_slots(keys, c) for c in out_cts]
        S = np.stack([d[0][:rows] for d in dec], axis=1)
        return S, min(b for _, b in dec)


def P_(a):
    return P(a)


def plain_scores(X: np.ndarray, W: np.ndarray, bias, t: int) -> np.ndarray:
    """The result the method must reach: [X W + b]_t centred into (-t/2, t/2]
    (section "Private inference protocol"; integer arithmetic, exact)."""
    X64, W64, b64 = (np.asarray(a, dtype=np.int64) for a in (X, W, bias))
    bound = int(np.abs(X64).max(initial=0)) * int(np.abs(W64).max(initial=0)) * X64.shape[1] + \
        int(np.abs(b64).max(initial=0))
    if bound < 2**62:   # every partial sum fits: int64 arithmetic is exact
        S = (X64 @ W64 + b64[None, :]) % t
    else:
        S = (X64.astype(object) @ W64.astype(object)) + b64.astype(object)[None, :]
        S = np.vectorize(lambda v: int(v) % t)(S).astype(np.int64)
    return np.where(S > (t - 1) // 2, S - t, S)


def fixed_point(a, bits: int) -> np.ndarray:
    """The paper's fixed-point conversion (section "Private inference
    protocol"): a value is multiplied by 2^bits and taken to the nearest
    integer (ties to even), int64."""
    return np.rint(np.asarray(a, dtype=np.float64) * float(2 ** bits)).astype(np.int64)


def plain_fixed_scores(Xs: np.ndarray, Ws: np.ndarray, bs) -> np.ndarray:
    """The exact integer result of the scaled computation, X_s W_s + b_s, with
    no reduction (it is what the CRT pair must give back); Python integers."""
    X64, W64, b64 = (np.asarray(a, dtype=np.int64) for a in (Xs, Ws, bs))
    bound = int(np.abs(X64).max(initial=0)) * int(np.abs(W64).max(initial=0)) * X64.shape[1] + \
        int(np.abs(b64).max(initial=0))
    if bound < 2**62:   # every partial sum fits: int64 arithmetic is exact
        return (X64 @ W64 + b64[None, :]).astype(object)
    return X64.astype(object) @ W64.astype(object) + b64.astype(object)[None, :]


def crt_pair(r0, r1, t0: int, t1: int) -> np.ndarray:
    """The integer z in (-t0 t1 / 2, t0 t1 / 2] with z = r0 mod t0 and z = r1 mod
    t1 (the Chinese remainder theorem over the paper's plaintext pair), for
    arrays of residues (any representatives); Python integers."""
    M = t0 * t1
    inv = pow(t0, -1, t1)
    r0 = np.asarray(r0, dtype=object)
    r1 = np.asarray(r1, dtype=object)
    out = np.empty(r0.shape, dtype=object)
    for idx in np.ndindex(r0.shape):
        a, b = int(r0[idx]) % t0, int(r1[idx]) % t1
        z = a + t0 * (((b - a) * inv) % t1)
        out[idx] = z - M if z > M // 2 else z
    return out


def argmax_lowest(S: np.ndarray) -> np.ndarray:
    """Predicted class = argmax_j score (section "Approximation of non-linear
    function in private inference"); ties go to the lowest class index."""
    return np.argmax(S, axis=1)
