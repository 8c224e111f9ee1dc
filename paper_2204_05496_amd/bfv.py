"""Python front end of liblrhe: the calls of the paper's private inference
protocol (section "Private inference protocol") on one MI355X.

    ctx = Context(n, q, P, t)             # parameters {n, T} of the protocol
    keys = ctx.keygen(seed)               # client: sk (host), pk, Galois keys (HBM)
    xct = ctx.encrypt_rows(keys, X, seed) # client: encode + encrypt |X| x f
    model = ctx.model(W, b)               # server: encode W^T and the biases
    y = ctx.matmul_fast(keys, model, xct, rows)      # server: Algorithm 1
    S, budget = ctx.scores_fast(keys, y, rows, classes)  # client: decrypt, decode
    cls = S.argmax(1)                     # predicted class

Ciphertext tensors are torch.int32 [count, 2, L, n] on the GPU holding uint32
residues (evaluation form).  All arithmetic happens in the HIP library.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import native as N


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclass
class Keys:
    ctx: "Context"
    sk: ctypes.c_void_p
    pk: ctypes.c_void_p
    gk: ctypes.c_void_p

    def close(self):
        lib = N.lib()
        if self.sk:
            lib.lrhe_sk_destroy(self.sk)
        if self.pk:
            lib.lrhe_pk_destroy(self.pk)
        if self.gk:
            lib.lrhe_gk_destroy(self.gk)
        self.sk = self.pk = self.gk = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Model:
    ctx: "Context"
    handle: ctypes.c_void_p
    f: int
    classes: int

    def close(self):
        if self.handle:
            N.lib().lrhe_model_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """BFV context on one device (device < 0: host-only client context)."""

    def __init__(self, n: int, q, P: int, t: int, device: int = 0, allow_insecure: bool = False):
        lib = N.lib()
        self._q = (ctypes.c_uint32 * len(q))(*q)
        prm = N.LrheParams(n, len(q), self._q, P, t, 1 if allow_insecure else 0)
        h = ctypes.c_void_p()
        N.check(lib.lrhe_ctx_create(ctypes.byref(prm), device, ctypes.byref(h)))
        self.h = h
        self.device = device
        nn, LL, ng, cw = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint64()
        N.check(lib.lrhe_ctx_info(h, ctypes.byref(nn), ctypes.byref(LL), ctypes.byref(ng), ctypes.byref(cw)))
        self.n, self.L, self.ngal, self.ct_words = nn.value, LL.value, ng.value, cw.value
        self.q, self.P, self.t = list(q), P, t
        g = ctypes.c_uint32()
        self.gal = []
        for i in range(self.ngal):
            N.check(lib.lrhe_galois_element(h, i, ctypes.byref(g)))
            self.gal.append(g.value)

    @classmethod
    def from_params(cls, p, device: int = 0):
        return cls(p.n, list(p.q), p.P, p.t, device=device, allow_insecure=p.insecure)

    def close(self):
        if getattr(self, "h", None):
            N.lib().lrhe_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- buffers
    def _dev(self):
        return _torch().device("cuda", self.device)

    def empty_ct(self, count: int):
        torch = _torch()
        return torch.empty((count, 2, self.L, self.n), dtype=torch.int32, device=self._dev())

    def workspace(self, op: int, rows: int = 0, f: int = 0, classes: int = 0):
        b = ctypes.c_uint64()
        N.check(N.lib().lrhe_workspace_bytes(self.h, op, rows, f, classes, ctypes.byref(b)))
        torch = _torch()
        return torch.empty(max(int(b.value), 256), dtype=torch.uint8, device=self._dev())

    def K(self, f: int) -> int:
        return -(-f // self.n)

    # ---------------------------------------------------------------- keys
    def keygen(self, seed: int, galois: bool = True) -> Keys:
        sk, pk, gk = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        N.check(N.lib().lrhe_keygen(self.h, seed, 1 if galois else 0, ctypes.byref(sk), ctypes.byref(pk),
                                    ctypes.byref(gk) if galois else None))
        return Keys(self, sk, pk, gk if galois else None)

    def export_pk(self, keys: Keys) -> np.ndarray:
        out = np.zeros((2, self.L, self.n), dtype=np.uint32)
        N.check(N.lib().lrhe_pk_export(self.h, keys.pk, N.ptr(out)))
        return out

    def export_gk(self, keys: Keys) -> np.ndarray:
        out = np.zeros((self.ngal, self.L, 2, self.L + 1, self.n), dtype=np.uint32)
        N.check(N.lib().lrhe_gk_export(self.h, keys.gk, N.ptr(out)))
        return out

    def export_sk(self, keys: Keys) -> np.ndarray:
        out = np.zeros(self.n, dtype=np.int8)
        N.check(N.lib().lrhe_sk_export(self.h, keys.sk, N.ptr(out)))
        return out

    # ---------------------------------------------------------------- wire format
    def _wire_bytes(self, kind: int, count: int = 1) -> int:
        b = ctypes.c_uint64()
        N.check(N.lib().lrhe_wire_bytes(self.h, kind, count, ctypes.byref(b)))
        return b.value

    def serialize_ct(self, ct) -> bytes:
        """Ciphertexts (device tensor, or host uint32 array) as one wire message."""
        host = isinstance(ct, np.ndarray)
        if host:
            ct = np.ascontiguousarray(ct, dtype=np.uint32)
        else:
            ct = ct.contiguous()
        count = ct.shape[0]
        out = np.empty(self._wire_bytes(N.WIRE_CT, count), dtype=np.uint8)
        N.check(N.lib().lrhe_ct_serialize(self.h, N.ptr(ct), count, N.CT_HOST if host else 0, N.ptr(out), out.size,
                                          None if host else _stream()))
        return out.tobytes()

    def deserialize_ct(self, msg: bytes, out=None, host: bool = False):
        """A ciphertext message into a device tensor (or into `out`; host=True: a
        host uint32 array)."""
        buf = np.frombuffer(msg, dtype=np.uint8)
        count = int.from_bytes(msg[40:48], "little") if len(msg) >= 64 else 0
        if out is None:
            out = np.zeros((count, 2, self.L, self.n), dtype=np.uint32) if host else self.empty_ct(count)
        got = ctypes.c_uint32()
        N.check(N.lib().lrhe_ct_deserialize(self.h, N.ptr(buf), buf.size, N.CT_HOST if host else 0, N.ptr(out),
                                            out.shape[0], ctypes.byref(got), None if host else _stream()))
        return out[:got.value]

    def serialize_key(self, keys: Keys, kind: int) -> bytes:
        """One key of `keys` (N.WIRE_GK, N.WIRE_PK or N.WIRE_SK) as a wire message."""
        key = {N.WIRE_GK: keys.gk, N.WIRE_PK: keys.pk, N.WIRE_SK: keys.sk}[kind]
        out = np.empty(self._wire_bytes(kind), dtype=np.uint8)
        N.check(N.lib().lrhe_key_serialize(self.h, kind, key, N.ptr(out), out.size))
        return out.tobytes()

    def load_keys(self, sk: bytes = None, pk: bytes = None, gk: bytes = None) -> Keys:
        """Keys from wire messages (any subset): the client keeps sk and pk, the
        server receives gk."""
        handles = []
        for msg, fn in ((sk, N.lib().lrhe_sk_deserialize), (pk, N.lib().lrhe_pk_deserialize),
                        (gk, N.lib().lrhe_gk_deserialize)):
            h = ctypes.c_void_p()
            if msg is not None:
                buf = np.frombuffer(msg, dtype=np.uint8)
                N.check(fn(self.h, N.ptr(buf), buf.size, ctypes.byref(h)))
            handles.append(h if msg is not None else None)
        return Keys(self, *handles)

    # ---------------------------------------------------------------- client
    def _as_dev_i64(self, X):
        torch = _torch()
        if isinstance(X, np.ndarray):
            X = torch.from_numpy(np.ascontiguousarray(X, dtype=np.int64))
        return X.to(device=self._dev(), dtype=torch.int64).contiguous()

    def encrypt_rows(self, keys: Keys, X, seed: int, id0: int = 0, out=None, ws=None):
        """Fast layout: [rows * K] ciphertexts (row i, chunk k at i K + k)."""
        Xd = self._as_dev_i64(X)
        rows, f = Xd.shape
        K = self.K(f)
        out = self.empty_ct(rows * K) if out is None else out
        ws = self.workspace(N.WS_ENCRYPT_ROWS, rows, f) if ws is None else ws
        N.check(N.lib().lrhe_encrypt_rows(self.h, keys.pk, N.ptr(Xd), rows, f, seed, id0, N.ptr(out), N.ptr(ws),
                                          ws.numel(), _stream()))
        return out

    def encrypt_cols(self, keys: Keys, X, seed: int, id0: int = 0, out=None, ws=None):
        """Standard layout: f ciphertexts, individuals in slots."""
        Xd = self._as_dev_i64(X)
        rows, f = Xd.shape
        out = self.empty_ct(f) if out is None else out
        ws = self.workspace(N.WS_ENCRYPT_COLS, rows, f) if ws is None else ws
        N.check(N.lib().lrhe_encrypt_cols(self.h, keys.pk, N.ptr(Xd), rows, f, seed, id0, N.ptr(out), N.ptr(ws),
                                          ws.numel(), _stream()))
        return out

    def decrypt_slots(self, keys: Keys, ct):
        cnt = ct.shape[0]
        slots = np.zeros((cnt, self.n), dtype=np.int64)
        bud = np.zeros(cnt, dtype=np.float64)
        N.check(N.lib().lrhe_decrypt_slots(self.h, keys.sk, N.ptr(ct.contiguous()), cnt, N.ptr(slots), N.ptr(bud),
                                           _stream()))
        return slots, bud

    def decrypt_slots_host(self, keys: Keys, ct_host: np.ndarray):
        ct_host = np.ascontiguousarray(ct_host, dtype=np.uint32)
        cnt = ct_host.shape[0]
        slots = np.zeros((cnt, self.n), dtype=np.int64)
        bud = np.zeros(cnt, dtype=np.float64)
        N.check(N.lib().lrhe_decrypt_slots_host(self.h, keys.sk, N.ptr(ct_host), cnt, N.ptr(slots), N.ptr(bud)))
        return slots, bud

    def _scores(self, fn, keys: Keys, y, rows: int, classes: int):
        S = np.zeros((rows, classes), dtype=np.int64)
        bud = ctypes.c_double()
        if isinstance(y, np.ndarray):
            y = np.ascontiguousarray(y, dtype=np.uint32)
            N.check(fn(self.h, keys.sk, N.ptr(y), rows, classes, N.CT_HOST, N.ptr(S), ctypes.byref(bud), None))
        else:
            N.check(fn(self.h, keys.sk, N.ptr(y.contiguous()), rows, classes, 0, N.ptr(S), ctypes.byref(bud),
                       _stream()))
        return S, bud.value

    def scores_fast(self, keys: Keys, y, rows: int, classes: int):
        """Class scores of Algorithm 1's outputs (device tensor or host uint32 array)."""
        return self._scores(N.lib().lrhe_decrypt_scores, keys, y, rows, classes)

    def scores_standard(self, keys: Keys, y, rows: int):
        """Class scores of the standard baseline's outputs (one ciphertext per class)."""
        return self._scores(N.lib().lrhe_decrypt_scores_standard, keys, y, rows, y.shape[0])

    def decrypt_check(self, keys: Keys, ct, expected):
        """Debug decryption against the expected slot values: raises LrheError with
        code LRHE_ENOISE when any slot differs.  Returns the noise budgets."""
        exp = np.ascontiguousarray(expected, dtype=np.int64)
        cnt = ct.shape[0]
        bud = np.zeros(cnt, dtype=np.float64)
        bad = ctypes.c_uint64()
        N.check(N.lib().lrhe_decrypt_check(self.h, keys.sk, N.ptr(ct.contiguous()), cnt, N.ptr(exp), 0, N.ptr(bud),
                                           ctypes.byref(bad), _stream()))
        return bud

    def host_transform(self, a: np.ndarray, mod_index: int, inverse: bool = False) -> np.ndarray:
        a = np.ascontiguousarray(a, dtype=np.uint32).copy()
        N.check(N.lib().lrhe_host_transform(self.h, mod_index, N.ptr(a), 1 if inverse else 0))
        return a

    # ---------------------------------------------------------------- server
    def model(self, W, bias) -> Model:
        Wd = self._as_dev_i64(W)
        f, classes = Wd.shape
        b = np.ascontiguousarray(bias, dtype=np.int64)
        h = ctypes.c_void_p()
        N.check(N.lib().lrhe_model_create(self.h, N.ptr(Wd), N.ptr(b), f, classes, _stream(), ctypes.byref(h)))
        return Model(self, h, f, classes)

    def matmul_fast(self, keys: Keys, model: Model, xct, rows: int, out=None, ws=None):
        nout = -(-rows * model.classes // self.n)
        out = self.empty_ct(nout) if out is None else out
        ws = self.workspace(N.WS_MATMUL_FAST, rows, model.f, model.classes) if ws is None else ws
        N.check(N.lib().lrhe_matmul_fast(self.h, keys.gk, model.handle, N.ptr(xct), rows, N.ptr(out), N.ptr(ws),
                                         ws.numel(), _stream()))
        return out

    def matmul_fast_noalloc(self, keys: Keys, model: Model, xct, rows: int, out):
        """Algorithm 1 with the library's fixed device scratch as workspace (no
        allocation in the call; out is caller-provided)."""
        N.check(N.lib().lrhe_matmul_fast_noalloc(self.h, keys.gk, model.handle, N.ptr(xct), rows, N.ptr(out),
                                                 _stream()))
        return out

    def matmul_fast_pairs(self, keys: Keys, model: Model, xct, rows: int, pair0: int, npairs: int, stage: int,
                          out=None, ws=None):
        out = self.empty_ct(npairs) if out is None else out
        ws = self.workspace(N.WS_MATMUL_FAST, npairs, model.f, 1) if ws is None else ws
        N.check(N.lib().lrhe_matmul_fast_pairs(self.h, keys.gk, model.handle, N.ptr(xct), rows, pair0, npairs, stage,
                                               N.ptr(out), N.ptr(ws), ws.numel(), _stream()))
        return out

    def matmul_standard(self, model: Model, fct, out=None):
        out = self.empty_ct(model.classes) if out is None else out
        N.check(N.lib().lrhe_matmul_standard(self.h, model.handle, N.ptr(fct), N.ptr(out), None, 0, _stream()))
        return out

    def tune_set(self, key: str, value: int):
        N.check(N.lib().lrhe_tune_set(self.h, key.encode(), value))

    def tune_get(self, key: str) -> int:
        v = ctypes.c_int()
        N.check(N.lib().lrhe_tune_get(self.h, key.encode(), ctypes.byref(v)))
        return v.value

    def tune_save(self, path: str, key: str):
        N.check(N.lib().lrhe_tune_save(self.h, path.encode(), key.encode()))

    def tune_load(self, path: str, key: str) -> bool:
        """Apply a cached entry; False when the file or key is absent."""
        rc = N.lib().lrhe_tune_load(self.h, path.encode(), key.encode())
        if rc == N.LRHE_EAGAIN:
            return False
        N.check(rc)
        return True

    def tuning(self) -> dict:
        names = ("le_intt", "le_mac", "le_moddown", "le_mask", "mac_mode", "fuse_intt", "le_mac_p")
        return {"large": {k: self.tune_get("large." + k) for k in names},
                "small": {k: self.tune_get("small." + k) for k in names},
                "tile": self.tune_get("tile"), "small_below": self.tune_get("small_below")}

    def autotune_fast(self, keys: Keys, model: Model, xct, rows: int, out=None, ws=None, reps: int = 2) -> dict:
        nout = -(-rows * model.classes // self.n)
        out = self.empty_ct(nout) if out is None else out
        ws = self.workspace(N.WS_MATMUL_FAST, rows, model.f, model.classes) if ws is None else ws
        N.check(N.lib().lrhe_autotune_fast(self.h, keys.gk, model.handle, N.ptr(xct), rows, N.ptr(out), N.ptr(ws),
                                           ws.numel(), _stream(), reps))
        return self.tuning()

    def to_coeff(self, ct):
        """Canonical coefficient form (device tensor, same shape), for parity checks."""
        out = _torch().empty_like(ct)
        polys = ct.numel() // (self.L * self.n)
        N.check(N.lib().lrhe_to_coeff(self.h, N.ptr(ct.contiguous()), polys, N.ptr(out), _stream()))
        return out


class Batch:
    """A fixed set of requests (xct, rows, model, y[, keys]) planned once; run()
    executes Algorithm 1 for all of them, capture() records the launches in a
    hipGraph.  A request without its own keys uses the batch's keys."""

    def __init__(self, ctx: Context, keys: Keys, requests):
        self.ctx, self.keys = ctx, keys
        self.requests = list(requests)   # keeps the tensors and keys alive
        arr = (N.LrheRequest * len(self.requests))()
        for k, req in enumerate(self.requests):
            xct, rows, model, y = req[:4]
            rkeys = req[4] if len(req) > 4 else None
            arr[k] = N.LrheRequest(N.ptr(xct), rows, model.handle, N.ptr(y), rkeys.gk if rkeys is not None else None)
        h = ctypes.c_void_p()
        N.check(N.lib().lrhe_batch_create(ctx.h, ctypes.cast(arr, ctypes.c_void_p), len(self.requests),
                                          ctypes.byref(h)))
        self.h = h
        wsb, npairs, tile, ng = ctypes.c_uint64(), ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        N.check(N.lib().lrhe_batch_info(h, ctypes.byref(wsb), ctypes.byref(npairs), ctypes.byref(tile),
                                        ctypes.byref(ng)))
        self.ws_bytes, self.npairs, self.tile, self.ngroups = wsb.value, npairs.value, tile.value, ng.value
        torch = _torch()
        self.ws = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=ctx._dev())

    def run(self):
        N.check(N.lib().lrhe_batch_run(self.ctx.h, self.keys.gk, self.h, N.ptr(self.ws), self.ws.numel(), _stream()))

    def capture(self, stream):
        """Capture on a (non-default) torch stream; later run() calls on any stream replay the graph."""
        N.check(N.lib().lrhe_batch_capture(self.ctx.h, self.keys.gk, self.h, N.ptr(self.ws), self.ws.numel(),
                                           ctypes.c_void_p(stream.cuda_stream)))

    def close(self):
        if getattr(self, "h", None):
            N.lib().lrhe_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server (native worker thread) over resident Galois keys."""

    def __init__(self, ctx: Context, keys: Keys, hbm_budget: int):
        self.ctx = ctx
        h = ctypes.c_void_p()
        N.check(N.lib().lrhe_server_create(ctx.h, keys.gk, hbm_budget, ctypes.byref(h)))
        self.h = h
        self._keep = {}       # request id -> buffers, model and keys it uses, until released
        self._keys = keys     # the server's own key set stays alive with it

    def submit(self, model: Model, xct, rows: int, y, keys: Keys = None):
        """Returns the request id, or None when admission is refused (LRHE_EAGAIN).
        `keys`: the client's keys when they are not the server's.  The server waits
        for the work queued on the current torch stream (the encryption of xct)."""
        rid = ctypes.c_uint64()
        if keys is not None:
            code = N.lib().lrhe_server_submit_keys(self.h, keys.gk, model.handle, N.ptr(xct), rows, N.ptr(y),
                                                   _stream(), ctypes.byref(rid))
        else:
            code = N.lib().lrhe_server_submit(self.h, model.handle, N.ptr(xct), rows, N.ptr(y), _stream(),
                                              ctypes.byref(rid))
        if code == N.LRHE_EAGAIN:
            return None
        N.check(code)
        self._keep[rid.value] = (xct, y, model, keys)
        return rid.value

    def release(self, rid: int):
        """Forget a finished request: the server's record and the buffers held for it."""
        N.check(N.lib().lrhe_server_release(self.h, rid))
        self._keep.pop(rid, None)

    def poll(self, rid: int):
        done, lat = ctypes.c_int(), ctypes.c_double()
        N.check(N.lib().lrhe_server_poll(self.h, rid, ctypes.byref(done), ctypes.byref(lat)))
        return bool(done.value), lat.value

    def drain(self):
        N.check(N.lib().lrhe_server_drain(self.h))

    def stats(self) -> dict:
        t, p, f, b, hd = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        N.check(N.lib().lrhe_server_stats(self.h, ctypes.byref(t), ctypes.byref(p), ctypes.byref(f), ctypes.byref(b),
                                          ctypes.byref(hd)))
        return {"ticks": t.value, "pairs": p.value, "free_slots": f.value, "tile": b.value, "held": hd.value}

    def close(self):
        if getattr(self, "h", None):
            N.lib().lrhe_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def to_numpy_u32(t) -> np.ndarray:
    """Device int32 tensor of residues -> host uint32 array."""
    return t.cpu().numpy().view(np.uint32)


def fixed_point(a, bits: int) -> np.ndarray:
    """Real values to the paper's fixed-point integers, nearest integer to
    a 2^bits (lrhe_fixed_point); same shape, int64."""
    x = np.ascontiguousarray(a, dtype=np.float64)
    out = np.empty(x.shape, dtype=np.int64)
    N.check(N.lib().lrhe_fixed_point(N.ptr(x), x.size, bits, N.ptr(out)))
    return out


def crt_combine(r0, r1, t0: int, t1: int) -> np.ndarray:
    """Scores mod t0 and mod t1 to the integer in (-t0 t1 / 2, t0 t1 / 2]
    congruent to both (lrhe_crt_combine); same shape, int64."""
    a = np.ascontiguousarray(r0, dtype=np.int64)
    b = np.ascontiguousarray(r1, dtype=np.int64)
    assert a.shape == b.shape
    out = np.empty(a.shape, dtype=np.int64)
    N.check(N.lib().lrhe_crt_combine(N.ptr(a), N.ptr(b), a.size, t0, t1, N.ptr(out)))
    return out
