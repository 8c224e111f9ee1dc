"""CPU tests of the wire format of the private inference protocol (ciphertexts
and keys as byte messages): the payload is the oracle's canonical
coefficient-form ciphertext, round trips are exact, keys reloaded in a new
context (a restart) are the same keys, and malformed, corrupted or foreign
messages are refused with LRHE_EINVAL.  Contexts are host-only."""
import numpy as np
import pytest

import workloads as WL
from oracle import oracle as O

HDR = 64


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
    return p, ctx, o, ctx.keygen(77), o.keygen(77, galois=False)


def fnv1a(b: bytes) -> int:
    h = 1469598103934665603
    for x in b:
        h = ((h ^ x) * 1099511628211) % 2 ** 64
    return h


def with_payload(msg: bytes, payload: bytes) -> bytes:
    """The same header with a new payload and its checksum recomputed."""
    return msg[:56] + fnv1a(payload).to_bytes(8, "little") + payload


def test_ct_payload_is_oracle_coefficients(tiny3, P):
    p, ctx, o, keys, ko = tiny3
    z = np.random.default_rng(3).integers(0, p.t, (3, p.n))
    cts = np.stack([o.encrypt_plain(ko, o.encode(z[c]), 9, c) for c in range(3)])       # coefficient form
    ev = np.stack([[[ctx.host_transform(cts[c, x, j].astype(np.uint32), j) for j in range(o.L)] for x in range(2)]
                   for c in range(3)])                                                   # library's evaluation form
    msg = ctx.serialize_ct(ev)
    assert len(msg) == HDR + cts.size * 4 and msg[:8] == b"LRHEWIR1"
    payload = np.frombuffer(msg[HDR:], dtype="<u4").reshape(cts.shape)
    assert np.array_equal(payload, cts.astype(np.uint32))
    back = ctx.deserialize_ct(msg, host=True)
    assert np.array_equal(back, ev)
    # the library decrypts the received ciphertexts with its own key (same seed as the oracle's)
    slots, bud = ctx.decrypt_slots_host(keys, back)
    assert np.array_equal(slots, o.centre(z)) and (bud > 0).all()


def test_keys_reloaded_in_new_context(tiny3, P):
    """sk, pk and gk through the wire into a fresh context: the same keys (exports
    equal), and the reloaded secret key decrypts what the original public key
    encrypted."""
    p, ctx, o, keys, ko = tiny3
    N = P.native
    msgs = {k: ctx.serialize_key(keys, k) for k in (N.WIRE_SK, N.WIRE_PK, N.WIRE_GK)}
    ctx2 = P.Context.from_params(p, device=-1)
    k2 = ctx2.load_keys(sk=msgs[N.WIRE_SK], pk=msgs[N.WIRE_PK], gk=msgs[N.WIRE_GK])
    assert np.array_equal(ctx2.export_sk(k2), ctx.export_sk(keys))
    assert np.array_equal(ctx2.export_pk(k2), ctx.export_pk(keys))
    assert np.array_equal(ctx2.export_gk(k2), ctx.export_gk(keys))
    # the library's keys are the oracle's (same seed): the reloaded sk decrypts an oracle ciphertext
    z = np.random.default_rng(4).integers(0, p.t, p.n)
    ct = o.encrypt_plain(o.keygen(77, galois=False), o.encode(z), 5, 0)
    ev = np.stack([[ctx.host_transform(ct[x, j].astype(np.uint32), j) for j in range(o.L)] for x in range(2)])[None]
    slots, bud = ctx2.decrypt_slots_host(k2, ev)
    assert np.array_equal(slots[0], o.centre(z)) and bud[0] > 0


def test_malformed_messages_refused(tiny3, P):
    p, ctx, o, keys, ko = tiny3
    N = P.native
    ev = np.zeros((2, 2, o.L, p.n), dtype=np.uint32)
    ev[:, :, :, 5] = 7
    msg = ctx.serialize_ct(ev)
    bad = [
        b"XXXXWIR1" + msg[8:],                                            # magic
        msg[:8] + (2).to_bytes(4, "little") + msg[12:],                   # version
        msg[:12] + (3).to_bytes(4, "little") + msg[16:],                  # kind
        msg[:-4],                                                         # truncated
        msg[:HDR + 10] + bytes([msg[HDR + 10] ^ 1]) + msg[HDR + 11:],     # payload bit flip (checksum)
    ]
    # a residue at the modulus itself, with a valid checksum
    pl = bytearray(msg[HDR:])
    pl[0:4] = int(p.q[0]).to_bytes(4, "little")
    bad.append(with_payload(msg, bytes(pl)))
    for m in bad:
        with pytest.raises(N.LrheError) as ei:
            ctx.deserialize_ct(m, host=True)
        assert ei.value.code == N.LRHE_EINVAL
    # another parameter set
    pt = WL.PARAMS["tiny"]
    other = P.Context.from_params(pt, device=-1)
    with pytest.raises(N.LrheError):
        other.deserialize_ct(msg, host=True)
    # too many ciphertexts for the buffer
    with pytest.raises(N.LrheError):
        ctx.deserialize_ct(msg, out=np.zeros((1, 2, o.L, p.n), dtype=np.uint32), host=True)
    # a secret key with a coefficient outside {-1, 0, 1}
    sk = ctx.serialize_key(keys, N.WIRE_SK)
    s = bytearray(sk[HDR:])
    s[0] = 2
    with pytest.raises(N.LrheError):
        ctx.load_keys(sk=with_payload(sk, bytes(s)))
    # a Galois key message read as a public key
    with pytest.raises(N.LrheError):
        ctx.load_keys(pk=ctx.serialize_key(keys, N.WIRE_GK))
