"""GPU test of the client/server split over the wire format (section "Private
inference protocol"): the client keygens, encrypts its rows and sends the
ciphertexts plus its Galois keys as byte messages; a server context of its
own reads them, runs Algorithm 1 and returns the result as a message; the
client decrypts it.  The server's output equals the one-process run bit for
bit and decrypts to X W + b mod t; a client restarted from its stored keys
encrypts to the same ciphertexts."""
import sys

import numpy as np
import pytest

import workloads as WL
from oracle import oracle as O

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-wire]", *a, flush=True)
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


@pytest.mark.parametrize("pname,rows,f,classes", [("tiny3", 5, 5000, 4), ("n16k", 2, 40000, 16)])
def test_client_server_over_wire(P, torch, pname, rows, f, classes):
    N = P.native
    p = WL.PARAMS[pname]
    wl = WL.make(f"wire_{rows}x{f}x{classes}", pname, rows, f, classes, 0.02, WL.BASE_SEED + 70)
    say(pname, rows, f, classes)
    # client
    client = P.Context.from_params(p, device=0)
    keys = client.keygen(4040)
    xct = client.encrypt_rows(keys, wl.X, seed=12)
    to_server = client.serialize_ct(xct)
    gk_msg = client.serialize_key(keys, N.WIRE_GK)
    sk_msg, pk_msg = client.serialize_key(keys, N.WIRE_SK), client.serialize_key(keys, N.WIRE_PK)
    # server: its own context, evaluation keys and inputs from the messages only
    server = P.Context.from_params(p, device=0)
    skeys = server.load_keys(gk=gk_msg)
    sx = server.deserialize_ct(to_server)
    assert torch.equal(sx, xct)
    model = server.model(wl.W, wl.b)
    y = server.matmul_fast(skeys, model, sx, rows)
    to_client = server.serialize_ct(y)
    # the one-process run with the client's own keys
    ref = client.matmul_fast(keys, client.model(wl.W, wl.b), xct, rows)
    torch.cuda.synchronize()
    assert torch.equal(y, ref)
    # client decrypts the returned message (host copy, no device needed for it)
    yh = client.deserialize_ct(to_client, host=True)
    S, budget = client.scores_fast(keys, yh, rows, classes)
    assert np.array_equal(S, O.plain_scores(wl.X, wl.W, wl.b, p.t)) and budget > 0
    # a restarted client: keys from storage give the same ciphertexts and decryptions
    client2 = P.Context.from_params(p, device=0)
    k2 = client2.load_keys(sk=sk_msg, pk=pk_msg)
    x2 = client2.encrypt_rows(k2, wl.X, seed=12)
    torch.cuda.synchronize()
    assert torch.equal(x2, xct)
    S2, _ = client2.scores_fast(k2, yh, rows, classes)
    assert np.array_equal(S2, S)
