"""GPU checks of the batched transform entry point (lrhe_ntt, row a12) against
definitions, not against the library's own host transform: the forward output
at index k is the evaluation a(psi^(2 brv(k) + 1)) for a primitive 2n-th root
psi (checked at sampled k by direct summation), the inverse undoes it, and
pointwise products of two transforms come back as the oracle's negacyclic
product.  Exact modular arithmetic: no tolerance."""
import sys

import numpy as np
import pytest

import workloads as WL
from oracle import oracle as O

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-ntt]", *a, flush=True)
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


def brv(k, bits):
    return int(format(k, f"0{bits}b")[::-1], 2)


def transform(P, ctx, torch, host, inverse):
    """lrhe_ntt in place on a device copy of host (polys, L, n) uint32."""
    d = torch.from_numpy(host.astype(np.int32)).cuda()
    P.native.check(P.native.lib().lrhe_ntt(ctx.h, P.native.ptr(d), host.shape[0], 1 if inverse else 0, None))
    torch.cuda.synchronize()
    return d.cpu().numpy().astype(np.uint32)


@pytest.mark.parametrize("pname", ["tiny", "n16k"])
def test_batched_transform_definition_and_product(P, torch, pname):
    p = WL.PARAMS[pname]
    n, qs = p.n, list(p.q)
    L, logn = len(qs), n.bit_length() - 1
    ctx = P.Context.from_params(p, device=0)
    say(pname, "n", n, "L", L)
    rng = np.random.default_rng(2024 + n)
    polys = 3
    a = np.stack([np.stack([rng.integers(0, q, n) for q in qs]) for _ in range(polys)]).astype(np.uint32)
    b = np.stack([np.stack([rng.integers(0, q, n) for q in qs]) for _ in range(polys)]).astype(np.uint32)
    # psi of each limb from the transform of the monomial X: index 0 holds psi^1
    mono = np.zeros((1, L, n), dtype=np.uint32)
    mono[0, :, 1] = 1
    M = transform(P, ctx, torch, mono, inverse=False)
    A = transform(P, ctx, torch, a, inverse=False)
    B = transform(P, ctx, torch, b, inverse=False)
    ks = [0, 1, n - 1] + [int(k) for k in rng.integers(0, n, 5)]
    for i, q in enumerate(qs):
        psi = int(M[0, i, 0])
        assert pow(psi, n, q) == q - 1, f"limb {i}: psi^n != -1"
        assert np.all(A[:, i] < q) and np.all(B[:, i] < q)
        for pi in range(polys):
            coeffs = [int(v) for v in a[pi, i]]
            for k in ks:
                z = pow(psi, 2 * brv(k, logn) + 1, q)
                acc, zj = 0, 1
                for c in coeffs:        # Horner would be faster; the plain sum is the definition
                    acc = (acc + c * zj) % q
                    zj = zj * z % q
                assert int(A[pi, i, k]) == acc, f"limb {i} poly {pi} index {k}"
    # inverse: round trip, and the pointwise product is the negacyclic product
    back = transform(P, ctx, torch, A, inverse=True)
    assert np.array_equal(back, a)
    AB = np.stack([[(A[pi, i].astype(np.uint64) * B[pi, i]) % q for i, q in enumerate(qs)] for pi in range(polys)])
    prod = transform(P, ctx, torch, AB.astype(np.uint32), inverse=True)
    o = O.Oracle(p.n, qs, p.P, p.t)
    for pi in range(polys):
        for i in range(L):
            ref = np.zeros(n, dtype=np.uint64)
            O.lib().ora_ring_mul(o.ctx, i, O.P(O.u64(a[pi, i])), O.P(O.u64(b[pi, i])), O.P(ref))
            assert np.array_equal(prod[pi, i].astype(np.uint64), ref), f"limb {i} poly {pi}"
