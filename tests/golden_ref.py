"""Reader of the stored oracle outputs under tests/golden/ (written by
tests/golden/make_golden.py from the CPU oracle alone) and the matching digest
of a GPU output, limb by limb."""
from __future__ import annotations

import hashlib
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
SAMPLE_POS = (0, 1, 2, 3, 4095, 8191, 12345, 16383)


def load(fname: str) -> dict:
    """{name: {(ciphertext, part, limb): (sha256, sampled values)}}"""
    out: dict = {}
    with open(os.path.join(GOLDEN, fname)) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            f = line.split()
            out.setdefault(f[0], {})[(int(f[1]), int(f[2]), int(f[3]))] = (f[4], [int(v) for v in f[5:]])
    return out


def mismatches(cts: np.ndarray, ref: dict) -> list:
    """Limbs of the canonical ciphertexts cts [count][2][L][n] whose bytes differ
    from the stored digest, or whose sampled values differ (empty = identical)."""
    bad = []
    assert len(ref) == cts.shape[0] * cts.shape[1] * cts.shape[2], "stored output has another shape"
    for (ci, part, limb), (h, vals) in sorted(ref.items()):
        v = np.ascontiguousarray(cts[ci, part, limb], dtype="<u4")
        got = [int(v[k]) for k in SAMPLE_POS]
        if hashlib.sha256(v.tobytes()).hexdigest() != h or got != vals:
            bad.append((ci, part, limb, got, vals))
    return bad
