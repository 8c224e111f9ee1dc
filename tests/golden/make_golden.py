"""Writes the stored expected outputs of the GPU parity tests at the benchmark's
sizes.  Calls only the CPU oracle (oracle/) and the seeded input generators
(workloads.py); nothing here touches the HIP path.

    python tests/golden/make_golden.py batch    # 512 x 40,000 x 16, n = 16384 (~40 min on 8 cores)
    python tests/golden/make_golden.py uneven   # 8 uneven requests of 1-4 individuals, n = 16384

Each output ciphertext is stored in canonical coefficient form (residues in
[0, q_i), uint32 little-endian, layout [2][L][n]) as one line per (part, limb):
its SHA-256 and the values at a few fixed positions.  The GPU tests hash the
same bytes of their own output, limb by limb.
"""
from __future__ import annotations

import hashlib
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as WL  # noqa: E402
from oracle import oracle as O  # noqa: E402

KEY_SEED = 2024          # key set of the n = 16384 parity tests and the benchmark
BATCH_ENC_SEED = 3       # encryption seed of the 512 x 40,000 benchmark batch
UNEVEN_ENC_SEED0 = 600   # request r is encrypted with seed UNEVEN_ENC_SEED0 + r
SAMPLE_POS = (0, 1, 2, 3, 4095, 8191, 12345, 16383)


def limb_lines(name: str, cts: np.ndarray) -> list[str]:
    out = []
    for ci, ct in enumerate(cts):
        for part in range(ct.shape[0]):
            for limb in range(ct.shape[1]):
                v = np.ascontiguousarray(ct[part, limb], dtype="<u4")
                h = hashlib.sha256(v.tobytes()).hexdigest()
                out.append(f"{name} {ci} {part} {limb} {h} " + " ".join(str(int(v[k])) for k in SAMPLE_POS))
    return out


def encrypt_rows_threaded(o, keys, X, seed, threads=8):
    """The oracle's row encryption, rows spread over threads (each C call
    releases the interpreter lock); the result does not depend on the order."""
    rows = X.shape[0]
    K = -(-X.shape[1] // o.n)
    out = np.zeros((rows, K, 2, o.L, o.n), dtype=np.uint64)

    def one(i):
        out[i] = o.encrypt_rows(keys, X[i:i + 1], seed=seed, row0=i)[0]

    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(one, range(rows)))
    return out


def uneven_small():
    """Requests shaped like the uneven-batching workload (features ~ U{10,000..40,000},
    one shared 40,000 x 16 master model), with 1-4 individuals each so the oracle
    stays cheap."""
    return WL.uneven_requests(count=8, seed=WL.BASE_SEED + 6, max_rows=4)


def write(path, header, lines):
    with open(path, "w") as fh:
        for h in header:
            fh.write("# " + h + "\n")
        for ln in lines:
            fh.write(ln + "\n")


def main(which):
    p = WL.PARAMS["n16k"]
    o = O.Oracle(p.n, list(p.q), p.P, p.t)
    t0 = time.time()
    keys = o.keygen(KEY_SEED)
    print(f"keygen {time.time() - t0:.1f} s", flush=True)
    if which == "batch":
        wl = WL.batch()
        xo = encrypt_rows_threaded(o, keys, wl.X, BATCH_ENC_SEED)
        print(f"encrypted {wl.rows} rows {time.time() - t0:.1f} s", flush=True)
        y = o.fast_matmul(keys, xo, o.encode_weights(wl.W), wl.b)
        print(f"Algorithm 1 done {time.time() - t0:.1f} s", flush=True)
        S, budget = o.scores_fast(keys, y, wl.rows, wl.classes)
        assert np.array_equal(S, O.plain_scores(wl.X, wl.W, wl.b, p.t)) and budget > 0
        write(os.path.join(HERE, "batch_512x40000x16_fast_output.txt"),
              [f"oracle output of Algorithm 1 on {wl.name} (n16k parameters), key seed {KEY_SEED}, "
               f"encryption seed {BATCH_ENC_SEED}, ciphertext id = i K + k",
               f"decrypts to X W + b mod t; noise budget left {budget:.1f} bits",
               "columns: name ciphertext part limb sha256(uint32 LE limb) values at " +
               " ".join(map(str, SAMPLE_POS))],
              limb_lines(wl.name, y))
    elif which == "uneven":
        lines = []
        for r, wl in enumerate(uneven_small()):
            xo = o.encrypt_rows(keys, wl.X, seed=UNEVEN_ENC_SEED0 + r)
            y = o.fast_matmul(keys, xo, o.encode_weights(wl.W), wl.b)
            S, budget = o.scores_fast(keys, y, wl.rows, wl.classes)
            assert np.array_equal(S, O.plain_scores(wl.X, wl.W, wl.b, p.t)) and budget > 0
            lines += limb_lines(f"req{r}_{wl.rows}x{wl.f}", y)
            print(f"request {r}: {wl.rows} x {wl.f} budget {budget:.1f} ({time.time() - t0:.1f} s)", flush=True)
        write(os.path.join(HERE, "uneven_small_n16k_outputs.txt"),
              [f"oracle outputs of Algorithm 1 on 8 uneven requests (workloads.uneven_requests(count=8, "
               f"seed=BASE_SEED + 6, max_rows=4)), n16k parameters, key seed {KEY_SEED}, request r "
               f"encrypted with seed {UNEVEN_ENC_SEED0} + r, ciphertext id = i K + k",
               "columns: name ciphertext part limb sha256(uint32 LE limb) values at " +
               " ".join(map(str, SAMPLE_POS))],
              lines)
    else:
        raise SystemExit("usage: make_golden.py batch|uneven")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "")
