"""Seeded synthetic inputs and parameter sets shared by the HIP path's tests and
benchmarks and by the CPU oracle.  Holds none of the method's arithmetic.

The paper's iDASH 2020 / TCGA mutation data (section "Dataset") is not
available, so every workload is a synthetic stand-in with the paper's shapes:
binary SNV-presence-like features (Bernoulli), up to 40,960 features per
individual (section "Private inference protocol", f = 40960), 543 test
patients and 11 cancer types (section "Privacy-preserving model evaluation"),
rounded here to the configurations below.  Weights and biases are integers in
[-127, 127] (int8 range).  Timing does not depend on the values.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 220405496


@dataclass(frozen=True)
class Params:
    """BFV parameters: ring degree n, data primes q (each < 2^30, = 1 mod 2n),
    special key-switching prime P (the next such prime), plaintext modulus t."""
    name: str
    n: int
    q: tuple
    P: int
    t: int
    insecure: bool = False   # log2(Q P) above the 128-bit bound for n (test-only)


# largest primes below 2^30 that are 1 mod 8192 (n = 4096)
_Q4096 = (1073692673, 1073668097, 1073651713, 1073643521)
# largest primes below 2^30 that are 1 mod 32768 (n = 16384)
_Q16384 = (1073643521, 1073479681, 1073184769, 1073053697, 1072857089, 1072496641, 1071513601, 1071415297)

# largest primes below 2^30 that are 1 mod 16384 (n = 8192): six data primes and P,
# log2(Q P) = 210 <= 218, the 128-bit bound at n = 8192
_Q8192 = (1073692673, 1073643521, 1073479681, 1073430529, 1073299457, 1073233921, 1073184769)

# the paper's plaintext moduli (section "Private inference protocol"): a CRT pair,
# t0 = 1073872897 (30 bits) and t1 = 114689 (16 bits), both 1 mod 2n at n = 8192,
# and its fixed-point scales: inputs x 2^6, weights x 2^14, biases x 2^20
T_PAIR = (1073872897, 114689)
S_X, S_W = 6, 14

PARAMS = {
    # tiny: n = 4096, t = 65537, two data primes + special prime
    "tiny": Params("tiny", 4096, _Q4096[:2], _Q4096[2], 65537),
    # tiny with three data primes (labelled insecure: 120 bits > 109 at n = 4096)
    "tiny3": Params("tiny3", 4096, _Q4096[:3], _Q4096[3], 65537, insecure=True),
    # n = 16384, seven data primes + special prime, t = 786433 (20-bit, = 1 mod 32768)
    "n16k": Params("n16k", 16384, _Q16384[:7], _Q16384[7], 786433),
    # the paper's parameter point: n = 8192, one context per plaintext modulus of the pair
    "paper_t0": Params("paper_t0", 8192, _Q8192[:6], _Q8192[6], T_PAIR[0]),
    "paper_t1": Params("paper_t1", 8192, _Q8192[:6], _Q8192[6], T_PAIR[1]),
}


@dataclass
class Workload:
    name: str
    params: str
    rows: int
    f: int
    classes: int
    p: float
    seed: int
    X: np.ndarray = field(repr=False, default=None)
    W: np.ndarray = field(repr=False, default=None)
    b: np.ndarray = field(repr=False, default=None)


def features(rows: int, f: int, p: float, seed: int) -> np.ndarray:
    """Binary mutation-presence-like features, Bernoulli(p), int64 [rows][f]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (rng.random((rows, f)) < p).astype(np.int64)


def weights(f: int, classes: int, seed: int) -> np.ndarray:
    """Integer weights uniform in [-127, 127], int64 [f][classes] (W is f x |Y|)."""
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    return rng.integers(-127, 128, size=(f, classes), dtype=np.int64)


def biases(classes: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed + 2))
    return rng.integers(-127, 128, size=classes, dtype=np.int64)


def make(name: str, params: str, rows: int, f: int, classes: int, p: float, seed: int) -> Workload:
    return Workload(name, params, rows, f, classes, p, seed,
                    features(rows, f, p, seed), weights(f, classes, seed), biases(classes, seed))


def tiny(seed: int = BASE_SEED + 1, params: str = "tiny") -> Workload:
    """1 individual x 256 features (p = 0.02), 4 classes, n = 4096."""
    return make("tiny_1x256x4", params, 1, 256, 4, 0.02, seed)


def single(seed: int = BASE_SEED + 2, f: int = 40000) -> Workload:
    """1 individual x 40,000 features (p = 0.01), 16 classes, n = 16384."""
    return make("single_1x40000x16", "n16k", 1, f, 16, 0.01, seed)


def batch(rows: int = 512, seed: int = BASE_SEED + 3, f: int = 40000) -> Workload:
    """512 individuals x 40,000 features (p = 0.01), 16 classes, n = 16384."""
    return make(f"batch_{rows}x{f}x16", "n16k", rows, f, 16, 0.01, seed)


def uneven_requests(count: int = 64, seed: int = BASE_SEED + 4, max_rows: int = 512,
                    f_lo: int = 10000, f_hi: int = 40000):
    """Requests with individuals ~ U{1..max_rows} and features ~ U{f_lo..f_hi};
    request r uses the first f_r rows of a seeded 40,000 x 16 master weight matrix."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rows = rng.integers(1, max_rows + 1, size=count)
    fs = rng.integers(f_lo, f_hi + 1, size=count)
    W = weights(f_hi, 16, seed)
    b = biases(16, seed)
    out = []
    for r in range(count):
        X = features(int(rows[r]), int(fs[r]), 0.01, seed + 1000 + r)
        out.append(Workload(f"req{r}", "n16k", int(rows[r]), int(fs[r]), 16, 0.01, seed + 1000 + r,
                            X, W[: int(fs[r])], b))
    return out


def binary_models(rows: int = 543, count: int = 11, seed: int = BASE_SEED + 60, params: str = "n16k",
                  f_lo: int = 10000, f_hi: int = 40000, p: float = 0.01):
    """One-vs-rest binary models (section "Binary models"): one model per cancer
    type, each with its own selected features (f_m ~ U{f_lo..f_hi}) and a single
    output (|Y| = 1), evaluated on the same individuals; model m's inputs are the
    individuals' values of its own features."""
    rng = np.random.Generator(np.random.PCG64(seed))
    fs = rng.integers(f_lo, f_hi + 1, size=count)
    out = []
    for m in range(count):
        f = int(fs[m])
        out.append(Workload(f"binary{m}", params, rows, f, 1, p, seed + 100 + m, features(rows, f, p, seed + 100 + m),
                            weights(f, 1, seed + 200 + m), biases(1, seed + 300 + m)))
    return out


def real_workload(name: str, rows: int, f: int, classes: int, p: float, seed: int) -> Workload:
    """Real-valued inputs of the paper's precision point (section "Private
    inference protocol"): features in [0, 2^8) (a Bernoulli(p) mask times
    U[0, 256), mutation-count-like and sparse), weights and biases in (-1, 1),
    float64.  The fixed-point scaling is the method's, not done here."""
    rng = np.random.Generator(np.random.PCG64(seed))
    X = (rng.random((rows, f)) < p) * rng.uniform(0.0, 256.0, size=(rows, f))
    W = rng.uniform(-1.0, 1.0, size=(f, classes))
    b = rng.uniform(-1.0, 1.0, size=classes)
    return Workload(name, "paper_t0", rows, f, classes, p, seed, X, W, b)


def paper_single(f: int = 40960, seed: int = BASE_SEED + 40) -> Workload:
    """One patient x 40,960 features x 11 cancer types, real-valued."""
    return real_workload(f"paper_1x{f}x11", 1, f, 11, 0.01, seed)


def paper_batch(rows: int = 543, f: int = 40960, seed: int = BASE_SEED + 41) -> Workload:
    """The paper's test set shape: 543 patients x 40,960 features x 11 cancer types."""
    return real_workload(f"paper_{rows}x{f}x11", rows, f, 11, 0.01, seed)


def poisson_arrivals(count: int, qps: float, seed: int = BASE_SEED + 5) -> np.ndarray:
    """Arrival times (seconds from start) of a Poisson process at rate qps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / qps, size=count))
