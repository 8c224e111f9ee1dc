"""Brute-force, big-integer definitions used to pin the oracle on tiny rings.

Everything here is the textbook definition written with Python integers:
schoolbook negacyclic products, CRT reconstruction, exact rounding.  It is
independent of the oracle's C code (which uses transforms and RNS formulas).
"""
from __future__ import annotations


def negacyclic(a, b, m=None):
    """a(X) b(X) mod (X^n + 1) over the integers (mod m if given)."""
    n = len(a)
    out = [0] * n
    for i in range(n):
        ai = int(a[i])
        if ai == 0:
            continue
        for j in range(n):
            k = i + j
            v = ai * int(b[j])
            if k < n:
                out[k] += v
            else:
                out[k - n] -= v
    if m is not None:
        out = [v % m for v in out]
    return out


def crt(residues, moduli):
    M = 1
    for m in moduli:
        M *= m
    x = 0
    for r, m in zip(residues, moduli):
        Mi = M // m
        x += int(r) * Mi * pow(Mi, -1, m)
    return x % M, M


def automorph(a, g):
    """a(X) -> a(X^g) mod (X^n + 1) over the integers."""
    n = len(a)
    out = [0] * n
    for k in range(n):
        idx = (g * k) % (2 * n)
        if idx < n:
            out[idx] += int(a[k])
        else:
            out[idx - n] -= int(a[k])
    return out


def smallest_generator(p):
    fac, m, d = [], p - 1, 2
    while d * d <= m:
        if m % d == 0:
            fac.append(d)
            while m % d == 0:
                m //= d
        d += 1
    if m > 1:
        fac.append(m)
    for g in range(2, p):
        if all(pow(g, (p - 1) // f, p) != 1 for f in fac):
            return g


def slot_exponents(n):
    """e_j = 3^j mod 2n for j < n/2, -3^(j - n/2) mod 2n otherwise."""
    e = [pow(3, j, 2 * n) for j in range(n // 2)]
    return e + [(2 * n - x) % (2 * n) for x in e]


def is_prime(m):
    if m < 2:
        return False
    for sp in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        if m % sp == 0:
            return m == sp
    d, s = m - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        x = pow(a, d, m)
        if x in (1, m - 1):
            continue
        for _ in range(s - 1):
            x = x * x % m
            if x == m - 1:
                break
        else:
            return False
    return True


def ntt_primes(n, count):
    """The largest primes below 2^30 that are 1 mod 2n."""
    out, c = [], ((1 << 30) - 1) // (2 * n) * (2 * n) + 1
    while len(out) < count:
        if c < (1 << 30) and is_prime(c):
            out.append(c)
        c -= 2 * n
    return out
