"""Number theory for the oracle (test infrastructure only).

Everything here is the plain definition: primality by trial division, roots
of unity by exhaustive search for the smallest one, CRT by the textbook
formula.
"""
from __future__ import annotations

import math

import numpy as np


def is_prime(n: int) -> bool:
    """Primality by trial division by every odd d <= sqrt(n)."""
    n = int(n)
    if n < 2:
        return False
    if n % 2 == 0:
        return n == 2
    r = math.isqrt(n)
    if r < 3:
        return True
    # vectorised trial division; values stay far below 2^63
    step = 1 << 20
    for lo in range(3, r + 1, step):
        d = np.arange(lo, min(lo + step, r + 1), 2, dtype=np.int64)
        if np.any(n % d == 0):
            return False
    return True


def ntt_primes(bits: int, two_n: int, count: int, exclude=()) -> list[int]:
    """The ``count`` largest primes p < 2^bits with p = 1 (mod two_n), descending."""
    out = []
    k = ((1 << bits) - 2) // two_n
    while len(out) < count:
        p = k * two_n + 1
        if p < (1 << (bits - 1)):
            raise ValueError("ran out of %d-bit primes" % bits)
        if p not in exclude and is_prime(p):
            out.append(p)
        k -= 1
    return out


def negacyclic_root(q: int, n: int) -> int:
    """Smallest x >= 2 with x^n = -1 (mod q): a primitive 2n-th root of unity.

    The solutions of x^n = -1 are exactly the odd powers of any one of them
    (n = power of two), and psi0 = g^((q-1)/2n) is one whenever g is a
    quadratic non-residue (psi0^n = g^((q-1)/2) = -1).  So the smallest
    solution is the minimum over psi0^k, k odd < 2n.
    """
    assert (q - 1) % (2 * n) == 0
    g = 2
    while pow(g, (q - 1) // 2, q) != q - 1:
        g += 1
    psi0 = pow(g, (q - 1) // (2 * n), q)
    sq = psi0 * psi0 % q
    best, x = q, psi0
    for _ in range(n):
        best = min(best, x)
        x = x * sq % q
    return best


def negacyclic_root_search(q: int, n: int) -> int:
    """The same root by exhaustive search (small q only; pins the fast form)."""
    for x in range(2, q):
        if pow(x, n, q) == q - 1:
            return x
    raise ValueError("no primitive 2n-th root modulo %d" % q)


def crt(residues, moduli) -> int:
    """The x in [0, prod(moduli)) with x = residues[i] (mod moduli[i])."""
    m = 1
    for q in moduli:
        m *= int(q)
    x = 0
    for r, q in zip(residues, moduli):
        q = int(q)
        mi = m // q
        x += int(r) * mi * pow(mi, -1, q)
    return x % m


def centered(x: int, m: int) -> int:
    """The representative of x mod m in (-m/2, m/2] (m odd: in (-m/2, m/2))."""
    r = int(x) % m
    return r - m if 2 * r > m else r


def round_div(a: int, b: int) -> int:
    """Nearest integer to a/b for b > 0 (ties toward +inf; callers rule ties out)."""
    return (2 * a + b) // (2 * b)
