"""The ring R = Z[X]/(X^N + 1) and its quotients R_M (test infrastructure only).

The ciphertext ring of the appendix "CKKS Scheme" is Z_p[x]/(x^N+1) with
p = q_1...q_l.  Here a polynomial is a Python list of N exact integers
(coefficient of X^i at index i); reduction mod M is explicit.

The product is the definition of multiplication in Z[X]/(X^N+1):
c_k = sum_{i+j=k} a_i b_j - sum_{i+j=k+N} a_i b_j.  ``negacyclic_mul``
evaluates it with one big-integer product (Kronecker substitution: pack the
coefficients as base-2^w digits, multiply, unpack), which is exact because
the digit width leaves room for every coefficient of the full product.
``schoolbook_mul`` is the double loop, kept to pin ``negacyclic_mul``.
"""
from __future__ import annotations

import numpy as np


def _offset(count: int, nbytes: int) -> int:
    """sum_{k<count} 2^(8*nbytes-1) * 2^(8*nbytes*k)."""
    return int.from_bytes((1 << (8 * nbytes - 1)).to_bytes(nbytes, "little") * count, "little")


def _pack(coeffs, nbytes: int) -> int:
    """The integer sum_k c_k 2^(8*nbytes*k) for signed c_k with |c_k| < 2^(8*nbytes-1)."""
    off = 1 << (8 * nbytes - 1)
    data = b"".join((int(c) + off).to_bytes(nbytes, "little") for c in coeffs)
    return int.from_bytes(data, "little") - _offset(len(coeffs), nbytes)


def _unpack(x: int, count: int, nbytes: int) -> list[int]:
    """Inverse of ``_pack`` for ``count`` signed digits."""
    off = 1 << (8 * nbytes - 1)
    data = (x + _offset(count, nbytes)).to_bytes(count * nbytes, "little")
    return [int.from_bytes(data[i * nbytes:(i + 1) * nbytes], "little") - off for i in range(count)]


def negacyclic_mul(a, b) -> list[int]:
    """Exact product of a and b in Z[X]/(X^N+1) (signed integer coefficients)."""
    n = len(a)
    assert len(b) == n
    amax = max((abs(int(x)) for x in a), default=0)
    bmax = max((abs(int(x)) for x in b), default=0)
    if amax == 0 or bmax == 0:
        return [0] * n
    bound = n * amax * bmax                       # |coefficient of the full product| <= bound
    nbytes = (bound.bit_length() + 2 + 7) // 8    # signed digit with a spare bit
    full = _unpack(_pack(a, nbytes) * _pack(b, nbytes), 2 * n, nbytes)
    return [full[k] - full[k + n] for k in range(n)]


def schoolbook_mul(a, b) -> list[int]:
    """The double-loop definition of the product in Z[X]/(X^N+1)."""
    n = len(a)
    c = [0] * n
    for i in range(n):
        for j in range(n):
            k = i + j
            if k < n:
                c[k] += int(a[i]) * int(b[j])
            else:
                c[k - n] -= int(a[i]) * int(b[j])
    return c


def reduce(a, m: int) -> list[int]:
    """Coefficients reduced to [0, m)."""
    return [int(x) % m for x in a]


def lift_c(a, m: int) -> list[int]:
    """Centred lift: each coefficient mapped to its representative in (-m/2, m/2)."""
    out = []
    for x in a:
        r = int(x) % m
        out.append(r - m if 2 * r > m else r)
    return out


def add(a, b, m: int) -> list[int]:
    return [(int(x) + int(y)) % m for x, y in zip(a, b)]


def sub(a, b, m: int) -> list[int]:
    return [(int(x) - int(y)) % m for x, y in zip(a, b)]


def neg(a, m: int) -> list[int]:
    return [(-int(x)) % m for x in a]


def scale(a, w: int, m: int) -> list[int]:
    return [(int(x) * int(w)) % m for x in a]


def mul(a, b, m: int) -> list[int]:
    """Product in R_m = Z_m[X]/(X^N+1) of any integer representatives."""
    return reduce(negacyclic_mul(a, b), m)


def automorphism(a, k: int) -> list[int]:
    """sigma_k: a(X) -> a(X^k) in Z[X]/(X^N+1), k odd.

    X^(i*k) = (-1)^floor(i*k/N) X^((i*k) mod N).
    """
    n = len(a)
    assert k % 2 == 1
    out = [0] * n
    for i, x in enumerate(a):
        e = i * k % (2 * n)
        if e < n:
            out[e] += int(x)
        else:
            out[e - n] -= int(x)
    return out


def ntt(a, q: int, psi: int) -> list[int]:
    """Negacyclic NTT by its definition: out[j] = sum_k a_k psi^((2j+1)k) mod q.

    psi is a primitive 2N-th root of unity mod q; output in natural order j.
    Evaluated with Horner's rule at all N points at once (exact integers).
    """
    n = len(a)
    pts = np.array([pow(psi, 2 * j + 1, q) for j in range(n)], dtype=object)
    acc = np.zeros(n, dtype=object)
    for k in range(n - 1, -1, -1):
        acc = (acc * pts + int(a[k])) % q
    return [int(x) for x in acc]


def ntt_at(a, q: int, psi: int, j: int) -> int:
    """One output of ``ntt``: a(psi^(2j+1)) mod q."""
    x = pow(psi, 2 * j + 1, q)
    acc = 0
    for k in range(len(a) - 1, -1, -1):
        acc = (acc * x + int(a[k])) % q
    return acc
