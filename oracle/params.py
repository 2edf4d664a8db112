"""Parameter sets (test infrastructure only).

Primes: the largest b-bit primes q = 1 (mod 2N), in descending order; the
first L form the ciphertext modulus Q = q_1...q_L and the next K form the
special modulus P used by key switching.  Key-switching digits are
contiguous groups of ``alpha`` primes of Q, in order.  These rules are this
build's reading: the paper states only "CKKS, N = 2^14" (Experiments
section) and leaves the moduli unstated.
"""
from __future__ import annotations

from dataclasses import dataclass, field

from synthetic import workloads as W

from . import nt


@dataclass(frozen=True)
class Params:
    name: str
    n: int
    q: tuple          # ciphertext primes, q[0] first
    p: tuple          # special primes
    t: int            # plaintext modulus
    alpha: int        # primes per key-switching digit
    insecure: bool = False

    @property
    def L(self) -> int:
        return len(self.q)

    @property
    def K(self) -> int:
        return len(self.p)

    @property
    def P(self) -> int:
        out = 1
        for x in self.p:
            out *= x
        return out

    def Q(self, level: int) -> int:
        out = 1
        for x in self.q[:level]:
            out *= x
        return out

    def dnum(self, level: int) -> int:
        """Number of digits with at least one prime at this level."""
        return -(-level // self.alpha)

    def digit_primes(self, j: int, level: int) -> tuple:
        """Primes of digit j that are still present at this level."""
        return self.q[j * self.alpha:min((j + 1) * self.alpha, level)]


def make(name: str, n: int, bits: int, L: int, K: int, alpha: int, t: int, insecure=False) -> Params:
    primes = nt.ntt_primes(bits, 2 * n, L + K, exclude={t})
    return Params(name, n, tuple(primes[:L]), tuple(primes[L:]), t, alpha, insecure)


_SPECS = W.PARAMS

_CACHE: dict = {}


def get(name: str) -> Params:
    if name not in _CACHE:
        _CACHE[name] = make(name, **_SPECS[name])
    return _CACHE[name]


def names() -> list[str]:
    return list(_SPECS)
