"""CRT batching of slot vectors into plaintexts mod t (test infrastructure only).

The appendix "CKKS Scheme" packs a vector of N/2 numbers into the slots of one
plaintext so that additions and multiplications act slot-wise, and defines
Rot(c, r) as a cyclic left shift of that vector by r.  The exact-arithmetic
counterpart used here (BFV batching, t prime, t = 1 mod 2N) has N slots
arranged as 2 rows of N/2:

  slot s = rho*N/2 + i  <->  evaluation point zeta^e(s),
  e(s) = 3^i mod 2N for rho = 0 and e(s) = -3^i mod 2N for rho = 1,

with zeta the smallest primitive 2N-th root of unity mod t.  A plaintext is the
unique m in Z_t[X]/(X^N+1) with m(zeta^e(s)) = v_s; the automorphism
X -> X^(3^r) then shifts both rows left by r, which is the appendix's Rot.
"""
from __future__ import annotations

import numpy as np

from . import nt


class BatchEncoder:
    def __init__(self, n: int, t: int):
        assert (t - 1) % (2 * n) == 0, "t must be 1 mod 2N"
        assert t < (1 << 21), "int64 evaluation below needs t < 2^21"
        self.n, self.t = n, t
        self.zeta = nt.negacyclic_root(t, n)
        half = n // 2
        exps = []
        for s in range(n):
            rho, i = divmod(s, half)
            e = pow(3, i, 2 * n)
            exps.append(e if rho == 0 else (2 * n - e) % (2 * n))
        self.exponent = np.array(exps, dtype=np.int64)          # e(s), odd, distinct
        self.points = np.array([pow(self.zeta, e, t) for e in exps], dtype=np.int64)

    def decode(self, m) -> np.ndarray:
        """Slot values m(zeta^e(s)) mod t, in [0, t); int64 [N] (Horner at all points)."""
        t = self.t
        acc = np.zeros(self.n, dtype=np.int64)
        for k in range(self.n - 1, -1, -1):
            acc = (acc * self.points + int(m[k]) % t) % t
        return acc

    def encode(self, v) -> list[int]:
        """The m in [0, t)^N with m(zeta^e(s)) = v_s mod t.

        Interpolation at the N odd powers x_j = zeta^(2j+1):
        m_k = N^-1 sum_j y_j x_j^-k, with y_j the slot value whose exponent is 2j+1.
        """
        n, t = self.n, self.t
        y = np.zeros(n, dtype=np.int64)
        y[(self.exponent - 1) // 2] = np.asarray(v, dtype=np.int64) % t
        inv_pts = np.array([pow(self.zeta, -(2 * j + 1), t) for j in range(n)], dtype=np.int64)
        ninv = pow(n, -1, t)
        cur = np.ones(n, dtype=np.int64)
        m = []
        for _ in range(n):
            m.append(int((y * cur).sum() % t) * ninv % t)
            cur = cur * inv_pts % t
        return m

    def centered(self, v) -> np.ndarray:
        """Slot values mapped to (-t/2, t/2)."""
        v = np.asarray(v, dtype=np.int64) % self.t
        return np.where(2 * v > self.t, v - self.t, v)
