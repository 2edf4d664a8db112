"""CKKS over R_Q = Z_Q[X]/(X^N+1) with exact ring arithmetic (test infrastructure only).

The paper runs CKKS (section "Experiments": N = 2^14; appendix "CKKS Scheme"): a
ciphertext holds a vector u of n = N/2 fixed-point slot values, and E, D, Add(c,u),
Add(c1,c2), Mult(c,u), Mult(c1,c2), Rot(c,r) act slot by slot, D reproducing the
result up to a small approximation error.  The paper gives only these slot
identities; the definitions below are the standard CKKS ones, on the same RNS
primes, keys and key switching as the BFV oracle:

  zeta = exp(i pi / N); slot i <-> evaluation point zeta^(e_i), e_i = 5^i mod 2N, i < N/2
  encode(z, Delta) = round(Delta * m) coefficient-wise, m the real polynomial of degree < N
                     with m(zeta^(e_i)) = z_i (and conj(z_i) at the conjugate points):
                     m_k = (2/N) Re( sum_i z_i zeta^(-e_i k) )
  decode(m, Delta) = ( m(zeta^(e_i)) / Delta )_i
  E(m)    = (-a s + e + m, a) mod Q_l            D(c) = lift_c([c0 + c1 s]_{Q_l})
  Add(c,u): c0 + m;   Mult(c,u): c_k * m mod Q_l (m a signed integer polynomial)
  Mult    d = (c0 c0', c0 c1' + c1 c0', c1 c1') mod Q_l exactly (no rounding); the scales
          multiply; relinearised with the BFV oracle's key switching
  Rescale c' = (c - lift_c([c]_{q_l})) / q_l mod Q_{l-1} (the BFV modulus switch): the
          scale divides by q_l
  Rot(c, r) = (sigma_k c0 + KS(sigma_k c1)_0, KS(sigma_k c1)_1), k = 5^r mod 2N
"""
from __future__ import annotations

import numpy as np

from . import bfv, ring
from .bfv import Ct
from .params import Params


def slot_exponents(n: int) -> list[int]:
    """e_i = 5^i mod 2N for the N/2 slots."""
    return [pow(5, i, 2 * n) for i in range(n // 2)]


def galois_element(prm: Params, r: int) -> int:
    """k = 5^r mod 2N; 5 has order N/2 mod 2N, so r is taken mod N/2."""
    return pow(5, r % (prm.n // 2), 2 * prm.n)


def _phase(e: np.ndarray, k: np.ndarray, n: int) -> np.ndarray:
    """exp(i pi (e k mod 2N) / N) with the exponent reduced exactly in integers."""
    return np.exp(1j * np.pi * ((np.outer(e, k) % (2 * n)).astype(np.float64)) / n)


def embed_inverse(z, n: int) -> np.ndarray:
    """The real polynomial m with m(zeta^(e_i)) = z_i: m_k = (2/N) Re(sum_i z_i zeta^(-e_i k)),
    evaluated in complex128 (row blocks of the N x N/2 matrix)."""
    z = np.asarray(z, dtype=np.complex128)
    e = np.array(slot_exponents(n), dtype=np.int64)
    out = np.empty(n)
    for k0 in range(0, n, 512):
        k = np.arange(k0, min(n, k0 + 512), dtype=np.int64)
        out[k0:k0 + len(k)] = (2.0 / n) * np.real(np.conj(_phase(e, k, n)).T @ z)
    return out


def embed(m, n: int) -> np.ndarray:
    """(m(zeta^(e_i)))_i for a polynomial with (float-representable) real coefficients."""
    m = np.asarray([float(x) for x in m])
    e = np.array(slot_exponents(n), dtype=np.int64)
    out = np.empty(n // 2, dtype=np.complex128)
    k = np.arange(n, dtype=np.int64)
    for i0 in range(0, n // 2, 256):
        out[i0:i0 + 256] = _phase(e[i0:i0 + 256], k, n) @ m
    return out


def encode(z, scale: float, n: int) -> list[int]:
    """round(Delta * m) for the slot vector z (real or complex, length <= N/2, zero padded)."""
    zz = np.zeros(n // 2, dtype=np.complex128)
    zz[:len(z)] = z
    return [int(v) for v in np.rint(scale * embed_inverse(zz, n)).astype(np.int64)]


def decode(m, scale: float, n: int) -> np.ndarray:
    """Slot values m(zeta^(e_i)) / Delta (complex)."""
    return embed(m, n) / scale


# ---------------------------------------------------------------- keys

def galois_key(prm: Params, s, r: int, a_res, e) -> bfv.KSKey:
    """Key for Rot(c, r): switches sigma_k(s) -> s, k = 5^r mod 2N."""
    return bfv.ksk_gen(prm, s, ring.automorphism(s, galois_element(prm, r)), a_res, e)


# ---------------------------------------------------------------- E / D

def encrypt(prm: Params, s, m, a_res, e, level: int | None = None) -> Ct:
    """(-a s + e + m, a) mod Q_l for an encoded (integer) plaintext m."""
    level = prm.L if level is None else level
    Q = prm.Q(level)
    a = bfv.from_rns(a_res, prm.q[:level])
    c0 = [(-x + int(ei) + int(mi)) % Q for x, ei, mi in zip(ring.negacyclic_mul(a, s), e, m)]
    return Ct(c0, a, level)


def decrypt(prm: Params, s, ct: Ct) -> list[int]:
    """lift_c([c0 + c1 s]_{Q_l}): Delta * (slot values) plus the noise, as signed integers."""
    Q = prm.Q(ct.level)
    x = [(a + b) % Q for a, b in zip(ct.c0, ring.negacyclic_mul(ct.c1, s))]
    return ring.lift_c(x, Q)


# ---------------------------------------------------------------- operations

def add_plain(prm: Params, ct: Ct, m) -> Ct:
    """Add(c, u) for an encoded u at the ciphertext's scale."""
    Q = prm.Q(ct.level)
    return Ct([(a + int(b)) % Q for a, b in zip(ct.c0, m)], list(ct.c1), ct.level)


def mul_plain(prm: Params, ct: Ct, m) -> Ct:
    """Mult(c, u) for an encoded u: both parts times the signed integer polynomial m."""
    Q = prm.Q(ct.level)
    return Ct(ring.mul(ct.c0, m, Q), ring.mul(ct.c1, m, Q), ct.level)


def tensor(prm: Params, a: Ct, b: Ct):
    """(d0, d1, d2) = (a0 b0, a0 b1 + a1 b0, a1 b1) mod Q_l, exact."""
    Q = prm.Q(a.level)
    d0 = ring.mul(a.c0, b.c0, Q)
    d1 = ring.add(ring.mul(a.c0, b.c1, Q), ring.mul(a.c1, b.c0, Q), Q)
    d2 = ring.mul(a.c1, b.c1, Q)
    return d0, d1, d2


def square_relin(prm: Params, a: Ct, rk: bfv.KSKey) -> Ct:
    """Mult(c, c) relinearised (scale squared; no rescale)."""
    return bfv.relinearize(prm, tensor(prm, a, a), rk, a.level)


def rescale(prm: Params, a: Ct) -> Ct:
    """Divide by the last prime with exact nearest rounding (the scale divides by q_l)."""
    return bfv.modswitch(prm, a)


def rotate(prm: Params, a: Ct, r: int, gk: bfv.KSKey) -> Ct:
    """Rot(c, r): the slot vector shifts left by r."""
    Q = prm.Q(a.level)
    k = galois_element(prm, r)
    c0 = ring.reduce(ring.automorphism(a.c0, k), Q)
    c1 = ring.reduce(ring.automorphism(a.c1, k), Q)
    k0, k1 = bfv.key_switch(prm, c1, gk, a.level)
    return Ct(ring.add(c0, k0, Q), k1, a.level)
