"""BFV over R_Q = Z_Q[X]/(X^N+1) with exact integer definitions (test infrastructure only).

Operation set of the appendix "CKKS Scheme": E, D, Add(c,u), Add(c1,c2),
Mult(c,u), Mult(c1,c2), Rot(c,r).  This module gives each of them its exact
definition in the integer (BFV) scheme implemented here, plus the key
switching that Mult(c1,c2) and Rot(c,r) imply, and modulus switching:

  [x]_M      residue in [0, M);  lift_c(x) = centred residue in (-M/2, M/2)
  Delta(m)   = round(Q_l * [m]_t / t)                          (pt-add scaling)
  E(m)       = (-a*s + e + Delta(m), a) mod Q_l                 (secret-key)
  D(c)       = [round(t * [c0 + c1*s]_Q / Q)]_t
  Mult       d_i = [round(t/Q * (lift_c(c) (x) lift_c(c'))_i)]_Q  (exact tensor over Z)
  KS(x; ksk) u = sum_j D_j * ksk_j mod Q_l*P, D_j = lift_c([x]_{Q_j})  (hybrid digits)
             result = (u - lift_c([u]_P)) / P mod Q_l            (exact round(u/P))
  Rot(c, r)  = (sigma_k c0 + KS(sigma_k c1)_0, KS(sigma_k c1)_1), k = 3^r mod 2N
  modswitch  c' = (c - lift_c([c]_{q_l})) / q_l mod Q_{l-1}    (exact round(c/q_l))

Every rounding is nearest-integer on an exact rational; Q, P, q_i and t are
odd, so no tie can occur.  Polynomials are lists of Python ints.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import nt, ring
from .params import Params


@dataclass
class Ct:
    """A ciphertext (c0, c1) with coefficients in [0, Q_level)."""
    c0: list
    c1: list
    level: int


@dataclass
class Ct3:
    """An unrelinearised product (d0, d1, d2): decrypts as d0 + d1 s + d2 s^2."""
    c0: list
    c1: list
    c2: list
    level: int


@dataclass
class KSKey:
    """Key-switching key: parts[j] = (b_j, a_j) with coefficients in [0, Q_L * P)."""
    parts: list


# ---------------------------------------------------------------- RNS boundary

def from_rns(res, moduli) -> list[int]:
    """CRT of per-modulus residue rows [len(moduli)][N] into integers in [0, prod)."""
    res = np.asarray(res)
    m = 1
    for q in moduli:
        m *= int(q)
    acc = np.zeros(res.shape[1], dtype=object)
    for row, q in zip(res, moduli):
        q = int(q)
        mi = m // q
        coef = mi * pow(mi, -1, q)
        acc = acc + row.astype(object) * coef
    return [int(x) % m for x in acc]


def to_rns(poly, moduli) -> np.ndarray:
    """Residues [len(moduli)][N] (uint64) of integer coefficients."""
    return np.array([[int(x) % int(q) for x in poly] for q in moduli], dtype=np.uint64)


def ct_to_rns(prm: Params, ct: Ct) -> np.ndarray:
    """A ciphertext as [2][level][N] uint64 residues over q_1..q_level."""
    qs = prm.q[:ct.level]
    return np.stack([to_rns(ct.c0, qs), to_rns(ct.c1, qs)])


# ---------------------------------------------------------------- plaintext scaling

def delta(prm: Params, m, level: int) -> list[int]:
    """Delta(m) = round(Q_l * [m]_t / t), coefficient-wise."""
    Q, t = prm.Q(level), prm.t
    return [nt.round_div(Q * (int(x) % t), t) for x in m]


# ---------------------------------------------------------------- keys

def gadget(prm: Params, j: int) -> int:
    """g_j = (Q/Q_j) * [(Q/Q_j)^-1]_{Q_j}: 1 mod the primes of digit j, 0 mod the rest of Q."""
    Q = prm.Q(prm.L)
    Qj = 1
    for x in prm.digit_primes(j, prm.L):
        Qj *= x
    return (Q // Qj) * pow(Q // Qj, -1, Qj)


def ksk_gen(prm: Params, s, s_prime, a_res, e) -> KSKey:
    """Key switching s' -> s: (b_j, a_j), b_j = -a_j*s + e_j + P*g_j*s' mod Q*P.

    a_res[j]: residues [L+K][N] of a_j over (q..., p...); e[j]: error polynomial.
    """
    moduli = list(prm.q) + list(prm.p)
    QP = prm.Q(prm.L) * prm.P
    parts = []
    for j in range(prm.dnum(prm.L)):
        a = from_rns(a_res[j], moduli)
        as_ = ring.negacyclic_mul(a, s)
        pg = prm.P * gadget(prm, j)
        b = [(-x + int(ej) + pg * int(sp)) % QP for x, ej, sp in zip(as_, e[j], s_prime)]
        parts.append((b, a))
    return KSKey(parts)


def relin_key(prm: Params, s, a_res, e) -> KSKey:
    """Relinearisation key: switches s^2 -> s."""
    return ksk_gen(prm, s, ring.negacyclic_mul(s, s), a_res, e)


def galois_element(prm: Params, r: int) -> int:
    """k = 3^r mod 2N; 3 has order N/2 mod 2N, so r is taken mod N/2."""
    return pow(3, r % (prm.n // 2), 2 * prm.n)


def galois_key(prm: Params, s, r: int, a_res, e) -> KSKey:
    """Galois key for a left rotation by r: switches sigma_k(s) -> s."""
    return ksk_gen(prm, s, ring.automorphism(s, galois_element(prm, r)), a_res, e)


# ---------------------------------------------------------------- E / D

def encrypt(prm: Params, s, m, a_res, e, level: int | None = None) -> Ct:
    """Secret-key encryption of plaintext m (coefficients mod t) at the given level.

    a_res: residues [level][N] of the uniform a over q_1..q_level.
    """
    level = prm.L if level is None else level
    Q = prm.Q(level)
    a = from_rns(a_res, prm.q[:level])
    as_ = ring.negacyclic_mul(a, s)
    d = delta(prm, m, level)
    c0 = [(-x + int(ei) + di) % Q for x, ei, di in zip(as_, e, d)]
    return Ct(c0, a, level)


def phase(prm: Params, s, ct: Ct) -> list[int]:
    """[c0 + c1*s]_Q."""
    Q = prm.Q(ct.level)
    c1s = ring.negacyclic_mul(ct.c1, s)
    return [(x + y) % Q for x, y in zip(ct.c0, c1s)]


def decrypt(prm: Params, s, ct: Ct) -> list[int]:
    """m = [round(t * [c0 + c1*s]_Q / Q)]_t, coefficient-wise."""
    Q, t = prm.Q(ct.level), prm.t
    return [nt.round_div(t * x, Q) % t for x in phase(prm, s, ct)]


def noise_budget(prm: Params, s, ct: Ct, m_expected) -> float:
    """Invariant noise budget in bits, measured against the expected plaintext.

    V = lift_c([t*(c0 + c1*s) - Q*m]_{tQ}); decryption returns m exactly when
    |V|_inf < Q/2, i.e. when the budget log2(Q) - 1 - log2|V|_inf is positive.
    """
    Q, t = prm.Q(ct.level), prm.t
    x = phase(prm, s, ct)
    vmax = max(abs(nt.centered(t * xi - Q * (int(mi) % t), t * Q)) for xi, mi in zip(x, m_expected))
    if vmax == 0:
        return float(Q.bit_length())
    return math.log2(Q) - 1 - math.log2(vmax)


# ---------------------------------------------------------------- linear ops

def add(prm: Params, a: Ct, b: Ct) -> Ct:
    assert a.level == b.level
    Q = prm.Q(a.level)
    return Ct(ring.add(a.c0, b.c0, Q), ring.add(a.c1, b.c1, Q), a.level)


def mul_scalar(prm: Params, a: Ct, w: int) -> Ct:
    Q = prm.Q(a.level)
    return Ct(ring.scale(a.c0, w, Q), ring.scale(a.c1, w, Q), a.level)


def mac(prm: Params, cts, weights) -> Ct:
    """sum_j w_j * ct_j mod Q (small signed integer weights)."""
    level = cts[0].level
    Q = prm.Q(level)
    n = prm.n
    c0 = [0] * n
    c1 = [0] * n
    for ct, w in zip(cts, weights):
        w = int(w)
        if w == 0:
            continue
        assert ct.level == level
        c0 = [x + w * y for x, y in zip(c0, ct.c0)]
        c1 = [x + w * y for x, y in zip(c1, ct.c1)]
    return Ct(ring.reduce(c0, Q), ring.reduce(c1, Q), level)


def add_plain(prm: Params, a: Ct, m) -> Ct:
    """Add(c, u): c0 + Delta(m)."""
    Q = prm.Q(a.level)
    return Ct(ring.add(a.c0, delta(prm, m, a.level), Q), list(a.c1), a.level)


def mul_plain(prm: Params, a: Ct, m) -> Ct:
    """Mult(c, u): c_k * lift_c(m mod t) mod Q."""
    Q = prm.Q(a.level)
    mc = ring.lift_c(m, prm.t)
    return Ct(ring.mul(a.c0, mc, Q), ring.mul(a.c1, mc, Q), a.level)


# ---------------------------------------------------------------- Mult(c1, c2)

def tensor(prm: Params, a: Ct, b: Ct):
    """(d0, d1, d2) = [round(t/Q * (lift_c(a) (x) lift_c(b)))]_Q with the tensor exact over Z."""
    assert a.level == b.level
    Q, t = prm.Q(a.level), prm.t
    a0, a1 = ring.lift_c(a.c0, Q), ring.lift_c(a.c1, Q)
    b0, b1 = ring.lift_c(b.c0, Q), ring.lift_c(b.c1, Q)
    d0 = ring.negacyclic_mul(a0, b0)
    d1 = [x + y for x, y in zip(ring.negacyclic_mul(a0, b1), ring.negacyclic_mul(a1, b0))]
    d2 = ring.negacyclic_mul(a1, b1)
    return tuple([nt.round_div(t * x, Q) % Q for x in d] for d in (d0, d1, d2))


def key_switch(prm: Params, x, key: KSKey, level: int):
    """KS(x; key) for x in R_{Q_l}: the pair round(sum_j D_j * key_j / P) mod Q_l."""
    digits = []
    for j in range(prm.dnum(level)):
        Qj = 1
        for qq in prm.digit_primes(j, level):
            Qj *= qq
        digits.append(ring.lift_c(x, Qj))
    return _ks_inner(prm, digits, key, level)


def _ks_inner(prm: Params, digits, key: KSKey, level: int):
    u0, u1 = ks_extended(prm, digits, key, level)
    return mod_down(prm, u0, level), mod_down(prm, u1, level)


def ks_extended(prm: Params, digits, key: KSKey, level: int):
    """The key switch before its division by P: u_k = sum_j D_j * key_j[k] mod Q_l P."""
    QP = prm.Q(level) * prm.P
    out = []
    for part in (0, 1):
        u = [0] * prm.n
        for j, D in enumerate(digits):
            k = [v % QP for v in key.parts[j][part]]
            u = [x + y for x, y in zip(u, ring.negacyclic_mul(D, k))]
        out.append([x % QP for x in u])
    return out[0], out[1]


def mod_down(prm: Params, x, level: int) -> list[int]:
    """ModDown: the nearest integer to x / P, mod Q_l, for x in [0, Q_l P)
    (x minus its centred residue mod P is divisible by P)."""
    Q, P = prm.Q(level), prm.P
    return [((v - nt.centered(v, P)) // P) % Q for v in x]


def relinearize(prm: Params, d, rk: KSKey, level: int) -> Ct:
    Q = prm.Q(level)
    k0, k1 = key_switch(prm, d[2], rk, level)
    return Ct(ring.add(d[0], k0, Q), ring.add(d[1], k1, Q), level)


def multiply(prm: Params, a: Ct, b: Ct, rk: KSKey) -> Ct:
    """Mult(c1, c2) followed by relinearisation."""
    return relinearize(prm, tensor(prm, a, b), rk, a.level)


def square(prm: Params, a: Ct, rk: KSKey) -> Ct:
    """The square activation sigma(x) = x^2 on a ciphertext."""
    return multiply(prm, a, a, rk)


# ---------------------------------------------------------------- deferred relinearisation
# Relinearisation is linear, so a square followed by a linear layer may relinearise the
# linear layer's outputs instead of its inputs: the layer's weighted sums run over the three
# parts (d0, d1, d2) and each output is key-switched once.

def square_unrelinearised(prm: Params, a: Ct) -> Ct3:
    d0, d1, d2 = tensor(prm, a, a)
    return Ct3(d0, d1, d2, a.level)


def modswitch3(prm: Params, a: Ct3) -> Ct3:
    """Drop q_l from each of the three parts (as modswitch)."""
    level = a.level
    assert level >= 2
    ql = prm.q[level - 1]
    Qn = prm.Q(level - 1)

    def one(c):
        return [((x - nt.centered(x, ql)) // ql) % Qn for x in c]

    return Ct3(one(a.c0), one(a.c1), one(a.c2), level - 1)


def mac3(prm: Params, cts, weights) -> Ct3:
    """sum_j w_j * ct_j mod Q over three-part products."""
    level = cts[0].level
    Q = prm.Q(level)
    acc = [[0] * prm.n for _ in range(3)]
    for ct, w in zip(cts, weights):
        w = int(w)
        if w == 0:
            continue
        assert ct.level == level
        for p, part in enumerate((ct.c0, ct.c1, ct.c2)):
            acc[p] = [x + w * y for x, y in zip(acc[p], part)]
    return Ct3(*[ring.reduce(a, Q) for a in acc], level)


def relinearize3(prm: Params, a: Ct3, rk: KSKey) -> Ct:
    return relinearize(prm, (a.c0, a.c1, a.c2), rk, a.level)


# ---------------------------------------------------------------- Rot(c, r)

def rotate(prm: Params, a: Ct, r: int, gk: KSKey) -> Ct:
    """Rot(c, r): both slot rows shift left by r."""
    Q = prm.Q(a.level)
    k = galois_element(prm, r)
    c0 = ring.reduce(ring.automorphism(a.c0, k), Q)
    c1 = ring.reduce(ring.automorphism(a.c1, k), Q)
    k0, k1 = key_switch(prm, c1, gk, a.level)
    return Ct(ring.add(c0, k0, Q), k1, a.level)


def rotate_hoisted(prm: Params, a: Ct, rs, gks) -> list[Ct]:
    """Several rotations of one ciphertext sharing a single digit decomposition.

    The digits D_j = lift_c([c1]_{Q_j}) are computed once; for each step the
    automorphism is applied to the digits over Z, which equals decomposing
    sigma_k(c1) because sigma_k only permutes and negates coefficients and the
    centred lift commutes with negation.
    """
    Q = prm.Q(a.level)
    digits = []
    for j in range(prm.dnum(a.level)):
        Qj = 1
        for qq in prm.digit_primes(j, a.level):
            Qj *= qq
        digits.append(ring.lift_c(a.c1, Qj))
    out = []
    for r, gk in zip(rs, gks):
        k = galois_element(prm, r)
        dk = [ring.automorphism(D, k) for D in digits]
        k0, k1 = _ks_inner(prm, dk, gk, a.level)
        c0 = ring.reduce(ring.automorphism(a.c0, k), Q)
        out.append(Ct(ring.add(c0, k0, Q), k1, a.level))
    return out


# ---------------------------------------------------------------- rotations with deferred ModDown
#
# A weighted sum of rotations (a convolution's taps) needs the division by P of the key
# switch only once, after the sum: each rotation is kept over Q_l P scaled by P,
#   Rot~(c, r) = (P sigma_k(c0) + u0, u1),  u = sum_j sigma_k(D_j) key_j  mod Q_l P,
#   Rot~(c, 0) = (P c0, P c1),
# which decrypts under s to P Rot(c, r) plus the key-switching error, and the sum (times
# any plaintext) is brought back to Q_l by one ModDown.  The P-multiples pass through the
# rounding exactly, so only the key-switching terms are rounded, once.

def _digits(prm: Params, x, level: int):
    out = []
    for j in range(prm.dnum(level)):
        Qj = 1
        for qq in prm.digit_primes(j, level):
            Qj *= qq
        out.append(ring.lift_c(x, Qj))
    return out


def rotations_extended(prm: Params, a: Ct, rs, gks) -> list:
    """[(e0, e1)] over Q_l P for each step r (0 = the ciphertext itself; its key is unused),
    from one digit decomposition of c1."""
    level = a.level
    QP = prm.Q(level) * prm.P
    P = prm.P
    digits = _digits(prm, a.c1, level)
    out = []
    for r, gk in zip(rs, gks):
        if r == 0:
            out.append(([(P * v) % QP for v in a.c0], [(P * v) % QP for v in a.c1]))
            continue
        k = galois_element(prm, r)
        u0, u1 = ks_extended(prm, [ring.automorphism(D, k) for D in digits], gk, level)
        c0 = ring.automorphism(a.c0, k)
        out.append(([(P * x + y) % QP for x, y in zip(c0, u0)], u1))
    return out


def mac_extended(prm: Params, exts, weights, level: int):
    """sum_j w_j * ext_j mod Q_l P (small signed integer weights)."""
    QP = prm.Q(level) * prm.P
    acc = [[0] * prm.n, [0] * prm.n]
    for ext, w in zip(exts, weights):
        w = int(w)
        if w == 0:
            continue
        for part in (0, 1):
            acc[part] = [x + w * y for x, y in zip(acc[part], ext[part])]
    return tuple([x % QP for x in a] for a in acc)


def mul_plain_extended(prm: Params, ext, m, level: int):
    """Both parts times the centred lift of the plaintext m (coefficients mod t), mod Q_l P."""
    QP = prm.Q(level) * prm.P
    ml = ring.lift_c(m, prm.t)
    return tuple(ring.reduce(ring.negacyclic_mul(part, ml), QP) for part in ext)


def mod_down_ct(prm: Params, ext, level: int) -> Ct:
    return Ct(mod_down(prm, ext[0], level), mod_down(prm, ext[1], level), level)


def rotate_sum_steps(span: int):
    """The two rounds of rotate_sum for span = 2^k: baby steps 1 .. b-1 and giant steps
    b, 2b, .., (g-1) b with b = 2^ceil(k/2), g = span / b."""
    k = span.bit_length() - 1
    assert span >= 2 and span == 1 << k
    b = 1 << ((k + 1) // 2)
    g = span // b
    return [list(range(1, b)), [b * j for j in range(1, g)]]


def rotate_sum(prm: Params, a: Ct, span: int, gks) -> Ct:
    """sum_{r < span} Rot(a, r), in two rounds of hoisted rotations kept over Q_l P:
    S1 = ModDown(sum_{r < b} Rot~(a, r)), then S = ModDown(sum_{j < g} Rot~(S1, j b))."""
    for steps in rotate_sum_steps(span):
        if not steps:
            continue
        ext = rotations_extended(prm, a, [0] + steps, [None] + [gks[r] for r in steps])
        a = mod_down_ct(prm, mac_extended(prm, ext, [1] * len(ext), a.level), a.level)
    return a


# ---------------------------------------------------------------- modulus switching

def modswitch(prm: Params, a: Ct) -> Ct:
    """Drop q_l: c' = (c - lift_c([c]_{q_l})) / q_l mod Q_{l-1}."""
    level = a.level
    assert level >= 2
    ql = prm.q[level - 1]
    Qn = prm.Q(level - 1)

    def one(c):
        return [((x - nt.centered(x, ql)) // ql) % Qn for x in c]

    return Ct(one(a.c0), one(a.c1), level - 1)
