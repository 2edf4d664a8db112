"""Counter-based random streams and the samplers built on them (test infrastructure only).

The client draws its randomness (secret key, the uniform a and Gaussian e of every
key-switching key and encryption) from ChaCha20 keystreams.  The block function is
the one of RFC 8439 (section 2.3): a 4x4 state of 32-bit words (four constants, an
8-word key, a 32-bit block counter, a 3-word nonce), ten double rounds of quarter
rounds, the input state added to the result, serialised little-endian.

Streams: key = seed as 8 little-endian bytes followed by 24 zero bytes; nonce = the
three words (purpose, index_hi, index_lo); block counter from 0; each 64-bit value is
two consecutive little-endian 32-bit keystream words (low word first).

Samplers, each with a fixed consumption of 64-bit values:
  ternary      (u mod 3) - 1
  uniform q    (u_hi * 2^64 + u_lo) mod q for two consecutive values (bias < 2^-88)
  Gaussian     CDT over k in [-19, 19], rho(k) = exp(-k^2 / (2 sigma^2)), sigma = 3.2:
               T_k = floor(2^64 * CDF(k)) for k = -19 .. 18, and e = -19 + #{k : u >= T_k}
"""
from __future__ import annotations

from decimal import Decimal, getcontext

MASK = 0xFFFFFFFF
SIGMA = Decimal("3.2")
BOUND = 19

# purposes of the streams (nonce word 0)
P_SECRET, P_KSK_A, P_KSK_E, P_ENC_A, P_ENC_E = 1, 2, 3, 4, 5


def _rotl(x: int, n: int) -> int:
    return ((x << n) | (x >> (32 - n))) & MASK


def quarter_round(a: int, b: int, c: int, d: int):
    a = (a + b) & MASK
    d = _rotl(d ^ a, 16)
    c = (c + d) & MASK
    b = _rotl(b ^ c, 12)
    a = (a + b) & MASK
    d = _rotl(d ^ a, 8)
    c = (c + d) & MASK
    b = _rotl(b ^ c, 7)
    return a, b, c, d


def block(key: bytes, counter: int, nonce: bytes) -> bytes:
    """The ChaCha20 block function: 64 keystream bytes."""
    assert len(key) == 32 and len(nonce) == 12
    const = [0x61707865, 0x3320646E, 0x79622D32, 0x6B206574]
    kw = [int.from_bytes(key[4 * i:4 * i + 4], "little") for i in range(8)]
    nw = [int.from_bytes(nonce[4 * i:4 * i + 4], "little") for i in range(3)]
    init = const + kw + [counter & MASK] + nw
    x = list(init)
    for _ in range(10):
        for (a, b, c, d) in ((0, 4, 8, 12), (1, 5, 9, 13), (2, 6, 10, 14), (3, 7, 11, 15),
                             (0, 5, 10, 15), (1, 6, 11, 12), (2, 7, 8, 13), (3, 4, 9, 14)):
            x[a], x[b], x[c], x[d] = quarter_round(x[a], x[b], x[c], x[d])
    return b"".join(((x[i] + init[i]) & MASK).to_bytes(4, "little") for i in range(16))


class Stream:
    """64-bit values of the keystream of (seed, purpose, index)."""

    def __init__(self, seed: int, purpose: int, index: int):
        self.key = int(seed).to_bytes(8, "little") + bytes(24)
        self.nonce = b"".join(int(w).to_bytes(4, "little")
                              for w in (purpose, (index >> 32) & MASK, index & MASK))
        self.counter = 0
        self.buf = []

    def next(self) -> int:
        if not self.buf:
            b = block(self.key, self.counter, self.nonce)
            self.counter += 1
            self.buf = [int.from_bytes(b[8 * i:8 * i + 8], "little") for i in range(8)]
            self.buf.reverse()
        return self.buf.pop()


def cdt_thresholds() -> list[int]:
    """T_k = floor(2^64 CDF(k)), k = -19 .. 18, computed with 60 significant digits."""
    getcontext().prec = 60
    rho = [(-(Decimal(k) ** 2) / (2 * SIGMA ** 2)).exp() for k in range(-BOUND, BOUND + 1)]
    total = sum(rho)
    out, acc = [], Decimal(0)
    for r in rho[:-1]:
        acc += r
        out.append(int((acc / total) * (Decimal(2) ** 64)))
    return out


def ternary(st: Stream, n: int) -> list[int]:
    return [st.next() % 3 - 1 for _ in range(n)]


def uniform(st: Stream, q: int, n: int) -> list[int]:
    out = []
    for _ in range(n):
        hi = st.next()
        lo = st.next()
        out.append(((hi << 64) | lo) % q)
    return out


def gaussian(st: Stream, n: int, table=None) -> list[int]:
    t = cdt_thresholds() if table is None else table
    out = []
    for _ in range(n):
        u = st.next()
        out.append(-BOUND + sum(1 for x in t if u >= x))
    return out


# --------------------------------------------------------------- scheme randomness
# Stream indices: a key-switching key is numbered 0 (relinearisation) or by its Galois
# element k; digit j, prime position i over (Q primes, P primes) of width w = L + K.
# Encryption number r: prime position i over q_1..q_level.

def secret(seed: int, n: int) -> list[int]:
    """The ternary secret key s."""
    return ternary(Stream(seed, P_SECRET, 0), n)


def ksk_randomness(seed: int, key: int, moduli, dnum: int, n: int):
    """(a, e) of one key-switching key: a[j][i] uniform mod moduli[i], e[j] Gaussian."""
    w = len(moduli)
    a = [[uniform(Stream(seed, P_KSK_A, (key << 32) | (j * w + i)), q, n) for i, q in enumerate(moduli)]
         for j in range(dnum)]
    table = cdt_thresholds()
    e = [gaussian(Stream(seed, P_KSK_E, (key << 32) | j), n, table) for j in range(dnum)]
    return a, e


def enc_randomness(seed: int, index: int, moduli, n: int):
    """(a, e) of encryption number `index`: a[i] uniform mod moduli[i] (q_1..q_level), e Gaussian."""
    a = [uniform(Stream(seed, P_ENC_A, (index << 32) | i), q, n) for i, q in enumerate(moduli)]
    e = gaussian(Stream(seed, P_ENC_E, index << 32), n)
    return a, e
