"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module holds *no* arithmetic of the homomorphic scheme: it only draws
random numbers.  Every random value the method consumes (the ternary secret,
the uniform ``a`` polynomials of encryptions and key-switching keys, the
Gaussian errors) is drawn here and handed to both implementations as an
input, so neither side needs a sampler of its own.  Images, integer weights
and the FP32 plaintext-branch features that stand in for the paper's datasets
(MNIST 28x28x1, CIFAR 32x32x3; Experiments section) are drawn here too.

Every stream is a counter-based Philox generator keyed by
``(seed, purpose, index...)`` through ``numpy.random.SeedSequence``, so any
piece can be regenerated on its own, in any order.
"""
from __future__ import annotations

import numpy as np

# Stream purposes.  Their numeric codes are part of the seed derivation and
# must never be renumbered.
PURPOSES = {
    "sk": 1,        # ternary secret key
    "ksk_a": 2,     # uniform a_j of a key-switching key (key id, digit)
    "ksk_e": 3,     # Gaussian e_j of a key-switching key (key id, digit)
    "enc_a": 4,     # uniform a of a fresh ciphertext (ciphertext index)
    "enc_e": 5,     # Gaussian e of a fresh ciphertext (ciphertext index)
    "img": 6,       # uint8 images
    "w": 7,         # integer layer weights (layer index)
    "feat": 8,      # FP32 plaintext-branch features (layer index)
    "req": 9,       # request mix / arrival times of the batched workloads
    "poly": 10,     # generic test polynomials
    "pw": 11,       # FP32 weights of the plaintext branch and the integration layer (tensor index)
    "pnoise": 12,   # Gaussian perturbation of the insensitive segment (image index range)
}

SIGMA = 3.2          # standard deviation of the error distribution
ERROR_BOUND = 19     # tail cut: |e| <= 19 (about 6 sigma)


def rng(seed: int, purpose: str, *index: int) -> np.random.Generator:
    """Independent Philox stream for ``(seed, purpose, index...)``."""
    words = [int(seed) & 0xFFFFFFFF, (int(seed) >> 32) & 0xFFFFFFFF, PURPOSES[purpose]]
    words += [int(i) & 0xFFFFFFFF for i in index]
    return np.random.Generator(np.random.Philox(np.random.SeedSequence(words)))


def ternary_secret(seed: int, n: int) -> np.ndarray:
    """Secret-key coefficients, uniform over {-1, 0, 1}; int8 [n]."""
    return rng(seed, "sk").integers(-1, 2, size=n, dtype=np.int8)


def uniform_residues(seed: int, purpose: str, index: tuple, moduli, n: int) -> np.ndarray:
    """Uniform residues, row i uniform in [0, moduli[i]); uint64 [len(moduli)][n].

    Independent uniform residues per modulus are, by the Chinese remainder
    theorem, a uniform element of Z_M with M the product of the moduli.
    """
    g = rng(seed, purpose, *index)
    out = np.empty((len(moduli), n), dtype=np.uint64)
    for i, q in enumerate(moduli):
        out[i] = g.integers(0, int(q), size=n, dtype=np.uint64)
    return out


def gaussian_error(seed: int, purpose: str, index: tuple, n: int) -> np.ndarray:
    """Rounded Gaussian errors, sigma = 3.2, cut at |e| <= 19; int8 [n]."""
    g = rng(seed, purpose, *index)
    e = np.rint(g.normal(0.0, SIGMA, size=n))
    return np.clip(e, -ERROR_BOUND, ERROR_BOUND).astype(np.int8)


def images(seed: int, count: int, height: int, width: int, channels: int = 1) -> np.ndarray:
    """Uniform uint8 images, [count][channels][height][width]."""
    return rng(seed, "img").integers(0, 256, size=(count, channels, height, width), dtype=np.uint8)


def int_weights(seed: int, layer: int, shape, bound: int) -> np.ndarray:
    """Integer weights uniform in [-bound, bound]; int32 of the given shape."""
    return rng(seed, "w", layer).integers(-bound, bound + 1, size=shape, dtype=np.int32)


def features(seed: int, layer: int, shape) -> np.ndarray:
    """FP32 plaintext-branch features, N(0, 2^2); float32 of the given shape."""
    return rng(seed, "feat", layer).normal(0.0, 2.0, size=shape).astype(np.float32)


def test_poly(seed: int, index: int, moduli, n: int) -> np.ndarray:
    """Generic uniform RNS test polynomial; uint64 [len(moduli)][n]."""
    return uniform_residues(seed, "poly", (index,), moduli, n)


def float_weights(seed: int, index: int, shape, scale: float) -> np.ndarray:
    """FP32 weights uniform in [-scale, scale]; float32 of the given shape."""
    return (rng(seed, "pw", index).uniform(-1.0, 1.0, size=shape) * scale).astype(np.float32)


def perturbation(seed: int, shape, sigma: float) -> np.ndarray:
    """Gaussian perturbation N(0, sigma^2) on the uint8 pixel scale; float32 of the given shape."""
    return rng(seed, "pnoise").normal(0.0, sigma, size=shape).astype(np.float32)
