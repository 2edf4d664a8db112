"""The real-valued network a CKKS workload evaluates, in FP64 (test infrastructure only).

Section "Experiments": the paper's ciphertext branch runs under CKKS on real values.
Here the inputs are pixel / 255, the weights W / 2^wbits (W the workload's integer
weights) and the plaintext-branch features are added as they are (FP32, no
quantisation); the activation is the square, a 'sum' layer sums each map, and the
dense layer multiplies the flattened vector.  Decrypting the CKKS evaluation must give
these values up to the scheme's approximation error.
"""
from __future__ import annotations

import numpy as np

from synthetic import workloads as W

from .network import conv2d, dense


def run(name: str, inputs, pixel_scale: float = 255.0, wscale: float | None = None) -> np.ndarray:
    """Outputs [1][n_out] (one HW-packed image)."""
    wl = W.WORKLOADS[name]
    wscale = float(2 ** wl["wbits"]) if wscale is None else wscale
    y0, size = wl["crop"]
    x = inputs["images"][:, :, y0:y0 + size, y0:y0 + size].astype(np.float64) / pixel_scale
    for li, lay in enumerate(wl["layers"]):
        w = inputs["weights"][li].astype(np.float64) / wscale
        if lay["kind"] == "conv":
            x = np.stack([_conv(x[b], w, lay["stride"], lay["pad"]) for b in range(x.shape[0])])
            f = inputs["features"][li]
            if f is not None:
                x = x + np.asarray(f, dtype=np.float64)[None]
            if lay["square"]:
                x = x * x
            if lay.get("sum"):
                x = x.reshape(x.shape[0], x.shape[1], -1).sum(axis=2)
        else:
            x = x.reshape(x.shape[0], -1) @ w.T
            if lay["square"]:
                x = x * x
    return x


def _conv(x, w, stride, pad):
    """The integer network's convolution definition evaluated on floats."""
    return np.asarray(conv2d(x.astype(object), w.astype(object), stride, pad), dtype=np.float64)
