"""The integer-quantised network that Dec(Eval(.)) must equal (test infrastructure only).

Layer semantics follow the appendix "Implementation Details": a fully
connected layer b_j = sum_i a_i w_{i,j}; a convolution
b_{y,x} = sum_{i,j} a_{s*y+i-p, s*x+j-p} f_{i,j} (the printed index ranges are
garbled; this is the standard reading, with zero padding p and stride s);
sum pooling adds without weights; the activation is the square (Experiments
details).  Plaintext-branch features enter the ciphertext branch by addition
after the convolution (section "The unidirectional connections"), quantised to
integers as q(f) = clamp(rint(8 f), -127, 127) computed in FP32.

Arithmetic is exact over Z (object arrays of Python ints) unless ``t`` is
given, in which case every layer is reduced mod t in int64; reduction mod t is
a ring homomorphism, so both give the same result mod t (a test pins this).
"""
from __future__ import annotations

import numpy as np

from synthetic import workloads as W


def quantise(f) -> np.ndarray:
    """q(f) = clamp(rint(8 f), -127, 127) evaluated in float32, as int64."""
    f = np.asarray(f, dtype=np.float32)
    return np.clip(np.rint(np.float32(8.0) * f), -127, 127).astype(np.int64)


def _red(x, t):
    return x if t is None else np.mod(x, t)


def conv2d(x, w, stride: int, pad: int, t=None):
    """x [..., C, H, W], w [O][C][k][k] -> [..., O, oh, ow] (leading axes are a batch)."""
    *lead, C, H, Wd = x.shape
    O, C2, k, _ = w.shape
    assert C == C2
    dt = object if t is None else np.int64
    xp = np.zeros(tuple(lead) + (C, H + 2 * pad, Wd + 2 * pad), dtype=dt)
    xp[..., pad:pad + H, pad:pad + Wd] = x
    oh = (H + 2 * pad - k) // stride + 1
    ow = (Wd + 2 * pad - k) // stride + 1
    out = np.zeros(tuple(lead) + (O, oh, ow), dtype=dt)
    wv = w.astype(dt)
    for o in range(O):
        for i in range(oh):
            for j in range(ow):
                patch = xp[..., stride * i:stride * i + k, stride * j:stride * j + k]
                out[..., o, i, j] = (patch * wv[o]).sum(axis=(-3, -2, -1))
    return _red(out, t)


def sum_pool(x, k: int, stride: int, t=None):
    """Local sum pooling: x [..., C, H, W] -> [..., C, oh, ow], each output the sum of its
    k x k window (no weights)."""
    *lead, C, H, Wd = x.shape
    oh, ow = (H - k) // stride + 1, (Wd - k) // stride + 1
    out = np.zeros(tuple(lead) + (C, oh, ow), dtype=x.dtype)
    for i in range(oh):
        for j in range(ow):
            out[..., i, j] = x[..., stride * i:stride * i + k, stride * j:stride * j + k].sum(axis=(-2, -1))
    return _red(out, t)


def dense(x, w, t=None):
    """x [..., n_in], w [n_out][n_in] -> [..., n_out]."""
    dt = object if t is None else np.int64
    return _red(x.astype(dt) @ w.astype(dt).T, t)


def run(name: str, inputs, images=None, t=None):
    """Outputs of the integer network of workload ``name`` (mod t if given).

    ``images`` selects image indices (default: all); the result has a leading
    batch axis [len(images)][...].
    """
    wl = W.WORKLOADS[name]
    y0, size = wl["crop"]
    dt = object if t is None else np.int64
    idx = np.arange(wl["batch"]) if images is None else np.asarray(images)
    x = inputs["images"][idx][:, :, y0:y0 + size, y0:y0 + size].astype(dt)
    batch = wl["packing"] in ("batch", "bhw")
    for li, lay in enumerate(wl["layers"]):
        w = inputs["weights"][li]
        if lay["kind"] == "pool":
            x = sum_pool(x, lay["k"], lay["stride"], t)
        elif lay["kind"] == "conv":
            x = conv2d(x, w, lay["stride"], lay["pad"], t)
            f = inputs["features"][li]
            if f is not None:
                fq = quantise(f[idx] if batch else f[None])
                x = _red(x + fq.astype(dt), t)
            if lay["square"]:
                x = _red(x * x, t)
            if lay.get("sum"):
                x = _red(x.reshape(x.shape[0], x.shape[1], -1).sum(axis=2), t)
        else:
            x = dense(x.reshape(x.shape[0], -1), w, t)
            f = inputs["features"][li]
            if f is not None:
                # plaintext terms of the integration layer's ciphertext neurons (batch packing)
                x = _red(x + quantise(f[idx]).astype(dt), t)
            if lay["square"]:
                x = _red(x * x, t)
    return x


def run_mod_t(name: str, inputs, t: int, images=None) -> np.ndarray:
    """Centred residues mod t of the network outputs, [batch][...]."""
    y = np.asarray(run(name, inputs, images, t), dtype=np.int64) % t
    return np.where(2 * y > t, y - t, y)


def first_layer_linear(name: str, inputs, images=None, t=None):
    """Output of the first layer's convolution (+features), before the square."""
    wl = W.WORKLOADS[name]
    y0, size = wl["crop"]
    dt = object if t is None else np.int64
    idx = np.arange(wl["batch"]) if images is None else np.asarray(images)
    x = inputs["images"][idx][:, :, y0:y0 + size, y0:y0 + size].astype(dt)
    lay = wl["layers"][0]
    x = conv2d(x, inputs["weights"][0], lay["stride"], lay["pad"], t)
    f = inputs["features"][0]
    if f is not None:
        fq = quantise(f[idx] if wl["packing"] in ("batch", "bhw") else f[None])
        x = _red(x + fq.astype(dt), t)
    return x
