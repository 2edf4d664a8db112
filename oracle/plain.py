"""Reference of the plaintext branch, the unidirectional connections' Resize and CRot,
and the plaintext neurons of the feature integration, in FP64 numpy (test
infrastructure only: the GPU path never calls this module).

Section "Our bi-CryptoNets": the plaintext branch sees the whole image with the
sensitive segment filled with zeros and the insensitive part perturbed; it runs
in full precision.  Section "The unidirectional connections": its layer-l maps are
resized to the ciphertext branch's map size (centre crop) and channel-rotated,
CRot^i(y) = sum_j W_CRot^{i,j} y^j, then added to the ciphertext branch.  Section
"The feature integration": plaintext neurons x_p^<1> = sigma(W'_p1 x_p + b'_1);
the ciphertext neurons receive W_p1 x_p + b_1 (first layer) and W_p2 x_p^<1> + b_2
(second layer) from the plaintext side.  sigma is the square (Experiments details);
the plaintext branch's own layers use ReLU (full precision, no HE constraint).
"""
from __future__ import annotations

import numpy as np

from synthetic import workloads as W


def _conv(x, w, b, stride, pad):
    """x [B][C][H][W], w [O][C][k][k] -> [B][O][oh][ow], the definition written out."""
    B, C, H, Wd = x.shape
    O, _, k, _ = w.shape
    xp = np.zeros((B, C, H + 2 * pad, Wd + 2 * pad))
    xp[:, :, pad:pad + H, pad:pad + Wd] = x
    oh = (H + 2 * pad - k) // stride + 1
    ow = (Wd + 2 * pad - k) // stride + 1
    out = np.zeros((B, O, oh, ow))
    for i in range(oh):
        for j in range(ow):
            patch = xp[:, :, stride * i:stride * i + k, stride * j:stride * j + k]
            out[:, :, i, j] = np.tensordot(patch, w, axes=([1, 2, 3], [1, 2, 3]))
    if b is not None:
        out += b[None, :, None, None]
    return out


def run(name: str, inputs) -> dict:
    """The plaintext side of workload `name` for all its images: z1 (features of ciphertext
    layer 1, [B][C1][oh][ow]), u1 and u2 (features of the two integration layers, [B][n]),
    and the intermediate x_p (flattened plaintext-branch output) and x_p^<1>."""
    wl = W.WORKLOADS[name]
    sp = W.plain_shapes(name)
    p, prm = wl["plain"], {k: np.asarray(v, dtype=np.float64) for k, v in inputs["plain"].items()}
    y0, size = wl["crop"]
    x = inputs["images"].astype(np.float64) + prm["noise"]        # perturbed image
    x[:, :, y0:y0 + size, y0:y0 + size] = 0.0                     # sensitive segment: zeros
    x = x / 255.0
    h1 = np.maximum(_conv(x, prm["w1"], prm["b1"], p["stride1"], p["pad1"]), 0.0)
    r, o = sp["resize"], sp["out_hw"]
    y1 = h1[:, :, r:r + o, r:r + o]                               # Resize: centre crop
    z1 = np.einsum("ij,bjhw->bihw", prm["crot"], y1)              # CRot: channel mix
    h2 = np.maximum(_conv(h1, prm["w2"], prm["b2"], p["stride2"], 0), 0.0)
    xp = h2.reshape(h2.shape[0], -1)
    xp1 = (xp @ prm["wpp"].T + prm["bpp"]) ** 2                   # plaintext neurons
    u1 = xp @ prm["wpc"].T + prm["bpc"]
    u2 = xp1 @ prm["wo"].T + prm["bo"]
    return dict(z1=z1, u1=u1, u2=u2, xp=xp, xp1=xp1)
