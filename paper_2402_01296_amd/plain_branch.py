"""The plaintext side of bi-CryptoNets in FP32 on the GPU: the plaintext branch,
Resize (centre crop) and CRot (channel mix) of the unidirectional connections,
and the plaintext neurons of the feature integration.

Section "Our bi-CryptoNets": the plaintext branch sees the whole image with the
sensitive segment zeroed and the insensitive part perturbed, in full precision;
it can run in parallel with the ciphertext branch.  Section "The unidirectional
connections": z_l = CRot_l(Resize_l(x_p,l)) is added to the ciphertext branch.
Section "The feature integration": x_p^<1> = sigma(W'_p1 x_p + b'_1); the
ciphertext neurons receive W_p1 x_p + b_1 and W_p2 x_p^<1> + b_2.  sigma is the
square; the plaintext branch's own layers use ReLU.

This is ordinary dense FP32 network work (not homomorphic), run with torch's
convolution and matrix kernels on its own stream, so it overlaps the
ciphertext branch's kernels.
"""
from __future__ import annotations

import numpy as np

from synthetic import workloads as W


class PlainBranch:
    def __init__(self, name: str, params: dict):
        import torch
        self.torch = torch
        torch.backends.cuda.matmul.allow_tf32 = False
        torch.backends.cudnn.allow_tf32 = False
        self.wl = W.WORKLOADS[name]
        self.p = self.wl["plain"]
        self.sp = W.plain_shapes(name)
        self.w = {k: torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32)).cuda()
                  for k, v in params.items() if k != "noise"}

    def first(self, images, noise):
        """Layer 1 of the plaintext branch and its connection to ciphertext layer 1.
        images: uint8 [B][C][H][W], noise: FP32 [B][C][H][W] (device).  Returns the layer-1
        map h1 and z1 = CRot(Resize(h1)), FP32 [B][C1][oh][ow]."""
        torch, F, w, p = self.torch, self.torch.nn.functional, self.w, self.p
        y0, size = self.wl["crop"]
        x = images.to(torch.float32) + noise
        x[:, :, y0:y0 + size, y0:y0 + size] = 0.0
        x = x / 255.0
        h1 = torch.relu(F.conv2d(x, w["w1"], w["b1"], stride=p["stride1"], padding=p["pad1"]))
        r, o = self.sp["resize"], self.sp["out_hw"]
        z1 = F.conv2d(h1[:, :, r:r + o, r:r + o], w["crot"][:, :, None, None])
        return h1, z1.contiguous()

    def rest(self, h1):
        """Layer 2 of the plaintext branch and the integration layer's plaintext side:
        u1 = W_p1 x_p + b_1 [B][n1/2] and u2 = W_p2 x_p^<1> + b_2 [B][n2]."""
        torch, F, w, p = self.torch, self.torch.nn.functional, self.w, self.p
        h2 = torch.relu(F.conv2d(h1, w["w2"], w["b2"], stride=p["stride2"]))
        xp = h2.reshape(h2.shape[0], -1)
        xp1 = torch.square(xp @ w["wpp"].T + w["bpp"])
        u1 = xp @ w["wpc"].T + w["bpc"]
        u2 = xp1 @ w["wo"].T + w["bo"]
        return u1.contiguous(), u2.contiguous()

    def __call__(self, images, noise):
        """All plaintext-side outputs: z1, u1, u2 (device FP32)."""
        h1, z1 = self.first(images, noise)
        u1, u2 = self.rest(h1)
        return dict(z1=z1, u1=u1, u2=u2)
