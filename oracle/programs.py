"""Homomorphic programs of the workloads, on the oracle's BFV (test infrastructure only).

The programs follow the appendix "Implementation Details":
  * batch packing: slot b holds image b; one ciphertext per input pixel, and
    a conv or dense layer is a multiply-accumulate of ciphertexts with scalar
    weights (Mult(c,u) by a constant, Add(c1,c2));
  * HW packing: one ciphertext per input channel, pixel (y, x) at slot
    row*y + x of slot row 0 (BHW packing: the same layout in one block of
    slots per image, `batch` images per ciphertext); a convolution rotates the channel ciphertext by
    each kernel offset, multiplies by the scalar kernel weight, sums, and
    multiplies by a mask that keeps the valid output slots;
  * sum pooling ("Homomorphic pooling layer") and the HW dense layer end with
    a rotate-and-sum leaving the sum of the first ``span`` slots in slot 0
    (bfv.rotate_sum: two rounds of hoisted rotations, baby and giant steps,
    each summed over Q_l P and brought down by one ModDown);
  * plaintext-branch features are added after the convolution (and its mask)
    as encoded plaintexts (section "The unidirectional connections");
  * each square activation is followed by relinearisation and, while at least
    two primes remain, a modulus switch.
Rotations of one ciphertext by several kernel offsets share one digit
decomposition (hoisting); a convolution keeps them over Q_l P and divides the
weighted, masked sum by P once per output (bfv.rotations_extended).
"""
from __future__ import annotations

import numpy as np

import synthetic
from synthetic import workloads as W

from . import bfv, network, params, plain
from .encoder import BatchEncoder

RELIN_KEY_ID = W.RELIN_KEY_ID
galois_key_id = W.rotation_key_id


def _span(max_slot: int) -> int:
    s = 1
    while s < max_slot + 1:
        s *= 2
    return s


def plan(name: str):
    """Static layout of a workload: per-layer geometry and the rotation steps it needs."""
    wl = W.WORKLOADS[name]
    shapes = W.layer_shapes(name)
    row = wl["crop"][1]
    ps = 1                      # spacing of valid positions (HW packing)
    steps = set()
    layers = []
    spatial = True
    moved_span = 0
    for li, lay in enumerate(wl["layers"]):
        (cin, *hw_in), out = shapes[li]
        info = dict(lay)
        info["in_shape"], info["out_shape"] = shapes[li][0], out
        if wl["packing"] in ("hw", "bhw"):
            if lay["kind"] == "pool":
                # local sum pooling: like a convolution without weights (channel by channel)
                offs = [ps * (row * di + dj) for di in range(lay["k"]) for dj in range(lay["k"])]
                info["offsets"] = offs
                steps.update(o for o in offs if o)
                ps_out = ps * lay["stride"]
                oh, ow = out[1], out[2]
                info["out_slots"] = [ps_out * (row * i + j) for i in range(oh) for j in range(ow)]
                ps = ps_out
            elif lay["kind"] == "dense" and lay.get("method") == "diag":
                # diagonal method: n1 + n2 - 1 rotations of the input (n1 inputs per channel).  With the
                # outputs in slots 0..n2-1 the steps are r = i - n2, i = 1 .. n1 + n2 - 1, i.e. 1 - n2 .. n1 - 1
                # (the mirror of the printed range n2 - 1 .. 1 - n1, which leaves the outputs at the top
                # of the input range instead)
                # inputs per channel at slots 0..n1-1: the image crop (row = crop width, so the
                # pixels are contiguous) or the previous diagonal layer's outputs
                if li == 0:
                    n1 = row * row
                elif layers[-1].get("method") == "diag":
                    n1 = layers[-1]["out"]
                else:
                    raise ValueError("the diagonal method needs its inputs at slots 0..n1-1")
                n2 = lay["out"]
                info["diag_n1"] = n1
                info["diag_steps"] = [i - n2 for i in range(1, n1 + n2)]
                steps.update(r for r in info["diag_steps"] if r)
                spatial = False
            elif lay["kind"] == "conv":
                offs = [ps * (row * di + dj) for di in range(lay["k"]) for dj in range(lay["k"])]
                info["offsets"] = offs
                steps.update(o for o in offs if o)
                ps_out = ps * lay["stride"]
                oh, ow = out[1], out[2]
                info["out_slots"] = [ps_out * (row * i + j) for i in range(oh) for j in range(ow)]
                ps = ps_out
                if lay.get("sum"):
                    span = _span(max(info["out_slots"]))
                    if wl.get("sum_after_dense"):
                        # the global sum moves after the following (scalar) dense layer
                        moved_span = span
                    else:
                        info["sum_span"] = span
                    steps.update(r for rs in bfv.rotate_sum_steps(span) for r in rs)
                    spatial = False
            elif moved_span:
                info["sum_span"] = moved_span
                moved_span = 0
            elif spatial:
                # dense over spatially laid out channels: weight vectors + rotate-and-sum
                prev = layers[-1]
                info["in_slots"] = prev["out_slots"]
                span = _span(max(prev["out_slots"]))
                info["sum_span"] = span
                steps.update(r for rs in bfv.rotate_sum_steps(span) for r in rs)
                spatial = False
        # a square followed by a scalar dense layer (weights per ciphertext: slot batching, or the
        # dense layer a global sum was moved after) leaves its products unrelinearised; the dense
        # layer's weighted sums run over the three parts and it relinearises its outputs
        scalar = lay["kind"] == "dense" and lay.get("method") != "diag" and "in_slots" not in info
        if layers and layers[-1].get("square") and scalar and not layers[-1].get("sum_span"):
            layers[-1]["defer_relin"] = True
            info["relin_in"] = True
        layers.append(info)
    if wl["packing"] == "bhw":
        n = params.get(wl["params"]).n
        bases = [W.image_base(b, wl["block"], n) for b in range(wl["batch"])]
    else:
        bases = [0]
    return dict(row=row, layers=layers, steps=sorted(steps), bases=bases)


class OracleSession:
    """Keys, encryptions and evaluation of one workload on the oracle."""

    def __init__(self, name: str, seeds=None, with_galois=True, plain_features=None):
        """plain_features: FP32 outputs 'z1', 'u1', 'u2' of the plaintext side for a workload with
        a plaintext branch (default: the FP64 reference of oracle.plain, rounded to FP32)."""
        self.name = name
        self.wl = W.WORKLOADS[name]
        self.prm = params.get(self.wl["params"])
        self.seeds = dict(W.SEEDS if seeds is None else seeds)
        self.enc = BatchEncoder(self.prm.n, self.prm.t)
        self.plan = plan(name)
        prm, n = self.prm, self.prm.n
        self.s = [int(x) for x in synthetic.ternary_secret(self.seeds["keys"], n)]
        moduli = list(prm.q) + list(prm.p)
        a_r, e_r = self.key_randomness(RELIN_KEY_ID)
        self.rk = bfv.relin_key(prm, self.s, a_r, e_r)
        self.gk = {}
        if with_galois:
            for r in self.plan["steps"]:
                self.gk[r] = self.galois(r)
        self.inputs = W.make_inputs(name, self.seeds)
        if "plain" in self.inputs:
            if plain_features is None:
                ref = plain.run(name, self.inputs)
                plain_features = {k: ref[k].astype(np.float32) for k in ("z1", "u1", "u2")}
            self.inputs = W.with_plain_features(self.inputs, name, plain_features)

    def key_randomness(self, key_id: int):
        prm = self.prm
        moduli = list(prm.q) + list(prm.p)
        d = prm.dnum(prm.L)
        a = [synthetic.uniform_residues(self.seeds["keys"], "ksk_a", (key_id, j), moduli, prm.n) for j in range(d)]
        e = [synthetic.gaussian_error(self.seeds["keys"], "ksk_e", (key_id, j), prm.n) for j in range(d)]
        return a, e

    def galois(self, r: int):
        if r not in self.gk:
            a_r, e_r = self.key_randomness(galois_key_id(r))
            self.gk[r] = bfv.galois_key(self.prm, self.s, r, a_r, e_r)
        return self.gk[r]

    # ------------------------------------------------------------ inputs

    def input_slots(self) -> np.ndarray:
        """Slot vectors of the input ciphertexts, [n_ct][N] int64."""
        wl, n = self.wl, self.prm.n
        y0, size = wl["crop"]
        crop = self.inputs["images"][:, :, y0:y0 + size, y0:y0 + size].astype(np.int64)
        if wl["packing"] == "batch":
            b = crop.shape[0]
            flat = crop.reshape(b, -1).T               # [C*H*W][batch], (c, y, x) order
            out = np.zeros((flat.shape[0], n), dtype=np.int64)
            out[:, :b] = flat
            return out
        c = crop.shape[1]
        out = np.zeros((c, n), dtype=np.int64)
        for b, base in enumerate(self.plan["bases"]):
            for ch in range(c):
                for y in range(size):
                    out[ch, base + size * y:base + size * y + size] = crop[b, ch, y]
        return out

    def encrypt_slots(self, slots, index: int, level=None) -> bfv.Ct:
        prm = self.prm
        level = prm.L if level is None else level
        a = synthetic.uniform_residues(self.seeds["enc"], "enc_a", (index,), prm.q[:level], prm.n)
        e = synthetic.gaussian_error(self.seeds["enc"], "enc_e", (index,), prm.n)
        return bfv.encrypt(prm, self.s, self.enc.encode(slots), a, e, level)

    def encrypt_inputs(self, indices=None):
        slots = self.input_slots()
        idx = range(len(slots)) if indices is None else indices
        return {i: self.encrypt_slots(slots[i], i) for i in idx}

    def decrypt_slots(self, ct: bfv.Ct) -> np.ndarray:
        return self.enc.centered(self.enc.decode(bfv.decrypt(self.prm, self.s, ct)))

    # ------------------------------------------------------------ plaintexts

    def feature_slots(self, li: int, o: int) -> np.ndarray:
        """Slot vector of the features added to output map o of layer li (per position)."""
        wl, n = self.wl, self.prm.n
        f = network.quantise(self.inputs["features"][li])
        info = self.plan["layers"][li]
        out = np.zeros(n, dtype=np.int64)
        if wl["packing"] == "batch":
            return f[:, o]                             # [batch][oh][ow]; caller picks (i, j)
        per_image = f if wl["packing"] == "bhw" else f[None]
        for b, base in enumerate(self.plan["bases"]):
            for pos, slot in enumerate(info["out_slots"]):
                i, j = divmod(pos, info["out_shape"][2])
                out[base + slot] = per_image[b, o, i, j]
        return out

    def mask_slots(self, li: int) -> np.ndarray:
        out = np.zeros(self.prm.n, dtype=np.int64)
        for base in self.plan["bases"]:
            out[[base + v for v in self.plan["layers"][li]["out_slots"]]] = 1
        return out

    # ------------------------------------------------------------ layers

    def conv_batch(self, li: int, cts: dict, outputs=None) -> dict:
        """Batch-packed conv (+features, square, modswitch) for output indices ``outputs``.

        cts maps input index (c*H*W + y*W + x) -> Ct; outputs are (o*oh + i)*ow + j.
        """
        prm, info = self.prm, self.plan["layers"][li]
        w = self.inputs["weights"][li]
        cin, h, wd = info["in_shape"]
        O, oh, ow = info["out_shape"]
        k, s, p = info["k"], info["stride"], info["pad"]
        outputs = range(O * oh * ow) if outputs is None else outputs
        res = {}
        for idx in outputs:
            o, rem = divmod(idx, oh * ow)
            i, j = divmod(rem, ow)
            terms, ws = [], []
            for c in range(cin):
                for di in range(k):
                    for dj in range(k):
                        y, x = s * i + di - p, s * j + dj - p
                        if 0 <= y < h and 0 <= x < wd:
                            terms.append(cts[(c * h + y) * wd + x])
                            ws.append(int(w[o, c, di, dj]))
            ct = bfv.mac(prm, terms, ws)
            if info.get("features"):
                fq = network.quantise(self.inputs["features"][li])[:, o, i, j]
                slots = np.zeros(prm.n, dtype=np.int64)
                slots[:len(fq)] = fq
                ct = bfv.add_plain(prm, ct, self.enc.encode(slots))
            res[idx] = self._activation(ct, info)
        return res

    def dense_scalar(self, li: int, cts: dict, outputs=None) -> dict:
        """Scalar dense layer over ciphertexts; with a global sum moved after it (HW packing),
        each output is then rotated-and-summed."""
        prm, info = self.prm, self.plan["layers"][li]
        w = self.inputs["weights"][li]
        n_out, n_in = w.shape
        outputs = range(n_out) if outputs is None else outputs
        res = {}
        for o in outputs:
            if info.get("relin_in"):
                # inputs are unrelinearised products: the sum over three parts, then one key switch
                ct = bfv.relinearize3(prm, bfv.mac3(prm, [cts[i] for i in range(n_in)], [int(x) for x in w[o]]),
                                      self.rk)
            else:
                ct = bfv.mac(prm, [cts[i] for i in range(n_in)], [int(x) for x in w[o]])
            if info.get("features"):
                # batch packing: slot b gets image b's feature of output o
                fq = network.quantise(self.inputs["features"][li])[:, o]
                slots = np.zeros(prm.n, dtype=np.int64)
                slots[:len(fq)] = fq
                ct = bfv.add_plain(prm, ct, self.enc.encode(slots))
            ct = self._activation(ct, info)
            if info.get("sum_span"):
                ct = self.rotate_sum(ct, info["sum_span"])
            res[o] = ct
        return res

    def rotated_input(self, li: int, ct):
        """One input channel of layer li rotated by every kernel offset (hoisted), each
        rotation complete (brought back to Q_l)."""
        offs = self.plan["layers"][li]["offsets"]
        nz = [o for o in offs if o]
        rots = bfv.rotate_hoisted(self.prm, ct, nz, [self.gk[o] for o in nz])
        table = dict(zip(nz, rots))
        table[0] = ct
        return [table[o] for o in offs]

    def extended_input(self, li: int, ct):
        """One input channel of HW conv / pooling layer li at every kernel offset, kept over
        Q_l P before ModDown (hoisted digits; the offset 0 tap is P times the input)."""
        offs = self.plan["layers"][li]["offsets"]
        nz = [o for o in offs if o]
        ext = bfv.rotations_extended(self.prm, ct, [0] + nz, [None] + [self.gk[o] for o in nz])
        table = dict(zip([0] + nz, ext))
        return [table[o] for o in offs]

    def conv_hw(self, li: int, cts: dict, outputs=None, ext=None) -> dict:
        """HW conv layer li for output maps ``outputs``: the taps of every input channel over
        Q_l P (``ext`` may carry them, channel -> list over the kernel offsets, as made by
        extended_input), summed with the weights, times the output mask, then one ModDown;
        then the features and the activation."""
        prm, info = self.prm, self.plan["layers"][li]
        w = self.inputs["weights"][li]
        O, cin, k, _ = w.shape
        level = cts[0].level
        if ext is None:
            ext = {c: self.extended_input(li, cts[c]) for c in range(cin)}
        mask = self.enc.encode(self.mask_slots(li))
        outputs = range(O) if outputs is None else outputs
        res = {}
        for o in outputs:
            terms, ws = [], []
            for c in range(cin):
                for t_i, e in enumerate(ext[c]):
                    di, dj = divmod(t_i, k)
                    terms.append(e)
                    ws.append(int(w[o, c, di, dj]))
            acc = bfv.mac_extended(prm, terms, ws, level)
            ct = bfv.mod_down_ct(prm, bfv.mul_plain_extended(prm, acc, mask, level), level)
            if info.get("features"):
                ct = bfv.add_plain(prm, ct, self.enc.encode(self.feature_slots(li, o)))
            ct = self._activation(ct, info)
            if info.get("sum_span"):
                ct = self.rotate_sum(ct, info["sum_span"])
            res[o] = ct
        return res

    def pool_hw(self, li: int, cts: dict) -> dict:
        """Local sum pooling, channel by channel: the window offsets' taps over Q_l P, summed,
        times the mask of the strided outputs, then one ModDown (appendix "Implementation
        Details", pooling layer: a convolution without weights)."""
        prm, info = self.prm, self.plan["layers"][li]
        mask = self.enc.encode(self.mask_slots(li))
        res = {}
        for c in sorted(cts):
            level = cts[c].level
            taps = self.extended_input(li, cts[c])
            acc = bfv.mac_extended(prm, taps, [1] * len(taps), level)
            res[c] = bfv.mod_down_ct(prm, bfv.mul_plain_extended(prm, acc, mask, level), level)
        return res

    def dense_diag(self, li: int, cts: dict) -> dict:
        """Fully connected layer by the diagonal method (appendix "Implementation Details"):
        channel c holds its n1 inputs at slots 0..n1-1; for i = 1 .. n1 + n2 - 1 the input is
        rotated by r = i - n2 and multiplied by the weight vector whose slot j is W[j][c*n1 + j + r]
        (0 where j + r is outside 0..n1-1); the products are summed.  Output j lands in slot j."""
        prm, info = self.prm, self.plan["layers"][li]
        w = self.inputs["weights"][li]
        n2 = w.shape[0]
        n1 = info["diag_n1"]
        acc = None
        for c in sorted(cts):
            nz = [r for r in info["diag_steps"] if r]
            table = dict(zip(nz, bfv.rotate_hoisted(prm, cts[c], nz, [self.gk[r] for r in nz])))
            table[0] = cts[c]
            for r in info["diag_steps"]:
                v = np.zeros(prm.n, dtype=np.int64)
                for j in range(n2):
                    if 0 <= j + r < n1:
                        v[j] = w[j, c * n1 + j + r]
                if not v.any():
                    continue
                term = bfv.mul_plain(prm, table[r], self.enc.encode(v))
                acc = term if acc is None else bfv.add(prm, acc, term)
        return {0: self._activation(acc, info)}

    def dense_hw(self, li: int, cts: dict, outputs=None) -> dict:
        prm, info = self.prm, self.plan["layers"][li]
        w = self.inputs["weights"][li]
        n_out = w.shape[0]
        cin = len(cts)
        slots_in = info["in_slots"]
        per = len(slots_in)
        outputs = range(n_out) if outputs is None else outputs
        res = {}
        for kk in outputs:
            acc = None
            for c in range(cin):
                v = np.zeros(prm.n, dtype=np.int64)
                for base in self.plan["bases"]:
                    v[[base + x for x in slots_in]] = w[kk, c * per:(c + 1) * per]
                term = bfv.mul_plain(prm, cts[c], self.enc.encode(v))
                acc = term if acc is None else bfv.add(prm, acc, term)
            acc = self.rotate_sum(acc, info["sum_span"])
            res[kk] = self._activation(acc, info)
        return res

    def rotate_sum(self, ct, span: int):
        return bfv.rotate_sum(self.prm, ct, span, self.gk)

    def _activation(self, ct, info):
        if info.get("square") and info.get("defer_relin"):
            ct = bfv.square_unrelinearised(self.prm, ct)
            if ct.level >= 2:
                ct = bfv.modswitch3(self.prm, ct)
        elif info.get("square"):
            ct = bfv.square(self.prm, ct, self.rk)
            if ct.level >= 2:
                ct = bfv.modswitch(self.prm, ct)
        return ct

    # ------------------------------------------------------------ whole program

    def run(self, cts: dict) -> dict:
        hw = self.wl["packing"] in ("hw", "bhw")
        spatial = True
        for li, info in enumerate(self.plan["layers"]):
            if info["kind"] == "pool":
                cts = self.pool_hw(li, cts)
            elif info.get("method") == "diag":
                cts = self.dense_diag(li, cts)
                spatial = False
            elif info["kind"] == "conv":
                cts = self.conv_hw(li, cts) if hw else self.conv_batch(li, cts)
                if info.get("sum"):
                    spatial = False
            elif hw and spatial:
                cts = self.dense_hw(li, cts)
                spatial = False
            else:
                cts = self.dense_scalar(li, cts)
        return cts

    def output_values(self, outs: dict) -> np.ndarray:
        """Decrypted network outputs: batch -> [batch][n_out]; HW -> [1][n_out] (slot 0);
        BHW -> [batch][n_out] (the first slot of each image's block); after a diagonal-method
        layer -> [1][n2] (slots 0..n2-1 of its one ciphertext)."""
        if self.plan["layers"][-1].get("method") == "diag":
            n2 = self.plan["layers"][-1]["out"]
            return self.decrypt_slots(outs[0])[None, :n2]
        vals = [self.decrypt_slots(outs[k]) for k in sorted(outs)]
        if self.wl["packing"] == "batch":
            b = self.wl["batch"]
            return np.stack([v[:b] for v in vals], axis=1)
        return np.array([[v[base] for v in vals] for base in self.plan["bases"]])
