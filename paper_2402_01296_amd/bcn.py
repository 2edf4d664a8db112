"""ctypes binding of the C ABI in include/bcn.h (argument marshalling only).

Device buffers are torch tensors on the GPU (float64 ciphertexts
[n][2][level][N], float32 features); the stream is torch's current stream.
Every arithmetic step runs in the HIP library; importing this module never
falls back to anything else: a missing library raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libbcn.so")

BCN_KEY_RELIN, BCN_KEY_ROTATION = 0, 1
BCN_CONV2D, BCN_DENSE, BCN_POOL = 0, 1, 2
BCN_DENSE_WEIGHT_VECTORS, BCN_DENSE_DIAGONAL = 0, 1
BCN_PACK_BATCH, BCN_PACK_HW = 0, 1
BCN_SAMPLE_TERNARY, BCN_SAMPLE_UNIFORM, BCN_SAMPLE_GAUSSIAN = 0, 1, 2
BCN_PURPOSE_SECRET, BCN_PURPOSE_KSK_A, BCN_PURPOSE_KSK_E, BCN_PURPOSE_ENC_A, BCN_PURPOSE_ENC_E = 1, 2, 3, 4, 5
BCN_OK, BCN_ERR_INVALID, BCN_ERR_LEVEL, BCN_ERR_KEY, BCN_ERR_NOMEM, BCN_ERR_HIP, BCN_ERR_INTERNAL = 0, -1, -2, -3, -4, -5, -6


class BcnError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("bcn error %d: %s" % (code, msg))
        self.code = code


class Params(C.Structure):
    _fields_ = [("n", C.c_uint32), ("q_bits", C.c_uint32), ("L", C.c_uint32), ("K", C.c_uint32),
                ("alpha", C.c_uint32), ("t", C.c_uint64)]


class LayerDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("packing", C.c_int32), ("in_c", C.c_int32), ("in_h", C.c_int32),
                ("in_w", C.c_int32), ("out_c", C.c_int32), ("k", C.c_int32), ("stride", C.c_int32),
                ("pad", C.c_int32), ("row", C.c_int32), ("pos_stride", C.c_int32),
                ("weights", C.POINTER(C.c_int32)), ("has_features", C.c_int32), ("feature_scale", C.c_float),
                ("feature_clamp", C.c_int32), ("batch", C.c_int32), ("square", C.c_int32),
                ("modswitch", C.c_int32), ("sum", C.c_int32), ("block", C.c_int32),
                ("method", C.c_int32), ("defer_relin", C.c_int32), ("in_parts", C.c_int32)]


class NttItem(C.Structure):
    _fields_ = [("ctx", C.c_void_p), ("data", C.c_void_p), ("n_polys", C.c_int32), ("n_limbs", C.c_int32),
                ("first_prime", C.c_int32)]


def ntt_multi(items, inverse=False):
    """One persistent launch transforming several contexts' limbs: items of
    (context, data [n_polys][n_limbs][N] device tensor, first_prime)."""
    arr = (NttItem * len(items))()
    for i, (ctx, data, first) in enumerate(items):
        arr[i].ctx = ctx.h
        arr[i].data = data.data_ptr()
        arr[i].n_polys, arr[i].n_limbs = data.shape[0], data.shape[1]
        arr[i].first_prime = first
    _check(lib().bcn_ntt_multi(arr, len(items), 1 if inverse else 0, _stream()))


_lib = None

_VP, _I, _U64P, _I64P, _I32P, _I8P = C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p

_SIGS = {
    "bcn_last_error": (C.c_char_p, []),
    "bcn_context_create": (_I, [C.POINTER(Params), _I, C.POINTER(_VP)]),
    "bcn_context_destroy": (None, [_VP]),
    "bcn_context_primes": (_I, [_VP, _U64P, _I, C.POINTER(_I), C.POINTER(_I), C.POINTER(_I)]),
    "bcn_secret_key_create": (_I, [_VP, _I8P, C.POINTER(_VP)]),
    "bcn_secret_key_destroy": (None, [_VP]),
    "bcn_eval_keys_create": (_I, [_VP, C.POINTER(_VP)]),
    "bcn_eval_keys_destroy": (None, [_VP]),
    "bcn_keygen": (_I, [_VP, _VP, _VP, _I, _I, _U64P, _I8P, _VP]),
    "bcn_eval_key_export": (_I, [_VP, _VP, _I, _I, _U64P, _VP]),
    "bcn_encode_encrypt": (_I, [_VP, _VP, _I64P, _U64P, _I8P, _I, _I, _VP, _VP]),
    "bcn_decrypt_decode": (_I, [_VP, _VP, _VP, _I, _I, _I64P, _VP]),
    "bcn_ct_export": (_I, [_VP, _VP, _I, _I, _U64P, _VP]),
    "bcn_ct_import": (_I, [_VP, _U64P, _I, _I, _VP, _VP]),
    "bcn_ntt": (_I, [_VP, _VP, _I, _I, _I, _I, _VP]),
    "bcn_mac": (_I, [_VP, _VP, _I, _VP, _I, _I, _I32P, _VP]),
    "bcn_add_plain": (_I, [_VP, _VP, _I, _I, _I64P, _VP]),
    "bcn_mul_plain": (_I, [_VP, _VP, _VP, _I, _I, _I64P, _VP]),
    "bcn_square_relin": (_I, [_VP, _VP, _VP, _VP, _I, _I, _I, _VP]),
    "bcn_rotate": (_I, [_VP, _VP, _VP, _I, _I, _I32P, _I, _VP, _VP]),
    "bcn_rotate_sum": (_I, [_VP, _VP, _VP, _I, _I, _I, _VP]),
    "bcn_modswitch": (_I, [_VP, _VP, _VP, _I, _I, _VP]),
    "bcn_layer_create": (_I, [_VP, C.POINTER(LayerDesc), _I, C.POINTER(_VP)]),
    "bcn_layer_destroy": (None, [_VP]),
    "bcn_layer_rotation_steps": (_I, [_VP, _I32P, _I]),
    "bcn_layer_shape": (_I, [_VP, C.POINTER(_I), C.POINTER(_I), C.POINTER(_I)]),
    "bcn_layer_parts": (_I, [_VP, C.POINTER(_I), C.POINTER(_I)]),
    "bcn_layer_eval": (_I, [_VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "bcn_layer_eval_batch": (_I, [_VP, _VP, _VP, _VP, _VP, _VP, _I, _VP]),
    "bcn_profile_enable": (_I, [_VP, _I]),
    "bcn_autotune": (_I, [_VP, C.c_char_p, _I, _VP]),
    "bcn_layer_autotune": (_I, [_VP, _VP, C.c_char_p, _I, _VP]),
    "bcn_profile_read": (_I, [_VP, C.c_char_p, _I, _VP, _VP, _VP, _VP, _I]),
    "bcn_square_relin_noalloc": (_I, [_VP, _VP, _VP, _VP, _I, _I, _I, _VP]),
    "bcn_context_create_ckks": (_I, [_VP, _I, _VP]),
    "bcn_ntt_multi": (_I, [_VP, _I, _I, _VP]),
    "bcn_ckks_encode": (_I, [_VP, _VP, _I, _I, C.c_double, _I, _VP, _VP]),
    "bcn_ckks_encode_encrypt": (_I, [_VP, _VP, _VP, C.c_double, _VP, _VP, _I, _I, _VP, _VP]),
    "bcn_ckks_decrypt_decode": (_I, [_VP, _VP, _VP, _I, _I, C.c_double, _VP, _VP]),
    "bcn_ckks_add_plain": (_I, [_VP, _VP, _I, _I, _VP, _VP]),
    "bcn_ckks_mul_plain": (_I, [_VP, _VP, _VP, _I, _I, _VP, _VP]),
    "bcn_ckks_square_relin_rescale": (_I, [_VP, _VP, _VP, _VP, _I, _I, _VP]),
    "bcn_scratch_info": (_I, [_VP, _VP, _VP, _VP, _VP, _VP]),
    "bcn_scratch_release": (_I, [_VP]),
    "bcn_rotate_sum_steps": (_I, [_I, _I32P, _I]),
    "bcn_sample": (_I, [_I, C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint64, _I, _I64P]),
    "bcn_gaussian_table": (_I, [_U64P]),
    "bcn_secret_key_generate": (_I, [_VP, C.c_uint64, C.POINTER(_VP)]),
    "bcn_keygen_seeded": (_I, [_VP, _VP, _VP, _I, _I, C.c_uint64, _VP]),
    "bcn_encrypt_seeded": (_I, [_VP, _VP, _I64P, C.c_uint64, C.c_uint64, _I, _I, _VP, _VP]),
    "bcn_ckks_encrypt_seeded": (_I, [_VP, _VP, _VP, C.c_double, C.c_uint64, C.c_uint64, _I, _I, _VP, _VP]),
}


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("HIP library missing: %s (run __graft_entry__.build())" % LIB_PATH)
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


def exported_symbols():
    return list(_SIGS)


def _check(rc):
    if rc != 0:
        raise BcnError(rc, lib().bcn_last_error().decode())


def _np_ptr(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(C.c_void_p)


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t):
    return C.c_void_p(t.data_ptr())


def sample(kind, seed, purpose, index, n, q=0):
    """n samples of `kind` (BCN_SAMPLE_*) from the ChaCha20 stream (seed, purpose, index)."""
    out = np.zeros(n, dtype=np.uint64 if kind == BCN_SAMPLE_UNIFORM else np.int64)
    _check(lib().bcn_sample(kind, seed, purpose, index, q, n, out.ctypes.data_as(C.c_void_p)))
    return out


def rotate_sum_steps(span):
    """The rotation steps bcn_rotate_sum(span) needs."""
    n = lib().bcn_rotate_sum_steps(span, None, 0)
    if n < 0:
        _check(n)
    out = np.zeros(max(n, 1), dtype=np.int32)
    lib().bcn_rotate_sum_steps(span, out.ctypes.data_as(C.c_void_p), n)
    return [int(x) for x in out[:n]]


def gaussian_table():
    out = np.zeros(38, dtype=np.uint64)
    _check(lib().bcn_gaussian_table(out.ctypes.data_as(C.c_void_p)))
    return [int(x) for x in out]


class Context:
    def __init__(self, n, q_bits, L, K, alpha, t, device=0, ckks=False):
        """A BFV context, or with ckks=True a CKKS context (t ignored)."""
        self.ckks = ckks
        self.p = Params(n, q_bits, L, K, alpha, 0 if ckks else t)
        h = C.c_void_p()
        create = lib().bcn_context_create_ckks if ckks else lib().bcn_context_create
        _check(create(C.byref(self.p), device, C.byref(h)))
        self.h = h
        self.n, self.L, self.K, self.alpha, self.t = n, L, K, alpha, t
        buf = np.zeros(64, dtype=np.uint64)
        nq, np_, nb = C.c_int(), C.c_int(), C.c_int()
        _check(lib().bcn_context_primes(h, buf.ctypes.data_as(C.c_void_p), 64, C.byref(nq), C.byref(np_),
                                        C.byref(nb)))
        self.primes = [int(x) for x in buf[:nq.value + np_.value + nb.value + (0 if ckks else 1)]]
        self.n_q, self.n_p, self.n_aux = nq.value, np_.value, nb.value

    @property
    def q(self):
        return self.primes[:self.n_q]

    @property
    def p_primes(self):
        return self.primes[self.n_q:self.n_q + self.n_p]

    def dnum(self, level=None):
        level = self.L if level is None else level
        return -(-level // self.alpha)

    def close(self):
        if self.h:
            lib().bcn_context_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ tensors
    def empty_ct(self, n, level):
        import torch
        return torch.empty((n, 2, level, self.n), dtype=torch.float64, device="cuda")

    # ------------------------------------------------------------ client side
    def secret_key(self, s):
        s, p = _np_ptr(s, np.int8)
        h = C.c_void_p()
        _check(lib().bcn_secret_key_create(self.h, p, C.byref(h)))
        return SecretKey(self, h)

    def secret_key_seeded(self, seed):
        h = C.c_void_p()
        _check(lib().bcn_secret_key_generate(self.h, seed, C.byref(h)))
        return SecretKey(self, h)

    def keygen_seeded(self, sk, ek, kind, step, seed):
        _check(lib().bcn_keygen_seeded(self.h, sk.h, ek.h, kind, step, seed, _stream()))

    def encrypt_seeded(self, sk, slots, seed, first=0, level=None):
        level = self.L if level is None else level
        slots, sp = _np_ptr(slots, np.int64)
        n = slots.shape[0]
        ct = self.empty_ct(n, level)
        _check(lib().bcn_encrypt_seeded(self.h, sk.h, sp, seed, first, n, level, _dptr(ct), _stream()))
        return ct

    def ckks_encrypt_seeded(self, sk, slots, scale, seed, first=0, level=None):
        level = self.L if level is None else level
        slots, sp = _np_ptr(slots, np.float64)
        n = slots.shape[0]
        ct = self.empty_ct(n, level)
        _check(lib().bcn_ckks_encrypt_seeded(self.h, sk.h, sp, C.c_double(scale), seed, first, n, level,
                                             _dptr(ct), _stream()))
        return ct

    def eval_keys(self):
        h = C.c_void_p()
        _check(lib().bcn_eval_keys_create(self.h, C.byref(h)))
        return EvalKeys(self, h)

    def keygen(self, sk, ek, kind, step, a, e):
        a, ap = _np_ptr(a, np.uint64)
        e, ep = _np_ptr(e, np.int8)
        _check(lib().bcn_keygen(self.h, sk.h, ek.h, kind, step, ap, ep, _stream()))

    def export_key(self, ek, kind, step=0):
        out = np.zeros((self.dnum(), 2, self.L + self.K, self.n), dtype=np.uint64)
        _check(lib().bcn_eval_key_export(self.h, ek.h, kind, step, out.ctypes.data_as(C.c_void_p), _stream()))
        return out

    def encrypt(self, sk, slots, a, e, level=None):
        level = self.L if level is None else level
        slots, sp = _np_ptr(slots, np.int64)
        a, ap = _np_ptr(a, np.uint64)
        e, ep = _np_ptr(e, np.int8)
        n = slots.shape[0]
        ct = self.empty_ct(n, level)
        _check(lib().bcn_encode_encrypt(self.h, sk.h, sp, ap, ep, n, level, _dptr(ct), _stream()))
        return ct

    def decrypt(self, sk, ct):
        n, _, level, _ = ct.shape
        out = np.zeros((n, self.n), dtype=np.int64)
        _check(lib().bcn_decrypt_decode(self.h, sk.h, _dptr(ct), n, level, out.ctypes.data_as(C.c_void_p),
                                        _stream()))
        return out

    def export(self, ct):
        n, _, level, _ = ct.shape
        out = np.zeros((n, 2, level, self.n), dtype=np.uint64)
        _check(lib().bcn_ct_export(self.h, _dptr(ct), n, level, out.ctypes.data_as(C.c_void_p), _stream()))
        return out

    def import_(self, arr):
        arr = np.ascontiguousarray(arr, dtype=np.uint64)
        n, _, level, _ = arr.shape
        ct = self.empty_ct(n, level)
        _check(lib().bcn_ct_import(self.h, arr.ctypes.data_as(C.c_void_p), n, level, _dptr(ct), _stream()))
        return ct

    # ------------------------------------------------------------ server side
    def ntt(self, data, first_prime, inverse=False):
        n_polys, n_limbs, _ = data.shape
        _check(lib().bcn_ntt(self.h, _dptr(data), n_polys, n_limbs, first_prime, 1 if inverse else 0, _stream()))

    def mac(self, ct, w):
        n_in, _, level, _ = ct.shape
        w, wp = _np_ptr(w, np.int32)
        out = self.empty_ct(w.shape[0], level)
        _check(lib().bcn_mac(self.h, _dptr(ct), n_in, _dptr(out), w.shape[0], level, wp, _stream()))
        return out

    def add_plain(self, ct, slots):
        n, _, level, _ = ct.shape
        slots, sp = _np_ptr(slots, np.int64)
        _check(lib().bcn_add_plain(self.h, _dptr(ct), n, level, sp, _stream()))

    def mul_plain(self, ct, slots):
        n, _, level, _ = ct.shape
        slots, sp = _np_ptr(slots, np.int64)
        out = self.empty_ct(n, level)
        _check(lib().bcn_mul_plain(self.h, _dptr(ct), _dptr(out), n, level, sp, _stream()))
        return out

    def square_relin(self, ek, ct, modswitch=False):
        n, _, level, _ = ct.shape
        out = self.empty_ct(n, level - 1 if modswitch else level)
        _check(lib().bcn_square_relin(self.h, ek.h, _dptr(ct), _dptr(out), n, level, 1 if modswitch else 0,
                                      _stream()))
        return out

    def square_relin_noalloc(self, ek, ct, out, modswitch=False):
        """The allocation-free square + relinearisation into caller-provided `out`."""
        n, _, level, _ = ct.shape
        _check(lib().bcn_square_relin_noalloc(self.h, ek.h, _dptr(ct), _dptr(out), n, level,
                                              1 if modswitch else 0, _stream()))
        return out

    def rotate(self, ek, ct, steps):
        n, _, level, _ = ct.shape
        steps, sp = _np_ptr(steps, np.int32)
        import torch
        out = torch.empty((n, len(steps), 2, level, self.n), dtype=torch.float64, device="cuda")
        _check(lib().bcn_rotate(self.h, ek.h, _dptr(ct), n, level, sp, len(steps), _dptr(out), _stream()))
        return out

    def rotate_sum(self, ek, ct, span):
        n, _, level, _ = ct.shape
        _check(lib().bcn_rotate_sum(self.h, ek.h, _dptr(ct), n, level, span, _stream()))

    def modswitch(self, ct):
        n, _, level, _ = ct.shape
        out = self.empty_ct(n, level - 1)
        _check(lib().bcn_modswitch(self.h, _dptr(ct), _dptr(out), n, level, _stream()))
        return out

    def layer(self, desc: dict, level: int):
        return Layer(self, desc, level)

    def autotune(self):
        buf = C.create_string_buffer(4096)
        _check(lib().bcn_autotune(self.h, buf, 4096, _stream()))
        return buf.value.decode()

    def autotune_layer(self, layer):
        buf = C.create_string_buffer(4096)
        _check(lib().bcn_layer_autotune(self.h, layer.h, buf, 4096, _stream()))
        return buf.value.decode()

    # ------------------------------------------------------------ measurement
    def profile(self, on: bool):
        _check(lib().bcn_profile_enable(self.h, 1 if on else 0))

    def profile_read(self):
        """{kernel: (launches, total_ms, algorithmic_bytes, algorithmic_fp64_ops)} since the last read."""
        cap = 64
        names = C.create_string_buffer(4096)
        la = np.zeros(cap, dtype=np.int32)
        ms = np.zeros(cap, dtype=np.float64)
        by = np.zeros(cap, dtype=np.float64)
        op = np.zeros(cap, dtype=np.float64)
        cnt = lib().bcn_profile_read(self.h, names, 4096, la.ctypes.data_as(C.c_void_p),
                                     ms.ctypes.data_as(C.c_void_p), by.ctypes.data_as(C.c_void_p),
                                     op.ctypes.data_as(C.c_void_p), cap)
        if cnt < 0:
            _check(cnt)
        keys = names.value.decode().split("\n")[:cnt]
        return {k: (int(la[i]), float(ms[i]), float(by[i]), float(op[i])) for i, k in enumerate(keys)}


    # ------------------------------------------------------------ CKKS
    def ckks_encrypt(self, sk, slots, scale, a, e, level=None):
        """Encode host slots [n][N/2] at `scale` and encrypt: device [n][2][level][N]."""
        level = self.L if level is None else level
        slots, sp = _np_ptr(slots, np.float64)
        a, ap = _np_ptr(a, np.uint64)
        e, ep = _np_ptr(e, np.int8)
        n = slots.shape[0]
        ct = self.empty_ct(n, level)
        _check(lib().bcn_ckks_encode_encrypt(self.h, sk.h, sp, C.c_double(scale), ap, ep, n, level, _dptr(ct),
                                             _stream()))
        return ct

    def ckks_decrypt(self, sk, ct, scale):
        """Decrypted, decoded slots (real parts), host [n][N/2]."""
        n, _, level, _ = ct.shape
        out = np.zeros((n, self.n // 2), dtype=np.float64)
        _check(lib().bcn_ckks_decrypt_decode(self.h, sk.h, _dptr(ct), n, level, C.c_double(scale),
                                             out.ctypes.data_as(C.c_void_p), _stream()))
        return out

    def ckks_encode(self, slots, level, scale, ntt=False):
        """Device slots [n][N/2] (float64) -> device residues [n][level][N]."""
        import torch
        slots = slots.contiguous()
        n = slots.shape[0]
        out = torch.empty((n, level, self.n), dtype=torch.float64, device="cuda")
        _check(lib().bcn_ckks_encode(self.h, _dptr(slots), n, level, C.c_double(scale), 1 if ntt else 0, _dptr(out),
                                     _stream()))
        return out

    def ckks_add_plain(self, ct, pt):
        n, _, level, _ = ct.shape
        _check(lib().bcn_ckks_add_plain(self.h, _dptr(ct), n, level, _dptr(pt), _stream()))

    def ckks_mul_plain(self, ct, pt_ntt):
        n, _, level, _ = ct.shape
        out = self.empty_ct(n, level)
        _check(lib().bcn_ckks_mul_plain(self.h, _dptr(ct), _dptr(out), n, level, _dptr(pt_ntt), _stream()))
        return out

    def ckks_square_relin_rescale(self, ek, ct):
        n, _, level, _ = ct.shape
        out = self.empty_ct(n, level - 1)
        _check(lib().bcn_ckks_square_relin_rescale(self.h, ek.h, _dptr(ct), _dptr(out), n, level, _stream()))
        return out

    # ------------------------------------------------------------ scratch arena
    def scratch_info(self):
        """{base, generation, bytes, high_bytes, retired_bytes} of the context's scratch arena."""
        base, gen = C.c_uint64(), C.c_uint64()
        by, hi, ret = C.c_size_t(), C.c_size_t(), C.c_size_t()
        _check(lib().bcn_scratch_info(self.h, C.byref(base), C.byref(gen), C.byref(by), C.byref(hi), C.byref(ret)))
        return {"base": base.value, "generation": gen.value, "bytes": by.value, "high_bytes": hi.value,
                "retired_bytes": ret.value}

    def scratch_release(self):
        _check(lib().bcn_scratch_release(self.h))


class SecretKey:
    def __init__(self, ctx, h):
        self.ctx, self.h = ctx, h

    def __del__(self):
        try:
            if self.h:
                lib().bcn_secret_key_destroy(self.h)
                self.h = None
        except Exception:
            pass


class EvalKeys:
    def __init__(self, ctx, h):
        self.ctx, self.h = ctx, h

    def __del__(self):
        try:
            if self.h:
                lib().bcn_eval_keys_destroy(self.h)
                self.h = None
        except Exception:
            pass


class Layer:
    """A prepared layer (weights uploaded, masks and weight vectors encoded)."""

    def __init__(self, ctx, desc: dict, level: int):
        self.ctx = ctx
        w = np.ascontiguousarray(desc["weights"] if desc.get("weights") is not None else np.zeros(1),
                                 dtype=np.int32)
        self._w = w
        d = LayerDesc()
        d.kind = desc["kind"]
        d.packing = desc["packing"]
        d.in_c, d.in_h, d.in_w = desc["in_c"], desc.get("in_h", 1), desc.get("in_w", 1)
        d.out_c = desc["out_c"]
        d.k, d.stride, d.pad = desc.get("k", 1), desc.get("stride", 1), desc.get("pad", 0)
        d.row, d.pos_stride = desc.get("row", 1), desc.get("pos_stride", 1)
        d.weights = w.ctypes.data_as(C.POINTER(C.c_int32))
        d.has_features = 1 if desc.get("features") else 0
        d.feature_scale = desc.get("feature_scale", 8.0)
        d.feature_clamp = desc.get("feature_clamp", 127)
        d.batch = desc.get("batch", 0)
        d.square = 1 if desc.get("square") else 0
        d.modswitch = 1 if desc.get("modswitch") else 0
        d.sum = int(desc.get("sum") or 0)
        d.block = int(desc.get("block") or 0)
        d.method = int(desc.get("method") or 0)
        d.defer_relin = 1 if desc.get("defer_relin") else 0
        d.in_parts = int(desc.get("in_parts") or 2)
        self.desc = d
        h = C.c_void_p()
        _check(lib().bcn_layer_create(ctx.h, C.byref(d), level, C.byref(h)))
        self.h = h
        buf = np.zeros(256, dtype=np.int32)
        cnt = lib().bcn_layer_rotation_steps(h, buf.ctypes.data_as(C.c_void_p), 256)
        if cnt < 0:
            _check(cnt)
        self.steps = [int(x) for x in buf[:cnt]]
        ni, no, lo = C.c_int(), C.c_int(), C.c_int()
        _check(lib().bcn_layer_shape(h, C.byref(ni), C.byref(no), C.byref(lo)))
        self.n_in, self.n_out, self.level_out = ni.value, no.value, lo.value
        pi, po = C.c_int(), C.c_int()
        _check(lib().bcn_layer_parts(h, C.byref(pi), C.byref(po)))
        self.in_parts, self.out_parts = pi.value, po.value
        self.level = level

    def _empty_out(self, rows):
        import torch
        return torch.empty((rows, self.out_parts, self.level_out, self.ctx.n), dtype=torch.float64, device="cuda")

    def __call__(self, ek, ct, features=None, out=None):
        if out is None:
            out = self._empty_out(self.n_out)
        fp = _dptr(features) if features is not None else None
        _check(lib().bcn_layer_eval(self.ctx.h, ek.h, self.h, _dptr(ct), _dptr(out), fp, _stream()))
        return out

    def batch(self, ek, ct, n_requests, features=None, out=None):
        """R requests at once: ct [R*n_in][in_parts][level][N] -> [R*n_out][out_parts][level_out][N]."""
        if out is None:
            out = self._empty_out(n_requests * self.n_out)
        fp = _dptr(features) if features is not None else None
        _check(lib().bcn_layer_eval_batch(self.ctx.h, ek.h, self.h, _dptr(ct), _dptr(out), fp, n_requests,
                                          _stream()))
        return out

    def __del__(self):
        try:
            if self.h:
                lib().bcn_layer_destroy(self.h)
                self.h = None
        except Exception:
            pass
