"""LocPIR gate bootstrapping on MI355X (gfx950): Python binding of liblocpir.

Argument marshalling only: every step of the path runs in the native library
(include/locpir.h).  Device buffers are torch tensors on a ROCm device
(uint32 stored as int32, since torch has no uint32 arithmetic we rely on);
streams are torch streams.  The library is built by ``_build.py``; if it is
missing, every call raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
import struct

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# LOCPIR_LIB names another build of the same library (e.g. an address- and
# undefined-behaviour-sanitizer build of the host code for CPU tests)
_LIB_PATH = os.environ.get("LOCPIR_LIB") or os.path.join(_HERE, "liblocpir.so")
_LIB = None

GATES = {"NAND": 0, "AND": 1, "OR": 2, "XOR": 3, "XNOR": 4, "NOR": 5, "MUX": 6, "NOT": 7, "COPY": 8}


class LocpirError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"locpir error {code}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("n", C.c_uint32), ("N", C.c_uint32), ("k", C.c_uint32), ("bg_bit", C.c_uint32),
                ("l", C.c_uint32), ("ks_base_bit", C.c_uint32), ("ks_t", C.c_uint32),
                ("lwe_sigma", C.c_double), ("bk_sigma", C.c_double)]

    def __repr__(self):
        return (f"Params(n={self.n}, N={self.N}, k={self.k}, bg_bit={self.bg_bit}, l={self.l}, "
                f"ks_base_bit={self.ks_base_bit}, ks_t={self.ks_t}, lwe_sigma={self.lwe_sigma}, "
                f"bk_sigma={self.bk_sigma})")


class KernelStat(C.Structure):
    _fields_ = [("name", C.c_char_p), ("launches", C.c_uint64), ("jobs", C.c_uint64), ("total_ms", C.c_double)]


class LaunchRecord(C.Structure):
    _fields_ = [("name", C.c_char_p), ("jobs", C.c_uint64), ("shape", C.c_int32), ("ms", C.c_double)]


class TuneEntry(C.Structure):
    _fields_ = [("jobs", C.c_uint32), ("br_waves", C.c_int32), ("ks_tile", C.c_int32), ("ks_split", C.c_int32),
                ("br_us", C.c_float), ("ks_us", C.c_float)]

    def as_dict(self) -> dict:
        return {"jobs": int(self.jobs), "br_waves": int(self.br_waves), "ks_tile": int(self.ks_tile),
                "ks_split": int(self.ks_split), "br_us": round(float(self.br_us), 3),
                "ks_us": round(float(self.ks_us), 3)}


TUNE_MAX_ROWS = 32
DEFAULT_TUNE_BUCKETS = (1, 16, 64, 128, 256, 384, 512, 768, 1024, 2048, 4096, 16384)


TICK_CAP_AUTO = 0xFFFFFFFF  # LP_TICK_CAP_AUTO


class ServerConfig(C.Structure):
    _fields_ = [("hbm_budget", C.c_size_t), ("max_inflight", C.c_uint32), ("simulate", C.c_int32),
                ("fail_ticket", C.c_uint64), ("max_tick_rotations", C.c_uint32)]


class HostQuery(C.Structure):
    _fields_ = [("l", C.c_uint32), ("n_boxes", C.c_uint32), ("m", C.c_uint32), ("is_signed", C.c_int32),
                ("x", C.c_void_p), ("y", C.c_void_p), ("bounds", C.c_void_p), ("payload", C.c_void_p)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("admitted", C.c_uint64), ("completed", C.c_uint64),
                ("failed", C.c_uint64), ("cancelled", C.c_uint64), ("ticks", C.c_uint64),
                ("fused_bootstraps", C.c_uint64), ("pending", C.c_uint32), ("active", C.c_uint32),
                ("bytes_in_use", C.c_size_t), ("peak_bytes", C.c_size_t), ("widest_tick", C.c_uint64)]


class BBoxQuery(C.Structure):
    _fields_ = [("l", C.c_uint32), ("n_boxes", C.c_uint32), ("m", C.c_uint32), ("is_signed", C.c_int32),
                ("d_x", C.c_void_p), ("d_y", C.c_void_p), ("d_bounds", C.c_void_p), ("d_payload", C.c_void_p)]


def lib() -> C.CDLL:
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(_LIB_PATH):
        raise LocpirError(-100, f"{_LIB_PATH} is not built (run __graft_entry__.build())")
    # torch ships its own HIP runtime with the same soname; loading torch
    # first makes liblocpir bind to that one runtime instead of a second copy
    # (a sanitizer build runs host-only tests and skips it)
    if not os.environ.get("LOCPIR_NO_TORCH"):
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
    L = C.CDLL(_LIB_PATH)
    vp, sz, u32, u64, i32 = C.c_void_p, C.c_size_t, C.c_uint32, C.c_uint64, C.c_int32
    PP = C.POINTER(Params)
    sig = {
        "lp_last_error": (C.c_char_p, []),
        "lp_version": (C.c_char_p, []),
        "lp_params_default": (i32, [PP]),
        "lp_params_lambda80": (i32, [PP]),
        "lp_keygen": (i32, [PP, u64, C.POINTER(vp), C.POINTER(vp)]),
        "lp_secret_key_import": (i32, [PP, vp, vp, C.POINTER(vp)]),
        "lp_secret_key_export": (i32, [vp, vp, vp]),
        "lp_cloud_key_import": (i32, [PP, vp, vp, C.POINTER(vp)]),
        "lp_cloud_key_export": (i32, [vp, vp, vp]),
        "lp_cloud_key_params": (i32, [vp, PP]),
        "lp_cloud_key_serialize": (i32, [vp, vp, C.POINTER(sz)]),
        "lp_cloud_key_deserialize": (i32, [vp, sz, C.POINTER(vp)]),
        "lp_bsk_words": (sz, [PP]),
        "lp_ksk_words": (sz, [PP]),
        "lp_encrypt_bits": (i32, [vp, vp, sz, u64, u64, vp]),
        "lp_encrypt_zeros": (i32, [vp, sz, u64, u64, vp]),
        "lp_preprocess": (i32, [vp, vp, vp, sz, vp, vp]),
        "lp_bbox_wire_bytes": (i32, [vp, u32, u32, u32, vp]),
        "lp_decrypt_bits": (i32, [vp, vp, sz, vp, vp]),
        "lp_device_key_create": (i32, [vp, vp, C.POINTER(vp)]),
        "lp_device_key_bytes": (i32, [vp, C.POINTER(sz)]),
        "lp_bootstrap_batch": (i32, [vp, i32, vp, vp, vp, sz, vp, vp]),
        "lp_bootstrap_batch_noks": (i32, [vp, i32, vp, vp, vp, sz, vp, vp]),
        "lp_bootstrap_batch_noalloc": (i32, [vp, i32, vp, vp, vp, sz, vp, vp]),
        "lp_debug_field_op_rates": (i32, [C.c_double, vp, vp, vp]),
        "lp_debug_external_product_mfma": (i32, [vp, vp, sz, vp, vp]),
        "lp_debug_split_profile": (i32, [vp, vp, sz, i32, vp, vp, vp]),
        "lp_keyswitch_batch": (i32, [vp, vp, sz, vp, vp]),
        "lp_eval_bbox_query": (i32, [vp, C.POINTER(BBoxQuery), vp, vp]),
        "lp_eval_bbox_batch": (i32, [C.POINTER(vp), C.POINTER(BBoxQuery), sz, C.POINTER(vp), vp]),
        "lp_eval_bbox_prepare": (i32, [C.POINTER(vp), C.POINTER(BBoxQuery), sz, vp]),
        "lp_bbox_counts": (i32, [u32, u32, u32, C.POINTER(u64), C.POINTER(u64), C.POINTER(u32)]),
        "lp_bbox_level_widths": (i32, [u32, u32, u32, C.POINTER(u32), C.POINTER(u32)]),
        "lp_debug_negacyclic_mul": (i32, [vp, vp, sz, vp, vp]),
        "lp_debug_blind_rotate": (i32, [vp, vp, sz, u32, vp, vp]),
        "lp_profile_enable": (i32, [i32]),
        "lp_profile_collect": (i32, [C.POINTER(KernelStat), C.POINTER(C.c_int)]),
        "lp_profile_collect_launches": (i32, [C.POINTER(LaunchRecord), C.POINTER(C.c_int)]),
        "lp_split_stall_count": (i32, [C.POINTER(u32)]),
        "lp_autotune": (i32, [vp, C.POINTER(u32), C.c_int, u32, vp, C.POINTER(TuneEntry)]),
        "lp_tune_set": (i32, [C.POINTER(TuneEntry), C.c_int]),
        "lp_tune_get": (i32, [C.POINTER(TuneEntry), C.POINTER(C.c_int)]),
        "lp_tune_pick": (i32, [u32, u32, C.POINTER(TuneEntry)]),
        "lp_server_create": (i32, [C.POINTER(ServerConfig), C.POINTER(vp)]),
        "lp_server_request_bytes": (i32, [vp, C.POINTER(HostQuery), C.POINTER(sz)]),
        "lp_server_submit": (i32, [vp, vp, C.POINTER(HostQuery), C.POINTER(u64)]),
        "lp_server_submit_blob": (i32, [vp, vp, sz, C.POINTER(HostQuery), C.POINTER(u64)]),
        "lp_server_poll": (i32, [vp, u64, i32, vp, C.POINTER(C.c_double)]),
        "lp_server_cancel": (i32, [vp, u64]),
        "lp_server_stats_get": (i32, [vp, C.POINTER(ServerStats)]),
        "lp_server_free": (None, [vp]),
        "lp_secret_key_free": (None, [vp]),
        "lp_cloud_key_free": (None, [vp]),
        "lp_device_key_free": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _LIB = L
    return L


def _check(code: int):
    if code != 0:
        raise LocpirError(code, lib().lp_last_error().decode(errors="replace"))


def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# ------------------------------------------------------------------ params
def params_default() -> Params:
    p = Params()
    _check(lib().lp_params_default(C.byref(p)))
    return p


def params_lambda80() -> Params:
    """The paper's lambda 80 set (Sec. 5: n = 540, sigma = 2^-20.2); the
    ring, gadget and key-switching parameters are those of the default set."""
    p = Params()
    _check(lib().lp_params_lambda80(C.byref(p)))
    return p


def bsk_words(p: Params) -> int:
    return int(lib().lp_bsk_words(C.byref(p)))


def ksk_words(p: Params) -> int:
    return int(lib().lp_ksk_words(C.byref(p)))


# ------------------------------------------------------------------ keys
class SecretKey:
    def __init__(self, handle, params: Params):
        self._h = handle
        self.params = params

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h and _LIB is not None:
            try:
                _LIB.lp_secret_key_free(h)
            except Exception:  # interpreter shutdown
                pass

    @classmethod
    def from_arrays(cls, params: Params, s, S):
        s = np.ascontiguousarray(s, np.uint8)
        S = np.ascontiguousarray(S, np.uint8)
        h = C.c_void_p()
        _check(lib().lp_secret_key_import(C.byref(params), _np_ptr(s), _np_ptr(S), C.byref(h)))
        return cls(h, params)

    def export(self):
        s = np.zeros(self.params.n, np.uint8)
        S = np.zeros(self.params.N, np.uint8)
        _check(lib().lp_secret_key_export(self._h, _np_ptr(s), _np_ptr(S)))
        return s, S

    def encrypt_bits(self, bits, seed: int, first_index: int = 0) -> np.ndarray:
        bits = np.ascontiguousarray(np.asarray(bits, np.uint8).reshape(-1))
        ct = np.zeros((len(bits), self.params.n + 1), np.uint32)
        _check(lib().lp_encrypt_bits(self._h, _np_ptr(bits), len(bits), seed, first_index, _np_ptr(ct)))
        return ct

    def encrypt_zeros(self, cnt: int, seed: int, first_index: int = 0) -> np.ndarray:
        """The client's fresh samples of zero for Preprocess (Sec. 3)."""
        ct = np.zeros((cnt, self.params.n + 1), np.uint32)
        _check(lib().lp_encrypt_zeros(self._h, cnt, seed, first_index, _np_ptr(ct)))
        return ct

    def decrypt_bits(self, ct):
        ct = np.ascontiguousarray(np.asarray(ct).view(np.uint32) if np.asarray(ct).dtype == np.int32
                                  else np.asarray(ct, np.uint32)).reshape(-1, self.params.n + 1)
        bits = np.zeros(len(ct), np.uint8)
        ph = np.zeros(len(ct), np.int32)
        _check(lib().lp_decrypt_bits(self._h, _np_ptr(ct), len(ct), _np_ptr(bits), _np_ptr(ph)))
        return bits, ph


class CloudKey:
    def __init__(self, handle, params: Params):
        self._h = handle
        self.params = params

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h and _LIB is not None:
            try:
                _LIB.lp_cloud_key_free(h)
            except Exception:  # interpreter shutdown
                pass

    @classmethod
    def from_arrays(cls, params: Params, bsk, ksk):
        bsk = np.ascontiguousarray(bsk, np.uint32)
        ksk = np.ascontiguousarray(ksk, np.uint32)
        if bsk.size != bsk_words(params) or ksk.size != ksk_words(params):
            raise LocpirError(-1, "key array sizes do not match the parameters")
        h = C.c_void_p()
        _check(lib().lp_cloud_key_import(C.byref(params), _np_ptr(bsk), _np_ptr(ksk), C.byref(h)))
        return cls(h, params)

    def export(self):
        bsk = np.zeros(bsk_words(self.params), np.uint32)
        ksk = np.zeros(ksk_words(self.params), np.uint32)
        _check(lib().lp_cloud_key_export(self._h, _np_ptr(bsk), _np_ptr(ksk)))
        return bsk, ksk

    def serialize(self) -> bytes:
        """PK as the client uploads it (lp_cloud_key_serialize)."""
        n = C.c_size_t()
        _check(lib().lp_cloud_key_serialize(self._h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(lib().lp_cloud_key_serialize(self._h, buf, C.byref(n)))
        return buf.raw[:n.value]

    @classmethod
    def deserialize(cls, blob: bytes) -> "CloudKey":
        h = C.c_void_p()
        _check(lib().lp_cloud_key_deserialize(blob, len(blob), C.byref(h)))
        p = Params()
        _check(lib().lp_cloud_key_params(h, C.byref(p)))
        return cls(h, p)


def keygen(params: Params | None, seed: int):
    params = params or params_default()
    sk, ck = C.c_void_p(), C.c_void_p()
    _check(lib().lp_keygen(C.byref(params), seed, C.byref(sk), C.byref(ck)))
    return SecretKey(sk, params), CloudKey(ck, params)


def bbox_counts(l: int, n_boxes: int, m: int):
    br, ks, lv = C.c_uint64(), C.c_uint64(), C.c_uint32()
    _check(lib().lp_bbox_counts(l, n_boxes, m, C.byref(br), C.byref(ks), C.byref(lv)))
    return int(br.value), int(ks.value), int(lv.value)


def bbox_level_widths(l: int, n_boxes: int, m: int) -> list:
    """Blind rotations per depth level as the library schedules the circuit."""
    n = C.c_uint32(0)
    _check(lib().lp_bbox_level_widths(l, n_boxes, m, None, C.byref(n)))
    arr = (C.c_uint32 * max(1, n.value))()
    _check(lib().lp_bbox_level_widths(l, n_boxes, m, arr, C.byref(n)))
    return [int(arr[k]) for k in range(n.value)]


# ------------------------------------------------------------------ device side
def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev_ptr(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise LocpirError(-1, "device buffers must be contiguous GPU tensors")
    return C.c_void_p(t.data_ptr())


def to_device(arr, device="cuda"):
    """Host uint32 array -> int32 GPU tensor holding the same bits."""
    torch = _torch()
    a = np.ascontiguousarray(np.asarray(arr, np.uint32)).view(np.int32)
    return torch.from_numpy(a.copy()).to(device)


def to_host(t) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint32)


class DeviceKey:
    """PK resident on the current GPU (BSK in the NTT domain + KSK)."""

    def __init__(self, cloud_key: CloudKey, stream=None):
        self.params = cloud_key.params
        h = C.c_void_p()
        _check(lib().lp_device_key_create(cloud_key._h, _stream_ptr(stream), C.byref(h)))
        self._h = h

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h and _LIB is not None:
            try:
                _LIB.lp_device_key_free(h)
            except Exception:  # interpreter shutdown
                pass

    @property
    def bytes(self) -> int:
        b = C.c_size_t()
        _check(lib().lp_device_key_bytes(self._h, C.byref(b)))
        return int(b.value)


def bootstrap_batch(dk: DeviceKey, gate: str, in0, in1=None, in2=None, out=None, stream=None):
    torch = _torch()
    cnt = in0.shape[0]
    if out is None:
        out = torch.empty((cnt, dk.params.n + 1), dtype=torch.int32, device=in0.device)
    _check(lib().lp_bootstrap_batch(dk._h, GATES[gate], _dev_ptr(in0), _dev_ptr(in1), _dev_ptr(in2), cnt,
                                    _dev_ptr(out), _stream_ptr(stream)))
    return out


def bootstrap_batch_noalloc(dk: DeviceKey, gate: str, in0, in1=None, in2=None, out=None, stream=None):
    """bootstrap_batch with every working buffer in the library's static
    device scratch (at most 1024 gates per call; calls overlapping on one GPU
    race).  `out` may be preallocated so the call allocates nothing."""
    torch = _torch()
    cnt = in0.shape[0]
    if out is None:
        out = torch.empty((cnt, dk.params.n + 1), dtype=torch.int32, device=in0.device)
    _check(lib().lp_bootstrap_batch_noalloc(dk._h, GATES[gate], _dev_ptr(in0), _dev_ptr(in1), _dev_ptr(in2), cnt,
                                            _dev_ptr(out), _stream_ptr(stream)))
    return out


def bootstrap_batch_noks(dk: DeviceKey, gate: str, in0, in1=None, in2=None, out=None, stream=None):
    """The gates of bootstrap_batch up to their key switch: [cnt][N+1]."""
    torch = _torch()
    cnt = in0.shape[0]
    if out is None:
        out = torch.empty((cnt, dk.params.N + 1), dtype=torch.int32, device=in0.device)
    _check(lib().lp_bootstrap_batch_noks(dk._h, GATES[gate], _dev_ptr(in0), _dev_ptr(in1), _dev_ptr(in2), cnt,
                                         _dev_ptr(out), _stream_ptr(stream)))
    return out


def keyswitch_batch(dk: DeviceKey, big, out=None, stream=None):
    torch = _torch()
    cnt = big.shape[0]
    if out is None:
        out = torch.empty((cnt, dk.params.n + 1), dtype=torch.int32, device=big.device)
    _check(lib().lp_keyswitch_batch(dk._h, _dev_ptr(big), cnt, _dev_ptr(out), _stream_ptr(stream)))
    return out


def preprocess(dk: DeviceKey, zero, bits, out=None, stream=None):
    """Algorithm 1 on the device: zero [cnt][n+1] int32 samples of zero, bits
    a uint8 device tensor of cnt bytes."""
    torch = _torch()
    cnt = zero.shape[0]
    if bits.dtype != torch.uint8 or bits.numel() != cnt:
        raise LocpirError(-1, "preprocess: bits must be a uint8 tensor with one byte per sample")
    if out is None:
        out = torch.empty_like(zero)
    _check(lib().lp_preprocess(dk._h, _dev_ptr(zero), _dev_ptr(bits), cnt, _dev_ptr(out), _stream_ptr(stream)))
    return out


class WireBytes(C.Structure):
    _fields_ = [("lwe_sample", C.c_size_t), ("public_key", C.c_size_t), ("service_samples", C.c_size_t),
                ("coordinate", C.c_size_t), ("query", C.c_size_t), ("result", C.c_size_t)]


def bbox_wire_bytes(params: Params, l: int, n_boxes: int, m: int) -> dict:
    w = WireBytes()
    _check(lib().lp_bbox_wire_bytes(C.byref(params), l, n_boxes, m, C.byref(w)))
    return {k: int(getattr(w, k)) for k, _ in WireBytes._fields_}


def eval_bbox_query(dk: DeviceKey, l, n_boxes, m, is_signed, x, y, bounds, payload, out=None, stream=None):
    torch = _torch()
    if out is None:
        out = torch.empty((m, dk.params.n + 1), dtype=torch.int32, device=x.device)
    q = BBoxQuery(l, n_boxes, m, int(bool(is_signed)), _dev_ptr(x), _dev_ptr(y), _dev_ptr(bounds),
                  _dev_ptr(payload))
    _check(lib().lp_eval_bbox_query(dk._h, C.byref(q), _dev_ptr(out), _stream_ptr(stream)))
    return out


def eval_bbox_batch(keys, queries, outs=None, stream=None):
    """queries: sequence of (l, n_boxes, m, is_signed, x, y, bounds, payload)
    with device tensors; keys: one DeviceKey per query.  Returns the outputs."""
    torch = _torch()
    nq = len(queries)
    if len(keys) != nq:
        raise LocpirError(-1, "one key per query")
    if outs is None:
        outs = [torch.empty((q[2], k.params.n + 1), dtype=torch.int32, device=q[4].device)
                for k, q in zip(keys, queries)]
    qarr = (BBoxQuery * nq)(*[BBoxQuery(q[0], q[1], q[2], int(bool(q[3])), _dev_ptr(q[4]), _dev_ptr(q[5]),
                                        _dev_ptr(q[6]), _dev_ptr(q[7])) for q in queries])
    karr = (C.c_void_p * nq)(*[k._h for k in keys])
    oarr = (C.c_void_p * nq)(*[_dev_ptr(o) for o in outs])
    _check(lib().lp_eval_bbox_batch(karr, qarr, nq, oarr, _stream_ptr(stream)))
    return outs


def eval_bbox_prepare(keys, queries, stream=None):
    """Compiles and caches the program eval_bbox_batch would run for these
    keys and query shapes (graphs captured), launching nothing."""
    nq = len(queries)
    if len(keys) != nq:
        raise LocpirError(-1, "one key per query")
    qarr = (BBoxQuery * nq)(*[BBoxQuery(q[0], q[1], q[2], int(bool(q[3])), _dev_ptr(q[4]), _dev_ptr(q[5]),
                                        _dev_ptr(q[6]), _dev_ptr(q[7])) for q in queries])
    karr = (C.c_void_p * nq)(*[k._h for k in keys])
    _check(lib().lp_eval_bbox_prepare(karr, qarr, nq, _stream_ptr(stream)))


def debug_negacyclic_mul(digits, poly, out=None, stream=None):
    torch = _torch()
    cnt = digits.shape[0]
    if out is None:
        out = torch.empty((cnt, 1024), dtype=torch.int32, device=digits.device)
    _check(lib().lp_debug_negacyclic_mul(_dev_ptr(digits), _dev_ptr(poly), cnt, _dev_ptr(out),
                                         _stream_ptr(stream)))
    return out


def debug_external_product_mfma(key_step, d, out=None, stream=None):
    """ExtProd of one blind-rotation step on the int8 matrix cores: key_step
    [2l][2][N] (device, Torus32), d [cnt][2N] TRLWE inputs (device)."""
    torch = _torch()
    cnt = d.shape[0]
    if out is None:
        out = torch.empty((cnt, 2048), dtype=torch.int32, device=d.device)
    _check(lib().lp_debug_external_product_mfma(_dev_ptr(key_step), _dev_ptr(d), cnt, _dev_ptr(out),
                                                _stream_ptr(stream)))
    return out


SPLIT_PHASES = ("digits", "barrier_a", "forward", "barrier_f", "partner_products", "drain_flag", "wait_partner",
                "fetch_own_sum", "inverse_1", "barrier_inv", "inverse_2", "barrier_c")


def debug_split_profile(dk: DeviceKey, ct, waves: int = 6, stream=None) -> dict:
    """Clock cycles per executed step of each phase, per wave index of a
    split workgroup (lp_debug_split_profile), and the launch time."""
    cyc = (C.c_double * (4 * len(SPLIT_PHASES)))()
    ms = C.c_double()
    _check(lib().lp_debug_split_profile(dk._h, _dev_ptr(ct), ct.shape[0], waves, cyc, C.byref(ms),
                                        _stream_ptr(stream)))
    return {"ms": float(ms.value),
            "waves": [{k: round(cyc[w * len(SPLIT_PHASES) + i], 1) for i, k in enumerate(SPLIT_PHASES)}
                      for w in range(4)]}


def debug_blind_rotate(dk: DeviceKey, ct, steps: int, out=None, stream=None):
    torch = _torch()
    cnt = ct.shape[0]
    if out is None:
        out = torch.empty((cnt, 2 * dk.params.N), dtype=torch.int32, device=ct.device)
    _check(lib().lp_debug_blind_rotate(dk._h, _dev_ptr(ct), cnt, steps, _dev_ptr(out), _stream_ptr(stream)))
    return out


FIELD_OPS = ("fwd_butterfly", "inv_butterfly", "digit_butterfly", "mulmod", "mulsum", "add", "u32_add")


def field_op_rates(target_ms: float = 4.0, stream=None) -> dict:
    """Measured throughput (operations per second, whole device) of the field
    operations the blind rotation is built from, each alone at full
    occupancy; see lp_debug_field_op_rates."""
    rates = (C.c_double * len(FIELD_OPS))()
    ms = (C.c_double * len(FIELD_OPS))()
    _check(lib().lp_debug_field_op_rates(float(target_ms), rates, ms, _stream_ptr(stream)))
    return {k: {"per_s": float(rates[i]), "ms": float(ms[i])} for i, k in enumerate(FIELD_OPS)}


# ------------------------------------------------------------------ profiling
def split_stall_count() -> int:
    """Waits of split blind rotations on the current device that ended
    without their partner workgroup (0 in normal operation)."""
    c = C.c_uint32(0)
    _check(lib().lp_split_stall_count(C.byref(c)))
    return int(c.value)


def profile_enable(on: bool = True):
    _check(lib().lp_profile_enable(1 if on else 0))


def profile_collect() -> dict:
    """{kernel name: {"launches", "jobs", "total_ms"}} since the last collect."""
    arr = (KernelStat * 8)()
    cnt = C.c_int(8)
    _check(lib().lp_profile_collect(arr, C.byref(cnt)))
    return {arr[i].name.decode(): {"launches": int(arr[i].launches), "jobs": int(arr[i].jobs),
                                   "total_ms": float(arr[i].total_ms)} for i in range(cnt.value)}


def profile_collect_launches(capacity: int = 1 << 16) -> list:
    """[{"name", "jobs", "shape", "ms"}] per recorded launch, oldest first."""
    arr = (LaunchRecord * capacity)()
    cnt = C.c_int(capacity)
    _check(lib().lp_profile_collect_launches(arr, C.byref(cnt)))
    return [{"name": arr[i].name.decode(), "jobs": int(arr[i].jobs), "shape": int(arr[i].shape),
             "ms": float(arr[i].ms)} for i in range(cnt.value)]


# ------------------------------------------------------------------ autotuning
def autotune(dk: DeviceKey, buckets=DEFAULT_TUNE_BUCKETS, br_steps: int = 64, stream=None) -> list:
    """Times the launch shapes at each batch size and installs the fastest
    per size for the current device (lp_autotune); returns the rows."""
    b = (C.c_uint32 * len(buckets))(*buckets)
    out = (TuneEntry * len(buckets))()
    _check(lib().lp_autotune(dk._h, b, len(buckets), br_steps, _stream_ptr(stream), out))
    return [r.as_dict() for r in out]


def tune_table() -> list:
    """The current device's installed rows (empty: built-in defaults)."""
    arr = (TuneEntry * TUNE_MAX_ROWS)()
    n = C.c_int(TUNE_MAX_ROWS)
    _check(lib().lp_tune_get(arr, C.byref(n)))
    return [arr[i].as_dict() for i in range(n.value)]


def set_tune_table(rows) -> None:
    """Installs rows (dicts with jobs, br_waves, ks_tile, ks_split); [] clears."""
    arr = (TuneEntry * max(1, len(rows)))()
    for i, r in enumerate(rows):
        arr[i] = TuneEntry(int(r["jobs"]), int(r["br_waves"]), int(r["ks_tile"]), int(r["ks_split"]),
                           float(r.get("br_us", 0.0)), float(r.get("ks_us", 0.0)))
    _check(lib().lp_tune_set(arr, len(rows)))


def tune_pick(jobs: int, n_lwe: int = 630) -> dict:
    """Shapes a launch of `jobs` jobs gets now (environment, table, defaults)."""
    r = TuneEntry()
    _check(lib().lp_tune_pick(jobs, n_lwe, C.byref(r)))
    d = r.as_dict()
    del d["br_us"], d["ks_us"]
    return d


def _kernel_sources_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in ("kernels.hip", "ntt32.h", "gl64.h", "jobs.h"):
        with open(os.path.join(os.path.dirname(__file__), "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def save_tune(path: str, rows=None, device_name: str = "") -> None:
    """Writes rows (default: the installed table) as a JSON cache tagged with
    the library version, a hash of the kernel sources and the device name."""
    import json
    doc = {"version": lib().lp_version().decode(), "kernels": _kernel_sources_hash(), "device": device_name,
           "rows": tune_table() if rows is None else list(rows)}
    with open(path, "w") as f:
        json.dump(doc, f, indent=1)


def load_tune(path: str, device_name: str = "") -> bool:
    """Installs a JSON cache written by save_tune if it matches this library,
    these kernel sources and the device name; returns whether it did."""
    import json
    try:
        with open(path) as f:
            doc = json.load(f)
    except (OSError, ValueError):
        return False
    if (doc.get("version") != lib().lp_version().decode() or doc.get("kernels") != _kernel_sources_hash()
            or doc.get("device") != device_name):
        return False
    set_tune_table(doc["rows"])
    return True


# ------------------------------------------------------------------ server
LP_EAGAIN = -6
LP_ECANCELED = -7


class Server:
    """Continuous-batching query server (lp_server_*).  Queries are host
    arrays (x, y, bounds, payload) of uint32 ciphertexts.  max_tick_rotations
    caps the blind rotations of one tick (0: a whole level per request;
    "auto": sized from the device's timed launch-shape table)."""

    def __init__(self, hbm_budget: int, max_inflight: int = 0, simulate: bool = False, fail_ticket: int = 0,
                 max_tick_rotations: "int | str" = 0):
        self._keep = {}
        cap = TICK_CAP_AUTO if max_tick_rotations == "auto" else int(max_tick_rotations)
        cfg = ServerConfig(hbm_budget, max_inflight, 1 if simulate else 0, fail_ticket, cap)
        h = C.c_void_p()
        _check(lib().lp_server_create(C.byref(cfg), C.byref(h)))
        self._h = h

    def close(self):
        h, self._h = getattr(self, "_h", None), None
        if h and _LIB is not None:
            _LIB.lp_server_free(h)
        self._keep = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _host_query(l, n_boxes, m, is_signed, x, y, bounds, payload):
        arrs = [np.ascontiguousarray(np.asarray(a, np.uint32)) for a in (x, y, bounds, payload)]
        return HostQuery(l, n_boxes, m, int(bool(is_signed)), *[_np_ptr(a) for a in arrs]), arrs

    def request_bytes(self, ck: CloudKey, l, n_boxes, m, is_signed, x, y, bounds, payload) -> int:
        q, _ = self._host_query(l, n_boxes, m, is_signed, x, y, bounds, payload)
        b = C.c_size_t()
        _check(lib().lp_server_request_bytes(ck._h, C.byref(q), C.byref(b)))
        return int(b.value)

    def submit(self, ck: CloudKey, l, n_boxes, m, is_signed, x, y, bounds, payload) -> int:
        q, arrs = self._host_query(l, n_boxes, m, is_signed, x, y, bounds, payload)
        t = C.c_uint64()
        _check(lib().lp_server_submit(self._h, ck._h, C.byref(q), C.byref(t)))
        self._keep[int(t.value)] = (ck, m, ck.params.n + 1)   # keep the key alive until done
        return int(t.value)

    def submit_blob(self, key_blob: bytes, l, n_boxes, m, is_signed, x, y, bounds, payload) -> int:
        """The request as the client sends it: PK as a serialized blob
        (CloudKey.serialize) that the server deserializes and owns."""
        q, arrs = self._host_query(l, n_boxes, m, is_signed, x, y, bounds, payload)
        t = C.c_uint64()
        _check(lib().lp_server_submit_blob(self._h, key_blob, len(key_blob), C.byref(q), C.byref(t)))
        n = struct.unpack_from("<I", key_blob, 8)[0]   # the header's LWE dimension
        self._keep[int(t.value)] = (None, m, n + 1)
        return int(t.value)

    def poll(self, ticket: int, wait: bool = True):
        """(status, result array or None, latency seconds)"""
        ck, m, w = self._keep[ticket]
        out = np.zeros((m, w), np.uint32)
        lat = C.c_double()
        st = lib().lp_server_poll(self._h, ticket, 1 if wait else 0, _np_ptr(out), C.byref(lat))
        if st == LP_EAGAIN:
            return st, None, None
        self._keep.pop(ticket, None)
        return st, (out if st == 0 else None), float(lat.value)

    def cancel(self, ticket: int):
        _check(lib().lp_server_cancel(self._h, ticket))

    def stats(self) -> dict:
        s = ServerStats()
        _check(lib().lp_server_stats_get(self._h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}
