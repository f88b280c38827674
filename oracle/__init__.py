"""CPU oracle for the LocPIR gate-bootstrapping path.

TEST INFRASTRUCTURE ONLY: imported by tests/, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``; never by the product package.
It shares no code with the GPU path (see locpir_oracle.h for what it
computes and which passage of the paper each part follows).

The C core (liboracle.so) is built by oracle/build.py.  This module wraps it
with numpy arrays and adds the plaintext side: the bounding-box circuit of
Algorithms 2-5 evaluated on booleans and the plaintext predicate.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from . import plain  # noqa: F401  (plaintext circuit and predicate)

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

GATES = {"NAND": 0, "AND": 1, "OR": 2, "XOR": 3, "XNOR": 4, "NOR": 5, "MUX": 6, "NOT": 7, "COPY": 8}

u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")


class OrcParams(C.Structure):
    _fields_ = [("n", C.c_uint32), ("N", C.c_uint32), ("bg_bit", C.c_uint32), ("l", C.c_uint32),
                ("ks_base_bit", C.c_uint32), ("ks_t", C.c_uint32),
                ("lwe_sigma", C.c_double), ("bk_sigma", C.c_double)]


@dataclass(frozen=True)
class Params:
    """TFHE Torus32 parameters.  Default: n=630 (sigma 2^-15), N=1024, k=1,
    Bg=2^7, l=3 (sigma 2^-25), key-switch base 2^2 with t=8."""
    n: int = 630
    N: int = 1024
    bg_bit: int = 7
    l: int = 3
    ks_base_bit: int = 2
    ks_t: int = 8
    lwe_sigma: float = 2.0 ** -15
    bk_sigma: float = 2.0 ** -25

    def c(self) -> OrcParams:
        return OrcParams(self.n, self.N, self.bg_bit, self.l, self.ks_base_bit, self.ks_t,
                         self.lwe_sigma, self.bk_sigma)

    @property
    def bsk_words(self) -> int:
        return self.n * 2 * self.l * 2 * self.N

    @property
    def ksk_words(self) -> int:
        return self.N * self.ks_t * ((1 << self.ks_base_bit) - 1) * (self.n + 1)


DEFAULT = Params()
# The paper's lambda 80 set as read here (Sec. 5 gives only n = 540 and
# sigma = 2^-20.2; ring, gadget and key-switching parameters as in DEFAULT).
LAMBDA80 = Params(n=540, lwe_sigma=2.0 ** -20.2)


def lib():
    """Load liboracle.so, building it first if it is missing."""
    global _LIB
    if _LIB is not None:
        return _LIB
    # LOCPIR_ORACLE_LIB names another build of the same C core (e.g. an
    # address- and undefined-behaviour-sanitizer build)
    path = os.environ.get("LOCPIR_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
    if not os.path.exists(path):
        from .build import build
        build()
    L = C.CDLL(path)
    P = C.POINTER(OrcParams)
    vp = C.c_void_p
    L.orc_ntt_prime.restype = C.c_uint64
    L.orc_mulmod.restype = C.c_uint64
    L.orc_mulmod.argtypes = [C.c_uint64, C.c_uint64]
    L.orc_negacyclic_mul_ntt.argtypes = [C.c_uint32, i64p, i64p, i64p]
    L.orc_negacyclic_mul_schoolbook.argtypes = [C.c_uint32, i64p, i64p, i64p]
    L.orc_rand_u64.restype = C.c_uint64
    L.orc_rand_u64.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64]
    L.orc_gauss_torus.restype = C.c_int32
    L.orc_gauss_torus.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, C.c_double]
    L.orc_keygen.argtypes = [P, C.c_uint64, u8p, u8p, u32p, u32p]
    L.orc_encrypt_bits.argtypes = [P, u8p, u8p, C.c_size_t, C.c_uint64, C.c_uint64, u32p]
    L.orc_encrypt_zeros.argtypes = [P, u8p, C.c_size_t, C.c_uint64, C.c_uint64, u32p]
    L.orc_decrypt_bits.argtypes = [P, u8p, u32p, C.c_size_t, u8p, i32p]
    L.orc_phase.restype = C.c_uint32
    L.orc_phase.argtypes = [C.c_uint32, u8p, u32p]
    L.orc_modswitch.restype = C.c_uint32
    L.orc_modswitch.argtypes = [C.c_uint32, C.c_uint32]
    L.orc_decompose.argtypes = [P, C.c_uint32, i32p]
    L.orc_poly_rotate.argtypes = [C.c_uint32, u32p, C.c_uint32, u32p]
    L.orc_sample_extract.argtypes = [C.c_uint32, u32p, u32p]
    L.orc_ctx_create.restype = vp
    L.orc_ctx_create.argtypes = [P, u32p, u32p]
    L.orc_ctx_free.argtypes = [vp]
    L.orc_external_product.argtypes = [vp, C.c_uint32, u32p, u32p]
    L.orc_blind_rotate.argtypes = [vp, u32p, C.c_uint32, u32p]
    L.orc_keyswitch.argtypes = [vp, u32p, u32p]
    L.orc_bootstrap_raw.argtypes = [vp, u32p, vp, vp]
    L.orc_gate.argtypes = [vp, C.c_int, vp, vp, vp, u32p]
    L.orc_gate_big_batch.restype = C.c_int
    L.orc_gate_big_batch.argtypes = [vp, C.c_int, C.c_size_t, vp, vp, vp, u32p]
    L.orc_gate_batch.restype = C.c_int
    L.orc_gate_batch.argtypes = [vp, C.c_int, C.c_size_t, vp, vp, vp, u32p]
    L.orc_bbox_query.argtypes = [vp, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int,
                                 u32p, u32p, u32p, u32p, u32p]
    L.orc_bbox_counts.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, C.POINTER(C.c_uint64),
                                  C.POINTER(C.c_uint64), C.POINTER(C.c_uint32)]
    _LIB = L
    return L


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# ---------------------------------------------------------------- arithmetic
def ntt_prime() -> int:
    return int(lib().orc_ntt_prime())


def mulmod(a: int, b: int) -> int:
    return int(lib().orc_mulmod(a, b))


def negacyclic_mul_ntt(a, b):
    a = np.ascontiguousarray(a, np.int64)
    b = np.ascontiguousarray(b, np.int64)
    out = np.zeros(len(a), np.int64)
    if lib().orc_negacyclic_mul_ntt(len(a), a, b, out) != 0:
        raise ValueError("unsupported N")
    return out


def negacyclic_mul_schoolbook(a, b):
    a = np.ascontiguousarray(a, np.int64)
    b = np.ascontiguousarray(b, np.int64)
    out = np.zeros(len(a), np.int64)
    lib().orc_negacyclic_mul_schoolbook(len(a), a, b, out)
    return out


def rand_u64(seed: int, stream: int, idx: int) -> int:
    return int(lib().orc_rand_u64(seed, stream, idx))


def gauss_torus(seed: int, stream: int, idx: int, sigma: float) -> int:
    return int(lib().orc_gauss_torus(seed, stream, idx, sigma))


def modswitch(x: int, N: int = 1024) -> int:
    return int(lib().orc_modswitch(x & 0xFFFFFFFF, N))


def decompose(a: int, P: Params = DEFAULT):
    d = np.zeros(P.l, np.int32)
    lib().orc_decompose(C.byref(P.c()), a & 0xFFFFFFFF, d)
    return [int(v) for v in d]


def poly_rotate(poly, k: int):
    poly = np.ascontiguousarray(poly, np.uint32)
    out = np.zeros_like(poly)
    lib().orc_poly_rotate(len(poly), poly, k, out)
    return out


def sample_extract(acc):
    acc = np.ascontiguousarray(acc, np.uint32).reshape(-1)
    N = len(acc) // 2
    out = np.zeros(N + 1, np.uint32)
    lib().orc_sample_extract(N, acc, out)
    return out


def phase(ct, key) -> int:
    ct = np.ascontiguousarray(ct, np.uint32)
    key = np.ascontiguousarray(key, np.uint8)
    return int(lib().orc_phase(len(key), key, ct))


# ---------------------------------------------------------------- keys
@dataclass
class Keys:
    params: Params
    seed: int
    s_lwe: np.ndarray   # [n] u8
    s_ring: np.ndarray  # [N] u8
    bsk: np.ndarray     # [n][2l][2][N] u32 (Torus32)
    ksk: np.ndarray     # [N][t][base-1][n+1] u32 (Torus32)


def keygen(seed: int, P: Params = DEFAULT) -> Keys:
    s = np.zeros(P.n, np.uint8)
    S = np.zeros(P.N, np.uint8)
    bsk = np.zeros(P.bsk_words, np.uint32)
    ksk = np.zeros(P.ksk_words, np.uint32)
    lib().orc_keygen(C.byref(P.c()), seed, s, S, bsk, ksk)
    return Keys(P, seed, s, S, bsk, ksk)


def encrypt_bits(keys: Keys, bits, seed: int, first_index: int = 0) -> np.ndarray:
    P = keys.params
    bits = np.ascontiguousarray(np.asarray(bits, np.uint8).reshape(-1))
    ct = np.zeros((len(bits), P.n + 1), np.uint32)
    lib().orc_encrypt_bits(C.byref(P.c()), keys.s_lwe, bits, len(bits), seed, first_index, ct)
    return ct


def encrypt_zeros(keys: Keys, cnt: int, seed: int, first_index: int = 0) -> np.ndarray:
    """The client's fresh samples of Sec. 3: encryptions of the torus value 0."""
    P = keys.params
    ct = np.zeros((cnt, P.n + 1), np.uint32)
    lib().orc_encrypt_zeros(C.byref(P.c()), keys.s_lwe, cnt, seed, first_index, ct)
    return ct


def preprocess(zero_ct, bits) -> np.ndarray:
    """Algorithm 1 (Preprocess): the cloud encrypts its plaintext service bits
    by adding the trivial sample (0, f(bit)) to one fresh client sample of
    zero each, f(1) = +1/8 and f(0) = -1/8 on the torus (the encoding of
    Encrypt in Sec. 2.2).  zero_ct: [cnt][n+1]; bits: cnt values in {0, 1}.
    An all-zero zero_ct gives the noiseless trivial samples of the bits."""
    zero_ct = np.asarray(zero_ct, np.uint32)
    bits = np.asarray(bits, np.uint8).reshape(-1)
    if zero_ct.ndim != 2 or len(zero_ct) != len(bits):
        raise ValueError("preprocess: one zero sample per bit")
    if bits.size and bits.max() > 1:
        raise ValueError("preprocess: bits must be 0/1")
    out = zero_ct.copy()
    out[:, -1] += np.where(bits == 1, np.uint32(1 << 29), np.uint32((1 << 32) - (1 << 29)))
    return out


def decrypt_bits(keys: Keys, ct):
    P = keys.params
    ct = np.ascontiguousarray(ct, np.uint32).reshape(-1, P.n + 1)
    bits = np.zeros(len(ct), np.uint8)
    ph = np.zeros(len(ct), np.int32)
    lib().orc_decrypt_bits(C.byref(P.c()), keys.s_lwe, ct, len(ct), bits, ph)
    return bits, ph


# ---------------------------------------------------------------- evaluation
class Ctx:
    """Oracle evaluation context (keys plus the transformed bootstrapping key)."""

    def __init__(self, keys: Keys):
        self.keys = keys
        self.P = keys.params
        self._c = lib().orc_ctx_create(C.byref(self.P.c()), keys.bsk, keys.ksk)
        if not self._c:
            raise ValueError("unsupported parameters")

    def __del__(self):
        if getattr(self, "_c", None):
            lib().orc_ctx_free(self._c)
            self._c = None

    def external_product(self, i: int, d):
        d = np.ascontiguousarray(d, np.uint32).reshape(-1)
        out = np.zeros(2 * self.P.N, np.uint32)
        lib().orc_external_product(self._c, i, d, out)
        return out

    def blind_rotate(self, ct, steps: int | None = None):
        ct = np.ascontiguousarray(ct, np.uint32).reshape(-1)
        acc = np.zeros(2 * self.P.N, np.uint32)
        lib().orc_blind_rotate(self._c, ct, self.P.n if steps is None else steps, acc)
        return acc

    def keyswitch(self, big):
        big = np.ascontiguousarray(big, np.uint32).reshape(-1)
        out = np.zeros(self.P.n + 1, np.uint32)
        lib().orc_keyswitch(self._c, big, out)
        return out

    def bootstrap_raw(self, ct):
        """(extracted LWE_N sample, key-switched LWE_n sample)"""
        ct = np.ascontiguousarray(ct, np.uint32).reshape(-1)
        big = np.zeros(self.P.N + 1, np.uint32)
        out = np.zeros(self.P.n + 1, np.uint32)
        lib().orc_bootstrap_raw(self._c, ct, _ptr(big), _ptr(out))
        return big, out

    def gate(self, gate: str, c1, c2=None, c3=None):
        out = np.zeros(self.P.n + 1, np.uint32)
        arrs = [None if c is None else np.ascontiguousarray(c, np.uint32).reshape(-1) for c in (c1, c2, c3)]
        lib().orc_gate(self._c, GATES[gate], *[_ptr(a) for a in arrs], out)
        return out

    def gate_batch(self, gate: str, c1, c2=None, c3=None):
        """cnt gates in parallel over the host's threads: returns (out, threads)."""
        w = self.P.n + 1
        arrs = [None if c is None else np.ascontiguousarray(c, np.uint32).reshape(-1, w) for c in (c1, c2, c3)]
        cnt = arrs[0].shape[0]
        out = np.zeros((cnt, w), np.uint32)
        th = lib().orc_gate_batch(self._c, GATES[gate], cnt, *[_ptr(a) for a in arrs], out)
        return out, th

    def gate_big_batch(self, gate: str, c1, c2=None, c3=None):
        """cnt bootstrapped gates up to their key switch: [cnt][N+1], the
        samples under the ring key that the key switch takes."""
        w = self.P.n + 1
        arrs = [None if c is None else np.ascontiguousarray(c, np.uint32).reshape(-1, w) for c in (c1, c2, c3)]
        cnt = arrs[0].shape[0]
        big = np.zeros((cnt, self.P.N + 1), np.uint32)
        if not lib().orc_gate_big_batch(self._c, GATES[gate], cnt, *[_ptr(a) for a in arrs], big):
            raise ValueError(f"{gate} does not bootstrap")
        return big

    def bbox_query(self, l, n_boxes, m, is_signed, x, y, bounds, payload):
        w = self.P.n + 1
        x = np.ascontiguousarray(x, np.uint32).reshape(l, w)
        y = np.ascontiguousarray(y, np.uint32).reshape(l, w)
        bounds = np.ascontiguousarray(bounds, np.uint32).reshape(n_boxes * 4 * l, w)
        payload = np.ascontiguousarray(payload, np.uint32).reshape(n_boxes * m, w)
        out = np.zeros((m, w), np.uint32)
        lib().orc_bbox_query(self._c, l, n_boxes, m, int(bool(is_signed)), x, y, bounds, payload, out)
        return out


def bbox_counts(l: int, n_boxes: int, m: int):
    br, ks, depth = C.c_uint64(), C.c_uint64(), C.c_uint32()
    lib().orc_bbox_counts(l, n_boxes, m, C.byref(br), C.byref(ks), C.byref(depth))
    return int(br.value), int(ks.value), int(depth.value)
