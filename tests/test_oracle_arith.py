"""Pins of the oracle's arithmetic against closed forms, library routines and
brute force (no GPU).  Each test names the fact it relies on."""
import random

import numpy as np
import pytest

import oracle as O

P = O.DEFAULT
MASK32 = 0xFFFFFFFF


def _is_prime(n: int) -> bool:
    # deterministic Miller-Rabin written with Python big integers
    if n < 2:
        return False
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def test_ntt_prime_properties():
    q = O.ntt_prime()
    assert _is_prime(q)
    assert q % 4096 == 1
    # exact lift needs q/2 above the largest external-product coefficient
    bound = 2 * P.l * P.N * (1 << (P.bg_bit - 1)) * (1 << 32)
    assert q // 2 > bound


def test_mulmod_against_python_bigint():
    q = O.ntt_prime()
    rng = random.Random(7)
    cases = [(0, 0), (1, q - 1), (q - 1, q - 1), (2**62, 2**63), (2**64 - 1, 2**64 - 1)]
    cases += [(rng.getrandbits(64), rng.getrandbits(64)) for _ in range(2000)]
    for a, b in cases:
        assert O.mulmod(a, b) == (a % q) * (b % q) % q


def _np_negacyclic(a, b):
    """Library routine: full convolution (numpy) folded with X^N = -1."""
    N = len(a)
    full = np.convolve(np.asarray(a, dtype=object), np.asarray(b, dtype=object))
    out = np.array(full[:N], dtype=object)
    out[: len(full) - N] -= full[N:]
    return np.array([int(v) for v in out], dtype=object)


@pytest.mark.parametrize("N", [2, 4, 16, 64])
def test_schoolbook_matches_numpy_convolution(N):
    rng = np.random.default_rng(N)
    for _ in range(5):
        a = rng.integers(-(2**20), 2**20, N)
        b = rng.integers(-(2**20), 2**20, N)
        assert list(O.negacyclic_mul_schoolbook(a, b)) == list(_np_negacyclic(a, b))


def test_schoolbook_monomials():
    # X^i * X^j = X^(i+j) if i+j < N else -X^(i+j-N)
    N = 32
    for i in range(N):
        for j in range(0, N, 5):
            a = np.zeros(N, np.int64)
            b = np.zeros(N, np.int64)
            a[i] = 1
            b[j] = 1
            exp = np.zeros(N, np.int64)
            if i + j < N:
                exp[i + j] = 1
            else:
                exp[i + j - N] = -1
            assert (O.negacyclic_mul_schoolbook(a, b) == exp).all()


@pytest.mark.parametrize("N", [2, 8, 64, 256, 1024, 2048])
def test_ntt_product_equals_schoolbook(N):
    rng = np.random.default_rng(100 + N)
    a = rng.integers(-64, 64, N)
    b = rng.integers(0, 2**32, N)
    assert (O.negacyclic_mul_ntt(a, b) == O.negacyclic_mul_schoolbook(a, b)).all()


def test_ntt_product_adversarial_extremes():
    # every digit at -Bg/2 against every coefficient at 2^32-1: the largest
    # magnitude a single product reaches
    N = 1024
    a = np.full(N, -64, np.int64)
    b = np.full(N, 2**32 - 1, np.int64)
    r = O.negacyclic_mul_ntt(a, b)
    assert (r == O.negacyclic_mul_schoolbook(a, b)).all()
    assert abs(int(r[-1])) == 64 * (2**32 - 1) * N  # last coefficient sums with one sign


def test_modswitch_closed_form():
    rng = random.Random(3)
    xs = [0, 1, 2**20 - 1, 2**20, 2**21, MASK32, 2**31, 2**31 - 1] + [rng.getrandbits(32) for _ in range(5000)]
    for x in xs:
        # round half up of x * 2N / 2^32, taken mod 2N
        assert O.modswitch(x) == ((x * 2048 + 2**31) >> 32) % 2048


def test_decompose_reconstruction_and_range():
    rng = random.Random(11)
    xs = [0, 1, MASK32, 2**31, 2**31 - 1, 0x81020400, 2**10, 2**10 - 1] + [rng.getrandbits(32) for _ in range(20000)]
    for a in xs:
        d = O.decompose(a)
        assert all(-64 <= v < 64 for v in d)
        rec = sum(v * (1 << (32 - 7 * (j + 1))) for j, v in enumerate(d))
        err = (a - rec) % 2**32
        err = err - 2**32 if err >= 2**31 else err
        assert abs(err) <= 2**10, (a, d, err)
    assert O.decompose(0) == [0, 0, 0]


def test_rotation_identities():
    N = 1024
    rng = np.random.default_rng(5)
    p = rng.integers(0, 2**32, N, dtype=np.uint32)
    assert (O.poly_rotate(p, 0) == p).all()
    assert (O.poly_rotate(p, N) == (-p.astype(np.int64)) % 2**32).all()      # X^N = -1
    assert (O.poly_rotate(p, 2 * N) == p).all()                            # X^2N = 1
    for a, b in [(3, 5), (1000, 1047), (2047, 1), (1500, 900)]:
        lhs = O.poly_rotate(O.poly_rotate(p, a), b)
        assert (lhs == O.poly_rotate(p, (a + b) % (2 * N))).all()
    # X * p shifts up with the top coefficient negated into position 0
    r = O.poly_rotate(p, 1)
    assert r[0] == (2**32 - int(p[-1])) % 2**32 and (r[1:] == p[:-1]).all()


def test_rotation_matches_monomial_product():
    N = 64
    rng = np.random.default_rng(9)
    p = rng.integers(0, 2**20, N).astype(np.int64)
    for k in (0, 1, 17, 63, 64, 65, 127):
        mono = np.zeros(N, np.int64)
        sign = -1 if k >= N else 1
        mono[k % N] = sign
        exp = O.negacyclic_mul_schoolbook(mono, p) % 2**32
        assert (O.poly_rotate(p.astype(np.uint32), k).astype(np.int64) == exp).all()


def test_splitmix64_published_first_output():
    # SplitMix64 seeded with 0: first output 0xE220A8397B1DCDAF.  The stream
    # key of (seed 0, stream 0) is that first output; the first draw of
    # stream 0 is the first output of a SplitMix64 seeded with it.
    def mix(z):
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & (2**64 - 1)
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & (2**64 - 1)
        return z ^ (z >> 31)
    G = 0x9E3779B97F4A7C15
    assert mix(G) == 0xE220A8397B1DCDAF
    key = 0xE220A8397B1DCDAF
    assert O.rand_u64(0, 0, 0) == mix((key + G) & (2**64 - 1))
    assert O.rand_u64(0, 0, 4) == mix((key + 5 * G) & (2**64 - 1))


def test_gaussian_statistics():
    sig = 2.0**-15 * 2**32
    e = np.array([O.gauss_torus(42, 3, i, 2.0**-15) for i in range(20000)], np.float64)
    assert abs(e.mean()) < 4 * sig / np.sqrt(len(e))
    assert 0.97 < e.std() / sig < 1.03


def test_layout_sizes_match_paper():
    # (n+1) words of 4 bytes per sample; the paper truncates to the printed digit
    import json, math, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "sizes.json")))
    kib = lambda n, cnt: (n + 1) * 4 * cnt / 1024
    trunc = lambda v, d: math.floor(v * 10**d) / 10**d
    assert trunc(kib(540, 1), 2) == g["tlwe_sample_kib_lambda80"]
    assert trunc(kib(540, 13), 1) == g["gps_coordinate_kib"]["lambda80_l13"]
    assert trunc(kib(540, 16), 1) == g["gps_coordinate_kib"]["lambda80_l16"]
    assert trunc(kib(630, 13), 0) == g["gps_coordinate_kib"]["lambda128_l13"]
    assert trunc(kib(630, 16), 1) == g["gps_coordinate_kib"]["lambda128_l16"]
    assert trunc(kib(540, 81), 0) == g["service_samples_kib"]["lambda80_81"]
    assert trunc(kib(630, 81), 0) == g["service_samples_kib"]["lambda128_81"]
    # result of m = 9 samples at n = 630: within 1 % of the printed 22.9 KB
    assert abs(9 * 631 * 4 / 1000 - g["result_kbytes_m9"]) / g["result_kbytes_m9"] < 0.01
