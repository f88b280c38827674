"""Pins of the oracle's keys, encryption and bootstrapping (no GPU): the
paper's decryption condition, closed forms of the blind rotation, the noise
model and truth tables."""
import numpy as np
import pytest

import oracle as O
from oracle import plain
from paper_2407_19871_amd import workloads as W

P = O.DEFAULT
Q32 = 2**32


def sgn32(v):
    v = np.asarray(v, np.int64) % Q32
    return np.where(v >= 2**31, v - Q32, v)


def ring_phase(keys, acc):
    """phase B - A*S of a TRLWE sample, by the schoolbook product"""
    N = P.N
    A = acc[:N].astype(np.int64)
    B = acc[N:].astype(np.int64)
    AS = O.negacyclic_mul_schoolbook(A, keys.s_ring.astype(np.int64))
    return (B - AS) % Q32


def test_encrypt_decrypt_roundtrip(okeys):
    bits = np.random.default_rng(1).integers(0, 2, 500).astype(np.uint8)
    ct = O.encrypt_bits(okeys, bits, seed=9)
    d, ph = O.decrypt_bits(okeys, ct)
    assert (d == bits).all()
    err = ph.astype(np.int64) - np.where(bits == 1, 2**29, -(2**29))
    assert np.abs(err).max() < 2**28               # |e| < 1/16 (Sec. 2.2)
    sig = P.lwe_sigma * Q32
    assert 0.85 < err.std() / sig < 1.15


def test_bsk_rows_are_tgsw_of_key_bits(okeys):
    # row (p, j) of BSK_i has phase E - s_i*g_j*S for p = 0 (mask gadget) and
    # E + s_i*g_j for p = 1 (body gadget), with |E| small
    N, l = P.N, P.l
    bsk = okeys.bsk.reshape(P.n, 2 * l, 2, N)
    for i in (0, 1, 200, 629):
        si = int(okeys.s_lwe[i])
        for r in range(2 * l):
            p, j = divmod(r, l)
            g = 1 << (32 - 7 * (j + 1))
            ph = ring_phase(okeys, bsk[i, r].reshape(-1))
            if p == 1:
                exp = np.zeros(N, np.int64)
                exp[0] = si * g
            else:
                exp = (-si * g * okeys.s_ring.astype(np.int64)) % Q32
            e = sgn32(ph - exp)
            assert np.abs(e).max() < 8 * P.bk_sigma * Q32 + 1


def test_ksk_rows_encrypt_scaled_ring_key(okeys):
    ksk = okeys.ksk.reshape(P.N, P.ks_t, 3, P.n + 1)
    for i in (0, 5, 1023):
        for j in (0, 3, 7):
            for v in (1, 2, 3):
                ph = O.phase(ksk[i, j, v - 1], okeys.s_lwe)
                msg = (v * int(okeys.s_ring[i]) << (32 - 2 * (j + 1))) % Q32
                assert abs(int(sgn32(ph - msg))) < 8 * P.lwe_sigma * Q32


def test_special_case_zero_key_noiseless_bsk():
    # s = 0 and sigma_bk = 0: every CMux adds a phase-0 sample, so after the
    # blind rotation ACC has phase exactly X^{-b~} v and the extracted sample
    # has phase +1/8 for b~ in [0, N), -1/8 otherwise.
    Pz = O.Params(bk_sigma=0.0)
    k = O.keygen(77, Pz)
    bsk = k.bsk.reshape(Pz.n, 2 * Pz.l, 2, Pz.N)
    for i in range(Pz.n):                      # remove the s_i * gadget terms
        if k.s_lwe[i]:
            for r in range(2 * Pz.l):
                p, j = divmod(r, Pz.l)
                bsk[i, r, p, 0] = np.uint32((int(bsk[i, r, p, 0]) - (1 << (32 - 7 * (j + 1)))) % 2**32)
    k.s_lwe[:] = 0
    ctx = O.Ctx(k)
    rng = np.random.default_rng(0)
    for b in [0, 2**20, 2**31 - 2**21, 2**31, 2**32 - 2**20 - 1] + list(rng.integers(0, 2**32, 4)):
        ct = rng.integers(0, 2**32, P.n + 1, dtype=np.uint64).astype(np.uint32)
        ct[P.n] = np.uint32(int(b))
        acc = ctx.blind_rotate(ct)
        bbar = O.modswitch(int(b))
        v = np.full(P.N, 2**29, np.uint32)
        exp = O.poly_rotate(v, (2 * P.N - bbar) % (2 * P.N))
        assert (ring_phase(k, acc) == exp.astype(np.int64)).all()
        big, _ = ctx.bootstrap_raw(ct)
        ph = O.phase(big, k.s_ring)
        assert ph == (2**29 if bbar < P.N else 2**32 - 2**29)


def test_blind_rotation_phase_is_rotated_test_vector(okeys, octx):
    # with the real key, ACC's phase equals X^{-phi~} v coefficientwise up to
    # the bootstrapping noise, where phi~ = b~ - sum a~_i s_i (mod 2N)
    rng = np.random.default_rng(4)
    for _ in range(2):
        ct = O.encrypt_bits(okeys, [int(rng.integers(2))], seed=int(rng.integers(1 << 30)))[0]
        acc = octx.blind_rotate(ct)
        phibar = (O.modswitch(int(ct[P.n])) - sum(O.modswitch(int(ct[i])) * int(okeys.s_lwe[i]) for i in range(P.n))) % 2048
        v = np.full(P.N, 2**29, np.uint32)
        exp = O.poly_rotate(v, (2 * P.N - phibar) % (2 * P.N)).astype(np.int64)
        e = sgn32(ring_phase(okeys, acc) - exp)
        assert np.abs(e).max() < 2**27
        # partial rotation after 10 steps: the same with only 10 key bits
        acc10 = octx.blind_rotate(ct, 10)
        phi10 = (O.modswitch(int(ct[P.n])) - sum(O.modswitch(int(ct[i])) * int(okeys.s_lwe[i]) for i in range(10))) % 2048
        exp10 = O.poly_rotate(v, (2 * P.N - phi10) % (2 * P.N)).astype(np.int64)
        assert np.abs(sgn32(ring_phase(okeys, acc10) - exp10)).max() < 2**26


def test_external_product_equals_schoolbook(okeys, octx):
    # ExtProd(BSK_i, D) = sum_{p,j} dec_j(D_p) * BSK_i[p,j] with schoolbook
    # products, mod 2^32
    N, l = P.N, P.l
    rng = np.random.default_rng(8)
    d = rng.integers(0, 2**32, 2 * N, dtype=np.uint64).astype(np.uint32)
    i = 17
    got = octx.external_product(i, d)
    bsk = okeys.bsk.reshape(P.n, 2 * l, 2, N)
    exp = np.zeros(2 * N, np.int64)
    for p in range(2):
        digs = np.array([O.decompose(int(v)) for v in d[p * N:(p + 1) * N]], np.int64)
        for j in range(l):
            for q in range(2):
                prod = O.negacyclic_mul_schoolbook(digs[:, j], bsk[i, p * l + j, q].astype(np.int64))
                exp[q * N:(q + 1) * N] += prod
    assert (got.astype(np.int64) == exp % Q32).all()


def test_keyswitch_preserves_phase(okeys, octx):
    rng = np.random.default_rng(12)
    for _ in range(3):
        bit = int(rng.integers(2))
        big = np.zeros(P.N + 1, np.uint32)
        big[:P.N] = rng.integers(0, 2**32, P.N, dtype=np.uint64).astype(np.uint32)
        dot = int(np.dot(big[:P.N].astype(np.int64), okeys.s_ring.astype(np.int64)) % Q32)
        mu = 2**29 if bit else 2**32 - 2**29
        big[P.N] = np.uint32((dot + mu) % Q32)
        out = octx.keyswitch(big)
        e = int(sgn32(O.phase(out, okeys.s_lwe) - mu))
        # rounding of N coefficients to 16 bits plus N*t KSK noises
        assert abs(e) < 2**26


TRUTH = {
    "NAND": lambda a, b: 1 - (a & b), "AND": lambda a, b: a & b, "OR": lambda a, b: a | b,
    "XOR": lambda a, b: a ^ b, "XNOR": lambda a, b: 1 - (a ^ b), "NOR": lambda a, b: 1 - (a | b),
}


@pytest.mark.parametrize("gate", list(TRUTH))
def test_gate_truth_tables(okeys, octx, gate):
    pairs = [(a, b) for a in (0, 1) for b in (0, 1)] * 2
    c1 = O.encrypt_bits(okeys, [a for a, _ in pairs], seed=21)
    c2 = O.encrypt_bits(okeys, [b for _, b in pairs], seed=22)
    out, _ = octx.gate_batch(gate, c1, c2)
    d, ph = O.decrypt_bits(okeys, out)
    assert list(d) == [TRUTH[gate](a, b) for a, b in pairs]
    assert np.abs(np.abs(ph.astype(np.int64)) - 2**29).max() < 2**28


def test_mux_not_copy_truth_tables(okeys, octx):
    trip = [(s, t, f) for s in (0, 1) for t in (0, 1) for f in (0, 1)]
    cs = O.encrypt_bits(okeys, [s for s, _, _ in trip], seed=31)
    ct = O.encrypt_bits(okeys, [t for _, t, _ in trip], seed=32)
    cf = O.encrypt_bits(okeys, [f for _, _, f in trip], seed=33)
    out, _ = octx.gate_batch("MUX", cs, ct, cf)
    d, ph = O.decrypt_bits(okeys, out)
    assert list(d) == [t if s else f for s, t, f in trip]
    assert np.abs(np.abs(ph.astype(np.int64)) - 2**29).max() < 2**28
    dn, _ = O.decrypt_bits(okeys, np.stack([octx.gate("NOT", c) for c in cs]))
    assert list(dn) == [1 - s for s, _, _ in trip]
    dc, _ = O.decrypt_bits(okeys, np.stack([octx.gate("COPY", c) for c in cs]))
    assert list(dc) == [s for s, _, _ in trip]


def test_bootstrap_noise_matches_model(okeys, octx):
    # model (torus^2 units): V_BR = n (k+1) l N (Bg^2/12) s_bk^2 for the
    # blind rotation; V_KS = N t (3/4) s_lwe^2 for the key-switching key noise
    # (a digit is non-zero 3/4 of the time) plus N (1/2) (2^-16)^2/12 for
    # rounding each coefficient to 16 bits.  The empirical std of the output
    # phase error must be within a factor 2 of sqrt(V_BR + V_KS).
    n, N, l, t = P.n, P.N, P.l, P.ks_t
    v_br = n * 2 * l * N * (128.0**2 / 12) * P.bk_sigma**2
    v_ks = N * t * 0.75 * P.lwe_sigma**2 + N * 0.5 * (2.0**-16) ** 2 / 12
    model = np.sqrt(v_br + v_ks) * Q32
    bits = np.random.default_rng(2).integers(0, 2, 256).astype(np.uint8)
    c1 = O.encrypt_bits(okeys, bits, seed=41)
    c2 = O.encrypt_bits(okeys, np.ones_like(bits), seed=42)
    out, _ = octx.gate_batch("AND", c1, c2)
    d, ph = O.decrypt_bits(okeys, out)
    assert (d == bits).all()
    err = ph.astype(np.int64) - np.where(bits == 1, 2**29, -(2**29))
    ratio = err.std() / model
    assert 0.5 < ratio < 2.0, ratio


@pytest.fixture(scope="module")
def okeys80():
    k = O.keygen(8, O.LAMBDA80)
    return k, O.Ctx(k)


def test_lambda80_gates_and_query(okeys80):
    """The lambda 80 set (n = 540): every two-input gate on all input pairs
    and a MUX on all triples decrypt to their truth tables within the phase
    bound, and a small query decrypts to the plaintext predicate."""
    keys, ctx = okeys80
    pairs = [(a, b) for a in (0, 1) for b in (0, 1)]
    c1 = O.encrypt_bits(keys, [a for a, _ in pairs], seed=81)
    c2 = O.encrypt_bits(keys, [b for _, b in pairs], seed=82)
    for gate, f in TRUTH.items():
        out, _ = ctx.gate_batch(gate, c1, c2)
        d, ph = O.decrypt_bits(keys, out)
        assert list(d) == [f(a, b) for a, b in pairs], gate
        assert np.abs(np.abs(ph.astype(np.int64)) - 2**29).max() < 2**28
    trip = [(s, t, f) for s in (0, 1) for t in (0, 1) for f in (0, 1)]
    cs, ct, cf = (O.encrypt_bits(keys, [v[i] for v in trip], seed=83 + i) for i in range(3))
    out, _ = ctx.gate_batch("MUX", cs, ct, cf)
    assert list(O.decrypt_bits(keys, out)[0]) == [t if s else f for s, t, f in trip]
    q = W.random_query(84, 13, 2, 3, force_inside=True)
    xb, yb, bb, pb = q.plain_bits()
    cts = O.encrypt_bits(keys, np.concatenate([xb, yb, bb, pb]), seed=85)
    l, N = q.l, q.n_boxes
    res = ctx.bbox_query(l, N, q.m, True, cts[:l], cts[l:2 * l], cts[2 * l:2 * l + 4 * l * N], cts[2 * l + 4 * l * N:])
    d, _ = O.decrypt_bits(keys, res)
    assert W.from_bits(d) == plain.predicate(q.x, q.y, q.boxes, q.payloads, l, q.m, True)


def test_zero_samples_and_preprocess(okeys):
    """Sec. 3 and Algorithm 1: the client's fresh samples carry phase e alone
    (Gaussian at the LWE width, inside the decryption bound), and Preprocess
    shifts each phase by exactly f(bit) = +-1/8 without touching the mask,
    so the services decrypt to the cloud's bits; an all-zero sample gives the
    noiseless trivial encryption."""
    z = O.encrypt_zeros(okeys, 4000, seed=31)
    _, ph0 = O.decrypt_bits(okeys, z)
    ph0 = ph0.astype(np.int64)
    sig = P.lwe_sigma * Q32
    assert np.abs(ph0).max() < 2**28
    assert abs(ph0.mean()) < 4 * sig / np.sqrt(len(ph0))
    assert 0.95 < ph0.std() / sig < 1.05
    # streams of their own: not the masks of Encrypt under the same seed
    assert not (z[:8, :P.n] == O.encrypt_bits(okeys, np.zeros(8, np.uint8), seed=31)[:, :P.n]).any(axis=1).all()
    bits = np.random.default_rng(32).integers(0, 2, 4000).astype(np.uint8)
    c = O.preprocess(z, bits)
    d, ph = O.decrypt_bits(okeys, c)
    assert (d == bits).all() and (c[:, :P.n] == z[:, :P.n]).all()
    shift = (ph.astype(np.int64) - ph0) % Q32
    assert (shift == np.where(bits == 1, 2**29, Q32 - 2**29)).all()
    t = O.preprocess(np.zeros((16, P.n + 1), np.uint32), bits[:16])
    dt, pht = O.decrypt_bits(okeys, t)
    assert (dt == bits[:16]).all() and (pht.astype(np.int64) == np.where(bits[:16] == 1, 2**29, -2**29)).all()
    with pytest.raises(ValueError):
        O.preprocess(z[:2], np.array([0, 2], np.uint8))
    with pytest.raises(ValueError):
        O.preprocess(z[:3], np.array([0, 1], np.uint8))


@pytest.mark.parametrize("seed,inside", [(41, True), (42, False)])
def test_protocol_query_through_oracle(okeys, octx, seed, inside):
    """The protocol of Sec. 3 end to end on the oracle: the client sends
    N*m fresh samples of zero and its encrypted coordinates; the cloud
    encrypts its services with Preprocess and enters its plaintext bounds
    as trivial samples; the result decrypts to the plaintext predicate."""
    q = W.random_query_u8(seed, force_inside=inside)
    l, N, m = q.l, q.n_boxes, q.m
    xb, yb, bb, pb = q.plain_bits()
    gps = O.encrypt_bits(okeys, np.concatenate([xb, yb]), seed=seed)
    zero = O.encrypt_zeros(okeys, N * m, seed=seed + 100)
    payload = O.preprocess(zero, pb)
    bounds = O.preprocess(np.zeros((4 * l * N, P.n + 1), np.uint32), bb)
    res = octx.bbox_query(l, N, m, False, gps[:l], gps[l:], bounds, payload)
    d, ph = O.decrypt_bits(okeys, res)
    assert W.from_bits(d) == plain.predicate(q.x, q.y, q.boxes, q.payloads, l, m, False)
    assert np.abs(np.abs(ph.astype(np.int64)) - 2**29).max() < 2**28


def test_gates_before_key_switching(okeys, octx):
    """The sample a gate hands to its key switch is an LWE encryption, under
    the ring key S, of the gate's value (+-1/8 with the bootstrap's noise);
    key switching it reproduces the whole gate bit for bit.  NOT and COPY do
    not bootstrap and are refused."""
    pairs = [(a, b) for a in (0, 1) for b in (0, 1)]
    c1 = O.encrypt_bits(okeys, [a for a, _ in pairs], seed=141)
    c2 = O.encrypt_bits(okeys, [b for _, b in pairs], seed=142)
    trip = [(s, t, f) for s in (0, 1) for t in (0, 1) for f in (0, 1)]
    cs, ct, cf = (O.encrypt_bits(okeys, [v[i] for v in trip], seed=143 + i) for i in range(3))
    cases = [(g, (c1, c2), [f(a, b) for a, b in pairs]) for g, f in TRUTH.items()]
    cases.append(("MUX", (cs, ct, cf), [t if s else f for s, t, f in trip]))
    for gate, ins, want in cases:
        big = octx.gate_big_batch(gate, *ins)
        assert big.shape == (len(want), P.N + 1)
        ph = np.array([sgn32(O.phase(b, okeys.s_ring)) for b in big])
        assert list((ph > 0).astype(int)) == want, gate
        assert np.abs(np.abs(ph) - 2**29).max() < 2**28, gate
        full, _ = octx.gate_batch(gate, *ins)
        assert all((octx.keyswitch(b) == o).all() for b, o in zip(big, full)), gate
    for gate in ("NOT", "COPY"):
        with pytest.raises(ValueError):
            octx.gate_big_batch(gate, c1)
