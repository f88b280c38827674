"""GPU parity: every stage of the gate bootstrap on the MI355X against the
CPU oracle, bit for bit, through the C ABI."""
import numpy as np
import pytest

import oracle as O
import paper_2407_19871_amd as lp

from gpu_common import as_u32, bits_of, cuda_or_skip, device_key_from_oracle, sync

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dkey(okeys):
    cuda_or_skip()
    return device_key_from_oracle(okeys)


def test_negacyclic_product_parity():
    cuda_or_skip()
    rng = np.random.default_rng(10)
    cnt = 7
    d = rng.integers(-64, 64, (cnt, 1024)).astype(np.int32)
    b = rng.integers(0, 2**32, (cnt, 1024), dtype=np.uint64).astype(np.uint32)
    d[0] = -64; b[0] = 0xFFFFFFFF          # largest magnitude
    d[1] = 63; b[1] = 0xFFFFFFFF
    d[2] = 0                                # zero product
    d[3] = 0; d[3, 0] = 1                   # identity
    d[4] = 0; d[4, 1023] = -1               # -X^1023
    out = as_u32(lp.debug_negacyclic_mul(lp.to_device(d.view(np.uint32)), lp.to_device(b)))
    for k in range(cnt):
        exp = O.negacyclic_mul_ntt(d[k].astype(np.int64), b[k].astype(np.int64)) % 2**32
        assert (out[k].astype(np.int64) == exp).all(), k


@pytest.mark.parametrize("steps", [1, 10, 630])
def test_blind_rotation_accumulator_parity(okeys, octx, dkey, steps):
    bits = [0, 1, 1, 0]
    ct = O.encrypt_bits(okeys, bits, seed=500 + steps)
    acc = as_u32(lp.debug_blind_rotate(dkey, lp.to_device(ct), steps))
    for k in range(len(bits)):
        assert (acc[k] == octx.blind_rotate(ct[k], steps)).all(), k


TRUTH = {
    "NAND": lambda a, b: 1 - (a & b), "AND": lambda a, b: a & b, "OR": lambda a, b: a | b,
    "XOR": lambda a, b: a ^ b, "XNOR": lambda a, b: 1 - (a ^ b), "NOR": lambda a, b: 1 - (a | b),
}


@pytest.mark.parametrize("gate", list(TRUTH))
def test_gate_parity_all_input_pairs(okeys, octx, dkey, gate):
    pairs = [(a, b) for a in (0, 1) for b in (0, 1)] * 3
    c1 = O.encrypt_bits(okeys, [a for a, _ in pairs], seed=61)
    c2 = O.encrypt_bits(okeys, [b for _, b in pairs], seed=62)
    got = as_u32(lp.bootstrap_batch(dkey, gate, lp.to_device(c1), lp.to_device(c2)))
    exp, _ = octx.gate_batch(gate, c1, c2)
    assert (got == exp).all()
    d, _ = bits_of(okeys, got)
    assert list(d) == [TRUTH[gate](a, b) for a, b in pairs]


def test_mux_not_copy_parity(okeys, octx, dkey):
    trip = [(s, t, f) for s in (0, 1) for t in (0, 1) for f in (0, 1)]
    cs = O.encrypt_bits(okeys, [s for s, _, _ in trip], seed=71)
    ct = O.encrypt_bits(okeys, [t for _, t, _ in trip], seed=72)
    cf = O.encrypt_bits(okeys, [f for _, _, f in trip], seed=73)
    got = as_u32(lp.bootstrap_batch(dkey, "MUX", lp.to_device(cs), lp.to_device(ct), lp.to_device(cf)))
    exp, _ = octx.gate_batch("MUX", cs, ct, cf)
    assert (got == exp).all()
    assert list(bits_of(okeys, got)[0]) == [t if s else f for s, t, f in trip]
    for g in ("NOT", "COPY"):
        got = as_u32(lp.bootstrap_batch(dkey, g, lp.to_device(cs)))
        assert (got == np.stack([octx.gate(g, c) for c in cs])).all()


@pytest.mark.parametrize("cnt", [1, 65, 300])
def test_keyswitch_parity(okeys, octx, dkey, cnt):
    rng = np.random.default_rng(cnt)
    big = rng.integers(0, 2**32, (cnt, 1025), dtype=np.uint64).astype(np.uint32)
    got = as_u32(lp.keyswitch_batch(dkey, lp.to_device(big)))
    for k in range(0, cnt, max(1, cnt // 20)):
        assert (got[k] == octx.keyswitch(big[k])).all(), k
    assert (got[-1] == octx.keyswitch(big[-1])).all()


def test_empty_batch_is_noop(dkey):
    torch = cuda_or_skip()
    z = torch.empty((0, 631), dtype=torch.int32, device="cuda")
    out = lp.bootstrap_batch(dkey, "NAND", z, z)
    sync()
    assert out.shape == (0, 631)
