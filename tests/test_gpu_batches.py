"""GPU parity of gate batches of the microbenchmark sizes (uniform random
bits, NAND gates sharing one key) and of ragged sizes; with the built-in
launch shapes 769 and 1024 run the two-wave rotation, the smaller sizes the
split one."""
import numpy as np
import pytest

import oracle as O
import paper_2407_19871_amd as lp
from paper_2407_19871_amd import workloads as W

from gpu_common import as_u32, bits_of, cuda_or_skip, device_key_from_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dkey(okeys):
    cuda_or_skip()
    return device_key_from_oracle(okeys)


@pytest.mark.parametrize("B", [1, 64, 97, 769, 1024])
def test_nand_batch_parity(okeys, octx, dkey, B):
    a = W.random_bits(1000 + B, B)
    b = W.random_bits(2000 + B, B)
    c1 = O.encrypt_bits(okeys, a, seed=3000 + B)
    c2 = O.encrypt_bits(okeys, b, seed=4000 + B)
    got = as_u32(lp.bootstrap_batch(dkey, "NAND", lp.to_device(c1), lp.to_device(c2)))
    exp, _ = octx.gate_batch("NAND", c1, c2)
    assert (got == exp).all()
    d, ph = bits_of(okeys, got)
    assert (d == 1 - (a & b)).all()
    assert np.abs(np.abs(ph.astype(np.int64)) - 2**29).max() < 2**28


def test_mux_batch_ragged(okeys, octx, dkey):
    B = 37
    s, t, f = (W.random_bits(k, B) for k in (1, 2, 3))
    cs, ct, cf = (O.encrypt_bits(okeys, v, seed=90 + i) for i, v in enumerate((s, t, f)))
    got = as_u32(lp.bootstrap_batch(dkey, "MUX", lp.to_device(cs), lp.to_device(ct), lp.to_device(cf)))
    exp, _ = octx.gate_batch("MUX", cs, ct, cf)
    assert (got == exp).all()
    assert (bits_of(okeys, got)[0] == np.where(s == 1, t, f)).all()


def test_nand_batch_full_size_sampled(okeys, octx, dkey):
    """The batched microbenchmark's largest launch (16384 NAND gates, one
    shared key): every output decrypts to the truth table, and 512 sampled
    outputs plus the first, the last and rows at power-of-two boundaries
    equal the oracle's gates bit for bit."""
    B = 16384
    a = W.random_bits(5001, B)
    b = W.random_bits(5002, B)
    c1 = O.encrypt_bits(okeys, a, seed=5003)
    c2 = O.encrypt_bits(okeys, b, seed=5004)
    got = as_u32(lp.bootstrap_batch(dkey, "NAND", lp.to_device(c1), lp.to_device(c2)))
    d, ph = bits_of(okeys, got)
    assert (d == 1 - (a & b)).all()
    assert np.abs(np.abs(ph.astype(np.int64)) - 2**29).max() < 2**28
    idx = np.random.default_rng(5005).choice(B, 512, replace=False)
    idx = np.unique(np.concatenate([idx, [0, 1, 63, 64, 1023, 1024, 8191, 8192, B - 1]]))
    exp, _ = octx.gate_batch("NAND", c1[idx], c2[idx])
    assert (got[idx] == exp).all()


@pytest.mark.parametrize("gate,B", [("NAND", 97), ("XNOR", 64), ("MUX", 45)])
def test_gates_before_key_switching(okeys, octx, dkey, gate, B):
    ins = [O.encrypt_bits(okeys, W.random_bits(160 + B + i, B), seed=170 + i) for i in range(3 if gate == "MUX" else 2)]
    d_ins = [lp.to_device(c) for c in ins]
    big = lp.bootstrap_batch_noks(dkey, gate, *d_ins)
    assert big.shape == (B, 1025)
    assert (as_u32(big) == octx.gate_big_batch(gate, *ins)).all()
    # key switching the samples gives the whole gate
    full = as_u32(lp.bootstrap_batch(dkey, gate, *d_ins))
    assert (as_u32(lp.keyswitch_batch(dkey, big)) == full).all()


def test_gates_before_key_switching_edges(dkey):
    import torch
    e = torch.empty((0, 631), dtype=torch.int32, device="cuda")
    assert lp.bootstrap_batch_noks(dkey, "NAND", e, e).shape == (0, 1025)
    with pytest.raises(lp.LocpirError):
        lp.bootstrap_batch_noks(dkey, "NOT", lp.to_device(np.zeros((3, 631), np.uint32)))


def test_gate_output_may_overwrite_an_input(okeys, dkey):
    ins = [O.encrypt_bits(okeys, W.random_bits(230 + i, 50), seed=240 + i) for i in range(3)]
    d = [lp.to_device(c) for c in ins]
    nand = as_u32(lp.bootstrap_batch(dkey, "NAND", d[0], d[1]))
    mux = as_u32(lp.bootstrap_batch(dkey, "MUX", d[0], d[1], d[2]))
    lp.bootstrap_batch(dkey, "MUX", d[0], d[1], d[2], out=d[2])
    lp.bootstrap_batch(dkey, "NAND", d[0], d[1], out=d[0])
    assert (as_u32(d[2]) == mux).all() and (as_u32(d[0]) == nand).all()
