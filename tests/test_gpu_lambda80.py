"""GPU parity under the paper's lambda 80 set (n = 540): gate batches and a
query equal the oracle bit for bit, and the query decrypts to the plaintext
predicate."""
import numpy as np
import pytest

import oracle as O
from oracle import plain
import paper_2407_19871_amd as lp
from paper_2407_19871_amd import workloads as W

from gpu_common import as_u32, cuda_or_skip

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def keys80():
    cuda_or_skip()
    ok = O.keygen(9, O.LAMBDA80)
    ck = lp.CloudKey.from_arrays(lp.params_lambda80(), ok.bsk, ok.ksk)
    return ok, O.Ctx(ok), lp.DeviceKey(ck)


@pytest.mark.parametrize("gate,B", [("NAND", 97), ("XNOR", 600)])
def test_lambda80_gate_batches(keys80, gate, B):
    ok, octx, dk = keys80
    a, b = W.random_bits(91 + B, B), W.random_bits(92 + B, B)
    c1, c2 = O.encrypt_bits(ok, a, seed=93), O.encrypt_bits(ok, b, seed=94)
    got = as_u32(lp.bootstrap_batch(dk, gate, lp.to_device(c1), lp.to_device(c2)))
    assert got.shape == (B, 541)
    exp, _ = octx.gate_batch(gate, c1, c2)
    assert (got == exp).all()


def test_lambda80_query(keys80):
    ok, octx, dk = keys80
    q = W.random_query(95, 13, 3, 4, force_inside=True)
    xb, yb, bb, pb = q.plain_bits()
    ct = O.encrypt_bits(ok, np.concatenate([xb, yb, bb, pb]), seed=96)
    l, N, m = q.l, q.n_boxes, q.m
    parts = (ct[:l], ct[l:2 * l], ct[2 * l:2 * l + 4 * l * N], ct[2 * l + 4 * l * N:])
    got = as_u32(lp.eval_bbox_query(dk, l, N, m, True, *[lp.to_device(v) for v in parts]))
    exp = octx.bbox_query(l, N, m, True, *parts)
    assert (got == exp).all()
    d, _ = O.decrypt_bits(ok, got)
    assert W.from_bits(d) == plain.predicate(q.x, q.y, q.boxes, q.payloads, l, m, True)


def test_lambda80_preprocess(keys80):
    import torch
    ok, _, dk = keys80
    z = O.encrypt_zeros(ok, 333, seed=97)
    bits = W.random_bits(98, 333)
    got = as_u32(lp.preprocess(dk, lp.to_device(z), torch.from_numpy(bits).to("cuda")))
    assert got.shape == (333, 541) and (got == O.preprocess(z, bits)).all()
