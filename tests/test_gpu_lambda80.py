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


def test_lambda80_fused_clients_and_mixed_refusal(keys80):
    """Two lambda 80 clients fused level by level equal each query alone and
    the oracle; a fused batch mixing the lambda 80 and lambda 128 sets is
    refused (one launch reads every pool with one sample stride)."""
    ok, octx, dk = keys80
    ok2 = O.keygen(10, O.LAMBDA80)
    dk2 = lp.DeviceKey(lp.CloudKey.from_arrays(lp.params_lambda80(), ok2.bsk, ok2.ksk))
    qs = [W.random_query(201, 13, 2, 3, force_inside=True), W.random_query_u8(202, force_inside=True)]
    owners = [(ok, octx, dk), (ok2, O.Ctx(ok2), dk2)]
    dev, host = [], []
    for k, (q, (o, _, _)) in enumerate(zip(qs, owners)):
        xb, yb, bb, pb = q.plain_bits()
        ct = O.encrypt_bits(o, np.concatenate([xb, yb, bb, pb]), seed=210 + k)
        l, N = q.l, q.n_boxes
        parts = (ct[:l], ct[l:2 * l], ct[2 * l:2 * l + 4 * l * N], ct[2 * l + 4 * l * N:])
        host.append(parts)
        dev.append((q.l, q.n_boxes, q.m, q.is_signed, *[lp.to_device(v) for v in parts]))
    outs = lp.eval_bbox_batch([dk, dk2], dev)
    for k, (q, (o, c, d)) in enumerate(zip(qs, owners)):
        got = as_u32(outs[k])
        assert got.shape == (q.m, 541)
        assert (got == as_u32(lp.eval_bbox_query(d, *dev[k]))).all()
        assert (got == c.bbox_query(q.l, q.n_boxes, q.m, q.is_signed, *host[k])).all()
        dd, _ = O.decrypt_bits(o, got)
        assert W.from_bits(dd) == plain.predicate(q.x, q.y, q.boxes, q.payloads, q.l, q.m, q.is_signed)
    k128 = O.keygen(11)
    dk128 = lp.DeviceKey(lp.CloudKey.from_arrays(lp.params_default(), k128.bsk, k128.ksk))
    with pytest.raises(lp.LocpirError):
        lp.eval_bbox_batch([dk, dk128], [dev[0], dev[0]])
