"""Fused evaluation of several queries under different keys, and hipGraph
replays: every result bit-identical to the query evaluated alone and to the
oracle, and the decrypted service equal to the plaintext predicate."""
import numpy as np
import pytest

import oracle as O
from oracle import plain
import paper_2407_19871_amd as lp
from paper_2407_19871_amd import workloads as W

from gpu_common import as_u32, bits_of, cuda_or_skip, device_key_from_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def clients():
    """three clients: (oracle keys, oracle ctx, device key)"""
    cuda_or_skip()
    out = []
    for seed in (21, 22, 23):
        k = O.keygen(seed)
        out.append((k, O.Ctx(k), device_key_from_oracle(k)))
    return out


def encrypt_query(keys, q, seed):
    xb, yb, bb, pb = q.plain_bits()
    ct = O.encrypt_bits(keys, np.concatenate([xb, yb, bb, pb]), seed=seed)
    l, N = q.l, q.n_boxes
    return ct[:l], ct[l:2 * l], ct[2 * l:2 * l + 4 * l * N], ct[2 * l + 4 * l * N:]


def device_query(q, parts):
    x, y, b, p = (lp.to_device(v) for v in parts)
    return (q.l, q.n_boxes, q.m, q.is_signed, x, y, b, p)


def test_fused_uneven_queries_match_alone_and_oracle(clients):
    torch = cuda_or_skip()
    qs = [W.random_query_u8(3, force_inside=True),
          W.random_query(31, 16, 3, 5, region=W.ZERO_STRADDLE, force_inside=True),
          W.random_query(32, 16, 2, 4, force_inside=False)]
    parts = [encrypt_query(clients[k][0], q, 100 + k) for k, q in enumerate(qs)]
    dqs = [device_query(q, p) for q, p in zip(qs, parts)]
    keys = [c[2] for c in clients]
    fused = [as_u32(o) for o in lp.eval_bbox_batch(keys, dqs)]
    for k, q in enumerate(qs):
        alone = as_u32(lp.eval_bbox_query(keys[k], *dqs[k]))
        assert (fused[k] == alone).all(), k
        okeys, octx, _ = clients[k]
        exp = octx.bbox_query(q.l, q.n_boxes, q.m, q.is_signed, *parts[k])
        assert (fused[k] == exp).all(), k
        d, _ = bits_of(okeys, fused[k])
        assert W.from_bits(d) == plain.predicate(q.x, q.y, q.boxes, q.payloads, q.l, q.m, q.is_signed)
    torch.cuda.synchronize()


def test_graph_replays_equal_eager(monkeypatch, clients):
    torch = cuda_or_skip()
    okeys, octx, dk = clients[0]
    q = W.random_query(41, 16, 2, 3, region=W.ZERO_STRADDLE, force_inside=True)
    parts = encrypt_query(okeys, q, 41)
    dq = device_query(q, parts)
    monkeypatch.setenv("LOCPIR_GRAPHS", "0")
    eager = as_u32(lp.eval_bbox_query(dk, *dq))
    monkeypatch.setenv("LOCPIR_GRAPHS", "1")
    c1 = lp.to_device(O.encrypt_bits(okeys, [1, 0], seed=5))
    for rep in range(3):
        got = as_u32(lp.eval_bbox_query(dk, *dq))
        assert (got == eager).all(), rep
        # the program's own eager work and a synchronisation between replays
        lp.bootstrap_batch(dk, "NAND", c1, c1)
        torch.cuda.synchronize()
    exp = octx.bbox_query(q.l, q.n_boxes, q.m, q.is_signed, *parts)
    assert (eager == exp).all()


def test_many_clients_scaled(clients):
    """Uneven queries from many clients (16- and 32-bit coordinates, 1..4
    boxes, 32-bit payloads), keys reused round-robin over three clients:
    every decrypted result equals the predicate, two are checked against the
    oracle bit for bit."""
    cuda_or_skip()
    rng = np.random.default_rng(7)
    qs, parts, keys, owners = [], [], [], []
    for k in range(12):
        l = 32 if k % 2 == 0 else 16
        q = W.random_query(700 + k, l, int(rng.integers(1, 5)), 32,
                           region=W.ZERO_STRADDLE if k % 3 == 0 else W.KOREA, force_inside=bool(k % 2))
        c = k % 3
        qs.append(q)
        parts.append(encrypt_query(clients[c][0], q, 800 + k))
        keys.append(clients[c][2])
        owners.append(c)
    outs = [as_u32(o) for o in lp.eval_bbox_batch(keys, [device_query(q, p) for q, p in zip(qs, parts)])]
    for k, q in enumerate(qs):
        d, _ = bits_of(clients[owners[k]][0], outs[k])
        assert W.from_bits(d) == plain.predicate(q.x, q.y, q.boxes, q.payloads, q.l, q.m, True), k
    for k in (1, 2):
        q = qs[k]
        exp = clients[owners[k]][1].bbox_query(q.l, q.n_boxes, q.m, True, *parts[k])
        assert (outs[k] == exp).all(), k
