"""Query server on the GPU: requests from several clients arriving together
and staggered; each result is bit-identical to the same query evaluated
alone, equal to the oracle for a small one, and decrypts to the predicate."""
import time

import numpy as np
import pytest

import oracle as O
from oracle import plain
import paper_2407_19871_amd as lp
from paper_2407_19871_amd import workloads as W

from gpu_common import bits_of, cuda_or_skip

pytestmark = pytest.mark.gpu


def enc(okeys, q, seed):
    xb, yb, bb, pb = q.plain_bits()
    ct = O.encrypt_bits(okeys, np.concatenate([xb, yb, bb, pb]), seed=seed)
    l, N = q.l, q.n_boxes
    return ct[:l], ct[l:2 * l], ct[2 * l:2 * l + 4 * l * N], ct[2 * l + 4 * l * N:]


def test_server_results_equal_alone_and_predicate():
    cuda_or_skip()
    p = lp.params_default()
    okeys = [O.keygen(s) for s in (61, 62)]
    cks = [lp.CloudKey.from_arrays(p, k.bsk, k.ksk) for k in okeys]
    qs = [W.random_query_u8(5, force_inside=True),
          W.random_query(51, 16, 2, 6, region=W.ZERO_STRADDLE, force_inside=True),
          W.random_query(52, 16, 3, 4, force_inside=False),
          W.random_query(53, 16, 1, 5, force_inside=True)]
    owner = [0, 1, 0, 1]
    parts = [enc(okeys[owner[k]], q, 900 + k) for k, q in enumerate(qs)]
    srv = lp.Server(64 << 30)
    tickets = [srv.submit(cks[owner[k]], q.l, q.n_boxes, q.m, q.is_signed, *parts[k]) for k, q in enumerate(qs[:3])]
    time.sleep(0.3)                                   # the fourth arrives while the others run
    tickets.append(srv.submit(cks[owner[3]], qs[3].l, qs[3].n_boxes, qs[3].m, qs[3].is_signed, *parts[3]))
    results = [srv.poll(t) for t in tickets]
    stats = srv.stats()
    srv.close()
    assert all(r[0] == 0 for r in results)
    assert stats["completed"] == 4 and stats["bytes_in_use"] == 0
    assert stats["ticks"] < sum(lp.bbox_counts(q.l, q.n_boxes, q.m)[2] for q in qs)  # levels were shared
    dks = [lp.DeviceKey(ck) for ck in cks]
    for k, q in enumerate(qs):
        got = results[k][1]
        alone = lp.to_host(lp.eval_bbox_query(dks[owner[k]], q.l, q.n_boxes, q.m, q.is_signed,
                                              *[lp.to_device(v) for v in parts[k]]))
        assert (got == alone).all(), k
        d, _ = bits_of(okeys[owner[k]], got)
        assert W.from_bits(d) == plain.predicate(q.x, q.y, q.boxes, q.payloads, q.l, q.m, q.is_signed), k
    ctx = O.Ctx(okeys[0])
    assert (results[0][1] == ctx.bbox_query(qs[0].l, 1, qs[0].m, False, *parts[0])).all()


def test_server_mixed_parameter_sets():
    """lambda 128 and lambda 80 clients in flight together: each result
    equals the same query alone under its own key and decrypts to the
    predicate."""
    cuda_or_skip()
    ok = [O.keygen(71), O.keygen(72, O.LAMBDA80)]
    cks = [lp.CloudKey.from_arrays(lp.params_default(), ok[0].bsk, ok[0].ksk),
           lp.CloudKey.from_arrays(lp.params_lambda80(), ok[1].bsk, ok[1].ksk)]
    qs = [W.random_query(73, 13, 2, 3, force_inside=True), W.random_query(74, 13, 2, 3, force_inside=True),
          W.random_query_u8(75, force_inside=True)]
    owner = [0, 1, 1]
    parts = [enc(ok[owner[k]], q, 950 + k) for k, q in enumerate(qs)]
    srv = lp.Server(64 << 30)
    tickets = [srv.submit(cks[owner[k]], q.l, q.n_boxes, q.m, q.is_signed, *parts[k]) for k, q in enumerate(qs)]
    results = [srv.poll(t) for t in tickets]
    srv.close()
    assert all(r[0] == 0 for r in results)
    dks = [lp.DeviceKey(ck) for ck in cks]
    for k, q in enumerate(qs):
        got = results[k][1]
        assert got.shape == (q.m, cks[owner[k]].params.n + 1)
        alone = lp.to_host(lp.eval_bbox_query(dks[owner[k]], q.l, q.n_boxes, q.m, q.is_signed,
                                              *[lp.to_device(v) for v in parts[k]]))
        assert (got == alone).all(), k
        d, _ = bits_of(ok[owner[k]], got)
        assert W.from_bits(d) == plain.predicate(q.x, q.y, q.boxes, q.payloads, q.l, q.m, q.is_signed), k


def test_server_tick_cap_leaves_results_unchanged():
    """A rotation cap below the widest levels splits them over several
    ticks (MUX pairs and key switches stay with their rotations): every
    result is bit-identical to the query evaluated alone."""
    cuda_or_skip()
    p = lp.params_default()
    okeys = O.keygen(71)
    ck = lp.CloudKey.from_arrays(p, okeys.bsk, okeys.ksk)
    qs = [W.random_query_u8(7, force_inside=True), W.random_query(72, 16, 3, 4, force_inside=True)]
    parts = [enc(okeys, q, 950 + k) for k, q in enumerate(qs)]
    cap = 25
    srv = lp.Server(64 << 30, max_tick_rotations=cap)
    tickets = [srv.submit(ck, q.l, q.n_boxes, q.m, q.is_signed, *parts[k]) for k, q in enumerate(qs)]
    results = [srv.poll(t) for t in tickets]
    stats = srv.stats()
    srv.close()
    assert all(r[0] == 0 for r in results)
    assert stats["widest_tick"] <= cap
    assert stats["ticks"] > max(lp.bbox_counts(q.l, q.n_boxes, q.m)[2] for q in qs)  # levels were split
    dk = lp.DeviceKey(ck)
    for k, q in enumerate(qs):
        alone = lp.to_host(lp.eval_bbox_query(dk, q.l, q.n_boxes, q.m, q.is_signed,
                                              *[lp.to_device(v) for v in parts[k]]))
        assert (results[k][1] == alone).all(), k
        d, _ = bits_of(okeys, results[k][1])
        assert W.from_bits(d) == plain.predicate(q.x, q.y, q.boxes, q.payloads, q.l, q.m, q.is_signed), k
