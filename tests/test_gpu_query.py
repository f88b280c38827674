"""GPU parity of whole bounding-box queries: every output ciphertext equal
to the oracle's, and the decrypted service equal to the plaintext predicate."""
import numpy as np
import pytest

import oracle as O
from oracle import plain
import paper_2407_19871_amd as lp
from paper_2407_19871_amd import workloads as W

from gpu_common import as_u32, bits_of, cuda_or_skip, device_key_from_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dkey(okeys):
    cuda_or_skip()
    return device_key_from_oracle(okeys)


def encrypt_query(okeys, q, seed):
    xb, yb, bb, pb = q.plain_bits()
    ct = O.encrypt_bits(okeys, np.concatenate([xb, yb, bb, pb]), seed=seed)
    l, N = q.l, q.n_boxes
    return ct[:l], ct[l:2 * l], ct[2 * l:2 * l + 4 * l * N], ct[2 * l + 4 * l * N:]


def run_both(okeys, octx, dkey, q, seed):
    x, y, bounds, pay = encrypt_query(okeys, q, seed)
    got = as_u32(lp.eval_bbox_query(dkey, q.l, q.n_boxes, q.m, q.is_signed, lp.to_device(x), lp.to_device(y),
                                    lp.to_device(bounds), lp.to_device(pay)))
    exp = octx.bbox_query(q.l, q.n_boxes, q.m, q.is_signed, x, y, bounds, pay)
    return got, exp


@pytest.mark.parametrize("seed,inside", [(1, True), (2, False)])
def test_u8_one_box_query(okeys, octx, dkey, seed, inside):
    q = W.random_query_u8(seed, force_inside=inside)
    got, exp = run_both(okeys, octx, dkey, q, 10 + seed)
    assert (got == exp).all()
    d, _ = bits_of(okeys, got)
    assert W.from_bits(d) == plain.predicate(q.x, q.y, q.boxes, q.payloads, 8, 8, False)


def test_signed_zero_straddling_query(okeys, octx, dkey):
    q = W.random_query(5, 16, 3, 4, region=W.ZERO_STRADDLE, force_inside=True)
    got, exp = run_both(okeys, octx, dkey, q, 55)
    assert (got == exp).all()
    d, _ = bits_of(okeys, got)
    assert W.from_bits(d) == plain.predicate(q.x, q.y, q.boxes, q.payloads, 16, 4, True)


def test_16bit_16box_query_full_size(okeys, octx, dkey):
    # 16-bit fixed point, 16 boxes tiling the Korea-like region, 32-bit payloads
    q = W.random_query(2, 16, 16, 32, force_inside=True)
    got, exp = run_both(okeys, octx, dkey, q, 2)
    assert (got == exp).all()
    d, _ = bits_of(okeys, got)
    assert W.from_bits(d) == plain.predicate(q.x, q.y, q.boxes, q.payloads, 16, 32, True)


def test_query_launch_records_follow_the_levels(okeys, dkey):
    # one blind rotation and one key switch per depth level, in level order,
    # each rotation as wide as the scheduler's level
    q = W.random_query(7, 16, 4, 3, force_inside=True)
    x, y, bounds, pay = encrypt_query(okeys, q, 70)
    args = [lp.to_device(v) for v in (x, y, bounds, pay)]
    lp.eval_bbox_query(dkey, q.l, q.n_boxes, q.m, True, *args)
    cuda_or_skip().cuda.synchronize()
    lp.profile_enable(True)
    lp.profile_collect_launches()
    lp.eval_bbox_query(dkey, q.l, q.n_boxes, q.m, True, *args)
    recs = lp.profile_collect_launches()
    lp.profile_enable(False)
    widths = lp.bbox_level_widths(q.l, q.n_boxes, q.m)
    assert [r["name"] for r in recs] == ["blind_rotate", "keyswitch"] * len(widths)
    assert [r["jobs"] for r in recs[0::2]] == widths
    assert all(r["shape"] == lp.tune_pick(r["jobs"])["br_waves"] and r["ms"] > 0 for r in recs[0::2])
