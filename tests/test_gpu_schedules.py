"""Schedule invariance: the same inputs give identical bits under every
launch shape (waves per bootstrap, including the rotation split over two
workgroups, key-switch tile and ring-index split), and equal the oracle."""
import numpy as np
import pytest

import oracle as O
import paper_2407_19871_amd as lp
from paper_2407_19871_amd import workloads as W

from gpu_common import as_u32, cuda_or_skip, device_key_from_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dkey(okeys):
    cuda_or_skip()
    return device_key_from_oracle(okeys)


@pytest.fixture(scope="module")
def inputs(okeys, octx):
    B = 9
    a, b = W.random_bits(11, B), W.random_bits(12, B)
    c1 = O.encrypt_bits(okeys, a, seed=13)
    c2 = O.encrypt_bits(okeys, b, seed=14)
    exp, _ = octx.gate_batch("AND", c1, c2)
    return c1, c2, exp


@pytest.mark.parametrize("waves", ["1", "2", "3", "4", "5", "6", "7"])
def test_blind_rotation_waves_per_bootstrap(monkeypatch, okeys, octx, dkey, waves):
    monkeypatch.setenv("LOCPIR_BR_WAVES", waves)
    ct = O.encrypt_bits(okeys, [1, 0, 1], seed=88)
    acc = as_u32(lp.debug_blind_rotate(dkey, lp.to_device(ct), 20))
    for k in range(3):
        assert (acc[k] == octx.blind_rotate(ct[k], 20)).all(), k


@pytest.mark.parametrize("waves", ["1", "2", "3", "4", "5", "6", "7"])
def test_gate_waves_per_bootstrap(monkeypatch, dkey, inputs, waves):
    monkeypatch.setenv("LOCPIR_BR_WAVES", waves)
    monkeypatch.setenv("LOCPIR_KS_SPLIT", "1")
    c1, c2, exp = inputs
    got = as_u32(lp.bootstrap_batch(dkey, "AND", lp.to_device(c1), lp.to_device(c2)))
    assert (got == exp).all()


@pytest.mark.parametrize("tile,split", [("1", "1"), ("4", "1"), ("1", "16"), ("4", "2"), ("8", "1"), ("8", "16"),
                                        ("16", "8")])
def test_keyswitch_shapes(monkeypatch, octx, dkey, tile, split):
    monkeypatch.setenv("LOCPIR_KS_TILE", tile)
    monkeypatch.setenv("LOCPIR_KS_SPLIT", split)
    rng = np.random.default_rng(int(tile) * 100 + int(split))
    big = rng.integers(0, 2**32, (21, 1025), dtype=np.uint64).astype(np.uint32)
    got = as_u32(lp.keyswitch_batch(dkey, lp.to_device(big)))
    for k in (0, 7, 20):
        assert (got[k] == octx.keyswitch(big[k])).all(), k


@pytest.mark.parametrize("waves", ["1", "2", "3", "4", "5", "6", "7"])
def test_query_under_each_rotation_shape(monkeypatch, okeys, octx, dkey, waves):
    """An 8-bit one-box query (107 bootstraps, 12 levels) with every level
    forced to one rotation shape equals the oracle."""
    from paper_2407_19871_amd import workloads as Wl
    monkeypatch.setenv("LOCPIR_BR_WAVES", waves)
    lp.set_tune_table(lp.tune_table())  # drops cached programs
    q = Wl.random_query_u8(55, force_inside=True)
    xb, yb, bb, pb = q.plain_bits()
    ct = O.encrypt_bits(okeys, np.concatenate([xb, yb, bb, pb]), seed=56)
    l, N, m = q.l, q.n_boxes, q.m
    parts = (ct[:l], ct[l:2 * l], ct[2 * l:2 * l + 4 * l * N], ct[2 * l + 4 * l * N:])
    got = as_u32(lp.eval_bbox_query(dkey, l, N, m, False, *[lp.to_device(v) for v in parts]))
    lp.set_tune_table(lp.tune_table())
    assert (got == octx.bbox_query(l, N, m, False, *parts)).all()
