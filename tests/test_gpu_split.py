"""Split blind rotation (br_waves 6: one bootstrap on two workgroups of four
waves, each owning one accumulator component and trading its key products
for the other component every step; br_waves 7: the same sized for two
workgroups per CU, up to 256 jobs): bit-exact against the oracle for the
accumulator after all n steps, for gates at one, ragged and maximal launch
widths, and for whole queries whose narrow levels run split, with the
exchange area reused launch after launch; a forced give-up fails the call
that launched it."""
import numpy as np
import pytest

import oracle as O
import paper_2407_19871_amd as lp
from oracle import plain
from paper_2407_19871_amd import workloads as W

from gpu_common import as_u32, cuda_or_skip, device_key_from_oracle

pytestmark = pytest.mark.gpu

SPLIT_MAX = {6: 128, 7: 256}  # widest launch of each split shape


@pytest.fixture(scope="module")
def dkey(okeys):
    cuda_or_skip()
    return device_key_from_oracle(okeys)


@pytest.fixture(scope="module")
def stalls_before(dkey):
    """The device's count of split waits that ran out of polls before the
    tests of this module."""
    return lp.split_stall_count()


@pytest.fixture(params=[6, 7])
def split_w(request):
    """The split shape under test."""
    return request.param


@pytest.fixture
def split_max(split_w):
    return SPLIT_MAX[split_w]


@pytest.fixture
def split_table(split_w, split_max):
    """Split rotations up to the shape's widest launch, one gadget level per
    wave above."""
    old = lp.tune_table()
    lp.set_tune_table([{"jobs": split_max, "br_waves": split_w, "ks_tile": 4, "ks_split": 8},
                       {"jobs": 1 << 22, "br_waves": 3, "ks_tile": 8, "ks_split": 8}])
    yield
    lp.set_tune_table(old)


def test_accumulator_after_all_steps(monkeypatch, okeys, octx, dkey, split_w):
    monkeypatch.setenv("LOCPIR_BR_WAVES", str(split_w))
    ct = O.encrypt_bits(okeys, [1, 0, 1], seed=91)
    acc = as_u32(lp.debug_blind_rotate(dkey, lp.to_device(ct), 630))
    for k in range(3):
        assert (acc[k] == octx.blind_rotate(ct[k], 630)).all(), k


@pytest.mark.parametrize("cnt", [1, 13, 120])
def test_gates_at_launch_widths(monkeypatch, okeys, octx, dkey, split_w, cnt):
    """One pair; a ragged block (idle pairs in the last block of 16
    tickets); nearly the widest launch."""
    monkeypatch.setenv("LOCPIR_BR_WAVES", str(split_w))
    a, b = W.random_bits(200 + cnt, cnt), W.random_bits(300 + cnt, cnt)
    c1 = O.encrypt_bits(okeys, a, seed=400 + cnt)
    c2 = O.encrypt_bits(okeys, b, seed=500 + cnt)
    got = as_u32(lp.bootstrap_batch(dkey, "XNOR", lp.to_device(c1), lp.to_device(c2)))
    exp, _ = octx.gate_batch("XNOR", c1, c2)
    assert (got == exp).all()
    d, _ = O.decrypt_bits(okeys, got)
    assert (d == (1 - (a ^ b))).all()


@pytest.mark.parametrize("cnt", [129, 200, 256])
def test_gates_at_two_per_cu_widths(monkeypatch, okeys, octx, dkey, cnt):
    """The split sized for two workgroups per CU past the one-per-CU width:
    ragged and full."""
    monkeypatch.setenv("LOCPIR_BR_WAVES", "7")
    a, b = W.random_bits(1200 + cnt, cnt), W.random_bits(1300 + cnt, cnt)
    c1 = O.encrypt_bits(okeys, a, seed=1400 + cnt)
    c2 = O.encrypt_bits(okeys, b, seed=1500 + cnt)
    lp.profile_enable(True)
    try:
        got = as_u32(lp.bootstrap_batch(dkey, "NOR", lp.to_device(c1), lp.to_device(c2)))
        recs = lp.profile_collect_launches()
    finally:
        lp.profile_enable(False)
    assert [r["shape"] for r in recs if r["name"] == "blind_rotate"] == [7]
    exp, _ = octx.gate_batch("NOR", c1, c2)
    assert (got == exp).all()


def test_mux_at_widest_split_launch(monkeypatch, okeys, octx, dkey, split_w, split_max):
    """64 (128) MUX gates are 128 (256) rotations, the widest launch of the
    shape."""
    monkeypatch.setenv("LOCPIR_BR_WAVES", str(split_w))
    cnt = split_max // 2
    s, t, f = (W.random_bits(600 + k, cnt) for k in range(3))
    cts = [O.encrypt_bits(okeys, v, seed=700 + k) for k, v in enumerate((s, t, f))]
    got = as_u32(lp.bootstrap_batch(dkey, "MUX", *[lp.to_device(c) for c in cts]))
    exp, _ = octx.gate_batch("MUX", *cts)
    assert (got == exp).all()


def test_wider_launch_falls_back(monkeypatch, okeys, octx, dkey, split_w, split_max):
    """A forced split shape on a launch wider than it takes runs the split
    sized for two workgroups per CU where that fits, else four waves two per
    CU (and is still exact)."""
    monkeypatch.setenv("LOCPIR_BR_WAVES", str(split_w))
    fallback = 7 if split_max < SPLIT_MAX[7] else 5
    assert lp.tune_pick(split_max)["br_waves"] == split_w
    assert lp.tune_pick(split_max + 1)["br_waves"] == fallback
    cnt = split_max + 3
    a, b = W.random_bits(801, cnt), W.random_bits(802, cnt)
    c1, c2 = O.encrypt_bits(okeys, a, seed=803), O.encrypt_bits(okeys, b, seed=804)
    lp.profile_enable(True)
    try:
        got = as_u32(lp.bootstrap_batch(dkey, "AND", lp.to_device(c1), lp.to_device(c2)))
        recs = lp.profile_collect_launches()
    finally:
        lp.profile_enable(False)
    assert [r["shape"] for r in recs if r["name"] == "blind_rotate"] == [fallback]
    exp, _ = octx.gate_batch("AND", c1, c2)
    assert (got == exp).all()


def _query_parts(okeys, q, seed):
    xb, yb, bb, pb = q.plain_bits()
    ct = O.encrypt_bits(okeys, np.concatenate([xb, yb, bb, pb]), seed=seed)
    l, N = q.l, q.n_boxes
    return (ct[:l], ct[l:2 * l], ct[2 * l:2 * l + 4 * l * N], ct[2 * l + 4 * l * N:])


@pytest.mark.parametrize("graphs", ["1", "0"])
def test_query_with_split_levels(monkeypatch, okeys, octx, dkey, split_w, split_max, split_table, graphs):
    """An 8-bit one-box query (12 levels, every one at most 32 rotations
    wide, so all of them split), run twice: the exchange area is reused by
    every level and every replay."""
    monkeypatch.setenv("LOCPIR_GRAPHS", graphs)
    q = W.random_query_u8(31, force_inside=True)
    parts = _query_parts(okeys, q, seed=32)
    l, N, m = q.l, q.n_boxes, q.m
    assert max(lp.bbox_level_widths(l, N, m)) <= split_max
    exp = octx.bbox_query(l, N, m, False, *parts)
    lp.profile_enable(True)
    try:
        for _ in range(2):
            res = as_u32(lp.eval_bbox_query(dkey, l, N, m, False, *[lp.to_device(v) for v in parts]))
            assert (res == exp).all()
        recs = lp.profile_collect_launches()
    finally:
        lp.profile_enable(False)
    assert {r["shape"] for r in recs if r["name"] == "blind_rotate"} == {split_w}
    d, _ = O.decrypt_bits(okeys, res)
    assert W.from_bits(d) == plain.predicate(q.x, q.y, q.boxes, q.payloads, l, m, False)


@pytest.fixture(scope="module")
def placement_query(okeys, octx):
    """9-bit signed coordinates against 11 boxes (1263 bootstraps) and the
    oracle's result."""
    q = W.random_query(41, 9, 11, 2, force_inside=True)
    parts = _query_parts(okeys, q, seed=42)
    return q, parts, octx.bbox_query(q.l, q.n_boxes, q.m, True, *parts)


@pytest.mark.parametrize("early", ["0", "1", None])
def test_query_xnor_placements(monkeypatch, okeys, dkey, placement_query, early):
    """With 11 boxes the MUX levels (88 rotations) split and the mixed ones
    (132) cannot, so the XNORs go early unless told otherwise; either
    placement gives the oracle's bits, with the launch widths it announces."""
    if early is None:
        monkeypatch.delenv("LOCPIR_XNOR_EARLY", raising=False)
    else:
        monkeypatch.setenv("LOCPIR_XNOR_EARLY", early)
    monkeypatch.delenv("LOCPIR_BR_WAVES", raising=False)
    old = lp.tune_table()
    lp.set_tune_table([])  # built-in shapes; also drops cached programs
    try:
        q, parts, exp = placement_query
        l, N, m = q.l, q.n_boxes, q.m
        widths = lp.bbox_level_widths(l, N, m)
        assert (widths[0] == l * 4 * N) == (early != "0")
        lp.profile_enable(True)
        lp.profile_collect_launches()
        try:
            res = as_u32(lp.eval_bbox_query(dkey, l, N, m, True, *[lp.to_device(v) for v in parts]))
            recs = lp.profile_collect_launches()
        finally:
            lp.profile_enable(False)
    finally:
        lp.set_tune_table(old)
    assert [r["jobs"] for r in recs if r["name"] == "blind_rotate"] == widths
    assert (res == exp).all()
    d, _ = O.decrypt_bits(okeys, res)
    assert W.from_bits(d) == plain.predicate(q.x, q.y, q.boxes, q.payloads, l, m, True)


def test_no_stalled_waits(dkey, stalls_before):
    """No split wait above ran out of polls."""
    assert lp.split_stall_count() == stalls_before


def test_give_up_path_is_bounded_and_reported(monkeypatch, okeys, octx, dkey, split_table):
    """Forced from the host with a one-poll limit, split waits give up: the
    kernel still finishes, the stalls are counted, and the call that launched
    them fails with LP_EDEVICE instead of returning an undefined result.  The
    next launches on the same query program's exchange area (eager, so that
    each launch reads the limit) are exact again, and so is a gate batch."""
    monkeypatch.setenv("LOCPIR_GRAPHS", "0")
    q = W.random_query_u8(61, force_inside=True)
    parts = _query_parts(okeys, q, seed=62)
    l, N, m = q.l, q.n_boxes, q.m
    args = [lp.to_device(v) for v in parts]
    before = lp.split_stall_count()
    monkeypatch.setenv("LOCPIR_SPLIT_SPIN", "1")
    with pytest.raises(lp.LocpirError) as e:
        lp.eval_bbox_query(dkey, l, N, m, False, *args)
    assert e.value.code == -3 and "split-rotation" in str(e.value)
    assert lp.split_stall_count() > before
    bits = np.array([0, 1, 1, 0, 1, 0, 0, 1], np.uint8)
    c = O.encrypt_bits(okeys, bits, seed=63)
    c1, c2 = lp.to_device(c[:4]), lp.to_device(c[4:])
    with pytest.raises(lp.LocpirError) as e:
        lp.bootstrap_batch(dkey, "NAND", c1, c2)
    assert e.value.code == -3
    monkeypatch.delenv("LOCPIR_SPLIT_SPIN")
    after = lp.split_stall_count()
    got = as_u32(lp.eval_bbox_query(dkey, l, N, m, False, *args))
    assert (got == octx.bbox_query(l, N, m, False, *parts)).all()
    exp, _ = octx.gate_batch("NAND", c[:4], c[4:])
    assert (as_u32(lp.bootstrap_batch(dkey, "NAND", c1, c2)) == exp).all()
    assert lp.split_stall_count() == after


def test_give_up_fails_the_server_request_only(monkeypatch, okeys, octx, split_table):
    """The server under the same forced limit: the request whose split
    rotations gave up ends with LP_EDEVICE and the server goes on; a server
    without the limit returns the exact result of the same request."""
    q = W.random_query_u8(64, force_inside=True)
    parts = _query_parts(okeys, q, seed=65)
    l, N, m = q.l, q.n_boxes, q.m
    ck = lp.CloudKey.from_arrays(lp.params_default(), okeys.bsk, okeys.ksk)
    monkeypatch.setenv("LOCPIR_SPLIT_SPIN", "1")
    srv = lp.Server(8 << 30)
    st, out, _ = srv.poll(srv.submit(ck, l, N, m, False, *parts))
    stats = srv.stats()
    srv.close()
    monkeypatch.delenv("LOCPIR_SPLIT_SPIN")
    assert st == -3 and out is None
    assert stats["failed"] == 1 and stats["bytes_in_use"] == 0
    srv = lp.Server(8 << 30)
    st, out, _ = srv.poll(srv.submit(ck, l, N, m, False, *parts))
    srv.close()
    assert st == 0
    assert (out == octx.bbox_query(l, N, m, False, *parts)).all()


def test_split_profile_reports_every_phase(okeys, dkey, split_w):
    """The profiling build of the split rotation: every wave reports every
    phase; the fourth wave stages the step's key while the level waves run
    their forward transforms, which take longer, so it then waits for them;
    all four meet at the barriers, so their step totals agree."""
    ct = lp.to_device(O.encrypt_bits(okeys, [1, 0, 1, 1, 0, 0, 1, 0], seed=5))
    r = lp.debug_split_profile(dkey, ct, split_w)
    assert r["ms"] > 0
    assert len(r["waves"]) == 4
    for w in r["waves"]:
        assert set(w) == set(lp.SPLIT_PHASES) and all(v >= 0 for v in w.values())
    assert r["waves"][0]["forward"] > r["waves"][3]["forward"] > 0
    assert r["waves"][3]["barrier_f"] > 10 * r["waves"][0]["barrier_f"]
    sums = [sum(w.values()) for w in r["waves"]]
    assert max(sums) < 1.05 * min(sums)


def test_area_reused_across_launch_widths(okeys, octx, dkey, split_table):
    """One exchange area (the allocation-free entry's static one) serves split
    launches of different widths back to back, each bit-exact against the
    oracle: no exchange word or step flag of one launch leaks into the next,
    whichever XCDs its pairs ran on."""
    for k, cnt in enumerate((128, 37, 128, 1, 64, 128)):
        bits = [W.random_bits(9100 + 10 * k + i, cnt) for i in range(2)]
        c1, c2 = (O.encrypt_bits(okeys, b, seed=9200 + 10 * k + i) for i, b in enumerate(bits))
        got = as_u32(lp.bootstrap_batch_noalloc(dkey, "NAND", lp.to_device(c1), lp.to_device(c2)))
        exp, _ = octx.gate_batch("NAND", c1, c2)
        assert (got == exp).all(), cnt


def test_agent_scope_exchange(monkeypatch, okeys, octx, dkey, split_table):
    """Pairs whose halves run on two XCDs trade at agent scope instead of
    through one XCD's L2.  Dispatch normally puts both halves on one XCD, so
    LOCPIR_SPLIT_AGENT=1 forces that path on every pair: gates at two widths
    and a whole query, run twice on one exchange area, stay bit-exact."""
    monkeypatch.setenv("LOCPIR_SPLIT_AGENT", "1")
    for cnt in (128, 37):
        a, b = W.random_bits(9300 + cnt, cnt), W.random_bits(9400 + cnt, cnt)
        c1, c2 = O.encrypt_bits(okeys, a, seed=9500 + cnt), O.encrypt_bits(okeys, b, seed=9600 + cnt)
        got = as_u32(lp.bootstrap_batch(dkey, "NAND", lp.to_device(c1), lp.to_device(c2)))
        exp, _ = octx.gate_batch("NAND", c1, c2)
        assert (got == exp).all(), cnt
    q = W.random_query_u8(33, force_inside=True)
    parts = _query_parts(okeys, q, seed=34)
    exp = octx.bbox_query(q.l, q.n_boxes, q.m, False, *parts)
    for _ in range(2):
        res = as_u32(lp.eval_bbox_query(dkey, q.l, q.n_boxes, q.m, False, *[lp.to_device(v) for v in parts]))
        assert (res == exp).all()
