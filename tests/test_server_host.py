"""Query-server host logic on the CPU (simulate mode: same admission and
scheduling, no GPU): budget-bound admission never drops or corrupts
requests, over-budget and malformed requests are refused, one failing
request does not disturb the others, cancellation ends a request."""
import time

import numpy as np
import pytest

import paper_2407_19871_amd as lp


@pytest.fixture(scope="module")
def ck():
    p = lp.params_default()
    # key contents do not matter in simulate mode; sizes do
    return lp.CloudKey.from_arrays(p, np.zeros(lp.bsk_words(p), np.uint32), np.zeros(lp.ksk_words(p), np.uint32))


def query(l, nb, m):
    w = 631
    return (l, nb, m, True, np.zeros((l, w), np.uint32), np.zeros((l, w), np.uint32),
            np.zeros((4 * l * nb, w), np.uint32), np.zeros((nb * m, w), np.uint32))


def test_budget_queues_requests_and_completes_all(ck):
    probe = lp.Server(1 << 40, simulate=True)
    one = probe.request_bytes(ck, *query(16, 2, 4))
    probe.close()
    srv = lp.Server(int(one * 2.5), simulate=True)
    tickets = [srv.submit(ck, *query(16, 2, 4)) for _ in range(7)]
    for t in tickets:
        st, out, lat = srv.poll(t, wait=True)
        assert st == 0 and out.shape == (4, 631) and lat >= 0
    s = srv.stats()
    assert s["completed"] == 7 and s["failed"] == 0 and s["admitted"] == 7
    assert s["peak_bytes"] <= int(one * 2.5)       # never more than two admitted together
    assert s["peak_bytes"] >= one
    assert s["bytes_in_use"] == 0
    srv.close()


def test_max_inflight_limits_admission(ck):
    srv = lp.Server(1 << 40, max_inflight=1, simulate=True)
    one = srv.request_bytes(ck, *query(8, 1, 2))
    tickets = [srv.submit(ck, *query(8, 1, 2)) for _ in range(4)]
    for t in tickets:
        assert srv.poll(t)[0] == 0
    assert srv.stats()["peak_bytes"] == one
    srv.close()


def test_over_budget_and_malformed_requests_are_refused(ck):
    srv = lp.Server(1 << 20, simulate=True)
    with pytest.raises(lp.LocpirError) as e:
        srv.submit(ck, *query(16, 2, 4))
    assert e.value.code == -5
    srv.close()
    srv = lp.Server(1 << 40, simulate=True)
    for bad in (query(0, 1, 1), query(16, 0, 1), query(16, 1, 0), query(65, 1, 1)):
        with pytest.raises(lp.LocpirError) as e:
            srv.submit(ck, *bad)
        assert e.value.code == -1
    srv.close()


def test_failing_request_does_not_disturb_others(ck):
    srv = lp.Server(1 << 40, simulate=True, fail_ticket=3)
    tickets = [srv.submit(ck, *query(8, 1, 2)) for _ in range(5)]
    res = {t: srv.poll(t)[0] for t in tickets}
    assert res[3] == -2                      # LP_ENOMEM from the injected failure
    assert all(res[t] == 0 for t in tickets if t != 3)
    s = srv.stats()
    assert s["failed"] == 1 and s["completed"] == 4 and s["bytes_in_use"] == 0
    srv.close()


def test_cancel_queued_request(ck):
    probe = lp.Server(1 << 40, simulate=True)
    one = probe.request_bytes(ck, *query(32, 8, 8))
    probe.close()
    srv = lp.Server(one, simulate=True)      # one request at a time
    t1 = srv.submit(ck, *query(32, 8, 8))
    t2 = srv.submit(ck, *query(32, 8, 8))
    srv.cancel(t2)
    assert srv.poll(t1)[0] == 0
    assert srv.poll(t2)[0] == lp.LP_ECANCELED
    s = srv.stats()
    assert s["cancelled"] == 1 and s["bytes_in_use"] == 0
    srv.close()


def test_continuous_batching_fuses_levels(ck):
    # two requests submitted together share ticks: fewer ticks than the sum
    # of their depths
    srv = lp.Server(1 << 40, simulate=True)
    _, _, depth = lp.bbox_counts(16, 4, 8)
    ts = [srv.submit(ck, *query(16, 4, 8)) for _ in range(2)]
    for t in ts:
        assert srv.poll(t)[0] == 0
    assert srv.stats()["ticks"] < 2 * depth
    srv.close()


def test_mixed_parameter_sets_run_in_separate_launches(ck):
    # a lambda 80 request (541-word samples) never shares a fused launch with
    # a lambda 128 one (631 words): each tick counts one launch pair per shape
    p80 = lp.params_lambda80()
    ck80 = lp.CloudKey.from_arrays(p80, np.zeros(lp.bsk_words(p80), np.uint32), np.zeros(lp.ksk_words(p80), np.uint32))
    l, nb, m = 8, 2, 3
    q80 = (l, nb, m, True, np.zeros((l, 541), np.uint32), np.zeros((l, 541), np.uint32),
           np.zeros((4 * l * nb, 541), np.uint32), np.zeros((nb * m, 541), np.uint32))
    srv = lp.Server(1 << 40, simulate=True)
    t = [srv.submit(ck, *query(l, nb, m)), srv.submit(ck80, *q80)]
    r = [srv.poll(x) for x in t]
    assert r[0][0] == 0 and r[0][1].shape == (m, 631)
    assert r[1][0] == 0 and r[1][1].shape == (m, 541)
    depth = lp.bbox_counts(l, nb, m)[2]
    s = srv.stats()
    assert s["ticks"] == 2 * depth and s["completed"] == 2 and s["bytes_in_use"] == 0
    srv.close()


def _late_widths(monkeypatch, l, nb, m):
    monkeypatch.setenv("LOCPIR_XNOR_EARLY", "0")  # the server's placement
    return lp.bbox_level_widths(l, nb, m)


@pytest.mark.parametrize("cap", [1, 7, 40])
def test_tick_cap_bounds_every_launch(monkeypatch, ck, cap):
    """A lone 16-box request under a rotation cap: no tick holds more than
    the cap (a MUX's two rotations stay together, so a cap of 1 still runs
    one gate), every level is split into enough ticks, and the request
    completes."""
    widths = _late_widths(monkeypatch, 16, 16, 8)
    srv = lp.Server(1 << 40, simulate=True, max_tick_rotations=cap)
    t = srv.submit(ck, *query(16, 16, 8))
    assert srv.poll(t)[0] == 0
    s = srv.stats()
    srv.close()
    assert s["widest_tick"] <= max(cap, 2)
    assert s["ticks"] >= sum(-(-w // max(cap, 2)) for w in widths)
    assert s["fused_bootstraps"] == sum(widths)
    assert s["completed"] == 1 and s["bytes_in_use"] == 0


def test_without_cap_a_tick_runs_whole_levels(monkeypatch, ck):
    widths = _late_widths(monkeypatch, 16, 4, 8)
    srv = lp.Server(1 << 40, simulate=True)
    assert srv.poll(srv.submit(ck, *query(16, 4, 8)))[0] == 0
    s = srv.stats()
    srv.close()
    assert s["ticks"] == len(widths) and s["widest_tick"] == max(widths)


def test_tick_cap_lets_narrow_requests_finish_first(monkeypatch, ck):
    """A one-box request beside a 64-box one under a cap of twice its widest
    level: its levels fit its share, so it finishes before the wide one,
    whose levels take several ticks each."""
    small = _late_widths(monkeypatch, 16, 1, 4)
    big = _late_widths(monkeypatch, 16, 64, 4)
    cap = 2 * max(small)
    srv = lp.Server(1 << 40, simulate=True, max_tick_rotations=cap)
    tb = srv.submit(ck, *query(16, 64, 4))
    ts = srv.submit(ck, *query(16, 1, 4))
    st_s, _, lat_s = srv.poll(ts, wait=True)
    st_b, _, lat_b = srv.poll(tb, wait=True)
    s = srv.stats()
    srv.close()
    assert st_s == 0 and st_b == 0
    assert s["widest_tick"] <= cap
    assert s["fused_bootstraps"] == sum(small) + sum(big)
    assert lat_s < lat_b
    assert s["ticks"] >= sum(-(-w // cap) for w in big)


TIMED_ROWS = [{"jobs": 128, "br_waves": 6, "ks_tile": 4, "ks_split": 16, "br_us": 94.9},
              {"jobs": 1024, "br_waves": 2, "ks_tile": 8, "ks_split": 16, "br_us": 34.6},
              {"jobs": 2048, "br_waves": 1, "ks_tile": 8, "ks_split": 16, "br_us": 27.0},
              {"jobs": 4096, "br_waves": 1, "ks_tile": 8, "ks_split": 16, "br_us": 25.5},
              {"jobs": 16384, "br_waves": 1, "ks_tile": 8, "ks_split": 16, "br_us": 24.1}]


UNTIMED_ROWS = [{k: v for k, v in r.items() if k != "br_us"} for r in TIMED_ROWS]


@pytest.mark.parametrize("rows,cap", [(None, 2048), (UNTIMED_ROWS, 2048), (TIMED_ROWS, 2048), (TIMED_ROWS[:2], 1024)])
def test_automatic_tick_cap(monkeypatch, ck, rows, cap):
    """LP_TICK_CAP_AUTO: the narrowest timed width within 15 % of the best
    rotation time per job (2048 for the measured MI355X table: 27.0 us
    against 24.1; 1024 when the table stops there), 2048 without a table or
    with rows installed untimed; a 256-box request's widest levels are split
    to it."""
    widths = _late_widths(monkeypatch, 16, 256, 4)
    assert max(widths) > 2048
    old = lp.tune_table()
    lp.set_tune_table(rows or [])
    try:
        srv = lp.Server(1 << 40, simulate=True, max_tick_rotations="auto")
        assert srv.poll(srv.submit(ck, *query(16, 256, 4)))[0] == 0
        s = srv.stats()
        srv.close()
    finally:
        lp.set_tune_table(old)
    assert s["widest_tick"] == cap
    assert s["fused_bootstraps"] == sum(widths)


def test_submit_blob_deserializes_and_owns_the_key(ck):
    """The request as the client sends it (Sec. 3: PK uploaded as a blob):
    the server deserializes the blob itself, the caller's bytes may go away
    at once, and a foreign or truncated blob is refused without queueing."""
    blob = ck.serialize()
    srv = lp.Server(1 << 40, simulate=True)
    t1 = srv.submit_blob(bytes(blob), *query(16, 2, 3))
    t2 = srv.submit(ck, *query(8, 1, 2))
    del blob
    st, out, lat = srv.poll(t1)
    assert st == 0 and out.shape == (3, 631) and lat >= 0
    assert srv.poll(t2)[0] == 0
    good = ck.serialize()
    with pytest.raises(lp.LocpirError) as e:
        srv.submit_blob(good[:-4], *query(8, 1, 2))       # truncated
    assert e.value.code == -1
    bad = bytearray(good)
    bad[:4] = b"XXXX"                                    # foreign magic
    with pytest.raises(lp.LocpirError):
        srv.submit_blob(bytes(bad), *query(8, 1, 2))
    s = srv.stats()
    assert s["submitted"] == 2 and s["completed"] == 2 and s["bytes_in_use"] == 0
    srv.close()
