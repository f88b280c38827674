"""Pins of the bounding-box circuit (Algorithms 2-5): brute force on
plaintext bits, the paper's worked examples, gate counts, and the encrypted
oracle against the plaintext predicate (no GPU)."""
import json
import os

import numpy as np
import pytest

import oracle as O
from oracle import plain
from paper_2407_19871_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("is_signed", [False, True])
def test_comparator_exhaustive_l8(is_signed):
    l = 8
    for a in range(256):
        ab = plain.to_bits(a, l)
        for b in range(256):
            got = plain.comp_s_bits(ab, plain.to_bits(b, l), is_signed)
            if is_signed:
                exp = int(plain.as_signed(a, l) < plain.as_signed(b, l))
            else:
                exp = int(a < b)
            assert got == exp


def test_msb_flip_on_unsigned_inputs_is_wrong_on_half_the_pairs():
    # reading of Algorithm 2 lines 2-3: with the flip the circuit orders
    # two's-complement values, so applied to unsigned codes it errs exactly
    # when the MSBs differ: 2 * 128 * 128 = 32768 of 65536 pairs
    l = 8
    wrong = sum(plain.comp_s_bits(plain.to_bits(a, l), plain.to_bits(b, l), True) != int(a < b)
                for a in range(256) for b in range(256))
    assert wrong == 32768


@pytest.mark.parametrize("l", [16, 32])
def test_comparator_random_wide(l):
    rng = np.random.default_rng(l)
    for _ in range(3000):
        a, b = (int(v) for v in rng.integers(0, 2**l, 2, dtype=np.uint64))
        if rng.random() < 0.2:
            b = a
        assert plain.comp_s_bits(plain.to_bits(a, l), plain.to_bits(b, l), True) == \
            int(plain.as_signed(a, l) < plain.as_signed(b, l))


@pytest.mark.parametrize("seed", range(30))
def test_bbox_circuit_equals_predicate(seed):
    q = W.random_query(seed, 16, 1 + seed % 9, 7, region=W.KOREA if seed % 2 else W.ZERO_STRADDLE,
                       force_inside=seed % 3 == 0)
    got = plain.bbox_circuit_bits(q.x, q.y, q.boxes, q.payloads, q.l, q.m, True)
    assert got == plain.predicate(q.x, q.y, q.boxes, q.payloads, q.l, q.m, True)


def test_guillotine_tilings_are_disjoint():
    for seed in range(20):
        q = W.random_query(seed, 16, 16, 4)
        S = lambda v: plain.as_signed(v, 16)
        for i, a in enumerate(q.boxes):
            for b in q.boxes[i + 1:]:
                overlap_x = max(S(a[0]), S(b[0])) < min(S(a[1]), S(b[1]))
                overlap_y = max(S(a[2]), S(b[2])) < min(S(a[3]), S(b[3]))
                assert not (overlap_x and overlap_y)


def test_worked_example_plaintext():
    g = json.load(open(os.path.join(GOLD, "worked_example.json")))
    b = g["box"]
    q = W.table1_query((g["x"], g["y"]), [["box", b["lat1"], b["lat2"], b["long1"], b["long2"],
                                           int(g["service_bits"], 2)]], l=16, m=3)
    x1, x2, y1, y2 = q.boxes[0]
    assert plain.comp_le_bits(plain.to_bits(x1, 16), plain.to_bits(q.x, 16), True) == 1
    assert plain.comp_s_bits(plain.to_bits(q.x, 16), plain.to_bits(x2, 16), True) == 1
    assert plain.comp_s_bits(plain.to_bits(q.y, 16), plain.to_bits(y2, 16), True) == g["expected"]["y_in_range"]
    out = plain.bbox_circuit_bits(q.x, q.y, q.boxes, q.payloads, 16, 3, True)
    assert format(out, "03b") == g["expected_service_bits"]


def test_table1_seoul_point_plaintext():
    t = json.load(open(os.path.join(GOLD, "table1_covid_boxes.json")))
    q = W.table1_query((37.55, 127.0), t["rows"], l=16, m=t["service_bits_m"])
    # the point lies in Seoul's box only (Incheon's latitude range matches, its
    # longitude range does not)
    out = plain.bbox_circuit_bits(q.x, q.y, q.boxes, q.payloads, 16, 9, True)
    assert out == 427
    assert plain.predicate(q.x, q.y, q.boxes, q.payloads, 16, 9, True) == 427


@pytest.mark.parametrize("l,N,m,br,ks,depth", [
    (8, 1, 8, 107, 75, 12),       # one 8-bit query, one box: "~110 bootstraps"
    (16, 16, 32, 4112, 3088, 24),  # 16-bit, 16 boxes, 32-bit payload: "~4k bootstraps"
    (16, 9, 9, 1908, 1332, 24),    # the paper's Table 2 shape (l = 16, N = m = 9)
    (13, 9, 9, 1584, 1116, 21),
])
def test_gate_counts(l, N, m, br, ks, depth):
    assert O.bbox_counts(l, N, m) == (br, ks, depth)


def test_comparator_costs_3l_bootstraps():
    # Sec. 6.2: l XNOR and l MUX per comparison, a MUX costing two bootstraps
    for l in (8, 13, 16, 32):
        br1, _, _ = O.bbox_counts(l, 1, 1)
        br2, _, _ = O.bbox_counts(l, 2, 1)
        per_box = br2 - br1 - 1           # one more XOR for the second box
        assert per_box == 4 * 3 * l + 3 + 1


def _encrypt_query(keys, q, seed):
    xb, yb, bb, pb = q.plain_bits()
    allb = np.concatenate([xb, yb, bb, pb])
    ct = O.encrypt_bits(keys, allb, seed=seed)
    l, N, m = q.l, q.n_boxes, q.m
    return ct[:l], ct[l:2 * l], ct[2 * l:2 * l + 4 * l * N], ct[2 * l + 4 * l * N:]


def test_worked_example_encrypted(okeys, octx):
    g = json.load(open(os.path.join(GOLD, "worked_example.json")))
    b = g["box"]
    q = W.table1_query((g["x"], g["y"]), [["box", b["lat1"], b["lat2"], b["long1"], b["long2"],
                                           int(g["service_bits"], 2)]], l=16, m=3)
    x, y, bounds, pay = _encrypt_query(okeys, q, 123)
    out = octx.bbox_query(16, 1, 3, True, x, y, bounds, pay)
    d, ph = O.decrypt_bits(okeys, out)
    assert W.from_bits(d) == 0
    assert np.abs(np.abs(ph.astype(np.int64)) - 2**29).max() < 2**28


def test_table1_two_cities_encrypted(okeys, octx):
    # Seoul and Incheon share the point's latitude range; only Seoul's box
    # holds the point
    t = json.load(open(os.path.join(GOLD, "table1_covid_boxes.json")))
    rows = [r for r in t["rows"] if r[0] in ("Seoul", "Incheon")]
    q = W.table1_query((37.55, 127.0), rows, l=16, m=9)
    x, y, bounds, pay = _encrypt_query(okeys, q, 321)
    out = octx.bbox_query(16, 2, 9, True, x, y, bounds, pay)
    d, _ = O.decrypt_bits(okeys, out)
    assert W.from_bits(d) == 427


def test_unsigned_u8_query_encrypted(okeys, octx):
    q = W.random_query_u8(1, force_inside=True)
    x, y, bounds, pay = _encrypt_query(okeys, q, 99)
    out = octx.bbox_query(8, 1, 8, False, x, y, bounds, pay)
    d, _ = O.decrypt_bits(okeys, out)
    assert W.from_bits(d) == plain.predicate(q.x, q.y, q.boxes, q.payloads, 8, 8, False) == q.payloads[0]
