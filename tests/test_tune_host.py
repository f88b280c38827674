"""Launch-shape table logic on the host: row lookup by job count, the
environment override, validation, and the JSON cache (no kernel launches)."""
import json

import pytest

import paper_2407_19871_amd as lp

ROWS = [{"jobs": 64, "br_waves": 1, "ks_tile": 4, "ks_split": 8},
        {"jobs": 1024, "br_waves": 3, "ks_tile": 16, "ks_split": 1}]


@pytest.fixture(autouse=True)
def clean_table(monkeypatch):
    for v in ("LOCPIR_BR_WAVES", "LOCPIR_KS_TILE", "LOCPIR_KS_SPLIT"):
        monkeypatch.delenv(v, raising=False)
    lp.set_tune_table([])
    yield
    lp.set_tune_table([])


def test_defaults_without_table():
    assert lp.tune_table() == []
    assert [lp.tune_pick(j)["br_waves"] for j in (1, 128, 129, 256, 257, 768, 769, 1024, 1025, 1280, 1281)] == \
        [6, 6, 7, 7, 5, 5, 2, 2, 2, 2, 1]
    assert [lp.tune_pick(j)["ks_tile"] for j in (1, 16, 256, 4096)] == [1, 4, 8, 8]
    # the default split grows until the key switch has >= 65536 blocks
    assert lp.tune_pick(1)["ks_split"] == 16
    assert lp.tune_pick(16384)["ks_split"] == 4


def test_row_lookup_first_bound_not_below_count():
    lp.set_tune_table(list(reversed(ROWS)))  # the library sorts
    assert [r["jobs"] for r in lp.tune_table()] == [64, 1024]
    got = [lp.tune_pick(j) for j in (1, 64, 65, 1024, 5000)]
    assert [g["br_waves"] for g in got] == [1, 1, 3, 3, 3]
    assert [g["ks_tile"] for g in got] == [4, 4, 16, 16, 16]
    assert [g["ks_split"] for g in got] == [8, 8, 1, 1, 1]


def test_environment_overrides_table(monkeypatch):
    lp.set_tune_table(ROWS)
    monkeypatch.setenv("LOCPIR_BR_WAVES", "1")
    monkeypatch.setenv("LOCPIR_KS_TILE", "8")
    g = lp.tune_pick(1024)
    assert g["br_waves"] == 1 and g["ks_tile"] == 8
    # the row's split belongs to tile 16, so tile 8 takes the default rule
    assert g["ks_split"] == lp.tune_pick(1024, 630)["ks_split"]
    monkeypatch.setenv("LOCPIR_BR_WAVES", "8")  # invalid values are ignored
    assert lp.tune_pick(1024)["br_waves"] == 3


def test_split_shapes_apply_up_to_their_widths(monkeypatch):
    """A row of split rotations serves launches of at most 128 jobs (6) or
    256 (7, two workgroups per CU); a wider launch that looks it up (the last
    row, or the environment) takes 7 where that fits, else four waves two
    per CU (5)."""
    lp.set_tune_table([{"jobs": 32, "br_waves": 1, "ks_tile": 4, "ks_split": 8},
                       {"jobs": 200, "br_waves": 6, "ks_tile": 8, "ks_split": 8}])
    got = [lp.tune_pick(j)["br_waves"] for j in (32, 33, 128, 129, 200, 5000)]
    assert got == [1, 6, 6, 7, 7, 5]
    monkeypatch.setenv("LOCPIR_BR_WAVES", "6")
    assert [lp.tune_pick(j)["br_waves"] for j in (1, 128, 129, 256, 257)] == [6, 6, 7, 7, 5]
    monkeypatch.setenv("LOCPIR_BR_WAVES", "7")
    assert [lp.tune_pick(j)["br_waves"] for j in (1, 256, 257)] == [7, 7, 5]


@pytest.mark.parametrize("bad", [
    {"jobs": 0, "br_waves": 1, "ks_tile": 4, "ks_split": 1},
    {"jobs": 8, "br_waves": 8, "ks_tile": 4, "ks_split": 1},
    {"jobs": 8, "br_waves": 0, "ks_tile": 4, "ks_split": 1},
    {"jobs": 8, "br_waves": 1, "ks_tile": 3, "ks_split": 1},
    {"jobs": 8, "br_waves": 1, "ks_tile": 4, "ks_split": 32},
    {"jobs": (1 << 22) + 1, "br_waves": 1, "ks_tile": 4, "ks_split": 1},
])
def test_invalid_rows_rejected(bad):
    lp.set_tune_table(ROWS)
    with pytest.raises(lp.LocpirError):
        lp.set_tune_table([bad])
    assert [r["jobs"] for r in lp.tune_table()] == [64, 1024]  # unchanged


def test_duplicate_bounds_rejected():
    with pytest.raises(lp.LocpirError):
        lp.set_tune_table([ROWS[0], dict(ROWS[0])])


def test_json_cache_round_trip(tmp_path):
    path = str(tmp_path / "tune.json")
    lp.set_tune_table(ROWS)
    lp.save_tune(path, device_name="devA")
    lp.set_tune_table([])
    assert not lp.load_tune(path, device_name="devB")  # other device
    assert lp.tune_table() == []
    assert lp.load_tune(path, device_name="devA")
    assert [(r["jobs"], r["br_waves"]) for r in lp.tune_table()] == [(64, 1), (1024, 3)]
    doc = json.load(open(path))
    doc["kernels"] = "0" * 16  # written for other kernel sources
    json.dump(doc, open(path, "w"))
    lp.set_tune_table([])
    assert not lp.load_tune(path, device_name="devA")
    assert not lp.load_tune(str(tmp_path / "missing.json"))
