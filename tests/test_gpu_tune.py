"""Autotuner on the GPU: it returns valid rows for every bucket, installs
them, and the launches that then use the tuned shapes stay bit-exact with
the oracle."""
import numpy as np
import pytest

import oracle as O
import paper_2407_19871_amd as lp
from paper_2407_19871_amd import workloads as W

from gpu_common import as_u32, bits_of, cuda_or_skip, device_key_from_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dkey(okeys):
    cuda_or_skip()
    return device_key_from_oracle(okeys)


@pytest.fixture
def clean_table():
    lp.set_tune_table([])
    yield
    lp.set_tune_table([])


def test_autotune_rows_and_parity(okeys, octx, dkey, clean_table):
    buckets = (1, 48, 300)
    rows = lp.autotune(dkey, buckets=buckets, br_steps=8)
    assert [r["jobs"] for r in rows] == list(buckets)
    for r in rows:
        assert r["br_waves"] in (1, 2, 3, 4, 5, 6, 7) and r["ks_tile"] in (1, 4, 8, 16) and r["ks_split"] in (1, 2, 4, 8, 16)
        assert r["br_us"] > 0 and r["ks_us"] > 0
    assert lp.tune_table() == rows
    for B in (1, 48, 300):
        pick = lp.tune_pick(B)
        row = next(r for r in rows if r["jobs"] >= B)
        assert (pick["br_waves"], pick["ks_tile"]) == (row["br_waves"], row["ks_tile"])
    B = 48
    a, b = W.random_bits(71, B), W.random_bits(72, B)
    c1, c2 = O.encrypt_bits(okeys, a, seed=73), O.encrypt_bits(okeys, b, seed=74)
    got = as_u32(lp.bootstrap_batch(dkey, "NAND", lp.to_device(c1), lp.to_device(c2)))
    exp, _ = octx.gate_batch("NAND", c1, c2)
    assert (got == exp).all()
    assert (bits_of(okeys, got)[0] == 1 - (a & b)).all()


def test_autotune_rejects_bad_arguments(dkey, clean_table):
    for buckets, steps in (((0,), 8), ((1 << 17,), 8), ((4, 4), 8), ((4,), 0), ((4,), 10_000)):
        with pytest.raises(lp.LocpirError):
            lp.autotune(dkey, buckets=buckets, br_steps=steps)
    assert lp.tune_table() == []
