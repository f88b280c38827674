"""The gate-batch entry point that allocates nothing
(lp_bootstrap_batch_noalloc): its outputs equal lp_bootstrap_batch's bit for
bit on consecutive calls that reuse the static scratch, each smaller than the
one before (a wide MUX batch, a split-rotation MUX batch at the split
maximum, a small NAND batch), and sizes above its maximum are refused."""
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


def _inputs(okeys, gate, B, seed):
    k = 3 if gate == "MUX" else 2
    bits = [W.random_bits(seed + i, B) for i in range(k)]
    cts = [O.encrypt_bits(okeys, v, seed=seed + 10 + i) for i, v in enumerate(bits)]
    return bits, cts


@pytest.mark.parametrize("gate,B", [("MUX", 300), ("MUX", 64), ("NAND", 45)])
def test_noalloc_equals_allocating_call(okeys, dkey, gate, B):
    torch = cuda_or_skip()
    bits, cts = _inputs(okeys, gate, B, 7000 + B)
    dev = [lp.to_device(c) for c in cts]
    exp = as_u32(lp.bootstrap_batch(dkey, gate, *dev))
    out = torch.empty((B, dkey.params.n + 1), dtype=torch.int32, device=dev[0].device)
    got = as_u32(lp.bootstrap_batch_noalloc(dkey, gate, *dev, out=out))
    assert (got == exp).all()
    # and the call again, now that the scratch holds this call's contents
    got2 = as_u32(lp.bootstrap_batch_noalloc(dkey, gate, *dev))
    assert (got2 == exp).all()
    d, _ = bits_of(okeys, got)
    if gate == "MUX":
        assert (d == np.where(bits[0] == 1, bits[1], bits[2])).all()
    else:
        assert (d == 1 - (bits[0] & bits[1])).all()


def test_noalloc_matches_oracle_after_larger_call(okeys, octx, dkey):
    """A wide call, then a smaller split-rotation call: the second equals the
    oracle's gates bit for bit (no state from the first leaks into it)."""
    _, big = _inputs(okeys, "MUX", 500, 7100)
    lp.bootstrap_batch_noalloc(dkey, "MUX", *[lp.to_device(c) for c in big])
    _, small = _inputs(okeys, "XNOR", 21, 7200)
    got = as_u32(lp.bootstrap_batch_noalloc(dkey, "XNOR", *[lp.to_device(c) for c in small]))
    exp, _ = octx.gate_batch("XNOR", *small)
    assert (got == exp).all()


def test_noalloc_refuses_batches_above_its_maximum(okeys, dkey):
    _, cts = _inputs(okeys, "NAND", 1025, 7300)
    dev = [lp.to_device(c) for c in cts]
    with pytest.raises(lp.LocpirError, match="1024"):
        lp.bootstrap_batch_noalloc(dkey, "NAND", *dev)
