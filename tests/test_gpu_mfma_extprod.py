"""The int8 matrix-core external product of one blind-rotation step
(lp_debug_external_product_mfma) equals the oracle's external product
(Sec. 2.2, Bootstrap: ExtProd(BSK_i, D), gadget digits times key rows in
Z[X]/(X^1024 + 1) mod 2^32) bit for bit: random accumulator differences at
ragged batch sizes around the 64-column tile, adversarial inputs (all digits
at their extremes), and a key step whose words sit at the limb boundaries
(0x80000000, 0x7FFFFFFF, 0xFFFFFFFF, 0x00000080, ...)."""
import numpy as np
import pytest

import oracle as O
import paper_2407_19871_amd as lp

from gpu_common import as_u32, cuda_or_skip

pytestmark = pytest.mark.gpu


def _key_step(okeys, i):
    P = okeys.params
    return np.ascontiguousarray(okeys.bsk.reshape(P.n, 2 * P.l, 2, P.N)[i])


def _check(octx, key_step, i, d):
    torch = cuda_or_skip()
    got = as_u32(lp.debug_external_product_mfma(lp.to_device(key_step), lp.to_device(d)))
    exp = np.stack([octx.external_product(i, d[b]) for b in range(d.shape[0])])
    assert got.shape == exp.shape
    bad = np.argwhere(got != exp)
    assert bad.size == 0, f"{len(bad)} words differ, first at {bad[:3].tolist()}"


@pytest.mark.parametrize("cnt", [1, 37, 64, 128, 200])
def test_mfma_extprod_random(okeys, octx, cnt):
    cuda_or_skip()
    i = 17
    d = np.random.default_rng(800 + cnt).integers(0, 2**32, size=(cnt, 2048), dtype=np.uint64).astype(np.uint32)
    _check(octx, _key_step(okeys, i), i, d)


def test_mfma_extprod_extreme_digits(okeys, octx):
    """Inputs whose digits are all -64, all +63, or alternate between them."""
    cuda_or_skip()
    i = 629
    lo = np.uint32((0x00000000 - 0x81020400) & 0xFFFFFFFF)   # every digit -64
    hi = np.uint32((0xFFFFFFFF - 0x81020400) & 0xFFFFFFFF)   # every digit +63
    rows = [np.full(2048, lo), np.full(2048, hi), np.where(np.arange(2048) % 2 == 0, lo, hi).astype(np.uint32),
            np.zeros(2048, np.uint32), np.full(2048, 0xFFFFFFFF, np.uint32)]
    _check(octx, _key_step(okeys, i), i, np.stack(rows).astype(np.uint32))


def test_mfma_extprod_boundary_key_words(okeys):
    """A key step made of words at the byte-limb boundaries, in an oracle
    context built on that key (the rows of every other step are the real
    ones)."""
    cuda_or_skip()
    P = okeys.params
    i = 3
    words = np.array([0x80000000, 0x7FFFFFFF, 0xFFFFFFFF, 0x00000080, 0x0000007F, 0x80808080, 0x7F7F7F7F,
                      0xFF80FF80, 0x00000000, 0x00000001], np.uint32)
    bsk = okeys.bsk.copy().reshape(P.n, 2 * P.l, 2, P.N)
    bsk[i] = words[np.random.default_rng(5).integers(0, len(words), size=bsk[i].shape)]
    keys = O.Keys(P, okeys.seed, okeys.s_lwe, okeys.s_ring, np.ascontiguousarray(bsk.reshape(-1)), okeys.ksk)
    ctx = O.Ctx(keys)
    d = np.random.default_rng(6).integers(0, 2**32, size=(40, 2048), dtype=np.uint64).astype(np.uint32)
    d[0] = np.uint32((0xFFFFFFFF - 0x81020400) & 0xFFFFFFFF)
    _check(ctx, np.ascontiguousarray(bsk[i]), i, d)
