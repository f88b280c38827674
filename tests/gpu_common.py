"""Shared helpers of the GPU parity tests (oracle keys imported into the
product library, so both sides use identical key material)."""
import numpy as np
import pytest

import oracle as O
import paper_2407_19871_amd as lp


def cuda_or_skip():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def device_key_from_oracle(okeys):
    p = lp.params_default()
    ck = lp.CloudKey.from_arrays(p, okeys.bsk, okeys.ksk)
    return lp.DeviceKey(ck)


def sync():
    import torch
    torch.cuda.synchronize()


def as_u32(t):
    return lp.to_host(t)


def bits_of(okeys, ct):
    d, ph = O.decrypt_bits(okeys, np.asarray(ct, np.uint32))
    return d, ph
