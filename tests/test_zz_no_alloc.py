"""The allocation-free forward pass (ms_mlp_forward_noalloc) against the
allocating entry point it shares its kernels with (ms_mlp_forward), through
the C ABI: two calls in a row, the second with a smaller batch, bitwise
equal (same kernels, same launch shapes); sizes beyond the scratch limit
are rejected before any work."""
import ctypes as C

import numpy as np
import pytest

from tests.gpu_util import device, say

pytestmark = pytest.mark.gpu


def _params(rng, i, w, o):
    return {"W0": rng.standard_normal((w, i)) / np.sqrt(i), "b0": 0.1 * rng.standard_normal(w),
            "W1": rng.standard_normal((w, w)) / np.sqrt(w), "b1": 0.1 * rng.standard_normal(w),
            "W2": rng.standard_normal((o, w)) / np.sqrt(w), "b2": 0.1 * rng.standard_normal(o)}


def test_forward_noalloc_matches_allocating_forward():
    import torch
    from paper_2508_13386_amd import ms
    dev = device()
    rng = np.random.default_rng(11)
    i, w, o = 96, 256, 48
    params = _params(rng, i, w, o)
    flat = ms.mlp_pack(params)
    Pd = torch.from_numpy(flat).cuda()
    for n in (300, 7):  # the second call is smaller and reuses the scratch
        Z = rng.standard_normal((n, i)).astype(np.float32)
        ref = ms.ms_mlp_forward(dev, params, Z)
        Zd = torch.from_numpy(Z).cuda()
        Yd = torch.full((n, o), float("nan"), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        ms.ms_mlp_forward_noalloc(dev, (i, w, o), Pd, Zd, Yd)
        dev.stream.synchronize()
        Y = Yd.cpu().numpy()
        say("noalloc forward n", n, "max |diff|", float(np.abs(Y - ref).max()))
        assert np.array_equal(Y, ref)
    # 4 n width above the scratch: rejected before anything is launched
    n_big = ms.MLP_NOALLOC_SCRATCH_FLOATS // (4 * w) + 1
    code = ms.lib().ms_mlp_forward_noalloc(C.byref(dev.desc), i, w, o, C.c_void_p(Pd.data_ptr()), n_big,
                                           C.c_void_p(Zd.data_ptr()), C.c_void_p(Yd.data_ptr()))
    assert code == ms.MS_E_ARG
