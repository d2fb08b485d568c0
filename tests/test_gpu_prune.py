"""Opacity pruning on the HIP path vs the oracle's definition: index work, so
the kept rows must match bit for bit (the keep decision is taken in binary32 on
both sides)."""
import numpy as np
import pytest

import oracle
from paper_2312_10070_amd import gsr

pytestmark = pytest.mark.gpu

WIDTH = {"means": 3, "scales": 3, "quats": 4, "opacities": 1, "colors": 3}


def torch_():
    import torch
    return torch


def groups(n, seed):
    rng = np.random.default_rng(seed)
    g = []
    for _ in range(3):
        d = {k: rng.normal(size=(n, w) if w > 1 else (n,)).astype(np.float32) for k, w in WIDTH.items()}
        g.append(d)
    o = rng.uniform(0, 1, n).astype(np.float32)
    o[::97] = np.float32(0.1)  # exactly at the threshold: kept
    if n > 5:
        o[5] = np.nan  # removed
    g[0]["opacities"] = o
    return g


@pytest.mark.parametrize("n,thre", [(0, 0.1), (1, 0.1), (3001, 0.1), (500_000, 0.5), (4099, 2.0), (4099, -1.0)])
def test_prune_matches_oracle(n, thre):
    torch = torch_()
    g = groups(n, n)
    m_ref, ref = oracle.prune(g, thre)
    dev = [{k: torch.from_numpy(v).cuda() for k, v in d.items()} for d in g]
    m, p, ea, es = gsr.prune(dev[0], thre, dev[1], dev[2])
    torch.cuda.synchronize()
    assert m == m_ref
    for got, want in zip((p, ea, es), ref):
        for k in WIDTH:
            np.testing.assert_array_equal(got[k].cpu().numpy(), want[k])


def test_prune_without_moments_and_bad_arguments():
    import ctypes
    torch = torch_()
    g = groups(1000, 7)
    dev = {k: torch.from_numpy(v).cuda() for k, v in g[0].items()}
    m, p, ea, es = gsr.prune(dev, 0.3)
    m_ref, (ref,) = oracle.prune(g[:1], 0.3)
    assert m == m_ref and ea is None and es is None
    for k in WIDTH:
        np.testing.assert_array_equal(p[k].cpu().numpy(), ref[k])
    ctx = gsr.Context.get(0)
    ins = (ctypes.c_void_p * 15)()
    outs = (ctypes.c_void_p * 15)()
    kept = ctypes.c_int64()
    for i, k in enumerate(gsr.PARAM_GROUPS):
        ins[i] = dev[k].data_ptr()
    # an output missing where its input is given
    assert ctx.lib.gsr_prune(ctx.h, 1000, 0.3, ins, outs, ctypes.byref(kept)) == gsr.GSR_EINVAL
    assert ctx.lib.gsr_prune(ctx.h, -1, 0.3, ins, outs, ctypes.byref(kept)) == gsr.GSR_EINVAL
    assert ctx.lib.gsr_prune(ctx.h, 1000, float("nan"), ins, outs, ctypes.byref(kept)) == gsr.GSR_EINVAL
