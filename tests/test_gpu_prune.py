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


def test_compact_by_mask_and_merge_match_oracle():
    torch = torch_()
    g = groups(20011, 3)
    rng = np.random.default_rng(11)
    keep = (rng.uniform(size=20011) < 0.37).astype(np.int32)
    dev = [{k: torch.from_numpy(v).cuda() for k, v in d.items()} for d in g]
    m, p, ea, es = gsr.compact(dev[0], torch.from_numpy(keep).cuda(), dev[1], dev[2])
    torch.cuda.synchronize()
    m_ref, ref = oracle.compact(g, keep)
    assert m == m_ref
    for got, want in zip((p, ea, es), ref):
        for k in WIDTH:
            np.testing.assert_array_equal(got[k].cpu().numpy(), want[k])
    # merge: a second sub-map overlapping the first
    sub = {k: v.copy() for k, v in g[1].items()}
    sub["means"] = np.concatenate([g[0]["means"][:5000] + rng.normal(0, 0.004, (5000, 3)),
                                   rng.uniform(-1, 1, (15011, 3))]).astype(np.float32)
    glob = {k: v.copy() for k, v in g[0].items()}
    glob["means"] = (glob["means"] * 0.5).astype(np.float32)
    merged = gsr.merge_submap({k: torch.from_numpy(v).cuda() for k, v in glob.items()},
                              {k: torch.from_numpy(v).cuda() for k, v in sub.items()}, rho=0.01)
    torch.cuda.synchronize()
    ref = oracle.merge_submap(glob, sub, rho=0.01)
    for k in WIDTH:
        np.testing.assert_array_equal(merged[k].cpu().numpy(), ref[k])
    assert len(glob["means"]) < len(ref["means"]) < len(glob["means"]) + len(sub["means"])


def test_submap_trigger_matches_oracle():
    # a host computation in the library (no kernel), checked on random pose pairs
    rng = np.random.default_rng(4)
    hits = 0
    for _ in range(400):
        qa, qb = rng.normal(size=4), rng.normal(size=4)
        qb = qa + rng.normal(0, 0.3, 4)
        a = np.concatenate([qa, rng.normal(0, 0.5, 3)]).astype(np.float32)
        b = np.concatenate([qb, a[4:] + rng.normal(0, 0.3, 3)]).astype(np.float32)
        got = gsr.submap_trigger(a, b, 0.5, 50.0)
        assert got == oracle.submap_trigger(a.astype(np.float64), b.astype(np.float64), 0.5, np.deg2rad(50.0))
        hits += got
    assert 0 < hits < 400
