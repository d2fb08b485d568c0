"""gsr_loss_track_noalloc (the tracking loss of Eq. 15 with its scratch in a
static device array, for callers that cannot allocate) against the
allocating gsr_loss_track and the oracle: two calls in a row, the second on
a smaller frame, so the second starts from the first call's leftover
histograms and tickets; an empty frame; argument errors."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2312_10070_amd import gsr

pytestmark = pytest.mark.gpu


def frame(seed, h, w):
    """A rendered-like frame and an observation with 20 % invalid depths and
    depths rounded to 1 mm (exact ties around the median)."""
    rng = np.random.default_rng(seed)
    C = rng.uniform(0, 1, (3, h, w)).astype(np.float32)
    D = rng.uniform(1, 5, (h, w)).astype(np.float32)
    A = rng.uniform(0, 1, (h, w)).astype(np.float32)
    Ct = np.clip(C + rng.normal(0, 0.05, C.shape), 0, 1).astype(np.float32)
    Dt = (np.round((D + rng.normal(0, 0.02, D.shape)) * 1000.0) / 1000.0).astype(np.float32)
    Dt[rng.uniform(size=Dt.shape) < 0.2] = 0.0
    return C, D, A, Ct, Dt


def run_noalloc(arrs, lambda_c=0.5, inlier_mult=50.0):
    import torch
    C, D, A, Ct, Dt = (torch.from_numpy(a).cuda() for a in arrs)
    loss = torch.full((1,), -7.0, device="cuda")
    med = torch.full((1,), -7.0, device="cuda")
    gC = torch.full_like(C, -7.0)
    gD = torch.full_like(D, -7.0)
    gsr.loss_track_noalloc(C, D, A, Ct, Dt, loss, gC, gD, med, lambda_c, inlier_mult)
    torch.cuda.synchronize()
    return loss.cpu().numpy(), gC.cpu().numpy(), gD.cpu().numpy(), med.cpu().numpy()


def run_alloc(arrs, lambda_c=0.5, inlier_mult=50.0):
    import torch
    C, D, A, Ct, Dt = (torch.from_numpy(a).cuda() for a in arrs)
    loss, gC, gD, med = gsr.loss_track(C, D, A, Ct, Dt, lambda_c, inlier_mult)
    torch.cuda.synchronize()
    return loss.cpu().numpy(), gC.cpu().numpy(), gD.cpu().numpy(), med.cpu().numpy()


def test_noalloc_matches_loss_track_twice_second_smaller():
    for seed, (h, w) in ((0, (480, 640)), (1, (120, 160))):
        arrs = frame(seed, h, w)
        got = run_noalloc(arrs)
        ref = run_alloc(arrs)
        # the same kernels and the same fixed-order reduction: bit for bit
        for a, b in zip(got, ref):
            np.testing.assert_array_equal(a, b)
        r = oracle.loss_track(*arrs, 0.5, 50.0)
        assert got[3][0] == r["median"]
        assert abs(got[0][0] - r["loss"]) <= 1e-5 * abs(r["loss"])
        np.testing.assert_allclose(got[1], r["gC"], rtol=1e-5, atol=1e-9)
        np.testing.assert_allclose(got[2], r["gD"], rtol=1e-5, atol=1e-9)


def test_noalloc_empty_frame_and_bad_arguments():
    import torch
    loss = torch.full((1,), -7.0, device="cuda")
    e = torch.empty(0, device="cuda")
    gsr.loss_track_noalloc(e, e, e, e, e, loss, e, e)
    torch.cuda.synchronize()
    assert loss.item() == 0.0
    lib = gsr.load()
    P = ctypes.c_void_p
    buf = torch.zeros(16, device="cuda")
    p = P(buf.data_ptr())
    stream = P(torch.cuda.current_stream().cuda_stream)
    # NULL loss and an oversized frame are refused on the host before any launch
    rc = lib.gsr_loss_track_noalloc(stream, p, p, p, p, p, 4, 0.5, 50.0, None, p, p, None)
    assert rc == gsr.GSR_EINVAL
    rc = lib.gsr_loss_track_noalloc(stream, p, p, p, p, p, 1 << 32, 0.5, 50.0, p, p, p, None)
    assert rc == gsr.GSR_EINVAL
    assert b"GSR_NOALLOC_MAX_PIXELS" in lib.gsr_last_error(None)
