"""The allocation-free grid scoring (prnu_score_grid_noalloc) through the C ABI, against
prnu_score_grid on the same inputs: two calls in a row on one context, the second on a
smaller frame and grid, then bf16 frames smaller than the fingerprint.  Both entry
points run the same kernels on the same candidates, so the scores must agree bit for bit
(stricter than the oracle bar of PCE within 1e-3 and exact shifts); the first case is
also checked against the FP64 oracle on a few candidates.
"""
import math
import sys

import numpy as np
import pytest

from oracle import prnu_oracle as O
from paper_2207_14507_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2207_14507_amd import prnu
    return prnu


def noalloc_scores(P, ctx, fp, frames, frame, opts, scales=None):
    import torch
    n = opts.full.n_scale * opts.full.n_rot
    dev = torch.device("cuda")
    pce = torch.full((n,), float("nan"), dtype=torch.float64, device=dev)
    rho = torch.full((n,), float("nan"), dtype=torch.float64, device=dev)
    dx = torch.full((n,), -12345, dtype=torch.int32, device=dev)
    dy = torch.full((n,), -12345, dtype=torch.int32, device=dev)
    if frames.dtype == np.uint16:
        ft = torch.from_numpy(frames.view(np.int16)).to(dev)
        st = torch.from_numpy(np.asarray(scales, np.float32)).to(dev)
    else:
        ft = torch.from_numpy(frames).to(dev)
        st = None
    torch.cuda.synchronize()
    P.prnu_score_grid_noalloc(ctx, fp, ft, frame, opts, pce, rho, dx, dy, scales=st)
    torch.cuda.synchronize()
    return pce.cpu().numpy(), rho.cpu().numpy(), dx.cpu().numpy(), dy.cpu().numpy()


def same(tag, a, b):
    for name, x, y in zip(("pce", "rho", "dx", "dy"), a, b):
        assert np.array_equal(x, y), (tag, name, int(np.flatnonzero(x != y)[0]))


def test_noalloc_equals_score_grid_on_two_calls_in_a_row(P):
    ctx = P.prnu_create(0)
    try:
        big = synth.walk_sequence(3, 0, 720, 1280, 1)
        small = synth.tiny(n_frames=2, config=27)
        cases = [("720p, 41x21 grid, R 64", big.K, big.frames, 0, (41, 0.85, 1.15, 21, -2.0, 2.0), 64),
                 ("256x256, 11x11 grid, R 16", small.K, small.frames, 1, (11, 0.95, 1.05, 11, -2.0, 2.0), 16)]
        for tag, K, frames, f, grid, R in cases:
            say(tag)
            fp = P.prnu_open_fingerprint(ctx, K)
            opts = P.make_opts(grid=grid, radius=R)
            ref = P.prnu_score_grid(ctx, fp, frames, f, opts)
            got = noalloc_scores(P, ctx, fp, frames, f, opts)
            same(tag, got, ref)
            if R == 64:
                cands = O.candidates(O.grid_values(*grid[:3]), O.grid_values(*grid[3:]))
                kn = O.mean_free(K)
                for i in (int(np.argmax(got[0])), 0, 430):
                    r = O.evaluate_candidate(K, frames[f], cands[i][0], cands[i][1], R, kn)
                    assert math.isclose(got[0][i], r.pce, rel_tol=1e-3), (i, got[0][i], r.pce)
                    assert (got[2][i], got[3][i]) == (r.dx, r.dy), i
            P.prnu_close_fingerprint(ctx, fp)
    finally:
        P.prnu_destroy(ctx)


def test_noalloc_bf16_frames_smaller_than_the_fingerprint(P):
    seq = synth.cropped_sequence(36, (256, 256), (216, 200), 2, radius=6)
    q = [synth.quantize_bf16(f) for f in seq.frames]
    bits = np.stack([b for b, _ in q])
    scales = np.array([s for _, s in q], np.float32)
    ctx = P.prnu_create(0)
    try:
        fp = P.prnu_open_fingerprint(ctx, seq.K)
        opts = P.make_opts(grid=(5, 0.97, 1.03, 5, -1.0, 1.0), radius=16)
        for f in range(2):
            ref = P.prnu_score_grid(ctx, fp, bits, f, opts, scales=scales)
            got = noalloc_scores(P, ctx, fp, bits, f, opts, scales)
            same(f"bf16 cropped f{f}", got, ref)
        # host frames are refused through the C ABI, nothing is queued
        import ctypes as C
        import torch
        keep = []
        fr = P.make_frames(bits, scales, keep)
        out = torch.zeros(25, dtype=torch.float64, device="cuda")
        st = P.lib.prnu_score_grid_noalloc(ctx, fp, C.byref(fr), 0, C.byref(opts), out.data_ptr(), None, None, None)
        assert st == P.PRNU_E_ARG
        P.prnu_close_fingerprint(ctx, fp)
    finally:
        P.prnu_destroy(ctx)
