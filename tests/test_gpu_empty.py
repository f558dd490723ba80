"""Empty inputs through the C ABI: no frames, no images, no candidates.

- A search over zero frames (plain, warm-started, coarse-to-fine; host or device
  memory; fp32 or bf16) succeeds with no results and an empty summary (0 frames, mean
  PCE 0, decision 0).
- A video of zero frames is done at submission: its poll returns at once with no
  results.
- Residuals of zero images are an empty array; the Eq. (2) estimate of zero images and
  a grid with no candidates are refused with PRNU_E_ARG, as is scoring a frame index
  outside the frames given.
- None of these leaves the context failed: a search afterwards gives the same result as
  before them.
"""
import sys

import numpy as np
import pytest

from paper_2207_14507_amd import synth

pytestmark = pytest.mark.gpu

GRID = (3, 0.98, 1.02, 3, -1.0, 1.0)


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


def fields(r):
    return (r.status, r.pce, r.rho, r.scale, r.rot_deg, r.dx, r.dy, r.cand_index)


def test_empty_inputs(P):
    import torch
    seq = synth.tiny(n_frames=2, config=27)
    M, N = seq.frames.shape[1:]
    plain = P.make_opts(grid=GRID, radius=16)
    warm = P.make_opts(grid=GRID, radius=16, warm=True, local=(3, 3, 0.005, 0.2), fallback_pce=60.0)
    refine = P.make_opts(grid=GRID, radius=16, refine=dict(half=1, max_iter=2))
    ctx = P.prnu_create(0, flags=P.PRNU_FLAG_NO_AUTOTUNE)
    try:
        fp = P.prnu_open_fingerprint(ctx, seq.K)
        before = [fields(r) for r in P.prnu_search_frames(ctx, fp, seq.frames, plain)[0]]
        none = np.zeros((0, M, N), np.float32)
        none_bf16 = np.zeros((0, M, N), np.uint16)
        none_dev = torch.empty((0, M, N), device="cuda")
        for name, frames, scales in [("host f32", none, None), ("host bf16", none_bf16, np.zeros(0, np.float32)),
                                     ("device f32", none_dev, None)]:
            for oname, o in [("plain", plain), ("warm", warm), ("refine", refine)]:
                say(f"empty search: {name}, {oname}")
                res, summ = P.prnu_search_frames(ctx, fp, frames, o, scales=scales)
                assert res == [] and summ.n_frames == 0 and summ.mean_pce == 0.0 and summ.decision == 0
        say("empty video")
        t = P.prnu_submit_video(ctx, fp, none, warm)
        st, res, summ = P.prnu_poll(ctx, t, 0, timeout_ms=10000)
        assert st == P.PRNU_OK and res == [] and summ.n_frames == 0 and summ.mean_pce == 0.0
        with pytest.raises(P.PrnuError) as e:  # retired
            P.prnu_poll(ctx, t, 0, timeout_ms=0)
        assert e.value.status == P.PRNU_E_HANDLE
        say("empty residuals and estimate")
        W = P.prnu_extract_residuals(ctx, none, 3.0)
        assert W.shape == (0, M, N)
        with pytest.raises(P.PrnuError) as e:
            P.prnu_estimate_fingerprint(ctx, none, none)
        assert e.value.status == P.PRNU_E_ARG
        say("refusals")
        with pytest.raises(P.PrnuError) as e:
            P.prnu_search_frames(ctx, fp, seq.frames, P.make_opts(grid=(0, 1.0, 1.0, 3, -1.0, 1.0), radius=16))
        assert e.value.status == P.PRNU_E_ARG
        with pytest.raises(P.PrnuError) as e:
            P.prnu_score_grid(ctx, fp, none, 0, plain)
        assert e.value.status == P.PRNU_E_ARG
        with pytest.raises(P.PrnuError) as e:
            P.prnu_score_grid(ctx, fp, seq.frames, 2, plain)
        assert e.value.status == P.PRNU_E_ARG
        after = [fields(r) for r in P.prnu_search_frames(ctx, fp, seq.frames, plain)[0]]
        assert after == before
        P.prnu_close_fingerprint(ctx, fp)
    finally:
        P.prnu_destroy(ctx)
