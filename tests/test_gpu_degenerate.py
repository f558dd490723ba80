"""Degenerate inputs of the search on the GPU, through the C ABI.

- A frame that is the mean-free fingerprint moved by d (no warp, no noise): NCC 1 at the
  identity candidate's peak and the peak at d (the closed form the oracle is pinned
  to).  Its PCE is not checked: the off-peak energy is the difference of two sums
  dominated by the peak, pure rounding.
- An all-zero frame: a zero correlation surface, PCE 0 and NCC 0 for every candidate,
  the peak at the first window position (-R, -R), and the lowest candidate index wins.
- A frame with a non-finite pixel: every candidate's PCE is NaN, the frame reports
  PRNU_E_NONFINITE, and the other frames of the call are unaffected.
"""
import math

import numpy as np
import pytest

from oracle import prnu_oracle as O
from paper_2207_14507_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2207_14507_amd import prnu
    return prnu


@pytest.fixture(scope="module")
def ctx(P):
    c = P.prnu_create(0)
    yield c
    P.prnu_destroy(c)


@pytest.mark.parametrize("shape,d", [((256, 256), (5, -7)), ((120, 160), (-3, 9)), ((1080, 1920), (12, -30))])
def test_shifted_fingerprint_gives_unit_ncc_at_the_shift(P, ctx, shape, d):
    K = synth.fingerprint(synth.rng(60, *shape), *shape)
    Kt, _ = O.mean_free(K)
    W = np.roll(Kt, (-d[0], -d[1]), axis=(0, 1)).astype(np.float32)   # W[p] = Kt[p + d]
    fp = P.prnu_open_fingerprint(ctx, K)
    R = 64 if shape[0] >= 1080 else 16
    opts = P.make_opts(grid=(3, 0.99, 1.01, 3, -0.5, 0.5), radius=R)
    pce, rho, dx, dy = P.prnu_score_grid(ctx, fp, W[None], 0, opts)
    # candidate 4 is the identity (scale 1, rotation 0)
    assert (dy[4], dx[4]) == d
    assert abs(rho[4] - 1.0) < 1e-4, rho[4]
    assert np.all(rho[[0, 1, 2, 3, 5, 6, 7, 8]] < 0.9)
    P.prnu_close_fingerprint(ctx, fp)


def test_zero_frame(P, ctx):
    seq = synth.tiny(n_frames=1, config=61)
    fp = P.prnu_open_fingerprint(ctx, seq.K)
    R = 16
    opts = P.make_opts(grid=(3, 0.98, 1.02, 3, -1.0, 1.0), radius=R)
    zero = np.zeros((1, 256, 256), np.float32)
    pce, rho, dx, dy = P.prnu_score_grid(ctx, fp, zero, 0, opts)
    assert np.all(pce == 0.0) and np.all(rho == 0.0)
    assert np.all(dx == -R) and np.all(dy == -R)
    o = O.evaluate_candidate(seq.K, zero[0], 1.0, 0.0, R)
    assert (o.pce, o.dx, o.dy) == (0.0, -R, -R)
    res, summ = P.prnu_search_frames(ctx, fp, zero, opts)
    assert res[0].status == 0 and res[0].cand_index == 0 and res[0].pce == 0.0
    P.prnu_close_fingerprint(ctx, fp)


@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_non_finite_frame(P, ctx, bad):
    seq = synth.tiny(n_frames=3, config=62)
    frames = seq.frames.copy()
    frames[1, 100, 37] = bad
    fp = P.prnu_open_fingerprint(ctx, seq.K)
    opts = P.make_opts(grid=(3, 0.98, 1.02, 3, -1.0, 1.0), radius=16)
    res, _ = P.prnu_search_frames(ctx, fp, frames, opts)
    assert res[1].status == P.PRNU_E_NONFINITE and math.isnan(res[1].pce)
    clean, _ = P.prnu_search_frames(ctx, fp, seq.frames[[0, 2]], opts)
    for r, c in zip([res[0], res[2]], clean):
        assert r.status == 0 and (r.pce, r.cand_index, r.dx, r.dy) == (c.pce, c.cand_index, c.dx, c.dy)
    pce, _, _, _ = P.prnu_score_grid(ctx, fp, frames, 1, opts)
    assert np.all(np.isnan(pce))
    P.prnu_close_fingerprint(ctx, fp)
