"""The whole identification flow on the GPU, through the C ABI: a reference fingerprint
from flat images (residuals, then Eq. (2)), residuals of stabilised frames, and the
EIS-inversion search against the estimated fingerprint.

Every step is checked against the oracle on the same inputs: the GPU residuals and
fingerprint within their fp32 tolerances, and the search's per-candidate PCE of the
GPU residuals against the oracle's PCE of the same (GPU-produced) residuals; the planted
transforms must be recovered.
"""
import numpy as np
import pytest

from oracle import denoise_oracle as D
from oracle import prnu_oracle as O
from paper_2207_14507_amd import synth
from test_gpu_parity import check_argmax, check_candidates, oracle_scores, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2207_14507_amd import prnu
    return prnu


def test_fingerprint_from_flat_images_then_search(P):
    M = N = 256
    g = synth.rng(50, 1)
    K = synth.fingerprint(g, M, N)
    # flat images: bright, nearly uniform scenes carrying the multiplicative PRNU
    flats = np.stack([(200.0 + 10.0 * synth.intensity(g, M, N)) * (1.0 + K) + g.standard_normal((M, N)) * 2.0
                      for _ in range(16)]).astype(np.float32)
    planted = [synth.Planted(1.015, -0.5, 3, -2), synth.Planted(0.985, 1.0, -4, 5), synth.Planted(1.0, 0.0, 0, 0)]
    frames = []
    for f, p in enumerate(planted):
        gf = synth.rng(50, 2, f)
        scene = synth.intensity(gf, M, N) * 255.0
        frames.append(synth.forward_warp(scene * (1.0 + K.astype(np.float64)), p) + gf.standard_normal((M, N)) * 2.0)
    frames = np.stack(frames).astype(np.float32)
    ctx = P.prnu_create(0)
    try:
        Wf = P.prnu_extract_residuals(ctx, flats, 3.0)
        Kh = P.prnu_estimate_fingerprint(ctx, flats, Wf)
        # the estimate against the oracle's chain on the same images
        Wo = np.stack([D.noise_residual(x, 3.0) for x in flats])
        Ko = O.estimate_fingerprint(flats, Wo)
        rel = float(np.linalg.norm(Kh - Ko) / np.linalg.norm(Ko))
        rho_k = float(np.corrcoef(Kh.ravel(), K.ravel())[0, 1])
        say(f"fingerprint: relative difference to the oracle {rel:.2e}, correlation with the planted PRNU {rho_k:.3f}")
        assert rel < 1e-4 and rho_k > 0.5
        Wr = P.prnu_extract_residuals(ctx, frames, 3.0)
        fp = P.prnu_open_fingerprint(ctx, Kh)
        grid = (5, 0.97, 1.03, 5, -1.0, 1.0)
        opts = P.make_opts(grid=grid, radius=16)
        res, _ = P.prnu_search_frames(ctx, fp, Wr, opts)
        cands = O.candidates(O.grid_values(*grid[:3]), O.grid_values(*grid[3:]))
        for f, (r, p) in enumerate(zip(res, planted)):
            say(f"frame {f}: scale {r.scale:.4f} rot {r.rot_deg:.2f} shift ({r.dx}, {r.dy}) PCE {r.pce:.1f}")
            assert abs(r.scale - p.scale) < 1e-9 and abs(r.rot_deg - p.rot_deg) < 1e-9
            assert (r.dx, r.dy) == (p.dx, p.dy)
            pce, rho, dx, dy = P.prnu_score_grid(ctx, fp, Wr, f, opts)
            o_pce, o_dx, o_dy, o_gap, _, near = oracle_scores(Kh, Wr[f], cands, 16)
            check_candidates(f"pipeline f{f}", pce, dx, dy, o_pce, o_dx, o_dy, o_gap, near)
            check_argmax(f"pipeline f{f}", o_pce, r.cand_index)
        P.prnu_close_fingerprint(ctx, fp)
    finally:
        P.prnu_destroy(ctx)
