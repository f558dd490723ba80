"""GPU parity of the general 8-parameter Eq. (4) warp and of Algorithm 1's
transform-initialised refinement, against the FP64 oracle, through the C ABI.
"""
import math
import sys

import numpy as np
import pytest

from oracle import prnu_oracle as O
from paper_2207_14507_amd import synth
from test_gpu_parity import check_one

pytestmark = pytest.mark.gpu

REL = 1e-3
GAP = 2e-3

TRUE_T = np.array([[1.012, 0.021, 0.0], [-0.016, 0.994, 0.0], [2.0e-4, -1.5e-4, 1.0]])


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
    return (r.pce, r.rho, r.scale, r.rot_deg, r.dx, r.dy, r.cand_index, r.n_evaluated, r.iterations, r.status)


def test_general_transforms_match_oracle(P):
    seq = synth.transform_sequence(81, 256, [(TRUE_T, 3, -2)])
    W = seq.frames[0]
    Ts = [TRUE_T, np.eye(3), O.similarity_matrix(1.01, 0.4),
          np.array([[1.03, -0.02, 0.0], [0.01, 0.98, 0.0], [0.0, 0.0, 1.0]]),
          np.array([[0.99, 0.0, 0.0], [0.0, 1.01, 0.0], [-3.0e-4, 2.0e-4, 1.0]])]
    ctx = P.prnu_create(0)
    try:
        fp = P.prnu_open_fingerprint(ctx, seq.K)
        pce, rho, dx, dy = P.prnu_score_transforms(ctx, fp, seq.frames, 0, np.stack(Ts), 16)
        kn = O.mean_free(seq.K)
        for i, T in enumerate(Ts):
            o, near = O.transform_near_peaks(seq.K, W, T, 16, GAP, kn)
            say(i, pce[i], o.pce)
            check_one(f"transform {i}", pce[i], dx[i], dy[i], o, near)
        assert pce[0] == max(pce) and (dx[0], dy[0]) == (3, -2)  # the planted transform scores best
        # the identity through the general path equals the similarity path bit for bit
        g, _, gx, gy = P.prnu_score_grid(ctx, fp, seq.frames, 0, P.make_opts(grid=(1, 1.0, 1.0, 1, 0.0, 0.0),
                                                                          radius=16))
        assert g[0] == pce[1] and (gx[0], gy[0]) == (dx[1], dy[1])
        with pytest.raises(P.PrnuError) as e:
            P.prnu_score_transforms(ctx, fp, seq.frames, 0, np.zeros((1, 3, 3)), 16)
        assert e.value.status == P.PRNU_E_ARG
    finally:
        P.prnu_destroy(ctx)


def test_points_beyond_the_horizon_read_zero(P):
    """A transform whose horizon crosses the frame: GPU PCE still within 1e-3 of the
    oracle, which zeroes those pixels."""
    seq = synth.planted_sequence(82, 256, [synth.Planted(1.0, 0.0, 0, 0)])
    T = np.linalg.inv(np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.01, 1.0]]))  # Z < 0 above row 28
    ctx = P.prnu_create(0)
    try:
        fp = P.prnu_open_fingerprint(ctx, seq.K)
        pce, _, dx, dy = P.prnu_score_transforms(ctx, fp, seq.frames, 0, T[None], 16)
        o = O.evaluate_transform(seq.K, seq.frames[0], T, 16)
        assert abs(pce[0] - o.pce) <= REL * max(abs(o.pce), 1.0), (pce[0], o.pce)
    finally:
        P.prnu_destroy(ctx)


def test_transform_initialised_refinement(P):
    seq = synth.transform_sequence(83, 256, [(TRUE_T, 1, 2), (TRUE_T, -2, 0)])
    refine = dict(half=5, rot_lo=-1.0, rot_hi=1.0)
    o = P.make_opts(radius=16, refine=refine)
    wild = O.similarity_matrix(1.25, 4.0)
    ctx = P.prnu_create(0)
    try:
        fp = P.prnu_open_fingerprint(ctx, seq.K)
        plain, _ = P.prnu_search_frames(ctx, fp, seq.frames, o)
        res, summ = P.prnu_search_with_transform(ctx, fp, seq.frames, o, np.stack([TRUE_T, wild]))
        kn = O.mean_free(seq.K)
        for f, H in enumerate((TRUE_T, wild)):
            oh = O.evaluate_transform(seq.K, seq.frames[f], H, 16, kn).pce
            oi = O.evaluate_transform(seq.K, seq.frames[f], np.eye(3), 16, kn).pce
            if abs(oh - oi) > GAP * max(abs(oh), abs(oi)):
                assert res[f].used_init == int(oh > oi), (f, oh, oi)
        assert res[0].used_init == 1 and res[1].used_init == 0
        # frame 1 ignored its transform: the same as the plain refinement
        assert fields(res[1]) == fields(plain[1])
        # frame 0 started from the transform's nearest similarity: the oracle from there
        s0, t0 = O.similarity_of(TRUE_T)
        ro = O.refine_frame(seq.K, seq.frames[0], O.RefineOptions(half=5, rot_lo=-1.0, rot_hi=1.0, radius=16,
                                                                  init_scale=s0, init_rot=t0))
        assert res[0].iterations == ro.iterations and res[0].n_evaluated == ro.n_evaluated
        assert abs(res[0].pce - ro.pce) <= REL * abs(ro.pce)
        assert math.isclose(summ.mean_pce, (res[0].pce + res[1].pce) / 2, rel_tol=1e-12)
    finally:
        P.prnu_destroy(ctx)


def test_general_transforms_at_1080p_sampled(P):
    """General transforms on a frame of the 1080p workload (full-size FFTs, radius 64),
    each against the oracle."""
    seq = synth.hd_sequence(n_frames=2)
    g = synth.rng(82, 1)
    Ts = [np.eye(3)]
    for _ in range(4):
        A = np.eye(3)
        A[:2, :2] += g.uniform(-0.01, 0.01, size=(2, 2))
        A[2, :2] = g.uniform(-2e-5, 2e-5, size=2)
        Ts.append(A)
    ctx = P.prnu_create(0)
    try:
        fp = P.prnu_open_fingerprint(ctx, seq.K)
        pce, rho, dx, dy = P.prnu_score_transforms(ctx, fp, seq.frames, 1, np.stack(Ts), 64)
        kn = O.mean_free(seq.K)
        for i, T in enumerate(Ts):
            r, near = O.transform_near_peaks(seq.K, seq.frames[1], T, 64, GAP, kn)
            say(f"transform {i}: gpu {pce[i]:.2f} oracle {r.pce:.2f}")
            check_one(f"hd transform {i}", pce[i], dx[i], dy[i], r, near)
        P.prnu_close_fingerprint(ctx, fp)
    finally:
        P.prnu_destroy(ctx)
