"""Write stored oracle outputs for the GPU parity tests.

Calls only the FP64 oracle (``oracle/``) on inputs drawn by the seeded generator;
nothing here comes from the GPU path.  Each grid file records, per frame, the PCE,
peak shift, NCC and relative gap between the two largest window values of every
candidate of the searched grid, plus the near-tied peak shifts of each candidate (every
shift of the peak window whose correlation is within NEAR of the peak, relative, with
the PCE of Eq. (3) taken there: the shifts an implementation may report when the peak
is ambiguous at its rounding), and a digest of the inputs so that a stale file is
detected.  The warm-chain files record the oracle's chained search (Algorithm 1 with
the local grid and the full-grid fallback) frame by frame.

    python tests/golden/make_golden.py tiny          # 256x256, 4 frames, 11x11 grid
    python tests/golden/make_golden.py hd  [--frames 0,1,2] [--procs 6]
    python tests/golden/make_golden.py uhd [--frames 0]     # bf16-stored 4K frames
    python tests/golden/make_golden.py uhd --near-only      # add the near-tied shifts to a
                                                            # stored file (see near_only)
    python tests/golden/make_golden.py warm_hd       # 1080p warm chain, 5 frames
    python tests/golden/make_golden.py warm_720      # 720p warm chain, 5 frames
    python tests/golden/make_golden.py p720          # 720 x 1280, 1 walk frame, 41x21 grid
    python tests/golden/make_golden.py portrait720   # 1280 x 720 (portrait), same
    python tests/golden/make_golden.py portrait1080  # 1920 x 1080 (portrait), same
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import prnu_oracle as O  # noqa: E402
from paper_2207_14507_amd import synth  # noqa: E402


def digest(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()[:16]


NEAR = 2e-3   # relative window-value gap within which a peak shift counts as near-tied
NEAR_MAX = 8  # near-tied shifts stored per candidate (the count is stored in full)

_K = None
_KN = None
_FR = None


def _init(K, frames):
    global _K, _KN, _FR
    _K, _FR = K, frames
    _KN = O.mean_free(K)


def near_arrays(near):
    """Fixed-size arrays (dx, dy, pce) of the first NEAR_MAX near-tied shifts, and the count."""
    n = len(near)
    dx = np.zeros(NEAR_MAX, np.int32)
    dy = np.zeros(NEAR_MAX, np.int32)
    pce = np.full(NEAR_MAX, np.nan)
    for i, t in enumerate(near[:NEAR_MAX]):
        dx[i], dy[i], pce[i] = t.dx, t.dy, t.pce
    return dx, dy, pce, n


def _eval(job):
    f, s, t, radius = job
    r, near = O.candidate_near_peaks(_K, _FR[f], s, t, radius, NEAR, _KN)
    gap = (r.peak - r.runner_up) / abs(r.peak) if r.peak != 0 else 0.0
    return (f, r.pce, r.dx, r.dy, r.rho, gap) + near_arrays(near)


def run(K, frames, cands, radius, frame_ids, procs):
    jobs = [(f, s, t, radius) for f in frame_ids for (s, t) in cands]
    with ProcessPoolExecutor(procs, initializer=_init, initargs=(K, frames)) as ex:
        out = list(ex.map(_eval, jobs, chunksize=8))
    nf, nc = len(frame_ids), len(cands)
    col = lambda i, dt=np.float64: np.array([o[i] for o in out], dtype=dt)
    res = dict(pce=col(1).reshape(nf, nc), dx=col(2, np.int32).reshape(nf, nc), dy=col(3, np.int32).reshape(nf, nc),
               rho=col(4).reshape(nf, nc), peak_gap=col(5).reshape(nf, nc),
               near_dx=col(6, np.int32).reshape(nf, nc, NEAR_MAX), near_dy=col(7, np.int32).reshape(nf, nc, NEAR_MAX),
               near_pce=col(8).reshape(nf, nc, NEAR_MAX), near_n=col(9, np.int32).reshape(nf, nc))
    return res


def _eval_near(job):
    f, s, t, radius = job
    _, near = O.candidate_near_peaks(_K, _FR[f], s, t, radius, NEAR, _KN)
    return near_arrays(near)


def near_only(path, K, frames, cands, radius, procs):
    """Adds the near-tied shifts to a stored grid file without recomputing its other
    arrays.  A candidate whose two largest window values differ by more than NEAR has
    only its peak within NEAR of the peak, so only the near-tied candidates are
    evaluated again; the others get their stored peak as the single entry."""
    g = dict(np.load(path, allow_pickle=False))
    ids = [int(x) for x in g["frames"]]
    nf, nc = g["pce"].shape
    n_dx = np.zeros((nf, nc, NEAR_MAX), np.int32)
    n_dy = np.zeros((nf, nc, NEAR_MAX), np.int32)
    n_pce = np.full((nf, nc, NEAR_MAX), np.nan)
    n_cnt = np.ones((nf, nc), np.int32)
    n_dx[:, :, 0], n_dy[:, :, 0], n_pce[:, :, 0] = g["dx"], g["dy"], g["pce"]
    weak = [(i, j) for i in range(nf) for j in range(nc) if not g["peak_gap"][i, j] > NEAR]
    jobs = [(ids[i], cands[j][0], cands[j][1], radius) for i, j in weak]
    with ProcessPoolExecutor(procs, initializer=_init, initargs=(K, frames)) as ex:
        out = list(ex.map(_eval_near, jobs, chunksize=4))
    for (i, j), (dx, dy, pce, n) in zip(weak, out):
        n_dx[i, j], n_dy[i, j], n_pce[i, j], n_cnt[i, j] = dx, dy, pce, n
    g.update(near_dx=n_dx, near_dy=n_dy, near_pce=n_pce, near_n=n_cnt)
    np.savez_compressed(path, **g)
    return len(weak)


def warm_frames(shape):
    """Five walk frames of one fingerprint; the third is drawn from an independent
    fingerprint (no match), so that its local search falls back to the full grid."""
    M, N = shape
    seq = synth.walk_sequence(31, 0, M, N, 5)
    other = synth.walk_sequence(31, 0, M, N, 5, independent_fp=True)
    frames = np.stack([seq.frames[0], seq.frames[1], other.frames[2], seq.frames[3], seq.frames[4]])
    return seq.K, frames, seq.planted


def run_warm(which):
    """The oracle's chained search on the batched workload's options: full grid on the
    first frame, 9 x 9 local grid (0.005, 0.1 deg) around the previous estimate, full
    41 x 21 grid as well when the local best is below PCE 60, shift radius 64."""
    shape = (1080, 1920) if which == "warm_hd" else (720, 1280)
    K, frames, planted = warm_frames(shape)
    o = O.WarmOptions()
    res = O.search_video(K, frames, o)
    F = len(frames)
    maxc = max(len(r.all) for r in res)
    cand = np.full((F, maxc, 2), np.nan)
    pce = np.full((F, maxc), np.nan)
    gap = np.full((F, maxc), np.nan)
    dx = np.zeros((F, maxc), np.int32)
    dy = np.zeros((F, maxc), np.int32)
    n_eval = np.zeros(F, np.int32)
    fell = np.zeros(F, np.int32)
    index = np.zeros(F, np.int32)
    wn = [near_arrays([]) for _ in range(F)]
    Kn = O.mean_free(K)
    for f, r in enumerate(res):
        n = len(r.all)
        n_eval[f], fell[f], index[f] = n, int(r.fell_back), r.index
        for i, c in enumerate(r.all):
            cand[f, i] = (c.scale, c.rot_deg)
            pce[f, i], dx[f, i], dy[f, i] = c.pce, c.dx, c.dy
            gap[f, i] = (c.peak - c.runner_up) / abs(c.peak) if c.peak != 0 else 0.0
        _, near = O.candidate_near_peaks(K, frames[f], r.best.scale, r.best.rot_deg, o.radius, NEAR, Kn)
        wn[f] = near_arrays(near)
        print(f"{which} frame {f}: {n} candidates, fell back {r.fell_back}, best {r.best.scale:.4f} "
              f"{r.best.rot_deg:.3f} ({r.best.dx}, {r.best.dy}) PCE {r.pce:.2f}", flush=True)
    return dict(cand=cand, pce=pce, dx=dx, dy=dy, peak_gap=gap, n_evaluated=n_eval, fell_back=fell, index=index,
                win_near_dx=np.stack([w[0] for w in wn]), win_near_dy=np.stack([w[1] for w in wn]),
                win_near_pce=np.stack([w[2] for w in wn]), win_near_n=np.array([w[3] for w in wn], np.int32),
                mean_pce=np.float64(O.video_decision([r.pce for r in res], o.tau)[0]),
                digest=np.array(digest(K, frames)),
                planted=np.array([[p.scale, p.rot_deg, p.dx, p.dy] for p in planted], dtype=np.float64))


# One walk frame of the other frame sizes on the full grid: (M, N, sequence of
# synth.walk_sequence config 3).  Their column lengths (720, 1280, 1920 rows) run the
# column plans that the 1080p and 4K files do not.
SINGLE = {"p720": (720, 1280, 0), "portrait720": (1280, 720, 1), "portrait1080": (1920, 1080, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["tiny", "hd", "uhd", "warm_hd", "warm_720"] + list(SINGLE))
    ap.add_argument("--frames", default="")
    ap.add_argument("--procs", type=int, default=max(1, (os.cpu_count() or 2) - 2))
    ap.add_argument("--near-only", action="store_true")
    a = ap.parse_args()
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    t0 = time.time()
    if a.which.startswith("warm"):
        path = os.path.join(HERE, f"oracle_{a.which}.npz")
        np.savez_compressed(path, **run_warm(a.which))
        print(f"wrote {path} in {time.time() - t0:.1f}s")
        return
    if a.which == "tiny":
        seq = synth.tiny(n_frames=4)
        grid = (11, 0.95, 1.05, 11, -2.0, 2.0)
        radius = 16
        frames = seq.frames
    elif a.which in SINGLE:
        M, N, seq_id = SINGLE[a.which]
        seq = synth.walk_sequence(3, seq_id, M, N, 1)
        grid = (41, 0.85, 1.15, 21, -2.0, 2.0)
        radius = 64
        frames = seq.frames
    elif a.which == "hd":
        seq = synth.hd_sequence()
        grid = (41, 0.85, 1.15, 21, -2.0, 2.0)
        radius = 64
        frames = seq.frames
    else:
        seq = synth.uhd_bf16_sequence()
        grid = (41, 0.85, 1.15, 21, -2.0, 2.0)
        radius = 64
        frames = np.stack([synth.dequantize_bf16(b, s) for b, s in zip(seq.bf16, seq.bf16_scale)])
    ids = [int(x) for x in a.frames.split(",")] if a.frames else list(range(len(frames)))
    cands = O.candidates(O.grid_values(*grid[:3]), O.grid_values(*grid[3:]))
    if a.near_only:
        path = os.path.join(HERE, f"oracle_{a.which}.npz")
        g = np.load(path, allow_pickle=False)
        stored = [int(x) for x in g["frames"]]
        if str(g["digest"]) != digest(seq.K, frames[stored]):
            raise SystemExit(f"{path} does not match the generator's inputs")
        n = near_only(path, seq.K, frames, cands, radius, a.procs)
        print(f"added near-tied shifts to {path} ({n} candidates evaluated again) in {time.time() - t0:.1f}s")
        return
    res = run(seq.K, frames, cands, radius, ids, a.procs)
    path = os.path.join(HERE, f"oracle_{a.which}.npz")
    np.savez_compressed(
        path, frames=np.array(ids, dtype=np.int32), **res,
        grid=np.array(grid, dtype=np.float64), radius=np.int32(radius),
        digest=np.array(digest(seq.K, frames[ids])),
        planted=np.array([[p.scale, p.rot_deg, p.dx, p.dy] for p in seq.planted], dtype=np.float64))
    print(f"wrote {path} ({len(ids)} frames x {len(cands)} candidates) in {time.time() - t0:.1f}s")


if __name__ == "__main__":
    main()
