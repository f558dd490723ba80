"""Write stored oracle outputs for the GPU parity tests.

Calls only the FP64 oracle (``oracle/``) on inputs drawn by the seeded generator;
nothing here comes from the GPU path.  Each output file records, per frame, the PCE,
peak shift, NCC and relative gap between the two largest window values of every
candidate of the searched grid, plus a digest of the inputs so that a stale file is
detected.

    python tests/golden/make_golden.py tiny          # 256x256, 4 frames, 11x11 grid
    python tests/golden/make_golden.py hd  [--frames 0,1,2] [--procs 6]
    python tests/golden/make_golden.py uhd [--frames 0]     # bf16-stored 4K frames
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


_K = None
_KN = None
_FR = None


def _init(K, frames):
    global _K, _KN, _FR
    _K, _FR = K, frames
    _KN = O.mean_free(K)


def _eval(job):
    f, s, t, radius = job
    r = O.evaluate_candidate(_K, _FR[f], s, t, radius, _KN)
    gap = (r.peak - r.runner_up) / abs(r.peak) if r.peak != 0 else 0.0
    return f, r.pce, r.dx, r.dy, r.rho, gap


def run(K, frames, cands, radius, frame_ids, procs):
    jobs = [(f, s, t, radius) for f in frame_ids for (s, t) in cands]
    with ProcessPoolExecutor(procs, initializer=_init, initargs=(K, frames)) as ex:
        out = list(ex.map(_eval, jobs, chunksize=8))
    nf, nc = len(frame_ids), len(cands)
    pce = np.array([o[1] for o in out]).reshape(nf, nc)
    dx = np.array([o[2] for o in out], dtype=np.int32).reshape(nf, nc)
    dy = np.array([o[3] for o in out], dtype=np.int32).reshape(nf, nc)
    rho = np.array([o[4] for o in out]).reshape(nf, nc)
    gap = np.array([o[5] for o in out]).reshape(nf, nc)
    return pce, dx, dy, rho, gap


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["tiny", "hd", "uhd"])
    ap.add_argument("--frames", default="")
    ap.add_argument("--procs", type=int, default=max(1, (os.cpu_count() or 2) - 2))
    a = ap.parse_args()
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    t0 = time.time()
    if a.which == "tiny":
        seq = synth.tiny(n_frames=4)
        grid = (11, 0.95, 1.05, 11, -2.0, 2.0)
        radius = 16
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
    pce, dx, dy, rho, gap = run(seq.K, frames, cands, radius, ids, a.procs)
    path = os.path.join(HERE, f"oracle_{a.which}.npz")
    np.savez_compressed(
        path, frames=np.array(ids, dtype=np.int32), pce=pce, dx=dx, dy=dy, rho=rho, peak_gap=gap,
        grid=np.array(grid, dtype=np.float64), radius=np.int32(radius),
        digest=np.array(digest(seq.K, frames[ids])),
        planted=np.array([[p.scale, p.rot_deg, p.dx, p.dy] for p in seq.planted], dtype=np.float64))
    print(f"wrote {path} ({len(ids)} frames x {len(cands)} candidates) in {time.time() - t0:.1f}s")


if __name__ == "__main__":
    main()
