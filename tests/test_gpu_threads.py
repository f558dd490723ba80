"""Several host threads on one context at once, through the C ABI: synchronous searches,
grid scoring with fingerprints opened and closed meanwhile, and serving-engine videos
submitted and polled.  Every result must equal, bit for bit, the same call made alone
beforehand: the calls serialise or batch inside the library, and each candidate is
computed independently of what shares its launch.

The binding's foreign calls release the interpreter lock, so the threads are inside the
library together.  Every wait is bounded (poll time-outs, joins with a time-out)."""
import sys
import threading
import time

import pytest

from paper_2207_14507_amd import synth

pytestmark = pytest.mark.gpu

GRID = (5, 0.97, 1.03, 5, -1.0, 1.0)


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
    return (r.status, r.pce, r.rho, r.scale, r.rot_deg, r.dx, r.dy, r.cand_index, r.fell_back, r.n_evaluated)


def run_video(P, ctx, fp, frames, opts, deadline_s=60.0):
    """Submit, then poll with short time-outs until done; BUSY (staging full) is retried."""
    t_end = time.monotonic() + deadline_s
    while True:
        try:
            t = P.prnu_submit_video(ctx, fp, frames, opts)
            break
        except P.PrnuError as e:
            if e.status != P.PRNU_E_BUSY or time.monotonic() > t_end:
                raise
            time.sleep(0.01)
    while True:
        st, res, summ = P.prnu_poll(ctx, t, len(frames), timeout_ms=200)
        if st == P.PRNU_OK:
            return [fields(r) for r in res], summ.mean_pce
        assert time.monotonic() < t_end, "video did not finish"


def test_concurrent_calls_on_one_context(P):
    seqs = [synth.tiny(n_frames=3, config=80 + i) for i in range(3)]
    vids = [synth.walk_sequence(84, i, 256, 256, 5, radius=8) for i in range(3)]
    opts = P.make_opts(grid=GRID, radius=16)
    vopts = P.make_opts(grid=GRID, radius=16, warm=True, local=(3, 3, 0.005, 0.2), fallback_pce=60.0)
    ctx = P.prnu_create(0, flags=P.PRNU_FLAG_NO_AUTOTUNE)
    alive = []
    try:
        fps = [P.prnu_open_fingerprint(ctx, s.K) for s in seqs]
        vfps = [P.prnu_open_fingerprint(ctx, v.K) for v in vids]
        # each call alone first
        ref_sync = [[fields(r) for r in P.prnu_search_frames(ctx, fp, s.frames, opts)[0]] for fp, s in zip(fps, seqs)]
        ref_grid = [x.copy() for x in P.prnu_score_grid(ctx, fps[0], seqs[0].frames, 1, opts)]
        ref_vid = [run_video(P, ctx, fp, v.frames, vopts) for fp, v in zip(vfps, vids)]
        say("references done")

        errors = []
        done = []

        def guarded(name, fn):
            def body():
                try:
                    fn()
                    done.append(name)
                except Exception as e:  # reported by the main thread
                    errors.append((name, repr(e)))
            return threading.Thread(target=body, name=name, daemon=True)

        def sync_worker(i):
            for _ in range(3):
                got = [fields(r) for r in P.prnu_search_frames(ctx, fps[i], seqs[i].frames, opts)[0]]
                assert got == ref_sync[i], f"search of sequence {i} differs"

        def grid_worker():
            for _ in range(3):
                h = P.prnu_open_fingerprint(ctx, seqs[0].K)
                got = P.prnu_score_grid(ctx, h, seqs[0].frames, 1, opts)
                P.prnu_close_fingerprint(ctx, h)
                for a, b in zip(got, ref_grid):
                    assert (a == b).all(), "grid scores with a reopened fingerprint differ"

        def video_worker(i):
            for _ in range(2):
                got = run_video(P, ctx, vfps[i], vids[i].frames, vopts)
                assert got == ref_vid[i], f"video {i} differs"

        threads = [guarded(f"sync{i}", lambda i=i: sync_worker(i)) for i in range(3)]
        threads += [guarded("grid", grid_worker)]
        threads += [guarded(f"video{i}", lambda i=i: video_worker(i)) for i in range(3)]
        for t in threads:
            t.start()
        t_end = time.monotonic() + 90.0
        for t in threads:
            t.join(max(0.0, t_end - time.monotonic()))
        alive = [t.name for t in threads if t.is_alive()]
        say("finished:", sorted(done), "errors:", errors, "still running:", alive)
        assert not alive, f"threads still running: {alive}"
        assert errors == []
        assert len(done) == len(threads)
        # the context is still usable and consistent afterwards
        again = [fields(r) for r in P.prnu_search_frames(ctx, fps[2], seqs[2].frames, opts)[0]]
        assert again == ref_sync[2]
    finally:
        if not alive:  # a thread still inside the library keeps the context
            P.prnu_destroy(ctx)
