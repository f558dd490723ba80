"""GPU tests of the launch runtime: captured launch graphs and the schedule autotuner.

A replayed graph must give the results of eager launches bit for bit, on every replay
and with other GPU work between the replays; a schedule (FFT batch, block order) changes
only the grouping of independent candidates, so every schedule gives the same results.
"""
import os
import sys

import numpy as np
import pytest

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


def fields(r):
    return (r.pce, r.rho, r.scale, r.rot_deg, r.dx, r.dy, r.cand_index, r.fell_back, r.n_evaluated, r.status)


def test_graph_replays_equal_eager_launches(P):
    import torch
    s = synth.walk_sequence(41, 0, 256, 256, 6, radius=12)
    o = P.make_opts(grid=(7, 0.96, 1.04, 7, -1.5, 1.5), radius=16, warm=True, local=(5, 5, 0.005, 0.2),
                    fallback_pce=60.0)
    g = P.prnu_create(0)
    e = P.prnu_create(0, flags=P.PRNU_FLAG_NO_GRAPHS)
    try:
        fg, fe = P.prnu_open_fingerprint(g, s.K), P.prnu_open_fingerprint(e, s.K)
        ref, _ = P.prnu_search_frames(e, fe, s.frames, o)
        x = torch.randn(1 << 20, device="cuda")
        for rep in range(4):
            say("replay round", rep)
            res, _ = P.prnu_search_frames(g, fg, s.frames, o)
            assert [fields(r) for r in res] == [fields(r) for r in ref], rep
            # other GPU work and synchronisations between the replays
            x = torch.sin(x) * 1.5 + 0.1
            torch.cuda.synchronize()
            again, _ = P.prnu_search_frames(e, fe, s.frames, o)
            assert [fields(r) for r in again] == [fields(r) for r in ref], rep
        cap, rep_n = P.prnu_graph_stats(g)
        say("captures", cap, "replays", rep_n)
        assert cap >= 1 and rep_n >= 10  # the local-grid launch set repeats every frame
        assert P.prnu_graph_stats(e) == (0, 0)
    finally:
        P.prnu_destroy(g)
        P.prnu_destroy(e)


def test_tuned_schedule_is_cached_and_reloaded(P, tmp_path):
    path = str(tmp_path / "tune.txt")
    ctx = P.prnu_create(0, tune_cache_path=path)
    try:
        t = P.prnu_tune(ctx, 256, 256, 16, P.PRNU_F32)
        say("tuned", t)
        assert not t["from_cache"] and t["ns_per_candidate"] > 0.0
        assert t["batch"] in (8, 16, 32, 48, 64, 96, 128, 192, 256, 320, 384, 448, 512, 640, 768) and t["order"] in (0, 1)
        b = P.prnu_tune(ctx, 256, 256, 16, P.PRNU_BF16)
        assert b["ns_per_candidate"] > 0.0
        with pytest.raises(P.PrnuError) as err:
            P.prnu_tune(ctx, 250, 250, 16, P.PRNU_F32)  # 250 is not a built length
        assert err.value.status == P.PRNU_E_SHAPE
    finally:
        P.prnu_destroy(ctx)
    lines = [l.split() for l in open(path) if not l.startswith("#")]
    assert ["256", "256", "16", "0", str(t["batch"]), str(t["order"])] in [l[:6] for l in lines]
    ctx = P.prnu_create(0, tune_cache_path=path)
    try:
        again = P.prnu_tune(ctx, 256, 256, 16, P.PRNU_F32)
        assert again["from_cache"] and (again["batch"], again["order"]) == (t["batch"], t["order"])
    finally:
        P.prnu_destroy(ctx)
    ctx = P.prnu_create(0, flags=P.PRNU_FLAG_NO_AUTOTUNE)
    try:
        d = P.prnu_tune(ctx, 256, 256, 16, P.PRNU_F32)
        assert d["ns_per_candidate"] == 0.0 and d["batch"] >= 1
    finally:
        P.prnu_destroy(ctx)



def test_cache_file_entries_are_checked(P, tmp_path):
    """Malformed lines of a schedule cache are skipped, and a cached batch whose workspace
    exceeds the tuning limit (8 GiB) is halved until it fits."""
    path = tmp_path / "tune.txt"
    path.write_text("# edited by hand\n"
                    "garbage line\n"
                    "256 256 16 0 32\n"            # too few fields
                    "256 256 16 0 0 0 5.0\n"       # batch 0
                    "256 256 16 0 64 7 5.0\n"      # unknown block order
                    "1080 1920 64 0 4096 1 9.0\n")  # 4096 1080p candidates: ~40 GiB of workspace
    ctx = P.prnu_create(0, tune_cache_path=str(path), flags=P.PRNU_FLAG_NO_AUTOTUNE)
    try:
        hd = P.prnu_tune(ctx, 1080, 1920, 64, P.PRNU_F32)
        say("capped", hd)
        assert hd["from_cache"] and hd["order"] == 1 and hd["batch"] == 512
        small = P.prnu_tune(ctx, 256, 256, 16, P.PRNU_F32)
        assert not small["from_cache"] and small["ns_per_candidate"] == 0.0
    finally:
        P.prnu_destroy(ctx)

def test_every_schedule_gives_the_same_results(P, tmp_path):
    """Force each (batch, order) through the cache file and compare with the default."""
    s = synth.walk_sequence(42, 0, 256, 256, 2, radius=12)
    o = P.make_opts(grid=(9, 0.95, 1.05, 9, -2.0, 2.0), radius=16)
    ctx = P.prnu_create(0, flags=P.PRNU_FLAG_NO_AUTOTUNE)
    try:
        ref, _ = P.prnu_search_frames(ctx, P.prnu_open_fingerprint(ctx, s.K), s.frames, o)
    finally:
        P.prnu_destroy(ctx)
    for batch in (5, 16, 81):
        for order in (0, 1):
            path = str(tmp_path / f"t_{batch}_{order}.txt")
            with open(path, "w") as f:
                f.write(f"256 256 16 0 {batch} {order} 1.0\n")
            ctx = P.prnu_create(0, tune_cache_path=path)
            try:
                assert P.prnu_tune(ctx, 256, 256, 16)["batch"] == batch
                res, _ = P.prnu_search_frames(ctx, P.prnu_open_fingerprint(ctx, s.K), s.frames, o)
                assert [fields(r) for r in res] == [fields(r) for r in ref], (batch, order)
            finally:
                P.prnu_destroy(ctx)
