"""CPU checks of the built HIP library: it loads, exports every entry point that
include/prnu.h declares, and its host-only calls behave without a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "prnu.h")
LIB = os.path.join(ROOT, "paper_2207_14507_amd", "libprnu.so")
EMU = os.path.join(ROOT, "paper_2207_14507_amd", "libprnu_emu.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(prnu_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    assert os.path.exists(LIB), "build the library first (python -m paper_2207_14507_amd.build)"
    lib = ctypes.CDLL(LIB)
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_the_header():
    from paper_2207_14507_amd import prnu as P
    assert sorted(P.EXPORTED) == declared_functions()


def test_status_strings_and_lengths():
    from paper_2207_14507_amd import prnu as P
    assert P.lib.prnu_status_string(P.PRNU_E_SHAPE) == b"unsupported or mismatched shape"
    lens = P.prnu_supported_lengths()
    for L in (256, 720, 1080, 1280, 1920, 2160, 3840):
        assert L in lens


def test_struct_layouts_match_the_header(tmp_path):
    """ctypes mirrors of the ABI structs have the C compiler's sizes and offsets."""
    import shutil
    import subprocess
    from paper_2207_14507_amd import prnu as P
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = [P.prnu_config, P.prnu_grid, P.prnu_search_opts, P.prnu_frames, P.prnu_frame_result,
               P.prnu_video_summary, P.prnu_kernel_stats]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "prnu.h"', "int main(void){"]
    for S in structs:
        lines.append(f'printf("%zu\\n", sizeof({S.__name__}));')
        for f, _ in S._fields_:
            lines.append(f'printf("%zu\\n", offsetof({S.__name__}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    want = []
    for S in structs:
        want.append(ctypes.sizeof(S))
        want.extend(getattr(S, f).offset for f, _ in S._fields_)
    assert got == want


def test_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2207_14507_amd import prnu as P
    ctx = ctypes.c_void_p()
    cfg = P.prnu_config(0, 0, 0, None, 0)
    st = P.lib.prnu_create(ctypes.byref(cfg), ctypes.byref(ctx))
    assert st == P.PRNU_E_DEVICE and not ctx.value


def _emu():
    return ctypes.CDLL(EMU)


def _lengths(lib, kind):
    buf = (ctypes.c_int * 64)()
    n = lib.prnu_emu_lengths(kind, buf, 64)
    return list(buf)[:n]


@pytest.mark.parametrize("kind", [0, 1, 2], ids=["row_plan", "col_plan", "col_plan_reversed"])
def test_emulated_device_fft_matches_numpy(kind):
    """The kernels' Stockham plans, index maps, butterflies (radices 5 to 16 forming
    their twiddle powers from W^k .. W^4k) and twiddle tables, run on the host, against
    numpy's FFT for every built length, both directions, batched."""
    lib = _emu()
    g = np.random.default_rng(kind)
    for L in _lengths(lib, kind):
        for inv in (0, 1):
            for B in (1, 3, 4, 8):
                x = (g.standard_normal((B, L)) + 1j * g.standard_normal((B, L))).astype(np.complex64)
                out = np.zeros_like(x)
                rc = lib.prnu_emu_fft(kind, L, inv, B, ctypes.c_void_p(x.ctypes.data), ctypes.c_void_p(out.ctypes.data))
                assert rc == 0
                x64 = x.astype(np.complex128)
                ref = np.fft.ifft(x64, axis=1) * L if inv else np.fft.fft(x64, axis=1)
                err = np.max(np.abs(out - ref)) / np.max(np.abs(ref))
                assert err < 2e-6, (kind, L, inv, B, err)


# ---------------------------------------------------------------------------
# Host logic of the library against the oracle (no device needed).

def test_candidate_grids_equal_the_oracles_bit_for_bit():
    """The runtime and the oracle generate every grid node as centre + k * step in FP64
    (independently written); the values must be identical, not merely close."""
    from oracle import prnu_oracle as O
    from paper_2207_14507_amd import prnu as P
    o = P.make_opts()
    assert P.prnu_candidates(o, 0) == O.full_grid(O.WarmOptions())
    for c in ((1.0, 0.0), (1.0123, 0.37), (0.9, -1.9)):
        assert P.prnu_candidates(o, 1, centre=c) == O.local_grid(O.WarmOptions(), c)
    ro = O.RefineOptions()
    for n, c in ((1, (1.0, 0.0)), (1, (1.02, 0.4)), (2, (1.02, 0.3)), (3, (0.987, -0.45))):
        assert P.prnu_candidates(P.make_opts(refine={}), 2, n, c) == O.refine_grid(ro, n, c), n
    small = dict(half=3, rot_lo=-1.0, rot_hi=1.0, scale_step=0.02, rot_step=0.25)
    assert P.prnu_candidates(P.make_opts(refine=small), 2, 1) == O.refine_grid(
        O.RefineOptions(half=3, rot_lo=-1.0, rot_hi=1.0, scale_step=0.02, rot_step=0.25), 1, (1.0, 0.0))


@pytest.mark.parametrize("bad", [
    dict(exclusion=9),
    dict(grid=(0, 0.9, 1.1, 5, -1, 1)),
    dict(grid=(5, 0.1, 1.1, 5, -1, 1)),
    dict(warm=True, refine={}),
    dict(refine=dict(max_iter=0)),
    dict(refine=dict(rot_step=0.0)),
    dict(refine=dict(rot_lo=2.0, rot_hi=-2.0)),
    dict(refine=dict(scale_step=0.2)),
    dict(warm=True, local=(0, 9, 0.005, 0.1)),
])
def test_option_validation_rejects(bad):
    from paper_2207_14507_amd import prnu as P
    assert P.prnu_check_opts(P.make_opts()) == P.PRNU_OK
    assert P.prnu_check_opts(P.make_opts(refine={})) == P.PRNU_OK
    assert P.prnu_check_opts(P.make_opts(**bad)) == P.PRNU_E_ARG
    assert P.lib.prnu_last_error()


def test_c_program_links_and_calls_the_host_entry_points(tmp_path):
    """A plain C99 program built against include/prnu.h and linked with libprnu.so: the
    options check, the candidate grid and the status strings work without a device, and
    prnu_create reports a missing device as PRNU_E_DEVICE (or succeeds where one exists)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    libdir = os.path.join(ROOT, "paper_2207_14507_amd")
    src = tmp_path / "client.c"
    src.write_text(r'''
#include <stdio.h>
#include <string.h>
#include "prnu.h"
int main(void) {
  prnu_search_opts o;
  memset(&o, 0, sizeof o);
  o.full.n_scale = 41; o.full.scale_lo = 0.85; o.full.scale_hi = 1.15;
  o.full.n_rot = 21; o.full.rot_lo_deg = -2.0; o.full.rot_hi_deg = 2.0;
  o.shift_radius = 64; o.exclusion = 11; o.local_n_scale = 9; o.local_n_rot = 9;
  o.local_dscale = 0.005; o.local_drot_deg = 0.1; o.fallback_pce = 60.0; o.tau = 19.5;
  if (prnu_check_opts(&o) != PRNU_OK) return 1;
  int32_t n = prnu_candidates(&o, 0, 1, 1.0, 0.0, NULL, 0);
  if (n != 861) return 2;
  double c[2 * 861];
  if (prnu_candidates(&o, 0, 1, 1.0, 0.0, c, 861) != 861) return 3;
  printf("%d %.17g %.17g %.17g %.17g\n", n, c[0], c[1], c[2 * 860], c[2 * 860 + 1]);
  o.exclusion = 9;
  if (prnu_check_opts(&o) != PRNU_E_ARG) return 4;
  if (!prnu_status_string(PRNU_E_SHAPE) || !prnu_status_string(PRNU_E_DEVICE)) return 5;
  prnu_ctx* ctx = NULL;
  prnu_status st = prnu_create(NULL, &ctx);
  if (st == PRNU_OK) prnu_destroy(ctx);
  else if (st != PRNU_E_DEVICE || ctx != NULL) return 6;
  printf("%d\n", (int)st);
  return 0;
}
''')
    exe = tmp_path / "client"
    subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src), "-L", libdir,
                    "-lprnu", f"-Wl,-rpath,{libdir}", "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, (out.returncode, out.stderr)
    first, status = out.stdout.split("\n")[:2]
    n, s0, t0, s1, t1 = first.split()
    assert int(n) == 861 and float(s0) == pytest.approx(0.85) and float(t0) == pytest.approx(-2.0)
    assert float(s1) == pytest.approx(1.15) and float(t1) == pytest.approx(2.0)
    assert int(status) in (0, -4)
