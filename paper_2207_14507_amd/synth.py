"""Seeded synthetic PRNU workloads (fingerprints, stabilised residual frames).

The paper evaluates on real stabilised videos whose fingerprints come from
flat images (Sec. 4); none of that data is available, so every input here is
synthetic with the shapes and statistics of that workload:

* fingerprint K ~ N(0, 0.02^2), float32, M rows x N columns;
* a smooth scene intensity I (Gaussian low-pass of white noise, clipped to
  [0.2, 0.9]) -- the PRNU is multiplicative (Sec. 2.2), so the frame carries
  I * K;
* a stabilised frame residual W = T_t(I * K) + N(0, 0.05^2), where T_t is the
  similarity special case of the EIS model of Eq. (4) with the parameter
  restrictions of Sec. 3.2 (t11 = t22, t12 = -t21, no projective terms) plus
  an integer translation.

This module only draws inputs.  It holds none of the search arithmetic (no
inverse warp, correlation or PCE); the forward resampling that plants the
transform is delegated to ``scipy.ndimage.map_coordinates`` (order 1, zero
outside the image).  Both the FP64 oracle and the HIP path consume these
arrays; neither is imported here.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np
from scipy import ndimage

SEED_BASE = 220714507

# Similarity-transform sampling ranges of the synthetic workloads.
FULL_SCALE = (0.85, 1.15)
FULL_ROT_DEG = (-2.0, 2.0)


def rng(config: int, *path: int) -> np.random.Generator:
    """Deterministic generator for config ``config`` and a sub-stream ``path``."""
    return np.random.default_rng(np.random.SeedSequence([SEED_BASE + int(config), *map(int, path)]))


@dataclasses.dataclass(frozen=True)
class Planted:
    """Planted forward stabilisation transform of one frame (Eq. 4, similarity form)."""
    scale: float
    rot_deg: float
    dx: int
    dy: int


def fingerprint(g: np.random.Generator, height: int, width: int, sigma: float = 0.02) -> np.ndarray:
    return (g.standard_normal((height, width)) * sigma).astype(np.float32)


def intensity(g: np.random.Generator, height: int, width: int) -> np.ndarray:
    """Smooth scene: white noise low-passed by a Gaussian of std width/32 px, standardised,
    mapped to 0.55 + 0.25 z and clipped to [0.2, 0.9]."""
    z = g.standard_normal((height, width))
    sig = width / 32.0
    fy = np.fft.fftfreq(height)[:, None]
    fx = np.fft.rfftfreq(width)[None, :]
    gain = np.exp(-2.0 * (math.pi * sig) ** 2 * (fy * fy + fx * fx))
    z = np.fft.irfft2(np.fft.rfft2(z) * gain, s=(height, width))
    z = (z - z.mean()) / max(z.std(), 1e-12)
    return np.clip(0.55 + 0.25 * z, 0.2, 0.9)


def forward_warp(img: np.ndarray, p: Planted) -> np.ndarray:
    """Stabilised frame: value at stabilised pixel q is img sampled at the original
    position s*Q(theta)(q - c) + c + d, Q(theta) = [[cos, sin], [-sin, cos]] acting on
    (column, row), c the image centre; bilinear, zero outside the image."""
    h, w = img.shape
    cx, cy = (w - 1) / 2.0, (h - 1) / 2.0
    th = math.radians(p.rot_deg)
    c, s = math.cos(th), math.sin(th)
    yy, xx = np.meshgrid(np.arange(h, dtype=np.float64), np.arange(w, dtype=np.float64), indexing="ij")
    ux, uy = xx - cx, yy - cy
    xs = p.scale * (c * ux + s * uy) + cx + p.dx
    ys = p.scale * (-s * ux + c * uy) + cy + p.dy
    return ndimage.map_coordinates(img, [ys, xs], order=1, mode="grid-constant", cval=0.0)


def forward_warp_matrix(img: np.ndarray, T: np.ndarray, dx: int, dy: int) -> np.ndarray:
    """Stabilised frame under a general Eq. (4) transform: value at stabilised pixel q is
    img sampled at pi(T (q - c, 1)) + c + d, pi(X, Y, Z) = (X/Z, Y/Z), c the image centre;
    bilinear, zero outside the image."""
    h, w = img.shape
    cx, cy = (w - 1) / 2.0, (h - 1) / 2.0
    T = np.asarray(T, dtype=np.float64)
    yy, xx = np.meshgrid(np.arange(h, dtype=np.float64), np.arange(w, dtype=np.float64), indexing="ij")
    ux, uy = xx - cx, yy - cy
    Z = T[2, 0] * ux + T[2, 1] * uy + T[2, 2]
    xs = (T[0, 0] * ux + T[0, 1] * uy + T[0, 2]) / Z + cx + dx
    ys = (T[1, 0] * ux + T[1, 1] * uy + T[1, 2]) / Z + cy + dy
    return ndimage.map_coordinates(img, [ys, xs], order=1, mode="grid-constant", cval=0.0)


def transform_sequence(config: int, size: int, planted) -> Sequence_:
    """size x size fingerprint and one frame per (T, dx, dy) general transform."""
    g = rng(config, size, 9)
    K = fingerprint(g, size, size)
    frames = []
    for f, (T, dx, dy) in enumerate(planted):
        gf = rng(config, size, 9, 1 + f)
        scene = intensity(gf, size, size)
        sig = forward_warp_matrix(scene * K.astype(np.float64), T, dx, dy)
        frames.append((sig + gf.standard_normal((size, size)) * 0.05).astype(np.float32))
    return Sequence_(K, np.stack(frames), [])


def make_frame(g: np.random.Generator, K: np.ndarray, p: Planted, noise: float = 0.05) -> np.ndarray:
    h, w = K.shape
    scene = intensity(g, h, w)
    sig = forward_warp(scene * K.astype(np.float64), p)
    return (sig + g.standard_normal((h, w)) * noise).astype(np.float32)


def grid_snap(v: float, n: int, lo: float, hi: float) -> float:
    """Nearest node of the uniform grid centre + k*step (odd n) to v."""
    centre, step = (lo + hi) / 2.0, (hi - lo) / (n - 1)
    k = int(round((v - centre) / step))
    k = max(-(n // 2), min(n // 2, k))
    return centre + k * step


def random_walk(g: np.random.Generator, n: int, radius: int, sigma_s: float = 0.003,
                sigma_t: float = 0.1, sigma_d: float = 2.0,
                s_range=FULL_SCALE, t_range=FULL_ROT_DEG) -> List[Planted]:
    """Per-frame transforms: a random walk from (1, 0 deg, 0, 0), clipped to the
    search ranges and the shift radius."""
    s, t, dx, dy = 1.0, 0.0, 0, 0
    out = []
    for _ in range(n):
        s = float(np.clip(s + g.normal(0.0, sigma_s), *s_range))
        t = float(np.clip(t + g.normal(0.0, sigma_t), *t_range))
        dx = int(np.clip(dx + int(round(g.normal(0.0, sigma_d))), -radius, radius))
        dy = int(np.clip(dy + int(round(g.normal(0.0, sigma_d))), -radius, radius))
        out.append(Planted(s, t, dx, dy))
    return out


# ----------------------------------------------------------------------------
# BF16 residual storage with a per-frame power-of-two scale.

def quantize_bf16(W: np.ndarray) -> Tuple[np.ndarray, float]:
    """sigma = smallest power of two >= max|W|; w = round-to-nearest-even bf16 of
    W / sigma (an exact division).  Returns (uint16 bit patterns, sigma)."""
    m = float(np.max(np.abs(W))) if W.size else 0.0
    sigma = 1.0 if m == 0.0 else float(2.0 ** math.ceil(math.log2(m)))
    x = (W.astype(np.float32) / np.float32(sigma)).astype(np.float32)
    bits = x.view(np.uint32).astype(np.uint64)
    bits = (bits + 0x7FFF + ((bits >> 16) & 1)) >> 16
    return bits.astype(np.uint16), sigma


def dequantize_bf16(bits: np.ndarray, sigma: float) -> np.ndarray:
    """Exact float32 value sigma * w of stored bf16 residuals."""
    f = (bits.astype(np.uint32) << 16).view(np.float32)
    return (f * np.float32(sigma)).astype(np.float32)


# ----------------------------------------------------------------------------
# Workloads.

@dataclasses.dataclass
class Sequence_:
    K: np.ndarray                 # fingerprint, float32 (M, N)
    frames: np.ndarray            # residuals, float32 (F, M, N)
    planted: List[Planted]
    bf16: np.ndarray | None = None        # uint16 (F, M, N) when stored in bf16
    bf16_scale: np.ndarray | None = None  # float32 (F,)
    offset: Tuple[int, int] = (0, 0)      # (row, column) of the frames' crop inside K


def tiny(n_frames: int = 4, size: int = 256, snap: bool = False, config: int = 1,
         grid=(11, 0.95, 1.05, 11, -2.0, 2.0), max_shift: int = 8) -> Sequence_:
    """256x256 parity workload: planted s in U[0.95,1.05], theta in U[-2,2] deg,
    dx, dy in U{-8..8}; with ``snap`` the (s, theta) are moved to grid nodes."""
    g = rng(config, size, int(snap))
    K = fingerprint(g, size, size)
    planted, frames = [], []
    ns, slo, shi, nt, tlo, thi = grid
    for f in range(n_frames):
        gf = rng(config, size, int(snap), 1 + f)
        s = float(gf.uniform(slo, shi))
        t = float(gf.uniform(tlo, thi))
        if snap:
            s, t = grid_snap(s, ns, slo, shi), grid_snap(t, nt, tlo, thi)
        p = Planted(s, t, int(gf.integers(-max_shift, max_shift + 1)), int(gf.integers(-max_shift, max_shift + 1)))
        planted.append(p)
        frames.append(make_frame(gf, K, p))
    return Sequence_(K, np.stack(frames), planted)


def planted_sequence(config: int, size: int, planted: Sequence[Planted]) -> Sequence_:
    """size x size fingerprint and one frame per given transform (seeded by config)."""
    g = rng(config, size, 7)
    K = fingerprint(g, size, size)
    frames = [make_frame(rng(config, size, 7, 1 + f), K, p) for f, p in enumerate(planted)]
    return Sequence_(K, np.stack(frames), list(planted))


def walk_sequence(config: int, seq: int, height: int, width: int, n_frames: int, radius: int = 64,
                  unwarped: Sequence[int] = (), independent_fp: bool = False, first: int = 0,
                  count: int | None = None) -> Sequence_:
    """Frames following a random walk of transforms; frames listed in ``unwarped`` carry
    no transform (s=1, theta=0, d=0) while the walk continues underneath.  With
    ``independent_fp`` the frames are generated from an independent fingerprint
    (non-matching case) while ``K`` is still the tested one.  ``first``/``count`` draw
    only frames first .. first + count - 1 of the same n_frames walk (each frame has its
    own seed, so the pieces of a long walk can be drawn in parallel)."""
    g = rng(config, seq, height, width)
    K = fingerprint(g, height, width)
    Ksrc = fingerprint(rng(config, seq, height, width, 99), height, width) if independent_fp else K
    walk = random_walk(rng(config, seq, 7), n_frames, radius)
    last = n_frames if count is None else min(n_frames, first + count)
    planted, frames = [], []
    for f, p in enumerate(walk):
        if f < first or f >= last:
            continue
        if f in unwarped:
            p = Planted(1.0, 0.0, 0, 0)
        planted.append(p)
        frames.append(make_frame(rng(config, seq, 100 + f), Ksrc, p))
    return Sequence_(K, np.stack(frames), planted)


def hd_sequence(n_frames: int = 30) -> Sequence_:
    """1080p workload: 1080x1920, 30 walk frames, three seeded frames (of the 30) unwarped;
    a shorter sequence is a prefix of the same walk."""
    idx = rng(2, 5).choice(30, size=3, replace=False)
    return walk_sequence(2, 0, 1080, 1920, n_frames, unwarped=set(int(i) for i in idx))


def mixed_sequences(frames_per_seq: int = 8) -> List[Sequence_]:
    """Batched warm-start workload: 8 sequences (3 x 720p, 4 x 1080p, 1 x 4K) with
    their own fingerprints."""
    shapes = [(720, 1280)] * 3 + [(1080, 1920)] * 4 + [(2160, 3840)]
    return [walk_sequence(3, i, h, w, frames_per_seq) for i, (h, w) in enumerate(shapes)]


def uhd_bf16_sequence(n_frames: int = 16) -> Sequence_:
    """Precision workload: 2160x3840 fingerprint, 16 walk frames stored in bf16."""
    s = walk_sequence(4, 0, 2160, 3840, n_frames)
    q = [quantize_bf16(f) for f in s.frames]
    s.bf16 = np.stack([b for b, _ in q])
    s.bf16_scale = np.array([sc for _, sc in q], dtype=np.float32)
    return s


def cropped_sequence(config: int, fp_shape: Tuple[int, int], frame_shape: Tuple[int, int], n_frames: int,
                     radius: int = 64, planted: Sequence[Planted] | None = None,
                     offset: Tuple[int, int] | None = None) -> Sequence_:
    """Frames smaller than the fingerprint: the sensor area they see is the crop of K at a
    seeded offset (row, column) in [0, M - M'] x [0, N - N'], and each frame is that crop
    of I * K under a planted transform about the frame's own centre, plus noise.  With no
    ``planted`` list the transforms follow the random walk of the 1080p workload."""
    (M, N), (Mf, Nf) = fp_shape, frame_shape
    if Mf > M or Nf > N:
        raise ValueError("frames must not be larger than the fingerprint")
    g = rng(config, M, N, Mf, Nf)
    K = fingerprint(g, M, N)
    if offset is None:
        offset = (int(g.integers(0, M - Mf + 1)), int(g.integers(0, N - Nf + 1)))
    oy, ox = offset
    crop = K[oy:oy + Mf, ox:ox + Nf]
    if planted is None:
        planted = random_walk(rng(config, M, N, Mf, Nf, 7), n_frames, radius)
    frames = [make_frame(rng(config, M, N, Mf, Nf, 100 + f), crop, p) for f, p in enumerate(planted)]
    return Sequence_(K, np.stack(frames), list(planted), offset=(oy, ox))
