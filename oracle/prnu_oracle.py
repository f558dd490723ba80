"""FP64 CPU oracle of the EIS-inversion grid search -- TEST INFRASTRUCTURE ONLY.

Only the tests, the package's ``smoke()`` check and the benchmark's CPU-baseline
leg may import this module.  It is a plain, slow, obviously correct restatement
of what the search computes, written from the paper (arXiv 2207.14507) and kept
independent of the GPU library: the two share no code, headers, tables or
helpers.

What it computes, per frame and candidate (scale s, rotation theta):

1. Mean-free fingerprint and its norm -- the NCC of Eq. (1).
2. Inverse of the similarity form of the EIS transform (Eq. (4) restricted as in
   Sec. 3.2: t11 = t22 = s cos(theta), t12 = -t21 = s sin(theta), t31 = t32 = 0):
   the residual is resampled bilinearly at B(q) = Q(-theta)(q - c)/s + c, with
   taps outside the image contributing zero.
3. Circular cross-correlation C(delta) = sum_p Kt[p] Rt[p - delta] over all M*N
   shifts (Eq. (1) evaluated at every shift; the FFT is only a faster route to the
   same sum and is pinned against the direct sum by the tests).
4. Peak-to-Correlation Energy of Eq. (3): signed peak within the shift radius,
   11x11 cyclic exclusion neighbourhood, off-peak energy summed directly.
5. Argmax over the candidate grid (the exhaustive step of CORRECTION, Sec. 3.2).
6. Warm start of consecutive frames around the previous estimate (Algorithm 1
   chains each frame's correction to the previous one; Sec. 3.2 starts the search
   from T_init) with a fallback to the full grid, and the video decision of Sec. 3.2
   (threshold on the mean of gamma).
7. The paper's own coarse-to-fine schedule of CORRECTION (Sec. 3.2, Eq. (8)): a
   dense first pass, then narrower grids around each estimate until it repeats.
8. The general 8-parameter form of Eq. (4), and the reference fingerprint of Eq. (2)
   from images and their residuals.
9. Frames smaller than the fingerprint (Sec. 2): the warped frame is zero-padded to
   the fingerprint's size and the peak is sought over the linear shifts
   0 <= delta <= (M - M', N - N') of Eq. (3), widened by the shift radius.

Readings of points the paper leaves open (angle units, rotation centre,
interpolation, shift domain, peak definition, tie rules, grid nodes, fallback)
are the ones listed in the design notes; each is restated where it is used.

Parity status: every function below is pinned by a CPU test (direct-sum
correlation, closed-form warps, closed-form PCE surfaces, planted-transform
recovery, identity rule).  The paper prints no worked example, so no value of
the paper itself pins the absolute PCE level.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

EXCLUSION = 11  # side of the cyclic exclusion neighbourhood D around the peak (Eq. 3)


# ---------------------------------------------------------------------------
# Eq. (1): mean-free operands and their norms.

def mean_free(X: np.ndarray) -> Tuple[np.ndarray, float]:
    """X - mean(X) over all elements, and its Euclidean norm (FP64)."""
    X = np.asarray(X, dtype=np.float64)
    Xt = X - X.mean()
    return Xt, float(math.sqrt(float(np.sum(Xt * Xt))))


# ---------------------------------------------------------------------------
# Eq. (2): the reference fingerprint from L images of the device.

def estimate_fingerprint(images: np.ndarray, residuals: np.ndarray) -> np.ndarray:
    """K = (sum_l I_l W_l) / (sum_l I_l I_l), pixel-wise, in FP64, from L images I_l and
    their noise residuals W_l = I_l - F(I_l) (the denoiser F is the caller's).  A pixel
    whose images are all zero has no estimate: it is set to 0."""
    I = np.asarray(images, dtype=np.float64)
    W = np.asarray(residuals, dtype=np.float64)
    num = np.zeros(I.shape[1:], dtype=np.float64)
    den = np.zeros(I.shape[1:], dtype=np.float64)
    for l in range(I.shape[0]):
        num += I[l] * W[l]
        den += I[l] * I[l]
    out = np.zeros_like(num)
    nz = den > 0
    out[nz] = num[nz] / den[nz]
    return out


# ---------------------------------------------------------------------------
# Candidate grids (the sets Lambda x Theta searched exhaustively in Sec. 3.2).

def grid_values(n: int, lo: float, hi: float) -> np.ndarray:
    """n uniform nodes over [lo, hi] generated as centre + k*step, k = -(n-1)/2..(n-1)/2,
    so that the centre is an exact node (n odd).  n == 1 gives the centre."""
    if n < 1:
        raise ValueError("grid needs at least one node")
    centre = (lo + hi) / 2.0
    step = (hi - lo) / (n - 1) if n > 1 else 0.0
    half = (n - 1) / 2.0
    return np.array([centre + (k - half) * step for k in range(n)], dtype=np.float64)


def local_values(centre: float, n: int, step: float) -> np.ndarray:
    """n nodes centre + (k - (n-1)/2)*step around a previous estimate (not clamped)."""
    half = (n - 1) / 2.0
    return np.array([centre + (k - half) * step for k in range(n)], dtype=np.float64)


def candidates(scales: Sequence[float], rots_deg: Sequence[float]) -> List[Tuple[float, float]]:
    """Scale-major, rotation-minor enumeration; the index in this list is the
    candidate index used for tie-breaking."""
    return [(float(s), float(t)) for s in scales for t in rots_deg]


# ---------------------------------------------------------------------------
# Eq. (4), similarity form: inverse warp of the residual.

def sample_points(height: int, width: int, scale: float, rot_deg: float) -> Tuple[np.ndarray, np.ndarray]:
    """B(q) for every output pixel q = (x = column, y = row): the inverse of the forward
    hypothesis T(p) = s Q(theta)(p - c) + c, Q(theta) = [[cos, sin], [-sin, cos]],
    about the image centre c = ((N-1)/2, (M-1)/2); theta in degrees."""
    th = math.radians(rot_deg)
    ct, st = math.cos(th), math.sin(th)
    cx, cy = (width - 1) / 2.0, (height - 1) / 2.0
    yy, xx = np.meshgrid(np.arange(height, dtype=np.float64), np.arange(width, dtype=np.float64),
                         indexing="ij")
    ux, uy = xx - cx, yy - cy
    bx = (ct * ux - st * uy) / scale + cx
    by = (st * ux + ct * uy) / scale + cy
    return bx, by


def inverse_warp(W: np.ndarray, scale: float, rot_deg: float) -> np.ndarray:
    """R(q) = bilinear interpolation of W at B(q); each of the four taps that falls
    outside the image contributes zero (the frame is zero-extended, consistent with the
    zero-padding convention that follows Eq. (1))."""
    W = np.asarray(W, dtype=np.float64)
    M, N = W.shape
    bx, by = sample_points(M, N, scale, rot_deg)
    return bilinear_zero(W, bx, by)


# ---------------------------------------------------------------------------
# Eq. (4), general 8-parameter form.

def similarity_matrix(scale: float, rot_deg: float) -> np.ndarray:
    """The similarity hypothesis as an Eq. (4) matrix in centred coordinates (origin at
    the image centre): t11 = t22 = s cos(theta), t12 = -t21 = s sin(theta), t31 = t32 = 0."""
    th = math.radians(rot_deg)
    c, s_ = scale * math.cos(th), scale * math.sin(th)
    return np.array([[c, s_, 0.0], [-s_, c, 0.0], [0.0, 0.0, 1.0]], dtype=np.float64)


def similarity_of(T: np.ndarray) -> Tuple[float, float]:
    """The (scale, rotation) nearest to the linear part of T: theta from the rotation
    that best aligns it, s from the square root of its determinant (the starting point
    (lambda^(0), theta^(0)) of the refinement taken from an initial transform)."""
    T = np.asarray(T, dtype=np.float64)
    th = math.atan2(T[0, 1] - T[1, 0], T[0, 0] + T[1, 1])
    det = T[0, 0] * T[1, 1] - T[0, 1] * T[1, 0]
    return math.sqrt(abs(det)), math.degrees(th)


def sample_points_matrix(height: int, width: int, T: np.ndarray) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """B(q) = pi(T^-1 (q - c, 1)) + c for a general Eq. (4) transform T (3 x 3,
    stabilised -> original, centred coordinates), pi(X, Y, Z) = (X / Z, Y / Z).  Output
    pixels whose homogeneous coordinate Z is not positive lie beyond the projective
    horizon: they are returned as invalid."""
    G = np.linalg.inv(np.asarray(T, dtype=np.float64))
    cx, cy = (width - 1) / 2.0, (height - 1) / 2.0
    yy, xx = np.meshgrid(np.arange(height, dtype=np.float64), np.arange(width, dtype=np.float64),
                         indexing="ij")
    ux, uy = xx - cx, yy - cy
    X = G[0, 0] * ux + G[0, 1] * uy + G[0, 2]
    Y = G[1, 0] * ux + G[1, 1] * uy + G[1, 2]
    Z = G[2, 0] * ux + G[2, 1] * uy + G[2, 2]
    valid = Z > 0
    Zs = np.where(valid, Z, 1.0)
    return X / Zs + cx, Y / Zs + cy, valid


def inverse_warp_matrix(W: np.ndarray, T: np.ndarray) -> np.ndarray:
    """The inverse warp of Eq. (4) for a general transform: bilinear at B(q), taps outside
    the image and points beyond the horizon contribute zero."""
    W = np.asarray(W, dtype=np.float64)
    M, N = W.shape
    bx, by, valid = sample_points_matrix(M, N, T)
    out = bilinear_zero(W, np.where(valid, bx, -10.0), np.where(valid, by, -10.0))
    return np.where(valid, out, 0.0)


def bilinear_zero(W: np.ndarray, bx: np.ndarray, by: np.ndarray) -> np.ndarray:
    """Bilinear interpolation of W at (bx, by) with the four taps explicit; a tap outside
    the image contributes zero."""
    M, N = W.shape
    x0 = np.floor(bx)
    y0 = np.floor(by)
    fx = bx - x0
    fy = by - y0
    x0 = x0.astype(np.int64)
    y0 = y0.astype(np.int64)
    out = np.zeros((M, N), dtype=np.float64)
    for ox, oy, wgt in ((0, 0, (1 - fx) * (1 - fy)), (1, 0, fx * (1 - fy)),
                        (0, 1, (1 - fx) * fy), (1, 1, fx * fy)):
        xi = x0 + ox
        yi = y0 + oy
        inside = (xi >= 0) & (xi < N) & (yi >= 0) & (yi < M)
        vals = np.zeros((M, N), dtype=np.float64)
        vals[inside] = W[yi[inside], xi[inside]]
        out += wgt * vals
    return out


# ---------------------------------------------------------------------------
# Eq. (1) at every circular shift.

def circular_xcorr(Kt: np.ndarray, Rt: np.ndarray) -> np.ndarray:
    """C[dy, dx] = sum_p Kt[p] * Rt[(p - delta) mod (M, N)], for every shift; array index
    (dy mod M, dx mod N).  Computed as IDFT2(DFT2(Kt) * conj(DFT2(Rt))) in FP64."""
    Kt = np.asarray(Kt, dtype=np.float64)
    Rt = np.asarray(Rt, dtype=np.float64)
    return np.real(np.fft.ifft2(np.fft.fft2(Kt) * np.conj(np.fft.fft2(Rt))))


# ---------------------------------------------------------------------------
# Eq. (3): Peak-to-Correlation Energy.

@dataclasses.dataclass
class PCEResult:
    pce: float
    peak: float     # C at the peak
    dx: int         # peak shift, column direction (signed)
    dy: int         # peak shift, row direction (signed)
    energy: float   # sum of C^2 over shifts outside D
    runner_up: float = -math.inf  # largest C in the search window at any other shift


def pce_from_surface(C: np.ndarray, radius: int, exclusion: int = EXCLUSION,
                     extent: Tuple[int, int] = (0, 0)) -> PCEResult:
    """Peak = signed maximum of C over -radius <= dy <= extent[0] + radius and
    -radius <= dx <= extent[1] + radius, first in row-major order from (-radius, -radius)
    on ties.  extent = (M - M', N - N') is the range of linear shifts of a smaller,
    zero-padded frame inside the fingerprint (Eq. 3 with frames of M' x N'); it is
    (0, 0) for equal sizes, where the window is |dy|, |dx| <= radius.
    D = peak +- exclusion//2 (indices mod M, N).
    PCE = sgn(C_pk) C_pk^2 / (sum_{delta not in D} C^2 / (M N - |D|)), the energy taken
    over all M N circular shifts.
    The common normalisation of rho cancels, so PCE depends on C only.  A surface with
    zero off-peak energy gives PCE 0."""
    M, N = C.shape
    ey, ex = extent
    best, bdy, bdx, second = -math.inf, 0, 0, -math.inf
    for dy in range(-radius, ey + radius + 1):
        for dx in range(-radius, ex + radius + 1):
            v = float(C[dy % M, dx % N])
            if v > best:
                best, bdy, bdx, second = v, dy, dx, best
            elif v > second:
                second = v
    h = exclusion // 2
    mask = np.ones((M, N), dtype=bool)
    for a in range(-h, h + 1):
        for b in range(-h, h + 1):
            mask[(bdy + a) % M, (bdx + b) % N] = False
    n_out = M * N - exclusion * exclusion
    energy = float(np.sum(C[mask] ** 2))
    if energy <= 0.0:
        return PCEResult(0.0, best, bdx, bdy, energy, second)
    pce = math.copysign(best * best, best) / (energy / n_out)
    return PCEResult(pce, best, bdx, bdy, energy, second)


# ---------------------------------------------------------------------------
# One candidate, one frame, one video.

@dataclasses.dataclass
class CandidateResult:
    scale: float
    rot_deg: float
    pce: float
    rho: float      # NCC at the peak, Eq. (1)
    dx: int
    dy: int
    peak: float
    runner_up: float = -math.inf  # second largest C in the search window


def zero_pad(R: np.ndarray, height: int, width: int) -> np.ndarray:
    """A frame smaller than the fingerprint, zero-padded to the fingerprint's size
    (Sec. 2, after Eq. (1)): the frame keeps rows 0..M'-1 and columns 0..N'-1 and every
    other element is zero."""
    Mf, Nf = R.shape
    if Mf > height or Nf > width:
        raise ValueError(f"frame {Mf}x{Nf} is larger than the fingerprint {height}x{width}")
    P = np.zeros((height, width), dtype=np.float64)
    P[:Mf, :Nf] = R
    return P


def _surface(K: np.ndarray, R: np.ndarray, Kt_norm) -> Tuple[np.ndarray, Tuple[int, int], float, float]:
    """Eq. (1) at every shift for a warped frame R of M' x N' <= K's M x N: the frame is
    zero-padded to M x N, both operands are made mean-free over all M N elements.
    Returns C, the linear-shift extent (M - M', N - N') and the two norms."""
    Kt, kn = Kt_norm if Kt_norm is not None else mean_free(K)
    M, N = Kt.shape
    extent = (M - R.shape[0], N - R.shape[1])
    if R.shape != (M, N):
        R = zero_pad(R, M, N)
    Rt, rn = mean_free(R)
    return circular_xcorr(Kt, Rt), extent, kn, rn


def _score(K: np.ndarray, R: np.ndarray, radius: int, Kt_norm) -> Tuple[PCEResult, float]:
    """Eq. (1) at every shift and Eq. (3) for a warped frame R of M' x N' <= K's M x N,
    the peak sought over the linear shifts widened by the radius."""
    C, extent, kn, rn = _surface(K, R, Kt_norm)
    p = pce_from_surface(C, radius, extent=extent)
    rho = p.peak / (kn * rn) if kn > 0 and rn > 0 else 0.0
    return p, rho


def pce_at_shift(C: np.ndarray, dy: int, dx: int, exclusion: int = EXCLUSION) -> float:
    """Eq. (3) with the peak taken at the shift (dy, dx) whatever its rank: sgn(C) C^2 over
    the mean of C^2 outside the cyclic exclusion block centred there.  At the signed
    maximum this is the PCE of pce_from_surface; at another shift it is the score a search
    reports had it resolved a near-tie of the peak (two shifts whose correlations agree to
    within the rounding of the arithmetic) the other way."""
    M, N = C.shape
    h = exclusion // 2
    mask = np.ones((M, N), dtype=bool)
    for a in range(-h, h + 1):
        for b in range(-h, h + 1):
            mask[(dy + a) % M, (dx + b) % N] = False
    energy = float(np.sum(C[mask] ** 2))
    if energy <= 0.0:
        return 0.0
    v = float(C[dy % M, dx % N])
    return math.copysign(v * v, v) / (energy / (M * N - exclusion * exclusion))


@dataclasses.dataclass
class NearPeak:
    dx: int
    dy: int
    value: float  # C at this shift
    pce: float    # Eq. (3) with the peak taken here


def near_peak_shifts(C: np.ndarray, radius: int, rel: float, extent: Tuple[int, int] = (0, 0),
                     exclusion: int = EXCLUSION) -> List[NearPeak]:
    """Every shift of the peak window (the one pce_from_surface searches) whose C is at
    least peak - rel * |peak|, in decreasing order of C (row-major order from (-radius,
    -radius) among equal values), each with its PCE by pce_at_shift.  The first entry is
    the peak itself.  With rel of the order of the arithmetic's rounding this is the set
    of shifts an implementation may legitimately report as the peak."""
    M, N = C.shape
    ey, ex = extent
    vals = []
    for dy in range(-radius, ey + radius + 1):
        for dx in range(-radius, ex + radius + 1):
            vals.append((float(C[dy % M, dx % N]), dy, dx))
    peak = max(v for v, _, _ in vals)
    floor = peak - rel * abs(peak)
    near = [(v, dy, dx) for v, dy, dx in vals if v >= floor]
    near.sort(key=lambda t: -t[0])  # stable: row-major order kept among equal values
    return [NearPeak(dx, dy, v, pce_at_shift(C, dy, dx, exclusion)) for v, dy, dx in near]


def transform_near_peaks(K: np.ndarray, W: np.ndarray, T: np.ndarray, radius: int, rel: float,
                         Kt_norm: Optional[Tuple[np.ndarray, float]] = None
                         ) -> Tuple[CandidateResult, List[NearPeak]]:
    """evaluate_transform together with near_peak_shifts of the same correlation surface."""
    C, extent, kn, rn = _surface(K, inverse_warp_matrix(W, T), Kt_norm)
    p = pce_from_surface(C, radius, extent=extent)
    rho = p.peak / (kn * rn) if kn > 0 and rn > 0 else 0.0
    res = CandidateResult(math.nan, math.nan, p.pce, rho, p.dx, p.dy, p.peak, p.runner_up)
    return res, near_peak_shifts(C, radius, rel, extent)


def candidate_near_peaks(K: np.ndarray, W: np.ndarray, scale: float, rot_deg: float, radius: int, rel: float,
                         Kt_norm: Optional[Tuple[np.ndarray, float]] = None
                         ) -> Tuple[CandidateResult, List[NearPeak]]:
    """evaluate_candidate together with near_peak_shifts of the same correlation surface."""
    C, extent, kn, rn = _surface(K, inverse_warp(W, scale, rot_deg), Kt_norm)
    p = pce_from_surface(C, radius, extent=extent)
    rho = p.peak / (kn * rn) if kn > 0 and rn > 0 else 0.0
    res = CandidateResult(scale, rot_deg, p.pce, rho, p.dx, p.dy, p.peak, p.runner_up)
    return res, near_peak_shifts(C, radius, rel, extent)


def evaluate_transform(K: np.ndarray, W: np.ndarray, T: np.ndarray, radius: int,
                       Kt_norm: Optional[Tuple[np.ndarray, float]] = None) -> CandidateResult:
    """PCE of one general Eq. (4) transform hypothesis (scale and rotation reported as NaN)."""
    p, rho = _score(K, inverse_warp_matrix(W, T), radius, Kt_norm)
    return CandidateResult(math.nan, math.nan, p.pce, rho, p.dx, p.dy, p.peak, p.runner_up)


def evaluate_candidate(K: np.ndarray, W: np.ndarray, scale: float, rot_deg: float,
                       radius: int, Kt_norm: Optional[Tuple[np.ndarray, float]] = None) -> CandidateResult:
    """PCE(K, T_t(W)) of one (scale, rotation) hypothesis, translation found as the
    correlation peak within the shift radius.  A frame smaller than K is warped about
    its own centre and then zero-padded (see _score); the peak's (dx, dy) is then the
    frame's position inside the fingerprint."""
    p, rho = _score(K, inverse_warp(W, scale, rot_deg), radius, Kt_norm)
    return CandidateResult(scale, rot_deg, p.pce, rho, p.dx, p.dy, p.peak, p.runner_up)


@dataclasses.dataclass
class FrameResult:
    index: int                 # candidate index of the winner in the evaluated list
    best: CandidateResult
    all: List[CandidateResult]
    fell_back: bool = False

    @property
    def pce(self) -> float:
        return self.best.pce


def argmax_first(values: Sequence[float]) -> int:
    """Index of the maximum, lowest index on ties."""
    bi, bv = 0, -math.inf
    for i, v in enumerate(values):
        if v > bv:
            bi, bv = i, v
    return bi


def search_frame(K: np.ndarray, W: np.ndarray, cands: Sequence[Tuple[float, float]], radius: int,
                 Kt_norm=None) -> FrameResult:
    """Exhaustive evaluation of every candidate and the argmax of PCE (CORRECTION's
    inner step, Sec. 3.2)."""
    Kt_norm = Kt_norm if Kt_norm is not None else mean_free(K)
    res = [evaluate_candidate(K, W, s, t, radius, Kt_norm) for s, t in cands]
    i = argmax_first([r.pce for r in res])
    return FrameResult(i, res[i], res)


@dataclasses.dataclass
class WarmOptions:
    """Full grid, shift radius and the warm-start parameters of the batched workload."""
    n_scale: int = 41
    scale_lo: float = 0.85
    scale_hi: float = 1.15
    n_rot: int = 21
    rot_lo: float = -2.0
    rot_hi: float = 2.0
    radius: int = 64
    warm: bool = True
    local_n_scale: int = 9
    local_n_rot: int = 9
    local_dscale: float = 0.005
    local_drot: float = 0.1
    fallback_pce: float = 60.0
    init: Optional[Tuple[float, float]] = None
    tau: float = 19.5


def full_grid(o: WarmOptions) -> List[Tuple[float, float]]:
    return candidates(grid_values(o.n_scale, o.scale_lo, o.scale_hi), grid_values(o.n_rot, o.rot_lo, o.rot_hi))


def local_grid(o: WarmOptions, centre: Tuple[float, float]) -> List[Tuple[float, float]]:
    return candidates(local_values(centre[0], o.local_n_scale, o.local_dscale),
                      local_values(centre[1], o.local_n_rot, o.local_drot))


def search_video(K: np.ndarray, frames: Sequence[np.ndarray], o: WarmOptions) -> List[FrameResult]:
    """Frame-by-frame search chained as in Algorithm 1 (each corrected frame seeds the
    next).  Without warm start every frame uses the full grid.  With warm start, a frame
    with a previous estimate (or T_init for the first frame) searches the local grid
    centred on it; when that local best has PCE below the fallback level, the full grid
    is searched as well and the result is the maximum over local followed by full (local
    wins ties).  The next frame centres on the result."""
    Kt_norm = mean_free(K)
    out: List[FrameResult] = []
    centre = o.init
    for W in frames:
        if not o.warm or centre is None:
            fr = search_frame(K, W, full_grid(o), o.radius, Kt_norm)
        else:
            loc = local_grid(o, centre)
            fr = search_frame(K, W, loc, o.radius, Kt_norm)
            if fr.pce < o.fallback_pce:
                full = search_frame(K, W, full_grid(o), o.radius, Kt_norm)
                allr = fr.all + full.all
                i = argmax_first([r.pce for r in allr])
                fr = FrameResult(i, allr[i], allr, fell_back=True)
        out.append(fr)
        centre = (fr.best.scale, fr.best.rot_deg)
    return out


# ---------------------------------------------------------------------------
# The paper's own coarse-to-fine schedule of CORRECTION (Sec. 3.2, Eq. (8)).

@dataclasses.dataclass
class RefineOptions:
    """Breadth-first refinement of Sec. 3.2.  Iteration n searches every pair of
    Lambda^(n) x Theta^(n), where each set is the previous estimate plus alpha * step_n
    for integer alpha in [-half, half].  The steps printed in Eq. (8) are garbled (they
    would grow with n although the text calls the sets progressively narrower); they are
    read as scale_step * 10^-(n-1) and rot_step * 10^-(n-1), i.e. 0.01 and 0.1 at n = 1,
    ten times finer at each further iteration.  At n = 1 the rotation set is the dense
    absolute grid {rot_lo, rot_lo + rot_step, ..., rot_hi} (the paper's {-5, -4.9, ...,
    5}).  The start (lambda^(0), theta^(0)) is (1, 0) or the given initial transform.
    The search stops when an iteration's estimate equals the previous one, or after
    max_iter iterations; gamma is the largest PCE observed."""
    half: int = 5
    scale_step: float = 0.01
    rot_step: float = 0.1
    rot_lo: float = -5.0
    rot_hi: float = 5.0
    max_iter: int = 3
    radius: int = 64
    init_scale: float = 1.0
    init_rot: float = 0.0


def refine_grid(o: RefineOptions, n: int, centre: Tuple[float, float]) -> List[Tuple[float, float]]:
    """Lambda^(n) x Theta^(n), scale-major."""
    factor = 10.0 ** (-(n - 1))
    scales = local_values(centre[0], 2 * o.half + 1, o.scale_step * factor)
    if n == 1:
        n_rot = int(round((o.rot_hi - o.rot_lo) / o.rot_step)) + 1
        rots = grid_values(n_rot, o.rot_lo, o.rot_hi)
    else:
        rots = local_values(centre[1], 2 * o.half + 1, o.rot_step * factor)
    return candidates(scales, rots)


@dataclasses.dataclass
class RefineResult:
    best: CandidateResult        # the candidate with the largest PCE over all iterations
    index: int                   # its index in the concatenation of the iterations' lists
    estimates: List[Tuple[float, float]]  # (lambda^(n), theta^(n)) for n = 1, 2, ...
    all: List[CandidateResult]   # every evaluated candidate, iterations in order

    @property
    def n_evaluated(self) -> int:
        return len(self.all)

    @property
    def pce(self) -> float:
        return self.best.pce

    @property
    def iterations(self) -> int:
        return len(self.estimates)


def refine_frame(K: np.ndarray, W: np.ndarray, o: RefineOptions, Kt_norm=None) -> RefineResult:
    """CORRECTION's schedule on one frame: exhaustive search of each iteration's grid,
    the next grid centred on the iteration's argmax (lowest index on ties), stop on a
    repeated estimate or after max_iter iterations."""
    Kt_norm = Kt_norm if Kt_norm is not None else mean_free(K)
    centre = (o.init_scale, o.init_rot)
    evaluated: List[CandidateResult] = []
    estimates: List[Tuple[float, float]] = []
    for n in range(1, o.max_iter + 1):
        fr = search_frame(K, W, refine_grid(o, n, centre), o.radius, Kt_norm)
        evaluated.extend(fr.all)
        est = (fr.best.scale, fr.best.rot_deg)
        estimates.append(est)
        if est == centre:
            break
        centre = est
    i = argmax_first([r.pce for r in evaluated])
    return RefineResult(evaluated[i], i, estimates, evaluated)


def video_decision(gammas: Sequence[float], tau: float) -> Tuple[float, bool]:
    """Sec. 3.2: decide H1 when the mean of the per-frame maximum PCE exceeds tau."""
    m = float(np.mean(np.asarray(gammas, dtype=np.float64))) if len(gammas) else 0.0
    return m, m > tau
