"""FP64 CPU oracle of the noise-residual extraction W(I) = I - F(I) -- TEST INFRASTRUCTURE ONLY.

Only the tests, the package's ``smoke()`` check and the benchmark's CPU-baseline leg may
import this module.  It shares no code, tables or constants with the GPU library.

The paper (Sec. 2, before Eq. (2)) defines the residual as the image minus its denoised
version, with F the wavelet denoiser of Mihcak, Kozintsev, Ramchandran and Moulin, and
gives no further detail.  This module follows that denoiser as PRNU work applies it:

1. A 4-level orthonormal 2-D wavelet decomposition with the 8-tap Daubechies filter
   (4 vanishing moments, minimum phase), periodic at the borders.
2. For every coefficient c of every detail subband, the local signal variance
   v = max(0, min over W in {3, 5, 7, 9} of mean(c^2 over the W x W window) - s0^2),
   the window zero outside the subband, s0 the noise standard deviation.
3. The denoised coefficient is the Wiener estimate c v / (v + s0^2); the noise residual
   keeps c s0^2 / (v + s0^2) in every detail subband and nothing of the coarsest
   approximation, so that the inverse transform of the residual coefficients is
   I - F(I) exactly (the transform is linear and orthonormal).

Readings of points the paper leaves open, stated where used: an image whose sides are
not multiples of 2^4 is extended by mirroring its last rows and columns (without
repeating the edge) and the residual is cropped back; s0 is a caller parameter (3 for
intensities in [0, 255]); analysis is correlation with the filter at even offsets.

Parity status: pinned by the filter's defining properties and its published values,
perfect reconstruction and energy preservation of the transform, closed-form subbands
of an impulse and of a constant, brute-force local variances, and the limits s0 -> 0
(no residual) and s0 -> infinity (every detail coefficient).  No value of the paper
pins the residual itself.
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np

LEVELS = 4
WINDOWS = (3, 5, 7, 9)


# ---------------------------------------------------------------------------
# The 8-tap Daubechies filter, by spectral factorisation.

def daubechies_lowpass(vanishing: int = 4) -> np.ndarray:
    """Minimum-phase orthonormal Daubechies lowpass filter with `vanishing` vanishing
    moments (2 * vanishing taps), sum sqrt(2).

    |H(w)|^2 = 2 cos^{2p}(w/2) P(sin^2(w/2)) with P(y) = sum_{k<p} C(p-1+k, k) y^k.
    With y = (2 - z - 1/z)/4, the roots of z^{p-1} P(y(z)) come in pairs (r, 1/r); H
    takes the roots inside the unit circle and p zeros at z = -1."""
    p = vanishing
    # P(y) as a polynomial in y, then y = (2 - z - z^-1)/4 substituted: multiply by
    # z^{p-1} to get an ordinary polynomial of degree 2(p-1) in z
    P = [math.comb(p - 1 + k, k) for k in range(p)]
    poly = np.zeros(2 * p - 1)
    base = np.array([-0.25, 0.5, -0.25])       # z * y(z) = (-z^2 + 2 z - 1)/4, highest power first
    for k, ck in enumerate(P):
        term = np.array([1.0])
        for _ in range(k):
            term = np.convolve(term, base)
        # term is z^k y^k (degree 2k); scale to z^{p-1} y^k: multiply by z^{p-1-k}
        term = np.concatenate([term, np.zeros(p - 1 - k)])
        poly[len(poly) - len(term):] += ck * term
    roots = np.roots(poly)
    inside = roots[np.abs(roots) < 1.0]
    h = np.array([1.0])
    for _ in range(p):
        h = np.convolve(h, [1.0, 1.0])
    for r in inside:
        h = np.convolve(h, [1.0, -r])
    h = np.real(h)
    return h * (math.sqrt(2.0) / h.sum())


def highpass_of(h: np.ndarray) -> np.ndarray:
    """Quadrature-mirror highpass g[k] = (-1)^k h[L-1-k]."""
    L = len(h)
    return np.array([(-1) ** k * h[L - 1 - k] for k in range(L)])


# ---------------------------------------------------------------------------
# Periodic orthonormal transform.

def analysis_1d(X: np.ndarray, f: np.ndarray, axis: int) -> np.ndarray:
    """out[n] = sum_k f[k] X[(2n + k) mod L] along `axis` (L even)."""
    X = np.moveaxis(np.asarray(X, dtype=np.float64), axis, -1)
    L = X.shape[-1]
    out = np.zeros(X.shape[:-1] + (L // 2,))
    for k, fk in enumerate(f):
        out += fk * X[..., (2 * np.arange(L // 2) + k) % L]
    return np.moveaxis(out, -1, axis)


def synthesis_1d(lo: np.ndarray, hi: np.ndarray, h: np.ndarray, g: np.ndarray, axis: int) -> np.ndarray:
    """Adjoint of the analysis: X[m] = sum_n h[m - 2n] lo[n] + g[m - 2n] hi[n], indices
    mod L (the inverse, the filters being orthonormal)."""
    lo = np.moveaxis(np.asarray(lo, dtype=np.float64), axis, -1)
    hi = np.moveaxis(np.asarray(hi, dtype=np.float64), axis, -1)
    n2 = lo.shape[-1]
    L = 2 * n2
    X = np.zeros(lo.shape[:-1] + (L,))
    for k in range(len(h)):
        idx = (2 * np.arange(n2) + k) % L
        np.add.at(X, (..., idx), h[k] * lo + g[k] * hi)
    return np.moveaxis(X, -1, axis)


def dwt2(X: np.ndarray, h: np.ndarray) -> Tuple[np.ndarray, Tuple[np.ndarray, np.ndarray, np.ndarray]]:
    """One level: the horizontal filter (along axis 1) first, then the vertical one
    (along axis 0).  Returns LL and the details (LH, HL, HH), the first letter naming
    the horizontal filter and the second the vertical one."""
    g = highpass_of(h)
    L = analysis_1d(X, h, 1)
    H = analysis_1d(X, g, 1)
    return analysis_1d(L, h, 0), (analysis_1d(L, g, 0), analysis_1d(H, h, 0), analysis_1d(H, g, 0))


def idwt2(LL: np.ndarray, details, h: np.ndarray) -> np.ndarray:
    g = highpass_of(h)
    LH, HL, HH = details
    L = synthesis_1d(LL, LH, h, g, 0)
    H = synthesis_1d(HL, HH, h, g, 0)
    return synthesis_1d(L, H, h, g, 1)


def wavedec2(X: np.ndarray, h: np.ndarray, levels: int = LEVELS):
    """[details of level 1 (finest), ..., details of level `levels`], coarsest LL."""
    out, A = [], np.asarray(X, dtype=np.float64)
    for _ in range(levels):
        A, d = dwt2(A, h)
        out.append(d)
    return out, A


def waverec2(details: Sequence, LL: np.ndarray, h: np.ndarray) -> np.ndarray:
    A = LL
    for d in reversed(details):
        A = idwt2(A, d, h)
    return A


# ---------------------------------------------------------------------------
# Local variance and the Wiener step.

def box_mean_zero(C2: np.ndarray, W: int) -> np.ndarray:
    """Mean of C2 over the W x W window centred on each element, the window reading
    zero outside the array and always divided by W^2."""
    r = W // 2
    M, N = C2.shape
    P = np.zeros((M + 2 * r, N + 2 * r))
    P[r:r + M, r:r + N] = C2
    S = np.zeros((M, N))
    for a in range(W):
        for b in range(W):
            S += P[a:a + M, b:b + N]
    return S / (W * W)


def local_variance(C: np.ndarray, sigma0: float, windows: Sequence[int] = WINDOWS) -> np.ndarray:
    """v = max(0, min_W mean_W(c^2) - s0^2): the smallest of the windowed estimates of
    the signal variance, clipped at zero."""
    C2 = np.asarray(C, dtype=np.float64) ** 2
    m = np.min(np.stack([box_mean_zero(C2, W) for W in windows]), axis=0)
    return np.maximum(0.0, m - sigma0 * sigma0)


def noise_part(C: np.ndarray, sigma0: float) -> np.ndarray:
    """The part of the coefficients the Wiener estimate removes: c s0^2 / (v + s0^2);
    zero where s0 = 0."""
    C = np.asarray(C, dtype=np.float64)
    s2 = sigma0 * sigma0
    if s2 == 0.0:
        return np.zeros_like(C)
    v = local_variance(C, sigma0)
    return C * (s2 / (v + s2))


# ---------------------------------------------------------------------------
# W(I) = I - F(I).

def mirror_extend(X: np.ndarray, M2: int, N2: int) -> np.ndarray:
    """X extended to M2 x N2 by mirroring its last rows and columns about the last
    one (row M + j holds row M - 2 - j)."""
    X = np.asarray(X, dtype=np.float64)
    M, N = X.shape
    rows = [i if i < M else 2 * (M - 1) - i for i in range(M2)]
    cols = [j if j < N else 2 * (N - 1) - j for j in range(N2)]
    return X[np.ix_(rows, cols)]


def padded_size(n: int, levels: int = LEVELS) -> int:
    q = 1 << levels
    return (n + q - 1) // q * q


def noise_residual(I: np.ndarray, sigma0: float = 3.0, levels: int = LEVELS) -> np.ndarray:
    """W(I) = I - F(I) with F the wavelet denoiser described in the module header."""
    I = np.asarray(I, dtype=np.float64)
    M, N = I.shape
    M2, N2 = padded_size(M, levels), padded_size(N, levels)
    if M2 - M >= M or N2 - N >= N:
        raise ValueError("image too small for the decomposition")
    X = mirror_extend(I, M2, N2)
    h = daubechies_lowpass(4)
    details, LL = wavedec2(X, h, levels)
    res = [tuple(noise_part(c, sigma0) for c in d) for d in details]
    R = waverec2(res, np.zeros_like(LL), h)
    return R[:M, :N]


def denoise(I: np.ndarray, sigma0: float = 3.0, levels: int = LEVELS) -> np.ndarray:
    """F(I): the Wiener estimates of every detail coefficient and the coarsest
    approximation, transformed back (cropped like the residual)."""
    I = np.asarray(I, dtype=np.float64)
    M, N = I.shape
    M2, N2 = padded_size(M, levels), padded_size(N, levels)
    X = mirror_extend(I, M2, N2)
    h = daubechies_lowpass(4)
    details, LL = wavedec2(X, h, levels)
    den = [tuple(c - noise_part(c, sigma0) for c in d) for d in details]
    return waverec2(den, LL, h)[:M, :N]
