"""Pins of the residual-extraction oracle (W(I) = I - F(I), wavelet denoiser) against
facts fixed by the mathematics: the published 8-tap Daubechies filter and its defining
properties, perfect reconstruction and energy preservation of the transform, closed-form
subbands of an impulse and of a constant, brute-force windowed means, and the limits of
the Wiener step."""
import math

import numpy as np
import pytest

from oracle import denoise_oracle as D

# Daubechies' orthonormal 8-tap filter (4 vanishing moments, minimum phase), as tabulated
# in the wavelet literature, scaled to sum sqrt(2)
PUBLISHED_DB8 = [0.2303778133088964, 0.7148465705529154, 0.6308807679298587, -0.0279837694168599,
                 -0.1870348117190931, 0.0308413818355607, 0.0328830116668852, -0.0105974017850690]


def test_filter_is_the_published_daubechies_filter():
    h = D.daubechies_lowpass(4)
    assert np.allclose(h, PUBLISHED_DB8, rtol=0, atol=1e-12)


def test_filter_properties():
    h = D.daubechies_lowpass(4)
    g = D.highpass_of(h)
    assert math.isclose(h.sum(), math.sqrt(2.0), rel_tol=1e-14)
    for k in range(4):   # orthonormal at even shifts, highpass orthogonal to lowpass
        assert math.isclose(float(np.dot(h[:8 - 2 * k], h[2 * k:])), 1.0 if k == 0 else 0.0, abs_tol=1e-14)
        assert abs(float(np.dot(h[:8 - 2 * k], g[2 * k:]))) < 1e-14
        assert abs(float(np.dot(g[:8 - 2 * k], h[2 * k:]))) < 1e-14
    for p in range(4):   # four vanishing moments of the highpass
        assert abs(sum(n ** p * g[n] for n in range(8))) < 1e-12
    assert abs(sum(n ** 4 * g[n] for n in range(8))) > 1.0
    # four zeros at z = -1 (divide them out exactly), the other three inside the unit
    # circle (minimum phase)
    q, rem = np.polydiv(h, [1.0, 4.0, 6.0, 4.0, 1.0])
    assert np.abs(rem).max() < 1e-12
    assert np.all(np.abs(np.roots(q)) < 0.9)


@pytest.mark.parametrize("shape,levels", [((32, 48), 3), ((64, 64), 4), ((16, 80), 4)])
def test_transform_is_orthonormal(shape, levels):
    X = np.random.default_rng(sum(shape)).standard_normal(shape)
    h = D.daubechies_lowpass(4)
    d, LL = D.wavedec2(X, h, levels)
    assert np.abs(D.waverec2(d, LL, h) - X).max() < 1e-12
    e = (LL ** 2).sum() + sum((c ** 2).sum() for t in d for c in t)
    assert math.isclose(e, (X ** 2).sum(), rel_tol=1e-12)


def test_impulse_subbands_are_filter_outer_products():
    """One level of a unit impulse at (r, c): subband (A, B)[n, m] = a[(r - 2n) mod M]
    * b[(c - 2m) mod N] with a, b the vertical and horizontal filters (zero outside
    their 8 taps)."""
    M, N, r, c = 16, 24, 5, 18
    X = np.zeros((M, N))
    X[r, c] = 1.0
    h = D.daubechies_lowpass(4)
    g = D.highpass_of(h)
    LL, (LH, HL, HH) = D.dwt2(X, h)

    def tap(f, i):
        return f[i] if 0 <= i < 8 else 0.0

    for got, fv, fh in ((LL, h, h), (LH, g, h), (HL, h, g), (HH, g, g)):
        want = np.array([[tap(fv, (r - 2 * n) % M) * tap(fh, (c - 2 * m) % N) for m in range(N // 2)]
                         for n in range(M // 2)])
        assert np.abs(got - want).max() < 1e-15


def test_constant_image():
    X = np.full((32, 48), 7.5)
    h = D.daubechies_lowpass(4)
    d, LL = D.wavedec2(X, h, 4)
    assert max(np.abs(c).max() for t in d for c in t) < 1e-12
    assert np.allclose(LL, 7.5 * 16.0, rtol=1e-14)   # sqrt(2)^2 per level and axis pair
    assert np.abs(D.noise_residual(X, 3.0)).max() < 1e-12


def test_windowed_means_brute_force():
    C = np.random.default_rng(3).standard_normal((7, 11))
    for W in (3, 5, 7, 9):
        got = D.box_mean_zero(C * C, W)
        r = W // 2
        for i in range(7):
            for j in range(11):
                s = sum(C[a, b] ** 2 for a in range(i - r, i + r + 1) for b in range(j - r, j + r + 1)
                        if 0 <= a < 7 and 0 <= b < 11)
                assert math.isclose(got[i, j], s / (W * W), rel_tol=1e-12)


def test_local_variance_takes_the_smallest_window_and_clips():
    """A coefficient field that is 2 on a 3 x 3 block and 0 elsewhere: at the block's
    centre the 3 x 3 mean of c^2 is 4, the 9 x 9 mean 36/81; elsewhere it is smaller."""
    C = np.zeros((21, 21))
    C[9:12, 9:12] = 2.0
    v = D.local_variance(C, 0.5)
    assert math.isclose(v[10, 10], 36.0 / 81.0 - 0.25, rel_tol=1e-12)
    assert np.all(v >= 0.0) and v[0, 0] == 0.0
    v0 = D.local_variance(C, 0.0)
    assert math.isclose(v0[10, 10], 36.0 / 81.0, rel_tol=1e-12)


def test_limits_of_the_wiener_step():
    I = np.random.default_rng(4).uniform(40, 220, (48, 64))
    assert np.abs(D.noise_residual(I, 0.0)).max() == 0.0
    # s0 -> infinity: every detail coefficient is noise, the residual is the image minus
    # its coarsest approximation (computed here through the transform alone)
    h = D.daubechies_lowpass(4)
    d, LL = D.wavedec2(I, h, 4)
    zero = [tuple(np.zeros_like(c) for c in t) for t in d]
    coarse = D.waverec2(zero, LL, h)
    assert np.abs(D.noise_residual(I, 1e9) - (I - coarse)).max() < 1e-6
    assert np.abs(D.denoise(I, 1e9) - coarse).max() < 1e-6


def test_mirror_extension_and_crop():
    X = np.arange(12.0).reshape(3, 4)
    E = D.mirror_extend(X, 5, 7)
    assert E[:3, :4].tolist() == X.tolist()
    assert E[3].tolist() == E[1].tolist() and E[4].tolist() == E[0].tolist()
    assert E[0, 4:].tolist() == [2.0, 1.0, 0.0]
    I = np.random.default_rng(5).uniform(40, 220, (37, 53))
    W = D.noise_residual(I, 3.0)
    F = D.denoise(I, 3.0)
    assert W.shape == I.shape and np.abs(I - F - W).max() < 1e-10


def test_residual_recovers_added_white_noise():
    """A smooth scene plus white noise of standard deviation s0: the residual is mostly
    that noise (the purpose of the denoiser)."""
    g = np.random.default_rng(6)
    yy, xx = np.mgrid[0:128, 0:128]
    scene = 120 + 60 * np.sin(xx / 17.0) * np.cos(yy / 23.0)
    noise = g.standard_normal((128, 128)) * 3.0
    W = D.noise_residual(scene + noise, 3.0)
    rho = float(np.sum(W * noise) / math.sqrt(np.sum(W * W) * np.sum(noise * noise)))
    assert rho > 0.8
    assert np.abs(D.noise_residual(scene, 3.0)).std() < 0.2 * noise.std()
