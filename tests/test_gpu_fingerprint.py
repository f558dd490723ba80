"""GPU parity of the reference-fingerprint estimate of Eq. (2) against the FP64 oracle."""
import numpy as np
import pytest

from oracle import prnu_oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2207_14507_amd import prnu
    return prnu


def _data(L, M, N, seed):
    g = np.random.default_rng(seed)
    K = (g.standard_normal((M, N)) * 0.02).astype(np.float32)
    I = g.uniform(0.2, 0.9, size=(L, M, N)).astype(np.float32)
    W = (I * K + g.standard_normal((L, M, N)) * 0.05).astype(np.float32)
    return K, I, W


@pytest.mark.parametrize("L,M,N", [(12, 256, 384), (5, 33, 41), (1, 64, 64)])
def test_estimate_matches_oracle(P, L, M, N):
    K, I, W = _data(L, M, N, 7 + M)
    ctx = P.prnu_create(0)
    try:
        got = P.prnu_estimate_fingerprint(ctx, I, W)
        ref = O.estimate_fingerprint(I, W)
        # FP64 sums on both sides, one rounding to float on the GPU
        assert np.allclose(got, ref, rtol=2e-7, atol=1e-9)
        I[:, 3, 5] = 0.0
        assert P.prnu_estimate_fingerprint(ctx, I, W)[3, 5] == 0.0
    finally:
        P.prnu_destroy(ctx)


def test_noise_free_model_and_device_inputs(P):
    import torch
    K, I, _ = _data(6, 128, 200, 11)
    W = (I.astype(np.float64) * K).astype(np.float32)
    ctx = P.prnu_create(0)
    try:
        host = P.prnu_estimate_fingerprint(ctx, I, W)
        assert np.allclose(host, O.estimate_fingerprint(I, W), rtol=2e-7, atol=1e-9)
        assert np.allclose(host, K, rtol=1e-5, atol=1e-7)
        # device inputs: one contiguous, one a strided view (staged by the library)
        di = torch.from_numpy(I).cuda()
        dw = torch.zeros((6, 128, 256), device="cuda")
        dw[:, :, :200] = torch.from_numpy(W).cuda()
        out = torch.empty((128, 200), device="cuda")
        P.prnu_estimate_fingerprint(ctx, di, dw[:, :, :200], out=out)
        assert np.array_equal(out.cpu().numpy(), host)
        with pytest.raises(P.PrnuError) as e:
            P.prnu_estimate_fingerprint(ctx, I, W[:5])
        assert e.value.status == P.PRNU_E_SHAPE
    finally:
        P.prnu_destroy(ctx)
