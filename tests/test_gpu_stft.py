"""The time-frequency front end and back end on the GPU against the FP64 reference.

Tolerances: the transform in float32 (FFT rounding grows as log2 nfft) is
compared as complex values, |X_gpu - X_ref| <= 2e-6 * max|X| (phases of bins with
almost no energy are ill-conditioned and are not compared on their own).  The
inverse divides by the window weight sum_t w^2, which near the first and last
frame tends to zero: it is compared where that weight is at least 0.1 (error
bound 1e-5 of max|y| over those samples), and checked finite everywhere.
"""
import numpy as np
import pytest

from oracle import stft_oracle as SO

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_1206_6468_amd import nfhmm
    return nfhmm


@pytest.fixture(scope="module")
def ctx(L):
    c = L.Context(0)
    yield c
    c.close()


# (nfft, hop, B, n): every supported nfft, several blocks of frames each, hops that
# do and do not divide nfft, a hop with a long lead-in (256 / 7), no overlap (hop = nfft)
CASES = [(1024, 256, 3, 40_000), (64, 16, 2, 1000), (2048, 512, 2, 30_000), (256, 100, 1, 5001),
         (4096, 1024, 1, 20_000), (128, 128, 2, 999), (256, 7, 1, 3000), (512, 128, 2, 9001)]


@pytest.mark.parametrize("nfft,hop,B,n", CASES)
def test_stft_matches_reference(L, ctx, nfft, hop, B, n):
    rng = np.random.default_rng(nfft + hop + n)
    x = rng.normal(size=(B, n)).astype(np.float32)
    mag, phase = L.stft(ctx, x, nfft, hop)
    rm, rp = SO.stft(x.astype(np.float64), nfft, hop)
    assert mag.shape == rm.shape == (B, SO.n_frames(nfft, hop, n), nfft // 2 + 1)
    Xg = mag.astype(np.float64) * np.exp(1j * phase.astype(np.float64))
    Xr = rm * np.exp(1j * rp)
    err = np.max(np.abs(Xg - Xr)) / np.max(np.abs(Xr))
    print(f"\nstft nfft={nfft} hop={hop}: max |dX| / max |X| = {err:.2e}")
    assert err < 2e-6
    assert np.all(mag >= 0) and np.all(np.abs(phase) <= np.pi + 1e-6)


@pytest.mark.parametrize("nfft,hop,B,n", CASES)
def test_istft_matches_reference(L, ctx, nfft, hop, B, n):
    # B mixtures, S = 2 masked versions of each sharing that mixture's phase
    rng = np.random.default_rng(7 + nfft + hop)
    S = 2
    ref = [SO.stft(rng.normal(size=n), nfft, hop) for _ in range(B)]
    T = ref[0][0].shape[0]
    gains = rng.uniform(0.2, 1.0, size=(B, S) + ref[0][0].shape)
    m = (gains * np.stack([r[0] for r in ref])[:, None]).astype(np.float32)
    p = np.stack([r[1] for r in ref]).astype(np.float32)
    y = L.istft(ctx, m, p, n, nfft, hop)
    assert y.shape == (B, S, n)
    ws = SO.window_weight(n, T, nfft, hop)
    ok = ws >= 0.1
    for b in range(B):
        yr = SO.istft(m[b].astype(np.float64), p[b].astype(np.float64), n, nfft, hop)
        err = np.max(np.abs(y[b][:, ok] - yr[:, ok])) / np.max(np.abs(yr[:, ok]))
        print(f"\nistft nfft={nfft} hop={hop} mixture {b}: max |dy| / max |y| = {err:.2e}")
        assert err < 1e-5
    assert np.all(np.isfinite(y))
    assert np.all(y[..., ws == 0.0] == 0.0)


def test_istft_frames_past_the_end_and_uncovered_tail(L, ctx):
    # T larger than the frame count of n (the extra frames fall past the end), and a
    # signal longer than the frames cover (its tail comes back as zeros)
    nfft, hop = 256, 64
    rng = np.random.default_rng(21)
    for T, n in [(40, 2000), (12, 2000)]:
        m = rng.uniform(size=(3, T, nfft // 2 + 1)).astype(np.float32)
        p = rng.uniform(-np.pi, np.pi, size=(T, nfft // 2 + 1)).astype(np.float32)
        y = L.istft(ctx, m, p, n, nfft, hop)
        yr = SO.istft(m.astype(np.float64), p.astype(np.float64), n, nfft, hop)
        ws = SO.window_weight(n, T, nfft, hop)
        ok = ws >= 0.1
        assert np.max(np.abs(y[:, ok] - yr[:, ok])) < 1e-5 * np.max(np.abs(yr[:, ok]))
        assert np.all(y[:, ws == 0.0] == 0.0)
        if T == 12:
            assert np.all(y[:, 11 * hop + nfft:] == 0.0)


def test_istft_phase_in_any_turn(L, ctx):
    # phases shifted by whole turns (as an unwrapped phase would be) resynthesise
    # the same signal
    nfft, hop, n = 1024, 256, 30_000
    rng = np.random.default_rng(5)
    mag, phase = SO.stft(rng.normal(size=n), nfft, hop)
    m = mag[None].astype(np.float32)
    p = phase.astype(np.float32)
    turns = rng.integers(-40, 41, size=p.shape)
    p2 = (p.astype(np.float64) + 2.0 * np.pi * turns).astype(np.float32)
    y1 = L.istft(ctx, m, p, n, nfft, hop)
    y2 = L.istft(ctx, m, p2, n, nfft, hop)
    ws = SO.window_weight(n, mag.shape[0], nfft, hop)
    ok = ws >= 0.1
    err = np.max(np.abs(y1[:, ok] - y2[:, ok])) / np.max(np.abs(y1[:, ok]))
    print(f"\nistft, phases off by up to 40 turns: max |dy| / max |y| = {err:.2e}")
    assert err < 1e-4


def test_round_trip_and_sources_sum_to_mixture(L, ctx):
    # analysis, three masks that sum to one, resynthesis with the mixture phase
    nfft, hop, n = 1024, 256, 64_000
    rng = np.random.default_rng(3)
    x = rng.normal(size=n).astype(np.float32)
    mag, phase = L.stft(ctx, x, nfft, hop)
    T = mag.shape[0]
    ws = SO.window_weight(n, T, nfft, hop)
    ok = ws >= 0.1
    y = L.istft(ctx, mag, phase, n, nfft, hop)
    assert np.max(np.abs(y[ok] - x[ok])) < 2e-5 * np.max(np.abs(x))
    m = rng.uniform(size=(3,) + mag.shape)
    m /= m.sum(0, keepdims=True)
    ys = L.istft(ctx, (m * mag[None]).astype(np.float32), phase, n, nfft, hop)
    assert np.max(np.abs(ys.sum(0)[ok] - x[ok])) < 2e-5 * np.max(np.abs(x))


def test_device_forms_equal_host_forms(L, ctx):
    import torch
    nfft, hop, B, n = 1024, 256, 2, 50_000
    rng = np.random.default_rng(9)
    x = rng.normal(size=(B, n)).astype(np.float32)
    mag, phase = L.stft(ctx, x, nfft, hop)
    dev = torch.device("cuda:0")
    dx = torch.as_tensor(x, device=dev)
    T = L.stft_frames(nfft, hop, n)
    dm = torch.empty((B, T, nfft // 2 + 1), dtype=torch.float32, device=dev)
    dp = torch.empty_like(dm)
    L.stft_device(ctx, dx, dm, dp, nfft, hop)
    dy = torch.empty((B, 1, n), dtype=torch.float32, device=dev)
    L.istft_device(ctx, dm.view(B, 1, T, -1), dp, dy, nfft, hop)
    torch.cuda.synchronize()
    assert np.array_equal(dm.cpu().numpy(), mag) and np.array_equal(dp.cpu().numpy(), phase)
    y = L.istft(ctx, mag[:, None], phase, n, nfft, hop)
    assert np.array_equal(dy.cpu().numpy(), y)
    with pytest.raises(ValueError):   # shapes are checked before anything is queued
        L.istft_device(ctx, dm.view(B, 1, T, -1), dp[:1], dy, nfft, hop)


def test_stft_rejects_bad_sizes(L, ctx):
    x = np.zeros(5000, dtype=np.float32)
    for nfft, hop in [(1000, 250), (8192, 256), (32, 8), (1024, 0), (1024, 2048)]:
        with pytest.raises(L.NfhmmError) as e:
            L.stft(ctx, x, nfft, hop)
        assert e.value.status == L.E_INVALID
    with pytest.raises(L.NfhmmError):
        L.stft(ctx, np.zeros(100, dtype=np.float32), 1024, 256)   # no whole frame
    with pytest.raises(L.NfhmmError) as e:   # more than 65535 sources in one call
        L.istft(ctx, np.zeros((256, 257, 1, 33), dtype=np.float32), np.zeros((256, 1, 33), dtype=np.float32),
                64, 64, 16)
    assert e.value.status == L.E_INVALID


def test_separation_pipeline_sources_sum_to_the_mixture(L, ctx):
    # the whole separation on the GPU: STFT of a mixture, the VI fit on its
    # magnitudes, the separated spectrograms back to signals with the mixture's
    # phase.  The separated magnitudes of every bin sum to the mixture's, so the
    # resynthesised sources sum to the mixture wherever a window covers.
    from gen import make_tiny
    nfft, hop = 256, 64
    p = make_tiny(S=2, N=5, K=8, F=nfft // 2 + 1, T=100, seed=3, iters=8)
    n = (p["T"] - 1) * hop + nfft
    rng = np.random.default_rng(17)
    i = np.arange(n)
    # two sources: a tone whose pitch steps every 1600 samples, and noise bursts
    s1 = np.sin(2 * np.pi * (0.02 + 0.01 * (i // 1600 % 3)) * i)
    s2 = rng.normal(size=n) * (np.sin(2 * np.pi * i / 2000) > 0)
    x = (s1 + 0.5 * s2).astype(np.float32)
    mag, phase = L.stft(ctx, x, nfft, hop)
    assert mag.shape == (p["T"], p["F"])
    p["V"] = mag
    out = L.fit(ctx, p)
    sep = out["sep"]
    assert np.all(np.isfinite(sep)) and np.all(sep >= 0)
    assert np.max(np.abs(sep.sum(0) - mag)) <= 1e-5 * np.max(mag)
    y = L.istft(ctx, sep, phase, n, nfft, hop)
    assert y.shape == (2, n) and np.all(np.isfinite(y))
    ws = SO.window_weight(n, p["T"], nfft, hop)
    ok = ws >= 0.1
    assert np.max(np.abs(y.sum(0)[ok] - x[ok])) < 2e-5 * np.max(np.abs(x))
    assert np.max(np.abs(y[0])) > 0 and np.max(np.abs(y[1])) > 0


def test_bench_launch_configuration(L, ctx):
    # the launches bench.py times: device forms on a stream of their own, 32
    # mixtures of 1000 frames (nfft 1024, hop 256), then 2 masked sources per
    # mixture in one inverse call; sampled mixtures checked against the reference
    import torch
    jobs, S, frames, nfft, hop = 32, 2, 1000, 1024, 256
    F = nfft // 2 + 1
    n = (frames - 1) * hop + nfft
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(31)
    x = rng.normal(size=(jobs, n)).astype(np.float32)
    masks = rng.uniform(size=(jobs, S, frames, F)).astype(np.float32)
    dx = torch.as_tensor(x, device=dev)
    mag = torch.empty((jobs, frames, F), device=dev)
    phase = torch.empty_like(mag)
    y = torch.empty((jobs, S, n), device=dev)
    torch.cuda.synchronize()   # the input copy (torch's stream) before the library's stream reads it
    st = torch.cuda.Stream()
    L.stft_device(ctx, dx, mag, phase, nfft, hop, stream=st)
    st.synchronize()
    src = (torch.as_tensor(masks, device=dev) * mag[:, None]).contiguous()
    torch.cuda.synchronize()
    L.istft_device(ctx, src, phase, y, nfft, hop, stream=st)
    st.synchronize()
    mg, ph, yg, sg = mag.cpu().numpy(), phase.cpu().numpy(), y.cpu().numpy(), src.cpu().numpy()
    ws = SO.window_weight(n, frames, nfft, hop)
    ok = ws >= 0.1
    for b in (0, 13, 31):
        rm, rp = SO.stft(x[b].astype(np.float64), nfft, hop)
        Xg = mg[b].astype(np.float64) * np.exp(1j * ph[b].astype(np.float64))
        assert np.max(np.abs(Xg - rm * np.exp(1j * rp))) < 2e-6 * np.max(rm)
        yr = SO.istft(sg[b].astype(np.float64), ph[b].astype(np.float64), n, nfft, hop)
        assert np.max(np.abs(yg[b][:, ok] - yr[:, ok])) < 1e-5 * np.max(np.abs(yr[:, ok]))
    assert np.all(np.isfinite(yg))
