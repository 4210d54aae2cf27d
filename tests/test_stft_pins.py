"""Pins of the FP64 time-frequency reference (oracle/stft_oracle.py), on the CPU.

Each pin checks the reference against something other than itself: the DFT
written out as a sum, closed forms of the Hann window and of a windowed pure
tone, and exact reconstruction.
"""
import numpy as np
import pytest

from oracle import stft_oracle as SO


def test_transform_is_the_windowed_dft_written_out():
    rng = np.random.default_rng(1)
    nfft, hop = 16, 5
    x = rng.normal(size=3 * hop + nfft)
    mag, phase = SO.stft(x, nfft, hop)
    T = SO.n_frames(nfft, hop, x.size)
    assert mag.shape == (T, nfft // 2 + 1) == (4, 9)
    w = [0.5 - 0.5 * np.cos(2 * np.pi * i / nfft) for i in range(nfft)]
    for t in range(T):
        for k in range(nfft // 2 + 1):
            s = sum(w[i] * x[t * hop + i] * np.exp(-2j * np.pi * k * i / nfft) for i in range(nfft))
            assert abs(mag[t, k] * np.exp(1j * phase[t, k]) - s) < 1e-12


def test_periodic_hann_closed_forms():
    for nfft in (64, 1024):
        w = SO.hann(nfft)
        assert w[0] == 0.0 and abs(w[nfft // 2] - 1.0) < 1e-15
        assert abs(w.sum() - nfft / 2) < 1e-9
        # at 75 % overlap the squared windows sum to 3/2 everywhere in the interior
        ws = SO.window_weight(8 * nfft, 29, nfft, nfft // 4)
        inner = ws[nfft:6 * nfft]
        assert np.max(np.abs(inner - 1.5)) < 1e-12


def test_windowed_tone_has_the_three_bin_shape():
    # x = cos(2 pi k0 i / nfft): the Hann window spreads it over bins k0 - 1, k0,
    # k0 + 1 with magnitudes nfft/8, nfft/4, nfft/8 and nothing elsewhere
    nfft, k0 = 256, 19
    i = np.arange(nfft)
    mag, _ = SO.stft(np.cos(2 * np.pi * k0 * i / nfft), nfft, nfft)
    want = np.zeros(nfft // 2 + 1)
    want[[k0 - 1, k0, k0 + 1]] = [nfft / 8, nfft / 4, nfft / 8]
    assert np.max(np.abs(mag[0] - want)) < 1e-10


@pytest.mark.parametrize("nfft,hop", [(64, 16), (64, 32), (256, 64), (128, 21)])
def test_inverse_reconstructs_where_windows_cover(nfft, hop):
    rng = np.random.default_rng(nfft + hop)
    n = 7 * nfft + 3
    x = rng.normal(size=n)
    mag, phase = SO.stft(x, nfft, hop)
    y = SO.istft(mag, phase, n, nfft, hop)
    T = mag.shape[0]
    ws = SO.window_weight(n, T, nfft, hop)
    cov = ws > 1e-3
    assert np.max(np.abs(y[cov] - x[cov])) < 1e-9
    assert np.all(y[ws == 0.0] == 0.0)
    # the samples after the last frame are not analysed and come back as zeros
    assert np.all(y[(T - 1) * hop + nfft:] == 0.0)


def test_masks_that_sum_to_one_give_sources_that_sum_to_the_mixture():
    rng = np.random.default_rng(5)
    nfft, hop, n = 128, 32, 1200
    x = rng.normal(size=n)
    mag, phase = SO.stft(x, nfft, hop)
    m = rng.uniform(size=(3,) + mag.shape)
    m /= m.sum(0, keepdims=True)
    y = SO.istft(m * mag[None], phase, n, nfft, hop)
    ws = SO.window_weight(n, mag.shape[0], nfft, hop)
    cov = ws > 1e-3
    assert np.max(np.abs(y.sum(0)[cov] - x[cov])) < 1e-9
