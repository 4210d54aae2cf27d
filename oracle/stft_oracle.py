"""FP64 reference of the time-frequency front end and back end (TEST INFRASTRUCTURE
ONLY: imported by tests/, never by the product path).

Section 5 of the paper analyses 16 kHz audio with 64 ms windows and a 16 ms hop
(1024-sample frames, hop 256, F = 513 bins); Section 1 takes each separated source
back to the time domain with the phase of the mixture.  The conventions written
out here are those the C ABI states (include/nfhmm.h, "time domain"):

  window    periodic Hann, w[i] = (1 - cos(2 pi i / nfft)) / 2
  framing   frame t covers x[t hop : t hop + nfft], no padding,
            T = 1 + (n - nfft) // hop
  transform X_t[k] = sum_i w[i] x[t hop + i] exp(-2 pi 1j k i / nfft), k <= nfft/2
  inverse   y[i] = sum_t w[j] z_t[j] / sum_t w[j]^2  (j = i - t hop over the frames
            covering i), z_t the inverse transform of the Hermitian spectrum
            mag_t exp(1j phase_t) with the imaginary parts of bins 0 and nfft/2
            dropped; y[i] = 0 where the window weights sum to zero.

numpy's FFT serves as a step; tests/test_stft_pins.py pins it (and everything
else here) to a brute-force DFT and to closed forms.
"""
from __future__ import annotations

import numpy as np


def hann(nfft: int) -> np.ndarray:
    """Periodic Hann window of nfft samples (float64)."""
    i = np.arange(nfft, dtype=np.float64)
    return 0.5 - 0.5 * np.cos(2.0 * np.pi * i / nfft)


def n_frames(nfft: int, hop: int, n: int) -> int:
    return 0 if n < nfft else 1 + (n - nfft) // hop


def stft(x, nfft: int = 1024, hop: int = 256):
    """(mag, phase) of x [n] (or [B][n]): [T][F] (or [B][T][F]), float64."""
    x = np.asarray(x, dtype=np.float64)
    one = x.ndim == 1
    x2 = x[None] if one else x
    T = n_frames(nfft, hop, x2.shape[1])
    w = hann(nfft)
    idx = np.arange(T)[:, None] * hop + np.arange(nfft)[None, :]
    X = np.fft.rfft(x2[:, idx] * w, axis=-1)        # [B][T][F]
    mag, phase = np.abs(X), np.angle(X)
    return (mag[0], phase[0]) if one else (mag, phase)


def istft(mag, phase, n: int, nfft: int = 1024, hop: int = 256):
    """Weighted overlap-add inverse: mag [T][F] or [B][T][F], phase [T][F] -> y [n] or [B][n]."""
    mag = np.asarray(mag, dtype=np.float64)
    phase = np.asarray(phase, dtype=np.float64)
    one = mag.ndim == 2
    m3 = mag[None] if one else mag
    B, T, F = m3.shape
    Y = m3 * np.exp(1j * phase)[None]
    Y[..., 0] = Y[..., 0].real
    Y[..., F - 1] = Y[..., F - 1].real
    z = np.fft.irfft(Y, n=nfft, axis=-1)             # [B][T][nfft]
    w = hann(nfft)
    y = np.zeros((B, n))
    wsum = np.zeros(n)
    for t in range(T):
        lo = t * hop
        hi = min(n, lo + nfft)
        if lo >= n:
            break
        y[:, lo:hi] += (z[:, t] * w)[:, : hi - lo]
        wsum[lo:hi] += (w * w)[: hi - lo]
    y = np.where(wsum > 0.0, y / np.where(wsum > 0.0, wsum, 1.0), 0.0)
    return y[0] if one else y


def window_weight(n: int, T: int, nfft: int = 1024, hop: int = 256) -> np.ndarray:
    """sum_t w[i - t hop]^2 at every sample i < n (the inverse's denominator)."""
    w2 = hann(nfft) ** 2
    s = np.zeros(n)
    for t in range(T):
        lo = t * hop
        hi = min(n, lo + nfft)
        if lo >= n:
            break
        s[lo:hi] += w2[: hi - lo]
    return s
