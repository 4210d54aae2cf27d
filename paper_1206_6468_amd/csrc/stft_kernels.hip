// Time-frequency front end and back end of the separation (Section 5 analyses
// 16 kHz audio with 64 ms windows and a 16 ms hop: 1024-sample frames, hop 256,
// F = 513 bins; Section 1 resynthesises each separated source with the phase
// of the mixture).
//
//   k_stft   one block per (signal, run of kStftFrames frames): per frame, the
//            frame times a periodic Hann window, an NFFT-point complex FFT in LDS
//            (radix-2, Stockham order, so no bit reversal), |X| and arg X of bins
//            0..NFFT/2.  The window and the twiddles are tabulated in LDS once per
//            block.
//   k_istft  one block per (source, run of G consecutive frames): per frame, the
//            Hermitian spectrum mag * exp(i phase), the inverse FFT, the window;
//            the windowed frame and the squared window are added into two rings
//            of NFFT samples in LDS (sample i at slot i mod NFFT).  Once frame t is
//            in, no later frame touches the samples [t hop, (t + 1) hop): they are
//            final, written out as sum / weight (weighted overlap-add), and their
//            slots cleared for the samples NFFT further on.  A block starts
//            ceil(NFFT / hop) - 1 frames before its run so that its first samples
//            see every frame covering them; those lead-in frames are computed but
//            write nothing.  Every sample is summed over its frames in increasing
//            t in one block: no atomics, no frame scratch in HBM, and a fixed
//            summation order.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "launch.h"

namespace nfhmm {

namespace {

constexpr int kStftThreads = 256;
#ifndef NFHMM_STFT_FRAMES
#define NFHMM_STFT_FRAMES 4
#endif
#ifndef NFHMM_ISTFT_RUN
#define NFHMM_ISTFT_RUN 8
#endif
constexpr int kStftFrames = NFHMM_STFT_FRAMES;    // frames per block of the transform
constexpr int kIstftRunPerLead = NFHMM_ISTFT_RUN; // inverse: run length per (lead-in + 1) frames

// periodic Hann window: w[i] = (1 - cos(2 pi i / NFFT)) / 2
template <int NFFT>
__device__ __forceinline__ float hann(int i) {
  return 0.5f - 0.5f * cospif(2.0f * (float)i / (float)NFFT);
}

// Twiddles into LDS, stage by stage: the stage combining transforms of size ns
// (1, 2, ..., NFFT/2) uses exp(sign i pi k / ns), k < ns, and finds them at
// tw[ns - 1 + k], so the lanes of a wave read consecutive words (one strided
// table of the NFFT/2 roots would put a wave's reads in one bank in the middle
// stages).  NFFT - 1 entries.
template <int NFFT>
__device__ __forceinline__ void twiddles(float *twr, float *twi, float sign) {
  for (int e = threadIdx.x; e < NFFT - 1; e += kStftThreads) {
    const int ns = 1 << (31 - __clz(e + 1));   // the largest power of two <= e + 1
    const int k = e + 1 - ns;
    float s, c;
    sincospif(sign * (float)k / (float)ns, &s, &c);
    twr[e] = c;
    twi[e] = s;
  }
}

// In-place NFFT-point FFT of (re, im) in LDS with the twiddles of its sign
// (forward -1, inverse +1, unscaled).  Stage s combines pairs of transforms of
// size ns = 2^s; butterfly j reads j and j + NFFT/2 and writes (j / ns) * 2 ns +
// j % ns and that + ns.  Expects the inputs and the table written before a
// barrier; ends with a barrier; the result is in (re, im).
template <int NFFT>
__device__ void fft_lds(float *re, float *im, float *re2, float *im2, const float *twr, const float *twi) {
  constexpr int kHalf = NFFT / 2;
  float *sr = re, *si = im, *dr = re2, *di = im2;
  for (int ns = 1; ns < NFFT; ns <<= 1) {
    for (int j = threadIdx.x; j < kHalf; j += kStftThreads) {
      const int k = j & (ns - 1);
      const float c = twr[ns - 1 + k], s = twi[ns - 1 + k];
      const float ar = sr[j], ai = si[j];
      const float br0 = sr[j + kHalf], bi0 = si[j + kHalf];
      const float br = br0 * c - bi0 * s, bi = br0 * s + bi0 * c;
      const int d = (j - k) * 2 + k;
      dr[d] = ar + br;
      di[d] = ai + bi;
      dr[d + ns] = ar - br;
      di[d + ns] = ai - bi;
    }
    __syncthreads();
    float *tr = sr, *ti = si;
    sr = dr; si = di; dr = tr; di = ti;
  }
  if (sr != re) {   // an odd number of stages left the result in the second buffer
    for (int i = threadIdx.x; i < NFFT; i += kStftThreads) {
      re[i] = sr[i];
      im[i] = si[i];
    }
    __syncthreads();
  }
}

// the window w[i] into LDS
template <int NFFT>
__device__ __forceinline__ void window(float *win) {
  for (int i = threadIdx.x; i < NFFT; i += kStftThreads) win[i] = hann<NFFT>(i);
}

template <int NFFT>
__global__ __launch_bounds__(kStftThreads) void k_stft(const float *__restrict__ x, int64_t n, int hop, int T,
                                                       float *__restrict__ mag, float *__restrict__ phase) {
  constexpr int F = NFFT / 2 + 1;
  __shared__ float re[NFFT], im[NFFT], re2[NFFT], im2[NFFT], twr[NFFT], twi[NFFT], win[NFFT];
  const int b = blockIdx.y;
  const int t0 = blockIdx.x * kStftFrames, t1 = min(T, t0 + kStftFrames);
  twiddles<NFFT>(twr, twi, -1.0f);
  window<NFFT>(win);
  for (int t = t0; t < t1; ++t) {
    const float *xs = x + (size_t)b * n + (size_t)t * hop;
    __syncthreads();   // the tables are written; the previous frame's bins are read
    for (int i = threadIdx.x; i < NFFT; i += kStftThreads) {
      re[i] = xs[i] * win[i];
      im[i] = 0.0f;
    }
    __syncthreads();
    fft_lds<NFFT>(re, im, re2, im2, twr, twi);
    const size_t o = ((size_t)b * T + t) * F;
    for (int k = threadIdx.x; k < F; k += kStftThreads) {
      mag[o + k] = hypotf(re[k], im[k]);
      phase[o + k] = atan2f(im[k], re[k]);
    }
  }
}

template <int NFFT>
__global__ __launch_bounds__(kStftThreads) void k_istft(const float *__restrict__ mag, const float *__restrict__ phase,
                                                        int S, int T, int hop, int G, int64_t n,
                                                        float *__restrict__ y) {
  constexpr int F = NFFT / 2 + 1;
  __shared__ float re[NFFT], im[NFFT], re2[NFFT], im2[NFFT], twr[NFFT], twi[NFFT], win[NFFT];
  __shared__ float acc[NFFT], wacc[NFFT];   // rings: slot i mod NFFT holds sample i
  const int sig = blockIdx.y, mix = sig / S;
  const int t0 = blockIdx.x * G, t1 = min(T, t0 + G);
  const int lead = (NFFT + hop - 1) / hop - 1;   // frames before t0 that cover samples >= t0 hop
  const int ts = max(0, t0 - lead);
  twiddles<NFFT>(twr, twi, 1.0f);
  window<NFFT>(win);
  for (int i = threadIdx.x; i < NFFT; i += kStftThreads) {
    acc[i] = 0.0f;
    wacc[i] = 0.0f;
  }
  float *ys = y + (size_t)sig * n;
  for (int t = ts; t < t1; ++t) {
    const float *ms = mag + ((size_t)sig * T + t) * F, *ps = phase + ((size_t)mix * T + t) * F;
    __syncthreads();   // the tables and rings are written; the previous frame is folded in
    for (int k = threadIdx.x; k < F; k += kStftThreads) {
      float s, c;
      sincosf(ps[k], &s, &c);
      const float a = ms[k];
      // a real signal: bins 0 and NFFT/2 are real (their imaginary parts are dropped)
      const float yr = a * c, yi = (k == 0 || k == F - 1) ? 0.0f : a * s;
      re[k] = yr;
      im[k] = yi;
      if (k > 0 && k < F - 1) {   // Hermitian half
        re[NFFT - k] = yr;
        im[NFFT - k] = -yi;
      }
    }
    __syncthreads();
    fft_lds<NFFT>(re, im, re2, im2, twr, twi);
    const int64_t base = (int64_t)t * hop;
    for (int j = threadIdx.x; j < NFFT; j += kStftThreads) {
      const int r = (int)((base + j) & (NFFT - 1));
      const float w = win[j];
      acc[r] += re[j] * (1.0f / (float)NFFT) * w;
      wacc[r] += w * w;
    }
    __syncthreads();
    // samples [t hop, t hop + hop) are final (the last frame also owns the rest of
    // the signal: its tail, then the samples no frame covers, which are zero)
    const int64_t hi = t == T - 1 ? n : min(n, base + hop);
    for (int64_t i = base + threadIdx.x; i < hi; i += kStftThreads) {
      if (i < base + NFFT) {
        const int r = (int)(i & (NFFT - 1));
        if (t >= t0) ys[i] = wacc[r] > 0.0f ? acc[r] / wacc[r] : 0.0f;
        acc[r] = 0.0f;
        wacc[r] = 0.0f;
      } else if (t >= t0) {
        ys[i] = 0.0f;
      }
    }
  }
}

}  // namespace

hipError_t launch_stft(int nfft, const float *x, int64_t n, int hop, int T, int B, float *mag, float *phase,
                       hipStream_t st) {
  const dim3 grid((unsigned)((T + kStftFrames - 1) / kStftFrames), B);
  switch (nfft) {
#define NFHMM_STFT_CASE(P) \
  case P: k_stft<P><<<grid, kStftThreads, 0, st>>>(x, n, hop, T, mag, phase); break;
    NFHMM_STFT_CASE(64) NFHMM_STFT_CASE(128) NFHMM_STFT_CASE(256) NFHMM_STFT_CASE(512)
    NFHMM_STFT_CASE(1024) NFHMM_STFT_CASE(2048) NFHMM_STFT_CASE(4096)
#undef NFHMM_STFT_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int istft_run(int nfft, int hop) {
  const int lead = (nfft + hop - 1) / hop - 1;
  return kIstftRunPerLead * (lead + 1);
}

hipError_t launch_istft(int nfft, const float *mag, const float *phase, int T, int B, int S, int hop, int64_t n,
                        float *y, hipStream_t st) {
  const int G = istft_run(nfft, hop);
  const dim3 grid((unsigned)((T + G - 1) / G), B * S);
  switch (nfft) {
#define NFHMM_ISTFT_CASE(P) \
  case P: k_istft<P><<<grid, kStftThreads, 0, st>>>(mag, phase, S, T, hop, G, n, y); break;
    NFHMM_ISTFT_CASE(64) NFHMM_ISTFT_CASE(128) NFHMM_ISTFT_CASE(256) NFHMM_ISTFT_CASE(512)
    NFHMM_ISTFT_CASE(1024) NFHMM_ISTFT_CASE(2048) NFHMM_ISTFT_CASE(4096)
#undef NFHMM_ISTFT_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace nfhmm
