// Time-frequency front end and back end of the separation (Section 5 analyses
// 16 kHz audio with 64 ms windows and a 16 ms hop: 1024-sample frames, hop 256,
// F = 513 bins; Section 1 resynthesises each separated source with the phase
// of the mixture).
//
// A real frame of NFFT samples is transformed as NFFT/2 complex points (even
// samples in the real, odd samples in the imaginary parts), with a pairwise
// fold or unfold between that transform and the real frame's bins.  The complex
// FFT of size L (the helpers' template parameter, L = NFFT/2 here) is a Stockham
// (self-sorting) transform in LDS: radix-4 passes, with one radix-2 pass first
// when log2 L is odd.  The pass combining transforms of size ns takes butterfly
// j (< L/R) from the R inputs j + r L/R, multiplies input r by
// exp(sign 2 pi i r k / (R ns)), k = j mod ns, does an R-point DFT and writes
// output r to (j - k) R + k + r ns.  The first pass (ns = 1, no twiddles) reads
// its inputs where they are, and the last pass (ns = L/4) leaves output r of
// butterfly j in registers as bin j + r L/4, so only the passes between touch
// LDS on both sides: 3 of 5 at L = 512 (NFFT = 1024).
//
//   k_stft   one block per (signal, run of kStftFrames frames): per frame, the
//            windowed frame, read from HBM as NFFT/2 complex values (even samples
//            real, odd imaginary), goes straight into the first pass of an
//            NFFT/2-point FFT; a last step unfolds bins k and NFFT/2 - k of the
//            real frame's transform from that FFT's bins k and NFFT/2 - k and
//            writes |X| and arg X of bins 0..NFFT/2 to HBM.  The window and the
//            twiddles are tabulated in LDS once per block.
//   k_istft  one block per (two sources of a mixture, run of G consecutive
//            frames; the sources share the phase's loads and sincos): per frame, the
//            Hermitian spectrum mag * exp(i phase) folded into NFFT/2 complex
//            values whose NFFT/2-point inverse FFT holds the even samples in its
//            real and the odd samples in its imaginary parts; the last pass adds
//            the windowed samples and the squared window into two rings of NFFT
//            samples in LDS (sample i at slot i mod NFFT).
//            Once frame t is in, no later frame touches the samples
//            [t hop, (t + 1) hop): they are final, written out as sum / weight
//            (weighted overlap-add), and their slots cleared for the samples NFFT
//            further on.  A block starts ceil(NFFT / hop) - 1 frames before its
//            run so that its first samples see every frame covering them; those
//            lead-in frames are computed but write nothing.  Every sample is
//            summed over its frames in increasing t in one block: no atomics, no
//            frame scratch in HBM, and a fixed summation order.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "launch.h"

namespace nfhmm {

namespace {

constexpr int kStftThreads = 256;
constexpr int kStftFrames = 8;         // frames per block of the transform
constexpr int kIstftRunPerLead = 8;    // inverse: run length per (lead-in + 1) frames
constexpr int kIstftPair = 2;                     // inverse: sources of one mixture per block

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// periodic Hann window: w[i] = (1 - cos(2 pi i / NFFT)) / 2
template <int NFFT>
__device__ __forceinline__ float hann(int i) {
  return 0.5f - 0.5f * cospif(2.0f * (float)i / (float)NFFT);
}

// the window w[i] into LDS
template <int NFFT>
__device__ __forceinline__ void window(float *win) {
  for (int i = threadIdx.x; i < NFFT; i += kStftThreads) win[i] = hann<NFFT>(i);
}

// ns of the first radix-4 pass that has twiddles (4, or 2 after a radix-2 pass)
template <int L>
constexpr int first_twiddled() { return ilog2(L) % 2 ? 2 : 4; }

// Word a of a transform buffer is kept at sw(a): bits 2-3 and 4-5 of a are
// XORed with bits 6-7.  The stores of the passes of size 4 and 16 (groups of 4
// or 16 words, 16 or 64 apart) then spread over every bank, for 32 or 64 banks,
// and 64 consecutive words stay conflict-free.  Bits 0-1 are kept, so the 2- and
// 4-word stores of the first pass stay contiguous and aligned.
__device__ __forceinline__ int sw(int a) { return a ^ (((a >> 6) & 3) * 20); }

// Twiddles of the radix-4 passes with ns > 1, pass by pass in the order they run:
// the pass of size ns keeps exp(sign i pi r k / (2 ns)) for r = 1, 2, 3 and
// k < ns at off + (r - 1) ns + k (off = 3 x the sizes of the passes before), so a
// wave's lanes read consecutive words.  Fewer than L entries.
template <int L, int SIGN>
__device__ __forceinline__ void twiddles(float *twr, float *twi) {
  int off = 0;
  for (int ns = first_twiddled<L>(); ns < L; ns *= 4) {
    for (int e = threadIdx.x; e < 3 * ns; e += kStftThreads) {
      const int r = e / ns + 1, k = e - (r - 1) * ns;
      float s, c;
      sincospif((float)SIGN * (float)(r * k) / (float)(2 * ns), &s, &c);
      twr[off + e] = c;
      twi[off + e] = s;
    }
    off += 3 * ns;
  }
}

// 4-point DFT in place, exp(SIGN 2 pi i / 4) = SIGN i
template <int SIGN>
__device__ __forceinline__ void dft4(float (&vr)[4], float (&vi)[4]) {
  const float ar = vr[0] + vr[2], ai = vi[0] + vi[2];
  const float br = vr[0] - vr[2], bi = vi[0] - vi[2];
  const float cr = vr[1] + vr[3], ci = vi[1] + vi[3];
  const float dr = (float)-SIGN * (vi[1] - vi[3]), di = (float)SIGN * (vr[1] - vr[3]);   // (v1 - v3) SIGN i
  vr[0] = ar + cr;
  vi[0] = ai + ci;
  vr[1] = br + dr;
  vi[1] = bi + di;
  vr[2] = ar - cr;
  vi[2] = ai - ci;
  vr[3] = br - dr;
  vi[3] = bi - di;
}

// inputs r = 1..3 of butterfly k of the pass of size ns times their twiddles
__device__ __forceinline__ void twiddle3(float (&vr)[4], float (&vi)[4], const float *twr, const float *twi,
                                         int off, int ns, int k) {
#pragma unroll
  for (int r = 1; r < 4; ++r) {
    const float c = twr[off + (r - 1) * ns + k], s = twi[off + (r - 1) * ns + k];
    const float x = vr[r], y = vi[r];
    vr[r] = x * c - y * s;
    vi[r] = x * s + y * c;
  }
}

// One radix-4 pass of size ns from (sr, si) to (dr, di), both in LDS; the
// calling thread takes butterflies j0, j0 + stride, ...
template <int L, int SIGN>
__device__ __forceinline__ void pass4(const float *sr, const float *si, float *dr, float *di, const float *twr,
                                      const float *twi, int off, int ns, int j0, int stride) {
  constexpr int Q = L / 4;
  for (int j = j0; j < Q; j += stride) {
    const int k = j & (ns - 1);
    float vr[4], vi[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      vr[r] = sr[sw(j + r * Q)];
      vi[r] = si[sw(j + r * Q)];
    }
    twiddle3(vr, vi, twr, twi, off, ns, k);
    dft4<SIGN>(vr, vi);
    const int d = (j - k) * 4 + k;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      dr[sw(d + r * ns)] = vr[r];
      di[sw(d + r * ns)] = vi[r];
    }
  }
}

// The passes between the first and the last.  The first pass has left its output
// in (sr, si) before a barrier; on return (sr, si) hold the input of the last pass
// (ns = L/4), written before a barrier, and the result is that pass's twiddle
// offset.
template <int L, int SIGN>
__device__ __forceinline__ int middle_passes(float *&sr, float *&si, float *&dr, float *&di, const float *twr,
                                             const float *twi, int j0 = threadIdx.x, int stride = kStftThreads) {
  int off = 0;
  for (int ns = first_twiddled<L>(); ns < L / 4; ns *= 4) {
    pass4<L, SIGN>(sr, si, dr, di, twr, twi, off, ns, j0, stride);
    off += 3 * ns;
    __syncthreads();
    float *tr = sr, *ti = si;
    sr = dr;
    si = di;
    dr = tr;
    di = ti;
  }
  return off;
}

// The last pass's butterfly j: inputs j + r L/4 from (sr, si); on return
// (vr[r], vi[r]) is bin j + r L/4.
template <int L, int SIGN>
__device__ __forceinline__ void last_pass(const float *sr, const float *si, const float *twr, const float *twi,
                                          int off, int j, float (&vr)[4], float (&vi)[4]) {
  constexpr int Q = L / 4;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    vr[r] = sr[sw(j + r * Q)];
    vi[r] = si[sw(j + r * Q)];
  }
  twiddle3(vr, vi, twr, twi, off, Q, j);
  dft4<SIGN>(vr, vi);
}

template <int NFFT>
__global__ __launch_bounds__(kStftThreads) void k_stft(const float *__restrict__ x, int64_t n, int hop, int T,
                                                       float *__restrict__ mag, float *__restrict__ phase) {
  // The real windowed frame u is transformed as z[m] = u[2m] + i u[2m+1] with an
  // H = NFFT/2 point FFT Z; with Ze = (Z[k] + conj Z[H-k]) / 2 and Zo = (Z[k] -
  // conj Z[H-k]) / 2i, X[k] = Ze + exp(-2 pi i k / NFFT) Zo and X[H-k] = conj(Ze -
  // exp(-2 pi i k / NFFT) Zo).
  constexpr int H = NFFT / 2, F = H + 1, Q = H / 4, P = H / 2 + 1;
  constexpr bool kOdd = ilog2(H) % 2 == 1;
  // the first pass writes 2 or 4 consecutive words per lane
  __shared__ __align__(16) float re[H];
  __shared__ __align__(16) float im[H];
  __shared__ __align__(16) float re2[H];
  __shared__ __align__(16) float im2[H];
  __shared__ float twr[H], twi[H], win[NFFT], er[P], ei[P];
  const int b = blockIdx.y;
  const int t0 = blockIdx.x * kStftFrames, t1 = min(T, t0 + kStftFrames);
  twiddles<H, -1>(twr, twi);
  window<NFFT>(win);
  for (int k = threadIdx.x; k < P; k += kStftThreads) sincospif(-2.0f * (float)k / (float)NFFT, &ei[k], &er[k]);
  // first pass: radix 4 (radix 2 when log2 H is odd) over H / kR butterflies,
  // input r of butterfly j being z[j + r H / kR]; each thread holds its
  // butterflies' samples for the next frame in registers, loaded while the
  // current frame's passes run
  constexpr int kR = kOdd ? 2 : 4, kBf = H / kR, kPer = (kBf + kStftThreads - 1) / kStftThreads;
  float xv[kPer][kR][2];
  auto load = [&](int t) {
    const float *xs = x + (size_t)b * n + (size_t)t * hop;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int j = threadIdx.x + q * kStftThreads;
#pragma unroll
      for (int r = 0; r < kR; ++r) {
        const int m = j + r * kBf;
        xv[q][r][0] = j < kBf ? xs[2 * m] : 0.0f;
        xv[q][r][1] = j < kBf ? xs[2 * m + 1] : 0.0f;
      }
    }
  };
  if (t0 < t1) load(t0);
  for (int t = t0; t < t1; ++t) {
    __syncthreads();   // the tables are written; the previous frame's bins are read
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int j = threadIdx.x + q * kStftThreads;
      if (j >= kBf) break;
      float vr[kR], vi[kR];
#pragma unroll
      for (int r = 0; r < kR; ++r) {
        const int m = j + r * kBf;
        vr[r] = xv[q][r][0] * win[2 * m];
        vi[r] = xv[q][r][1] * win[2 * m + 1];
      }
      if constexpr (kOdd) {
        reinterpret_cast<float2 *>(re)[sw(2 * j) >> 1] = make_float2(vr[0] + vr[1], vr[0] - vr[1]);
        reinterpret_cast<float2 *>(im)[sw(2 * j) >> 1] = make_float2(vi[0] + vi[1], vi[0] - vi[1]);
      } else {
        dft4<-1>(vr, vi);
        reinterpret_cast<float4 *>(re)[sw(4 * j) >> 2] = make_float4(vr[0], vr[1], vr[2], vr[3]);
        reinterpret_cast<float4 *>(im)[sw(4 * j) >> 2] = make_float4(vi[0], vi[1], vi[2], vi[3]);
      }
    }
    if (t + 1 < t1) load(t + 1);
    __syncthreads();
    float *sr = re, *si = im, *dr = re2, *di = im2;
    const int off = middle_passes<H, -1>(sr, si, dr, di, twr, twi);
    // last pass: Z[j + r H/4] into the free buffer, for the pairs (k, H - k)
    for (int j = threadIdx.x; j < Q; j += kStftThreads) {
      float vr[4], vi[4];
      last_pass<H, -1>(sr, si, twr, twi, off, j, vr, vi);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        dr[sw(j + r * Q)] = vr[r];
        di[sw(j + r * Q)] = vi[r];
      }
    }
    __syncthreads();
    const size_t o = ((size_t)b * T + t) * F;
    for (int k = threadIdx.x; k < P; k += kStftThreads) {
      const int h = k == 0 ? 0 : H - k;
      const float zkr = dr[sw(k)], zki = di[sw(k)], zhr = dr[sw(h)], zhi = di[sw(h)];
      const float eer = 0.5f * (zkr + zhr), eei = 0.5f * (zki - zhi);      // Ze
      const float oor = 0.5f * (zki + zhi), ooi = -0.5f * (zkr - zhr);     // Zo
      const float c = er[k], s = ei[k];
      const float pr = c * oor - s * ooi, pi = c * ooi + s * oor;        // exp(-2 pi i k / NFFT) Zo
      const float xr = eer + pr, xi = eei + pi;
      mag[o + k] = hypotf(xr, xi);
      phase[o + k] = atan2f(xi, xr);
      if (k == 0 || k < H - k) {   // X[H] = Ze - Zo at k = 0, else X[H - k] = conj(Ze - e Zo)
        const float yr = eer - pr, yi = k == 0 ? eei - pi : -(eei - pi);
        mag[o + H - k] = hypotf(yr, yi);
        phase[o + H - k] = atan2f(yi, yr);
      }
    }
  }
}

template <int NFFT>
__global__ __launch_bounds__(kStftThreads) void k_istft(const float *__restrict__ mag, const float *__restrict__ phase,
                                                        int S, int T, int hop, int G, int64_t n,
                                                        float *__restrict__ y) {
  // The real frame of a Hermitian spectrum X comes from an H = NFFT/2 point
  // complex inverse transform: with Z[k] = (X[k] + conj X[H-k]) + i e_k (X[k] -
  // conj X[H-k]), e_k = exp(2 pi i k / NFFT), its inverse z gives z[m] =
  // y[2m] + i y[2m+1].  A block takes kIstftPair sources of one mixture, which
  // share the phase (its loads and sincos, folded for both sources by the same
  // thread) and the squared-window ring; their transforms run side by side, the
  // block's threads split between them, so every pass keeps all threads busy and
  // each barrier serves both.
  constexpr int H = NFFT / 2, F = H + 1, Q = H / 4, P = H / 2 + 1;   // P pairs (k, H - k), k <= H/2
  constexpr bool kOdd = ilog2(H) % 2 == 1;
  constexpr int TPS = kStftThreads / kIstftPair;   // threads per source in the passes
  // the first pass writes 2 or 4 consecutive words per lane
  __shared__ __align__(16) float re[kIstftPair][H];
  __shared__ __align__(16) float im[kIstftPair][H];
  __shared__ __align__(16) float re2[kIstftPair][H];
  __shared__ __align__(16) float im2[kIstftPair][H];
  __shared__ float twr[H], twi[H], win[NFFT], er[P], ei[P];
  __shared__ float acc[kIstftPair][NFFT], wacc[NFFT];   // rings: slot i mod NFFT holds sample i
  const int groups = (S + kIstftPair - 1) / kIstftPair;
  const int mix = blockIdx.y / groups, s0 = (blockIdx.y - mix * groups) * kIstftPair;
  const int ns = min(kIstftPair, S - s0);
  const int t0 = blockIdx.x * G, t1 = min(T, t0 + G);
  const int lead = (NFFT + hop - 1) / hop - 1;   // frames before t0 that cover samples >= t0 hop
  const int ts = max(0, t0 - lead);
  const int sl = threadIdx.x / TPS, lt = threadIdx.x - sl * TPS;   // this thread's source in the passes
  twiddles<H, 1>(twr, twi);
  window<NFFT>(win);
  for (int k = threadIdx.x; k < P; k += kStftThreads) sincospif(2.0f * (float)k / (float)NFFT, &ei[k], &er[k]);
  for (int i = threadIdx.x; i < NFFT; i += kStftThreads) {
#pragma unroll
    for (int s = 0; s < kIstftPair; ++s) acc[s][i] = 0.0f;
    wacc[i] = 0.0f;
  }
  // each thread's pairs of bins (k, H - k) of the next frame, loaded while the
  // current frame's passes run
  constexpr int kPerP = (P + kStftThreads - 1) / kStftThreads;
  float ma[kPerP][kIstftPair], mb[kPerP][kIstftPair], pa[kPerP], pb[kPerP];
  auto load = [&](int t) {
    const float *ps = phase + ((size_t)mix * T + t) * F;
#pragma unroll
    for (int q = 0; q < kPerP; ++q) {
      const int k = threadIdx.x + q * kStftThreads;
      const bool in = k < P;
      pa[q] = in ? ps[k] : 0.0f;
      pb[q] = in ? ps[H - k] : 0.0f;
#pragma unroll
      for (int s = 0; s < kIstftPair; ++s) {
        const float *ms = mag + (((size_t)mix * S + s0 + s) * T + t) * F;
        ma[q][s] = in && s < ns ? ms[k] : 0.0f;
        mb[q][s] = in && s < ns ? ms[H - k] : 0.0f;
      }
    }
  };
  if (ts < t1) load(ts);
  for (int t = ts; t < t1; ++t) {
    __syncthreads();   // the tables and rings are written; the previous frame is folded in
    // this frame's bins, folded for every source: the phase's sincos once
#pragma unroll
    for (int q = 0; q < kPerP; ++q) {
      const int k = threadIdx.x + q * kStftThreads;
      if (k >= P) break;
      // the hardware sine and cosine, accurate to about 1e-6 on [-pi, pi]: the phase
      // is first reduced by whole turns (no change for a phase already in range,
      // as those of the transform are)
      float ca, sa, cb, sb;
      const float ra = pa[q] - 6.28318530717958648f * rintf(pa[q] * 0.159154943091895336f);
      const float rb = pb[q] - 6.28318530717958648f * rintf(pb[q] * 0.159154943091895336f);
      __sincosf(ra, &sa, &ca);
      __sincosf(rb, &sb, &cb);
      const float c = er[k], d = ei[k];
#pragma unroll
      for (int s = 0; s < kIstftPair; ++s) {
        // a = X[k], b = X[H - k]; bins 0 and H of a real signal are real (their
        // imaginary parts are dropped)
        const float ar = ma[q][s] * ca, ai = k == 0 ? 0.0f : ma[q][s] * sa;
        const float br = mb[q][s] * cb, bi = k == 0 ? 0.0f : mb[q][s] * sb;
        // Z[k] = u + i e v, u = a + conj b, v = a - conj b
        const float ur = ar + br, ui = ai - bi, vr = ar - br, vi = ai + bi;
        re[s][sw(k)] = ur - (c * vi + d * vr);
        im[s][sw(k)] = ui + (c * vr - d * vi);
        if (k > 0 && k < H - k) {
          // Z[H - k] from the same pair: roles of a and b swapped, e_{H-k} = -conj e_k
          const float ur2 = br + ar, ui2 = bi - ai, vr2 = br - ar, vi2 = bi + ai;
          re[s][sw(H - k)] = ur2 - (-c * vi2 + d * vr2);
          im[s][sw(H - k)] = ui2 + (-c * vr2 - d * vi2);
        }
      }
    }
    if (t + 1 < t1) load(t + 1);
    __syncthreads();
    // first pass (ns = 1, twiddles 1) from (re, im) to (re2, im2), source sl
    if constexpr (kOdd) {
      for (int j = lt; j < H / 2; j += TPS) {
        const float xr = re[sl][sw(j)], xi = im[sl][sw(j)], zr = re[sl][sw(j + H / 2)], zi = im[sl][sw(j + H / 2)];
        reinterpret_cast<float2 *>(re2[sl])[sw(2 * j) >> 1] = make_float2(xr + zr, xr - zr);
        reinterpret_cast<float2 *>(im2[sl])[sw(2 * j) >> 1] = make_float2(xi + zi, xi - zi);
      }
    } else {
      for (int j = lt; j < Q; j += TPS) {
        float vr[4], vi[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          vr[r] = re[sl][sw(j + r * Q)];
          vi[r] = im[sl][sw(j + r * Q)];
        }
        dft4<1>(vr, vi);
        reinterpret_cast<float4 *>(re2[sl])[sw(4 * j) >> 2] = make_float4(vr[0], vr[1], vr[2], vr[3]);
        reinterpret_cast<float4 *>(im2[sl])[sw(4 * j) >> 2] = make_float4(vi[0], vi[1], vi[2], vi[3]);
      }
    }
    __syncthreads();
    float *sr = re2[sl], *si = im2[sl], *dr = re[sl], *di = im[sl];
    const int off = middle_passes<H, 1>(sr, si, dr, di, twr, twi, lt, TPS);
    // last pass: z[m], m = j + r H/4, is samples 2m (real part) and 2m + 1
    // (imaginary part) of the frame; scaled and windowed into source sl's ring
    // (the squared window once, by the first source's threads)
    const int64_t base = (int64_t)t * hop;
    for (int j = lt; j < Q; j += TPS) {
      float vr[4], vi[4];
      last_pass<H, 1>(sr, si, twr, twi, off, j, vr, vi);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 2 * (j + r * Q);
        const int q0 = (int)((base + i) & (NFFT - 1)), q1 = (int)((base + i + 1) & (NFFT - 1));
        const float w0 = win[i], w1 = win[i + 1];
        acc[sl][q0] += vr[r] * (1.0f / (float)NFFT) * w0;
        acc[sl][q1] += vi[r] * (1.0f / (float)NFFT) * w1;
        if (sl == 0) {
          wacc[q0] += w0 * w0;
          wacc[q1] += w1 * w1;
        }
      }
    }
    __syncthreads();
    // samples [t hop, t hop + hop) are final (the last frame also owns the rest of
    // the signal: its tail, then the samples no frame covers, which are zero)
    const int64_t hi = t == T - 1 ? n : min(n, base + hop);
    for (int64_t i = base + threadIdx.x; i < hi; i += kStftThreads) {
      if (i < base + NFFT) {
        const int r = (int)(i & (NFFT - 1));
        const float w = wacc[r];
#pragma unroll
        for (int s = 0; s < kIstftPair; ++s) {
          if (s < ns && t >= t0) y[((size_t)mix * S + s0 + s) * n + i] = w > 0.0f ? acc[s][r] / w : 0.0f;
          acc[s][r] = 0.0f;
        }
        wacc[r] = 0.0f;
      } else if (t >= t0) {
#pragma unroll
        for (int s = 0; s < kIstftPair; ++s)
          if (s < ns) y[((size_t)mix * S + s0 + s) * n + i] = 0.0f;
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
  const dim3 grid((unsigned)((T + G - 1) / G), B * ((S + kIstftPair - 1) / kIstftPair));
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
