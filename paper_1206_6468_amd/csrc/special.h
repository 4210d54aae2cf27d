// Digamma and log-gamma in float32 for the expected log mixture weights of
// Eqs. 7-8 (psi(alpha_k) - psi(sum_k alpha_k)) and the Dirichlet terms of the
// evidence lower bound.  Written from the textbook series, not from any vendor
// library:
//   psi:    recurrence psi(x) = psi(x + n) - sum_{i<n} 1/(x + i)
//           (Abramowitz & Stegun 6.3.5) to x >= 6, then the asymptotic series
//           ln x - 1/(2x) - sum_n B_2n / (2n x^2n)  (A&S 6.3.18).
//   lngamma: recurrence lnG(x) = lnG(x + n) - ln prod_{i<n}(x + i) to x >= 8,
//           then Stirling's series (A&S 6.1.41):
//           (x - 1/2) ln x - x + ln(2 pi)/2 + 1/(12x) - 1/(360x^3) + 1/(1260x^5).
// The shift sums are formed as p'/p of the product p = prod (x + i), so each
// costs one division and no cancellation (all terms positive).
#pragma once

#include <math.h>

#ifndef NFHMM_HD
#if defined(__HIPCC__)
#define NFHMM_HD __host__ __device__ __forceinline__
#else
#define NFHMM_HD inline
#endif
#endif

namespace nfhmm {

// psi(x) = ln(xs) + rest with xs = x shifted to >= 6: returns rest, writes xs.
// Differences psi(a) - psi(b) are then formed as ln(xs_a / xs_b) + (rest_a - rest_b),
// which avoids cancelling two large logarithms.
NFHMM_HD float digamma_parts(float x, float &xs) {
  float shift = 0.0f;
  if (x < 6.0f) {
    float p = 1.0f, dp = 0.0f;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      const float xi = x + (float)i;
      dp = dp * xi + p;
      p = p * xi;
    }
    shift = dp / p;
    x += 6.0f;
  }
  const float r = 1.0f / x;
  const float r2 = r * r;
  const float series = r2 * (1.0f / 12.0f - r2 * (1.0f / 120.0f - r2 * (1.0f / 252.0f - r2 * (1.0f / 240.0f))));
  xs = x;
  return -0.5f * r - series - shift;
}

// psi(x) for x > 0
NFHMM_HD float digammaf(float x) {
  float shift = 0.0f;
  if (x < 6.0f) {
    // sum_{i<6} 1/(x+i) = p'/p with p = prod_{i<6} (x+i); x+6 >= 6 afterwards
    float p = 1.0f, dp = 0.0f;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      const float xi = x + (float)i;
      dp = dp * xi + p;
      p = p * xi;
    }
    shift = dp / p;
    x += 6.0f;
  }
  const float r = 1.0f / x;
  const float r2 = r * r;
  // B2/2 = 1/12, B4/4 = -1/120, B6/6 = 1/252, B8/8 = -1/240
  const float series = r2 * (1.0f / 12.0f - r2 * (1.0f / 120.0f - r2 * (1.0f / 252.0f - r2 * (1.0f / 240.0f))));
  return logf(x) - 0.5f * r - series - shift;
}

// ln Gamma(x) for x > 0
NFHMM_HD float lgammaf_pos(float x) {
  float lshift = 0.0f;
  if (x < 8.0f) {
    float p = x;
#pragma unroll
    for (int i = 1; i < 8; ++i) p *= (x + (float)i);
    lshift = logf(p);
    x += 8.0f;
  }
  const float r = 1.0f / x;
  const float r2 = r * r;
  const float series = r * (1.0f / 12.0f - r2 * (1.0f / 360.0f - r2 * (1.0f / 1260.0f)));
  const float half_log_2pi = 0.91893853320467274f;
  return (x - 0.5f) * logf(x) - x + half_log_2pi + series - lshift;
}

// Error-free sum and Neumaier-compensated accumulation (float32 hi + lo).
struct Comp {
  float hi, lo;
};

NFHMM_HD Comp comp_zero() { Comp c; c.hi = 0.0f; c.lo = 0.0f; return c; }

NFHMM_HD void comp_add(Comp &c, float x) {
  const float t = c.hi + x;
  if (fabsf(c.hi) >= fabsf(x)) c.lo += (c.hi - t) + x;
  else c.lo += (x - t) + c.hi;
  c.hi = t;
}

NFHMM_HD Comp comp_merge(Comp a, Comp b) {
  comp_add(a, b.hi);
  a.lo += b.lo;
  return a;
}

}  // namespace nfhmm
