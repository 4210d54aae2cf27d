// Digamma and log-gamma in float32 for the expected log mixture weights of
// Eqs. 7-8 (psi(alpha_k) - psi(sum_k alpha_k)) and the Dirichlet terms of the
// evidence lower bound.  Written from the textbook series, not from any vendor
// library:
//   psi:    recurrence psi(x) = psi(x + n) - sum_{i<n} 1/(x + i)
//           (Abramowitz & Stegun 6.3.5) to x >= 4, then the asymptotic series
//           ln x - 1/(2x) - sum_n B_2n / (2n x^2n)  (A&S 6.3.18).
//   lngamma: recurrence lnG(x) = lnG(x + n) - ln prod_{i<n}(x + i) to x >= 4,
//           then Stirling's series (A&S 6.1.40):
//           (x - 1/2) ln x - x + ln(2 pi)/2 + sum_n B_2n / (2n (2n-1) x^(2n-1)).
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

// psi and ln Gamma share one shift: for x < 4, p = x (x+1) (x+2) (x+3), dp = p'
// (accumulated by the product rule, all terms positive) and xs = x + 4; else
// p = 1, dp = 0, xs = x.  Then, with the Bernoulli numbers B_2n,
//   psi(x) = ln xs - 1/(2 xs) - sum_{n=1..5} B_2n / (2n xs^2n) - dp / p
//   lnG(x) = (xs - 1/2) ln xs - xs + ln(2 pi)/2
//            + sum_{n=1..5} B_2n / (2n (2n-1) xs^(2n-1)) - ln p
// (truncation below 1e-8 for xs >= 4), so a caller that needs both -- and
// differences psi(a) - psi(b), formed as ln(xs_a / xs_b) + (rest_a - rest_b) to
// avoid cancelling two large logarithms -- evaluates ln xs once.
struct Shift8 {
  float xs, p, dp;
};

// Reciprocal, natural logarithm and exponential from the hardware
// approximations on the device (about 1 ulp; the logarithm as log2 x * ln 2, the
// exponential as 2^(x log2 e)), the C library on the host.  fast_ln is for
// normal x > 0 (the device instruction flushes subnormal inputs).
NFHMM_HD float fast_rcp(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}
NFHMM_HD float fast_ln(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_logf(x) * 0.69314718055994531f;
#else
  return logf(x);
#endif
}
NFHMM_HD float fast_exp(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_exp2f(x * 1.4426950408889634f);
#else
  return expf(x);
#endif
}

// ln x for any x > 0, subnormal included (scaled by 2^32 into the normal range
// first): the hardware log2 on the device, as fast_ln.
NFHMM_HD float ln_pos(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const bool tiny = x < 1.17549435e-38f;
  const float l2 = __builtin_amdgcn_logf(tiny ? x * 4294967296.0f : x) - (tiny ? 32.0f : 0.0f);
  return l2 * 0.69314718055994531f;
#else
  return logf(x);
#endif
}

// Without branches: the product is formed for every x and selected, so lanes of
// one wavefront with x on both sides of 4 do not diverge.
NFHMM_HD Shift8 shift8(float x) {
  float p = x, dp = 1.0f;
#pragma unroll
  for (int i = 1; i < 4; ++i) {
    const float xi = x + (float)i;
    dp = dp * xi + p;
    p = p * xi;
  }
  const bool sh = x < 4.0f;
  Shift8 r;
  r.xs = sh ? x + 4.0f : x;
  r.p = sh ? p : 1.0f;
  r.dp = sh ? dp : 0.0f;
  return r;
}

// psi(x) - ln xs
NFHMM_HD float psi_rest(const Shift8 &s) {
  const float r = fast_rcp(s.xs);
  const float r2 = r * r;
  // B2/2 = 1/12, B4/4 = -1/120, B6/6 = 1/252, B8/8 = -1/240, B10/10 = 1/132
  const float series =
      r2 * (1.0f / 12.0f - r2 * (1.0f / 120.0f - r2 * (1.0f / 252.0f - r2 * (1.0f / 240.0f - r2 * (1.0f / 132.0f)))));
  return -0.5f * r - series - s.dp * fast_rcp(s.p);
}

// ln Gamma(x) given lxs = ln xs
NFHMM_HD float lgamma_from(const Shift8 &s, float lxs) {
  const float r = fast_rcp(s.xs);
  const float r2 = r * r;
  // B2/2 = 1/12, B4/12 = -1/360, B6/30 = 1/1260, B8/56 = -1/1680, B10/90 = 1/1188
  const float series =
      r * (1.0f / 12.0f - r2 * (1.0f / 360.0f - r2 * (1.0f / 1260.0f - r2 * (1.0f / 1680.0f - r2 * (1.0f / 1188.0f)))));
  const float half_log_2pi = 0.91893853320467274f;
  // p >= 6x for a shifted x: below the normal range only for x < 2e-39
  const float lp = s.p == 1.0f ? 0.0f : (s.p >= 1.17549435e-38f ? fast_ln(s.p) : logf(s.p));
  return (s.xs - 0.5f) * lxs - s.xs + half_log_2pi + series - lp;
}

// ln Gamma(x) given lxs = ln xs, for x >= 1: the shift product p is then 1 or at
// least 1 * 2 * 3 * 4, never below the normal range, so ln p needs no guard
NFHMM_HD float lgamma_from_ge1(const Shift8 &s, float lxs) {
  const float r = fast_rcp(s.xs);
  const float r2 = r * r;
  const float series =
      r * (1.0f / 12.0f - r2 * (1.0f / 360.0f - r2 * (1.0f / 1260.0f - r2 * (1.0f / 1680.0f - r2 * (1.0f / 1188.0f)))));
  const float half_log_2pi = 0.91893853320467274f;
  const float lp = s.p == 1.0f ? 0.0f : fast_ln(s.p);
  return (s.xs - 0.5f) * lxs - s.xs + half_log_2pi + series - lp;
}

// psi(x) for x > 0
NFHMM_HD float digammaf(float x) {
  const Shift8 s = shift8(x);
  return fast_ln(s.xs) + psi_rest(s);
}

// ln Gamma(x) for x > 0
NFHMM_HD float lgammaf_pos(float x) {
  const Shift8 s = shift8(x);
  return lgamma_from(s, fast_ln(s.xs));
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
