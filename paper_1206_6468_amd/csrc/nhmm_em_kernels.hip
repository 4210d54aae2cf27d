// HIP kernels of EM learning of one source's N-HMM (Section 2.1 of the paper:
// states D_t follow a Markov chain; each quantum of frame t draws an element Z
// from theta_t(D_t) and a frequency from beta(D_t, Z)).  The paper states that EM
// finds the maximum-likelihood dictionaries and transitions, with the per-frame
// weights as nuisance parameters; the steps below are derived from that model.
//
// One iteration, from parameters (beta, theta, A, pi):
//   k_em_frame   per (frame t, state d), one wavefront: P_t(f | d) = sum_z theta_t(d, z) beta(d, z, f),
//                the frame log-likelihood ll[t][d] = sum_f V_tf ln P_t(f | d) (the
//                multinomial constant dropped), and the theta update
//                theta'_t(d, z) ~ theta_t(d, z) sum_f beta(d, z, f) V_tf / P_t(f | d),
//                which needs no chain posterior (gamma_t(d) is a common factor)
//   k_em_prep    the chain's log evidence ll - max_d ll per frame
//   k_em_chain   the two sweeps of the forward-backward, side by side (one
//                wavefront each): the forward messages and ln P(V), the backward
//                messages; or the same, time-parallel: k_em_sweep_cols,
//                k_em_sweep_scan, k_em_sweep_fin
//   k_em_post    ln gamma_t(d) from the two messages, one wavefront per frame
//   k_em_xi      the pairwise marginals xi_t(i, j) summed over the frames of a
//                chunk in log space (running maximum and scaled sum), per (chunk,
//                row i), lane = column j
//   k_em_xi_reduce  the chunks' sums in order: A' ~ sum_t xi_t (rows normalised),
//                pi' = gamma_0, and the largest ln gamma of each state
//   k_em_beta    partial sums over frame chunks of
//                sum_t gamma_t(d) theta_t(d, z) V_tf / P_t(f | d)
//   k_em_beta_reduce  beta'(d, z, f) ~ beta(d, z, f) times that sum, normalised over f
// A row that receives no expected counts keeps its previous values.  Every sum runs
// in a fixed order, so a result does not depend on scheduling.  beta and theta are
// double between iterations, A and pi float32 logarithms (nhmm_em.h says why).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "launch.h"
#include "nhmm_em.h"
#include "special.h"
#include "wave.h"

namespace nfhmm {

// The descriptors are read from device memory, so the pointers in them would be
// generic (flat) to the compiler; every access below goes through these
// global-memory views instead.
typedef __attribute__((address_space(1))) double gdouble;
__device__ __forceinline__ const gdouble *gptr(const double *p) { return (const gdouble *)p; }
__device__ __forceinline__ gdouble *gptr(double *p) { return (gdouble *)p; }

__device__ __forceinline__ double wave_sum_d(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;   // the butterfly leaves the same value in every lane
}

// One wavefront per (frame t, state d), four per block; KR >= K elements in
// registers.  In every kernel below grid y is the problem of the batch and `it`
// the iteration: a problem whose iterations are done, and blocks or wavefronts
// past its own extent, return.
template <int KR>
__global__ __launch_bounds__(256) void k_em_frame(const EmDesc *__restrict__ Es, int it) {
  const EmDesc &E = Es[blockIdx.y];
  // block = (state d, four consecutive frames), one frame per wavefront: the four
  // read the same rows of beta together, so three of them find them in the L1
  // cache.  The wavefront's (frame, state) is a scalar: theta's row then sits in
  // scalar registers.
  const int G = (E.T + 3) / 4;
  if (it >= E.iters || (int)blockIdx.x >= G * E.N) return;
  const int d = blockIdx.x / G, lane = threadIdx.x & 63;
  const int t = __builtin_amdgcn_readfirstlane((blockIdx.x - d * G) * 4 + (threadIdx.x >> 6));
  if (t >= E.T) return;
  const int K = E.K, F = E.F;
  const size_t row = ((size_t)t * E.N + d) * K;
  const gdouble *theta = gptr(E.theta);
  double th[KR];
#pragma unroll
  for (int z = 0; z < KR; ++z) {
    const double x = theta[row + min(z, K - 1)];
    th[z] = z < K ? x : 0.0;
  }
  const gdouble *bd = gptr(E.beta) + (size_t)d * K * F;
  const gfloat *v = gptr(E.V) + (size_t)t * F;
  double nt[KR];
#pragma unroll
  for (int z = 0; z < KR; ++z) nt[z] = 0.0;
  double ll = 0.0;
  // the next bin's column of beta and its count are loaded while this bin's are
  // used (the loads of a bin past F read bin F - 1 and are not used)
  // rows z >= K load row K - 1 again (no branches around the loads); their theta
  // is 0, so they add exact zeros to P, and their sums are not used
  double bn[KR];
  float vn;
  {
    const int f0 = min(lane, F - 1);
#pragma unroll
    for (int z = 0; z < KR; ++z) bn[z] = bd[(size_t)min(z, K - 1) * F + f0];
    vn = v[f0];
  }
  for (int f = lane; f < F; f += 64) {
    double bz[KR];
#pragma unroll
    for (int z = 0; z < KR; ++z) bz[z] = bn[z];
    const float vv = vn;
    const int fn = min(f + 64, F - 1);
#pragma unroll
    for (int z = 0; z < KR; ++z) bn[z] = bd[(size_t)min(z, K - 1) * F + fn];
    vn = v[fn];
    if (!(vv > 0.0f)) continue;   // V = 0: no term in ll, no counts to share
    double P = 0.0;
#pragma unroll
    for (int z = 0; z < KR; ++z) P = fma(th[z], bz[z], P);
    ll += (double)vv * log(P);
    const double R = (double)vv / P;
#pragma unroll
    for (int z = 0; z < KR; ++z) nt[z] = fma(bz[z], R, nt[z]);
  }
  ll = wave_sum_d(ll);
  // every lane holds the sums; lane z writes element z of the new weights
  double tot = 0.0, mine = 0.0;
#pragma unroll
  for (int z = 0; z < KR; ++z) {
    if (z < K) {
      const double sz = th[z] * wave_sum_d(nt[z]);
      tot += sz;
      if (lane == z) mine = sz;
    }
  }
  if (lane == 0) gptr(E.ll)[(size_t)t * E.N + d] = ll;
  if (lane < K) gptr(E.theta_new)[row + lane] = tot > 0.0 ? mine / tot : theta[row + lane];
}

// The chain's log evidence of frame t (one wavefront, lane = state): the frame's
// log-likelihoods relative to their largest, which off[t] keeps (in double) for
// ln P(V).
__global__ __launch_bounds__(64) void k_em_prep(const EmDesc *__restrict__ Es, int it) {
  const EmDesc &E = Es[blockIdx.y];
  const int t = blockIdx.x, lane = threadIdx.x;
  if (it >= E.iters || t >= E.T) return;
  const bool live = lane < E.N;
  const double x = live ? E.ll[(size_t)t * E.N + lane] : -INFINITY;
  double m = x;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  const bool fin = m > -INFINITY;
  E.x[(size_t)t * 64 + lane] = (live && fin) ? (float)(x - m) : -INFINITY;
  if (lane == 0) E.off[t] = m;
}

// log-sum-exp over the live lanes of a wavefront (-inf if all are -inf)
__device__ __forceinline__ float lse_lanes(float x, bool live) {
  const float mx = wave_max(live ? x : -INFINITY);
  if (!(mx > -INFINITY)) return mx;
  return mx + __logf(wave_sum(live ? __expf(x - mx) : 0.0f));
}

// The forward-backward of the source chain, lane r = state r, in log space with
// the messages normalised per frame (the smallest probabilities the iterations
// need are far below the float32 range, and a message entry far below its
// frame's largest can still carry a marginal when the other direction's message
// favours it, so no message entry is ever flushed):
//   forward   la_t(n) = x_t(n) + lse_m(la_{t-1}(m) + ln A(m, n)), la_0 = ln pi + x_0;
//             ln Z = the sum of the frames' normalisers
//   backward  s_{t-1}(i) = lse_j(ln A(i, j) + x_t(j) + lb_t(j)), lb_{t-1} = s_{t-1}
//             normalised, lb_{T-1} = 0; both are stored, s for the pairwise
//             marginals: ln xi_t(i, j) = ln gamma_{t-1}(i) + ln A(i, j) + x_t(j) +
//             lb_t(j) - s_{t-1}(i).
// Each lane's log-sum-exp takes the largest of its N terms and sums the rest
// relative to it, so only terms negligible against that lane's own sum are lost.
//
// Two schedules.  k_em_chain runs the two sweeps side by side, one wavefront each,
// T dependent steps.  The time-parallel one cuts each sweep into chunks of
// kEmSweepChunk frames and uses that a sweep is linear in its message:
//   k_em_sweep_cols  wavefront (direction, chunk, state m) sweeps the chunk from
//                    the unit message of m: the chunk's transfer column (end
//                    message as normalised logarithms) and its log scale
//   k_em_sweep_scan  one wavefront per direction carries the true message across
//                    the chunks with those columns (a log-sum-exp per lane over
//                    the N columns), storing each chunk's start message (and
//                    ln P(V))
//   k_em_sweep_fin   wavefront (direction, chunk) sweeps its chunk again from that
//                    start, storing the messages
// The critical path is about 2 kEmSweepChunk + T / kEmSweepChunk steps instead of
// T, for N times the work; the runtime picks it for batches too small to fill the
// GPU.  Both give the same messages up to rounding.
constexpr int kAhead = 8;   // frames of evidence loaded ahead of the sweep

// A sweep's block is one wavefront, and LDS executes a wavefront's operations in
// issue order, so a read sees every lane's earlier write to buf and a write cannot
// pass an earlier read: only the compiler must not move them across each other.
// (A barrier would also wait for every global access in flight -- the evidence
// loaded ahead and the stored messages.)
__device__ __forceinline__ void lds_order() { __asm__ volatile("" ::: "memory"); }

// lse_m(buf[m] + c[m]) over NR terms for this lane: four independent partial
// maxima and sums, so that the dependent chains are NR/4 long (-inf if every term
// is -inf).
template <int NR>
__device__ __forceinline__ float lse_terms(const float *buf, const float (&c)[NR]) {
  float m4[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
#pragma unroll
  for (int m = 0; m < NR; ++m) m4[m & 3] = fmaxf(m4[m & 3], buf[m] + c[m]);
  const float mx = fmaxf(fmaxf(m4[0], m4[1]), fmaxf(m4[2], m4[3]));
  if (!(mx > -INFINITY)) return -INFINITY;
  float s4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int m = 0; m < NR; ++m) s4[m & 3] += __expf(buf[m] + c[m] - mx);
  return mx + __logf((s4[0] + s4[1]) + (s4[2] + s4[3]));
}

// Forward steps t = t0 .. t1-1 from la, the normalised message of frame t0-1.  ac
// is column r of ln A.  Returns the sum of the normalisers; STORE keeps the
// messages.  Each frame's evidence row is loaded kAhead frames before its step
// (clamped to the last frame: always in bounds), in whole rounds of kAhead steps;
// the last few steps load their own.
template <int NR, bool STORE>
__device__ __forceinline__ double fwd_steps(const gfloat *x, gfloat *lag, const float (&ac)[NR], float *buf,
                                            bool live, int r, int t0, int t1, int T, float &la) {
  double z = 0.0;
  auto step = [&](int t, float xt) {
    buf[r] = la;
    lds_order();
    const float s = lse_terms<NR>(buf, ac);
    lds_order();
    const float l = (live && s > -INFINITY) ? xt + s : -INFINITY;
    const float c = lse_lanes(l, live);
    la = (live && c > -INFINITY) ? l - c : -INFINITY;
    if (STORE) lag[(size_t)t * 64 + r] = la;
    z += (double)c;
  };
  float xq[kAhead];
#pragma unroll
  for (int q = 0; q < kAhead; ++q) xq[q] = x[(size_t)min(t0 + q, T - 1) * 64 + r];
  int t = t0;
  for (; t + kAhead <= t1; t += kAhead) {
#pragma unroll
    for (int q = 0; q < kAhead; ++q) {
      const float xt = xq[q];
      xq[q] = x[(size_t)min(t + q + kAhead, T - 1) * 64 + r];
      step(t + q, xt);
    }
  }
  for (; t < t1; ++t) step(t, x[(size_t)t * 64 + r]);
  return z;
}

// Backward steps t = t0, t0-1, .., t1+1 from lb, the message of frame t0; each
// gives s_{t-1} and lb_{t-1}.  ar is row r of ln A.  Returns the sum of the
// normalisers; STORE keeps s and the messages.  Evidence is loaded ahead as above
// (clamped to frame 0).
template <int NR, bool STORE>
__device__ __forceinline__ double bwd_steps(const gfloat *x, gfloat *sIg, gfloat *lbg, const float (&ar)[NR],
                                            float *buf, bool live, int r, int t0, int t1, float &lb) {
  double z = 0.0;
  auto step = [&](int t, float xt) {
    buf[r] = live ? xt + lb : -INFINITY;
    lds_order();
    const float s = lse_terms<NR>(buf, ar);
    lds_order();
    const float sI = live ? s : -INFINITY;
    const float cb = lse_lanes(sI, live);
    lb = (live && cb > -INFINITY) ? sI - cb : -INFINITY;
    if (STORE) {
      sIg[(size_t)(t - 1) * 64 + r] = sI;
      lbg[(size_t)(t - 1) * 64 + r] = lb;
    }
    z += (double)cb;
  };
  float xq[kAhead];
#pragma unroll
  for (int q = 0; q < kAhead; ++q) xq[q] = x[(size_t)max(t0 - q, 0) * 64 + r];
  int t = t0;
  for (; t - kAhead >= t1; t -= kAhead) {
#pragma unroll
    for (int q = 0; q < kAhead; ++q) {
      const float xt = xq[q];
      xq[q] = x[(size_t)max(t - q - kAhead, 0) * 64 + r];
      step(t - q, xt);
    }
  }
  for (; t > t1; --t) step(t, x[(size_t)t * 64 + r]);
  return z;
}

// Column r (forward) or row r (backward) of ln A; -inf past N.
template <int NR>
__device__ __forceinline__ void a_lane(const float *lnA, int N, int r, bool col, float (&a)[NR]) {
  const bool live = r < N;
#pragma unroll
  for (int j = 0; j < NR; ++j)
    a[j] = (live && j < N) ? lnA[col ? (size_t)j * N + r : (size_t)r * N + j] : -INFINITY;
}

// The normalised first forward message, and its normaliser.
__device__ __forceinline__ float fwd_first(const EmDesc &E, bool live, int r, double &z) {
  const float l0 = live ? E.lnpi[r] + E.x[r] : -INFINITY;
  const float c = lse_lanes(l0, live);
  z = (double)c;
  return (live && c > -INFINITY) ? l0 - c : -INFINITY;
}

// ln P(V) = sum_t off_t + ln Z of the relative evidence
__device__ __forceinline__ void put_trace(const EmDesc &E, int it, int r, double z) {
  double off = 0.0;
  for (int t = r; t < E.T; t += 64) off += E.off[t];
  off = wave_sum_d(off);
  if (r == 0) E.trace[it] = off + z;
}

// The sequential schedule: block 0 sweeps forward, block 1 backward (problems on
// the time-parallel one return).
template <int NR>
__global__ __launch_bounds__(64) void k_em_chain(const EmDesc *__restrict__ Es, int it) {
  const EmDesc &E = Es[blockIdx.y];
  if (it >= E.iters || E.nsw > 0) return;
  const int r = threadIdx.x, N = E.N, T = E.T;
  const bool live = r < N;
  __shared__ float buf[64];
  float a[NR];
  if (blockIdx.x == 0) {
    a_lane<NR>(E.lnA, N, r, true, a);
    double z;
    float la = fwd_first(E, live, r, z);
    E.la[r] = la;
    z += fwd_steps<NR, true>(gptr(E.x), gptr(E.la), a, buf, live, r, 1, T, T, la);
    put_trace(E, it, r, z);
  } else {
    a_lane<NR>(E.lnA, N, r, false, a);
    float lb = live ? 0.0f : -INFINITY;
    E.lbn[(size_t)(T - 1) * 64 + r] = lb;
    bwd_steps<NR, true>(gptr(E.x), gptr(E.sI), gptr(E.lbn), a, buf, live, r, T - 1, 0, lb);
  }
}

// Forward chunk c covers the steps t = 1 + c L .. min(1 + (c + 1) L, T) - 1, and
// backward chunk c the steps t = T - 1 - c L down to max(T - 1 - (c + 1) L, 0) + 1
// (L = kEmSweepChunk).
__device__ __forceinline__ int fwd_chunk_begin(int c) { return 1 + c * kEmSweepChunk; }
__device__ __forceinline__ int bwd_chunk_begin(int T, int c) { return T - 1 - c * kEmSweepChunk; }

// Block (direction, chunk c, state m): the chunk swept from the unit message of
// m.  tm[dir][c][m][n] = the normalised end message (lane n, logarithms),
// tz[dir][c][m] = the sum of its normalisers.
template <int NR>
__global__ __launch_bounds__(64) void k_em_sweep_cols(const EmDesc *__restrict__ Es, int it) {
  const EmDesc &E = Es[blockIdx.y];
  const int N = E.N, C = E.nsw, T = E.T;
  if (it >= E.iters || (int)blockIdx.x >= 2 * C * N) return;
  const int dir = blockIdx.x / (C * N), rem = blockIdx.x - dir * C * N, c = rem / N, m = rem - c * N;
  const int r = threadIdx.x;
  const bool live = r < N;
  __shared__ float buf[64];
  float a[NR];
  float msg = (r == m) ? 0.0f : -INFINITY;
  double z;
  if (dir == 0) {
    a_lane<NR>(E.lnA, N, r, true, a);
    const int t0 = fwd_chunk_begin(c);
    z = fwd_steps<NR, false>(gptr(E.x), nullptr, a, buf, live, r, t0, min(t0 + kEmSweepChunk, T), T, msg);
  } else {
    a_lane<NR>(E.lnA, N, r, false, a);
    const int t0 = bwd_chunk_begin(T, c);
    z = bwd_steps<NR, false>(gptr(E.x), nullptr, nullptr, a, buf, live, r, t0, max(t0 - kEmSweepChunk, 0), msg);
  }
  const size_t col = (size_t)(dir * C + c) * N + m;
  gptr(E.tm)[col * 64 + r] = msg;
  if (r == 0) gptr(E.tz)[(size_t)(dir * C + c) * 64 + m] = z;
}

// One chunk's transfer columns as lane r sees them: tm(m, r) for the N states m
// (clamped past N: their weights are -inf) and the log scale of column r.
template <int NR>
struct ScanCols {
  float t[NR];
  double h;
};
template <int NR>
__device__ __forceinline__ void load_cols(const gfloat *tm, const gdouble *tz, int N, int r, ScanCols<NR> &k) {
#pragma unroll
  for (int m = 0; m < NR; ++m) k.t[m] = tm[(size_t)min(m, N - 1) * 64 + r];
  k.h = tz[r];
}

// The message v at a chunk's start (normalised logs) carried across it:
// v'(n) = lse_m(v(m) + h(m) + tm(m, n)), returned normalised, its normaliser added
// to z.  The weights v + h are taken relative to their largest (in double), so
// that the float log-sum-exp sees values of moderate size.
template <int NR>
__device__ __forceinline__ float scan_step(const ScanCols<NR> &k, float *buf, bool live, int r, int N, float v,
                                           double &z) {
  const double w = (live && v > -INFINITY) ? (double)v + k.h : -INFINITY;
  const double mw = (double)wave_max((float)w);   // the shift: any value near the largest
  buf[r] = (w > -INFINITY) ? (float)(w - mw) : -INFINITY;
  lds_order();
  float cm[NR];
#pragma unroll
  for (int m = 0; m < NR; ++m) cm[m] = m < N ? k.t[m] : -INFINITY;
  const float e = live ? lse_terms<NR>(buf, cm) : -INFINITY;
  lds_order();
  const float c = lse_lanes(e, live);
  z = (mw > -INFINITY && c > -INFINITY) ? z + (mw + (double)c) : -INFINITY;
  return (live && c > -INFINITY) ? e - c : -INFINITY;
}

// Block dir: the scan over the chunks, each chunk's columns loaded one chunk
// ahead.  ts[dir][c] = the message at chunk c's start (c >= 1); forward also
// ln P(V).
template <int NR>
__global__ __launch_bounds__(64) void k_em_sweep_scan(const EmDesc *__restrict__ Es, int it) {
  const EmDesc &E = Es[blockIdx.y];
  const int N = E.N, C = E.nsw, dir = blockIdx.x;
  if (it >= E.iters || C == 0) return;
  const int r = threadIdx.x;
  const bool live = r < N;
  __shared__ float buf[64];
  const gfloat *tm = gptr(E.tm) + (size_t)dir * C * N * 64;
  const gdouble *tz = gptr(E.tz) + (size_t)dir * C * 64;
  gfloat *ts = gptr(E.ts) + (size_t)dir * C * 64;
  double z = 0.0;
  float v = live ? 0.0f : -INFINITY;   // backward: lb_{T-1}
  if (dir == 0) v = fwd_first(E, live, r, z);
  const int steps = dir == 0 ? C : C - 1;   // forward carries on to the end, for ln Z
  auto load = [&](int c, ScanCols<NR> &k) {
    c = min(c, steps - 1);
    load_cols<NR>(tm + (size_t)c * N * 64, tz + (size_t)c * 64, N, r, k);
  };
  auto step = [&](int c, const ScanCols<NR> &k) {
    v = scan_step<NR>(k, buf, live, r, N, v, z);
    if (c + 1 < C) ts[(size_t)(c + 1) * 64 + r] = v;
  };
  ScanCols<NR> ka, kb;
  load(0, ka);
  int c = 0;
  for (; c + 2 <= steps; c += 2) {
    load(c + 1, kb);
    step(c, ka);
    load(c + 2, ka);
    step(c + 1, kb);
  }
  if (c < steps) step(c, ka);
  if (dir == 0) put_trace(E, it, r, z);
}

// Block (direction, chunk): the chunk swept again from its true start, storing
// the messages as k_em_chain does.
template <int NR>
__global__ __launch_bounds__(64) void k_em_sweep_fin(const EmDesc *__restrict__ Es, int it) {
  const EmDesc &E = Es[blockIdx.y];
  const int N = E.N, C = E.nsw, T = E.T;
  if (it >= E.iters || (int)blockIdx.x >= 2 * C) return;
  const int dir = blockIdx.x / C, c = blockIdx.x - dir * C, r = threadIdx.x;
  const bool live = r < N;
  __shared__ float buf[64];
  float a[NR];
  if (dir == 0) {
    a_lane<NR>(E.lnA, N, r, true, a);
    float la;
    if (c == 0) {
      double z;
      la = fwd_first(E, live, r, z);
      E.la[r] = la;
    } else {
      la = E.ts[(size_t)c * 64 + r];
    }
    const int t0 = fwd_chunk_begin(c);
    fwd_steps<NR, true>(gptr(E.x), gptr(E.la), a, buf, live, r, t0, min(t0 + kEmSweepChunk, T), T, la);
  } else {
    a_lane<NR>(E.lnA, N, r, false, a);
    float lb;
    if (c == 0) {
      lb = live ? 0.0f : -INFINITY;
      E.lbn[(size_t)(T - 1) * 64 + r] = lb;
    } else {
      lb = E.ts[(size_t)(C + c) * 64 + r];
    }
    const int t0 = bwd_chunk_begin(T, c);
    bwd_steps<NR, true>(gptr(E.x), gptr(E.sI), gptr(E.lbn), a, buf, live, r, t0, max(t0 - kEmSweepChunk, 0), lb);
  }
}

// ln gamma_t = la_t + lb_t normalised over the states: one wavefront per frame.
__global__ __launch_bounds__(64) void k_em_post(const EmDesc *__restrict__ Es, int it) {
  const EmDesc &E = Es[blockIdx.y];
  const int t = blockIdx.x, r = threadIdx.x;
  if (it >= E.iters || t >= E.T) return;
  const bool live = r < E.N;
  const float g = live ? E.la[(size_t)t * 64 + r] + E.lbn[(size_t)t * 64 + r] : -INFINITY;
  const float cg = lse_lanes(g, live);   // every lane: the reduction reads lane 63
  if (live) E.lgam[(size_t)t * E.N + r] = (cg > -INFINITY) ? g - cg : -INFINITY;
}

// sum over the frames t of chunk c (t >= 1) of xi_t(i, j), as a running maximum M
// and a sum S scaled by exp(-M): block (c, i), lane j.  Terms and sums below
// kEmLogTiny count as zero, as in a double-precision evaluation.  Lane 0 also
// keeps the chunk's largest ln gamma_t(i).
__global__ __launch_bounds__(64) void k_em_xi(const EmDesc *__restrict__ Es, int it) {
  const EmDesc &E = Es[blockIdx.y];
  const int N = E.N;
  if (it >= E.iters || (int)blockIdx.x >= E.nchunk * N) return;
  const int c = blockIdx.x / N, i = blockIdx.x - c * N, j = threadIdx.x;
  const bool live = j < N;
  const float aij = live ? E.lnA[(size_t)i * N + j] : -INFINITY;
  const int t0 = c * kEmChunk, t1 = min(E.T, t0 + kEmChunk);
  float M = -INFINITY, S = 0.0f, gmx = -INFINITY;
  for (int t = t0; t < t1; ++t) {
    gmx = fmaxf(gmx, E.lgam[(size_t)t * N + i]);
    if (t == 0) continue;
    const float lg = E.lgam[(size_t)(t - 1) * N + i];
    if (!(lg >= kEmLogTiny)) continue;   // uniform over the block
    const float v = lg + aij + E.x[(size_t)t * 64 + j] + E.lbn[(size_t)t * 64 + j] - E.sI[(size_t)(t - 1) * 64 + i];
    if (live && v >= kEmLogTiny) {
      const float d = v - M;
      const float e = __expf(-fabsf(d));
      S = d > 0.0f ? fmaf(S, e, 1.0f) : S + e;
      M = fmaxf(M, v);
    }
  }
  E.xpart[((size_t)c * N + i) * 64 + j] = make_float2(M, S);
  if (j == 0) E.gpart[(size_t)c * N + i] = gmx;
}

// Row i of the new ln A from the chunks' sums (merged in chunk order; kept if the
// row received nothing), ln pi'(i) = ln gamma_0(i), and gmax(i).  One wavefront
// per row, lane j.
__global__ __launch_bounds__(64) void k_em_xi_reduce(const EmDesc *__restrict__ Es, int it) {
  const EmDesc &E = Es[blockIdx.y];
  const int i = blockIdx.x, j = threadIdx.x, N = E.N;
  if (it >= E.iters || i >= N) return;
  const bool live = j < N;
  float M = -INFINITY, S = 0.0f, gmx = -INFINITY;
  for (int c = 0; c < E.nchunk; ++c) {
    const float2 p = E.xpart[((size_t)c * N + i) * 64 + j];
    if (p.y > 0.0f) {
      const float d = p.x - M;
      if (d > 0.0f) { S = fmaf(S, __expf(-d), p.y); M = p.x; }
      else S = fmaf(p.y, __expf(d), S);
    }
    gmx = fmaxf(gmx, E.gpart[(size_t)c * N + i]);
  }
  float lr = (live && S > 0.0f) ? M + __logf(S) : -INFINITY;
  if (lr < kEmLogTiny) lr = -INFINITY;   // an expected count that underflows a double
  const float rmx = wave_max(lr);
  const float rs = wave_sum(rmx > -INFINITY && lr > -INFINITY ? __expf(lr - rmx) : 0.0f);
  const float lrs = rmx + __logf(rs);
  if (live) E.lnA_new[(size_t)i * N + j] = rmx > -INFINITY ? lr - lrs : E.lnA[(size_t)i * N + j];
  if (j == 0) {
    const float g0 = E.lgam[i];
    E.lnpi_new[i] = g0 >= kEmLogTiny ? g0 : -INFINITY;
    E.gmax[i] = gmx;
  }
}

// Partial sums of the beta update over one chunk of frames: lane = bin f of a
// 64-bin tile, block (tile, state d, chunk).  theta_t(d, .) and gamma_t(d) are the
// same for every lane: the chunk's are staged in LDS first, and each lane's counts
// of the chunk's frames loaded at once, so that the frames' loads overlap instead
// of each frame waiting for its own.  KR >= K elements in registers.
template <int KR>
__global__ __launch_bounds__(64) void k_em_beta(const EmDesc *__restrict__ Es, int it) {
  const EmDesc &E = Es[blockIdx.y];
  const int K = E.K, F = E.F, N = E.N, ftiles = (F + 63) / 64;
  if (it >= E.iters || (int)blockIdx.x >= ftiles * N * E.nchunk) return;
  // block = (bin tile, state d, frame chunk c)
  const int ft = blockIdx.x % ftiles, dc = blockIdx.x / ftiles, d = dc % N, c = dc / N;
  const int lane = threadIdx.x, f = ft * 64 + lane;
  const bool in = f < F;
  const float gmx = gptr(E.gmax)[d];
  const gdouble *beta = gptr(E.beta), *theta = gptr(E.theta);
  const gfloat *V = gptr(E.V), *lgam = gptr(E.lgam);
  const int t0 = c * kEmChunk, nt = min(E.T, t0 + kEmChunk) - t0;
  __shared__ double ths[kEmChunk][KR];   // theta_t(d, z) of the chunk's frames (0 for z >= K)
  __shared__ double gs[kEmChunk];        // gamma_t(d) relative to the state's largest
  for (int i = lane; i < kEmChunk * KR; i += 64) {
    const int tt = i / KR, z = i - tt * KR;
    ths[tt][z] = (tt < nt && z < K) ? theta[((size_t)(t0 + tt) * N + d) * K + z] : 0.0;
  }
  if (lane < kEmChunk) {
    // gamma relative to the state's largest: the row is normalised over f, so the
    // per-state scale cancels, and frames far below the largest still count
    const float lg = lane < nt ? lgam[(size_t)(t0 + lane) * N + d] : -INFINITY;
    gs[lane] = lg >= kEmLogTiny ? exp((double)(lg - gmx)) : 0.0;
  }
  float vq[kEmChunk];
#pragma unroll
  for (int i = 0; i < kEmChunk; ++i) vq[i] = (in && i < nt) ? V[(size_t)(t0 + i) * F + f] : 0.0f;
  double bz[KR], acc[KR];
#pragma unroll
  for (int z = 0; z < KR; ++z) {
    // rows z >= K load row K - 1 again (no branches around the loads); theta is 0
    // for those rows, and their sums are not stored
    bz[z] = in ? beta[((size_t)d * K + min(z, K - 1)) * F + f] : 0.0;
    acc[z] = 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kEmChunk; ++i) {
    if (i >= nt) continue;   // uniform over the block
    double tz[KR];
    double P = 0.0;
#pragma unroll
    for (int z = 0; z < KR; ++z) {
      tz[z] = ths[i][z];
      P = fma(tz[z], bz[z], P);
    }
    const double g = gs[i];
    const float vv = vq[i];
    const double gr = (vv > 0.0f && g > 0.0) ? g * ((double)vv / P) : 0.0;
#pragma unroll
    for (int z = 0; z < KR; ++z) acc[z] = fma(tz[z], gr, acc[z]);
  }
  if (in) {
    gdouble *out = gptr(E.bpart) + ((size_t)c * N + d) * K * F;
#pragma unroll
    for (int z = 0; z < KR; ++z)
      if (z < K) out[(size_t)z * F + f] = acc[z];
  }
}

// beta'(d, z, .) for one row (d, z): the chunks' partial sums in order, times
// beta(d, z, f), normalised over f (the row is kept if it received nothing).
__global__ __launch_bounds__(256) void k_em_beta_reduce(const EmDesc *__restrict__ Es, int it) {
  const EmDesc &E = Es[blockIdx.y];
  const int rw = blockIdx.x, F = E.F, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (it >= E.iters || rw >= E.N * E.K) return;
  const size_t NKF = (size_t)E.N * E.K * F;
  __shared__ double red[4];
  __shared__ double total;
  const gdouble *brow = gptr(E.beta) + (size_t)rw * F, *bpart = gptr(E.bpart);
  gdouble *nrow = gptr(E.beta_new) + (size_t)rw * F;
  double s = 0.0;
  for (int f = tid; f < F; f += 256) {
    double acc = 0.0;
    // unrolled so that eight chunks' loads are in flight together; the sum keeps
    // its order
#pragma unroll 8
    for (int c = 0; c < E.nchunk; ++c) acc += bpart[(size_t)c * NKF + (size_t)rw * F + f];
    const double x = brow[f] * acc;
    nrow[f] = x;
    s += x;
  }
  s = wave_sum_d(s);
  if (lane == 0) red[wave] = s;
  __syncthreads();
  if (tid == 0) total = ((red[0] + red[1]) + red[2]) + red[3];
  __syncthreads();
  const double tot = total;
  for (int f = tid; f < F; f += 256) nrow[f] = tot > 0.0 ? nrow[f] / tot : brow[f];
}

// float32 parameters <-> working parameters (grid-stride over the largest array)
__global__ void k_em_import(int N, int K, int F, int T, const float *W, const float *theta, const float *A,
                            const float *pi, double *beta, double *th, float *lnA, float *lnpi) {
  const size_t nb = (size_t)N * K * F, nt = (size_t)T * N * K, na = (size_t)N * N;
  const size_t n = nb > nt ? nb : nt;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    if (i < nb) beta[i] = (double)W[i];
    if (i < nt) th[i] = (double)theta[i];
    if (i < na) lnA[i] = A[i] > 0.0f ? logf(A[i]) : -INFINITY;
    if (i < (size_t)N) lnpi[i] = pi[i] > 0.0f ? logf(pi[i]) : -INFINITY;
  }
}

__global__ void k_em_export(int N, int K, int F, int T, const double *beta, const double *th, const float *lnA,
                            const float *lnpi, float *W, float *theta, float *A, float *pi) {
  const size_t nb = (size_t)N * K * F, nt = (size_t)T * N * K, na = (size_t)N * N;
  const size_t n = nb > nt ? nb : nt;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    if (W && i < nb) W[i] = (float)beta[i];
    if (theta && i < nt) theta[i] = (float)th[i];
    if (A && i < na) A[i] = expf(lnA[i]);
    if (pi && i < (size_t)N) pi[i] = expf(lnpi[i]);
  }
}

hipError_t launch_em_frames(const EmBatch &B, int it, hipStream_t st) {
  const dim3 g((unsigned)((B.maxT + 3) / 4 * B.maxN), (unsigned)B.n);
  if (B.maxK <= 4) k_em_frame<4><<<g, 256, 0, st>>>(B.d, it);
  else if (B.maxK <= 8) k_em_frame<8><<<g, 256, 0, st>>>(B.d, it);
  else if (B.maxK <= 10) k_em_frame<10><<<g, 256, 0, st>>>(B.d, it);   // the paper's K
  else if (B.maxK <= 12) k_em_frame<12><<<g, 256, 0, st>>>(B.d, it);
  else if (B.maxK <= 16) k_em_frame<16><<<g, 256, 0, st>>>(B.d, it);
  else if (B.maxK <= 24) k_em_frame<24><<<g, 256, 0, st>>>(B.d, it);
  else k_em_frame<kEmMaxK><<<g, 256, 0, st>>>(B.d, it);
  k_em_prep<<<dim3((unsigned)B.maxT, (unsigned)B.n), 64, 0, st>>>(B.d, it);
  return hipGetLastError();
}

hipError_t launch_em_chain(const EmBatch &B, int it, hipStream_t st) {
  const dim3 g2(2, (unsigned)B.n), gc((unsigned)(2 * B.maxSw * B.maxN), (unsigned)B.n),
      gf((unsigned)(2 * B.maxSw), (unsigned)B.n);
#define NFHMM_EM_SWEEPS(NR)                                                 \
  do {                                                                      \
    if (B.anySeq) k_em_chain<NR><<<g2, 64, 0, st>>>(B.d, it);               \
    if (B.maxSw > 0) {                                                      \
      k_em_sweep_cols<NR><<<gc, 64, 0, st>>>(B.d, it);                      \
      k_em_sweep_scan<NR><<<g2, 64, 0, st>>>(B.d, it);                      \
      k_em_sweep_fin<NR><<<gf, 64, 0, st>>>(B.d, it);                       \
    }                                                                       \
  } while (0)
  switch ((B.maxN + 15) & ~15) {
    case 16: NFHMM_EM_SWEEPS(16); break;
    case 32: NFHMM_EM_SWEEPS(32); break;
    case 48: NFHMM_EM_SWEEPS(48); break;
    case 64: NFHMM_EM_SWEEPS(64); break;
    default: return hipErrorInvalidValue;
  }
#undef NFHMM_EM_SWEEPS
  k_em_post<<<dim3((unsigned)B.maxT, (unsigned)B.n), 64, 0, st>>>(B.d, it);
  k_em_xi<<<dim3((unsigned)(B.maxChunk * B.maxN), (unsigned)B.n), 64, 0, st>>>(B.d, it);
  k_em_xi_reduce<<<dim3((unsigned)B.maxN, (unsigned)B.n), 64, 0, st>>>(B.d, it);
  return hipGetLastError();
}

hipError_t launch_em_beta(const EmBatch &B, int it, hipStream_t st) {
  const dim3 g((unsigned)((B.maxF + 63) / 64 * B.maxN * B.maxChunk), (unsigned)B.n);
  if (B.maxK <= 4) k_em_beta<4><<<g, 64, 0, st>>>(B.d, it);
  else if (B.maxK <= 8) k_em_beta<8><<<g, 64, 0, st>>>(B.d, it);
  else if (B.maxK <= 10) k_em_beta<10><<<g, 64, 0, st>>>(B.d, it);
  else if (B.maxK <= 12) k_em_beta<12><<<g, 64, 0, st>>>(B.d, it);
  else if (B.maxK <= 16) k_em_beta<16><<<g, 64, 0, st>>>(B.d, it);
  else if (B.maxK <= 24) k_em_beta<24><<<g, 64, 0, st>>>(B.d, it);
  else k_em_beta<kEmMaxK><<<g, 64, 0, st>>>(B.d, it);
  k_em_beta_reduce<<<dim3((unsigned)(B.maxN * B.maxK), (unsigned)B.n), 256, 0, st>>>(B.d, it);
  return hipGetLastError();
}

static int em_grid(size_t n) { return (int)(n / 256 + 1 < 2048 ? n / 256 + 1 : 2048); }

hipError_t launch_em_import(int N, int K, int F, int T, const float *W, const float *theta, const float *A,
                            const float *pi, double *beta, double *th, float *lnA, float *lnpi, hipStream_t st) {
  const size_t n = std::max((size_t)N * K * F, (size_t)T * N * K);
  k_em_import<<<em_grid(n), 256, 0, st>>>(N, K, F, T, W, theta, A, pi, beta, th, lnA, lnpi);
  return hipGetLastError();
}

hipError_t launch_em_export(int N, int K, int F, int T, const double *beta, const double *th, const float *lnA,
                            const float *lnpi, float *W, float *theta, float *A, float *pi, hipStream_t st) {
  const size_t n = std::max((size_t)N * K * F, (size_t)T * N * K);
  k_em_export<<<em_grid(n), 256, 0, st>>>(N, K, F, T, beta, th, lnA, lnpi, W, theta, A, pi);
  return hipGetLastError();
}

}  // namespace nfhmm
