// Host runtime and C ABI (include/nfhmm.h).
//
// A job owns one device allocation (its arena) holding every array of
// jobdesc.h.  The engine advances a set of resident jobs in rounds: each round
// is one iteration of every resident job, issued as a handful of grouped
// launches whose blocks are dealt out over all jobs (work lists).  Blocking
// fits run rounds until their jobs are done; the serving loop runs the same
// rounds on a scheduler thread and admits queued jobs between rounds.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/nfhmm.h"
#include "host_copy.h"
#include "jobdesc.h"
#include "launch.h"
#include "nhmm_em.h"
#include "table_ring.h"

using namespace nfhmm;

// Working memory of nfhmm_fit_device_noalloc (see "scratch of the no-alloc fit" below).
constexpr size_t kNoAllocScratchBytes = size_t(96) << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {

thread_local std::string g_err = "";

nfhmm_status fail(nfhmm_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_OK(expr)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(NFHMM_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

inline int64_t rup(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// ------------------------------------------------------------------ scratch of the no-alloc fit
// Working memory of nfhmm_fit_device_noalloc: one static device array per GPU,
// held until the process ends.  In host code `scratch` names a host-side stand-in,
// not the device array: its device address is taken once per device with
// hipGetSymbolAddress (in nfhmm_create, with that device current) and only that
// address is passed to kernels.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};

// Take the current device's scratch address (device `dev` must be current).
hipError_t scratch_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev]) return hipSuccess;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[dev] = static_cast<char *>(ptr);
  return hipSuccess;
}

char *scratch_of(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[dev];
}

// ------------------------------------------------------------------ dims / layout
struct Dims {
  int S, N, K, M, Mp, F, Fp, T, iters;
  bool bf16;
};

bool dims_ok(const nfhmm_problem *p, std::string *why) {
  auto bad = [&](const char *m) { if (why) *why = m; return false; };
  if (!p) return bad("problem is NULL");
  if (p->S < 1 || p->S > NFHMM_MAX_SOURCES) return bad("S out of range [1, 8]");
  if (p->N < 1 || p->N > NFHMM_MAX_STATES) return bad("N out of range [1, 64]");
  if (p->K < 1) return bad("K must be >= 1");
  if ((int64_t)p->S * p->N * p->K > NFHMM_MAX_ELEMENTS) return bad("S*N*K exceeds NFHMM_MAX_ELEMENTS");
  if (p->F < 1 || p->F > (1 << 20)) return bad("F out of range");
  if (p->T < 1 || p->T > (1 << 22)) return bad("T out of range");
  if (p->iters < 0 || p->iters > (1 << 20)) return bad("iters out of range");
  if (!(p->gamma >= 0.0f) || !std::isfinite(p->gamma)) return bad("gamma must be finite and >= 0");
  const int64_t M = (int64_t)p->S * p->N * p->K;
  const int64_t Mp = rup(M, 32), Fp = rup(p->F, 32);
  if (p->T * std::max(Mp, Fp) * p->S >= (int64_t)1 << 31) return bad("T * max(M, F) * S too large");
  if (Fp * Mp >= (int64_t)1 << 31) return bad("F * M too large");
  if (!p->V || !p->W || !p->A || !p->pi) return bad("V, W, A and pi are required");
  return true;
}

Dims dims_of(const nfhmm_problem *p, nfhmm_precision prec) {
  Dims d;
  d.S = p->S; d.N = p->N; d.K = p->K; d.M = p->S * p->N * p->K;
  d.Mp = (int)rup(d.M, 32); d.F = (int)p->F; d.Fp = (int)rup(p->F, 32); d.T = (int)p->T;
  d.iters = p->iters; d.bf16 = prec == NFHMM_BF16;
  return d;
}

// Byte offsets of every array inside a job's arena.
struct Layout {
  size_t V_in, W_in, A_in, pi_in, alpha_init;                // host-input copies
  size_t V, Wfm, Wmf, Wfm_h, Wmf_h, wh, Rh, w, R;
  size_t alpha, c, phi, ev, sh, fwd, bwd, lnz, post, vll, clw, elbo, sep, status, chainflag, bnd, bgain, bchk;
  size_t out_alpha, out_post, out_sep, out_elbo;              // host-output staging
  size_t total;
};

}  // namespace

namespace {

Layout plan(const Dims &d, bool host_in, bool host_out, bool has_init) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += (bytes + 255) / 256 * 256; return o; };
  const size_t T = d.T, S = d.S, N = d.N, M = d.M, Mp = d.Mp, F = d.F, Fp = d.Fp;
  const size_t nlt = (Fp + 63) / 64 + 1, it = std::max(d.iters, 1);
  const size_t none = ~size_t(0);
  L.V_in = host_in ? take(T * F * 4) : none;
  L.W_in = host_in ? take(M * F * 4) : none;
  L.A_in = host_in ? take(S * N * N * 4) : none;
  L.pi_in = host_in ? take(S * N * 4) : none;
  L.alpha_init = (host_in && has_init) ? take(T * M * 4) : none;
  L.V = take(T * Fp * 4);
  L.Wfm = take(Fp * Mp * 4);
  L.Wmf = take(Fp * Mp * 4);
  L.Wfm_h = d.bf16 ? take(Fp * Mp * 2) : none;
  L.Wmf_h = d.bf16 ? take(Fp * Mp * 2) : none;
  L.wh = d.bf16 ? take(T * Mp * 2) : none;
  L.Rh = d.bf16 ? take(T * Fp * 2) : none;
  L.w = d.bf16 ? none : take(T * Mp * 4);
  L.R = d.bf16 ? none : take(T * Fp * 4);
  L.alpha = take(T * Mp * 4);
  L.c = take(T * Mp * 4);
  L.phi = take(S * T * 64 * 4);
  L.ev = take(S * T * 64 * 4);
  L.sh = take(S * T * 4);
  L.fwd = take(S * T * 64 * 4);
  L.bwd = take(S * T * 64 * 4);
  L.lnz = take(S * 8);
  L.post = take(S * T * N * 4);
  L.vll = take(nlt * T * 8);
  L.clw = take((Mp + kBoundRows - 1) / kBoundRows * T * 8);
  L.elbo = take(it * T * 8);
  L.sep = take(S * T * Fp * 4);
  L.status = take(4);
  L.chainflag = take(S * 4);
  int fbC = 1, fbL = 1;
  fb_geometry((int)T, &fbC, &fbL);
  L.bnd = take(S * 2 * 4 * (size_t)fbC * 64 * 4);
  L.bgain = take(S * 2 * (size_t)fbC * 8);
  L.bchk = take(S * 2 * (size_t)fbC * 8);
  L.out_alpha = host_out ? take(T * M * 4) : none;
  L.out_post = host_out ? take(S * T * N * 4) : none;
  L.out_sep = host_out ? take(S * T * F * 4) : none;
  L.out_elbo = host_out ? take(it * 8) : none;
  L.total = off;
  return L;
}

// ------------------------------------------------------------------ host validation
// The checks run over every input element at submit, so their loops are kept
// free of early exits and calls: one pass of compares and adds that the host
// compiler turns into vector code; only a failing input is scanned again to
// name the offending entry.

// finite and >= 0 (NaN fails both compares)
inline int bad_value(float v) { return !(v >= 0.0f && v <= 3.40282347e38f); }

bool all_finite_nonneg(const float *x, int64_t n) {
  constexpr int64_t kBlock = 4096;
  for (int64_t b = 0; b < n; b += kBlock) {
    const int64_t e = std::min(n, b + kBlock);
    int bad = 0;
    for (int64_t i = b; i < e; ++i) bad |= bad_value(x[i]);
    if (bad) return false;
  }
  return true;
}

// check_V false: the caller checks V itself (the serving path does, while copying it)
nfhmm_status validate_host(const nfhmm_problem *p, std::string *msg, bool check_V = true) {
  std::string why;
  if (!dims_ok(p, &why)) { *msg = why; return NFHMM_E_INVALID; }
  const int64_t S = p->S, N = p->N, K = p->K, M = S * N * K, F = p->F, T = p->T;
  char buf[256];
  if (check_V && !all_finite_nonneg(p->V, T * F)) {
    for (int64_t i = 0; i < T * F; ++i) {
      const float v = p->V[i];
      if (bad_value(v)) {
        snprintf(buf, sizeof buf, "V[%lld][%lld] = %g is not finite and >= 0", (long long)(i / F), (long long)(i % F), v);
        *msg = buf;
        return NFHMM_E_INVALID;
      }
    }
  }
  std::vector<unsigned char> bin_has(F, 0);
  for (int64_t k = 0; k < M; ++k) {
    const float *row = p->W + k * F;
    // eight independent partial sums (in double) so that the loop vectorises
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int bad = 0;
    int64_t l = 0;
    for (; l + 8 <= F; l += 8)
      for (int q = 0; q < 8; ++q) {
        const float w = row[l + q];
        bad |= bad_value(w);
        acc[q] += w;
        bin_has[l + q] |= (unsigned char)(w > 0.0f);
      }
    for (; l < F; ++l) {
      const float w = row[l];
      bad |= bad_value(w);
      acc[0] += w;
      bin_has[l] |= (unsigned char)(w > 0.0f);
    }
    if (bad) {
      for (l = 0; l < F; ++l)
        if (bad_value(row[l])) {
          snprintf(buf, sizeof buf, "W[%lld][%lld] = %g is not finite and >= 0", (long long)k, (long long)l, row[l]);
          *msg = buf;
          return NFHMM_E_INVALID;
        }
    }
    const double s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    if (std::fabs(s - 1.0) > 1e-4) {
      snprintf(buf, sizeof buf, "dictionary element %lld sums to %.7g, not 1", (long long)k, s);
      *msg = buf;
      return NFHMM_E_INVALID;
    }
  }
  for (int64_t l = 0; l < F; ++l) {
    if (bin_has[l]) continue;
    for (int64_t t = 0; t < T; ++t)
      if (p->V[t * F + l] > 0.0f) {
        snprintf(buf, sizeof buf, "bin %lld has V > 0 but every dictionary element is 0 there", (long long)l);
        *msg = buf;
        return NFHMM_E_INVALID;
      }
  }
  for (int64_t s = 0; s < S; ++s) {
    double ps = 0.0;
    for (int64_t i = 0; i < N; ++i) {
      const float v = p->pi[s * N + i];
      if (!(v >= 0.0f) || !std::isfinite(v)) { *msg = "pi has a negative or non-finite entry"; return NFHMM_E_INVALID; }
      ps += v;
      double rs = 0.0;
      for (int64_t j = 0; j < N; ++j) {
        const float a = p->A[(s * N + i) * N + j];
        if (!(a >= 0.0f) || !std::isfinite(a)) { *msg = "A has a negative or non-finite entry"; return NFHMM_E_INVALID; }
        rs += a;
      }
      if (std::fabs(rs - 1.0) > 1e-4) {
        snprintf(buf, sizeof buf, "row %lld of A[%lld] sums to %.7g, not 1", (long long)i, (long long)s, rs);
        *msg = buf;
        return NFHMM_E_INVALID;
      }
    }
    if (std::fabs(ps - 1.0) > 1e-4) {
      snprintf(buf, sizeof buf, "pi[%lld] sums to %.7g, not 1", (long long)s, ps);
      *msg = buf;
      return NFHMM_E_INVALID;
    }
  }
  if (p->alpha_init)
    for (int64_t i = 0; i < T * M; ++i) {
      const float a = p->alpha_init[i];
      if (!(a > 0.0f) || !std::isfinite(a)) { *msg = "alpha_init has an entry that is not finite and > 0"; return NFHMM_E_INVALID; }
    }
  return NFHMM_OK;
}

// ------------------------------------------------------------------ jobs
enum JobState { kQueued, kResident, kDone };

struct Job {
  uint64_t id = 0;
  nfhmm_problem prob{};       // pointers: device (device path) or job-owned host copies / user host memory
  Dims d{};
  nfhmm_result res{};         // destination of the outputs (host or device)
  bool host_in = false, host_out = false;
  Layout L{};
  char *arena = nullptr;
  size_t arena_bytes = 0;
  size_t charged = 0;         // bytes counted against the serving budget while admitted
  bool in_slab = false;       // arena carved from the serving slab
  size_t out_pin = ~size_t(0);  // offset of the outputs in the pinned ring (serving)
  bool out_direct[4] = {};      // alpha, post, sep, elbo: the caller's array is pinned, copied into directly
  int dev_flag = 0;             // the device status word, delivered with the outputs
  JobDesc desc{};
  nfhmm_status status = NFHMM_OK;
  std::string error;
  JobState state = kQueued;
  bool cancel = false;
  int start_round = 0;
  int finish_round = -1;      // round after which the job's outputs were queued
  double t_submit = 0.0, t_done = 0.0;
  std::unique_ptr<float[]> hV, hW, hA, hpi, hinit;   // serving: owned host copies of the inputs
};

void fill_desc(Job &j, float gamma) {
  JobDesc &D = j.desc;
  const Dims &d = j.d;
  const Layout &L = j.L;
  char *a = j.arena;
  auto F32 = [&](size_t off) { return off == ~size_t(0) ? nullptr : reinterpret_cast<float *>(a + off); };
  auto U16 = [&](size_t off) { return off == ~size_t(0) ? nullptr : reinterpret_cast<uint16_t *>(a + off); };
  D = JobDesc{};
  D.S = d.S; D.N = d.N; D.K = d.K; D.M = d.M; D.Mp = d.Mp; D.F = d.F; D.Fp = d.Fp; D.T = d.T;
  D.NK = d.N * d.K; D.iters = d.iters; D.start_round = j.start_round; D.bf16 = d.bf16 ? 1 : 0;
  D.gamma = gamma; D.nlt = (d.Fp + 63) / 64;
  const int ftail = d.F % 64;
  if (d.F >= 64 && ftail >= 1 && ftail <= 4) { D.Fm = d.F - ftail; D.Ft = ftail; }
  else { D.Fm = d.Fp; D.Ft = 0; }
  D.nsl = (D.Fm + 63) / 64;
  const double C = std::lgamma((double)d.M + (double)gamma * d.S * d.K) - (double)d.S * d.K * std::lgamma(1.0 + gamma);
  D.elbo_const = (double)d.T * C;
  if (j.host_in) {
    D.V_in = F32(L.V_in); D.W_in = F32(L.W_in); D.A_in = F32(L.A_in); D.pi_in = F32(L.pi_in);
    D.alpha_init = j.prob.alpha_init ? F32(L.alpha_init) : nullptr;
  } else {
    D.V_in = j.prob.V; D.W_in = j.prob.W; D.A_in = j.prob.A; D.pi_in = j.prob.pi; D.alpha_init = j.prob.alpha_init;
  }
  D.V = F32(L.V); D.Wfm = F32(L.Wfm); D.Wmf = F32(L.Wmf);
  D.Wfm_h = U16(L.Wfm_h); D.Wmf_h = U16(L.Wmf_h); D.wh = U16(L.wh); D.Rh = U16(L.Rh);
  D.w = F32(L.w); D.R = F32(L.R);
  D.alpha = F32(L.alpha); D.c = F32(L.c);
  D.phi = F32(L.phi); D.ev = F32(L.ev); D.sh = F32(L.sh); D.fwd = F32(L.fwd); D.bwd = F32(L.bwd);
  D.lnz = reinterpret_cast<float2 *>(a + L.lnz); D.post = F32(L.post);
  D.vll = reinterpret_cast<float2 *>(a + L.vll);
  D.clw = reinterpret_cast<float2 *>(a + L.clw);
  D.elbo = reinterpret_cast<float2 *>(a + L.elbo);
  D.sep = F32(L.sep);
  D.status = reinterpret_cast<int *>(a + L.status);
  D.chainflag = reinterpret_cast<int *>(a + L.chainflag);
  fb_geometry(d.T, &D.fbC, &D.fbL);
  D.bnd = F32(L.bnd);
  D.bgain = reinterpret_cast<float2 *>(a + L.bgain);
  D.bchk = reinterpret_cast<float2 *>(a + L.bchk);
  if (j.host_out) {
    D.out_alpha = j.res.alpha ? F32(L.out_alpha) : nullptr;
    D.out_post = j.res.post ? F32(L.out_post) : nullptr;
    D.out_sep = j.res.sep ? F32(L.out_sep) : nullptr;
    D.out_elbo = j.res.elbo ? reinterpret_cast<double *>(a + L.out_elbo) : nullptr;
  } else {
    D.out_alpha = j.res.alpha; D.out_post = j.res.post; D.out_sep = j.res.sep; D.out_elbo = j.res.elbo;
  }
}

// ------------------------------------------------------------------ work-list tables
// One table describes a set of jobs for every launch of a round: the job
// descriptors and, per launch kind, the prefix sums of blocks per job.
enum ListKind {
  kSpecF, kSpecH, kCntF, kCntH, kFBR, kFB, kPost, kChain, kUpd, kFrames, kRecon, kIters,
  kBegin, kTrans, kLam, kRatio, kNumLists
};

struct Table {
  WorkList lists[kNumLists];
  int nmax = 1, mpmax = 32, upd_stride = 32;
  // spectrum block tiles: FP32 always 64 x 64 (four blocks per CU; measured 1 %
  // faster than 128 x 64 for the paper-typical batch); BF16 128 x 128, or 64 x 64
  // when the batch would not fill the chip
  bool spec_small = false;
  char *dev = nullptr, *host = nullptr;
  size_t cap = 0;
};

// Stream and event operations of the table ring (table_ring.h).
struct HipRingOps {
  using Stream = hipStream_t;
  using Event = hipEvent_t;
  bool create(hipEvent_t *e) { return hipEventCreateWithFlags(e, hipEventDisableTiming) == hipSuccess; }
  bool record(hipEvent_t e, hipStream_t st) { return hipEventRecord(e, st) == hipSuccess; }
  bool sync(hipEvent_t e) { return hipEventSynchronize(e) == hipSuccess; }
  bool stream_wait(hipStream_t st, hipEvent_t e) { return hipStreamWaitEvent(st, e, 0) == hipSuccess; }
  void destroy(hipEvent_t e) { (void)hipEventDestroy(e); }
};
constexpr int kTableSlots = 16;

// below this many 128 x 128 blocks the BF16 spectrum runs on 64 x 64 tiles
// (four times the blocks), so that a small batch still spreads over the 256 CUs
constexpr int kSmallBatchBlocks = 256;

int spec_blocks(const JobDesc &D, bool small) {
  const int bm = small ? kSpecSmallBM : kSpecBM, bn = small ? kSpecSmallBN : kSpecBN;
  return ((D.Fm + bm - 1) / bm) * ((D.T + bn - 1) / bn);
}

int blocks_of(ListKind k, const JobDesc &D, bool bf16, int upd_wpb, bool spec_small) {
  const int ct = (D.T + 63) / 64;       // 64-frame tiles (reconstruction)
  const int spec = spec_blocks(D, spec_small);
  const int cnt = bf16 ? ((D.Mp + kCntHBM - 1) / kCntHBM) * ((D.T + kCntHBN - 1) / kCntHBN)
                       : ((D.Mp + kCntBM - 1) / kCntBM) * ((D.T + kCntBN - 1) / kCntBN);
  switch (k) {
    case kSpecF: return bf16 ? 0 : spec_blocks(D, true);
    case kSpecH: return bf16 ? spec : 0;
    case kCntF: return bf16 ? 0 : cnt;
    case kCntH: return bf16 ? cnt : 0;
    case kFBR: return 2 * D.S * D.fbC;
    case kFB: return 2 * D.S;
    case kPost: return D.S * ((D.T + 3) / 4);
    case kChain: return D.S;
    case kUpd: return (D.T + upd_wpb - 1) / upd_wpb;
    case kFrames: return D.T;
    case kRecon: return D.S * D.nlt * ct;
    case kIters: return D.iters;
    case kBegin: return (D.T + 3) / 4 + D.Mp / 4 + (D.alpha_init ? 0 : kBeginFillBlocks);
    case kTrans: return (D.Mp / 32) * (D.Fp / 32);
    case kLam: return D.alpha_init ? 0 : (D.F + kStartLamBinsPerBlock - 1) / kStartLamBinsPerBlock;
    case kRatio: return D.alpha_init ? 0 : D.T;
    default: return 0;
  }
}

}  // namespace

// ------------------------------------------------------------------ context
struct nfhmm_ctx {
  int device = 0;
  size_t budget = 0;
  int max_slots = 64;
  // Streams: lane 0's pair doubles as the context's own (stream / fb_stream).
  // HIP maps streams onto a few hardware queues per process (4 by default); the
  // context creates exactly 2 per lane so that the chain stream of a lane never
  // shares a queue with that lane's contraction stream.
  hipStream_t stream = nullptr, fb_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // execution lanes of the blocking engine: jobs are split into groups, each
  // advancing on its own pair of streams, so that one group's update and launch
  // gaps overlap the other group's contractions
  static constexpr int kMaxGroups = 2;
  int groups = 2;
  struct Lane { hipStream_t main, fb; hipEvent_t fork, join, done; } lanes[kMaxGroups] = {};
  // work-list tables: data per slot, reuse and recycling by the ring
  Table tables[kTableSlots];
  HipRingOps ring_ops;
  TableRing<HipRingOps> ring{ring_ops, kTableSlots};
  std::map<size_t, std::vector<char *>> arena_cache;   // fit paths: reusable arenas by size

  // Held while host code issues device work: by a blocking fit or chain call
  // for its whole length, by the serving scheduler for each round.  The two
  // share the streams, the table ring and the event pools.
  std::mutex engine_mu;

  // serving state
  std::mutex mu;
  std::condition_variable cv, cv_done;
  std::thread sched;
  bool stop = false;
  std::atomic<uint64_t> next_id{1};
  std::deque<Job *> queue;
  std::vector<Job *> resident;
  std::map<uint64_t, std::unique_ptr<Job>> jobs;
  size_t bytes_in_use = 0;
  int round = 0;
  std::string sched_error;
  // serving memory: one device slab of `budget` bytes, sub-allocated first fit
  // (no hipMalloc / hipFree per job: both synchronise the device)
  char *slab = nullptr;
  bool slab_tried = false;
  std::map<size_t, size_t> slab_free;   // offset -> bytes of each free range
  // host-array copies (serving and host fits): one pinned host ring, so that
  // host<->device copies are asynchronous (a copy from or to pageable memory
  // holds the calling thread until the stream reaches it, which would drain the
  // device between rounds)
  struct PinRegion { size_t off, len; hipEvent_t ev; bool done; };
  char *pin = nullptr;
  size_t pin_size = 0, pin_head = 0;
  bool pin_tried = false;
  std::deque<PinRegion> pin_regs;
  // host copies (serving inputs at submit; the ring on both sides), made on the
  // first submit or host-array fit: eleven workers beside the calling thread
  // (measured: 7 -> 11 raised saturated serving from pageable arrays by about
  // 10 %, 15 no further), fewer on a host with fewer cores
  static int copy_workers() {
    const int hc = (int)std::thread::hardware_concurrency();
    return std::max(1, std::min(11, hc > 2 ? hc - 2 : 1));
  }
  std::unique_ptr<CopyPool> copies;

  // measurement: (kind, start, end) event triples of timed launches
  bool profiling = false;
  unsigned profile_mask = ~0u;   // kinds timed while profiling
  struct Rec { int kind; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> event_pool;
  // pinned word for the no-alloc fit's status read-back (allocated at create)
  int *status_host = nullptr;
  // status words of a blocking batch, gathered on the device and read back in
  // one copy (instead of one synchronous copy per job)
  int *status_dev = nullptr, *status_pin = nullptr;
  int status_cap = 0;
};

namespace {

uint64_t new_id(nfhmm_ctx *ctx) { return ctx->next_id.fetch_add(1); }

hipError_t table_reserve(Table &t, size_t bytes) {
  if (t.cap >= bytes) return hipSuccess;
  if (t.dev) { (void)hipFree(t.dev); t.dev = nullptr; }
  if (t.host) { (void)hipHostFree(t.host); t.host = nullptr; }
  size_t cap = std::max<size_t>(bytes * 2, 1 << 16);
  hipError_t e = hipMalloc(&t.dev, cap);
  if (e != hipSuccess) return e;
  e = hipHostMalloc(&t.host, cap, hipHostMallocDefault);
  if (e != hipSuccess) return e;
  t.cap = cap;
  return hipSuccess;
}

// Build (or reuse) the table for `jobs`, to be read by launches on `st`.  The
// caller holds the returned lease until its last launch reading the table has
// been queued on `st`; the lease then records that use, and the ring rewrites the
// slot only after every recorded use has finished.
struct TableLease {
  nfhmm_ctx *ctx = nullptr;
  int slot = -1;
  hipStream_t st = nullptr;
  TableLease() = default;
  TableLease(const TableLease &) = delete;
  TableLease &operator=(const TableLease &) = delete;
  ~TableLease() {
    if (slot >= 0) (void)ctx->ring.used(slot, st);
  }
};

nfhmm_status get_table(nfhmm_ctx *ctx, const std::vector<Job *> &jobs, hipStream_t st, Table **out,
                       TableLease &lease) {
  std::vector<uint64_t> key;
  for (Job *j : jobs) key.push_back(j->id);
  bool rewrite = false;
  const int slot = ctx->ring.acquire(key, st, &rewrite);
  if (slot < 0) return fail(NFHMM_E_DEVICE, "work-list table ring: a stream or event operation failed");
  Table &t = ctx->tables[slot];
  lease.ctx = ctx;
  lease.slot = slot;
  lease.st = st;
  *out = &t;
  if (!rewrite) return NFHMM_OK;
  const int n = (int)jobs.size();
  const size_t desc_bytes = rup((int64_t)n * sizeof(JobDesc), 256);
  const size_t list_bytes = rup((int64_t)(n + 1) * sizeof(int), 256);
  const size_t total = desc_bytes + kNumLists * list_bytes;
  HIP_OK(table_reserve(t, total));
  JobDesc *hd = reinterpret_cast<JobDesc *>(t.host);
  t.nmax = 1;
  t.mpmax = 32;
  int snmax = 1;
  for (int i = 0; i < n; ++i) {
    hd[i] = jobs[i]->desc;
    t.nmax = std::max(t.nmax, jobs[i]->d.N);
    t.mpmax = std::max(t.mpmax, jobs[i]->d.Mp);
    snmax = std::max(snmax, jobs[i]->d.S * jobs[i]->d.N);
  }
  t.upd_stride = update_stride(t.mpmax, snmax);
  int big = 0;
  for (int i = 0; i < n; ++i) big += spec_blocks(jobs[i]->desc, false);
  t.spec_small = big < kSmallBatchBlocks;
  for (int k = 0; k < kNumLists; ++k) {
    int *hs = reinterpret_cast<int *>(t.host + desc_bytes + k * list_bytes);
    int acc = 0;
    for (int i = 0; i < n; ++i) {
      hs[i] = acc;
      acc += blocks_of((ListKind)k, jobs[i]->desc, jobs[i]->d.bf16, update_waves(t.upd_stride), t.spec_small);
    }
    hs[n] = acc;
    t.lists[k].jobs = reinterpret_cast<const JobDesc *>(t.dev);
    t.lists[k].start = reinterpret_cast<const int *>(t.dev + desc_bytes + k * list_bytes);
    t.lists[k].njobs = n;
    t.lists[k].total = acc;
  }
  HIP_OK(hipMemcpyAsync(t.dev, t.host, total, hipMemcpyHostToDevice, st));
  if (!ctx->ring.written(slot, st)) return fail(NFHMM_E_DEVICE, "work-list table ring: event record failed");
  return NFHMM_OK;
}

nfhmm_status arena_alloc(nfhmm_ctx *ctx, Job &j, bool cached) {
  j.arena_bytes = j.L.total;
  if (cached) {
    auto it = ctx->arena_cache.find(j.arena_bytes);
    if (it != ctx->arena_cache.end() && !it->second.empty()) {
      j.arena = it->second.back();
      it->second.pop_back();
      return NFHMM_OK;
    }
  }
  hipError_t e = hipMalloc(&j.arena, j.arena_bytes);
  if (e != hipSuccess) {
    j.arena = nullptr;
    return fail(e == hipErrorOutOfMemory ? NFHMM_E_NOMEM : NFHMM_E_DEVICE, "hipMalloc(%zu): %s", j.arena_bytes,
                hipGetErrorString(e));
  }
  return NFHMM_OK;
}

void arena_release(nfhmm_ctx *ctx, Job &j, bool cached) {
  if (!j.arena) return;
  if (cached) ctx->arena_cache[j.arena_bytes].push_back(j.arena);
  else (void)hipFree(j.arena);
  j.arena = nullptr;
}

// Serving arenas: carved from the context's slab when a budget is set (falls back
// to hipMalloc if the slab cannot be allocated).  Returns false, with nothing
// allocated, when the slab has no free range large enough right now.
bool serving_alloc(nfhmm_ctx *ctx, Job &j, nfhmm_status *err) {
  *err = NFHMM_OK;
  const size_t need = (j.L.total + 255) / 256 * 256;
  if (ctx->budget && !ctx->slab_tried) {
    ctx->slab_tried = true;
    if (hipMalloc(&ctx->slab, ctx->budget) == hipSuccess) ctx->slab_free[0] = ctx->budget;
    else { ctx->slab = nullptr; (void)hipGetLastError(); }
  }
  if (!ctx->slab) {
    *err = arena_alloc(ctx, j, false);
    return *err == NFHMM_OK;
  }
  for (auto it = ctx->slab_free.begin(); it != ctx->slab_free.end(); ++it) {
    if (it->second < need) continue;
    const size_t off = it->first, len = it->second;
    ctx->slab_free.erase(it);
    if (len > need) ctx->slab_free[off + need] = len - need;
    j.arena = ctx->slab + off;
    j.arena_bytes = need;
    j.in_slab = true;
    return true;
  }
  return false;
}

void serving_free(nfhmm_ctx *ctx, Job &j) {
  if (!j.arena) return;
  if (!j.in_slab) { arena_release(ctx, j, false); return; }
  size_t off = (size_t)(j.arena - ctx->slab), len = j.arena_bytes;
  auto next = ctx->slab_free.lower_bound(off);
  if (next != ctx->slab_free.end() && off + len == next->first) {   // merge with the following range
    len += next->second;
    next = ctx->slab_free.erase(next);
  }
  if (next != ctx->slab_free.begin()) {                              // and with the preceding one
    auto prev = std::prev(next);
    if (prev->first + prev->second == off) {
      prev->second += len;
      len = 0;
    }
  }
  if (len) ctx->slab_free[off] = len;
  j.arena = nullptr;
  j.in_slab = false;
}

constexpr size_t kPinBytes = size_t(1) << 30;

// Reserve len bytes of the pinned ring (FIFO: regions are released in the order
// they were reserved; the live ones occupy [tail, head) circularly).  Returns the
// offset, or ~0 if there is no room right now.
size_t pin_reserve(nfhmm_ctx *ctx, size_t len, hipEvent_t ev) {
  len = (len + 255) / 256 * 256;
  if (!ctx->pin_tried) {
    ctx->pin_tried = true;
    if (hipHostMalloc((void **)&ctx->pin, kPinBytes, hipHostMallocDefault) == hipSuccess) ctx->pin_size = kPinBytes;
    else { ctx->pin = nullptr; (void)hipGetLastError(); }
  }
  if (!ctx->pin || len == 0 || len >= ctx->pin_size) return ~size_t(0);
  size_t off;
  if (ctx->pin_regs.empty()) {
    off = 0;
  } else {
    const size_t tail = ctx->pin_regs.front().off, head = ctx->pin_head;
    if (head > tail) {
      if (ctx->pin_size - head >= len) off = head;
      else if (tail > len) off = 0;
      else return ~size_t(0);
    } else {
      if (tail - head > len) off = head;
      else return ~size_t(0);
    }
  }
  ctx->pin_head = off + len;
  ctx->pin_regs.push_back({off, len, ev, false});
  return off;
}

void pin_pop(nfhmm_ctx *ctx) {
  while (!ctx->pin_regs.empty() && ctx->pin_regs.front().done) {
    if (ctx->pin_regs.front().ev) (void)hipEventDestroy(ctx->pin_regs.front().ev);
    ctx->pin_regs.pop_front();
  }
  if (ctx->pin_regs.empty()) ctx->pin_head = 0;
}

// Mark upload regions whose copies have completed; drop finished regions.
void pin_poll(nfhmm_ctx *ctx) {
  for (auto &r : ctx->pin_regs)
    if (!r.done && r.ev && hipEventQuery(r.ev) == hipSuccess) r.done = true;
  pin_pop(ctx);
}

void pin_release(nfhmm_ctx *ctx, size_t off) {
  for (auto &r : ctx->pin_regs)
    if (r.off == off && !r.done) { r.done = true; break; }
  pin_pop(ctx);
}

// Is p in pinned (page-locked) host memory?  A pageable pointer is not known to
// HIP: the query then fails or reports unregistered memory, and its error is
// cleared so that no later call reports it.
bool host_pinned(const void *p) {
  if (!p) return false;
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeHost;
}

nfhmm_status download_outputs(Job &j, hipStream_t st) {
  const Dims &d = j.d;
  char *a = j.arena;
  if (j.res.alpha) HIP_OK(hipMemcpyAsync(j.res.alpha, a + j.L.out_alpha, (size_t)d.T * d.M * 4, hipMemcpyDeviceToHost, st));
  if (j.res.post)
    HIP_OK(hipMemcpyAsync(j.res.post, a + j.L.out_post, (size_t)d.S * d.T * d.N * 4, hipMemcpyDeviceToHost, st));
  if (j.res.sep) HIP_OK(hipMemcpyAsync(j.res.sep, a + j.L.out_sep, (size_t)d.S * d.T * d.F * 4, hipMemcpyDeviceToHost, st));
  if (j.res.elbo && d.iters > 0)
    HIP_OK(hipMemcpyAsync(j.res.elbo, a + j.L.out_elbo, (size_t)d.iters * 8, hipMemcpyDeviceToHost, st));
  return NFHMM_OK;
}

// Staged forms of the two copies (serving and host-array fits), through the
// pinned ring (pageable copies if the ring has no room).
nfhmm_status upload_staged(nfhmm_ctx *ctx, Job &j, hipStream_t st) {
  const Dims &d = j.d;
  const size_t nb[5] = {(size_t)d.T * d.F * 4, (size_t)d.M * d.F * 4, (size_t)d.S * d.N * d.N * 4,
                        (size_t)d.S * d.N * 4, j.prob.alpha_init ? (size_t)d.T * d.M * 4 : 0};
  const void *src[5] = {j.prob.V, j.prob.W, j.prob.A, j.prob.pi, j.prob.alpha_init};
  const size_t dst[5] = {j.L.V_in, j.L.W_in, j.L.A_in, j.L.pi_in, j.L.alpha_init};
  // arrays already in pinned memory go up directly (the blocking calls read the
  // caller's arrays while they run); the others through the ring
  bool direct[5];
  size_t total = 0, sub[5];
  for (int i = 0; i < 5; ++i) {
    direct[i] = nb[i] > 0 && host_pinned(src[i]);
    sub[i] = total;
    if (!direct[i]) total += (nb[i] + 255) / 256 * 256;
  }
  for (int i = 0; i < 5; ++i)
    if (direct[i]) HIP_OK(hipMemcpyAsync(j.arena + dst[i], src[i], nb[i], hipMemcpyHostToDevice, st));
  if (total == 0) return NFHMM_OK;
  hipEvent_t ev = nullptr;
  HIP_OK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  const size_t off = pin_reserve(ctx, total, ev);
  if (off == ~size_t(0)) {
    (void)hipEventDestroy(ev);
    for (int i = 0; i < 5; ++i)
      if (nb[i] && !direct[i]) HIP_OK(hipMemcpyAsync(j.arena + dst[i], src[i], nb[i], hipMemcpyHostToDevice, st));
    return NFHMM_OK;
  }
  CopyPool::Piece pc[5];
  int np = 0;
  for (int i = 0; i < 5; ++i)
    if (!direct[i]) pc[np++] = {ctx->pin + off + sub[i], src[i], nb[i]};
  ctx->copies->run(pc, np);
  for (int i = 0; i < 5; ++i)
    if (nb[i] && !direct[i])
      HIP_OK(hipMemcpyAsync(j.arena + dst[i], ctx->pin + off + sub[i], nb[i], hipMemcpyHostToDevice, st));
  HIP_OK(hipEventRecord(ev, st));
  return NFHMM_OK;
}

// The outputs of a host-memory job; a direct piece goes from the arena straight
// into the caller's pinned array, the others through the pinned ring.
struct OutPiece { void *dst; size_t src, bytes; bool direct; };
void out_pieces(Job &j, OutPiece (&p)[5]) {
  const Dims &d = j.d;
  p[0] = {j.res.alpha, j.L.out_alpha, (size_t)d.T * d.M * 4, j.out_direct[0]};
  p[1] = {j.res.post, j.L.out_post, (size_t)d.S * d.T * d.N * 4, j.out_direct[1]};
  p[2] = {j.res.sep, j.L.out_sep, (size_t)d.S * d.T * d.F * 4, j.out_direct[2]};
  p[3] = {d.iters > 0 ? j.res.elbo : nullptr, j.L.out_elbo, (size_t)d.iters * 8, j.out_direct[3]};
  p[4] = {&j.dev_flag, j.L.status, 4, false};
}

nfhmm_status download_staged(nfhmm_ctx *ctx, Job &j, hipStream_t st) {
  OutPiece p[5];
  out_pieces(j, p);
  size_t total = 0;
  for (auto &q : p)
    if (q.dst && !q.direct) total += (q.bytes + 255) / 256 * 256;
  const size_t off = pin_reserve(ctx, total, nullptr);
  if (off == ~size_t(0)) return download_outputs(j, st);
  j.out_pin = off;
  size_t o = off;
  for (auto &q : p) {
    if (!q.dst) continue;
    if (q.direct) {
      HIP_OK(hipMemcpyAsync(q.dst, j.arena + q.src, q.bytes, hipMemcpyDeviceToHost, st));
      continue;
    }
    HIP_OK(hipMemcpyAsync(ctx->pin + o, j.arena + q.src, q.bytes, hipMemcpyDeviceToHost, st));
    o += (q.bytes + 255) / 256 * 256;
  }
  return NFHMM_OK;
}

// After the download has completed: ring -> the caller's output arrays.
void deliver_staged(nfhmm_ctx *ctx, Job &j) {
  if (j.out_pin == ~size_t(0)) return;
  OutPiece p[5];
  out_pieces(j, p);
  size_t o = j.out_pin;
  CopyPool::Piece pc[5];
  int n = 0;
  for (auto &q : p) {
    if (!q.dst || q.direct) continue;
    pc[n++] = {q.dst, ctx->pin + o, q.bytes};
    o += (q.bytes + 255) / 256 * 256;
  }
  ctx->copies->run(pc, n);
  pin_release(ctx, j.out_pin);
  j.out_pin = ~size_t(0);
}

// ------------------------------------------------------------------ engine
// Start jobs: pack inputs, then the default start (or the warm start).
nfhmm_status engine_begin(nfhmm_ctx *ctx, const std::vector<Job *> &jobs, hipStream_t st) {
  if (jobs.empty()) return NFHMM_OK;
  {
    // packing of every job in three launches (one per step), not five per job,
    // then R of the default starts
    Table *t;
    TableLease lease;
    nfhmm_status s = get_table(ctx, jobs, st, &t, lease);
    if (s != NFHMM_OK) return s;
    HIP_OK(launch_begin(t->lists[kBegin], t->lists[kTrans], st));
    HIP_OK(launch_start_ratio(t->lists[kLam], t->lists[kRatio], st));
  }
  std::vector<Job *> uni, warm;
  for (Job *j : jobs) (j->desc.alpha_init ? warm : uni).push_back(j);
  if (!uni.empty()) {
    Table *t;
    TableLease lease;
    nfhmm_status s = get_table(ctx, uni, st, &t, lease);
    if (s != NFHMM_OK) return s;
    HIP_OK(launch_counts(t->lists[kCntF], false, st));
    HIP_OK(launch_counts(t->lists[kCntH], true, st));
    HIP_OK(launch_update(t->lists[kUpd], kUpdUniform, 0, t->upd_stride, st));
  }
  if (!warm.empty()) {
    Table *t;
    TableLease lease;
    nfhmm_status s = get_table(ctx, warm, st, &t, lease);
    if (s != NFHMM_OK) return s;
    HIP_OK(launch_update(t->lists[kUpd], kUpdFromAlpha, 0, t->upd_stride, st));
  }
  return NFHMM_OK;
}

hipEvent_t pooled_event(nfhmm_ctx *ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

// Brackets one launch with timing events when the context is profiling.
struct Timed {
  nfhmm_ctx *ctx;
  int kind;
  hipStream_t st;
  hipEvent_t a = nullptr;
  Timed(nfhmm_ctx *c, int k, hipStream_t s) : ctx(c), kind(k), st(s) {
    if (ctx->profiling && ((ctx->profile_mask >> k) & 1u)) {
      a = pooled_event(ctx);
      (void)hipEventRecord(a, st);
    }
  }
  ~Timed() {
    if (!a) return;
    hipEvent_t b = pooled_event(ctx);
    (void)hipEventRecord(b, st);
    ctx->recs.push_back({kind, a, b});
  }
};

// One iteration of every job in `jobs` (round index `round`).
nfhmm_status engine_iterate(nfhmm_ctx *ctx, const std::vector<Job *> &jobs, int round, hipStream_t st,
                            hipStream_t fb, hipEvent_t ev_fork, hipEvent_t ev_join) {
  if (jobs.empty()) return NFHMM_OK;
  Table *t;
  TableLease lease;   // the chains on fb are covered: st waits for them before the update
  nfhmm_status s = get_table(ctx, jobs, st, &t, lease);
  if (s != NFHMM_OK) return s;
  HIP_OK(hipEventRecord(ev_fork, st));
  HIP_OK(hipStreamWaitEvent(fb, ev_fork, 0));
  {
    Timed tm(ctx, NFHMM_K_CHAINS, fb);
    HIP_OK(launch_chain_fb(t->lists[kFBR], t->lists[kFB], t->nmax, fb));
  }
  {
    Timed tm(ctx, NFHMM_K_POSTERIOR, fb);
    HIP_OK(launch_posterior(t->lists[kPost], t->lists[kChain], t->nmax, fb));
  }
  HIP_OK(hipEventRecord(ev_join, fb));
  {
    Timed tm(ctx, NFHMM_K_SPECTRUM, st);
    HIP_OK(launch_spectrum(t->lists[kSpecF], false, true, st));
    HIP_OK(launch_spectrum(t->lists[kSpecH], true, t->spec_small, st));
  }
  {
    Timed tm(ctx, NFHMM_K_COUNTS, st);
    HIP_OK(launch_counts(t->lists[kCntF], false, st));
    HIP_OK(launch_counts(t->lists[kCntH], true, st));
  }
  HIP_OK(hipStreamWaitEvent(st, ev_join, 0));
  {
    Timed tm(ctx, NFHMM_K_UPDATE, st);
    HIP_OK(launch_update(t->lists[kUpd], kUpdMessages, round, t->upd_stride, st));
  }
  return NFHMM_OK;
}

nfhmm_status engine_finish(nfhmm_ctx *ctx, const std::vector<Job *> &jobs, hipStream_t st) {
  if (jobs.empty()) return NFHMM_OK;
  Table *t;
  TableLease lease;
  nfhmm_status s = get_table(ctx, jobs, st, &t, lease);
  if (s != NFHMM_OK) return s;
  HIP_OK(launch_finish(t->lists[kFrames], t->lists[kRecon], t->lists[kIters], st));
  return NFHMM_OK;
}

// Run a fixed set of jobs to completion (all start at round 0).  After packing
// and the start (on st), the jobs are dealt into up to ctx->groups groups that
// each run their rounds on their own lane; st waits for all lanes at the end.
nfhmm_status run_blocking(nfhmm_ctx *ctx, std::vector<Job *> &jobs, hipStream_t st) {
  int max_it = 0;
  for (Job *j : jobs) {
    j->start_round = 0;
    fill_desc(*j, j->prob.gamma);
    max_it = std::max(max_it, j->d.iters);
  }
  nfhmm_status s;
  // host inputs through the pinned ring (the copy pool fills it while the DMA of
  // the previous job's arrays runs); pageable copies when the ring has no room
  for (Job *j : jobs)
    if (j->host_in && (s = upload_staged(ctx, *j, st)) != NFHMM_OK) return s;
  if ((s = engine_begin(ctx, jobs, st)) != NFHMM_OK) return s;
  std::vector<Job *> done0;
  for (Job *j : jobs)
    if (j->d.iters == 0) done0.push_back(j);
  if ((s = engine_finish(ctx, done0, st)) != NFHMM_OK) return s;
  const int G = std::max(1, std::min<int>(ctx->groups, (int)jobs.size()));
  std::vector<std::vector<Job *>> grp(G);
  for (size_t i = 0; i < jobs.size(); ++i) grp[i * G / jobs.size()].push_back(jobs[i]);
  HIP_OK(hipEventRecord(ctx->ev_fork, st));
  for (int g = 0; g < G; ++g) HIP_OK(hipStreamWaitEvent(ctx->lanes[g].main, ctx->ev_fork, 0));
  for (int r = 0; r < max_it; ++r) {
    for (int g = 0; g < G; ++g) {
      nfhmm_ctx::Lane &ln = ctx->lanes[g];
      std::vector<Job *> act, fin;
      for (Job *j : grp[g]) {
        if (r < j->d.iters) act.push_back(j);
        if (r + 1 == j->d.iters) fin.push_back(j);
      }
      if ((s = engine_iterate(ctx, act, r, ln.main, ln.fb, ln.fork, ln.join)) != NFHMM_OK) return s;
      if ((s = engine_finish(ctx, fin, ln.main)) != NFHMM_OK) return s;
    }
  }
  for (int g = 0; g < G; ++g) {
    HIP_OK(hipEventRecord(ctx->lanes[g].done, ctx->lanes[g].main));
    HIP_OK(hipStreamWaitEvent(st, ctx->lanes[g].done, 0));
  }
  // every job's status word into one pinned array, read after the one
  // synchronisation below
  const int n = (int)jobs.size();
  if (n > ctx->status_cap) {
    if (ctx->status_dev) (void)hipFree(ctx->status_dev);
    if (ctx->status_pin) (void)hipHostFree(ctx->status_pin);
    ctx->status_dev = ctx->status_pin = nullptr;
    ctx->status_cap = 0;
    const int cap = (n + 255) / 256 * 256;
    HIP_OK(hipMalloc((void **)&ctx->status_dev, (size_t)cap * 4));
    HIP_OK(hipHostMalloc((void **)&ctx->status_pin, (size_t)cap * 4, hipHostMallocDefault));
    ctx->status_cap = cap;
  }
  {
    Table *t;
    TableLease lease;
    if ((s = get_table(ctx, jobs, st, &t, lease)) != NFHMM_OK) return s;
    HIP_OK(launch_status_gather(t->lists[kBegin], ctx->status_dev, st));
    HIP_OK(hipMemcpyAsync(ctx->status_pin, ctx->status_dev, (size_t)n * 4, hipMemcpyDeviceToHost, st));
  }
  // host outputs through the pinned ring, then the copy pool into the caller's
  // arrays; every region taken here is given back before returning
  nfhmm_status ds = NFHMM_OK;
  for (Job *j : jobs)
    if (j->host_out && ds == NFHMM_OK) ds = download_staged(ctx, *j, st);
  const hipError_t se = hipStreamSynchronize(st);
  for (Job *j : jobs) {
    if (se == hipSuccess && ds == NFHMM_OK) {
      deliver_staged(ctx, *j);
    } else if (j->out_pin != ~size_t(0)) {
      pin_release(ctx, j->out_pin);
      j->out_pin = ~size_t(0);
    }
  }
  pin_poll(ctx);   // the upload regions, whose copies are done
  if (ds != NFHMM_OK) return ds;
  HIP_OK(se);
  nfhmm_status first = NFHMM_OK;
  for (int i = 0; i < n; ++i) {
    Job *j = jobs[i];
    const int flag = ctx->status_pin[i];
    if (flag & (kBadV | kBadW)) {
      j->status = NFHMM_E_INVALID;
      j->error = (flag & kBadV) ? "V has a negative or non-finite entry" : "a dictionary element is not normalised";
    } else if (flag & kNonFinite) {
      j->status = NFHMM_E_NONFINITE;
      j->error = "the evidence lower bound became non-finite";
    }
    if (first == NFHMM_OK && j->status != NFHMM_OK) {
      first = j->status;
      g_err = j->error;
    }
  }
  return first;
}

nfhmm_status make_job(const nfhmm_problem *p, nfhmm_precision prec, const nfhmm_result *r, bool host_in,
                      bool host_out, Job &j) {
  std::string why;
  if (prec != NFHMM_FP32 && prec != NFHMM_BF16) return fail(NFHMM_E_INVALID, "unknown precision %d", (int)prec);
  if (!dims_ok(p, &why)) return fail(NFHMM_E_INVALID, "%s", why.c_str());
  if (!r) return fail(NFHMM_E_INVALID, "result is NULL");
  j.prob = *p;
  j.d = dims_of(p, prec);
  j.res = *r;
  j.host_in = host_in;
  j.host_out = host_out;
  if (host_out) {
    const void *outs[4] = {r->alpha, r->post, r->sep, r->elbo};
    for (int i = 0; i < 4; ++i) j.out_direct[i] = host_pinned(outs[i]);
  }
  j.L = plan(j.d, host_in, host_out, p->alpha_init != nullptr);
  return NFHMM_OK;
}

// ------------------------------------------------------------------ serving loop
void finish_job_locked(nfhmm_ctx *ctx, Job *j, nfhmm_status st, const std::string &err) {
  j->status = st;
  j->error = err;
  j->state = kDone;
  j->t_done = now_s();
  ctx->bytes_in_use -= j->charged;
  j->charged = 0;
}

void scheduler(nfhmm_ctx *ctx) {
  (void)hipSetDevice(ctx->device);
  // Rounds run on lane 0's streams.  The blocking engine's second lane is idle
  // here, so its two streams carry the host<->device copies: inputs go up on
  // one and outputs come down on the other, beside the rounds instead of
  // between them, ordered by events.
  hipStream_t st = ctx->stream, up = ctx->lanes[1].main, down = ctx->lanes[1].fb;
  hipEvent_t ev_up = nullptr;
  (void)hipEventCreateWithFlags(&ev_up, hipEventDisableTiming);
  struct Pending { Job *job; hipEvent_t ev; };
  std::vector<Pending> pending;        // off the device or cancelled; outputs / last work in flight
  std::deque<hipEvent_t> inflight;     // end markers of the rounds still on the device
  std::vector<hipEvent_t> spare;
  auto new_event = [&]() {
    hipEvent_t e = nullptr;
    if (!spare.empty()) { e = spare.back(); spare.pop_back(); }
    else (void)hipEventCreateWithFlags(&e, hipEventDisableTiming);
    return e;
  };
  for (;;) {
    std::vector<Job *> admitted, act;
    {
      std::unique_lock<std::mutex> lk(ctx->mu);
      ctx->cv.wait(lk, [&] { return ctx->stop || !ctx->queue.empty() || !ctx->resident.empty() || !pending.empty(); });
      if (ctx->stop && ctx->queue.empty() && ctx->resident.empty() && pending.empty()) break;
      // drop cancelled queued jobs
      for (auto it = ctx->queue.begin(); it != ctx->queue.end();) {
        if ((*it)->cancel) {
          finish_job_locked(ctx, *it, NFHMM_E_CANCELLED, "cancelled");
          it = ctx->queue.erase(it);
        } else ++it;
      }
      // admission: first in, first out, within budget and slots; then the
      // arenas, stopping (in order) at the first job the slab cannot place yet
      std::vector<size_t> fp;
      for (Job *j : ctx->queue) fp.push_back(j->L.total);
      std::vector<int> adm(fp.size(), 0);
      nfhmm_admission_plan((int)fp.size(), fp.data(), ctx->bytes_in_use, ctx->budget, (int)ctx->resident.size(),
                           ctx->max_slots, adm.data());
      for (size_t i = 0; i < adm.size(); ++i) {
        if (adm[i] != 1) break;
        Job *j = ctx->queue[i];
        nfhmm_status err;
        if (!serving_alloc(ctx, *j, &err)) {
          if (err == NFHMM_OK) break;            // no free range yet: wait for a job to leave
          finish_job_locked(ctx, j, err, g_err); // the device refused the memory
          ctx->cv_done.notify_all();
          continue;
        }
        admitted.push_back(j);
      }
      for (Job *j : admitted) {
        ctx->queue.erase(std::find(ctx->queue.begin(), ctx->queue.end(), j));
        j->charged = j->L.total;
        ctx->bytes_in_use += j->charged;
      }
      for (auto it = ctx->queue.begin(); it != ctx->queue.end();) {   // jobs failed above
        if ((*it)->state == kDone) it = ctx->queue.erase(it);
        else ++it;
      }
    }
    std::lock_guard<std::mutex> eng(ctx->engine_mu);
    // start the admitted jobs
    std::vector<Job *> started;
    pin_poll(ctx);
    for (Job *j : admitted) {
      j->start_round = ctx->round;
      fill_desc(*j, j->prob.gamma);
      nfhmm_status s = upload_staged(ctx, *j, up);
      std::lock_guard<std::mutex> lk(ctx->mu);
      if (s != NFHMM_OK) {   // finished (with this status) once the stream has passed it
        j->status = s;
        j->error = g_err;
        pending.push_back({j, nullptr});
      } else {
        j->state = kResident;
        started.push_back(j);
      }
    }
    if (!started.empty()) {
      (void)hipEventRecord(ev_up, up);
      (void)hipStreamWaitEvent(st, ev_up, 0);
    }
    nfhmm_status s = engine_begin(ctx, started, st);
    std::vector<Job *> zero_iter;
    {
      std::lock_guard<std::mutex> lk(ctx->mu);
      for (Job *j : started) {
        if (j->d.iters == 0) zero_iter.push_back(j);
        else ctx->resident.push_back(j);
      }
      // cancelled resident jobs leave now; their arenas are released once the
      // work already queued for them has finished
      std::vector<Job *> keep;
      for (Job *j : ctx->resident) {
        if (j->cancel) {
          j->status = NFHMM_E_CANCELLED;
          pending.push_back({j, nullptr});
        } else keep.push_back(j);
      }
      ctx->resident.swap(keep);
      act = ctx->resident;
    }
    const int r = ctx->round;
    std::vector<Job *> fin = zero_iter;
    if (s == NFHMM_OK) s = engine_iterate(ctx, act, r, st, ctx->fb_stream, ctx->ev_fork, ctx->ev_join);
    for (Job *j : act)
      if (r - j->start_round + 1 == j->d.iters) fin.push_back(j);
    if (s == NFHMM_OK) s = engine_finish(ctx, fin, st);
    // one marker for everything queued so far: the last work of finished and
    // cancelled jobs is complete once it has passed; their outputs follow on the
    // download stream
    hipEvent_t mark = new_event();
    (void)hipEventRecord(mark, st);
    for (Job *j : fin) pending.push_back({j, nullptr});
    bool fresh = false;
    for (auto &pd : pending) fresh |= !pd.ev;
    if (fresh) (void)hipStreamWaitEvent(down, mark, 0);
    for (Job *j : fin)
      if (s == NFHMM_OK) s = download_staged(ctx, *j, down);
    for (auto &pd : pending)
      if (!pd.ev) {
        pd.ev = new_event();
        (void)hipEventRecord(pd.ev, down);
      }
    inflight.push_back(mark);
    {
      std::lock_guard<std::mutex> lk(ctx->mu);
      std::vector<Job *> keep;
      for (Job *j : ctx->resident)
        if (std::find(fin.begin(), fin.end(), j) == fin.end()) keep.push_back(j);
      ctx->resident.swap(keep);
      ctx->round++;
      if (s != NFHMM_OK) ctx->sched_error = g_err;
    }
    // at most two rounds on the device; with nothing left to run, wait for all
    const bool idle = ctx->resident.empty();
    while (inflight.size() > 2 || (idle && !inflight.empty())) {
      (void)hipEventSynchronize(inflight.front());
      spare.push_back(inflight.front());
      inflight.pop_front();
    }
    if (idle)   // nothing to run: wait for the outputs still coming down
      for (auto &pd : pending) (void)hipEventSynchronize(pd.ev);
    // retire the jobs whose outputs have landed
    std::vector<Pending> still;
    for (auto &pd : pending) {
      if (hipEventQuery(pd.ev) != hipSuccess) { still.push_back(pd); continue; }
      spare.push_back(pd.ev);
      Job *j = pd.job;
      const bool staged = j->out_pin != ~size_t(0);
      deliver_staged(ctx, *j);
      int flag = j->dev_flag;
      if (!staged && j->status == NFHMM_OK) (void)hipMemcpy(&flag, j->desc.status, 4, hipMemcpyDeviceToHost);
      serving_free(ctx, *j);
      std::lock_guard<std::mutex> lk(ctx->mu);
      nfhmm_status js = j->status;
      std::string err = j->error;
      if (js == NFHMM_OK && s != NFHMM_OK) { js = s; err = ctx->sched_error; }
      else if (js == NFHMM_OK && (flag & (kBadV | kBadW))) { js = NFHMM_E_INVALID; err = "invalid input detected on the device"; }
      else if (js == NFHMM_OK && (flag & kNonFinite)) { js = NFHMM_E_NONFINITE; err = "the evidence lower bound became non-finite"; }
      else if (js == NFHMM_E_CANCELLED) err = "cancelled";
      finish_job_locked(ctx, j, js, err);
      ctx->cv_done.notify_all();
    }
    pending.swap(still);
  }
  (void)hipStreamSynchronize(st);
  (void)hipStreamSynchronize(up);
  (void)hipStreamSynchronize(down);
  (void)hipEventDestroy(ev_up);
  for (hipEvent_t e : inflight) (void)hipEventDestroy(e);
  for (hipEvent_t e : spare) (void)hipEventDestroy(e);
}

}  // namespace

// ================================================================== C ABI
extern "C" {

nfhmm_status nfhmm_create(nfhmm_ctx **out, int device, size_t hbm_budget_bytes, int max_slots) {
  if (!out) return fail(NFHMM_E_INVALID, "out is NULL");
  *out = nullptr;
  int n = 0;
  HIP_OK(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(NFHMM_E_DEVICE, "device %d not present (%d devices)", device, n);
  HIP_OK(hipSetDevice(device));
  HIP_OK(scratch_setup(device));
  std::unique_ptr<nfhmm_ctx> c(new nfhmm_ctx());
  HIP_OK(hipHostMalloc((void **)&c->status_host, 256, hipHostMallocDefault));
  c->device = device;
  c->budget = hbm_budget_bytes;
  c->max_slots = max_slots > 0 ? max_slots : 64;
  HIP_OK(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
  HIP_OK(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
  for (auto &ln : c->lanes) {
    HIP_OK(hipStreamCreateWithFlags(&ln.main, hipStreamNonBlocking));
    HIP_OK(hipStreamCreateWithFlags(&ln.fb, hipStreamNonBlocking));
    HIP_OK(hipEventCreateWithFlags(&ln.fork, hipEventDisableTiming));
    HIP_OK(hipEventCreateWithFlags(&ln.join, hipEventDisableTiming));
    HIP_OK(hipEventCreateWithFlags(&ln.done, hipEventDisableTiming));
  }
  c->stream = c->lanes[0].main;
  c->fb_stream = c->lanes[0].fb;
  *out = c.release();
  return NFHMM_OK;
}

void nfhmm_destroy(nfhmm_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (Job *j : ctx->queue) j->cancel = true;
    ctx->stop = true;
  }
  ctx->cv.notify_all();
  if (ctx->sched.joinable()) ctx->sched.join();
  (void)hipDeviceSynchronize();
  for (auto &kv : ctx->jobs)
    if (kv.second->arena && !kv.second->in_slab) (void)hipFree(kv.second->arena);
  if (ctx->slab) (void)hipFree(ctx->slab);
  for (auto &r : ctx->pin_regs)
    if (r.ev) (void)hipEventDestroy(r.ev);
  if (ctx->pin) (void)hipHostFree(ctx->pin);
  for (auto &kv : ctx->arena_cache)
    for (char *a : kv.second) (void)hipFree(a);
  for (auto &r : ctx->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
  for (auto &t : ctx->tables) {
    if (t.dev) (void)hipFree(t.dev);
    if (t.host) (void)hipHostFree(t.host);
  }
  if (ctx->status_host) (void)hipHostFree(ctx->status_host);
  if (ctx->status_dev) (void)hipFree(ctx->status_dev);
  if (ctx->status_pin) (void)hipHostFree(ctx->status_pin);
  (void)hipEventDestroy(ctx->ev_fork);
  (void)hipEventDestroy(ctx->ev_join);
  for (auto &ln : ctx->lanes) {
    (void)hipEventDestroy(ln.fork);
    (void)hipEventDestroy(ln.join);
    (void)hipEventDestroy(ln.done);
    (void)hipStreamDestroy(ln.main);
    (void)hipStreamDestroy(ln.fb);
  }
  delete ctx;
}

const char *nfhmm_last_error(const nfhmm_ctx *) { return g_err.c_str(); }

size_t nfhmm_footprint_bytes(const nfhmm_problem *p, nfhmm_precision prec) {
  if (!dims_ok(p, nullptr)) return 0;
  return plan(dims_of(p, prec), true, true, p->alpha_init != nullptr).total;
}

nfhmm_status nfhmm_validate(const nfhmm_problem *p, char *msg, size_t msglen) {
  std::string m;
  nfhmm_status s = validate_host(p, &m);
  if (msg && msglen) snprintf(msg, msglen, "%s", m.c_str());
  if (s != NFHMM_OK) g_err = m;
  return s;
}

int nfhmm_admission_plan(int n_queued, const size_t *footprints, size_t bytes_in_use, size_t budget, int resident,
                         int max_slots, int *admit) {
  int n = 0;
  bool blocked = false;
  size_t used = bytes_in_use;
  for (int i = 0; i < n_queued; ++i) {
    admit[i] = 0;
    if (budget && footprints[i] > budget) {
      admit[i] = -1;
      continue;
    }
    if (blocked) continue;
    const bool slot = resident + n < max_slots;
    const bool fits = !budget || used + footprints[i] <= budget;
    if (slot && fits) {
      admit[i] = 1;
      used += footprints[i];
      ++n;
    } else {
      blocked = true;
    }
  }
  return n;
}

nfhmm_status nfhmm_fit_batch(nfhmm_ctx *ctx, int n, const nfhmm_problem *ps, nfhmm_precision prec,
                             nfhmm_result *rs) {
  if (!ctx) return fail(NFHMM_E_INVALID, "ctx is NULL");
  if (n < 0 || (n > 0 && (!ps || !rs))) return fail(NFHMM_E_INVALID, "bad batch arguments");
  HIP_OK(hipSetDevice(ctx->device));
  std::vector<std::unique_ptr<Job>> owned;
  std::vector<Job *> jobs;
  for (int i = 0; i < n; ++i) {
    std::string m;
    if (validate_host(&ps[i], &m) != NFHMM_OK) return fail(NFHMM_E_INVALID, "job %d: %s", i, m.c_str());
    owned.emplace_back(new Job());
    Job &j = *owned.back();
    j.id = new_id(ctx);
    nfhmm_status s = make_job(&ps[i], prec, &rs[i], true, true, j);
    if (s != NFHMM_OK) return s;
    jobs.push_back(&j);
  }
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (!ctx->copies) ctx->copies.reset(new CopyPool(nfhmm_ctx::copy_workers()));
  }
  std::lock_guard<std::mutex> eng(ctx->engine_mu);
  nfhmm_status s = NFHMM_OK;
  for (Job *j : jobs)
    if ((s = arena_alloc(ctx, *j, true)) != NFHMM_OK) break;
  if (s == NFHMM_OK) s = run_blocking(ctx, jobs, ctx->stream);
  (void)hipStreamSynchronize(ctx->stream);
  for (Job *j : jobs) arena_release(ctx, *j, true);
  return s;
}

nfhmm_status nfhmm_fit(nfhmm_ctx *ctx, const nfhmm_problem *p, nfhmm_precision prec, nfhmm_result *r) {
  return nfhmm_fit_batch(ctx, 1, p, prec, r);
}

nfhmm_status nfhmm_fit_batch_device(nfhmm_ctx *ctx, int n, const nfhmm_problem *ps, nfhmm_precision prec,
                                    nfhmm_result *rs, void *hip_stream) {
  if (!ctx) return fail(NFHMM_E_INVALID, "ctx is NULL");
  if (n < 0 || (n > 0 && (!ps || !rs))) return fail(NFHMM_E_INVALID, "bad batch arguments");
  HIP_OK(hipSetDevice(ctx->device));
  hipStream_t st = hip_stream ? reinterpret_cast<hipStream_t>(hip_stream) : ctx->stream;
  std::vector<std::unique_ptr<Job>> owned;
  std::vector<Job *> jobs;
  for (int i = 0; i < n; ++i) {
    owned.emplace_back(new Job());
    Job &j = *owned.back();
    j.id = new_id(ctx);
    nfhmm_status s = make_job(&ps[i], prec, &rs[i], false, false, j);
    if (s != NFHMM_OK) return fail(s, "job %d: %s", i, g_err.c_str());
    jobs.push_back(&j);
  }
  std::lock_guard<std::mutex> eng(ctx->engine_mu);
  nfhmm_status s = NFHMM_OK;
  for (Job *j : jobs)
    if ((s = arena_alloc(ctx, *j, true)) != NFHMM_OK) break;
  if (s == NFHMM_OK) s = run_blocking(ctx, jobs, st);
  (void)hipStreamSynchronize(st);
  for (Job *j : jobs) arena_release(ctx, *j, true);
  return s;
}

nfhmm_status nfhmm_fit_device(nfhmm_ctx *ctx, const nfhmm_problem *dev_p, nfhmm_precision prec,
                              nfhmm_result *dev_r, void *hip_stream) {
  return nfhmm_fit_batch_device(ctx, 1, dev_p, prec, dev_r, hip_stream);
}

nfhmm_status nfhmm_fit_device_noalloc(nfhmm_ctx *ctx, const nfhmm_problem *dev_p, nfhmm_precision prec,
                                      nfhmm_result *dev_r, void *hip_stream) {
  if (!ctx) return fail(NFHMM_E_INVALID, "ctx is NULL");
  Job j;
  nfhmm_status s = make_job(dev_p, prec, dev_r, false, false, j);
  if (s != NFHMM_OK) return s;
  // scratch: the table image, then the job's arena
  const size_t arena_off = (size_t)rup((int64_t)sizeof(OneJobTable), 256);
  const size_t need = arena_off + j.L.total;
  if (need > kNoAllocScratchBytes)
    return fail(NFHMM_E_NOMEM, "the job needs %zu bytes of working memory; nfhmm_fit_device_noalloc has %zu",
                need, kNoAllocScratchBytes);
  HIP_OK(hipSetDevice(ctx->device));
  char *base = scratch_of(ctx->device);
  if (!base) return fail(NFHMM_E_DEVICE, "no scratch address for device %d", ctx->device);
  hipStream_t st = hip_stream ? reinterpret_cast<hipStream_t>(hip_stream) : ctx->stream;
  std::lock_guard<std::mutex> eng(ctx->engine_mu);
  j.arena = base + arena_off;
  j.start_round = 0;
  fill_desc(j, j.prob.gamma);
  const JobDesc &D = j.desc;
  // the work lists of this one job, as the batched engine would build them
  OneJobTable img;
  static_assert(kNumLists <= kOneJobLists, "table image too small");
  std::memset(&img, 0, sizeof img);
  img.desc = D;
  const int stride = update_stride(std::max(32, j.d.Mp), std::max(1, j.d.S * j.d.N));
  const bool small = spec_blocks(D, false) < kSmallBatchBlocks;
  WorkList wl[kNumLists];
  for (int k = 0; k < kNumLists; ++k) {
    img.start[k][0] = 0;
    img.start[k][1] = blocks_of((ListKind)k, D, j.d.bf16, update_waves(stride), small);
    wl[k].jobs = reinterpret_cast<const JobDesc *>(base);
    wl[k].start = reinterpret_cast<const int *>(base + offsetof(OneJobTable, start)) + 2 * k;
    wl[k].njobs = 1;
    wl[k].total = img.start[k][1];
  }
  const int nmax = std::max(1, j.d.N);
  HIP_OK(launch_put_table(img, base, st));   // also clears the status word
  HIP_OK(launch_begin(wl[kBegin], wl[kTrans], st));
  if (D.alpha_init) {
    HIP_OK(launch_update(wl[kUpd], kUpdFromAlpha, 0, stride, st));
  } else {
    HIP_OK(launch_start_ratio(wl[kLam], wl[kRatio], st));
    HIP_OK(launch_counts(wl[kCntF], false, st));
    HIP_OK(launch_counts(wl[kCntH], true, st));
    HIP_OK(launch_update(wl[kUpd], kUpdUniform, 0, stride, st));
  }
  // each iteration on the one stream: the chains, then the contractions, then Eq. 6
  for (int r = 0; r < j.d.iters; ++r) {
    HIP_OK(launch_chain_fb(wl[kFBR], wl[kFB], nmax, st));
    HIP_OK(launch_posterior(wl[kPost], wl[kChain], nmax, st));
    HIP_OK(launch_spectrum(wl[kSpecF], false, true, st));
    HIP_OK(launch_spectrum(wl[kSpecH], true, small, st));
    HIP_OK(launch_counts(wl[kCntF], false, st));
    HIP_OK(launch_counts(wl[kCntH], true, st));
    HIP_OK(launch_update(wl[kUpd], kUpdMessages, r, stride, st));
  }
  HIP_OK(launch_finish(wl[kFrames], wl[kRecon], wl[kIters], st));
  HIP_OK(hipMemcpyAsync(ctx->status_host, D.status, 4, hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  const int flag = *ctx->status_host;
  if (flag & kBadV) return fail(NFHMM_E_INVALID, "V has a negative or non-finite entry");
  if (flag & kBadW) return fail(NFHMM_E_INVALID, "a dictionary element is not normalised");
  if (flag & kNonFinite) return fail(NFHMM_E_NONFINITE, "the evidence lower bound became non-finite");
  return NFHMM_OK;
}

nfhmm_status nfhmm_submit(nfhmm_ctx *ctx, const nfhmm_problem *p, nfhmm_precision prec, nfhmm_result *r,
                          uint64_t *job_id) {
  if (!ctx || !job_id) return fail(NFHMM_E_INVALID, "ctx or job_id is NULL");
  std::string m;
  if (validate_host(p, &m, false) != NFHMM_OK) return fail(NFHMM_E_INVALID, "%s", m.c_str());
  std::unique_ptr<Job> j(new Job());
  nfhmm_status s = make_job(p, prec, r, true, true, *j);
  if (s != NFHMM_OK) return s;
  const Dims &d = j->d;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (!ctx->copies) ctx->copies.reset(new CopyPool(nfhmm_ctx::copy_workers()));
  }
  // the caller may reuse its arrays once submit returns: take copies
  const size_t nV = (size_t)d.T * d.F, nW = (size_t)d.M * d.F, nA = (size_t)d.S * d.N * d.N,
               npi = (size_t)d.S * d.N, ni = p->alpha_init ? (size_t)d.T * d.M : 0;
  j->hV.reset(new float[nV]);
  j->hW.reset(new float[nW]);
  j->hA.reset(new float[nA]);
  j->hpi.reset(new float[npi]);
  if (ni) j->hinit.reset(new float[ni]);
  const CopyPool::Piece pc[5] = {{j->hV.get(), p->V, nV * 4, true}, {j->hW.get(), p->W, nW * 4},
                                 {j->hA.get(), p->A, nA * 4}, {j->hpi.get(), p->pi, npi * 4},
                                 {j->hinit.get(), p->alpha_init, ni * 4}};
  if (!ctx->copies->run(pc, 5)) {   // V failed the check made while copying it: name the entry
    validate_host(p, &m);
    return fail(NFHMM_E_INVALID, "%s", m.c_str());
  }
  // a valid job that can never fit the budget (checked after the inputs, so
  // that an invalid input is reported as such whatever its size)
  if (ctx->budget && j->L.total > ctx->budget)
    return fail(NFHMM_E_NOMEM, "job needs %zu device bytes, budget is %zu", j->L.total, ctx->budget);
  j->prob.V = j->hV.get();
  j->prob.W = j->hW.get();
  j->prob.A = j->hA.get();
  j->prob.pi = j->hpi.get();
  j->prob.alpha_init = ni ? j->hinit.get() : nullptr;
  j->t_submit = now_s();
  j->id = new_id(ctx);
  std::lock_guard<std::mutex> lk(ctx->mu);
  *job_id = j->id;
  ctx->queue.push_back(j.get());
  ctx->jobs[j->id] = std::move(j);
  if (!ctx->sched.joinable()) ctx->sched = std::thread(scheduler, ctx);
  ctx->cv.notify_all();
  return NFHMM_OK;
}

nfhmm_status nfhmm_poll(nfhmm_ctx *ctx, uint64_t job_id, int *done) {
  if (!ctx || !done) return fail(NFHMM_E_INVALID, "ctx or done is NULL");
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto it = ctx->jobs.find(job_id);
  if (it == ctx->jobs.end()) return fail(NFHMM_E_NOTFOUND, "unknown job %llu", (unsigned long long)job_id);
  *done = it->second->state == kDone;
  return NFHMM_OK;
}

nfhmm_status nfhmm_wait(nfhmm_ctx *ctx, uint64_t job_id, double *latency_s) {
  if (!ctx) return fail(NFHMM_E_INVALID, "ctx is NULL");
  std::unique_lock<std::mutex> lk(ctx->mu);
  auto it = ctx->jobs.find(job_id);
  if (it == ctx->jobs.end()) return fail(NFHMM_E_NOTFOUND, "unknown job %llu", (unsigned long long)job_id);
  Job *j = it->second.get();
  ctx->cv_done.wait(lk, [&] { return j->state == kDone; });
  if (latency_s) *latency_s = j->t_done - j->t_submit;
  const nfhmm_status st = j->status;
  const std::string err = j->error;
  ctx->jobs.erase(it);
  if (st != NFHMM_OK) return fail(st, "%s", err.c_str());
  return NFHMM_OK;
}

nfhmm_status nfhmm_cancel(nfhmm_ctx *ctx, uint64_t job_id) {
  if (!ctx) return fail(NFHMM_E_INVALID, "ctx is NULL");
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto it = ctx->jobs.find(job_id);
  if (it == ctx->jobs.end()) return fail(NFHMM_E_NOTFOUND, "unknown job %llu", (unsigned long long)job_id);
  it->second->cancel = true;
  ctx->cv.notify_all();
  return NFHMM_OK;
}

nfhmm_status nfhmm_profile_enable(nfhmm_ctx *ctx, int enable) {
  if (!ctx) return fail(NFHMM_E_INVALID, "ctx is NULL");
  HIP_OK(hipSetDevice(ctx->device));
  HIP_OK(hipDeviceSynchronize());
  for (auto &r : ctx->recs) {
    ctx->event_pool.push_back(r.a);
    ctx->event_pool.push_back(r.b);
  }
  ctx->recs.clear();
  ctx->profiling = enable != 0;
  return NFHMM_OK;
}

nfhmm_status nfhmm_set_lanes(nfhmm_ctx *ctx, int lanes) {
  if (!ctx || lanes < 1 || lanes > nfhmm_ctx::kMaxGroups) return fail(NFHMM_E_INVALID, "lanes must be 1 or 2");
  ctx->groups = lanes;
  return NFHMM_OK;
}

nfhmm_status nfhmm_profile_select(nfhmm_ctx *ctx, unsigned mask) {
  if (!ctx) return fail(NFHMM_E_INVALID, "ctx is NULL");
  ctx->profile_mask = mask;
  return NFHMM_OK;
}

nfhmm_status nfhmm_profile_read(nfhmm_ctx *ctx, int kind, int64_t *launches, double *total_ms) {
  if (!ctx || kind < 0 || kind >= NFHMM_K_COUNT) return fail(NFHMM_E_INVALID, "bad arguments");
  HIP_OK(hipSetDevice(ctx->device));
  int64_t n = 0;
  double ms = 0.0;
  for (auto &r : ctx->recs) {
    if (r.kind != kind) continue;
    HIP_OK(hipEventSynchronize(r.b));
    float e = 0.0f;
    HIP_OK(hipEventElapsedTime(&e, r.a, r.b));
    ms += e;
    ++n;
  }
  if (launches) *launches = n;
  if (total_ms) *total_ms = ms;
  return NFHMM_OK;
}

// ------------------------------------------------------------------ time domain
namespace {
constexpr int64_t kMaxFrames = int64_t(1) << 30;   // frame indices and run ends stay in int
bool stft_sizes_ok(int32_t nfft, int32_t hop, int32_t B) {
  return nfft >= 64 && nfft <= 4096 && (nfft & (nfft - 1)) == 0 && hop >= 1 && hop <= nfft && B >= 1 &&
         B <= 65535;
}
}  // namespace

int64_t nfhmm_stft_frames(int32_t nfft, int32_t hop, int64_t n) {
  if (nfft <= 0 || hop <= 0 || n < nfft) return 0;
  return 1 + (n - nfft) / hop;
}

nfhmm_status nfhmm_stft_device(nfhmm_ctx *ctx, int32_t nfft, int32_t hop, int32_t B, const float *x, int64_t n,
                               float *mag, float *phase, void *hip_stream) {
  if (!ctx || !x || !mag || !phase) return fail(NFHMM_E_INVALID, "NULL argument");
  if (!stft_sizes_ok(nfft, hop, B)) return fail(NFHMM_E_INVALID, "bad nfft, hop or B");
  const int64_t T = nfhmm_stft_frames(nfft, hop, n);
  if (T < 1 || T > kMaxFrames) return fail(NFHMM_E_INVALID, "the signal has no whole frame (n < nfft) or too many");
  HIP_OK(hipSetDevice(ctx->device));
  hipStream_t st = hip_stream ? reinterpret_cast<hipStream_t>(hip_stream) : ctx->stream;
  HIP_OK(launch_stft(nfft, x, n, hop, (int)T, B, mag, phase, st));
  return NFHMM_OK;
}

nfhmm_status nfhmm_istft_device(nfhmm_ctx *ctx, int32_t nfft, int32_t hop, int32_t B, int32_t S, const float *mag,
                                const float *phase, int64_t T, float *y, int64_t n, void *hip_stream) {
  if (!ctx || !mag || !phase || !y) return fail(NFHMM_E_INVALID, "NULL argument");
  if (!stft_sizes_ok(nfft, hop, B) || S < 1 || (int64_t)B * S > 65535)
    return fail(NFHMM_E_INVALID, "bad nfft, hop, B or S");
  if (T < 1 || T > kMaxFrames || n < 1) return fail(NFHMM_E_INVALID, "bad T or n");
  HIP_OK(hipSetDevice(ctx->device));
  hipStream_t st = hip_stream ? reinterpret_cast<hipStream_t>(hip_stream) : ctx->stream;
  HIP_OK(launch_istft(nfft, mag, phase, (int)T, B, S, hop, n, y, st));
  return NFHMM_OK;
}

nfhmm_status nfhmm_stft(nfhmm_ctx *ctx, int32_t nfft, int32_t hop, int32_t B, const float *x, int64_t n,
                        float *mag, float *phase) {
  if (!ctx || !x || !mag || !phase) return fail(NFHMM_E_INVALID, "NULL argument");
  if (!stft_sizes_ok(nfft, hop, B)) return fail(NFHMM_E_INVALID, "bad nfft, hop or B");
  const int64_t T = nfhmm_stft_frames(nfft, hop, n);
  if (T < 1 || T > kMaxFrames) return fail(NFHMM_E_INVALID, "the signal has no whole frame (n < nfft) or too many");
  HIP_OK(hipSetDevice(ctx->device));
  std::lock_guard<std::mutex> eng(ctx->engine_mu);
  hipStream_t st = ctx->stream;
  const size_t bx = (size_t)B * n * 4, bo = (size_t)B * T * (nfft / 2 + 1) * 4;
  char *d = nullptr;
  HIP_OK(hipMallocAsync((void **)&d, bx + 2 * bo, st));
  float *dx = reinterpret_cast<float *>(d), *dm = reinterpret_cast<float *>(d + bx),
        *dp = reinterpret_cast<float *>(d + bx + bo);
  hipError_t e = hipMemcpyAsync(dx, x, bx, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = launch_stft(nfft, dx, n, hop, (int)T, B, dm, dp, st);
  if (e == hipSuccess) e = hipMemcpyAsync(mag, dm, bo, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(phase, dp, bo, hipMemcpyDeviceToHost, st);
  (void)hipFreeAsync(d, st);
  const hipError_t es = hipStreamSynchronize(st);
  HIP_OK(e);
  HIP_OK(es);
  return NFHMM_OK;
}

nfhmm_status nfhmm_istft(nfhmm_ctx *ctx, int32_t nfft, int32_t hop, int32_t B, int32_t S, const float *mag,
                         const float *phase, int64_t T, float *y, int64_t n) {
  if (!ctx || !mag || !phase || !y) return fail(NFHMM_E_INVALID, "NULL argument");
  if (!stft_sizes_ok(nfft, hop, B) || S < 1 || (int64_t)B * S > 65535)
    return fail(NFHMM_E_INVALID, "bad nfft, hop, B or S");
  if (T < 1 || T > kMaxFrames || n < 1) return fail(NFHMM_E_INVALID, "bad T or n");
  HIP_OK(hipSetDevice(ctx->device));
  std::lock_guard<std::mutex> eng(ctx->engine_mu);
  hipStream_t st = ctx->stream;
  const size_t F = nfft / 2 + 1, bm = (size_t)B * S * T * F * 4, bp = (size_t)B * T * F * 4,
               by = (size_t)B * S * n * 4;
  char *d = nullptr;
  HIP_OK(hipMallocAsync((void **)&d, bm + bp + by, st));
  float *dm = reinterpret_cast<float *>(d), *dp = reinterpret_cast<float *>(d + bm),
        *dy = reinterpret_cast<float *>(d + bm + bp);
  hipError_t e = hipMemcpyAsync(dm, mag, bm, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(dp, phase, bp, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = launch_istft(nfft, dm, dp, (int)T, B, S, hop, n, dy, st);
  if (e == hipSuccess) e = hipMemcpyAsync(y, dy, by, hipMemcpyDeviceToHost, st);
  (void)hipFreeAsync(d, st);
  const hipError_t es = hipStreamSynchronize(st);
  HIP_OK(e);
  HIP_OK(es);
  return NFHMM_OK;
}

// ------------------------------------------------------------------ EM learning of a source model
}  // extern "C"

namespace {

nfhmm_status em_check(const nfhmm_nhmm_problem *p, const nfhmm_nhmm_result *r, bool values, std::string *msg) {
  auto bad = [&](const char *m) { *msg = m; return NFHMM_E_INVALID; };
  if (!p || !r) return bad("problem or result is NULL");
  if (p->N < 1 || p->N > NFHMM_MAX_STATES) return bad("N out of range [1, 64]");
  if (p->K < 1 || p->K > kEmMaxK) return bad("K out of range [1, 32]");
  if (p->F < 1 || p->F > (1 << 20) || p->T < 1 || p->T > (1 << 22)) return bad("F or T out of range");
  if (p->iters < 1 || p->iters > (1 << 20)) return bad("iters out of range [1, 2^20]");
  if ((int64_t)p->T * p->N * std::max<int64_t>(p->K, 64) >= (int64_t)1 << 31 ||
      (int64_t)p->N * p->K * p->F * ((p->T + kEmChunk - 1) / kEmChunk) >= (int64_t)1 << 31)
    return bad("T * N * K or the M-step's partial sums too large");
  if (!p->V || !p->W || !p->theta || !p->A || !p->pi) return bad("V, W, theta, A and pi are required");
  if (!values) return NFHMM_OK;
  const int64_t N = p->N, K = p->K, F = p->F, T = p->T;
  char buf[256];
  if (!all_finite_nonneg(p->V, T * F)) return bad("V has a negative or non-finite entry");
  std::vector<unsigned char> counted(F, 0);
  for (int64_t i = 0; i < T * F; ++i) counted[i % F] |= (unsigned char)(p->V[i] > 0.0f);
  for (int64_t d = 0; d < N; ++d) {
    std::vector<unsigned char> cover(F, 0);
    for (int64_t z = 0; z < K; ++z) {
      const float *row = p->W + (d * K + z) * F;
      double sum = 0.0;
      for (int64_t f = 0; f < F; ++f) {
        if (bad_value(row[f])) return bad("W has a negative or non-finite entry");
        sum += row[f];
        cover[f] |= (unsigned char)(row[f] > 0.0f);
      }
      if (std::fabs(sum - 1.0) > 1e-4) {
        snprintf(buf, sizeof buf, "dictionary row (%lld, %lld) sums to %.7g, not 1", (long long)d, (long long)z, sum);
        *msg = buf;
        return NFHMM_E_INVALID;
      }
    }
    for (int64_t f = 0; f < F; ++f)
      if (counted[f] && !cover[f]) {
        snprintf(buf, sizeof buf, "state %lld's dictionary is 0 in bin %lld, which has counts", (long long)d,
                 (long long)f);
        *msg = buf;
        return NFHMM_E_INVALID;
      }
  }
  for (int64_t i = 0; i < T * N; ++i) {
    double sum = 0.0;
    for (int64_t z = 0; z < K; ++z) {
      const float x = p->theta[i * K + z];
      if (!(x > 0.0f) || !std::isfinite(x)) return bad("theta has an entry that is not finite and > 0");
      sum += x;
    }
    if (std::fabs(sum - 1.0) > 1e-4) return bad("a row of theta does not sum to 1");
  }
  double ps = 0.0;
  for (int64_t i = 0; i < N; ++i) {
    if (bad_value(p->pi[i])) return bad("pi has a negative or non-finite entry");
    ps += p->pi[i];
    double rs = 0.0;
    for (int64_t j = 0; j < N; ++j) {
      if (bad_value(p->A[i * N + j])) return bad("A has a negative or non-finite entry");
      rs += p->A[i * N + j];
    }
    if (std::fabs(rs - 1.0) > 1e-4) return bad("a row of A does not sum to 1");
  }
  if (std::fabs(ps - 1.0) > 1e-4) return bad("pi does not sum to 1");
  return NFHMM_OK;
}

// Where one EM problem's arrays sit in its arena.
struct EmLayout {
  size_t V, W32, th32, A32, pi32, b[2], th[2], lA[2], lpi[2], ll, off, x, la, lgam, gmax, lbn, sI, xpart, gpart,
      bpart, trace, tm, tz, ts, total;
  int nsw;
};

// The forward-backward runs time-parallel (in chunks of kEmSweepChunk frames) for
// chains of at least four chunks, when the whole batch's chains are too few to
// fill the GPU: it costs N times the sequential sweep's work, spread over N times
// as many wavefronts.  Past about 2^19 state-frames the sequential sweeps of the
// batch's problems, side by side, take less time.  The choice depends on the
// batch (a problem's results then agree with learning it alone to rounding, not
// bit for bit, when a batch crosses that line and the problem alone does not).
constexpr int64_t kEmSweepWork = (int64_t)1 << 19;
int em_sweep_chunks(const nfhmm_nhmm_problem &p, int64_t batch_work) {
  const int c = (p.T - 1 + kEmSweepChunk - 1) / kEmSweepChunk;
  return (batch_work <= kEmSweepWork && c >= 4) ? c : 0;
}
int64_t em_batch_work(const nfhmm_nhmm_problem *ps, int n) {
  int64_t w = 0;
  for (int i = 0; i < n; ++i) w += (int64_t)ps[i].N * ps[i].T;
  return w;
}

EmLayout em_layout(const nfhmm_nhmm_problem &p, bool host, int nsw) {
  const size_t N = p.N, K = p.K, F = p.F, T = p.T, it = p.iters;
  const size_t nchunk = (T + kEmChunk - 1) / kEmChunk;
  EmLayout L{};
  size_t off = 0;
  auto take = [&](size_t b) { size_t o = off; off += (b + 255) / 256 * 256; return o; };
  // the caller's float32 arrays (host: copies in the arena), then the working ones
  L.V = host ? take(T * F * 4) : ~size_t(0);
  L.W32 = take(N * K * F * 4); L.th32 = take(T * N * K * 4); L.A32 = take(N * N * 4); L.pi32 = take(N * 4);
  for (int i = 0; i < 2; ++i) {
    L.b[i] = take(N * K * F * 8);
    L.th[i] = take(T * N * K * 8);
    L.lA[i] = take(N * N * 4);
    L.lpi[i] = take(N * 4);
  }
  L.ll = take(T * N * 8); L.off = take(T * 8); L.x = take(T * 64 * 4); L.la = take(T * 64 * 4);
  L.lgam = take(T * N * 4); L.gmax = take(N * 4);
  L.lbn = take(T * 64 * 4); L.sI = take(T * 64 * 4);
  L.xpart = take(nchunk * N * 64 * 8); L.gpart = take(nchunk * N * 4);
  L.bpart = take(nchunk * N * K * F * 8); L.trace = take(it * 8);
  const size_t C = (size_t)nsw;
  L.nsw = nsw;
  L.tm = take(2 * C * N * 64 * 4); L.tz = take(2 * C * 64 * 8); L.ts = take(2 * C * 64 * 4);
  L.total = off;
  return L;
}

// The grids of a batch span the largest sizes in it; their product must fit.
bool em_batch_fits(const nfhmm_nhmm_problem *ps, int n) {
  int64_t N = 0, F = 0, T = 0, C = 0;
  for (int i = 0; i < n; ++i) {
    N = std::max<int64_t>(N, ps[i].N); F = std::max<int64_t>(F, ps[i].F); T = std::max<int64_t>(T, ps[i].T);
    C = std::max<int64_t>(C, (ps[i].T + kEmChunk - 1) / kEmChunk);
  }
  return T * N < ((int64_t)1 << 31) && (F + 63) / 64 * N * C < ((int64_t)1 << 31);
}

// EM of n independent problems in one run: host or device arrays in and out, the
// work on st.  Each problem has its own arena; every iteration's kernels cover all
// problems still iterating in the same launches.
nfhmm_status em_run(nfhmm_ctx *ctx, int n, const nfhmm_nhmm_problem *ps, nfhmm_nhmm_result *rs, bool host,
                    hipStream_t st) {
  std::vector<EmLayout> lay(n);
  std::vector<Job> jobs(n);   // only their arenas are used: allocated and cached like a fit's
  nfhmm_status s = NFHMM_OK;
  int done = 0;
  const int64_t work = em_batch_work(ps, n);
  for (; done < n && s == NFHMM_OK; ++done) {
    lay[done] = em_layout(ps[done], host, em_sweep_chunks(ps[done], work));
    jobs[done].L.total = lay[done].total;
    s = arena_alloc(ctx, jobs[done], true);
  }
  if (s != NFHMM_OK) {
    for (int i = 0; i + 1 < done; ++i) arena_release(ctx, jobs[i], true);
    return s;
  }
  hipError_t e = hipSuccess;
  auto cp = [&](void *dst, const void *src, size_t b, hipMemcpyKind k) {
    if (e == hipSuccess) e = hipMemcpyAsync(dst, src, b, k, st);
  };
  const hipMemcpyKind in = host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  // descriptors of both parities: iteration i reads parity i & 1 and writes the other
  std::vector<EmDesc> hd(2 * (size_t)n);
  EmBatch B{};
  B.n = n;
  int max_it = 0;
  for (int i = 0; i < n; ++i) {
    const nfhmm_nhmm_problem &p = ps[i];
    const EmLayout &L = lay[i];
    char *a = jobs[i].arena;
    auto F32 = [&](size_t o) { return reinterpret_cast<float *>(a + o); };
    auto F64 = [&](size_t o) { return reinterpret_cast<double *>(a + o); };
    const size_t N = p.N, K = p.K, F = p.F, T = p.T;
    if (host) cp(F32(L.V), p.V, T * F * 4, in);
    cp(F32(L.W32), p.W, N * K * F * 4, in);
    cp(F32(L.th32), p.theta, T * N * K * 4, in);
    cp(F32(L.A32), p.A, N * N * 4, in);
    cp(F32(L.pi32), p.pi, N * 4, in);
    if (e == hipSuccess)
      e = launch_em_import((int)N, (int)K, (int)F, (int)T, F32(L.W32), F32(L.th32), F32(L.A32), F32(L.pi32),
                           F64(L.b[0]), F64(L.th[0]), F32(L.lA[0]), F32(L.lpi[0]), st);
    for (int c = 0; c < 2; ++c) {
      const int nx = c ^ 1;
      EmDesc &E = hd[(size_t)c * n + i];
      E.N = (int)N; E.K = (int)K; E.F = (int)F; E.T = (int)T; E.nchunk = (int)((T + kEmChunk - 1) / kEmChunk);
      E.iters = p.iters;
      E.V = host ? F32(L.V) : p.V;
      E.beta = F64(L.b[c]); E.theta = F64(L.th[c]); E.lnA = F32(L.lA[c]); E.lnpi = F32(L.lpi[c]);
      E.beta_new = F64(L.b[nx]); E.theta_new = F64(L.th[nx]); E.lnA_new = F32(L.lA[nx]); E.lnpi_new = F32(L.lpi[nx]);
      E.ll = F64(L.ll); E.off = F64(L.off); E.x = F32(L.x); E.la = F32(L.la);
      E.lgam = F32(L.lgam); E.gmax = F32(L.gmax);
      E.lbn = F32(L.lbn); E.sI = F32(L.sI);
      E.xpart = reinterpret_cast<float2 *>(a + L.xpart); E.gpart = F32(L.gpart);
      E.bpart = F64(L.bpart); E.trace = F64(L.trace);
      E.nsw = L.nsw; E.tm = F32(L.tm); E.tz = F64(L.tz); E.ts = F32(L.ts);
    }
    B.maxN = std::max(B.maxN, (int)N); B.maxK = std::max(B.maxK, (int)K); B.maxF = std::max(B.maxF, (int)F);
    B.maxT = std::max(B.maxT, (int)T); B.maxChunk = std::max(B.maxChunk, hd[i].nchunk);
    B.maxSw = std::max(B.maxSw, L.nsw); B.anySeq = B.anySeq || L.nsw == 0;
    max_it = std::max(max_it, p.iters);
  }
  EmDesc *dd = nullptr;
  if (e == hipSuccess) e = hipMallocAsync((void **)&dd, hd.size() * sizeof(EmDesc), st);
  cp(dd, hd.data(), hd.size() * sizeof(EmDesc), hipMemcpyHostToDevice);
  for (int it = 0; it < max_it && e == hipSuccess; ++it) {
    B.d = dd + (size_t)(it & 1) * n;
    e = launch_em_frames(B, it, st);
    if (e == hipSuccess) e = launch_em_chain(B, it, st);
    if (e == hipSuccess) e = launch_em_beta(B, it, st);
  }
  // each problem's learned parameters, as float32, into its staging arrays, then out
  const hipMemcpyKind out = host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  for (int i = 0; i < n; ++i) {
    const nfhmm_nhmm_problem &p = ps[i];
    const nfhmm_nhmm_result &r = rs[i];
    const EmLayout &L = lay[i];
    char *a = jobs[i].arena;
    auto F32 = [&](size_t o) { return reinterpret_cast<float *>(a + o); };
    auto F64 = [&](size_t o) { return reinterpret_cast<double *>(a + o); };
    const size_t N = p.N, K = p.K, F = p.F, T = p.T;
    const int fin = p.iters & 1;
    if (e == hipSuccess)
      e = launch_em_export((int)N, (int)K, (int)F, (int)T, F64(L.b[fin]), F64(L.th[fin]), F32(L.lA[fin]),
                           F32(L.lpi[fin]), F32(L.W32), F32(L.th32), F32(L.A32), F32(L.pi32), st);
    if (r.W) cp(r.W, F32(L.W32), N * K * F * 4, out);
    if (r.theta) cp(r.theta, F32(L.th32), T * N * K * 4, out);
    if (r.A) cp(r.A, F32(L.A32), N * N * 4, out);
    if (r.pi) cp(r.pi, F32(L.pi32), N * 4, out);
    if (r.loglik) cp(r.loglik, a + L.trace, (size_t)p.iters * 8, out);
  }
  if (dd) (void)hipFreeAsync(dd, st);
  const hipError_t es = hipStreamSynchronize(st);
  for (int i = 0; i < n; ++i) arena_release(ctx, jobs[i], true);
  HIP_OK(e);
  HIP_OK(es);
  return NFHMM_OK;
}

}  // namespace

extern "C" {

nfhmm_status nfhmm_learn_nhmm(nfhmm_ctx *ctx, const nfhmm_nhmm_problem *p, nfhmm_nhmm_result *r) {
  return nfhmm_learn_nhmm_batch(ctx, 1, p, r);
}

nfhmm_status nfhmm_learn_nhmm_batch(nfhmm_ctx *ctx, int n, const nfhmm_nhmm_problem *ps, nfhmm_nhmm_result *rs) {
  if (!ctx) return fail(NFHMM_E_INVALID, "ctx is NULL");
  if (n < 1 || n > kEmMaxBatch || !ps || !rs) return fail(NFHMM_E_INVALID, "bad batch arguments");
  std::string m;
  for (int i = 0; i < n; ++i)
    if (em_check(&ps[i], &rs[i], true, &m) != NFHMM_OK) {
      if (n == 1) return fail(NFHMM_E_INVALID, "%s", m.c_str());
      return fail(NFHMM_E_INVALID, "problem %d: %s", i, m.c_str());
    }
  if (!em_batch_fits(ps, n)) return fail(NFHMM_E_INVALID, "the batch's largest sizes together are too large: split it");
  HIP_OK(hipSetDevice(ctx->device));
  std::lock_guard<std::mutex> eng(ctx->engine_mu);
  return em_run(ctx, n, ps, rs, true, ctx->stream);
}

nfhmm_status nfhmm_learn_nhmm_device(nfhmm_ctx *ctx, const nfhmm_nhmm_problem *dev_p, nfhmm_nhmm_result *dev_r,
                                     void *hip_stream) {
  if (!ctx) return fail(NFHMM_E_INVALID, "ctx is NULL");
  std::string m;
  if (em_check(dev_p, dev_r, false, &m) != NFHMM_OK) return fail(NFHMM_E_INVALID, "%s", m.c_str());
  HIP_OK(hipSetDevice(ctx->device));
  std::lock_guard<std::mutex> eng(ctx->engine_mu);
  return em_run(ctx, 1, dev_p, dev_r, false, hip_stream ? reinterpret_cast<hipStream_t>(hip_stream) : ctx->stream);
}

nfhmm_status nfhmm_chain_posterior(nfhmm_ctx *ctx, int N, int64_t T, const float *logev, const float *A,
                                   const float *pi, float *post, double *lnZ) {
  if (!ctx || !logev || !A || !pi) return fail(NFHMM_E_INVALID, "NULL argument");
  if (N < 1 || N > NFHMM_MAX_STATES || T < 1 || T > (1 << 24)) return fail(NFHMM_E_INVALID, "bad N or T");
  HIP_OK(hipSetDevice(ctx->device));
  std::lock_guard<std::mutex> eng(ctx->engine_mu);
  hipStream_t st = ctx->stream;
  const size_t T_ = (size_t)T;
  // layout: logev, A, pi, phi, ev, sh, fwd, bwd, nrm, post
  size_t off = 0;
  auto take = [&](size_t b) { size_t o = off; off += (b + 255) / 256 * 256; return o; };
  const size_t o_lev = take(T_ * N * 4), o_A = take((size_t)N * N * 4), o_pi = take((size_t)N * 4);
  const size_t o_phi = take(T_ * 64 * 4), o_ev = take(T_ * 64 * 4), o_sh = take(T_ * 4);
  const size_t o_f = take(T_ * 64 * 4), o_b = take(T_ * 64 * 4), o_n = take(T_ * 4), o_p = take(T_ * N * 4);
  const size_t o_flag = take(4);
  int fbC = 1, fbL = 1;
  fb_geometry((int)T, &fbC, &fbL);
  const size_t o_bnd = take((size_t)2 * 4 * fbC * 64 * 4), o_bg = take((size_t)2 * fbC * 8);
  const size_t o_chk = take((size_t)2 * fbC * 8);
  const size_t o_desc = take(sizeof(JobDesc)), o_start = take(8 * sizeof(int));
  char *a = nullptr;
  HIP_OK(hipMalloc(&a, off));
  std::unique_ptr<char, void (*)(char *)> guard(a, [](char *p) { (void)hipFree(p); });
  HIP_OK(hipMemcpyAsync(a + o_lev, logev, T_ * N * 4, hipMemcpyHostToDevice, st));
  HIP_OK(hipMemcpyAsync(a + o_A, A, (size_t)N * N * 4, hipMemcpyHostToDevice, st));
  HIP_OK(hipMemcpyAsync(a + o_pi, pi, (size_t)N * 4, hipMemcpyHostToDevice, st));
  JobDesc D{};
  D.S = 1; D.N = N; D.K = 1; D.M = N; D.T = (int)T; D.iters = 0;
  D.A_in = reinterpret_cast<const float *>(a + o_A);
  D.pi_in = reinterpret_cast<const float *>(a + o_pi);
  D.phi = reinterpret_cast<float *>(a + o_phi);
  D.ev = reinterpret_cast<float *>(a + o_ev);
  D.sh = reinterpret_cast<float *>(a + o_sh);
  D.fwd = reinterpret_cast<float *>(a + o_f);
  D.bwd = reinterpret_cast<float *>(a + o_b);
  D.lnz = reinterpret_cast<float2 *>(a + o_n);
  D.post = reinterpret_cast<float *>(a + o_p);
  D.chainflag = reinterpret_cast<int *>(a + o_flag);
  D.fbC = fbC;
  D.fbL = fbL;
  D.bnd = reinterpret_cast<float *>(a + o_bnd);
  D.bgain = reinterpret_cast<float2 *>(a + o_bg);
  D.bchk = reinterpret_cast<float2 *>(a + o_chk);
  const int npost = (int)((T_ + 3) / 4);
  const int start[8] = {0, 2 * fbC, 0, 2, 0, npost, 0, 1};    // rounds, fix-up, posterior, exact
  HIP_OK(hipMemcpyAsync(a + o_desc, &D, sizeof D, hipMemcpyHostToDevice, st));
  HIP_OK(hipMemcpyAsync(a + o_start, start, sizeof start, hipMemcpyHostToDevice, st));
  HIP_OK(launch_chain_prep(D, reinterpret_cast<const float *>(a + o_lev), st));
  WorkList wl[4];
  for (int i = 0; i < 4; ++i) {
    wl[i].jobs = reinterpret_cast<const JobDesc *>(a + o_desc);
    wl[i].start = reinterpret_cast<const int *>(a + o_start) + 2 * i;
    wl[i].njobs = 1;
    wl[i].total = start[2 * i + 1];
  }
  HIP_OK(launch_chain_fb(wl[0], wl[1], N, st));
  HIP_OK(launch_posterior(wl[2], wl[3], N, st));
  std::vector<float> sh(T_);
  float lnz2[2] = {0.0f, 0.0f};
  if (post) HIP_OK(hipMemcpyAsync(post, a + o_p, T_ * N * 4, hipMemcpyDeviceToHost, st));
  HIP_OK(hipMemcpyAsync(sh.data(), a + o_sh, T_ * 4, hipMemcpyDeviceToHost, st));
  HIP_OK(hipMemcpyAsync(lnz2, a + o_n, 8, hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  if (lnZ) {
    double z = 0.0;
    for (size_t t = 0; t < T_; ++t) z += (double)sh[t];
    z += (double)lnz2[0] + (double)lnz2[1];
    *lnZ = z;
  }
  return NFHMM_OK;
}

nfhmm_status nfhmm_special_functions(nfhmm_ctx *ctx, int64_t n, const float *x, float *psi, float *lgam) {
  if (!ctx || (n > 0 && !x) || n < 0) return fail(NFHMM_E_INVALID, "bad arguments");
  if (n == 0) return NFHMM_OK;
  HIP_OK(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  char *a = nullptr;
  const size_t b = (size_t)n * 4;
  HIP_OK(hipMalloc(&a, 3 * b));
  std::unique_ptr<char, void (*)(char *)> guard(a, [](char *p) { (void)hipFree(p); });
  HIP_OK(hipMemcpyAsync(a, x, b, hipMemcpyHostToDevice, st));
  HIP_OK(launch_special(n, reinterpret_cast<const float *>(a), psi ? reinterpret_cast<float *>(a + b) : nullptr,
                        lgam ? reinterpret_cast<float *>(a + 2 * b) : nullptr, st));
  if (psi) HIP_OK(hipMemcpyAsync(psi, a + b, b, hipMemcpyDeviceToHost, st));
  if (lgam) HIP_OK(hipMemcpyAsync(lgam, a + 2 * b, b, hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  return NFHMM_OK;
}

}  // extern "C"
