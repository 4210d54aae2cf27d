// EM learning of a source's N-HMM (Section 2.1), for one source or a batch of
// independent ones: descriptor and launchers of the kernels in nhmm_em_kernels.hip.
//
// Shapes: V [T][F] counts; beta [N][K][F] (each row of F values a distribution);
// theta [T][N][K] per-frame weights of each state's elements (rows over K sum to
// 1); A [N][N] row-stochastic; pi [N].
//
// Working precision.  With thousands of quanta per frame the frame likelihoods of
// two states differ by hundreds to thousands of nats, and EM drives transitions,
// initial probabilities and weights that the data do not use towards values far
// below the float32 range -- values that a later iteration may bring back, since
// EM's updates are multiplicative and a zero never recovers.  So between
// iterations beta and theta are kept in double, and A and pi as float32
// logarithms; the chain runs in log space and hands the beta update ln gamma.
// What counts as zero is what a double-precision evaluation flushes (kEmLogTiny).
// The ABI's float32 parameters are read at the start and written at the end.
#pragma once
#include <hip/hip_runtime.h>

#include "jobdesc.h"

namespace nfhmm {

constexpr int kEmMaxK = 32;      // elements per state
constexpr int kEmMaxBatch = 65535;   // problems per batch (grid y)
constexpr int kEmChunk = 32;     // frames per partial sum of the beta update's and the xi sums over t
constexpr int kEmSweepChunk = 32;   // frames per chunk of the time-parallel forward-backward
// ln 2^-1075, below which the exponential of a double rounds to zero (the
// subnormal doubles above it still count): probabilities (marginals, pairwise
// marginals, transitions, initial probabilities) below it count as zero, as they
// do in a double-precision evaluation of the same updates -- where a state or a
// transition whose every count underflows keeps its previous parameters.
constexpr float kEmLogTiny = -745.1332191019412f;

struct EmDesc {
  int N, K, F, T, nchunk;
  int nsw;                  // chunks of the time-parallel forward-backward (0: the sequential one)
  int iters;                // the problem's iteration count: later iterations skip it
  const float *V;           // [T][F]
  const double *beta;       // [N][K][F]   parameters this iteration starts from
  const double *theta;      // [T][N][K]
  const float *lnA;         // [N][N]      ln A (-inf where A = 0)
  const float *lnpi;        // [N]
  double *beta_new;         // [N][K][F]   parameters it produces
  double *theta_new;        // [T][N][K]
  float *lnA_new;           // [N][N]
  float *lnpi_new;          // [N]
  double *ll;               // [T][N]      frame log-likelihoods sum_f V ln P_t(f | d)
  double *off;              // [T]         their largest value per frame
  float *x;                 // [T][64]     ll - off: the chain's log evidence (row per frame)
  float *la;                // [T][64]     log forward messages, normalised per frame
  float *lbn;               // [T][64]     log backward messages, normalised per frame
  float *sI;                // [T][64]     the backward messages before that normalisation
  float *lgam;              // [T][N]      ln gamma_t(d), the log state marginals
  float *gmax;              // [N]         max_t ln gamma_t(d)
  float2 *xpart;            // [nchunk][N][64] per frame chunk: sum of xi_t(i, j) as (max, scaled sum)
  float *gpart;             // [nchunk][N] per frame chunk: max ln gamma_t(i)
  double *bpart;            // [nchunk][N][K][F] partial sums over frame chunks of the beta update
  double *trace;            // [iters]     ln P(V) of the parameters each iteration started from
  float *tm;                // [2][nsw][N][64] per direction and chunk: transfer columns (normalised logarithms)
  double *tz;               // [2][nsw][64]    their log scales
  float *ts;                // [2][nsw][64]    each chunk's start message
};

// A batch of independent problems: their descriptors for one iteration (device
// memory, n of them) and the largest sizes among them, which set the grids (grid
// y is the problem; blocks past a problem's own extent return at once) and the
// register tiles (KR >= K, NR >= N: the extra terms are exact zeros, so a
// problem's results do not depend on what else is in the batch).
struct EmBatch {
  const EmDesc *d;
  int n, maxN, maxK, maxF, maxT, maxChunk;
  int maxSw;     // the most sweep chunks of a problem (0: none is time-parallel)
  bool anySeq;   // some problem takes the sequential forward-backward
};

// E-step per (frame, state) -- frame log-likelihoods and the theta update, which
// needs no chain posterior -- and the chain's log-evidence rows.
hipError_t launch_em_frames(const EmBatch &B, int it, hipStream_t st);
// The chain (the forward-backward, sequential or time-parallel per problem, then
// gamma and the pairwise marginals over frame chunks): gamma, the new ln A and
// ln pi, and ln P(V) for iteration `it`.
hipError_t launch_em_chain(const EmBatch &B, int it, hipStream_t st);
// The beta update (after the chain).
hipError_t launch_em_beta(const EmBatch &B, int it, hipStream_t st);
// Conversions between the ABI's float32 parameters and the working ones.
hipError_t launch_em_import(int N, int K, int F, int T, const float *W, const float *theta, const float *A,
                            const float *pi, double *beta, double *th, float *lnA, float *lnpi, hipStream_t st);
// Any output pointer may be null.
hipError_t launch_em_export(int N, int K, int F, int T, const double *beta, const double *th, const float *lnA,
                            const float *lnpi, float *W, float *theta, float *A, float *pi, hipStream_t st);

}  // namespace nfhmm
