// Per-job descriptor shared by the host runtime and the kernels.
//
// Device layouts of one job (all row-major, padded with zeros):
//   V      [T][Fp]     mixture spectrogram, frame-major (Fp = F rounded up to 32,
//                      Mp = S*N*K rounded up to 32)
//   Wfm    [Fp][Mp]    beta_l(k) with k contiguous: the operand of Lambda = beta w
//   Wmf    [Mp][Fp]    beta_l(k) with l contiguous: the operand of beta^T R
//   alpha  [T][Mp]     Dirichlet parameters alpha-hat (Eq. 6), stored when an output
//   w      [T][Mp]     exp(psi(alpha_k) - psi(alpha_0)): the carried state
//                      (float32, or bfloat16 in wh)
//   R      [T][Fp]     V / Lambda (float32, or bfloat16 in Rh)
//   c      [T][Mp]     expected counts sum_l V z (the first term of Eq. 6)
//   phi    [S][T][64]  gamma * sum_j psi(alpha_(s,n,j)): Eq. 8 up to a per-frame constant
//   ev     [S][T][64]  exp(gamma*phi - sh): linear-domain chain evidence
//   sh     [S][T]      per-frame log shift of ev
//   fwd    [S][T][64]  scaled forward messages;  bwd: scaled backward messages
//   lnz    [S]         ln Z of each chain minus sum_t sh_t (hi, lo)
//   post   [S][T][N]   state marginals d-hat
//   vll    [nvl][T]    per (128-row tile, frame) partials of sum_l V ln Lambda (hi, lo);
//                      the last slot holds the tail bins when Ft > 0
// Bins: F = 2^k + 1 (a 2^(k+1)-point STFT) would waste most of a 64-row tile, so
// when F mod 64 is 1..4 the contractions run over Fm = F - (F mod 64) bins and
// the Ft tail bins are handled by k_update (their Lambda row: a dot product with
// the w it has just formed) and by the epilogue of k_counts (a rank-Ft update).
//   clw    [nkt][T]    per (64-row tile, frame) partials of -sum_k c ln w (hi, lo)
//   elbo   [iters][T]  per-frame bound contributions (hi, lo)
//   sep    [S][T][Fp]  reconstructions, then masked separations
//   chainflag [S]      1 if the chain's scaled messages lost posterior mass
#pragma once
#include <stdint.h>

namespace nfhmm {

constexpr int kLanes = 64;     // states per chain row (wavefront width)
constexpr int kMaxSources = 8;

// Block tiles of the two contractions: 2 x 2 wavefronts of 16*W rows x 16*W
// columns each.  Lambda (spectrum): bins x frames; counts: elements x frames.
constexpr int kSpecWM = 4, kSpecWN = 4;
constexpr int kCntWM = 2, kCntWN = 2;     // FP32 counts
constexpr int kCntHWM = 4, kCntHWN = 4;   // BF16 counts
constexpr int kSpecBM = 32 * kSpecWM, kSpecBN = 32 * kSpecWN;
constexpr int kCntBM = 32 * kCntWM, kCntBN = 32 * kCntWN;
constexpr int kCntHBM = 32 * kCntHWM, kCntHBN = 32 * kCntHWN;
constexpr int kBoundRows = 64;            // rows per partial of the bound's counts term
constexpr int kSpecSmallBM = 64, kSpecSmallBN = 64;   // spectrum tile for small batches
constexpr float kEvHeadroomLog = 44.3614195558365f;   // 64 ln 2: ev <= 2^64

// Chunks of the time-parallel forward-backward: about kFbChunk frames each, at
// most kFbMaxChunks per chain.  A job's chunking depends on its T only, so its
// results do not depend on what else runs beside it.
constexpr int kFbChunk = 64;
constexpr int kFbMaxChunks = 256;
inline void fb_geometry(int T, int *C, int *L) {
  int c = (T + kFbChunk - 1) / kFbChunk;
  c = c < 1 ? 1 : (c > kFbMaxChunks ? kFbMaxChunks : c);
  const int l = (T + c - 1) / c;
  *L = l;
  *C = (T + l - 1) / l;
}

enum Status : int { kOk = 0, kBadV = 1, kBadW = 2, kNonFinite = 4 };

struct JobDesc {
  int S, N, K, M, Mp, F, Fp, T;
  int NK;            // N*K
  int iters;
  int start_round;   // round in which this job runs its iteration 0
  int bf16;          // contraction operands in bfloat16
  float gamma;
  int nlt;           // ceil(Fp / 64): row tiles of the reconstruction
  int Fm;            // bins of the spectrum contraction (rows) and of the counts (k)
  int Ft;            // tail bins [Fm, F) handled outside the MFMA tiles (0..4)
  int nsl;           // ceil(Fm / 64): 64-bin slots of the spectrum's bound partials
                     // in vll (the tail bins' partial is slot nsl)
  int fbC, fbL;      // chunks of the forward-backward and frames per chunk
  double elbo_const; // T * (lnG(M + gamma S K) - S K lnG(1 + gamma))
  // inputs in the ABI layouts (device)
  const float *V_in, *W_in, *A_in, *pi_in, *alpha_init;
  // working layouts
  float *V, *Wfm, *Wmf;
  uint16_t *Wfm_h, *Wmf_h, *wh, *Rh;
  float *alpha, *w, *R, *c;
  float *phi, *ev, *sh, *fwd, *bwd, *post;
  float2 *vll, *clw, *elbo, *lnz;
  float *bnd;        // boundary messages of the chunked sweep [S][2][4][fbC][64]
  float2 *bgain;     // forward log gains of the chunks [S][2 rounds][fbC]
  float2 *bchk;      // round-2 verdicts (1 / 0) and log factors of the chunk starts [S][2][fbC]
  float *sep;
  int *status;
  int *chainflag;    // [S] set when a chain needs the exact log-space pass
  // outputs in the ABI layouts (device), any may be null
  float *out_alpha, *out_post, *out_sep;
  double *out_elbo;
};

// Work lists of one launch: block b of a grouped kernel belongs to the job j with
// start[j] <= b < start[j+1] (start[] is an exclusive prefix sum over the jobs).
struct WorkList {
  const JobDesc *jobs;
  const int *start;
  int njobs;
  int total;
};

}  // namespace nfhmm
