// HIP kernels (gfx950) of variational inference in the Bayesian N-FHMM.
//
// One iteration of the loop (Section 3.2 of the paper):
//   k_spectrum   Lambda = beta w,  R = V / Lambda, partials of sum V ln Lambda
//                (the normaliser kappa = ln Lambda of Eq. 7)            [MFMA]
//   k_counts     c = w (.) beta^T R: sum_l V z, the first term of Eq. 6 [MFMA]
//   k_fb_round (x2), k_fb_fixup
//                forward and backward recursions of every source chain on the
//                evidence of Eq. 8, swept in parallel over chunks of frames
//   k_posterior  d-hat from the messages (k_chain_exact where flagged)
//   k_update     Eq. 6, then psi / w / Eq. 8 for the next iteration, and the
//                per-frame bound contributions
// The chain kernels run on their own stream beside k_spectrum -> k_counts: given
// the current alpha-hat the chains and the contractions do not depend on each other.
//
// Z-hat of Eq. 7 is never formed: z[t,l,k] = beta[l,k] w[t,k] / Lambda[l,t]
// with w = exp(psi(alpha_tk) - psi(alpha_t0)), so sum_l V z is c[t,k] above.
#include <hip/hip_runtime.h>

#include "jobdesc.h"
#include "launch.h"
#include "special.h"
#include "wave.h"

namespace nfhmm {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ int find_job(const int *start, int njobs, int b) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Blocks are dealt round-robin to the 8 XCDs (block b -> XCD b % 8).  Give each
// XCD one contiguous range of logical tiles so that tiles sharing a job's
// dictionary and frame panels share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int n) {
  const int q = n >> 3, r = n & 7, x = b & 7, i = b >> 3;
  return x * q + min(x, r) + i;
}

// float -> bfloat16, round to nearest even (the gfx950 conversion instruction)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ------------------------------------------------------------------ packing
// Each packing step is a block body taking its block index; the kernels below
// run it over a work list that covers every job starting together (one launch
// per step; the allocation-free path builds a one-job list).

// V_in [T][F] -> V [T][Fp]; checks V finite and >= 0.  One wavefront per row.
__device__ __forceinline__ void pack_v_row(const JobDesc &J, int t, int lane) {
  bool bad = false;
  for (int l = lane; l < J.Fp; l += 64) {
    float v = 0.0f;
    if (l < J.F) {
      v = J.V_in[(size_t)t * J.F + l];
      if (!(v >= 0.0f) || isinf(v)) { bad = true; v = 0.0f; }
    }
    J.V[(size_t)t * J.Fp + l] = v;
  }
  if (__ballot(bad) != 0 && lane == 0) atomicOr(J.status, kBadV);
}

// W_in [M][F] -> Wmf [Mp][Fp] (+ bf16); checks rows finite, >= 0, summing to 1.
// One wavefront per row.
__device__ __forceinline__ void pack_wmf_row(const JobDesc &J, int k, int lane) {
  float s = 0.0f;
  bool bad = false;
  for (int l = lane; l < J.Fp; l += 64) {
    float v = 0.0f;
    if (k < J.M && l < J.F) {
      v = J.W_in[(size_t)k * J.F + l];
      if (!(v >= 0.0f) || isinf(v)) { bad = true; v = 0.0f; }
    }
    s += v;
    J.Wmf[(size_t)k * J.Fp + l] = v;
    if (J.bf16) J.Wmf_h[(size_t)k * J.Fp + l] = f2bf(v);
  }
  const float tot = wave_sum(s);
  const bool anybad = __ballot(bad) != 0;
  if (lane == 0 && k < J.M && (anybad || fabsf(tot - 1.0f) > 1e-4f)) atomicOr(J.status, kBadW);
}

// Wmf [Mp][Fp] -> Wfm [Fp][Mp] (+ bf16), 32x32 tiles through LDS.
__device__ __forceinline__ void transpose_tile(const JobDesc &J, int bx, int by) {
  __shared__ float tile[32][33];
  const int k0 = bx * 32, l0 = by * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 256 threads: 8 rows per pass
  for (int r = ty; r < 32; r += 8) tile[r][tx] = J.Wmf[(size_t)(k0 + r) * J.Fp + l0 + tx];
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const float v = tile[tx][r];
    J.Wfm[(size_t)(l0 + r) * J.Mp + k0 + tx] = v;
    if (J.bf16) J.Wfm_h[(size_t)(l0 + r) * J.Mp + k0 + tx] = f2bf(v);
  }
}

// w = 1 on the M real elements (z-hat proportional to beta), 0 on the padding:
// part b of nb of the job's T x Mp values.
__device__ __forceinline__ void fill_w_ones_part(const JobDesc &J, int b, int nb) {
  const size_t n = (size_t)J.T * J.Mp;
  for (size_t i = (size_t)b * blockDim.x + threadIdx.x; i < n; i += (size_t)nb * blockDim.x) {
    const float v = ((int)(i % J.Mp) < J.M) ? 1.0f : 0.0f;
    if (J.bf16) J.wh[i] = f2bf(v); else J.w[i] = v;
  }
}

// Batched forms over a work list.  Per job, k_begin_pack has ceil(T / 4) blocks
// packing V and Mp / 4 packing the dictionary (a row per wavefront), then
// (default start only) kBeginFillBlocks setting w = 1; k_begin_transpose one
// block per 32 x 32 tile.
__global__ void k_status_clear(WorkList wl) {
  for (int i = threadIdx.x; i < wl.njobs; i += blockDim.x) *wl.jobs[i].status = 0;
}

// dst[i] = status word of job i of the list
__global__ void k_status_gather(WorkList wl, int *dst) {
  for (int i = threadIdx.x; i < wl.njobs; i += blockDim.x) dst[i] = *wl.jobs[i].status;
}

__global__ __launch_bounds__(256) void k_begin_pack(WorkList wl) {
  const int b = blockIdx.x;
  const int jb = find_job(wl.start, wl.njobs, b);
  const JobDesc &J = wl.jobs[jb];
  const int local = b - wl.start[jb];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nv = (J.T + 3) / 4, nw = J.Mp / 4;   // blocks of four rows (one per wavefront)
  if (local < nv) {
    const int t = 4 * local + wave;
    if (t < J.T) pack_v_row(J, t, lane);
  } else if (local < nv + nw) {
    pack_wmf_row(J, 4 * (local - nv) + wave, lane);
  } else {
    fill_w_ones_part(J, local - nv - nw, kBeginFillBlocks);
  }
}

__global__ __launch_bounds__(256) void k_begin_transpose(WorkList wl) {
  const int b = blockIdx.x;
  const int jb = find_job(wl.start, wl.njobs, b);
  const JobDesc &J = wl.jobs[jb];
  const int local = b - wl.start[jb], nx = J.Mp / 32;
  transpose_tile(J, local % nx, local / nx);
}

// The default start (w = 1, Section 3.2's first iteration from a flat alpha-hat):
// Lambda = beta 1 is the same in every frame, the row sum of each bin's
// dictionary values, so the start forms it once per job (k_start_lambda: 16 bins
// per block, into the job's sep buffer, free until the separation) and then R =
// V / Lambda per frame (k_start_ratio), as the spectrum kernel's epilogue and
// the tail-bin path would.
__global__ __launch_bounds__(256) void k_start_lambda(WorkList wl) {
  const int b = blockIdx.x;
  const int jb = find_job(wl.start, wl.njobs, b);
  const JobDesc &J = wl.jobs[jb];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l0 = (b - wl.start[jb]) * kStartLamBinsPerBlock + wave * (kStartLamBinsPerBlock / 4);
  for (int i = 0; i < kStartLamBinsPerBlock / 4; ++i) {
    const int l = l0 + i;
    if (l >= J.F) break;   // uniform over the wave
    float acc = 0.0f;
    for (int k = lane; k < J.M; k += 64)
      acc += J.bf16 ? bf2f(J.Wfm_h[(size_t)l * J.Mp + k]) : J.Wfm[(size_t)l * J.Mp + k];
    const float lam = wave_sum(acc);
    if (lane == 0) J.sep[l] = lam;
  }
}

__global__ __launch_bounds__(256) void k_start_ratio(WorkList wl) {
  const int b = blockIdx.x;
  const int jb = find_job(wl.start, wl.njobs, b);
  const JobDesc &J = wl.jobs[jb];
  const int t = b - wl.start[jb];
  // every bin of the padded row: the contraction reads [0, Fm), which for a
  // ragged F without tail bins runs past F (V = 0 there, so R = 0)
  for (int l = threadIdx.x; l < J.Fp; l += blockDim.x) {
    const float v = J.V[(size_t)t * J.Fp + l], lam = l < J.F ? J.sep[l] : 1.0f;
    const float rr = v > 0.0f ? (l < J.Fm ? v * fast_rcp(lam) : v / lam) : 0.0f;
    if (J.bf16) J.Rh[(size_t)t * J.Fp + l] = f2bf(rr);
    else J.R[(size_t)t * J.Fp + l] = rr;
  }
}

// ------------------------------------------------------------------ MFMA tiles
// C[i][j] = sum_k A[i][k] B[j][k] for a (32*WM) x (32*WN) block tile: 256 threads
// = 4 waves in a 2x2 grid, each wave (16*WM) x (16*WN) = WM x WN MFMA 16x16 tiles
// held in accumulator registers.  Operand k-slices pass through LDS: loaded
// straight into it for the two contractions of every iteration (below,
// gemm_nt_f32_dma / gemm_nt_bf16_dma), and for the once-per-job reconstruction,
// whose k range is arbitrary, with its ragged stages masked in LDS.  A larger wave tile
// reuses every fragment read from LDS across more MFMAs.  Within every 16 (f32)
// or 32 (bf16) wide k-chunk lane (r, q) of a fragment supplies the q-th group of
// consecutive k; A and B use the same grouping, so every k is summed once.
// Output tile element (row, col) lives in lane (lr, lq) of wave (wr, wc) at
// acc[i][j][r] with row = wr*16*WM + i*16 + 4*lq + r, col = wc*16*WN + j*16 + lr.
struct Frag {
  int wr, wc, lr, lq;
};
__device__ __forceinline__ Frag frag_of(int tid) {
  const int wave = tid >> 6, lane = tid & 63;
  Frag f;
  f.wr = wave >> 1; f.wc = wave & 1; f.lr = lane & 15; f.lq = lane >> 4;
  return f;
}

constexpr int kBKf = 32;                            // f32: 32 k per stage
constexpr int kBKh = 64;                            // bf16: 64 k per stage

// f32 main loop with the operands loaded straight into LDS (global_load_lds,
// 16 bytes per lane; no staging registers and no LDS store instructions).  A
// wavefront instruction fills eight rows of 32 floats, contiguous in LDS, so the
// rows are not padded; instead row r keeps the 16-byte chunk ch of its global
// row at position ch ^ (r & 7), which lets the fragment reads of eight
// consecutive rows fall on eight different bank groups.  Rows past the end of
// an operand read its last row (their outputs are not stored); the k range must
// be whole stages of 32.
typedef __attribute__((address_space(1))) const void gcvoid;
typedef __attribute__((address_space(3))) void lvoid;
constexpr int kDmaRow = 32;   // floats per LDS row (one k-stage)

template <int ROWS>
__device__ __forceinline__ void dma_rows(const float *__restrict__ src, int ld, int nrows, int row0, int k,
                                         float *lds, int wave, int lane) {
  constexpr int kGroups = ROWS / 32;   // eight-row groups per wavefront
#pragma unroll
  for (int h = 0; h < kGroups; ++h) {
    const int g = wave * kGroups + h;
    const int r = g * 8 + (lane >> 3);
    const int ch = (lane & 7) ^ (r & 7);
    const int grow = min(row0 + r, nrows - 1);
    __builtin_amdgcn_global_load_lds((gcvoid *)(src + (size_t)grow * ld + k + ch * 4),
                                     (lvoid *)(lds + g * 8 * kDmaRow), 16, 0, 0);
  }
}

template <int WM, int WN>
__device__ __forceinline__ void mma_stage_f32_dma(const float *As, const float *Bs, const Frag &f,
                                                  floatx4 (&acc)[WM][WN]) {
  const int sw = f.lr & 7;   // every fragment row is 16-aligned, so row & 7 = lr & 7
#pragma unroll
  for (int kk = 0; kk < kBKf; kk += 16) {
    const int chunk = ((kk >> 2) + f.lq) ^ sw;
    float4 a[WM], b[WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
      a[i] = *(const float4 *)(As + (f.wr * 16 * WM + i * 16 + f.lr) * kDmaRow + chunk * 4);
#pragma unroll
    for (int j = 0; j < WN; ++j)
      b[j] = *(const float4 *)(Bs + (f.wc * 16 * WN + j * 16 + f.lr) * kDmaRow + chunk * 4);
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) {
          const float av = p == 0 ? a[i].x : p == 1 ? a[i].y : p == 2 ? a[i].z : a[i].w;
          const float bv = p == 0 ? b[j].x : p == 1 ? b[j].y : p == 2 ? b[j].z : b[j].w;
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[i][j], 0, 0, 0);
        }
  }
}

template <int WM, int WN>
__device__ void gemm_nt_f32_dma(const float *__restrict__ A, int lda, int arows, int row0, const float *__restrict__ B,
                                int ldb, int bcols, int col0, int kb, int ke, floatx4 (&acc)[WM][WN]) {
  constexpr int BM = 32 * WM, BN = 32 * WN;
  // two stages in four separate arrays, and the loop unrolled by two, so that
  // every access names its buffer and the compiler can tell that the loads in
  // flight into one stage do not touch the stage being read
  __shared__ __attribute__((aligned(16))) float As0[BM * kDmaRow], As1[BM * kDmaRow];
  __shared__ __attribute__((aligned(16))) float Bs0[BN * kDmaRow], Bs1[BN * kDmaRow];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const Frag f = frag_of(tid);
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  dma_rows<BM>(A, lda, arows, row0, kb, As0, wave, lane);
  dma_rows<BN>(B, ldb, bcols, col0, kb, Bs0, wave, lane);
  __syncthreads();
  for (int k = kb; k < ke; k += 2 * kBKf) {
    if (k + kBKf < ke) {   // stage 1 was last read before the previous barrier
      dma_rows<BM>(A, lda, arows, row0, k + kBKf, As1, wave, lane);
      dma_rows<BN>(B, ldb, bcols, col0, k + kBKf, Bs1, wave, lane);
    }
    // a raised wave priority while the stage's MFMAs issue: of the waves sharing a
    // SIMD, one that has begun its cluster keeps the matrix pipe (measured +1.4 %
    // on the loop; no gain in the bf16 loop, which is not issue-bound)
    __builtin_amdgcn_s_setprio(1);
    mma_stage_f32_dma<WM, WN>(As0, Bs0, f, acc);
    __builtin_amdgcn_s_setprio(0);
    // the MFMAs stay before the barrier (and its wait for the loads in flight),
    // which the scheduler would otherwise move above them
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();   // each wavefront waits for its own loads first
    if (k + kBKf >= ke) break;
    if (k + 2 * kBKf < ke) {
      dma_rows<BM>(A, lda, arows, row0, k + 2 * kBKf, As0, wave, lane);
      dma_rows<BN>(B, ldb, bcols, col0, k + 2 * kBKf, Bs0, wave, lane);
    }
    __builtin_amdgcn_s_setprio(1);
    mma_stage_f32_dma<WM, WN>(As1, Bs1, f, acc);
    __builtin_amdgcn_s_setprio(0);
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();
  }
}

// The same for a k range [kb, ke) in any position (the reconstruction: one
// source's elements): whole stages of 32 from kb rounded down to ke rounded up
// (within the padded rows), loaded straight into LDS as above; in the first and
// last stage the B entries outside [kb, ke) are set to zero in LDS, between two
// barriers, before their MFMAs.
template <int BN>
__device__ __forceinline__ void mask_stage_b(float *Bs, int ks, int kb, int ke, int tid) {
  if (ks >= kb && ks + kBKf <= ke) return;   // uniform over the block
  for (int idx = tid; idx < BN * kDmaRow; idx += blockDim.x) {
    const int r = idx / kDmaRow, kl = idx - r * kDmaRow, k = ks + kl;
    if (k < kb || k >= ke) Bs[r * kDmaRow + (((kl >> 2) ^ (r & 7)) << 2) + (kl & 3)] = 0.0f;
  }
  __syncthreads();
}

template <int WM, int WN>
__device__ void gemm_nt_f32_dma_kmask(const float *__restrict__ A, int lda, int arows, int row0,
                                      const float *__restrict__ B, int ldb, int bcols, int col0, int kb, int ke,
                                      floatx4 (&acc)[WM][WN]) {
  constexpr int BM = 32 * WM, BN = 32 * WN;
  __shared__ __attribute__((aligned(16))) float As0[BM * kDmaRow], As1[BM * kDmaRow];
  __shared__ __attribute__((aligned(16))) float Bs0[BN * kDmaRow], Bs1[BN * kDmaRow];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const Frag f = frag_of(tid);
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int k0 = kb & ~(kBKf - 1), k1 = (ke + kBKf - 1) & ~(kBKf - 1);
  dma_rows<BM>(A, lda, arows, row0, k0, As0, wave, lane);
  dma_rows<BN>(B, ldb, bcols, col0, k0, Bs0, wave, lane);
  __syncthreads();
  mask_stage_b<BN>(Bs0, k0, kb, ke, tid);
  for (int k = k0; k < k1; k += 2 * kBKf) {
    if (k + kBKf < k1) {
      dma_rows<BM>(A, lda, arows, row0, k + kBKf, As1, wave, lane);
      dma_rows<BN>(B, ldb, bcols, col0, k + kBKf, Bs1, wave, lane);
    }
    mma_stage_f32_dma<WM, WN>(As0, Bs0, f, acc);
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();
    if (k + kBKf >= k1) break;
    mask_stage_b<BN>(Bs1, k + kBKf, kb, ke, tid);
    if (k + 2 * kBKf < k1) {
      dma_rows<BM>(A, lda, arows, row0, k + 2 * kBKf, As0, wave, lane);
      dma_rows<BN>(B, ldb, bcols, col0, k + 2 * kBKf, Bs0, wave, lane);
    }
    mma_stage_f32_dma<WM, WN>(As1, Bs1, f, acc);
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();
    if (k + 2 * kBKf < k1) mask_stage_b<BN>(Bs0, k + 2 * kBKf, kb, ke, tid);
  }
}

// Wait until at most N vector-memory operations of this wavefront are still in
// flight (gfx9 s_waitcnt encoding: vmcnt in bits 3:0 and 15:14; expcnt and
// lgkmcnt left at their no-wait maxima).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt is six bits");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// bf16 main loop with the same direct-to-LDS scheme: a k-stage of 64 values is
// again eight 16-byte chunks per row.  kend is a multiple of 32; in a final half
// stage the chunks at or past kend load the row's last chunk again (in bounds,
// and every stage is the same loads), and the A rows' copies are then set to
// zero in LDS.
template <int ROWS>
__device__ __forceinline__ void dma_rows_h(const uint16_t *__restrict__ src, int ld, int nrows, int row0, int k,
                                           int kend, uint16_t *lds, int wave, int lane) {
  constexpr int kGroups = ROWS / 32;
#pragma unroll
  for (int h = 0; h < kGroups; ++h) {
    const int g = wave * kGroups + h;
    const int r = g * 8 + (lane >> 3);
    const int ch = (lane & 7) ^ (r & 7);
    const int grow = min(row0 + r, nrows - 1);
    const int kk = min(k + ch * 8, kend - 8);
    __builtin_amdgcn_global_load_lds((gcvoid *)(src + (size_t)grow * ld + kk), (lvoid *)(lds + g * 8 * kBKh), 16,
                                     0, 0);
  }
}

// A stage's fragment reads take this lane's offsets within the stage, formed once
// per block (ao / bo: A and B rows, one per 32-wide half of the stage's k) and
// hidden from the optimiser, so that every read address is the stage array plus
// one offset plus a constant: the LDS lowering then still sees which stage array
// each read belongs to (it follows only a few levels of address arithmetic), and
// the compiler's wait before the read counts only the loads into that array.
template <int WM, int WN>
__device__ __forceinline__ void mma_stage_bf16_dma(const uint16_t *As, const uint16_t *Bs, const int (&ao)[2],
                                                   const int (&bo)[2], floatx4 (&acc)[WM][WN]) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    bf16x8 a[WM], b[WN];
#pragma unroll
    for (int i = 0; i < WM; ++i) a[i] = *(const bf16x8 *)(As + ao[h] + i * 16 * kBKh);
#pragma unroll
    for (int j = 0; j < WN; ++j) b[j] = *(const bf16x8 *)(Bs + bo[h] + j * 16 * kBKh);
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int j = 0; j < WN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  }
}

template <int WM, int WN>
struct Bf16Operands {
  const uint16_t *A, *B;
  int lda, arows, row0, ldb, bcols, col0, kend, wave, lane;
  __device__ __forceinline__ void load(int stage, uint16_t *lds) const {
    dma_rows_h<32 * WM>(A, lda, arows, row0, stage * kBKh, kend, lds, wave, lane);
    dma_rows_h<32 * WN>(B, ldb, bcols, col0, stage * kBKh, kend, lds + 32 * WM * kBKh, wave, lane);
  }
};

// Two stage buffers, one stage in flight.  Before each stage: this wavefront's
// loads of it have landed (vmcnt 0), then a barrier without a fence shows that
// every wavefront's part has landed and that every wavefront is done with the
// other buffer, which the next stage's loads then refill while this one's MFMAs
// run.  The two steps of a round are written out by recursion over the buffers
// (each names its buffer at compile time; the same loop written as one body
// unrolled by two came out at 224 registers in the counts kernel against 132
// here, and 2 % slower).  A final half stage runs after the loop, with its
// zeros set in LDS.
template <int U>
__device__ __forceinline__ uint16_t *stage_buf(uint16_t *L0, uint16_t *L1) {
  if constexpr (U == 0) return L0;
  else return L1;
}

template <int WM, int WN, int U>
__device__ __forceinline__ void bf16_steps(const Bf16Operands<WM, WN> &op, const int (&ao)[2], const int (&bo)[2],
                                           floatx4 (&acc)[WM][WN], int s0, int nrun, int nst, uint16_t *L0,
                                           uint16_t *L1) {
  if constexpr (U < 2) {
    const int s = s0 + U;
    if (s >= nrun) return;
    wait_vmcnt<0>();
    __builtin_amdgcn_s_barrier();
    if (s + 1 < nst) op.load(s + 1, stage_buf<(U + 1) % 2>(L0, L1));
    uint16_t *cur = stage_buf<U>(L0, L1);
    mma_stage_bf16_dma<WM, WN>(cur, cur + 32 * WM * kBKh, ao, bo, acc);
    // the MFMAs stay before the next stage's wait and barrier
    __builtin_amdgcn_sched_barrier(0);
    bf16_steps<WM, WN, U + 1>(op, ao, bo, acc, s0, nrun, nst, L0, L1);
  }
}

template <int WM, int WN>
__device__ void gemm_nt_bf16_dma(const uint16_t *__restrict__ A, int lda, int arows, int row0,
                                 const uint16_t *__restrict__ B, int ldb, int bcols, int col0, int kend,
                                 floatx4 (&acc)[WM][WN]) {
  constexpr int kStage = 32 * (WM + WN) * kBKh;
  __shared__ __attribute__((aligned(16))) uint16_t L0[kStage], L1[kStage];
  const int tid = threadIdx.x;
  const Frag f = frag_of(tid);
  const Bf16Operands<WM, WN> op{A, B, lda, arows, row0, ldb, bcols, col0, kend, tid >> 6, tid & 63};
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  int ao[2], bo[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int chunk = (h * 4 + f.lq) ^ (f.lr & 7);   // every fragment row is 16-aligned: row & 7 = lr & 7
    ao[h] = (f.wr * 16 * WM + f.lr) * kBKh + chunk * 8;
    bo[h] = (f.wc * 16 * WN + f.lr) * kBKh + chunk * 8;
  }
  __asm__ volatile("" : "+v"(ao[0]), "+v"(ao[1]), "+v"(bo[0]), "+v"(bo[1]));
  const int nst = (kend + kBKh - 1) / kBKh;
  const bool half = (kend & (kBKh - 1)) != 0;
  const int nrun = half ? nst - 1 : nst;
  if (nst > 0) op.load(0, L0);
  for (int s0 = 0; s0 < nrun; s0 += 2) bf16_steps<WM, WN, 0>(op, ao, bo, acc, s0, nrun, nst, L0, L1);
  if (half) {
    uint16_t *cur = ((nst - 1) & 1) ? L1 : L0;
    wait_vmcnt<0>();
    __syncthreads();
    // zero in A's rows the chunks at or past kend: B's copies of its last chunk
    // then meet zeros
    const int c0 = (kend & (kBKh - 1)) >> 3;
    for (int idx = tid; idx < 32 * WM * 8; idx += 256) {
      const int r = idx >> 3, c = idx & 7;
      if (c >= c0) *(uint4 *)(cur + r * kBKh + ((c ^ (r & 7)) << 3)) = make_uint4(0, 0, 0, 0);
    }
    __syncthreads();
    mma_stage_bf16_dma<WM, WN>(cur, cur + 32 * WM * kBKh, ao, bo, acc);
  }
}

// ------------------------------------------------------------------ Eq. 7: Lambda, R
// Rows l (frequency, [0, Fm)), columns t (frames), k over all M elements.
// Block tiles: FP32 64 x 64; BF16 128 bins x 128 frames for large batches (its
// stages wait on the operand requests from L1 to L2, and the larger tile asks for
// fewer bytes per flop), 64 x 64 when the batch would not fill the chip.  Either
// way the per-frame partials of sum V ln Lambda go to one slot per 64 bins (nsl
// slots), so the bound does not depend on the tile chosen.  Two blocks of four
// wavefronts per CU fit the LDS; the registers are held to that.
template <bool kBF16, int WM, int WN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_spectrum(WorkList wl) {
  static_assert(WM == 2 || WM == 4, "a wave row covers 32 or 64 bins");
  constexpr int BM = 32 * WM, BN = 32 * WN;
  const int b = xcd_remap(blockIdx.x, wl.total);
  const int jb = find_job(wl.start, wl.njobs, b);
  const JobDesc &J = wl.jobs[jb];
  const int T = J.T, Fp = J.Fp, Fm = J.Fm, nsl = J.nsl;
  const gfloat *Vin = gptr(J.V);
  gfloat *Rout = gptr(J.R);
  gu16 *Rh = gptr(J.Rh);
  gfloat2 *vll = gptr(J.vll);
  const int tile = b - wl.start[jb];
  const int nrt = (Fm + BM - 1) / BM;
  const int rt = tile % nrt, ct = tile / nrt;
  const int row0 = rt * BM, col0 = ct * BN;
  floatx4 acc[WM][WN];
  if constexpr (kBF16) gemm_nt_bf16_dma<WM, WN>(J.Wfm_h, J.Mp, J.Fm, row0, J.wh, J.Mp, J.T, col0, J.Mp, acc);
  else gemm_nt_f32_dma<WM, WN>(J.Wfm, J.Mp, J.Fm, row0, J.w, J.Mp, J.T, col0, 0, J.Mp, acc);

  const Frag f = frag_of(threadIdx.x);
  __shared__ Comp part[2][BN];
#pragma unroll
  for (int j = 0; j < WN; ++j) {
    const int t = col0 + f.wc * 16 * WN + j * 16 + f.lr;
    // one partial per 32 bins (i / 2), so that a 64-bin slot is summed in the same
    // order whichever tile covers it: the bound does not depend on the batch
    Comp cs2[WM / 2];
#pragma unroll
    for (int h = 0; h < WM / 2; ++h) cs2[h] = comp_zero();
    if (t < T) {
#pragma unroll
      for (int i = 0; i < WM; ++i) {
        const int l = row0 + f.wr * 16 * WM + i * 16 + 4 * f.lq;
        if (l < Fm) {
          const vf4 v = *(const gfloat4 *)(Vin + (size_t)t * Fp + l);
          const float lam[4] = {acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]};
          const float vv[4] = {v.x, v.y, v.z, v.w};
          float rr[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            rr[r] = vv[r] > 0.0f ? vv[r] * fast_rcp(lam[r]) : 0.0f;
            if (vv[r] > 0.0f) comp_add(cs2[i >> 1], vv[r] * ln_pos(lam[r]));
          }
          if constexpr (kBF16) {
            vu2 h;
            h.x = (uint32_t)f2bf(rr[0]) | ((uint32_t)f2bf(rr[1]) << 16);
            h.y = (uint32_t)f2bf(rr[2]) | ((uint32_t)f2bf(rr[3]) << 16);
            *(guint2 *)(Rh + (size_t)t * Fp + l) = h;
          } else {
            *(gfloat4 *)(Rout + (size_t)t * Fp + l) = vf4{rr[0], rr[1], rr[2], rr[3]};
          }
        }
      }
    }
    // reduce over the 4 lane groups that share column t
#pragma unroll
    for (int h = 0; h < WM / 2; ++h)
#pragma unroll
      for (int o = 16; o < 64; o <<= 1) {
        Comp d;
        d.hi = __shfl_xor(cs2[h].hi, o);
        d.lo = __shfl_xor(cs2[h].lo, o);
        cs2[h] = comp_merge(cs2[h], d);
      }
    const Comp cs = cs2[0];
    if constexpr (WM == 4) {   // a wave row is one 64-bin slot: its two halves merged as two wave rows are
      const int slot = rt * 2 + f.wr;
      const Comp tot = comp_merge(cs2[0], cs2[WM / 2 - 1]);
      if (f.lq == 0 && t < T && slot < nsl) vll[(size_t)slot * T + t] = vf2{tot.hi, tot.lo};
    } else {                   // the two wave rows form one slot
      if (f.lq == 0 && f.wr == 1) part[f.wc][j * 16 + f.lr] = cs;
      __syncthreads();
      if (f.lq == 0 && f.wr == 0 && t < T) {
        const Comp tot = comp_merge(cs, part[f.wc][j * 16 + f.lr]);
        vll[(size_t)rt * T + t] = vf2{tot.hi, tot.lo};
      }
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------------ Eq. 6 first term: c
// Rows k (elements), columns t (frames), contraction over the Fm bins, plus the
// rank-Ft update of the tail bins in the epilogue.
// Block tiles: FP32 64 x 64; BF16 128 x 128, for the same reason as the spectrum's
// (half the operand bytes per flop).  Either way the partials of the bound go to
// one slot per 64 rows.
template <bool kBF16>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kBF16 ? 2 : 1))) void k_counts(WorkList wl) {
  constexpr int WM = kBF16 ? kCntHWM : kCntWM, WN = kBF16 ? kCntHWN : kCntWN, BM = 32 * WM, BN = 32 * WN;
  static_assert(WM == 2 || WM == 4, "a wave row covers 32 or 64 rows");
  static_assert(kCntBM == kBoundRows, "the FP32 row tile is one partial slot");
  const int b = xcd_remap(blockIdx.x, wl.total);
  const int jb = find_job(wl.start, wl.njobs, b);
  const JobDesc &J = wl.jobs[jb];
  const int T = J.T, Fp = J.Fp, Fm = J.Fm, Ft = J.Ft, Mp = J.Mp;
  const gfloat *Rin = gptr(J.R), *Wmf = gptr(J.Wmf), *win = gptr(J.w);
  const gu16 *Rh = gptr(J.Rh), *Wmf_h = gptr(J.Wmf_h), *wh = gptr(J.wh);
  gfloat *cout = gptr(J.c);
  gfloat2 *clw = gptr(J.clw);
  const int tile = b - wl.start[jb];
  const int nrt = (Mp + BM - 1) / BM;
  const int rt = tile % nrt, ct = tile / nrt;
  const int row0 = rt * BM, col0 = ct * BN;
  floatx4 acc[WM][WN];
  if constexpr (kBF16) gemm_nt_bf16_dma<WM, WN>(J.Wmf_h, J.Fp, J.Mp, row0, J.Rh, J.Fp, J.T, col0, J.Fm, acc);
  else gemm_nt_f32_dma<WM, WN>(J.Wmf, J.Fp, J.Mp, row0, J.R, J.Fp, J.T, col0, 0, J.Fm, acc);
  const Frag f = frag_of(threadIdx.x);
  __shared__ Comp part[2][BN];
#pragma unroll
  for (int j = 0; j < WN; ++j) {
    const int t = col0 + f.wc * 16 * WN + j * 16 + f.lr;
    Comp cs = comp_zero();     // -sum_k c ln w over this tile's rows: a bound term
    if (t < T) {
#pragma unroll
      for (int i = 0; i < WM; ++i) {
        const int k = row0 + f.wr * 16 * WM + i * 16 + 4 * f.lq;
        if (k >= Mp) continue;
        // tail bins: acc += beta[l][k] R[t][l] for l in [Fm, F)
        for (int l = Fm; l < Fm + Ft; ++l) {
          float rl;
          float wk[4];
          if constexpr (kBF16) {
            rl = bf2f(Rh[(size_t)t * Fp + l]);
#pragma unroll
            for (int r = 0; r < 4; ++r) wk[r] = bf2f(Wmf_h[(size_t)(k + r) * Fp + l]);
          } else {
            rl = Rin[(size_t)t * Fp + l];
#pragma unroll
            for (int r = 0; r < 4; ++r) wk[r] = Wmf[(size_t)(k + r) * Fp + l];
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[i][j][r] = fmaf(wk[r], rl, acc[i][j][r]);
        }
        vf4 w;
        if constexpr (kBF16) {
          const vu2 h = *(const guint2 *)(wh + (size_t)t * Mp + k);
          w = vf4{bf2f((uint16_t)(h.x & 0xffff)), bf2f((uint16_t)(h.x >> 16)),
                  bf2f((uint16_t)(h.y & 0xffff)), bf2f((uint16_t)(h.y >> 16))};
        } else {
          w = *(const gfloat4 *)(win + (size_t)t * Mp + k);
        }
        const vf4 c = vf4{w.x * acc[i][j][0], w.y * acc[i][j][1], w.z * acc[i][j][2], w.w * acc[i][j][3]};
        *(gfloat4 *)(cout + (size_t)t * Mp + k) = c;
        if (w.x > 0.0f) comp_add(cs, -c.x * ln_pos(w.x));
        if (w.y > 0.0f) comp_add(cs, -c.y * ln_pos(w.y));
        if (w.z > 0.0f) comp_add(cs, -c.z * ln_pos(w.z));
        if (w.w > 0.0f) comp_add(cs, -c.w * ln_pos(w.w));
      }
    }
#pragma unroll
    for (int o = 16; o < 64; o <<= 1) {
      Comp d;
      d.hi = __shfl_xor(cs.hi, o);
      d.lo = __shfl_xor(cs.lo, o);
      cs = comp_merge(cs, d);
    }
    if constexpr (WM == 4) {   // a wave row is one 64-row slot
      const int slot = rt * 2 + f.wr;
      if (f.lq == 0 && t < T && slot * kBoundRows < Mp) clw[(size_t)slot * T + t] = vf2{cs.hi, cs.lo};
    } else {                   // the two wave rows form one slot
      if (f.lq == 0 && f.wr == 1) part[f.wc][j * 16 + f.lr] = cs;
      __syncthreads();
      if (f.lq == 0 && f.wr == 0 && t < T) {
        const Comp tot = comp_merge(cs, part[f.wc][j * 16 + f.lr]);
        clw[(size_t)rt * T + t] = vf2{tot.hi, tot.lo};
      }
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------------ forward-backward
// One 64-lane wavefront per (job, source, direction, chunk).  Lane n < N owns
// state n.  Messages are linear vectors with per-frame log offsets (the scaled
// recursion of Rabiner's tutorial, which the paper cites): the evidence row of
// frame t is ev = exp(gamma*phi - sh_t) <= 2^64, and each message is rescaled by
// the power of two 2^-k_t that brings its normaliser into [1/2, 1), so
//   ln Z = sum_t sh_t + lnz,   lnz = ln sum_n u_{T-1}(n) + ln 2 * sum_t k_t
// is exact integer bookkeeping.
// Lane N (the first unused lane) holds one extra row of the transition
// operator so that the normaliser comes out of the same FMA pass: all ones in
// the forward direction (sum of the incoming message), the column sums of A in
// the backward direction (sum of the outgoing message).  For N = 64 a reduction
// is used instead.
// The largest entry of every forward message and of every backward message times
// the evidence is kept above 2^-20: a frame where all of them would fall below is
// redone in log space with its own shift (the forward adds the shift's change to
// its log gain).  States that end up more than ~100 nats below a frame's best are
// flushed to zero; k_posterior detects the frames where that could matter and
// k_chain_exact then recomputes the chain entirely in log space.
//
// Time-parallel sweep.  The T frames are cut into C chunks of L frames:
//   round 1  every chunk is swept from a uniform start (the first forward chunk
//            from pi, the last backward chunk from b = 1: both exact);
//   round 2  every chunk whose round-1 start disagrees with its neighbour's
//            round-1 end is swept again from that end;
//   fix-up   one wavefront per chain and direction walks the chunks in order and
//            sweeps again every chunk whose start disagrees with the final end of
//            its neighbour, so the result is that of the sequential recursion
//            whatever the chain's memory.
// Two boundary messages agree when every state matches to 2^-20 relative, or both
// lie below 2^-60 of the largest state (where k_posterior's 40-nat check takes
// over).  A chunk forgets its start geometrically, so after round 2 the fix-up
// normally sweeps nothing and the critical path is about 2L steps instead of T.
// Boundary messages are stored with their largest entry scaled by a power of two
// into [1/2, 1); a forward chunk's log gain G (exponents times ln 2, plus the
// log-space shifts) is relative to its start, and lnz = sum_c G_c + ln sum_n u_{T-1}.
//
// Each sweep runs in blocks of kFbBlock frames whose evidence rows are loaded one
// block ahead, before that block's message stores, so the waits for the loads
// never include the stores (stores and loads share one counter on gfx9).
constexpr float kRescue = 9.5367431640625e-07f;      // 2^-20
constexpr float kChunkTol = 9.5367431640625e-07f;    // 2^-20
constexpr float kChunkFloor = 8.673617379884035e-19f;  // 2^-60
constexpr int kFbBlock = 8;

// One recursion step: every lane publishes x through LDS, then forms
// y = sum_m x_m coef[m]; tot is the normaliser (lane N's row, or a reduction).
template <int NR>
__device__ __forceinline__ float chain_apply(float *buf, int &p, const float (&coef)[NR], float x, int lane, int N,
                                             bool sumlane, bool live, bool fwd, float &tot) {
  float y0 = 0.0f, y1 = 0.0f, y2 = 0.0f, y3 = 0.0f;
  if (lane < NR) buf[p * NR + lane] = x;
  // The block is one wavefront and LDS executes a wavefront's operations in issue
  // order, so the reads below see every lane's write; only the compiler must not
  // move them across (no instruction, no wait on the outstanding global stores).
  __asm__ volatile("" ::: "memory");
  float4 v[NR / 4];
#pragma unroll
  for (int q = 0; q < NR / 4; ++q) v[q] = *(const float4 *)(buf + p * NR + 4 * q);
  p ^= 1;
  // four independent accumulators: the dependent chain is NR/4 FMAs long
#pragma unroll
  for (int q = 0; q < NR / 4; ++q) {
    y0 = fmaf(v[q].x, coef[4 * q + 0], y0);
    y1 = fmaf(v[q].y, coef[4 * q + 1], y1);
    y2 = fmaf(v[q].z, coef[4 * q + 2], y2);
    y3 = fmaf(v[q].w, coef[4 * q + 3], y3);
  }
  const float y = (y0 + y1) + (y2 + y3);
  if (sumlane) tot = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(y), N));
  else tot = wave_sum(live ? (fwd ? x : y) : 0.0f);
  return y;
}

// Scale a boundary message by the power of two that brings its largest entry into
// [1/2, 1); returns the exponent removed (0 for a zero or non-finite message).
__device__ __forceinline__ int canon_msg(float &x, bool live) {
  const float mx = wave_max(live ? x : 0.0f);
  if (!(mx > 0.0f && mx < INFINITY)) return 0;
  const int k = __builtin_amdgcn_frexp_expf(mx);
  x = ldexpf(x, -k);
  return k;
}

// Do two messages agree up to a positive factor?  Each is divided by its largest
// entry; on agreement lr = ln(max b / max a), the log of the factor that turns a
// into b (a forward gain measured from a start a then holds from b once lr is
// added).  Two zero messages agree; a zero and a non-zero one do not.
__device__ __forceinline__ bool msgs_agree(float a, float b, bool live, float &lr) {
  const float ma = wave_max(live ? a : 0.0f), mb = wave_max(live ? b : 0.0f);
  lr = 0.0f;
  if (!(ma > 0.0f) || !(mb > 0.0f)) return !(ma > 0.0f) && !(mb > 0.0f) && ma == 0.0f && mb == 0.0f;
  const float an = a / ma, bn = b / mb;
  const bool ok = !live || fabsf(an - bn) <= kChunkTol * fmaxf(an, bn) + kChunkFloor;
  lr = logf(mb) - logf(ma);
  return __ballot(!ok) == 0;
}

// Forward sweep over frames [t0, t1).  For t0 == 0 it starts from pi; otherwise u
// is the message of frame t0 - 1.  On return u is the message of frame t1 - 1 and
// g its log gain relative to the start.
template <int NR>
__device__ void fwd_sweep(const JobDesc &J, int s, const float (&coef)[NR], float *buf, int t0, int t1, float &u,
                          double &g) {
  const int lane = threadIdx.x & 63, N = J.N, T = J.T;
  const bool sumlane = N < 64, live = lane < N;
  const gfloat *ev = gptr(J.ev + (size_t)s * T * 64 + lane);
  const gfloat *phi = gptr(J.phi + (size_t)s * T * 64 + lane);
  gfloat *fwd = gptr(J.fwd + (size_t)s * T * 64 + lane);
  const gfloat *sh = gptr(J.sh + (size_t)s * T);
  int p = 0, ksum = 0;
  float lam = 0.0f, yr = 0.0f;
  int t = t0;
  if (t0 == 0) {
    const float p0 = live ? J.pi_in[(size_t)s * N + lane] : 0.0f;
    u = p0 * ev[0];
    if (__ballot(live && u > kRescue) == 0) {   // frame 0 in log space
      const float x = live ? logf(p0) + phi[0] : -INFINITY;
      const float mx = wave_max(x);
      u = (live && mx > -INFINITY) ? expf(x - mx + kEvHeadroomLog) : 0.0f;
      lam += (mx - kEvHeadroomLog) - sh[0];
    }
    fwd[0] = u;
    t = 1;
  }
  // one step at frame t with evidence e; false (yr kept) if the frame needs the rescue
#define NFHMM_FSTEP(t, e, ok)                                                               \
  {                                                                                         \
    float tot_;                                                                             \
    const float y_ = chain_apply<NR>(buf, p, coef, u, lane, N, sumlane, live, true, tot_); \
    const int k_ = __builtin_amdgcn_frexp_expf(tot_);                                      \
    ksum += k_;                                                                             \
    yr = ldexpf(y_, -k_);                                                                   \
    const float un_ = yr * (e);                                                             \
    ok = __ballot(live && un_ > kRescue) != 0;                                              \
    if (ok) {                                                                               \
      u = un_;                                                                              \
      fwd[(size_t)(t) * 64] = u;                                                            \
    }                                                                                       \
  }
  while (t < t1) {
    bool ok = true;
    if (t1 - t >= 2 * kFbBlock) {
      float ea[kFbBlock], eb[kFbBlock];
#pragma unroll
      for (int i = 0; i < kFbBlock; ++i) ea[i] = ev[(size_t)(t + i) * 64];
      while (ok && t1 - t >= 2 * kFbBlock) {
#pragma unroll
        for (int i = 0; i < kFbBlock; ++i) eb[i] = ev[(size_t)(t + kFbBlock + i) * 64];
#pragma unroll
        for (int i = 0; i < kFbBlock; ++i) {
          NFHMM_FSTEP(t, ea[i], ok);
          if (!ok) break;
          ++t;
        }
        if (!ok) break;
#pragma unroll
        for (int i = 0; i < kFbBlock; ++i) ea[i] = ev[(size_t)min(t + kFbBlock + i, t1 - 1) * 64];
#pragma unroll
        for (int i = 0; i < kFbBlock; ++i) {
          NFHMM_FSTEP(t, eb[i], ok);
          if (!ok) break;
          ++t;
        }
      }
    } else {
      const float e1 = ev[(size_t)t * 64];
      NFHMM_FSTEP(t, e1, ok);
      if (ok) ++t;
    }
    if (!ok) {   // frame t in log space with its own shift
      const float x = live ? logf(yr) + phi[(size_t)t * 64] : -INFINITY;
      const float mx = wave_max(x);
      u = (live && mx > -INFINITY) ? expf(x - mx + kEvHeadroomLog) : 0.0f;
      lam += (mx - kEvHeadroomLog) - sh[t];
      fwd[(size_t)t * 64] = u;
      ++t;
    }
  }
#undef NFHMM_FSTEP
  g = 0.69314718055994530942 * (double)ksum + (double)lam;
}

// Backward sweep over frames [t0, t1), from t1 - 1 down to t0.  For t1 == T it
// starts from b_{T-1} = 1; otherwise q is e_{t1} * b_{t1}, the evidence-weighted
// message of frame t1.  On return q = e_{t0} * b_{t0} (any positive scale).
template <int NR>
__device__ void bwd_sweep(const JobDesc &J, int s, const float (&coef)[NR], float *buf, int t0, int t1, float &q) {
  const int lane = threadIdx.x & 63, N = J.N, T = J.T;
  const bool sumlane = N < 64, live = lane < N;
  const gfloat *ev = gptr(J.ev + (size_t)s * T * 64 + lane);
  const gfloat *phi = gptr(J.phi + (size_t)s * T * 64 + lane);
  gfloat *bwd = gptr(J.bwd + (size_t)s * T * 64 + lane);
  int p = 0;
  float bb = 0.0f;
  int t = t1 - 1;
  if (t1 == T) {   // b_{T-1} = 1; q = e_{T-1} * b_{T-1}
    const float bcur = live ? 1.0f : 0.0f;
    bwd[(size_t)(T - 1) * 64] = bcur;
    q = bcur * ev[(size_t)(T - 1) * 64];
    if (__ballot(live && q > kRescue) == 0) {
      const float x = live ? phi[(size_t)(T - 1) * 64] : -INFINITY;
      const float mx = wave_max(x);
      q = (live && mx > -INFINITY) ? expf(x - mx + kEvHeadroomLog) : 0.0f;
    }
    t = T - 2;
  }
#define NFHMM_BSTEP(t, e, ok)                                                                \
  {                                                                                          \
    float tot_;                                                                              \
    const float y_ = chain_apply<NR>(buf, p, coef, q, lane, N, sumlane, live, false, tot_); \
    bb = ldexpf(y_, -__builtin_amdgcn_frexp_expf(tot_));                                    \
    bwd[(size_t)(t) * 64] = bb;                                                              \
    const float qn_ = bb * (e);                                                              \
    ok = __ballot(live && qn_ > kRescue) != 0;                                               \
    if (ok) q = qn_;                                                                         \
  }
  while (t >= t0) {
    bool ok = true;
    if (t - t0 + 1 >= 2 * kFbBlock) {
      float ea[kFbBlock], eb[kFbBlock];
#pragma unroll
      for (int i = 0; i < kFbBlock; ++i) ea[i] = ev[(size_t)(t - i) * 64];
      while (ok && t - t0 + 1 >= 2 * kFbBlock) {
#pragma unroll
        for (int i = 0; i < kFbBlock; ++i) eb[i] = ev[(size_t)(t - kFbBlock - i) * 64];
#pragma unroll
        for (int i = 0; i < kFbBlock; ++i) {
          NFHMM_BSTEP(t, ea[i], ok);
          if (!ok) break;
          --t;
        }
        if (!ok) break;
#pragma unroll
        for (int i = 0; i < kFbBlock; ++i) ea[i] = ev[(size_t)max(t - kFbBlock - i, t0) * 64];
#pragma unroll
        for (int i = 0; i < kFbBlock; ++i) {
          NFHMM_BSTEP(t, eb[i], ok);
          if (!ok) break;
          --t;
        }
      }
    } else {
      const float e1 = ev[(size_t)t * 64];
      NFHMM_BSTEP(t, e1, ok);
      if (ok) --t;
    }
    if (!ok) {   // q = b e underflows at frame t: that frame in log space
      const float x = live ? logf(bb) + phi[(size_t)t * 64] : -INFINITY;
      const float mx = wave_max(x);
      q = (live && mx > -INFINITY) ? expf(x - mx + kEvHeadroomLog) : 0.0f;
      --t;
    }
  }
#undef NFHMM_BSTEP
}

// Lane n's coefficients of the step operator (see chain_apply): column n of A
// forward (lane N: ones), row n of A backward (lane N: the column sums of A,
// formed by lane m for column m and then read across).
template <int NR>
__device__ __forceinline__ void chain_coef(const float *A, int N, int lane, bool fwd, float (&coef)[NR]) {
  const bool live = lane < N;
  if (fwd) {
#pragma unroll
    for (int m = 0; m < NR; ++m) coef[m] = (m < N && live) ? A[(size_t)m * N + lane] : ((m < N && lane == N) ? 1.0f : 0.0f);
  } else {
    float colsum = 0.0f;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      coef[i] = (i < N && live) ? A[(size_t)lane * N + i] : 0.0f;
      if (i < N && live) colsum += A[(size_t)i * N + lane];
    }
#pragma unroll
    for (int m = 0; m < NR; ++m) {
      const float cs = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(colsum), m));
      if (lane == N && m < N) coef[m] = cs;
    }
  }
}

// Boundary slots of chain s: [dir][slot][chunk][64] with slots 0/1 = round-1
// start/end and 2/3 = round-2 start/end; forward gains [round][chunk].
__device__ __forceinline__ float *bnd_of(const JobDesc &J, int s, int dir) {
  return J.bnd + ((size_t)s * 2 + dir) * 4 * (size_t)J.fbC * 64;
}
__device__ __forceinline__ void put_gain(float2 *gp, double g) {
  const float hi = (float)g;
  *gp = make_float2(hi, (float)(g - (double)hi));
}

// Rounds 1 and 2 of the chunked sweep: one wavefront per (job, source, direction,
// chunk).  In round 2 each chunk also decides, for the chunk after it in sweep
// order, whether that chunk's round-2 start agrees with this chunk's round-2 end
// (the same test the next chunk made to pick its start, then the agreement
// test), and records the verdict and the log factor between the two in bchk:
// the fix-up then only reads verdicts.
template <int NR>
__global__ __launch_bounds__(64) void k_fb_round(WorkList wl, int round) {
  const int b = blockIdx.x;
  const int jb = find_job(wl.start, wl.njobs, b);
  const JobDesc &J = wl.jobs[jb];
  const int C = J.fbC, L = J.fbL, T = J.T, N = J.N;
  const int local = b - wl.start[jb];
  const int s = local / (2 * C), rem = local - s * 2 * C;
  const int dir = rem / C, c = rem - dir * C;
  const int lane = threadIdx.x;
  const bool live = lane < N;
  const int t0 = c * L, t1 = min(T, t0 + L);
  float *bs = bnd_of(J, s, dir) + lane;
  float2 *gs = J.bgain + (size_t)s * 2 * C;
  const bool exact = dir == 0 ? c == 0 : c == C - 1;
  const int prev_c = dir == 0 ? c - 1 : c + 1, next_c = dir == 0 ? c + 1 : c - 1;
  float x;
  bool swept = true;
  if (round == 1) {
    if (dir == 0 && c == 0 && lane == 0) J.chainflag[s] = 0;
    x = live ? 0.5f : 0.0f;
  } else {
    const float in1 = bs[(size_t)c * 64];
    bool keep = exact;
    x = 0.0f;
    if (!exact) {
      x = bs[(size_t)(C + prev_c) * 64];   // the neighbour's round-1 end
      float lr;
      keep = msgs_agree(in1, x, live, lr);
    }
    if (keep) {
      x = bs[(size_t)(C + c) * 64];        // round-1 end stands
      bs[(size_t)(2 * C + c) * 64] = in1;
      bs[(size_t)(3 * C + c) * 64] = x;
      if (dir == 0 && lane == 0) gs[C + c] = gs[c];
      swept = false;
    }
  }
  if (swept) {
    const int slot = round == 1 ? 0 : 2;
    bs[(size_t)(slot * C + c) * 64] = x;
    __shared__ __attribute__((aligned(16))) float buf[2 * NR];
    float coef[NR];
    chain_coef<NR>(J.A_in + (size_t)s * N * N, N, lane, dir == 0, coef);
    double g = 0.0;
    if (dir == 0) fwd_sweep<NR>(J, s, coef, buf, t0, t1, x, g);
    else bwd_sweep<NR>(J, s, coef, buf, t0, t1, x);
    const int k = canon_msg(x, live);
    bs[(size_t)((slot + 1) * C + c) * 64] = x;
    if (dir == 0 && lane == 0) put_gain(gs + (round - 1) * C + c, g + 0.69314718055994530942 * (double)k);
  }
  if (round == 2 && next_c >= 0 && next_c < C) {
    // the next chunk's round-2 start: its round-1 start if that agreed with our
    // round-1 end, else our round-1 end
    const float in1n = bs[(size_t)next_c * 64], out1 = bs[(size_t)(C + c) * 64];
    float lr;
    const float in2n = msgs_agree(in1n, out1, live, lr) ? in1n : out1;
    const bool ok = msgs_agree(in2n, x, live, lr);
    if (lane == 0) J.bchk[((size_t)s * 2 + dir) * C + next_c] = make_float2(ok ? 1.0f : 0.0f, lr);
  }
}

// Fix-up of the chunked sweep: one wavefront per (job, source, direction).  The
// verdicts of round 2 are read 64 chunks at a time to find the first chunk (in
// sweep order) whose start disagrees with the end before it, summing the forward
// gains up to there; from that chunk on, the chunks are walked in order and swept
// again wherever the start differs from the final end before them.  The forward
// wavefront also forms lnz.
template <int NR>
__global__ __launch_bounds__(64) void k_fb_fixup(WorkList wl) {
  const int b = blockIdx.x;
  const int jb = find_job(wl.start, wl.njobs, b);
  const JobDesc &J = wl.jobs[jb];
  const int C = J.fbC, L = J.fbL, T = J.T, N = J.N;
  const int local = b - wl.start[jb];
  const int s = local >> 1, dir = local & 1;
  const int lane = threadIdx.x;
  const bool live = lane < N;
  const float *bs = bnd_of(J, s, dir) + lane;
  const float2 *gs = J.bgain + (size_t)s * 2 * C + C;   // round-2 gains
  const float2 *chk = J.bchk + ((size_t)s * 2 + dir) * C;
  const float *in2 = bs + (size_t)2 * C * 64, *out2 = bs + (size_t)3 * C * 64;
  // pass 1: first chunk (in sweep order, from 1) whose start disagrees
  Comp tot = comp_zero();
  int first = C;
  for (int i0 = 1; i0 < C; i0 += 64) {
    const int i = i0 + lane;
    const bool in = i < C;
    const int c = dir == 0 ? i : C - 1 - i;
    const float2 v = in ? chk[c] : make_float2(1.0f, 0.0f);
    const float2 g = (in && dir == 0) ? gs[c] : make_float2(0.0f, 0.0f);
    const uint64_t bad = __ballot(in && v.x == 0.0f);
    const int l0 = bad ? __builtin_ctzll(bad) : 64;
    Comp part = comp_zero();
    if (in && lane < l0) {
      comp_add(part, g.x);
      comp_add(part, g.y);
      comp_add(part, v.y);
    }
    tot = comp_merge(tot, wave_comp(part));
    if (bad) { first = i0 + l0; break; }
  }
  float prev;
  if (first == C) {
    prev = out2[(size_t)(dir == 0 ? C - 1 : 0) * 64];
  } else {
    // pass 2: walk from the first disagreement
    __shared__ __attribute__((aligned(16))) float buf[2 * NR];
    float coef[NR];
    chain_coef<NR>(J.A_in + (size_t)s * N * N, N, lane, dir == 0, coef);
    const int cb = dir == 0 ? first - 1 : C - first;   // chunk before the first disagreement
    prev = out2[(size_t)cb * 64];
    for (int i = first; i < C; ++i) {
      const int c = dir == 0 ? i : C - 1 - i;
      const float a = in2[(size_t)c * 64];
      float lr;
      if (i > first && msgs_agree(a, prev, live, lr)) {
        prev = out2[(size_t)c * 64];
        if (dir == 0) {
          comp_add(tot, gs[c].x);
          comp_add(tot, gs[c].y);
          comp_add(tot, lr);
        }
        continue;
      }
      const int t0 = c * L, t1 = min(T, t0 + L);
      float x = prev;
      double g = 0.0;
      if (dir == 0) fwd_sweep<NR>(J, s, coef, buf, t0, t1, x, g);
      else bwd_sweep<NR>(J, s, coef, buf, t0, t1, x);
      g += 0.69314718055994530942 * (double)canon_msg(x, live);
      const float gh = (float)g;
      comp_add(tot, gh);
      comp_add(tot, (float)(g - (double)gh));
      prev = x;
    }
  }
  if (dir == 0) {
    const float2 g0 = gs[0];
    const float last = wave_sum(live ? prev : 0.0f);
    if (lane == 0) {
      const double z = (double)tot.hi + (double)tot.lo + (double)g0.x + (double)g0.y + log((double)last);
      const float hi = (float)z;
      J.lnz[s] = make_float2(hi, (float)(z - (double)hi));
    }
  }
}

// d-hat of every (job, source, frame) from the scaled messages: one wavefront per
// (source, frame), four per block.  A chain is flagged for the exact log-space
// pass when at some frame the best forward x backward product falls more than
// 40 nats below (best forward) x (best backward), or is not finite: only then can
// states flushed by the scaled recursion carry posterior mass.
constexpr float kAgreeNats = 40.0f;

__global__ __launch_bounds__(256) void k_posterior(WorkList wl) {
  const int b = blockIdx.x;
  const int jb = find_job(wl.start, wl.njobs, b);
  const JobDesc &J = wl.jobs[jb];
  const int local = b - wl.start[jb];
  const int groups = (J.T + 3) >> 2;
  const int s = local / groups;
  const int t = (local - s * groups) * 4 + (threadIdx.x >> 6);
  if (t >= J.T) return;
  const int lane = threadIdx.x & 63;
  const bool live = lane < J.N;
  const size_t o = ((size_t)s * J.T + t) * 64 + lane;
  const float lf = live ? logf(J.fwd[o]) : -INFINITY;
  const float lb = live ? logf(J.bwd[o]) : -INFINITY;
  const float x = lf + lb;
  const float mx = wave_max(x);
  const float e = live ? expf(x - mx) : 0.0f;
  const float d = e / wave_sum(e);
  if (live) J.post[((size_t)s * J.T + t) * J.N + lane] = d;
  const float agree = mx - wave_max(lf) - wave_max(lb);
  if (lane == 0 && !(agree >= -kAgreeNats)) atomicOr(J.chainflag + s, 1);
}

// Exact log-space forward-backward of a flagged chain (one wavefront per chain;
// returns at once for unflagged chains).  Each lane n evaluates
//   l_t(n) = gamma*phi_t(n) + lse_m( la_{t-1}(m) + ln A[m][n] )
// with its own maximum, so no value is flushed; messages are kept log-normalised
// and the increments of ln Z go to sh (with nrm = 1).  The backward sweep then
// forms d-hat = exp(la + lb - lse(la + lb)) directly.
template <int NR>
__global__ __launch_bounds__(64) void k_chain_exact(WorkList wl) {
  const int b = blockIdx.x;
  const int jb = find_job(wl.start, wl.njobs, b);
  const JobDesc &J = wl.jobs[jb];
  const int s = b - wl.start[jb];
  if (J.chainflag[s] == 0) return;
  const int lane = threadIdx.x;
  const int N = J.N, T = J.T;
  const bool live = lane < N;
  const float *A = J.A_in + (size_t)s * N * N;
  const float *phi = J.phi + (size_t)s * T * 64;
  float *la = J.fwd + (size_t)s * T * 64;     // log forward messages (overwrites the scaled ones)
  float *sh = J.sh + (size_t)s * T;
  __shared__ float buf[NR];
  float lac[NR];
  // forward: column n of ln A
#pragma unroll
  for (int m = 0; m < NR; ++m) lac[m] = (live && m < N) ? logf(A[(size_t)m * N + lane]) : -INFINITY;
  const float *pi = J.pi_in + (size_t)s * N;
  float cur = live ? logf(pi[lane]) + phi[lane] : -INFINITY;
  auto lse_lanes = [&](float x) -> float {
    const float mx = wave_max(x);
    if (!(mx > -INFINITY)) return mx;
    return mx + logf(wave_sum(live ? expf(x - mx) : 0.0f));
  };
  float c = lse_lanes(cur);
  cur = live ? cur - c : -INFINITY;
  la[lane] = cur;
  Comp lz = comp_zero();              // ln Z = sum_t c_t; the shifts sh are cleared
  comp_add(lz, c);
  if (lane == 0) sh[0] = 0.0f;
  for (int t = 1; t < T; ++t) {
    if (lane < NR) buf[lane] = cur;
    __syncthreads();
    float mx = -INFINITY;
#pragma unroll
    for (int m = 0; m < NR; ++m) mx = fmaxf(mx, buf[m] + lac[m]);
    float acc = 0.0f;
    if (mx > -INFINITY) {
#pragma unroll
      for (int m = 0; m < NR; ++m) acc += expf(buf[m] + lac[m] - mx);
    }
    __syncthreads();
    const float l = (live && mx > -INFINITY) ? phi[(size_t)t * 64 + lane] + mx + logf(acc) : -INFINITY;
    c = lse_lanes(l);
    cur = live ? l - c : -INFINITY;
    la[(size_t)t * 64 + lane] = cur;
    comp_add(lz, c);
    if (lane == 0) sh[t] = 0.0f;
  }
  if (lane == 0) J.lnz[s] = make_float2(lz.hi, lz.lo);
  // backward with row m of ln A in lane m; d-hat on the way
#pragma unroll
  for (int n = 0; n < NR; ++n) lac[n] = (live && n < N) ? logf(A[(size_t)lane * N + n]) : -INFINITY;
  float lb = live ? 0.0f : -INFINITY;
  for (int t = T - 1; t >= 0; --t) {
    if (t < T - 1) {
      const float w = live ? lb + phi[(size_t)(t + 1) * 64 + lane] : -INFINITY;
      if (lane < NR) buf[lane] = w;
      __syncthreads();
      float mx = -INFINITY;
#pragma unroll
      for (int n = 0; n < NR; ++n) mx = fmaxf(mx, buf[n] + lac[n]);
      float acc = 0.0f;
      if (mx > -INFINITY) {
#pragma unroll
        for (int n = 0; n < NR; ++n) acc += expf(buf[n] + lac[n] - mx);
      }
      __syncthreads();
      const float l = (live && mx > -INFINITY) ? mx + logf(acc) : -INFINITY;
      const float cb = lse_lanes(l);
      lb = (live && cb > -INFINITY) ? l - cb : -INFINITY;
    }
    const float x = live ? la[(size_t)t * 64 + lane] + lb : -INFINITY;
    const float z = lse_lanes(x);
    if (live) J.post[((size_t)s * T + t) * N + lane] = expf(x - z);
  }
}

// ------------------------------------------------------------------ Eq. 6 + Eq. 7/8 inputs
// One wavefront per (job, frame), kUpdWaves(Mp) frames of one job per block; no
// block-level synchronisation (LDS holds each wave's own rows).  Modes:
//   kUpdMessages: alpha = c + gamma B'd + 1 with this iteration's d-hat, and the
//                 frame's bound contribution for iteration (round - start);
//   kUpdUniform:  the default start: alpha = c + gamma/N + 1 (c computed with w = 1);
//   kUpdFromAlpha: alpha read from alpha_init ([T][M], warm start / resume).
// Then, in every mode: alpha_0, w = exp(psi(alpha) - psi(alpha_0)), gamma*phi
// (Eq. 8, up to a per-frame constant) with its shifted exponential for the next
// chain pass, and the Lambda rows of the tail bins.  alpha itself is stored only
// when it is an output (the job's last iteration, or a start with no iterations):
// it is c + gamma B'd + 1 and nothing else reads it but the reconstruction.
//
// Two forms of the element passes.  The streamed form (any size) walks the row
// in chunks of 64 x kUpdU elements.  The resident form (rows of at most 1024
// elements and at most one tail bin: every paper-sized job) issues every load of
// the frame -- its row of c (or of alpha_init), the tail bin's dictionary row,
// that bin's count, the frame's d-hat and bound partials -- before anything else,
// keeps alpha in registers (four float4 per lane, elements 256 j + 4 lane + e),
// and stores nothing before its last load has been consumed: global loads and
// stores share one counter on gfx9, so a load issued after a store would also
// wait for that store.  The two forms sum the tail bins' Lambda in different
// orders, so a job takes the same form for all its updates (a resumed fit then
// repeats the uninterrupted one bit for bit).
__device__ __forceinline__ void lds_order() { __asm__ volatile("" ::: "memory"); }

constexpr int kUpdU = 4;   // elements per lane whose loads are issued together (streamed form)
constexpr int kMaxTail = 4;   // tail bins handled here (F mod 64 <= 4)
constexpr int kUpdResident = 1024;   // largest Mp of the resident form

// What the update needs besides the element rows: the contraction-side partials
// of the bound, the chain's part, and d-hat of every source at frame t in sD.
struct UpdPre {
  vf2 vtail;   // tail part of sum V ln Lambda (previous call)
  Comp pv;     // contraction-side parts of the bound
  Comp chain;  // ln Z parts and -sum_n d (gamma phi)
};

__device__ __forceinline__ UpdPre update_prelude(const JobDesc &J, int t, int lane, float *sD, bool msg) {
  const int S = J.S, N = J.N, Mp = J.Mp, T = J.T, Ft = J.Ft, nsl = J.nsl;
  const gfloat *post_in = gptr(J.post), *phi_in = gptr(J.phi), *sh_in = gptr(J.sh);
  const gfloat2 *lnz = gptr(J.lnz), *clw = gptr(J.clw), *vll = gptr(J.vll);
  gfloat *post = gptr(J.post);
  const bool live = lane < N;
  UpdPre u;
  u.vtail = vf2{0.0f, 0.0f};
  u.pv = comp_zero();
  u.chain = comp_zero();
  if (msg) {
    if (Ft > 0) u.vtail = vll[(size_t)nsl * T + t];
    const int nkt = (Mp + kBoundRows - 1) / kBoundRows;
    for (int r = lane; r < nsl; r += 64) {
      const vf2 v = vll[(size_t)r * T + t];
      Comp d; d.hi = v.x; d.lo = v.y;
      u.pv = comp_merge(u.pv, d);
    }
    for (int r = lane; r < nkt; r += 64) {
      const vf2 v = clw[(size_t)r * T + t];
      Comp d; d.hi = v.x; d.lo = v.y;
      u.pv = comp_merge(u.pv, d);
    }
    const int nl = live ? lane : 0;
    float dv[kMaxSources], pf[kMaxSources], shv[kMaxSources];
#pragma unroll
    for (int s = 0; s < kMaxSources; ++s) {
      const int ss = s < S ? s : 0;
      dv[s] = post_in[((size_t)ss * T + t) * N + nl];
      pf[s] = phi_in[((size_t)ss * T + t) * 64 + nl];
      shv[s] = sh_in[(size_t)ss * T + t];
    }
    // d-hat of every source at frame t, -sum_n d (gamma phi) and ln Z's part
    Comp cc = comp_zero();
#pragma unroll
    for (int s = 0; s < kMaxSources; ++s) {
      if (s < S) {
        if (live) {
          sD[s * N + lane] = dv[s];
          comp_add(cc, -dv[s] * pf[s]);
        }
        comp_add(u.chain, shv[s]);
      }
    }
    u.chain = comp_merge(u.chain, wave_comp(cc));
    if (t == 0) {
      for (int s = 0; s < S; ++s) {
        const vf2 z = lnz[s];
        comp_add(u.chain, z.x);
        comp_add(u.chain, z.y);
      }
    }
  } else {
    for (int i = lane; i < S * N; i += 64) {
      sD[i] = 1.0f / (float)N;
      post[((size_t)(i / N) * T + t) * N + (i % N)] = 1.0f / (float)N;
    }
  }
  lds_order();
  return u;
}

// One element of the second pass: psi(alpha) into sE (for Eq. 8), w, and the
// bound's lnG(alpha).  alpha >= 1 (Eq. 6) for every element in a c-based mode.
struct ElemOut {
  float w, ps;
};
__device__ __forceinline__ ElemOut update_elem(float a, bool in, float inv_xs0, float rest0, bool want_lg, double &lg) {
  // straight-line code, results selected at the end: a branch around the
  // exponential or lnG would split the element's computation and keep its
  // temporaries live across the branch
  const Shift8 z = shift8(in ? a : 1.0f);
  const float rest = psi_rest(z);
  const float lxs = fast_ln(z.xs);
  const float w = (z.xs * inv_xs0) * fast_exp(rest - rest0);
  const float l = lgamma_from_ge1(z, lxs);
  ElemOut o;
  o.ps = in ? lxs + rest : 0.0f;
  o.w = in ? w : 0.0f;
  lg += (want_lg && in) ? (double)l : 0.0;
  return o;
}

// The tail bins' R and V ln Lambda, Eq. 8 up to a per-frame constant, and the
// frame's bound contribution.
template <bool kBF16>
__device__ __forceinline__ void update_finish(const JobDesc &J, int t, int lane, const float *sE, bool msg, int it,
                                              const float (&tacc)[kMaxTail], const float (&vt)[kMaxTail], double lg,
                                              const Shift8 &z0, const UpdPre &u) {
  const int S = J.S, N = J.N, K = J.K, T = J.T, Fp = J.Fp, Fm = J.Fm, Ft = J.Ft, nsl = J.nsl;
  const float gamma = J.gamma;
  gfloat2 *vll = gptr(J.vll), *elbo = gptr(J.elbo);
  gfloat *Rout = gptr(J.R), *phi = gptr(J.phi), *ev = gptr(J.ev), *sh = gptr(J.sh);
  gu16 *Rh = gptr(J.Rh);
  const bool live = lane < N;

  // ---- tail bins of the next contraction: R = V / Lambda, and their V ln Lambda
  Comp vl = comp_zero();
#pragma unroll
  for (int jt = 0; jt < kMaxTail; ++jt) {
    if (jt < Ft) {
      const float lam = wave_sum(tacc[jt]);
      const int l = Fm + jt;
      const float v = vt[jt];
      const float rr = v > 0.0f ? v / lam : 0.0f;
      if (v > 0.0f) comp_add(vl, v * ln_pos(lam));
      if (lane == 0) {
        if constexpr (kBF16) Rh[(size_t)t * Fp + l] = f2bf(rr);
        else Rout[(size_t)t * Fp + l] = rr;
      }
    }
  }

  // ---- Eq. 8 up to a per-frame constant: gamma * sum_j psi(alpha_(s,n,j)).  The
  //      term -gamma K psi(alpha_0) is the same for every state of the frame and
  //      changes neither the chain posterior nor the bound, so it is left out.
  for (int s = 0; s < S; ++s) {
    float x = -INFINITY;
    if (live) {
      float acc = 0.0f;
      const float *seg = sE + (s * N + lane) * K;
      for (int j = 0; j < K; ++j) acc += seg[j];
      x = gamma * acc;
    }
    const float mx = wave_max(x);
    const size_t o = ((size_t)s * T + t) * 64 + lane;
    phi[o] = live ? x : 0.0f;
    ev[o] = live ? expf(x - mx + kEvHeadroomLog) : 0.0f;
    if (lane == 0) sh[(size_t)s * T + t] = mx - kEvHeadroomLog;
  }

  // ---- bound contribution of frame t:
  //   sum_k lnG(alpha_k) - lnG(alpha_0) + sum V ln Lambda - sum c ln w
  //   + sum_s (ln Z_s part - sum_n d (gamma phi))
  if (msg) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) lg += __shfl_xor(lg, o);
    Comp tot;
    tot.hi = (float)lg;
    tot.lo = (float)(lg - (double)tot.hi);
    tot = comp_merge(tot, wave_comp(u.pv));
    comp_add(tot, -lgamma_from_ge1(z0, fast_ln(z0.xs)));
    tot = comp_merge(tot, u.chain);
    comp_add(tot, u.vtail.x);
    comp_add(tot, u.vtail.y);
    if (lane == 0) elbo[(size_t)it * T + t] = vf2{tot.hi, tot.lo};
  }
  if (lane == 0 && Ft > 0) vll[(size_t)nsl * T + t] = vf2{vl.hi, vl.lo};
}

__device__ __forceinline__ double wave_sum_f64(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

// Streamed form: any Mp, any mode.
template <bool kBF16>
__device__ __forceinline__ void update_frame(const JobDesc &J, int t, int lane, float *sE, int mode, int round) {
  const int S = J.S, N = J.N, K = J.K, M = J.M, Mp = J.Mp, T = J.T, Fp = J.Fp;
  const int Fm = J.Fm, Ft = J.Ft;
  const int it = round - J.start_round, iters = J.iters;
  const float gamma = J.gamma;
  const gfloat *c = gptr(J.c), *alpha_init = gptr(J.alpha_init), *Vin = gptr(J.V);
  const gfloat *Wfm = gptr(J.Wfm);
  const gu16 *Wfm_h = gptr(J.Wfm_h);
  gfloat *alpha = gptr(J.alpha), *wout = gptr(J.w);
  gu16 *wh = gptr(J.wh);

  float *sD = sE + Mp;
  const size_t row = (size_t)t * Mp;
  const bool msg = mode == kUpdMessages;
  const bool store_alpha = msg ? (it == iters - 1) : (iters == 0);
  const UpdPre u = update_prelude(J, t, lane, sD, msg);

  // ---- Eq. 6; element k belongs to state g = k / K (kept incrementally).  Loads
  //      past the end read the last element (in bounds) and are not used.
  // alpha_0: per-lane sums in double, then a butterfly over the lanes, which
  // leaves the same value in every lane.  Every term is a float >= 1 and the sum
  // stays far below 2^53 ulps of the smallest, so the double sum is exact and
  // does not depend on the order.  Sub-chunks of 64 elements past Mp are skipped
  // (a uniform test).
  double asum = 0.0;
  {
    const int step_g = 64 / K, step_r = 64 % K;
    int g = lane / K, r = lane - (lane / K) * K;
    const bool from_alpha = mode == kUpdFromAlpha;
    for (int base = 0; base < Mp; base += 64 * kUpdU) {
      float cv[kUpdU];
#pragma unroll
      for (int u = 0; u < kUpdU; ++u) {
        if (base + 64 * u >= Mp) break;
        const int k = min(base + 64 * u + lane, M - 1);
        cv[u] = from_alpha ? alpha_init[(size_t)t * M + k] : c[row + k];
      }
#pragma unroll
      for (int u = 0; u < kUpdU; ++u) {
        if (base + 64 * u >= Mp) break;
        const int k = base + 64 * u + lane;
        float a = from_alpha ? cv[u] : cv[u] + gamma * sD[min(g, S * N - 1)] + 1.0f;
        a = k < M ? a : 0.0f;
        asum += (double)a;
        if (k < Mp) sE[k] = a;   // Mp is a multiple of 32: the last sub-chunk may be half full
        g += step_g;
        r += step_r;
        if (r >= K) { r -= K; ++g; }
      }
    }
  }
  asum = wave_sum_f64(asum);
  const float a0 = (float)asum;
  const Shift8 z0 = shift8(a0);
  const float rest0 = psi_rest(z0);
  const float inv_xs0 = 1.0f / z0.xs;
  lds_order();

  // ---- w = exp(psi(alpha) - psi(alpha_0)) = (xs / xs0) exp(rest - rest0);
  //      sE keeps psi(alpha_k) for Eq. 8; sum_k lnG(alpha_k) for the bound;
  //      tail bins: Lambda[l][t] = sum_k beta[l][k] w_k for the next contraction
  double lg = 0.0;
  float tacc[kMaxTail] = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int base = 0; base < Mp; base += 64 * kUpdU) {
    float tw[kMaxTail][kUpdU];
#pragma unroll
    for (int jt = 0; jt < kMaxTail; ++jt) {
      if (jt < Ft) {
#pragma unroll
        for (int u = 0; u < kUpdU; ++u) {
          if (base + 64 * u >= Mp) break;
          const size_t o = (size_t)(Fm + jt) * Mp + min(base + 64 * u + lane, M - 1);
          tw[jt][u] = kBF16 ? bf2f(Wfm_h[o]) : Wfm[o];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kUpdU; ++u) {
      if (base + 64 * u >= Mp) break;
      const int k = base + 64 * u + lane;
      const bool in = k < M;
      const float a = in ? sE[k] : 1.0f;
      ElemOut e = update_elem(a, in, inv_xs0, rest0, msg, lg);
      if (store_alpha && in) alpha[row + k] = a;
      if (k < Mp) {
        sE[k] = e.ps;
        if constexpr (kBF16) {
          const uint16_t h = f2bf(e.w);
          wh[row + k] = h;
          e.w = bf2f(h);
        } else {
          wout[row + k] = e.w;
        }
      }
#pragma unroll
      for (int jt = 0; jt < kMaxTail; ++jt)
        if (jt < Ft) tacc[jt] = fmaf(tw[jt][u], e.w, tacc[jt]);
    }
  }
  lds_order();
  float vt[kMaxTail];
#pragma unroll
  for (int jt = 0; jt < kMaxTail; ++jt) vt[jt] = jt < Ft ? Vin[(size_t)t * Fp + Fm + jt] : 0.0f;
  update_finish<kBF16>(J, t, lane, sE, msg, it, tacc, vt, lg, z0, u);
}

// Resident form: Mp <= kUpdResident, Ft <= 1, any mode.
// Every load is issued unconditionally or under a lane mask, with no use inside
// the masked region, so that the compiler places no wait before the last one.
template <bool kBF16>
__device__ __forceinline__ void update_frame_resident(const JobDesc &J, int t, int lane, float *sE, int mode,
                                                      int round) {
  const int S = J.S, N = J.N, K = J.K, M = J.M, Mp = J.Mp, T = J.T, Fp = J.Fp, Fm = J.Fm, Ft = J.Ft;
  const int nsl = J.nsl;
  const int it = round - J.start_round, iters = J.iters;
  const float gamma = J.gamma;
  const gfloat *c = gptr(J.c), *Vin = gptr(J.V), *Wfm = gptr(J.Wfm), *alpha_init = gptr(J.alpha_init);
  const gfloat *post_in = gptr(J.post), *phi_in = gptr(J.phi), *sh_in = gptr(J.sh);
  const gfloat2 *lnz = gptr(J.lnz), *clw = gptr(J.clw), *vll = gptr(J.vll);
  const gu16 *Wfm_h = gptr(J.Wfm_h);
  gfloat *alpha = gptr(J.alpha), *wout = gptr(J.w), *post = gptr(J.post);
  gu16 *wh = gptr(J.wh);
  float *sD = sE + Mp;
  const size_t row = (size_t)t * Mp;
  const bool msg = mode == kUpdMessages, from_alpha = mode == kUpdFromAlpha;
  const bool store_alpha = msg ? (it == iters - 1) : (iters == 0);
  const bool live = lane < N;
  const int k0 = 4 * lane;

  // ---- every load first: the row of c and the tail bin's row of beta (chunks
  //      past Mp read the row's last chunk and are masked out below), the tail
  //      bin's count, and the frame's d-hat, chain terms and bound partials
  vf4 cv[4];
  vf4 twf[4];
  vu2 twh[4];
  const size_t trow = (size_t)(Ft > 0 ? Fm : 0) * Mp;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int kk = min(256 * j + k0, Mp - 4);
    if (from_alpha) {   // [T][M] rows: not 16-byte aligned in general
#pragma unroll
      for (int e = 0; e < 4; ++e) cv[j][e] = alpha_init[(size_t)t * M + min(256 * j + k0 + e, M - 1)];
    } else {
      cv[j] = *(const gfloat4 *)(c + row + kk);
    }
    if constexpr (kBF16) twh[j] = *(const guint2 *)(Wfm_h + trow + kk);
    else twf[j] = *(const gfloat4 *)(Wfm + trow + kk);
  }
  const float vt0 = Vin[(size_t)t * Fp + (Ft > 0 ? Fm : 0)];
  // (source, state) pair i = s N + n in lane i % 64 of slot i / 64; two slots
  // cover S N <= 128 and are loaded here, any others in a loop below
  const int SN = S * N;
  float dq[2] = {0.0f, 0.0f}, fq[2] = {0.0f, 0.0f}, shl = 0.0f;
  vf2 vtail = vf2{0.0f, 0.0f}, pv_sl = vf2{0.0f, 0.0f}, pv_kt = vf2{0.0f, 0.0f}, z_s = vf2{0.0f, 0.0f};
  const int nkt = (Mp + kBoundRows - 1) / kBoundRows;   // <= 64 here
  if (msg) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int i = min(lane + 64 * q, SN - 1), s = i / N, n = i - s * N;
      dq[q] = post_in[((size_t)s * T + t) * N + n];
      fq[q] = phi_in[((size_t)s * T + t) * 64 + n];
    }
    shl = sh_in[(size_t)min(lane, S - 1) * T + t];
    // clamped, unconditional loads, masked after use-free: a load under a lane
    // mask whose result needs a copy makes the compiler wait inside the mask
    vtail = vll[(size_t)(Ft > 0 ? nsl : 0) * T + t];
    pv_sl = vll[(size_t)min(lane, nsl - 1) * T + t];
    pv_kt = clw[(size_t)min(lane, nkt - 1) * T + t];
    z_s = lnz[min(lane, S - 1)];
  }

  // ---- d-hat into LDS (uniform start: 1/N, which is also the posterior output)
  Comp chain = comp_zero(), pv = comp_zero();
  if (msg) {
    Comp cc = comp_zero();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (lane + 64 * q < SN) {
        sD[lane + 64 * q] = dq[q];
        comp_add(cc, -dq[q] * fq[q]);
      }
    }
    for (int i = lane + 128; i < SN; i += 64) {   // more than 128 (source, state) pairs
      const int s = i / N, n = i - s * N;
      const float dv = post_in[((size_t)s * T + t) * N + n];
      sD[i] = dv;
      comp_add(cc, -dv * phi_in[((size_t)s * T + t) * 64 + n]);
    }
    if (lane < S) comp_add(cc, shl);
    chain = wave_comp(cc);
    Comp d;
    d.hi = lane < nsl ? pv_sl.x : 0.0f; d.lo = lane < nsl ? pv_sl.y : 0.0f; pv = comp_merge(pv, d);
    d.hi = lane < nkt ? pv_kt.x : 0.0f; d.lo = lane < nkt ? pv_kt.y : 0.0f; pv = comp_merge(pv, d);
    for (int r = lane + 64; r < nsl; r += 64) {   // only for more than 4096 bins
      const vf2 v = vll[(size_t)r * T + t];
      d.hi = v.x; d.lo = v.y;
      pv = comp_merge(pv, d);
    }
    if (t == 0) {
      for (int s = 0; s < S; ++s) {
        const float zx = __shfl(z_s.x, s), zy = __shfl(z_s.y, s);
        comp_add(chain, zx);
        comp_add(chain, zy);
      }
    }
  } else {
    for (int i = lane; i < S * N; i += 64) sD[i] = 1.0f / (float)N;
  }
  lds_order();

  // ---- Eq. 6 in registers; alpha_0 as the exact double sum
  const int step_g = 256 / K, step_r = 256 % K;
  int g0 = k0 / K, r0 = k0 - (k0 / K) * K;   // state and position of element 256 j + k0
  double asum = 0.0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    int g = g0, r = r0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = 256 * j + k0 + e;
      float a = from_alpha ? cv[j][e] : cv[j][e] + gamma * sD[min(g, S * N - 1)] + 1.0f;
      a = k < M ? a : 0.0f;
      cv[j][e] = a;
      asum += (double)a;
      if (++r == K) { r = 0; ++g; }
    }
    g0 += step_g;
    r0 += step_r;
    if (r0 >= K) { r0 -= K; ++g0; }
  }
  asum = wave_sum_f64(asum);
  const float a0 = (float)asum;
  const Shift8 z0 = shift8(a0);
  const float rest0 = psi_rest(z0);
  const float inv_xs0 = 1.0f / z0.xs;

  // ---- w, psi, lnG, and the stores (no global load follows them)
  if (!msg) {
    for (int i = lane; i < S * N; i += 64) post[((size_t)(i / N) * T + t) * N + (i % N)] = 1.0f / (float)N;
  }
  double lg = 0.0;
  float tacc[kMaxTail] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int kj = 256 * j + k0;
    vf4 tw;
    if constexpr (kBF16)
      tw = vf4{__uint_as_float(twh[j].x << 16), __uint_as_float(twh[j].x & 0xffff0000u),
               __uint_as_float(twh[j].y << 16), __uint_as_float(twh[j].y & 0xffff0000u)};
    else
      tw = twf[j];
    vf4 ps, wv;
    uint32_t hw[2] = {0u, 0u};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      ElemOut o = update_elem(cv[j][e], kj + e < M, inv_xs0, rest0, msg, lg);
      if constexpr (kBF16) {
        const uint16_t h = f2bf(o.w);
        hw[e >> 1] |= (uint32_t)h << (16 * (e & 1));
        o.w = bf2f(h);
      }
      wv[e] = o.w;
      ps[e] = o.ps;
      tacc[0] = fmaf(tw[e], o.w, tacc[0]);
    }
    if (kj < Mp) {
      *(vf4 *)(sE + kj) = ps;
      if (store_alpha) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (kj + e < M) alpha[row + kj + e] = cv[j][e];
      }
      if constexpr (kBF16) *(guint2 *)(wh + row + kj) = vu2{hw[0], hw[1]};
      else *(gfloat4 *)(wout + row + kj) = wv;
    }
    // one chunk of four elements at a time: the sums are pinned here, else the
    // compiler sinks their additions to the end and holds all sixteen terms
    __asm__ volatile("" : "+v"(lg), "+v"(tacc[0]));
  }
  lds_order();
  UpdPre u;
  u.vtail = Ft > 0 ? vtail : vf2{0.0f, 0.0f};
  u.pv = pv;
  u.chain = chain;
  const float vt[kMaxTail] = {vt0, 0.0f, 0.0f, 0.0f};
  update_finish<kBF16>(J, t, lane, sE, msg, it, tacc, vt, lg, z0, u);
}

// Five wavefronts per SIMD: the resident form needs 98 registers, which would
// allow four; held to 96 it spills a few values once per frame.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_update(WorkList wl, int mode,
                                                                                         int round, int stride) {
  extern __shared__ float smem[];   // per wave: [Mp] alpha, then psi(alpha); then [S N] d-hat
  const int b = blockIdx.x;
  const int jb = find_job(wl.start, wl.njobs, b);
  const JobDesc &J = wl.jobs[jb];
  const int wpb = blockDim.x >> 6;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int t = (b - wl.start[jb]) * wpb + wave;
  const bool bf16 = J.bf16;
  if (t >= J.T) return;
  float *sE = smem + (size_t)wave * stride;
  const bool resident = J.Mp <= kUpdResident && J.Ft <= 1;
  if (resident) {
    if (bf16) update_frame_resident<true>(J, t, lane, sE, mode, round);
    else update_frame_resident<false>(J, t, lane, sE, mode, round);
  } else {
    if (bf16) update_frame<true>(J, t, lane, sE, mode, round);
    else update_frame<false>(J, t, lane, sE, mode, round);
  }
}

// ------------------------------------------------------------------ Section 4
// Vhat^(s) = beta_s E[theta]_s with E[theta_t] = alpha_t / alpha_t0 (Section 4),
// computed as alpha_t0 Vhat^(s): the product with alpha-hat itself.  The common
// factor alpha_t0 of a frame's column cancels in the ratio mask, the only use of
// Vhat.  Rows l, columns t, k over source s's elements.  Work: per job S * nlt *
// ceil(T/64) tiles.
__global__ __launch_bounds__(256) void k_reconstruct(WorkList wl) {
  const int b = xcd_remap(blockIdx.x, wl.total);
  const int jb = find_job(wl.start, wl.njobs, b);
  const JobDesc &J = wl.jobs[jb];
  int tile = b - wl.start[jb];
  const int nct = (J.T + 63) / 64;
  const int per_s = J.nlt * nct;
  const int s = tile / per_s;
  tile -= s * per_s;
  const int rt = tile % J.nlt, ct = tile / J.nlt;
  const int row0 = rt * 64, col0 = ct * 64;
  const int kb = s * J.NK, ke = kb + J.NK;
  floatx4 acc[2][2];
  gemm_nt_f32_dma_kmask<2, 2>(J.Wfm, J.Mp, J.Fp, row0, J.alpha, J.Mp, J.T, col0, kb, ke, acc);
  const Frag f = frag_of(threadIdx.x);
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int t = col0 + f.wc * 32 + j * 16 + f.lr;
    if (t >= J.T) continue;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int l = row0 + f.wr * 32 + i * 16 + 4 * f.lq;
      if (l >= J.Fp) continue;
      *(float4 *)(J.sep + ((size_t)s * J.T + t) * J.Fp + l) =
          make_float4(acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]);
    }
  }
}

// Ratio mask V* = V Vhat^(s) / sum_s' Vhat^(s') and export of every output in the
// ABI layouts.  One block per (job, frame).
__global__ __launch_bounds__(256) void k_mask_export(WorkList wl) {
  const int b = blockIdx.x;
  const int jb = find_job(wl.start, wl.njobs, b);
  const JobDesc &J = wl.jobs[jb];
  const int t = b - wl.start[jb];
  const int S = J.S;
  for (int l = threadIdx.x; l < J.F; l += 256) {
    const float v = J.V[(size_t)t * J.Fp + l];
    float tot = 0.0f;
    for (int s = 0; s < S; ++s) tot += J.sep[((size_t)s * J.T + t) * J.Fp + l];
    for (int s = 0; s < S; ++s) {
      const float vh = J.sep[((size_t)s * J.T + t) * J.Fp + l];
      const float o = v > 0.0f ? (tot > 0.0f ? v * (vh / tot) : v / (float)S) : 0.0f;
      if (J.out_sep) J.out_sep[((size_t)s * J.T + t) * J.F + l] = o;
    }
  }
  if (J.out_alpha)
    for (int k = threadIdx.x; k < J.M; k += 256) J.out_alpha[(size_t)t * J.M + k] = J.alpha[(size_t)t * J.Mp + k];
  if (J.out_post)
    for (int i = threadIdx.x; i < S * J.N; i += 256) {
      const int s = i / J.N, n = i % J.N;
      J.out_post[((size_t)s * J.T + t) * J.N + n] = J.post[((size_t)s * J.T + t) * J.N + n];
    }
}

// Sum of the per-frame contributions of every iteration (fixed order,
// compensated), plus the constant T * C.  One block per (job, iteration).
__global__ __launch_bounds__(256) void k_elbo_reduce(WorkList wl) {
  __shared__ Comp red[4];
  const int b = blockIdx.x;
  const int jb = find_job(wl.start, wl.njobs, b);
  const JobDesc &J = wl.jobs[jb];
  const int it = b - wl.start[jb];
  Comp s = comp_zero();
  for (int t = threadIdx.x; t < J.T; t += 256) {
    const float2 v = J.elbo[(size_t)it * J.T + t];
    Comp d; d.hi = v.x; d.lo = v.y;
    s = comp_merge(s, d);
  }
  s = wave_comp(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    Comp a = red[0];
    for (int w2 = 1; w2 < 4; ++w2) a = comp_merge(a, red[w2]);
    const double L = (double)a.hi + (double)a.lo + J.elbo_const;
    if (J.out_elbo) J.out_elbo[it] = L;
    if (!isfinite(L)) atomicOr(J.status, kNonFinite);
  }
}

// ------------------------------------------------------------------ building blocks
__global__ void k_special(int64_t n, const float *x, float *psi, float *lg) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (psi) psi[i] = digammaf(x[i]);
    if (lg) lg[i] = lgammaf_pos(x[i]);
  }
}

// Chain-only problem: phi <- logev rows (padded to 64), ev / sh as k_update makes them.
__global__ void k_chain_prep(JobDesc J, const float *logev) {
  const int t = blockIdx.x, lane = threadIdx.x;
  const bool live = lane < J.N;
  const float x = live ? logev[(size_t)t * J.N + lane] : -INFINITY;
  const float mx = wave_max(x);
  J.phi[(size_t)t * 64 + lane] = live ? x : 0.0f;
  J.ev[(size_t)t * 64 + lane] = (live && mx > -INFINITY) ? expf(x - mx + kEvHeadroomLog) : 0.0f;
  if (lane == 0) J.sh[t] = mx - kEvHeadroomLog;
}

// One job's table image -> dst (4-byte words), and the job's status word cleared.
__global__ void k_put_table(OneJobTable img, int *dst) {
  constexpr int kWords = (int)(sizeof(OneJobTable) / 4);
  const int *src = reinterpret_cast<const int *>(&img);
  for (int i = threadIdx.x; i < kWords; i += blockDim.x) dst[i] = src[i];
  if (threadIdx.x == 0) *img.desc.status = 0;
}

// ------------------------------------------------------------------ launchers
static inline hipError_t last() { return hipGetLastError(); }

hipError_t launch_put_table(const OneJobTable &img, void *dst, hipStream_t st) {
  static_assert(sizeof(OneJobTable) % 4 == 0, "the image is copied in 4-byte words");
  k_put_table<<<1, 64, 0, st>>>(img, reinterpret_cast<int *>(dst));
  return last();
}

hipError_t launch_status_gather(const WorkList &wl, int *dst, hipStream_t st) {
  if (wl.njobs > 0) k_status_gather<<<1, 256, 0, st>>>(wl, dst);
  return last();
}

hipError_t launch_begin(const WorkList &pack, const WorkList &trans, hipStream_t st) {
  if (pack.njobs > 0) k_status_clear<<<1, 256, 0, st>>>(pack);
  if (pack.total > 0) k_begin_pack<<<pack.total, 256, 0, st>>>(pack);
  if (trans.total > 0) k_begin_transpose<<<trans.total, 256, 0, st>>>(trans);
  return last();
}

hipError_t launch_start_ratio(const WorkList &lam, const WorkList &ratio, hipStream_t st) {
  if (lam.total > 0) k_start_lambda<<<lam.total, 256, 0, st>>>(lam);
  if (ratio.total > 0) k_start_ratio<<<ratio.total, 256, 0, st>>>(ratio);
  return last();
}

hipError_t launch_spectrum(const WorkList &wl, bool bf16, bool small, hipStream_t st) {
  if (wl.total <= 0) return last();
  if (!bf16) k_spectrum<false, 2, 2><<<wl.total, 256, 0, st>>>(wl);
  else if (small) k_spectrum<true, 2, 2><<<wl.total, 256, 0, st>>>(wl);
  else k_spectrum<true, kSpecWM, kSpecWN><<<wl.total, 256, 0, st>>>(wl);
  return last();
}

hipError_t launch_counts(const WorkList &wl, bool bf16, hipStream_t st) {
  if (wl.total <= 0) return last();
  if (bf16) k_counts<true><<<wl.total, 256, 0, st>>>(wl);
  else k_counts<false><<<wl.total, 256, 0, st>>>(wl);
  return last();
}

hipError_t launch_chain_fb(const WorkList &rounds, const WorkList &fixup, int nmax, hipStream_t st) {
  if (rounds.total <= 0) return last();
  const int nr = (nmax + 3) & ~3;
#define NFHMM_FB_CASE(R)                                    \
  case R:                                                   \
    k_fb_round<R><<<rounds.total, 64, 0, st>>>(rounds, 1); \
    k_fb_round<R><<<rounds.total, 64, 0, st>>>(rounds, 2); \
    k_fb_fixup<R><<<fixup.total, 64, 0, st>>>(fixup);      \
    break;
  switch (nr) {
    NFHMM_FB_CASE(4) NFHMM_FB_CASE(8) NFHMM_FB_CASE(12) NFHMM_FB_CASE(16)
    NFHMM_FB_CASE(20) NFHMM_FB_CASE(24) NFHMM_FB_CASE(28) NFHMM_FB_CASE(32)
    NFHMM_FB_CASE(36) NFHMM_FB_CASE(40) NFHMM_FB_CASE(44) NFHMM_FB_CASE(48)
    NFHMM_FB_CASE(52) NFHMM_FB_CASE(56) NFHMM_FB_CASE(60) NFHMM_FB_CASE(64)
    default: return hipErrorInvalidValue;
  }
#undef NFHMM_FB_CASE
  return last();
}

hipError_t launch_posterior(const WorkList &post, const WorkList &chains, int nmax, hipStream_t st) {
  if (post.total > 0) k_posterior<<<post.total, 256, 0, st>>>(post);
  if (chains.total <= 0) return last();
  const int nr = (nmax + 3) & ~3;
#define NFHMM_EX_CASE(R) \
  case R: k_chain_exact<R><<<chains.total, 64, 0, st>>>(chains); break;
  switch (nr) {
    NFHMM_EX_CASE(4) NFHMM_EX_CASE(8) NFHMM_EX_CASE(12) NFHMM_EX_CASE(16)
    NFHMM_EX_CASE(20) NFHMM_EX_CASE(24) NFHMM_EX_CASE(28) NFHMM_EX_CASE(32)
    NFHMM_EX_CASE(36) NFHMM_EX_CASE(40) NFHMM_EX_CASE(44) NFHMM_EX_CASE(48)
    NFHMM_EX_CASE(52) NFHMM_EX_CASE(56) NFHMM_EX_CASE(60) NFHMM_EX_CASE(64)
    default: return hipErrorInvalidValue;
  }
#undef NFHMM_EX_CASE
  return last();
}

int update_stride(int mp_max, int sn_max) { return mp_max + ((sn_max + 3) & ~3); }
int update_waves(int stride) { return max(1, min(4, 14336 / max(stride, 1))); }

hipError_t launch_update(const WorkList &wl, int mode, int round, int stride, hipStream_t st) {
  const int wpb = update_waves(stride);
  if (wl.total > 0) k_update<<<wl.total, 64 * wpb, (size_t)wpb * stride * sizeof(float), st>>>(wl, mode, round, stride);
  return last();
}

hipError_t launch_finish(const WorkList &frames, const WorkList &tiles, const WorkList &iters, hipStream_t st) {
  if (tiles.total > 0) k_reconstruct<<<tiles.total, 256, 0, st>>>(tiles);
  if (frames.total > 0) k_mask_export<<<frames.total, 256, 0, st>>>(frames);
  if (iters.total > 0) k_elbo_reduce<<<iters.total, 256, 0, st>>>(iters);
  return last();
}

hipError_t launch_special(int64_t n, const float *x, float *psi, float *lg, hipStream_t st) {
  const int blocks = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  if (n > 0) k_special<<<blocks, 256, 0, st>>>(n, x, psi, lg);
  return last();
}

hipError_t launch_chain_prep(const JobDesc &J, const float *logev, hipStream_t st) {
  k_chain_prep<<<J.T, 64, 0, st>>>(J, logev);
  return last();
}


}  // namespace nfhmm
