// Host-side launchers of the kernels in nfhmm_kernels.hip.
#pragma once
#include <hip/hip_runtime.h>

#include "jobdesc.h"

namespace nfhmm {

enum UpdateMode : int { kUpdMessages = 0, kUpdUniform = 1, kUpdFromAlpha = 2 };

// The work-list table of a single job as one image: its descriptor and, per launch
// kind, the block range [0, blocks).  launch_put_table writes it to device memory
// from the kernel's own argument (no host staging buffer) and clears the job's
// status word.
constexpr int kOneJobLists = 16;
struct OneJobTable {
  JobDesc desc;
  int start[kOneJobLists][2];
};
hipError_t launch_put_table(const OneJobTable &img, void *dst, hipStream_t st);

// Every job of a work list starting together: clear the status words, pack V and
// the dictionary (and set w = 1 for a default start), transpose the dictionary.
// Blocks per job: pack ceil(T / 4) + Mp / 4 (+ kBeginFillBlocks for a default
// start), trans (Mp / 32) (Fp / 32).
constexpr int kBeginFillBlocks = 32;
hipError_t launch_begin(const WorkList &pack, const WorkList &trans, hipStream_t st);
// R = V / Lambda of a default start, where Lambda = beta 1 is one value per bin:
// lam has ceil(F / 16) blocks per default-start job, ratio T (0 for warm starts).
constexpr int kStartLamBinsPerBlock = 16;
hipError_t launch_start_ratio(const WorkList &lam, const WorkList &ratio, hipStream_t st);
// dst[i] = the status word of job i of wl (device memory, wl.njobs ints)
hipError_t launch_status_gather(const WorkList &wl, int *dst, hipStream_t st);
// FP32: 64 x 64 block tiles.  BF16: kSpecBM x kSpecBN, or with small 64 x 64 (work
// lists built with kSpecSmallBM / BN)
hipError_t launch_spectrum(const WorkList &wl, bool bf16, bool small, hipStream_t st);
hipError_t launch_counts(const WorkList &wl, bool bf16, hipStream_t st);
// Chunked forward-backward: rounds 1 and 2 (one block per source, direction and
// chunk), then the fix-up (one block per source and direction).
hipError_t launch_chain_fb(const WorkList &rounds, const WorkList &fixup, int nmax, hipStream_t st);
// d-hat from the messages (post: one block per source and 4 frames), then the exact
// log-space pass over flagged chains (chains: one block per source).
hipError_t launch_posterior(const WorkList &post, const WorkList &chains, int nmax, hipStream_t st);
// k_update: floats of LDS per frame (elements padded to mp_max, then the S*N
// chain posteriors) and frames per block (one wavefront each)
int update_stride(int mp_max, int sn_max);
int update_waves(int stride);
hipError_t launch_update(const WorkList &wl, int mode, int round, int stride, hipStream_t st);
hipError_t launch_finish(const WorkList &frames, const WorkList &tiles, const WorkList &iters, hipStream_t st);
hipError_t launch_special(int64_t n, const float *x, float *psi, float *lg, hipStream_t st);
hipError_t launch_chain_prep(const JobDesc &J, const float *logev, hipStream_t st);

// Short-time Fourier transform (stft_kernels.hip).  B signals x[B][n]; frame t
// covers samples [t hop, t hop + nfft); nfft is a power of two in [64, 4096].
// mag, phase: [B][T][nfft/2 + 1].
hipError_t launch_stft(int nfft, const float *x, int64_t n, int hop, int T, int B, float *mag, float *phase,
                       hipStream_t st);
// Inverse of B mixtures' S magnitude sets mag[B][S][T][nfft/2 + 1], source (b, s)
// with phase[b][T][nfft/2 + 1]: y[B][S][n] by weighted overlap-add.  B * S <= 65535.
hipError_t launch_istft(int nfft, const float *mag, const float *phase, int T, int B, int S, int hop, int64_t n,
                        float *y, hipStream_t st);
// frames per block of the inverse (a multiple of the frames that cover one sample)
int istft_run(int nfft, int hop);

}  // namespace nfhmm
