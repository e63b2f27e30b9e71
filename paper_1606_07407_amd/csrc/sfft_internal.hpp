// Internal structures shared by the host plan code and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace sfft {

constexpr int kWG = 256;          // threads per work-group (4 waves of 64)
constexpr size_t kLdsLimit = 160 * 1024 - 4096;  // dynamic LDS per work-group (the rest
                                                 // is the kernels' static LDS)
constexpr int kMaxD2 = 256;       // largest number of unwrapped coordinates (FP32: also 2 (S+1) <= 128)
constexpr int kMaxRT = 8;         // MFMA row tiles: 2 (S+1) real rows <= 128
constexpr int kChunk = 16;        // sampler: A-fragment pairs staged in LDS per chunk
constexpr int kF64Chunk = 256;    // FP64 sampler: modes whose coefficients are staged at once
constexpr size_t kF64StageBytes = 16384;  // FP64 sampler: LDS for that stage and the wave sums
constexpr int kTwiddleBits = 6;   // DFT twiddles exp(-2 pi i t / L) = T1[t >> 6] * T2[t & 63]
// Largest FFT lengths held in LDS (FP32, FP64); Bluestein lengths up to 4 times
// these run in 2 or 4 parts through the workspace.
constexpr int kLdsFftMax32 = 8192;
constexpr int kLdsFftMax64 = 4096;
constexpr int kBluesteinParts = 4;
// LDS entries of the Bluestein twiddle tables for an L-point convolution whose
// FFTs have M points (M-point pair, then the L-point pair when L > M).
__host__ __device__ inline int bs_tab_entries(int L, int M) {
  const int n1m = (M >> kTwiddleBits) > 0 ? (M >> kTwiddleBits) : 1;
  return n1m + (1 << kTwiddleBits) + (L > M ? (L >> kTwiddleBits) + (1 << kTwiddleBits) : 0);
}
// FFT radix schedules of a power-of-two length L = 2^n (n = 4 q + b): radix-2
// (b odd) and radix-4 (b >= 2) head passes, then radix 16; or, when b = 3,
// one radix-8 head pass in place of the radix-2 and radix-4 ones.
constexpr int kFftRadix24Head = 1;
constexpr int kFftRadix8Head = 2;
// Sampler column-tile bands: rounds with p below 320, 640, 1600, and above.
constexpr int kNtBands = 4;
__host__ __device__ inline int nt_band(int p) {
  return p < 320 ? 0 : p < 640 ? 1 : p < 1600 ? 2 : 3;
}

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

// Elements of an n-point DFT buffer in LDS with its padding (one after every 16).
__host__ __device__ inline int lds_padded(int n) { return n + (n >> 4); }

// LDS carve-up of the registry merge step (shared by host sizing and device).
struct MergeLds {
  size_t accpos, ids, key0, runflag, runpos, cnt, matchrun, keep, bytes;
};
__host__ __device__ inline MergeLds merge_lds(int k_max, int cap) {
  MergeLds m;
  size_t o = 0;
  m.accpos = o;   o = align16(o + 4 * (size_t)k_max);
  m.ids = o;      o = align16(o + 4 * (size_t)(2 * k_max + 2));
  m.key0 = o;     o = align16(o + 8 * (size_t)(2 * k_max + 2));
  m.runflag = o;  o = align16(o + 4 * (size_t)k_max);
  m.runpos = o;   o = align16(o + 4 * (size_t)k_max);
  m.cnt = o;      o = align16(o + 4 * (size_t)(cap + 1));
  m.matchrun = o; o = align16(o + 4 * (size_t)cap);
  m.keep = o;     o = align16(o + 4 * (size_t)(2 * cap + 2));
  m.bytes = o;
  return m;
}

// LDS carve-up of the decode step: accept flags [k_max] | classifier parameters
// (FP32) | residual-mode counts per bucket [p_max] (feature export only).
__host__ __device__ inline size_t decode_lds_w(int k_max) { return align16(4 * (size_t)k_max); }
__host__ __device__ inline size_t decode_lds_cnt(int k_max) {
  return decode_lds_w(k_max) + align16(4 * (size_t)4866);
}

// Byte offsets of one work-group slot's workspace (each 256-byte aligned).
struct WsLayout {
  size_t ypl;      // int64  [k_max][d2]        planted modes, unwrapped
  size_t ccomp;    // cplx T [m_max][S1]        per-mode coefficient rows
  size_t afrag;    // float  [pairs_max][RT][64] MFMA A fragments (FP32 path)
  size_t sy[2];    // int64  [cap][d2]          registry keys by slot (two banks)
  size_t sa[2];    // double2[cap]              registry coefficients by slot
  size_t sE[2];    // float2 [cap][S]           shift phases E_s(y) by slot (FP32 plans)
  size_t ord[2];   // int32  [cap]              slots in lexicographic order of y
  size_t dirty;    // int32  [cap]              slots whose exponential-sum rows are stale
  size_t V;        // cplx T [S1][vstride]      samples, then spectra
  size_t chirp;    // cplx T [p_max]            Bluestein chirp
  size_t bhat;     // cplx T [L_max]            DFT of the chirp filter
  size_t big;      // cplx T [L_max]            halves of a DFT longer than LDS holds (else empty)
  size_t cand;     // int32  [k_max]            candidate buckets
  size_t acc_y;    // int64  [k_max][d2]        decoded frequencies
  size_t acc_a;    // double2[k_max]            decoded coefficients
  size_t acc_ok;   // int32  [k_max]            accept flags, then ranks
  size_t run;      // int32  [k_max]            merge bookkeeping
  size_t pl_sorted;// int32  [k_max]            planted modes in lexicographic order (export)
  size_t feat_tmp; // float  [k_max][8]         candidate features (export)
  size_t merge;    // MergeLds carve-up when it does not stay in LDS (merge_global)
  size_t wtmp;     // int64  [k_max][d]         outputs before ranking (wrap_rank only)
  size_t bytes;    // size of one slot
};

// Everything a kernel needs about a plan (passed by value).
struct KParams {
  int d, d1, d2, S, S1, RT;
  int64_t N, NB;          // NB = N^d1 (d1: the largest block)
  int k_max, cap, m_max, pairs_max;
  int max_rounds, prime_rule, p_min, ladder_K, robust, precision;
  double c, tau, tau_noise, eta;
  int p_max, L_max, log2_Lmax, vstride;
  const int32_t* primes;  // ascending primes usable by the prime rule, up to p_max
  int n_primes;
  char* ws;               // slots back to back
  size_t ws_slot;
  WsLayout lay;
  int* queue;             // work-queue counter (zeroed before each launch)
  int classifier;         // 0 plain ratio test, 1 learned classifier
  const uint16_t* mlp_w;  // BF16 parameters of the learned classifier
  double mlp_thr, feat_scale;
  int n_slots;
  int lds_bytes;
  int merge_global;       // 1: the merge/sort arrays live in the slot, not in LDS
  int verify;             // verification round when |R| reaches k
  int p_vmax;             // largest prime a verification round can use
  double verify_eta;
  int residual;           // 0: registry subtracted from the spectra, 1: from the samples
  int sub_cs;             // FP32 spectrum subtraction: sets per LDS-staged block (0: unstaged)
  int tw_half;            // FP32 sampler: twiddle table of p/2 + 1 points (long lines; the
                          // recovery then runs as the several-groups launches)
  int sched_nt[kNtBands]; // sampler column tiles per wave per p band (0: built-in choice)
  int sched_fft;          // kFftRadix24Head or kFftRadix8Head
  int sched_dft_batch;    // FP32: most sets per batched Bluestein pass (0: all that fit)
  // Partition of the d coordinates into d2 blocks (device tables): block q holds
  // coordinates perm[blk[q]] .. perm[blk[q+1] - 1], the first the least
  // significant base-N digit; y_q lies in [band[2q], band[2q+1]].
  const int32_t* blk;     // [d2 + 1] block starts
  const int32_t* perm;    // [d] coordinate order
  const int64_t* band;    // [d2][2] inclusive band of each coordinate
  int wrap_rank;          // lexicographic order of w differs from that of y
  // 2D tilting: y = (tb w0 - ta w1, ta w0 + tb w1), w = (tb y0 + ta y1,
  // -ta y0 + tb y1) / tc2 (tilt = 0: the partition above)
  int tilt;
  int64_t ta, tb, tc2;
};

// Modes the sampler's LDS residue arrays hold: the planted modes, plus the
// registry when the residual is subtracted from the samples.
__host__ __device__ inline int sampler_m_max(const KParams& kp) {
  return kp.residual == 1 ? kp.m_max : 2 * ((kp.k_max + 1) / 2);
}

// Whether the several-groups recovery gives a round's noise and DFTs a launch of their
// own, dealt out over the groups: when a round's DFT work is large (S1 L_max >= 2^18
// points; measured: c5 45.2 -> 40.6 ms, the d = 1000 sweep 9-15% faster, while the d =
// 100 sweep at k = 256 and 512, 21 sets of 4096 and 8192 points, was 19% and 4% slower
// with the extra launch per round).  Otherwise the one-group launch transforms them.
__host__ __device__ inline bool split_dft_launch(const KParams& kp) {
  return (int64_t)kp.S1 * kp.L_max >= ((int64_t)1 << 18);
}

// Per-work-group Bluestein chirp, filter spectrum and parts buffer of the DFT launch
// of the several-groups recovery (byte offsets, 256-aligned, and the total).
struct SplitDftScratch {
  size_t chirp, bhat, big, bytes;
};
__host__ __device__ inline SplitDftScratch split_dft_scratch(const KParams& kp) {
  const size_t cs = kp.precision == 1 ? 8 : 16;
  const int maxL = kp.precision == 1 ? kLdsFftMax32 : kLdsFftMax64;
  auto a256 = [](size_t x) { return (x + 255) & ~(size_t)255; };
  SplitDftScratch s;
  s.chirp = 0;
  s.bhat = a256(cs * (size_t)kp.p_max);
  s.big = s.bhat + a256(cs * (size_t)kp.L_max);
  s.bytes = s.big + a256(kp.L_max > maxL ? cs * (size_t)kp.L_max : 0);
  return s;
}

struct KBatch {
  int B;
  const int64_t* mode_off;
  const int64_t* freqs;
  const double* coeffs;
  const int32_t* k;
  const double* sigma;
  uint64_t seed;
};

struct KOut {
  int64_t* freqs;
  double* coeffs;
  int32_t* k_found;
  int32_t* status;
  int32_t* rounds;
  int64_t* samples;
  int32_t* trace;
  float* feat;            // bucket-feature export (NULL: off)
  uint8_t* label;
  int32_t* meta;
  int64_t* count;
  int64_t cap;
  int64_t* phase;         // [B][max_rounds][8] wall-clock ticks per phase (NULL: off)
};

// A session of caller-supplied samples (device arrays owned by the session).
struct WgState;
struct KSess {
  int B;
  const int32_t* k;   // [B] sparsities
  WgState* state;     // [B] round state between launches
  int32_t* req_p;     // [B] prime of the requested round, 0 once finished
  int32_t* req_m;     // [B] its unwrapped axis, 1-based
  int32_t* trace;     // [B][max_rounds][8]
};

// Launchers (defined in the .hip file).  Return a hipError_t as int.
int launch_zero_queue(const KParams& kp, int64_t* count, void* stream);
int launch_mlp_forward(const void* w, const float* x, int64_t n, float* prob, void* stream);
// Gradient: per-group partial sums in `part` (kMlpGradGroups rows of
// kMlpPartStride floats), then added in group order into grad and loss.
constexpr int kMlpParamCount = 4866;
constexpr int kMlpGradGroups = 64;
constexpr int kMlpPartStride = kMlpParamCount + 1;
int launch_mlp_grad(const void* w, const float* x, const uint8_t* y, int64_t n, int64_t rows,
                    uint64_t seed, uint64_t step, float* part, float* grad, float* loss,
                    void* stream);
int launch_mlp_init(const void* w, float* master, float* m, float* v, void* stream);
int launch_mlp_adam(float* master, float* m, float* v, const float* g, void* w, float lr,
                    float bc1, float bc2, void* stream);
int launch_mlp_accum(const float* src, float* dst, float scale, void* stream);
int launch_fill(float* a, int n, float v, void* stream);
int launch_recover(const KParams& kp, const KBatch& kb, const KOut& ko, int grid, void* stream);
// Several work-groups per signal (batches smaller than the chip): `state` holds
// kb.B round states (split_state_bytes() each), ngrp groups sample each line and,
// when split_dft_launch(kp), transform its sets, each group with
// split_dft_scratch(kp).bytes of `dft_scratch` (kb.B * ngrp of them; else unused).
size_t split_state_bytes();
int launch_recover_split(const KParams& kp, const KBatch& kb, const KOut& ko, void* state,
                         int ngrp, void* dft_scratch, void* stream);
// Fixed device scratch of sfft_recover_static (see the .hip file): its size,
// the part the queue counter takes, the per-device address lookup (call once
// per device with that device current), the slots of a given size it holds,
// and the launch that uses it instead of the plan's workspace.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
constexpr size_t kStaticQueueBytes = 256;
int static_scratch_setup(int dev);
int static_scratch_slots(size_t ws_slot);
int launch_recover_static(const KParams& kp, const KBatch& kb, const KOut& ko, int dev,
                          void* stream);
int launch_sample_lines(const KParams& kp, const KBatch& kb, int round, int p, int m,
                        const int64_t* res_off, const int64_t* res_y, const double* res_c,
                        void* V, void* stream);
int launch_dft(const KParams& kp, void* data, int count, int p, void* stream);
int set_kernel_lds_limits(int lds_bytes);
size_t session_state_bytes();
// what: 0 init, 1 feed (samples), 2 points (t), 3 finish (ko)
int launch_session(const KParams& kp, const KSess& ss, int what, const void* samples, double* t,
                   const KOut* ko, void* stream);

}  // namespace sfft
