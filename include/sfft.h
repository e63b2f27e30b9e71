/*
 * sfft.h -- C ABI of the MI355X (gfx950) sparse Fourier recovery library.
 *
 * The library recovers k-sparse spectra of d-dimensional signals
 *     f(t) = sum_j a_j exp(2 pi i w_j . t),  w_j in [-N/2, N/2)^d integer,
 * (the problem statement of "High-Dimensional Sparse Fourier Algorithms",
 * Choi, Christlieb, Wang: Section 2.2 eq. (9), Section 4.1.2 eq. (32)) with
 * the MultiPhaseshift method of Section 4.1.2: partial unwrapping of the d
 * coordinates into d2 = d/d1 coordinates of bandwidth N^d1 (eq. (35)),
 * sampling along the unwrapped axis m at h/p and at the same points shifted
 * by eps along each axis n (eq. (41)), prime-length DFTs, the collision test
 * of eq. (42), phase-ratio decoding of eq. (41), and adaptive subtraction of
 * the modes already found (Section 5.0).
 *
 * Conventions (every entry point):
 *   - Plain C types only.  "device" pointers are HIP device memory on the
 *     current device; "host" pointers are ordinary host memory.
 *   - The caller owns every buffer it passes.  A plan owns its workspace.
 *   - Argument errors are detected on the host before any launch and
 *     returned synchronously; sfft_last_error() then describes them.  Launch
 *     failures return SFFT_EDEVICE.  Data-dependent outcomes (a signal that
 *     did not converge) are written to the per-signal status output.
 *   - Entry points taking a `stream` (a hipStream_t, NULL = default stream)
 *     only enqueue work; outputs are valid after the stream synchronises.
 *   - A plan may be used by one stream at a time; calls on one plan that
 *     overlap in time race on its workspace.
 */
#ifndef SFFT_H
#define SFFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sfft_plan_s* sfft_plan;

typedef enum {
  SFFT_OK = 0,
  SFFT_NOT_CONVERGED = 1, /* per-signal: max_rounds reached with |R| < k          */
  SFFT_RESIDUAL_NONZERO = 2, /* per-signal: |R| = k but the last verification round
                                still found residual energy (verify = 1)          */
  SFFT_EINVAL = -1,       /* invalid argument (see sfft_last_error())             */
  SFFT_ERANGE = -2,       /* sizes beyond what the plan or the device supports    */
  SFFT_ENOMEM = -3,       /* device allocation failed                             */
  SFFT_EDEVICE = -4       /* HIP runtime error                                    */
} sfft_status;

enum { SFFT_PRIME_PAPER = 0, SFFT_PRIME_SMOOTH = 1 };
enum { SFFT_FP64 = 0, SFFT_FP32 = 1 };
enum { SFFT_CLS_PLAIN = 0, SFFT_CLS_MLP = 1 };
enum { SFFT_RESIDUAL_SPECTRUM = 0, SFFT_RESIDUAL_SAMPLES = 1 };

/* Learned bucket classifier (not in the paper): an 8-64-64-2 ReLU network with
 * BF16 parameters, evaluated with FP32 accumulation.  Parameter blob: the
 * SFFT_MLP_PARAMS BF16 values W1 [64][8], b1 [64], W2 [64][64], b2 [64],
 * W3 [2][64], b3 [2], row-major, back to back.  Output 1 is "the bucket holds
 * exactly one mode".  Features of a candidate bucket h, with r_s =
 * F_s[h] / F_0[h], y the decoded unwrapped frequency and z = r_s exp(-i pi K y_n
 * / N^d1) for a set shifted by K eps along axis n: the coarse and fine sets of
 * the projection axis m and of the axis n* != m whose fine |r| is furthest from
 * 1 (ties to the smaller n; n* = m when d2 = 1; fine = coarse without a
 * ladder), each as asinh((Re z - 1) / s), asinh(Im z / s), s = feature_scale;
 * inputs are rounded to BF16 before the network. */
#define SFFT_MLP_PARAMS 4866
#define SFFT_MLP_FEATURES 8

/* Method parameters (the inputs c, k, N, d, d1, d2, eps of the MultiPhaseshift
 * listing, plus the readings the paper leaves open). */
typedef struct {
  int32_t d;          /* dimension, >= 1                                            */
  int32_t d1;         /* unwrapping block size; d % d1 == 0; d2 = d / d1 <= 256;
                         FP32 also needs 2 (S+1) <= 128 (else SFFT_ERANGE).
                         Ignored when `blocks` is given                             */
  int64_t N;          /* per-dimension bandwidth, even, >= 2; N^d1 <= 2^40 (with
                         `blocks`: N^(largest block) <= 2^40)                       */
  int32_t k_max;      /* largest sparsity of any signal recovered with this plan    */
  double c;           /* p_i = i-th prime >= max(ceil(c k*), p_min); c > 1          */
  int32_t prime_rule; /* SFFT_PRIME_PAPER, or SFFT_PRIME_SMOOTH (p - 1 7-smooth)    */
  int32_t p_min;      /* floor on c k* (0 = the paper's rule)                       */
  int32_t ladder_K;   /* 1: one shift eps per axis (paper).  K > 1: also K*eps      */
  double tau;         /* collision-test tolerance; <= 0 means tau = eps            */
  double tau_noise;   /* extra tolerance tau_noise * sqrt(p) / |F_0[h]| (>= 0)      */
  double eta;         /* prune |a| < eta; buckets with |F_0|/p < eta are skipped    */
  int32_t max_rounds; /* round cap, 1..256                                          */
  int32_t precision;  /* SFFT_FP64: FP64 end to end.  SFFT_FP32: FP32 samples,
                         exponential sums and DFTs, FP64 decode and registry        */
  int32_t robust;     /* 0: paper's test.  1: also residue y_m = h (mod p) and
                         ladder-consistency checks                                  */
  int32_t classifier; /* SFFT_CLS_PLAIN: the ratio-magnitude test of eq. (42).
                         SFFT_CLS_MLP: accept iff the network's probability of one
                         mode exceeds mlp_threshold (the decode checks still apply) */
  const void* mlp_weights; /* device, SFFT_MLP_PARAMS BF16 values; NULL with PLAIN      */
  double mlp_threshold;    /* acceptance threshold on the probability, (0, 1)          */
  double feature_scale;    /* s of the features; <= 0 means s = tau                    */
  int32_t verify;          /* 1: verification round when |R| reaches k (not in the
                              paper): the residual is sampled once on the tilted line
                              t_h = (h/p) U v, v_n = q^(n-1) mod p, q = 1 + (i mod
                              (p-1)), p the round-i prime for k* = 1, and transformed;
                              buckets with |F[h]|/p >= verify_eta send the loop on with
                              k* = their count.  0: stop at |R| = k (the listing)     */
  double verify_eta;       /* residual-energy floor of the verification; <= 0: eta     */
  int32_t residual;        /* where the modes found so far are subtracted (Section 5.0):
                              SFFT_RESIDUAL_SAMPLES: g(t) as an exponential sum over the
                              samples of every set, on the matrix cores with the planted
                              sum (the listing's step); SFFT_RESIDUAL_SPECTRUM: the
                              closed form of its DFT (eq. (41)), p sum a E_s over the
                              entries of each bucket, subtracted from the spectra in
                              FP64 -- the same spectra with O(|R| (S+1)) instead of
                              O(p |R| (S+1)) work                                      */
  /* Kernel schedules: how the kernels tile their work.  Every choice gives the
   * same results up to FP32 rounding; 0 takes the built-in choice, and
   * sfft_autotune picks them by measurement. */
  int32_t sched_nt[4];     /* FP32 sampler: 16-point column tiles per wave in rounds
                              with p < 320, < 640, < 1600 and >= 1600: 2 to 4, or up
                              to 8 in the last two bands (below 640 points the chunked
                              FP32 accumulation needs at most 4); 0 = chosen from p */
  int32_t sched_fft;       /* passes of the power-of-two FFTs inside Bluestein, L = 2^n:
                              1 = a radix-2 (n odd) and a radix-4 (n mod 4 >= 2) head
                              pass, then radix 16; 2 = the same, except one radix-8
                              head pass when n = 3 mod 4; 0 = 1                      */
  int32_t sched_dft_batch; /* most sample sets transformed together in one Bluestein
                              pass over the LDS buffer: 1 = one set at a time,
                              2..64, 0 = as many as fit                              */
  /* General partitions (Section 4.1: a block's coordinates need not be in their
   * natural order and blocks need not have one size; Section 4.1.2: d prime).
   * Host arrays, read only by sfft_plan_create (and sfft_autotune), owned by the
   * caller.  Block q (sizes d_0, d_1, ...) holds the coordinates
   * order[s_q], ..., order[s_q + d_q - 1], s_q = d_0 + ... + d_{q-1}, the first
   * the least significant base-N digit: y_q = sum_r w[order[s_q + r]] N^r.  One
   * shift eps = 1 / (2 N^(largest block)) serves every axis; each coordinate's
   * decoded value must lie in its own block's band.  Zero-filled fields give
   * the uniform partition of d1 in the natural order (eq. (35)). */
  const int32_t* blocks;   /* n_blocks sizes, each >= 1, summing to d; NULL: d / d1
                              blocks of d1                                           */
  int32_t n_blocks;        /* 1..256 with `blocks` (this is d2); 0 without           */
  const int32_t* order;    /* a permutation of 0..d-1; NULL: 0, 1, ..., d-1          */
  /* 2D tilting (Section 3.3, eq. (27), Theorem 1), for d = 2 with d1 = 1 and no
   * blocks or order: the recovery runs on lines t = U t~, U = [[b, a], [-a, b]]
   * (the rotation by sin = a/c, cos = b/c, scaled by c), so y = U^T w, and each
   * answer is rotated back exactly, w = U y / c^2.  A decoded y is no mode unless
   * U y is divisible by c^2 with the quotient in [-N/2, N/2)^2.  One shift
   * eps = 1 / ((a + b) N) serves both axes.  With b > 2N and gcd(a, b) = 1 no two
   * frequencies share a rotated coordinate, which recovers frequencies on the
   * vertices of axis-aligned rectangles (every parallel projection collides). */
  int32_t tilt;            /* 0: off.  1: on                                         */
  int32_t tilt_a, tilt_b, tilt_c; /* the triple: a^2 + b^2 = c^2, 1 <= a < b, b > 2N,
                              gcd(a, b) = 1; all 0: the plan takes the triple with
                              the smallest a + b (then the smallest b)               */
  /* Work-groups per signal in sfft_recover (0..16).  The S+1 sample sets of a round
   * are sampled at points h/p that split into independent column blocks (the
   * loop over the sets in Algorithm MultiPhaseshift needs no order), so a batch
   * smaller than the device runs each ordinary round's sampling on several
   * work-groups, and, when a round's DFTs are large ((S+1) L_max >= 2^18 points,
   * L_max the longest Bluestein length), its noise and DFTs too (each group some
   * of the sets), and the rest of the round on one (two or three launches per
   * round, no host synchronisation; results identical bit for bit).  Such plans
   * reserve one set of Bluestein tables per work-group the device holds at
   * sfft_plan_create (split_groups sets per workspace slot when it is given).
   * 0: automatic (as many as fill the device, at most 8, when the batch takes at
   * most half of it and k_max >= 256); 1: one work-group per signal (one
   * launch); 2..16.  Split, the phase timestamps' sampling interval (marks 0 to
   * 1) also holds the gap between the launches and the noise. */
  int32_t split_groups;
} sfft_params;

/* A batch of synthetic black-box signals with planted spectra.  All pointers
 * are device pointers.  Signal b is sum_{j in [mode_off[b], mode_off[b+1])}
 * coeffs[j] exp(2 pi i freqs[j] . t) plus complex Gaussian noise of standard
 * deviation sigma[b] per sample: Philox4x64-10 with key (seed, b) and counter
 * (h / 2, sample set, round, 0), output words 0, 1 for even h and 2, 3 for odd
 * h, Box-Muller on their top 53 bits (in FP64 on the FP64 path, in FP32 from
 * the exact integer 1 - u1 on the FP32 path). */
typedef struct {
  int32_t B;                /* number of signals, 1..max_batch                    */
  const int64_t* mode_off;  /* [B + 1], mode_off[0] = 0, non-decreasing           */
  const int64_t* freqs;     /* [mode_off[B]][d] integer frequencies in band       */
  const double* coeffs;     /* [mode_off[B]][2] complex coefficients (re, im)     */
  const int32_t* k;         /* [B] sparsity given to the method, 1..k_max         */
  const double* sigma;      /* [B] noise standard deviation, >= 0                 */
  uint64_t seed;            /* noise key material                                 */
} sfft_signal_batch;

#define SFFT_TRACE_W 8 /* per round: i, k*, p, m, candidates, accepted, |R|, verify;
                          a verification row has k* = 0, m = 0, candidates = buckets
                          with residual energy, verify = 1 */

/* Outputs of sfft_recover (device pointers; the optional ones may be NULL). */
typedef struct {
  int64_t* freqs;    /* [B][k_max][d] recovered w, lexicographic order, zero-padded */
  double* coeffs;    /* [B][k_max][2] recovered a (re, im), same order              */
  int32_t* k_found;  /* [B] number of modes written: min(|R| at the end, k_max)    */
  int32_t* status;   /* [B] SFFT_OK, SFFT_NOT_CONVERGED, SFFT_RESIDUAL_NONZERO
                      * (or SFFT_ERANGE)                                          */
  int32_t* rounds;   /* [B] rounds run (optional)                                   */
  int64_t* samples;  /* [B] signal samples taken (optional)                         */
  int32_t* trace;    /* [B][max_rounds][SFFT_TRACE_W] per-round record (optional);
                      * rows after the last round run are zeroed                   */
  /* Bucket-feature export (optional; all four NULL to disable).  Every candidate
   * bucket of every round appends one record at an atomically claimed index
   * (order across signals is not deterministic); records beyond feat_cap are
   * counted but dropped.  *feat_count is zeroed by the call. */
  float* feat;        /* [feat_cap][SFFT_MLP_FEATURES] features (before BF16 rounding)  */
  uint8_t* label;     /* [feat_cap] 1 iff the residual holds exactly one mode in h  */
  int32_t* feat_meta; /* [feat_cap][4] signal, round, bucket h, accepted (0/1)      */
  int64_t* feat_count;/* [1] records produced                                       */
  int64_t feat_cap;
  /* Phase timestamps (optional, NULL = off): [B][max_rounds][SFFT_TRACE_W] device
   * wall-clock ticks (100 MHz) taken by each work-group at the start of round i
   * (0) and after its sampler (1), DFTs (2), registry subtraction (7), selection
   * (3), test and decode (4) and merge (5); a verification round writes 0 and 6.
   * Unused entries are left as they were. */
  int64_t* phase;
} sfft_outputs;

/* Create a plan: validates `params` (SFFT_EINVAL / SFFT_ERANGE), derives the
 * prime tables, the largest prime any round can use and the DFT sizes, and
 * allocates all device workspace for up to `max_batch` signals on the
 * current device (SFFT_ENOMEM).  `*out` is set only on SFFT_OK.  Primes reach
 * 16384 (FP32) or 8192 (FP64): Bluestein lengths up to 16384 / 8192 points stay
 * in LDS, longer ones (up to twice that) run as two in-LDS halves through the
 * workspace.  SFFT_ERANGE also when a step's LDS carve-up at the largest prime
 * exceeds the work-group's LDS.  FP32 plans whose sampler cannot hold the whole
 * table of p twiddles next to its staged operands keep p/2 + 1 of them (omega^(p-x)
 * = conj omega^x); sfft_recover then always runs the several-groups launches (see
 * split_groups, at most one signal per workspace slot) and sfft_recover_static
 * refuses the plan (SFFT_ERANGE). */
sfft_status sfft_plan_create(const sfft_params* params, int32_t max_batch, sfft_plan* out);

/* Release a plan and its workspace (synchronises the device first).  NULL is
 * accepted. */
sfft_status sfft_plan_destroy(sfft_plan plan);

/* Recover every signal of `batch` (MultiPhaseshift, Section 4.1.2 listing):
 * one persistent launch in which each work-group takes signals from a queue
 * and runs all rounds of one signal (sample, DFT, select, test, decode,
 * registry update) before taking the next; or, for batches smaller than the
 * device (see split_groups), several work-groups per signal over two or
 * three launches per round.  Allocates nothing. */
sfft_status sfft_recover(sfft_plan plan, const sfft_signal_batch* batch,
                         const sfft_outputs* out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): sfft_recover with the
 * per-work-group workspace and the work-queue counter taken from a fixed
 * device array of the library (64 MiB per device, held until the process
 * ends) instead of the plan's workspace.  Same arguments, outputs and results
 * as sfft_recover (feature export is not offered: those fields must be NULL);
 * as many work-groups run as workspace slots fit in the array
 * (sfft_static_scratch_slots), each taking signals from the queue.  The call
 * allocates nothing and clears the part of the array it uses with a kernel
 * before the recovery.  Every call on one device shares that device's array:
 * calls that overlap in time on one device (any plan, any stream) race and
 * must be serialised by the caller.  SFFT_ERANGE when one workspace slot of
 * the plan does not fit in the array; otherwise as sfft_recover. */
sfft_status sfft_recover_static(sfft_plan plan, const sfft_signal_batch* batch,
                                const sfft_outputs* out, void* stream);
/* Workspace slots of this plan that fit in the fixed array (0: the plan is too
 * large for sfft_recover_static). */
int32_t sfft_static_scratch_slots(sfft_plan plan);

/* Bucket features for training the learned classifier (not in the paper; the
 * inputs are the spectra of Algorithm MultiPhaseshift's rounds): runs the same
 * recovery as sfft_recover on `batch` and writes, for every candidate bucket
 * of every round, one record of the export described in sfft_outputs -- the
 * SFFT_MLP_FEATURES features (device float [feat_cap][8], before BF16
 * rounding), the label (device uint8 [feat_cap]: 1 iff the residual holds
 * exactly one mode in the bucket), and (signal, round, bucket, accepted)
 * (device int32 [feat_cap][4]) -- at an atomically claimed index, so the
 * order across signals is not deterministic.  *feat_count (device int64) is
 * zeroed by the call and ends as the number of records produced; records past
 * feat_cap are counted but dropped.  No recovery outputs are written.  The
 * plan's classifier decides which buckets are accepted (the plain test for
 * the training data).  SFFT_EINVAL for a NULL array or feat_cap < 0.
 * Allocates nothing. */
sfft_status sfft_export_bucket_features(sfft_plan plan, const sfft_signal_batch* batch,
                                        float* feat, uint8_t* label, int32_t* feat_meta,
                                        int64_t feat_cap, int64_t* feat_count, void* stream);

/* The line sampler on its own (eqs. (36), (41), adaptive residual of
 * Section 5.0): for each signal b writes the S+1 sample sets of round `round`
 * (1-based; keys the noise counter) along unwrapped axis m (1-based) with
 * prime p:
 *   V[b][s][h] = f_b(t_{s,h}) - sum_{e} res_coeffs[e] exp(2 pi i y_e . t~_{s,h})
 * for h < p, where set 0 is unshifted and set s >= 1 is shifted by K_s eps
 * along axis n_s (s = 1..d2: K = 1, n = s; s = d2+1..2 d2: K = ladder_K,
 * n = s - d2).  res_off[b]..res_off[b+1] index the residual modes of signal b
 * (res_y: [*][d2] int64 unwrapped frequencies, res_coeffs: [*][2] double);
 * res_off may be NULL (no residual).  V is complex of the plan's precision
 * (float2 or double2), [B][S+1][p], device.  p must be prime and at most the
 * plan's largest prime. */
sfft_status sfft_sample_lines(sfft_plan plan, const sfft_signal_batch* batch, int32_t round,
                              int32_t p, int32_t m, const int64_t* res_off,
                              const int64_t* res_y, const double* res_coeffs, void* V,
                              void* stream);

/* Batched DFT of Section 2.1, X[h] = sum_j x[j] exp(-2 pi i h j / p), on
 * `count` sequences of length p stored back to back in `data` (complex of the
 * plan's precision, device), in place.  Any p in [2, plan's largest prime]. */
sfft_status sfft_dft(sfft_plan plan, void* data, int32_t count, int32_t p, void* stream);

/* Caller-supplied samples (signals the library cannot evaluate: the paper's
 * black-box f of eq. (32)).  A session runs the rounds of Section 5.0 one at a
 * time: sfft_session_request names the line each signal needs next, the caller
 * evaluates f on it, sfft_session_feed runs the rest of the round (DFT, registry
 * subtraction in the spectra, selection, decode and merge), and
 * sfft_session_finish writes the answers as sfft_recover does.  Every call is
 * asynchronous on `stream`.  The plan must have residual =
 * SFFT_RESIDUAL_SPECTRUM (else SFFT_EINVAL) and must outlive the session; one
 * session is used on one stream at a time.  With verify = 1 the verification
 * round asks for the tilted line of the plan's verification (m < 0 below).  The session allocates
 * B workspace slots of the plan's size (hipMalloc in create, freed in destroy). */
typedef struct sfft_session_s* sfft_session;

/* k: [B] sparsities (device int32, 1..k_max; others end with SFFT_EINVAL). */
sfft_status sfft_session_create(sfft_plan plan, int32_t B, const int32_t* k, void* stream,
                                sfft_session* out);
sfft_status sfft_session_destroy(sfft_session session);

/* The lines of the next round (device int32 [B] each): p[b] the prime (0 once
 * signal b is finished), m[b] the unwrapped axis (1..d2), or m[b] = -q for a
 * verification round, whose one line is t_h = (h/p) U v with v_n = q^(n-1)
 * mod p (n = 1..d2; only set 0 of the samples is read).  Otherwise the samples are
 * f(t) at t_h = (h/p) U e_m + eps K_s U e_{n_s}, h = 0..p-1, for the sets
 * s = 0..S (eqs. (36), (41)): set 0 unshifted, s = 1..d2 shifted by eps along
 * n_s = s, and with ladder_K > 1 also s = d2+1..2 d2 shifted by K eps along
 * n_s = s - d2; U is the plan's unwrapping (eq. (35), its partition, or the
 * rotation of 2D tilting), eps = 1 / (2 NB) with NB the largest bandwidth of an
 * unwrapped coordinate. */
sfft_status sfft_session_request(sfft_session session, int32_t* p, int32_t* m, void* stream);

/* Convenience: the points of the requested lines, t[b][s][h][0..d) doubles
 * (device, [B][S+1][max_prime][d]; rows h >= p[b] and finished signals are not
 * written). */
sfft_status sfft_session_points(sfft_session session, double* t, void* stream);

/* The samples of the requested lines, complex of the plan's precision (float2
 * or double2), device, [B][S+1][max_prime] (h < p[b] read; finished signals
 * ignored).  Runs one round of every unfinished signal. */
sfft_status sfft_session_feed(sfft_session session, const void* samples, void* stream);

/* Outputs as for sfft_recover (feature export and phase timestamps are not
 * offered: those fields must be NULL).  rounds and samples count the fed
 * rounds; a signal still unfinished ends with SFFT_NOT_CONVERGED. */
sfft_status sfft_session_finish(sfft_session session, const sfft_outputs* out, void* stream);

/* Learned classifier kernels.  `w` points to SFFT_MLP_PARAMS BF16 values
 * (device); x holds n feature rows of SFFT_MLP_FEATURES floats (device), which
 * are rounded to BF16 on input; y holds n labels in {0, 1}.
 *
 * sfft_mlp_forward: prob[i] = probability of one mode for row i (device, n).
 * sfft_mlp_grad: mean softmax cross-entropy over the rows (per row
 *   logsumexp(z) - z[label], finite for any logits) and its gradient with
 *   respect to the parameters (device: grad [SFFT_MLP_PARAMS], loss [1], both
 *   overwritten); the forward and backward passes of training.  The sums over
 *   rows are added in a fixed order: the same inputs give the same bits.
 *   Allocates and frees 1.2 MB of partial sums and synchronises `stream`.
 * sfft_mlp_train: Adam (beta1 0.9, beta2 0.999, eps 1e-8) on FP32 master
 *   parameters initialised from `w`, `epochs` passes of ceil(n / batch) steps
 *   over minibatches drawn with replacement (counter-based hash of seed, step,
 *   row); `w` is overwritten with the BF16 rounding of the trained masters;
 *   loss_hist (device, [epochs], optional) receives the mean minibatch loss of
 *   each epoch.  Deterministic for a given seed.  Allocates and frees its
 *   optimiser state and gradient partial sums (about 1.3 MB) and synchronises
 *   `stream` before returning. */
sfft_status sfft_mlp_forward(const void* w, const float* x, int64_t n, float* prob, void* stream);
sfft_status sfft_mlp_grad(const void* w, const float* x, const uint8_t* y, int64_t n, float* grad,
                          float* loss, void* stream);
sfft_status sfft_mlp_train(void* w, const float* x, const uint8_t* y, int64_t n, int32_t epochs,
                           int32_t batch, double lr, uint64_t seed, float* loss_hist,
                           void* stream);

/* Largest prime a round of this plan can use, and the number of sample sets
 * per round (S+1). */
int32_t sfft_plan_max_prime(sfft_plan plan);
int32_t sfft_plan_num_sets(sfft_plan plan);

/* One candidate measured by sfft_autotune. */
typedef struct {
  double c;                /* oversampling factor                                    */
  int32_t sched_nt[4];     /* schedules, as in sfft_params                           */
  int32_t sched_fft;       /* as run: 0 in the candidate's params is logged as 1     */
  int32_t sched_dft_batch;
  int32_t status;          /* SFFT_OK, or why the candidate's plan was refused       */
  int32_t exact;           /* signals with status SFFT_OK whose recovered support
                              equals the batch's planted support                    */
  double ms;               /* median duration of the timed launches                 */
} sfft_tune_entry;

/* Autotuner (a measurement around the method, not part of it): picks c and the
 * kernel schedules for `batch` by timing whole recoveries on `stream`.
 * Stage 1 measures every c of c_values (host array of n_c values; n_c = 0 keeps
 * params->c) with the schedules of *params.  Stage 2 changes one schedule at a
 * time from the best so far -- sched_fft; for FP32 plans also sched_dft_batch
 * over {0, 1, 2, 4, 8} and each band of sched_nt over its allowed values -- and
 * keeps a change only when it is more than 2% faster with at least as many
 * exact recoveries.  Candidates rank by exact recoveries, then by the median
 * of `steps` timed launches (HIP events on `stream`) after `warmup` untimed
 * ones.  A candidate whose plan cannot be created (e.g. a c whose first prime
 * needs more LDS than a work-group has) is logged with that status and skipped.
 * On SFFT_OK, *params holds the winner (only c and the sched_* fields change),
 * log[0 .. min(*n_log, log_cap)) the candidates in the order measured (log may
 * be NULL when log_cap = 0) and *n_log their number.  Creates one plan per
 * candidate and the output buffers of the batch (device memory, all freed
 * before returning); copies the batch's planted frequencies and each
 * candidate's results to the host; synchronises `stream`.  SFFT_EINVAL for bad
 * arguments; plan and launch errors other than a refused candidate are
 * returned as they are. */
sfft_status sfft_autotune(sfft_params* params, const sfft_signal_batch* batch,
                          const double* c_values, int32_t n_c, int32_t warmup, int32_t steps,
                          sfft_tune_entry* log, int32_t log_cap, int32_t* n_log, void* stream);

/* Text of the last error on this thread ("" if none). */
const char* sfft_last_error(void);

/* Library version, major * 10000 + minor * 100 + patch. */
int32_t sfft_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SFFT_H */
