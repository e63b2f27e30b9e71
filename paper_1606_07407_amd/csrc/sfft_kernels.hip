// HIP kernels of the MultiPhaseshift recovery (gfx950).
//
// recover_kernel: one persistent launch.  Each work-group takes a signal from
// a work queue and runs every round of MultiPhaseshift for it (Section 4.1.2
// listing):  plan the round (k*, p, m) -> mode preparation -> line sampler
// (planted signal minus the registry as one exponential sum) -> S+1 prime
// length DFTs (Bluestein in LDS) -> top-k* bucket selection -> collision test
// and FP64 phase-ratio decode -> registry merge and prune, until |R| = k or
// the round cap, then wraps the unwrapped frequencies back to d dimensions.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <type_traits>

#include "sfft_device.hpp"
#include "sfft_internal.hpp"
#include "sfft_mlp.hpp"

namespace sfft {

// ------------------------------------------------------------ helpers -----
__device__ __forceinline__ int64_t pmod64(int64_t a, int64_t m) {
  int64_t r = a % m;
  return r < 0 ? r + m : r;
}

// a mod p in [0, p) for |a| < 2^52 and 2 <= p < 2^20: the FP64 quotient
// estimate is off by at most one, corrected in each direction.
__device__ __forceinline__ int pmod_small(int64_t a, int p, double inv_p) {
  const int64_t q = (int64_t)floor((double)a * inv_p);
  int64_t r = a - q * (int64_t)p;
  if (r < 0) r += p;
  if (r >= p) r -= p;
  return (int)r;
}

// Unwrapped shift phase exp(2 pi i eps K y) with eps = 1 / (2 NB):
// q = K y mod 2 NB exactly, angle = pi q / NB.
__device__ __forceinline__ cpx<double> shift_phase(int64_t y, int64_t K, int64_t NB) {
  const int64_t q = pmod64(K * y, 2 * NB);
  double c, s;
  expipi((double)q / (double)NB, &c, &s);
  return cmk<double>(c, s);
}

// Shift table: set s = 1..d2 -> (n = s, K = 1); s = d2+1..2 d2 -> (n = s - d2, K).
__device__ __forceinline__ void shift_of(const KParams& kp, int s, int* n0, int64_t* K) {
  if (s <= kp.d2) {
    *n0 = s - 1;
    *K = 1;
  } else {
    *n0 = s - kp.d2 - 1;
    *K = kp.ladder_K;
  }
}

// p = i-th prime >= max(ceil(c k*), p_min); -1 if beyond the table.
__device__ inline int prime_for_round(const KParams& kp, int kstar, int i) {
  double x = ceil(kp.c * (double)kstar);
  if (x < (double)kp.p_min) x = (double)kp.p_min;
  if (x > 2.0e9) return -1;
  const int xi = (int)x;
  int lo = 0, hi = kp.n_primes;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (kp.primes[mid] < xi)
      lo = mid + 1;
    else
      hi = mid;
  }
  const int idx = lo + i - 1;
  return (idx < kp.n_primes) ? kp.primes[idx] : -1;
}

template <typename T>
__device__ __forceinline__ cpx<T>* ws_cpx(char* slot, size_t off) {
  return reinterpret_cast<cpx<T>*>(slot + off);
}

// Scatter coefficient rows of modes [j0, j1) into MFMA A-fragment order.
// A[row][k] for K step `pair`: row = 16 t + (lane & 15) -> set row >> 1,
// Re/Im row & 1; k = lane >> 4 -> mode 2 pair + (k >> 1), Re/Im k & 1;
// value Re C, -Im C (row Re) or Im C, Re C (row Im).
__device__ inline void scatter_afrag(const KParams& kp, const cpx<float>* ccomp, float* afrag,
                                     int j0, int j1) {
  const int RT = kp.RT, S1 = kp.S1;
  const int per_mode = RT * 32;
  const int n = (j1 - j0) * per_mode;
  for (int q = threadIdx.x; q < n; q += kWG) {
    const int j = j0 + q / per_mode;
    const int rem = q - (j - j0) * per_mode;
    const int t = rem >> 5;
    const int li = rem & 31;
    const int jsel = j & 1;
    // lanes whose k >> 1 == jsel: k in {2 jsel, 2 jsel + 1}
    const int k = 2 * jsel + (li >> 4);
    const int lane = k * 16 + (li & 15);
    const int row = 16 * t + (lane & 15);
    const int s = row >> 1;
    float v = 0.f;
    if (s < S1) {
      const cpx<float> c = ccomp[(size_t)j * S1 + s];
      const int rpart = row & 1, tpart = k & 1;
      v = (rpart == 0) ? (tpart == 0 ? c.x : -c.y) : (tpart == 0 ? c.y : c.x);
    }
    afrag[((size_t)(j >> 1) * RT + t) * 64 + lane] = v;
  }
}

// lexicographic compare of two d2-vectors: -1, 0, 1
__device__ __forceinline__ int lexcmp(const int64_t* a, const int64_t* b, int n) {
  for (int i = 0; i < n; ++i) {
    if (a[i] < b[i]) return -1;
    if (a[i] > b[i]) return 1;
  }
  return 0;
}

// Shared per-work-group scalars.
struct WgState {
  int sig, k, M_pl, nR, cur, i, p, m0, kstar, ncand, nacc, status, L, log2L, nU, flag;
  int kv, verified;  // k* after a verification that found residual energy; clean check
  int nslots, sb;    // registry slots in use, storage bank (cur: index of the sorted order)
  int64_t off, samples;
  double sigma;
  uint64_t prefix;
  int need;
  int split;         // several groups per signal: 1 while an ordinary round awaits its
                     // samples, 3 while a verification line awaits its sums, 2 once the
                     // signal is finished
};

// --------------------------------------------------- per-signal set-up -----
// Planted modes: y = U^T w (eq. (35); block q of a general partition holds the
// coordinates perm[blk[q]] .. perm[blk[q+1] - 1], the first the least
// significant base-N digit; tilted: the rotation of eq. (27), y = U^T w with
// U = [[b, a], [-a, b]]) and the coefficient rows
// C[j][0] = a_j, C[j][s] = a_j exp(2 pi i eps K_s y_{j,n_s}).
template <typename T>
__device__ void planted_setup(const KParams& kp, const KBatch& kb, char* slot, WgState& st) {
  int64_t* ypl = reinterpret_cast<int64_t*>(slot + kp.lay.ypl);
  cpx<T>* cc = ws_cpx<T>(slot, kp.lay.ccomp);
  const int d = kp.d, d2 = kp.d2, S1 = kp.S1;
  for (int j = threadIdx.x; j < st.M_pl; j += kWG) {
    const int64_t* w = kb.freqs + (st.off + j) * d;
    if (kp.tilt) {
      ypl[(size_t)j * 2] = kp.tb * w[0] - kp.ta * w[1];
      ypl[(size_t)j * 2 + 1] = kp.ta * w[0] + kp.tb * w[1];
    } else {
      for (int q = 0; q < d2; ++q) {
        int64_t y = 0, pw = 1;
        for (int l = kp.blk[q]; l < kp.blk[q + 1]; ++l) {
          y += w[kp.perm[l]] * pw;
          pw *= kp.N;
        }
        ypl[(size_t)j * d2 + q] = y;
      }
    }
    const cpx<double> a = cmk<double>(kb.coeffs[2 * (st.off + j)], kb.coeffs[2 * (st.off + j) + 1]);
    cc[(size_t)j * S1] = cmk<T>((T)a.x, (T)a.y);
    for (int s = 1; s < S1; ++s) {
      int n0;
      int64_t K;
      shift_of(kp, s, &n0, &K);
      const cpx<double> e = shift_phase(ypl[(size_t)j * d2 + n0], K, kp.NB);
      const cpx<double> v = cmul(a, e);
      cc[(size_t)j * S1 + s] = cmk<T>((T)v.x, (T)v.y);
    }
  }
  if (threadIdx.x == 0 && (st.M_pl & 1)) {
    for (int s = 0; s < S1; ++s) cc[(size_t)st.M_pl * S1 + s] = cmk<T>(0, 0);
  }
  __syncthreads();
}

// Registry storage: entries live in slots that never move while the signal is
// processed (new entries take the next free slot, pruned ones get a zero
// coefficient and leave the order); ord[st.cur] lists the live slots in
// lexicographic order of y.
__device__ __forceinline__ int64_t* reg_y(const KParams& kp, char* slot, int bank) {
  return reinterpret_cast<int64_t*>(slot + kp.lay.sy[bank]);
}
__device__ __forceinline__ double2* reg_a(const KParams& kp, char* slot, int bank) {
  return reinterpret_cast<double2*>(slot + kp.lay.sa[bank]);
}
__device__ __forceinline__ int* reg_ord(const KParams& kp, char* slot, int which) {
  return reinterpret_cast<int*>(slot + kp.lay.ord[which]);
}
__device__ __forceinline__ cpx<float>* reg_E(const KParams& kp, char* slot, int bank) {
  return reinterpret_cast<cpx<float>*>(slot + kp.lay.sE[bank]);
}

// Exponential-sum operand of mode row j, set s: complex c into the MFMA A
// fragments (FP32 path; same lane order as scatter_afrag) or the coefficient
// rows (FP64 path).  Used for the registry rows when the residual is
// subtracted from the samples.
template <typename T>
__device__ __forceinline__ void put_row(const KParams& kp, char* slot, int j, int s,
                                        cpx<double> c) {
  if constexpr (sizeof(T) == 4) {
    float* af = reinterpret_cast<float*>(slot + kp.lay.afrag);
    const float cx = (float)c.x, cy = (float)c.y;
    const int jsel = j & 1;
#pragma unroll
    for (int rpart = 0; rpart < 2; ++rpart) {
      const int row = 2 * s + rpart;
      float* base = af + ((size_t)(j >> 1) * kp.RT + (row >> 4)) * 64 + (row & 15);
      base[(2 * jsel) * 16] = rpart == 0 ? cx : cy;       // K index of Re omega
      base[(2 * jsel + 1) * 16] = rpart == 0 ? -cy : cx;  // K index of Im omega
    }
  } else {
    cpx<double>* cc = reinterpret_cast<cpx<double>*>(slot + kp.lay.ccomp);
    cc[(size_t)j * kp.S1 + s] = c;
  }
}

// Registry rows of the exponential sum, mode row 2 P0 + slot: C[s] = -a E_s(y),
// E_0 = 1, E_s the shift phase of set s.  All slots, or only those flagged
// dirty (flags cleared).  The partner of an odd last slot gets a zero row.
template <typename T>
__device__ void rebuild_rows(const KParams& kp, char* slot, WgState& st, int P0, bool only_dirty) {
  const int S1 = kp.S1, d2 = kp.d2, n = st.nslots;
  const int64_t* sy = reg_y(kp, slot, st.sb);
  const double2* sa = reg_a(kp, slot, st.sb);
  int* dirty = reinterpret_cast<int*>(slot + kp.lay.dirty);
  for (int q = threadIdx.x; q < n * S1; q += kWG) {
    const int e = q / S1, s = q - e * S1;
    if (only_dirty && !dirty[e]) continue;
    const cpx<double> a = cmk<double>(-sa[e].x, -sa[e].y);
    cpx<double> v = a;
    if (s > 0 && (a.x != 0.0 || a.y != 0.0)) {
      int n0;
      int64_t K;
      shift_of(kp, s, &n0, &K);
      v = cmul(a, shift_phase(sy[(size_t)e * d2 + n0], K, kp.NB));
    }
    put_row<T>(kp, slot, 2 * P0 + e, s, v);
  }
  if (n & 1)
    for (int s = threadIdx.x; s < S1; s += kWG) put_row<T>(kp, slot, 2 * P0 + n, s, cmk<double>(0, 0));
  __syncthreads();
  if (only_dirty) {
    for (int e = threadIdx.x; e < n; e += kWG) dirty[e] = 0;
    __syncthreads();
  }
}

// ------------------------------------------------------------ sampling ----
// Line sampler for round st.i with prime st.p along axis st.m0 (0-based):
// writes V[s][h] = f(t_h) + noise for all sets, f the planted signal (rows
// [0, 2 P0)), minus g(t_h) (registry rows [2 P0, 2 P0 + 2 ceil(nslots / 2)))
// when the residual is subtracted from the samples; otherwise the registry is
// subtracted after the DFT (subtract_registry).
// grp / ngrp: ngrp work-groups share the line, this one computing its share of
// the points (see expsum_mfma); noise = false leaves the noise to the caller.
// HALF (FP32): the twiddle table holds only omega_p^x for x <= p/2 (plans whose lines
// are too long for the whole table next to the staged A fragments).
template <typename T, int RT, bool HALF = false>
__device__ void sample_round(const KParams& kp, const KBatch& kb, char* slot, WgState& st,
                             int P0, char* lds, cpx<T>* V, int vstride, int grp = 0,
                             int ngrp = 1, bool noise = true) {
  const int p = st.p, m0 = st.m0, d2 = kp.d2;
  const int nreg = (kp.residual == 1) ? st.nslots : 0;
  const int npairs = P0 + (nreg + 1) / 2;
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(lds);
  // residues and column steps fit 16 bits (p <= 16384)
  const int msm = sampler_m_max(kp);
  // LDS: twiddle table [p_max, or p_max / 2 + 1] | residues | column steps | A stage
  const size_t ntab = HALF ? (size_t)(kp.p_max / 2 + 1) : (size_t)kp.p_max;
  uint16_t* rr = reinterpret_cast<uint16_t*>(lds + align16(ntab * sizeof(cpx<T>)));
  uint16_t* rs = reinterpret_cast<uint16_t*>(reinterpret_cast<char*>(rr) +
                                             align16(2 * (size_t)(msm + 4)));
  float* abuf = reinterpret_cast<float*>(reinterpret_cast<char*>(rs) +
                                         align16(2 * (size_t)(msm + 4)));
  const int64_t* ypl = reinterpret_cast<const int64_t*>(slot + kp.lay.ypl);
  const int64_t* ry = reg_y(kp, slot, st.sb);
  const int ntw = HALF ? p / 2 + 1 : p;
  for (int x = threadIdx.x; x < ntw; x += kWG) {
    double c, s;
    expipi(2.0 * (double)x / (double)p, &c, &s);  // omega_p^x = exp(2 pi i x / p)
    tw[x] = cmk<T>((T)c, (T)s);
  }
  // four residues per thread at a time: their coordinate loads in flight together
  const int nrr = 2 * npairs + 4;
  for (int j0 = threadIdx.x; j0 < nrr; j0 += 4 * kWG) {
    int64_t yv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = j0 + u * kWG;
      yv[u] = 0;
      if (j < st.M_pl)
        yv[u] = ypl[(size_t)j * d2 + m0];
      else if (j < nrr && j >= 2 * P0 && j - 2 * P0 < nreg)
        yv[u] = ry[(size_t)(j - 2 * P0) * d2 + m0];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = j0 + u * kWG;
      if (j < nrr) {
        const int r = (int)pmod64(yv[u], p);
        rr[j] = (uint16_t)r;
        rs[j] = (uint16_t)((16 * r) % p);
      }
    }
  }
  __syncthreads();
  if constexpr (sizeof(T) == 4) {
    const float* af = reinterpret_cast<const float*>(slot + kp.lay.afrag);
    // RT * NT accumulator tiles per wave: at most 24 (96 accumulator registers)
    constexpr int NTMAX = (RT <= 3) ? 8 : (RT <= 6) ? 4 : 2;
    const int nt_plan = kp.sched_nt[nt_band(p)];
    const int nt = min(nt_plan > 0 ? nt_plan : choose_nt(p), NTMAX);
    const cpx<float>* twc = (const cpx<float>*)tw;
    cpx<float>* Vf = (cpx<float>*)V;
#define SFFT_EXPSUM(NTV)                                                                   \
  expsum_mfma<RT, (NTV <= NTMAX ? NTV : NTMAX), HALF>(af, rr, rs, twc, abuf, npairs, p, kp.S1, \
                                                      Vf, vstride, grp, ngrp)
    // widths above NTMAX are never taken (nt <= NTMAX) and not instantiated
    switch (nt) {
      case 8: if constexpr (NTMAX >= 8) SFFT_EXPSUM(8); break;
      case 7: if constexpr (NTMAX >= 7) SFFT_EXPSUM(7); break;
      case 6: if constexpr (NTMAX >= 6) SFFT_EXPSUM(6); break;
      case 5: if constexpr (NTMAX >= 5) SFFT_EXPSUM(5); break;
      case 4: if constexpr (NTMAX >= 4) SFFT_EXPSUM(4); break;
      case 3: if constexpr (NTMAX >= 3) SFFT_EXPSUM(3); break;
      default: SFFT_EXPSUM(2); break;
    }
#undef SFFT_EXPSUM
  } else {
    const cpx<double>* cc = reinterpret_cast<const cpx<double>*>(slot + kp.lay.ccomp);
    const cpx<double>* twd = (const cpx<double>*)tw;
    cpx<double>* Vd = (cpx<double>*)V;
    cpx<double>* stage = reinterpret_cast<cpx<double>*>(abuf);
    // short lines (p <= 64): one point per lane, so that fewer lanes idle past p
    const int sb = f64_set_block(kp.S1);
    const int M2 = 2 * npairs;
    if (p <= 64) {
      if (sb == 4)
        expsum_f64_tiled<4, 1>(cc, rr, twd, stage, M2, p, kp.S1, Vd, vstride, grp, ngrp);
      else if (sb == 3)
        expsum_f64_tiled<3, 1>(cc, rr, twd, stage, M2, p, kp.S1, Vd, vstride, grp, ngrp);
      else
        expsum_f64_tiled<2, 1>(cc, rr, twd, stage, M2, p, kp.S1, Vd, vstride, grp, ngrp);
    } else if (sb == 4) {
      expsum_f64_tiled<4, 4>(cc, rr, twd, stage, M2, p, kp.S1, Vd, vstride, grp, ngrp);
    } else if (sb == 3) {
      expsum_f64_tiled<3, 4>(cc, rr, twd, stage, M2, p, kp.S1, Vd, vstride, grp, ngrp);
    } else {
      expsum_f64_tiled<2, 4>(cc, rr, twd, stage, M2, p, kp.S1, Vd, vstride, grp, ngrp);
    }
  }
  __syncthreads();
  if (noise) {
    add_noise<T>(V, vstride, p, 0, kp.S1, kb.seed, (uint64_t)st.sig, st.i, st.sigma);
    __syncthreads();
  }
}

// The prime-length DFTs of sets grp, grp + ngrp, ... of a round (defined with the DFT
// step below).
template <typename T>
__device__ __noinline__ void dft_sets(const KParams& kp, const WgState& st, char* lds, cpx<T>* V,
                                      int vstride, int nsets, cpx<T>* chirp, cpx<T>* bhat,
                                      cpx<T>* G, int grp, int ngrp, bool noise, uint64_t seed);

// The S+1 (or `nsets`) DFTs of a round with the slot's Bluestein tables and parts buffer.
template <typename T>
__device__ __forceinline__ void dft_round(const KParams& kp, char* slot, WgState& st, char* lds,
                                          cpx<T>* V, int vstride, int nsets) {
  dft_sets<T>(kp, st, lds, V, vstride, nsets, ws_cpx<T>(slot, kp.lay.chirp),
              ws_cpx<T>(slot, kp.lay.bhat), ws_cpx<T>(slot, kp.lay.big), 0, 1, false, 0);
}

// The n (<= NMAX) twiddles omega_p^{((h0 + u) r) mod p}, u < n, of one mode of the
// verification sums (table `tw` of p points in LDS).
template <typename T, int NMAX>
__device__ __forceinline__ void verify_twiddles(const cpx<T>* tw, uint32_t h0, uint32_t r, int p,
                                                float inv_p, int n, cpx<T>* t) {
  uint32_t idx = mulmod24(h0, r, (uint32_t)p, inv_p);
#pragma unroll
  for (int u = 0; u < NMAX; ++u) {
    if (u < n) {
      t[u] = tw[idx];
      const uint32_t nx = idx + r;
      idx = min(nx, nx - (uint32_t)p);
    }
  }
}

// Verification samples (the check at |R| = k): the residual, planted modes
// minus registry, on the tilted line t_h = (h/p) U v, v_n = q^(n-1) mod p, so
// the bucket of a mode is (y . v) mod p, exact in integers:
//   V[h] = sum_j C[j][0] omega_p^{(h r_j) mod p} - sum_e a_e omega_p^{(h r_e) mod p},
// then noise (set 0 of round st.i) and the DFT of that one sequence.  Writes
// the number of buckets with |F[h]| >= verify_eta p to st.ncand.  `extra`
// (NULL in the recovery kernel): samples added before the DFT -- the caller's
// f(t_h) in a session, where there are no planted modes.
template <typename T>
__device__ void verify_round(const KParams& kp, const KBatch& kb, char* slot, WgState& st,
                            char* lds, cpx<T>* V, int* sh_part, const cpx<T>* extra,
                            int part_mode = 0, int h_lo = 0, int h_hi = 0) {
  const int p = st.p, d2 = kp.d2;
  const int M = st.M_pl + st.nslots;
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(lds);
  // LDS: twiddles [p] | residues [m_max + 4] | coefficients [m_max] | partial sums
  uint16_t* rr = reinterpret_cast<uint16_t*>(lds + align16((size_t)p * sizeof(cpx<T>)));
  cpx<T>* coef = reinterpret_cast<cpx<T>*>(reinterpret_cast<char*>(rr) +
                                           align16(2 * (size_t)(kp.m_max + 4)));
  cpx<T>* part = coef + kp.m_max;
  const int64_t* ypl = reinterpret_cast<const int64_t*>(slot + kp.lay.ypl);
  const int64_t* ry = reg_y(kp, slot, st.sb);
  const double2* ra = reg_a(kp, slot, st.sb);
  const cpx<T>* cc = ws_cpx<T>(slot, kp.lay.ccomp);
  const int64_t q = 1 + (st.i % (p - 1));
  // part_mode 1: only the sums of points h_lo .. h_hi - 1 (one group of the
  // several-groups sampling launch); 2: only what follows the sums (noise, DFT, count)
  if (part_mode != 2) {
    for (int x = threadIdx.x; x < p; x += kWG) {
      double c, sn;
      expipi(2.0 * (double)x / (double)p, &c, &sn);
      tw[x] = cmk<T>((T)c, (T)sn);
    }
    const double inv_pd = 1.0 / (double)p;
    for (int j = threadIdx.x; j < M; j += kWG) {
      const int64_t* y = (j < st.M_pl) ? ypl + (size_t)j * d2 : ry + (size_t)(j - st.M_pl) * d2;
      int64_t r = 0, v = 1;
      // the coordinates are read 8 at a time (their loads in flight together), then
      // folded in coordinate order
      constexpr int NB8 = 8;
      for (int n0 = 0; n0 < d2; n0 += NB8) {
        int64_t yv[NB8];
#pragma unroll
        for (int u = 0; u < NB8; ++u) yv[u] = (n0 + u < d2) ? y[n0 + u] : 0;
        if constexpr (sizeof(T) == 4) {
          int r32 = (int)r, v32 = (int)v;
#pragma unroll
          for (int u = 0; u < NB8; ++u) {
            if (n0 + u < d2) {
              r32 = (r32 + v32 * pmod_small(yv[u], p, inv_pd)) % p;
              v32 = (v32 * (int)q) % p;
            }
          }
          r = r32;
          v = v32;
        } else {
#pragma unroll
          for (int u = 0; u < NB8; ++u) {
            if (n0 + u < d2) {
              r = (r + v * pmod64(yv[u], p)) % p;
              v = (v * q) % p;
            }
          }
        }
      }
      rr[j] = (uint16_t)r;
      if (j < st.M_pl) {
        coef[j] = cc[(size_t)j * kp.S1];
      } else {
        const double2 a = ra[j - st.M_pl];
        coef[j] = cmk<T>((T)-a.x, (T)-a.y);
      }
    }
    __syncthreads();
    // G threads per point when p is small; partial sums reduced through LDS.
    // FP32: each thread takes 4 consecutive points (index stepped by r) so one
    // residue and coefficient read feeds 4 products.
    const float inv_p = 1.0f / (float)p;
    int G;
    constexpr int kNpMax = 16;  // points per thread of the long-line form below
    if (part_mode == 1) {
      // this group's points: ceil(n / 256) consecutive points per thread, each point's
      // sum over the modes in order, as in every form below with one thread per point
      // (G = 1, which is what p > 2 * 256 gives)
      const int np = (h_hi - h_lo + kWG - 1) / kWG;
      const int h0 = h_lo + np * (int)threadIdx.x;
      if (h0 < h_hi && np <= 4) {
        // up to 4 points per thread: the coefficient and twiddles of mode j + 1 are read
        // while mode j's products are formed (the sums stay in mode order)
        cpx<T> acc[4], tv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] = cmk<T>(0, 0);
        cpx<T> c = cmk<T>(0, 0);
        if (M > 0) {
          c = coef[0];
          verify_twiddles<T, 4>(tw, (uint32_t)h0, rr[0], p, inv_p, np, tv);
        }
        for (int j = 0; j < M; ++j) {
          const int jn = min(j + 1, M - 1);
          const cpx<T> cn = coef[jn];
          cpx<T> tn[4];
          verify_twiddles<T, 4>(tw, (uint32_t)h0, rr[jn], p, inv_p, np, tn);
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (u < np) acc[u] = cadd(acc[u], cmul(c, tv[u]));
          c = cn;
#pragma unroll
          for (int u = 0; u < 4; ++u) tv[u] = tn[u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (u < np && h0 + u < h_hi) V[h0 + u] = acc[u];
      } else if (h0 < h_hi) {
        cpx<T> acc[kNpMax];
#pragma unroll
        for (int u = 0; u < kNpMax; ++u) acc[u] = cmk<T>(0, 0);
        for (int j = 0; j < M; ++j) {
          const uint32_t r = rr[j];
          const cpx<T> c = coef[j];
          uint32_t idx = mulmod24((uint32_t)h0, r, (uint32_t)p, inv_p);
#pragma unroll
          for (int u = 0; u < kNpMax; ++u) {
            if (u < np) {
              acc[u] = cadd(acc[u], cmul(c, tw[idx]));
              const uint32_t nx = idx + r;
              idx = min(nx, nx - (uint32_t)p);
            }
          }
        }
#pragma unroll
        for (int u = 0; u < kNpMax; ++u)
          if (u < np && h0 + u < h_hi) V[h0 + u] = acc[u];
      }
      __syncthreads();
      return;
    }
    if (sizeof(T) == 4 && p > 4 * kWG && p <= kNpMax * kWG) {
      // lines longer than 4 points per thread: ceil(p / 256) consecutive points on every
      // thread, in one pass (4 points per thread would leave a second pass to a few
      // threads and double the time)
      G = 1;
      const int np = (p + kWG - 1) / kWG;
      const int h0 = np * (int)threadIdx.x;
      if (h0 < p) {
        cpx<T> acc[kNpMax];
#pragma unroll
        for (int u = 0; u < kNpMax; ++u) acc[u] = cmk<T>(0, 0);
        for (int j = 0; j < M; ++j) {
          const uint32_t r = rr[j];
          const cpx<T> c = coef[j];
          uint32_t idx = mulmod24((uint32_t)h0, r, (uint32_t)p, inv_p);
#pragma unroll
          for (int u = 0; u < kNpMax; ++u) {
            if (u < np) {
              acc[u] = cadd(acc[u], cmul(c, tw[idx]));
              const uint32_t nx = idx + r;
              idx = min(nx, nx - (uint32_t)p);
            }
          }
        }
#pragma unroll
        for (int u = 0; u < kNpMax; ++u)
          if (u < np && h0 + u < p) V[h0 + u] = acc[u];
      }
    } else if constexpr (sizeof(T) == 4) {
      const int npg = (p + 3) / 4;
      G = max(1, kWG / npg);
      for (int t = threadIdx.x; t < G * npg; t += kWG) {
        const int h0 = 4 * (t % npg), g = t / npg;
        cpx<T> acc[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] = cmk<T>(0, 0);
        for (int j = g; j < M; j += G) {
          const uint32_t r = rr[j];
          const cpx<T> c = coef[j];
          uint32_t idx = mulmod24((uint32_t)h0, r, (uint32_t)p, inv_p);
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            acc[u] = cadd(acc[u], cmul(c, tw[idx]));
            const uint32_t nx = idx + r;
            idx = min(nx, nx - (uint32_t)p);
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (h0 + u < p) {
            if (G == 1)
              V[h0 + u] = acc[u];
            else
              part[g * p + h0 + u] = acc[u];
          }
        }
      }
    } else {
      G = (p < kWG) ? kWG / p : 1;
      for (int t = threadIdx.x; t < G * p; t += kWG) {
        const int h = t % p, g = t / p;
        cpx<T> acc = cmk<T>(0, 0);
        for (int j = g; j < M; j += G)
          acc = cadd(acc, cmul(coef[j], tw[mulmod((uint32_t)h, (uint32_t)rr[j], p, inv_p)]));
        if (G == 1)
          V[h] = acc;
        else
          part[g * p + h] = acc;
      }
    }
    __syncthreads();
    if (G > 1) {
      for (int h = threadIdx.x; h < p; h += kWG) {
        cpx<T> acc = part[h];
        for (int g = 1; g < G; ++g) acc = cadd(acc, part[g * p + h]);
        V[h] = acc;
      }
      __syncthreads();
    }
  }  // part_mode != 2
  if (extra) {
    for (int h = threadIdx.x; h < p; h += kWG) V[h] = cadd(V[h], extra[h]);
    __syncthreads();
  }
  add_noise<T>(V, kp.vstride, p, 0, 1, kb.seed, (uint64_t)st.sig, st.i, st.sigma);
  __syncthreads();
  dft_round<T>(kp, slot, st, lds, V, kp.vstride, 1);
  const double thr = kp.verify_eta * (double)p;
  int cnt = 0;
  for (int h = threadIdx.x; h < p; h += kWG)
    cnt += (hypot((double)V[h].x, (double)V[h].y) >= thr) ? 1 : 0;
  const int tot = block_sum(cnt, sh_part);
  if (threadIdx.x == 0) st.ncand = tot;
  __syncthreads();
}

// --------------------------------------------------------------- DFTs ------
// The DFTs of sets grp, grp + ngrp, ... (several at a time: batches grp, grp + ngrp,
// ... of `cap` consecutive sets) with this work-group's Bluestein tables and parts
// buffer; `noise`: the sets' noise is added first (several-groups launches, where the
// sampling launch leaves it out).  Every set is transformed the same way whichever
// group takes it.
template <typename T>
__device__ __noinline__ void dft_sets(const KParams& kp, const WgState& st, char* lds, cpx<T>* V,
                                      int vstride,
                         int nsets, cpx<T>* chirp, cpx<T>* bhat, cpx<T>* G, int grp, int ngrp,
                         bool noise, uint64_t seed) {
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(lds);
  constexpr int ML = MaxL<T>::value;
  const int R = st.L > ML ? st.L / ML : 1;  // parts through the slot beyond the LDS maximum
  const int M = st.L / R;
  // sets of short lengths are transformed together, the twiddle tables then sitting
  // after the whole buffer (L_max points, at most the in-LDS maximum) so that up to
  // min(L_max, ML) / L sets fit
  constexpr int MAXV = MaxL<T>::value / kWG;
  const int Lb = min(kp.L_max, ML);
  const bool batched = R == 1 && kp.sched_dft_batch != 1 && st.L <= MAXV * kWG &&
                       2 * st.L <= Lb;
  const BsTabs<T> tb = bs_tables<T>(st.L, M, buf + lds_padded(batched ? Lb : M));
  // s = -1 computes chirp and filter; one call site for every FFT of the step
  for (int s = -1; s < (batched ? 0 : nsets); s = (s < 0 ? grp : s + ngrp)) {
    if (s >= 0 && noise) {
      add_noise<T>(V, vstride, st.p, s, s + 1, seed, (uint64_t)st.sig, st.i, st.sigma);
      __syncthreads();
    }
    bluestein_run<T>(s < 0, s < 0 ? nullptr : V + (size_t)s * vstride, st.p, st.L, R,
                     st.log2L - (R >> 1), chirp, bhat, G, buf, tb, kp.sched_fft);
  }
  if (batched) {
    int cap = min(Lb, MAXV * kWG) / st.L;
    if (kp.sched_dft_batch > 1) cap = min(cap, kp.sched_dft_batch);
    for (int s0 = grp * cap; s0 < nsets; s0 += ngrp * cap) {
      const int g = min(cap, nsets - s0);
      if (noise) {
        add_noise<T>(V, vstride, st.p, s0, s0 + g, seed, (uint64_t)st.sig, st.i, st.sigma);
        __syncthreads();
      }
      bluestein_dft_batch<T, MAXV>(V + (size_t)s0 * vstride, vstride, g, st.p, st.L, st.log2L,
                                   chirp, bhat, buf, tb.T1M, kp.sched_fft);
    }
  }
}


// ------------------------------------------- residual in the spectrum ------
// Adaptive subtraction of the registry (Section 5.0) applied to the spectra:
// by eq. (41) the DFT of g(t) = sum_e a_e exp(2 pi i y_e . t) on the sampling
// line of set s is p sum_{e: y_{e,m} = h mod p} a_e E_s(y_e) in bucket h, with
// E_0 = 1 and E_s = exp(2 pi i eps K_s y_{e,n_s}), so
//   F_s[h] <- F_s[h] - p sum_{e in bucket h} a_e E_s(y_e)
// equals the DFT of the residual samples f - g.  FP64 sums (entries of a
// bucket in registry order), one rounding to T per spectrum value.
// FP32 plans: entries grouped by bucket with a bitonic sort of (bucket, registry
// position) keys, and the shift phases read from the per-slot cache.
__device__ void subtract_registry_f32(const KParams& kp, char* slot, WgState& st, char* lds,
                                      cpx<float>* V, int vstride, int nsets, int* sh_part) {
  const int nR = st.nR;
  const int p = st.p, d2 = kp.d2, m0 = st.m0, S = kp.S;
  const int64_t* sy = reg_y(kp, slot, st.sb);
  const double2* sa = reg_a(kp, slot, st.sb);
  const cpx<float>* sE = reg_E(kp, slot, st.sb);
  const int* ord = reg_ord(kp, slot, st.cur);
  int N2 = 1;
  while (N2 < nR) N2 <<= 1;
  // LDS: bucket start [p + 1] | keys [N2], key = bucket << 16 | registry position,
  // then the slot of each sorted position | coefficients in sorted order [nR]
  int* start = reinterpret_cast<int*>(lds);
  int* key = start + (p + 1);
  double2* asort = reinterpret_cast<double2*>(lds + align16(4 * ((size_t)p + 1 + N2)));
  for (int h = threadIdx.x; h <= p; h += kWG) start[h] = 0;
  __syncthreads();
  const double inv_pd = 1.0 / (double)p;
  for (int e = threadIdx.x; e < N2; e += kWG) {
    if (e < nR) {
      int h = pmod_small(sy[(size_t)ord[e] * d2 + m0], p, inv_pd);
      h = min(max(h, 0), p - 1);
      key[e] = (h << 16) | e;
      atomicAdd(&start[h], 1);
    } else {
      key[e] = 0x7fffffff;
    }
  }
  __syncthreads();
  block_exscan(start, p + 1, sh_part);
  for (int size = 2; size <= N2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < N2 / 2; t += kWG) {
        const int lo_i = 2 * t - (t & (stride - 1));
        const int hi_i = lo_i + stride;
        const bool asc = ((lo_i & size) == 0);
        const int a = key[lo_i], b = key[hi_i];
        if ((a > b) == asc) {
          key[lo_i] = b;
          key[hi_i] = a;
        }
      }
      __syncthreads();
    }
  }
  for (int g = threadIdx.x; g < nR; g += kWG) {
    const int sl = ord[key[g] & 0xffff];
    key[g] = sl;
    asort[g] = sa[sl];
  }
  __syncthreads();
  const double pd = (double)p;
  // set index fastest: neighbouring threads share a bucket's entries and read
  // consecutive cached phases.  U items per thread at a time, so that the
  // phase loads of their first entries are in flight together.
  constexpr int U = 8;
  const int nq = p * nsets;
  for (int q0 = threadIdx.x; q0 < nq; q0 += U * kWG) {
    int hh[U], ss[U], bb0[U], bb1[U];
    cpx<float> E0[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = q0 + u * kWG;
      hh[u] = 0;
      ss[u] = 0;
      bb0[u] = 0;
      bb1[u] = 0;
      E0[u] = cmk<float>(1.f, 0.f);
      if (q < nq) {
        hh[u] = q / nsets;
        ss[u] = q - hh[u] * nsets;
        bb0[u] = start[hh[u]];
        bb1[u] = start[hh[u] + 1];
        if (bb1[u] > bb0[u] && ss[u] > 0) E0[u] = sE[(size_t)key[bb0[u]] * S + ss[u] - 1];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (bb1[u] == bb0[u]) continue;
      const int s = ss[u];
      double ax = 0.0, ay = 0.0;
      for (int g = bb0[u]; g < bb1[u]; ++g) {
        const cpx<float> E = (g == bb0[u]) ? E0[u]
                             : (s > 0 ? sE[(size_t)key[g] * S + s - 1] : cmk<float>(1.f, 0.f));
        const double2 a = asort[g];
        ax += a.x * (double)E.x - a.y * (double)E.y;
        ay += a.x * (double)E.y + a.y * (double)E.x;
      }
      cpx<float>* v = V + (size_t)s * vstride + hh[u];
      *v = cmk<float>((float)((double)v->x - pd * ax), (float)((double)v->y - pd * ay));
    }
  }
  __syncthreads();
}

// FP32 plans whose LDS holds it (kp.sub_cs > 0): the entries are grouped by
// bucket with a counting sort (counts, exclusive scan, placement by atomic cursors,
// then each bucket's few entries put back in registry order), and the sets are
// taken kp.sub_cs at a time: the shift phases of every entry for those sets are
// first copied from the per-slot cache into LDS (independent loads, all in flight
// together), then one item per (bucket, set) sums its entries from LDS.  The sums
// run over each bucket's entries in registry order, as in the sorted form above.
__device__ void subtract_registry_f32_staged(const KParams& kp, char* slot, WgState& st,
                                             char* lds, cpx<float>* V, int vstride, int nsets,
                                             int* sh_part) {
  const int nR = st.nR;
  const int p = st.p, d2 = kp.d2, m0 = st.m0, S = kp.S, CS = kp.sub_cs;
  const int64_t* sy = reg_y(kp, slot, st.sb);
  const double2* sa = reg_a(kp, slot, st.sb);
  const cpx<float>* sE = reg_E(kp, slot, st.sb);
  const int* ord = reg_ord(kp, slot, st.cur);
  // LDS: cursors c[p + 1] | entries grouped by bucket [cap] (registry position, then
  // slot) | coefficients [cap] (first the entries' buckets) | phases [cap][CS]
  int* c = reinterpret_cast<int*>(lds);
  int* list = c + (p + 1);
  double2* asort = reinterpret_cast<double2*>(lds + align16(4 * ((size_t)p + 1 + kp.cap)));
  int* hb = reinterpret_cast<int*>(asort);
  cpx<float>* Es = reinterpret_cast<cpx<float>*>(asort + kp.cap);
  for (int h = threadIdx.x; h <= p; h += kWG) c[h] = 0;
  __syncthreads();
  const double inv_pd = 1.0 / (double)p;
  // four entries per thread at a time: their slot and coordinate loads in flight together
  for (int e0 = threadIdx.x; e0 < nR; e0 += 4 * kWG) {
    int sl[4];
    int64_t yv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) sl[u] = (e0 + u * kWG < nR) ? ord[e0 + u * kWG] : 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) yv[u] = (e0 + u * kWG < nR) ? sy[(size_t)sl[u] * d2 + m0] : 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * kWG;
      if (e < nR) {
        int h = pmod_small(yv[u], p, inv_pd);
        h = min(max(h, 0), p - 1);
        hb[e] = h;
        atomicAdd(&c[h], 1);
      }
    }
  }
  __syncthreads();
  block_exscan(c, p + 1, sh_part);
  // placement: afterwards c[h] is the end of bucket h (the start of bucket h + 1)
  for (int e = threadIdx.x; e < nR; e += kWG) list[atomicAdd(&c[hb[e]], 1)] = e;
  __syncthreads();
  for (int h = threadIdx.x; h < p; h += kWG) {
    const int b0 = (h == 0) ? 0 : c[h - 1], b1 = c[h];
    for (int g = b0 + 1; g < b1; ++g) {
      const int v = list[g];
      int q = g - 1;
      while (q >= b0 && list[q] > v) {
        list[q + 1] = list[q];
        --q;
      }
      list[q + 1] = v;
    }
  }
  __syncthreads();
  for (int g0 = threadIdx.x; g0 < nR; g0 += 4 * kWG) {
    int sl[4];
    double2 av[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) sl[u] = (g0 + u * kWG < nR) ? ord[list[g0 + u * kWG]] : 0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      av[u] = (g0 + u * kWG < nR) ? sa[sl[u]] : make_double2(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int g = g0 + u * kWG;
      if (g < nR) {
        list[g] = sl[u];
        asort[g] = av[u];
      }
    }
  }
  __syncthreads();
  const double pd = (double)p;
  for (int s0 = 0; s0 < nsets; s0 += CS) {
    const int cs = min(CS, nsets - s0);
    // U copies per thread at a time: their global loads are issued together, before
    // any of the LDS stores
    constexpr int U = 8;
    const int nq = nR * cs;
    for (int q0 = threadIdx.x; q0 < nq; q0 += U * kWG) {
      cpx<float> ev[U];
      int dst[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int q = q0 + u * kWG;
        ev[u] = cmk<float>(1.f, 0.f);
        dst[u] = -1;
        if (q < nq) {
          const int g = q / cs, w = q - g * cs;
          dst[u] = g * CS + w;
          if (s0 + w > 0) ev[u] = sE[(size_t)list[g] * S + s0 + w - 1];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (dst[u] >= 0) Es[dst[u]] = ev[u];
    }
    __syncthreads();
    // set index fastest: neighbouring threads read neighbouring phases
    for (int q = threadIdx.x; q < p * cs; q += kWG) {
      const int h = q / cs, u = q - h * cs;
      const int b0 = (h == 0) ? 0 : c[h - 1], b1 = c[h];
      if (b1 == b0) continue;
      double ax = 0.0, ay = 0.0;
      for (int g = b0; g < b1; ++g) {
        const cpx<float> E = Es[(size_t)g * CS + u];
        const double2 a = asort[g];
        ax += a.x * (double)E.x - a.y * (double)E.y;
        ay += a.x * (double)E.y + a.y * (double)E.x;
      }
      cpx<float>* v = V + (size_t)(s0 + u) * vstride + h;
      *v = cmk<float>((float)((double)v->x - pd * ax), (float)((double)v->y - pd * ay));
    }
    __syncthreads();
  }
}

template <typename T>
__device__ void subtract_registry(const KParams& kp, char* slot, WgState& st, char* lds,
                                  cpx<T>* V, int vstride, int nsets, int* sh_part) {
  const int nR = st.nR;
  if (nR == 0) return;
  if constexpr (sizeof(T) == 4) {
    if (kp.sub_cs > 0)
      subtract_registry_f32_staged(kp, slot, st, lds, V, vstride, nsets, sh_part);
    else
      subtract_registry_f32(kp, slot, st, lds, V, vstride, nsets, sh_part);
    return;
  }
  const int p = st.p, d2 = kp.d2, m0 = st.m0;
  const int64_t* sy = reg_y(kp, slot, st.sb);
  const double2* sa = reg_a(kp, slot, st.sb);
  const int* ord = reg_ord(kp, slot, st.cur);
  // LDS: bucket start [p + 1] | entries grouped by bucket [nR] | bucket of entry [nR]
  int* start = reinterpret_cast<int*>(lds);
  int* grp = start + (p + 1);
  int* hb = grp + nR;
  for (int h = threadIdx.x; h <= p; h += kWG) start[h] = 0;
  __syncthreads();
  for (int e = threadIdx.x; e < nR; e += kWG) {
    const int h = (int)pmod64(sy[(size_t)ord[e] * d2 + m0], p);
    hb[e] = h;
    atomicAdd(&start[h], 1);
  }
  __syncthreads();
  block_exscan(start, p + 1, sh_part);
  // deterministic placement: rank of e among the entries of its bucket
  // (registry order), counted by the entries' own scan of their bucket run
  for (int e = threadIdx.x; e < nR; e += kWG) {
    const int h = hb[e];
    int r = 0;
    for (int f = 0; f < e; ++f) r += (hb[f] == h) ? 1 : 0;
    grp[start[h] + r] = e;
  }
  __syncthreads();
  const double pd = (double)p;
  for (int q = threadIdx.x; q < p * nsets; q += kWG) {
    const int h = q % p, s = q / p;
    const int b0 = start[h], b1 = start[h + 1];
    if (b1 == b0) continue;
    int n0 = 0;
    int64_t K = 0;
    if (s > 0) shift_of(kp, s, &n0, &K);
    double ax = 0.0, ay = 0.0;
    for (int g = b0; g < b1; ++g) {
      const int sl = ord[grp[g]];
      double2 a = sa[sl];
      if (s > 0) {
        const cpx<double> E = shift_phase(sy[(size_t)sl * d2 + n0], K, kp.NB);
        a = make_double2(a.x * E.x - a.y * E.y, a.x * E.y + a.y * E.x);
      }
      ax += a.x;
      ay += a.y;
    }
    cpx<T>* v = V + (size_t)s * vstride + h;
    *v = cmk<T>((T)((double)v->x - pd * ax), (T)((double)v->y - pd * ay));
  }
  __syncthreads();
}

// ------------------------------------------------ top-k* selection ---------
// Candidates: buckets with |F_0[h]|/p >= eta, and among them the k* largest
// |F_0| (ties by ascending h), written in ascending h to cand[].
template <typename T>
__device__ void select_round(const KParams& kp, char* slot, WgState& st, char* lds,
                             const cpx<T>* F0, int* sh_part) {
  const int p = st.p;
  // keys: the bits of |F_0| (FP32: 32, FP64: 64), 0 for buckets below the floor
  using Key = typename std::conditional<sizeof(T) == 4, uint32_t, uint64_t>::type;
  Key* keys = reinterpret_cast<Key*>(lds);
  int* flag = reinterpret_cast<int*>(lds + align16((size_t)kp.p_max * sizeof(Key)));
  int* hist = flag + kp.p_max;  // 256 bins
  int* cand = reinterpret_cast<int*>(slot + kp.lay.cand);
  const double thr = kp.eta * (double)p;
  int cnt = 0;
  for (int h = threadIdx.x; h < p; h += kWG) {
    const double mag = hypot((double)F0[h].x, (double)F0[h].y);
    const int pass = (mag >= thr) ? 1 : 0;
    Key key;
    if constexpr (sizeof(T) == 4) {
      key = __float_as_uint((float)mag);
    } else {
      key = (uint64_t)__double_as_longlong(mag);
    }
    keys[h] = pass ? key : (Key)0;
    flag[h] = pass;
    cnt += pass;
  }
  cnt = block_sum(cnt, sh_part);
  if (cnt > st.kstar) {
    // radix select of the k*-th largest key among the passing buckets, 8 bits a
    // pass from the top (FP32 keys have 32 bits, FP64 keys 64)
    if (threadIdx.x == 0) {
      st.prefix = 0ull;
      st.need = st.kstar;
    }
    __syncthreads();
    constexpr int kTopPass = sizeof(T) == 4 ? 3 : 7;
    for (int pass = kTopPass; pass >= 0; --pass) {
      const int shift = pass * 8;
      for (int b = threadIdx.x; b < 256; b += kWG) hist[b] = 0;
      __syncthreads();
      const uint64_t himask = (pass == 7) ? 0ull : ~((1ull << (shift + 8)) - 1ull);
      const uint64_t prefix = st.prefix;
      for (int h = threadIdx.x; h < p; h += kWG) {
        const uint64_t kh = keys[h];
        if (flag[h] && ((kh ^ prefix) & himask) == 0ull)
          atomicAdd(&hist[(int)((kh >> shift) & 255ull)], 1);
      }
      __syncthreads();
      // counts from the top bin down: sh_part[t] = keys in bins >= 255 - t
      // (inclusive scan over the reversed histogram); the first t where it
      // reaches `need` names the bin
      const int need = st.need;
      const int tid = threadIdx.x;
      sh_part[tid] = (tid < 256) ? hist[255 - tid] : 0;
      __syncthreads();
      for (int off = 1; off < kWG; off <<= 1) {
        const int v = (tid >= off) ? sh_part[tid - off] : 0;
        __syncthreads();
        sh_part[tid] += v;
        __syncthreads();
      }
      const int above = (tid == 0) ? 0 : sh_part[tid - 1];
      if (tid < 256 && above < need && sh_part[tid] >= need) {
        st.prefix = prefix | ((uint64_t)(255 - tid) << shift);
        st.need = need - above;
      }
      __syncthreads();
    }
    const uint64_t T_ = st.prefix;
    const int take = st.need;
    // rank among keys equal to the threshold, by ascending h
    for (int h = threadIdx.x; h < p; h += kWG)
      flag[h] = (flag[h] && (uint64_t)keys[h] == T_) ? 1 : 0;
    __syncthreads();
    block_exscan(flag, p, sh_part);
    for (int h = threadIdx.x; h < p; h += kWG) {
      const uint64_t kh = keys[h];
      const bool eq = (kh == T_) && kh != 0ull;
      const bool sel = (kh > T_) || (eq && flag[h] < take);
      flag[h] = sel ? 1 : 0;
    }
    __syncthreads();
  }
  const int n = block_exscan(flag, p, sh_part);
  // flag now holds the output position of each selected h; recompute selection
  for (int h = threadIdx.x; h < p; h += kWG) {
    const int pos = flag[h];
    const int nxt = (h + 1 < p) ? flag[h + 1] : n;
    if (nxt > pos) cand[pos] = h;
  }
  if (threadIdx.x == 0) st.ncand = n;
  __syncthreads();
}

// ------------------------------------------- collision test and decode ------
// LDS carve-up of the decode step: accept flags [k_max] | classifier
// parameters (FP32) | residual-mode counts per bucket [p_max] (export only).

// Ratio F_s[h] / F_0[h] in FP64.
template <typename T>
__device__ __forceinline__ void ratio_of(cpx<T> v, double f0x, double f0y, double den,
                                         double* rx, double* ry) {
  const double fx = (double)v.x;
  const double fy = (double)v.y;
  *rx = (fx * f0x + fy * f0y) / den;
  *ry = (fy * f0x - fx * f0y) / den;
}

template <typename T>
__device__ __forceinline__ void ratio(const cpx<T>* V, int vstride, int s, int h, double f0x,
                                      double f0y, double den, double* rx, double* ry) {
  ratio_of<T>(V[(size_t)s * vstride + h], f0x, f0y, den, rx, ry);
}

// The 8 classifier features of bucket h (see include/sfft.h): ratios of the
// coarse and fine sets of axis m and of the most collision-suspicious other
// axis, with the decoded phase removed, as asinh of their deviation from 1.
template <typename T>
__device__ void bucket_features(const KParams& kp, const cpx<T>* V, int vstride, int h,
                                const int64_t* y, int m0, double f0x, double f0y, float* f) {
  const double den = f0x * f0x + f0y * f0y;
  const bool lad = kp.ladder_K > 1;
  const int d2 = kp.d2;
  auto set_of = [&](int n0, bool fine) { return (fine && lad) ? d2 + n0 + 1 : n0 + 1; };
  int nstar = m0;
  double best = -1.0;
  for (int n0 = 0; n0 < d2; ++n0) {
    if (n0 == m0) continue;
    double rx, ry;
    ratio<T>(V, vstride, set_of(n0, true), h, f0x, f0y, den, &rx, &ry);
    const double dv = fabs(hypot(rx, ry) - 1.0);
    if (dv > best) {
      best = dv;
      nstar = n0;
    }
  }
  const double sc = kp.feat_scale;
  const int ax[4] = {m0, m0, nstar, nstar};
  for (int q = 0; q < 4; ++q) {
    const bool fine = (q & 1) != 0;
    const int64_t K = (fine && lad) ? kp.ladder_K : 1;
    double rx, ry;
    ratio<T>(V, vstride, set_of(ax[q], fine), h, f0x, f0y, den, &rx, &ry);
    const int64_t qq = pmod64(K * y[ax[q]], 2 * kp.NB);
    double c, sn;
    expipi(-(double)qq / (double)kp.NB, &c, &sn);
    const double zx = rx * c - ry * sn, zy = rx * sn + ry * c;
    f[2 * q] = (float)asinh((zx - 1.0) / sc);
    f[2 * q + 1] = (float)asinh(zy / sc);
  }
}

// Decode every candidate (eq. (41), ladder refinement; band, residue and
// ladder-consistency checks), then accept it by the ratio-magnitude test of
// eq. (42) (| |F_s[h]| / |F_0[h]| - 1 | < tau (+ tau_noise sqrt(p) / |F_0[h]|)
// for every shifted set) or by the learned classifier; a = F_0[h] / p.  FP64.
template <typename T>
__device__ void decode_round(const KParams& kp, const KOut& ko, char* slot, WgState& st,
                             const cpx<T>* V, int vstride, char* lds, int* sh_part) {
  int* acc_list = reinterpret_cast<int*>(lds);
  float* Wl = reinterpret_cast<float*>(lds + decode_lds_w(kp.k_max));
  const int* cand = reinterpret_cast<const int*>(slot + kp.lay.cand);
  int64_t* acc_y = reinterpret_cast<int64_t*>(slot + kp.lay.acc_y);
  double2* acc_a = reinterpret_cast<double2*>(slot + kp.lay.acc_a);
  int* acc_ok = reinterpret_cast<int*>(slot + kp.lay.acc_ok);
  float* ftmp = reinterpret_cast<float*>(slot + kp.lay.feat_tmp);
  const bool use_mlp = kp.classifier == 1;
  const bool exporting = ko.feat != nullptr;
  if (use_mlp) mlp_load(kp.mlp_w, Wl);
  const int p = st.p, d2 = kp.d2, S = kp.S;
  const int64_t NB = kp.NB;
  const double NBd = (double)NB;
  // coordinate n lies in [band[2n], band[2n+1]]
  for (int c = threadIdx.x; c < st.ncand; c += kWG) {
    const int h = cand[c];
    const double f0x = (double)V[h].x, f0y = (double)V[h].y;
    const double den = f0x * f0x + f0y * f0y;
    int64_t* y = acc_y + (size_t)c * d2;
    bool valid = true;
    const bool lad = kp.ladder_K > 1;
    // the values of coordinate n + 1 are loaded before coordinate n is decoded, so
    // that their latency overlaps its arithmetic (V is only read here)
    cpx<T> vc = V[(size_t)vstride + h];
    cpx<T> vf = lad ? V[(size_t)(d2 + 1) * vstride + h] : cmk<T>((T)0, (T)0);
    for (int n = 0; n < d2; ++n) {
      cpx<T> vc1 = vc, vf1 = vf;
      if (n + 1 < d2) {
        vc1 = V[(size_t)(n + 2) * vstride + h];
        if (lad) vf1 = V[(size_t)(d2 + n + 2) * vstride + h];
      }
      double rx, ry;
      ratio_of<T>(vc, f0x, f0y, den, &rx, &ry);
      double th = atan2(ry, rx);
      if (th >= M_PI) th = -M_PI;
      const double yc_real = th * NBd / M_PI;
      int64_t yn = llround(yc_real);
      if (lad) {
        const int64_t K = kp.ladder_K;
        double sx, sy;
        ratio_of<T>(vf, f0x, f0y, den, &sx, &sy);
        double thf = atan2(sy, sx);
        if (thf >= M_PI) thf = -M_PI;
        const int64_t q = pmod64(K * yn, 2 * NB);
        double delta = thf - M_PI * (double)q / NBd;
        delta = delta - 2.0 * M_PI * floor((delta + M_PI) / (2.0 * M_PI));
        yn = yn + llround(delta * NBd / (M_PI * (double)K));
        if (kp.robust && fabs(yc_real - (double)yn) > NBd / (4.0 * (double)K)) valid = false;
      }
      if (yn < kp.band[2 * n] || yn > kp.band[2 * n + 1]) valid = false;
      y[n] = yn;
      vc = vc1;
      vf = vf1;
    }
    if (kp.tilt && valid) {
      // tilted: y must be U^T w for an integer w in the box (U y divisible by c^2)
      const int64_t u0 = kp.tb * y[0] + kp.ta * y[1], u1 = kp.tb * y[1] - kp.ta * y[0];
      if (u0 % kp.tc2 != 0 || u1 % kp.tc2 != 0) {
        valid = false;
      } else {
        const int64_t w0 = u0 / kp.tc2, w1 = u1 / kp.tc2;
        if (w0 < -(kp.N / 2) || w0 >= kp.N / 2 || w1 < -(kp.N / 2) || w1 >= kp.N / 2) valid = false;
      }
    }
    if (kp.robust && pmod64(y[st.m0], p) != h) valid = false;
    bool ok;
    float f[kMlpIn];
    if (use_mlp || exporting) bucket_features<T>(kp, V, vstride, h, y, st.m0, f0x, f0y, f);
    if (use_mlp) {
      float xb[kMlpIn];
      for (int i = 0; i < kMlpIn; ++i) xb[i] = bf16_round(f[i]);
      ok = valid && (double)mlp_prob(Wl, xb) > kp.mlp_thr;
    } else {
      const double absF0 = sqrt(den);
      double thr = kp.tau;
      if (kp.tau_noise > 0.0) thr += kp.tau_noise * sqrt((double)p) / absF0;
      ok = valid;
      cpx<T> vs = ok ? V[(size_t)vstride + h] : cmk<T>((T)0, (T)0);
      for (int s = 1; s <= S && ok; ++s) {
        const cpx<T> vn = (s < S) ? V[(size_t)(s + 1) * vstride + h] : vs;
        double rx, ry;
        ratio_of<T>(vs, f0x, f0y, den, &rx, &ry);
        if (!(fabs(hypot(rx, ry) - 1.0) < thr)) ok = false;
        vs = vn;
      }
    }
    if (exporting) {
      for (int i = 0; i < kMlpIn; ++i) ftmp[(size_t)c * kMlpIn + i] = f[i];
    }
    acc_list[c] = ok ? 1 : 0;
    acc_ok[c] = ok ? 1 : 0;
    acc_a[c] = make_double2(f0x / (double)p, f0y / (double)p);
  }
  __syncthreads();
}

// Number accepted and their ranks (ascending h) in acc_list.
__device__ inline void decode_finish(const KParams& kp, WgState& st, char* lds, int* sh_part) {
  int* acc_list = reinterpret_cast<int*>(lds);
  const int n = block_exscan(acc_list, st.ncand, sh_part);
  if (threadIdx.x == 0) st.nacc = n;
  __syncthreads();
}

// lower_bound of row y among n rows (lexicographic order); rows given directly
// or through an index permutation.
__device__ inline int lower_bound_rows(const int64_t* rows, const int* perm, int n, int w,
                                       const int64_t* y) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const int r = perm ? perm[mid] : mid;
    if (lexcmp(rows + (size_t)r * w, y, w) < 0)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// The merge and sort arrays: in LDS, or in the signal's workspace slot when
// they would be the largest LDS consumer of the plan (large k_max).  Offset 0
// (the accept-flag scan) always stays in LDS.
__device__ __forceinline__ char* merge_base(const KParams& kp, char* slot, char* lds) {
  return kp.merge_global ? slot + kp.lay.merge : lds;
}

// Export: planted modes sorted lexicographically once per signal (bitonic
// sort of indices in LDS), for the residual-mode counts of the labels.
__device__ void export_sort_planted(const KParams& kp, char* slot, WgState& st, char* lds) {
  const MergeLds ml = merge_lds(kp.k_max, kp.cap);
  char* mb = merge_base(kp, slot, lds);
  int* ids = reinterpret_cast<int*>(mb + ml.ids);
  int64_t* key0 = reinterpret_cast<int64_t*>(mb + ml.key0);
  const int64_t* ypl = reinterpret_cast<const int64_t*>(slot + kp.lay.ypl);
  int* out = reinterpret_cast<int*>(slot + kp.lay.pl_sorted);
  const int n = st.M_pl, d2 = kp.d2;
  int N2 = 1;
  while (N2 < n) N2 <<= 1;
  for (int q = threadIdx.x; q < N2; q += kWG) {
    ids[q] = q < n ? q : 0x7fffffff;
    key0[q] = q < n ? ypl[(size_t)q * d2] : INT64_MAX;
  }
  __syncthreads();
  for (int size = 2; size <= N2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < N2 / 2; t += kWG) {
        const int lo_i = 2 * t - (t & (stride - 1));
        const int hi_i = lo_i + stride;
        const bool asc = ((lo_i & size) == 0);
        const int a = ids[lo_i], b = ids[hi_i];
        int cmp;
        if (key0[lo_i] != key0[hi_i]) {
          cmp = key0[lo_i] < key0[hi_i] ? -1 : 1;
        } else if (a == 0x7fffffff || b == 0x7fffffff) {
          cmp = (a == b) ? 0 : (a < b ? -1 : 1);
        } else {
          cmp = lexcmp(ypl + (size_t)a * d2, ypl + (size_t)b * d2, d2);
          if (cmp == 0) cmp = (a < b) ? -1 : (a > b ? 1 : 0);
        }
        if ((cmp > 0) == asc) {
          ids[lo_i] = b;
          ids[hi_i] = a;
          const int64_t k0 = key0[lo_i];
          key0[lo_i] = key0[hi_i];
          key0[hi_i] = k0;
        }
      }
      __syncthreads();
    }
  }
  for (int q = threadIdx.x; q < n; q += kWG) out[q] = ids[q];
  __syncthreads();
}

// Export: label of each candidate = exactly one residual mode (planted minus
// the registry, |coefficient| >= eta) in its bucket; then one record per
// candidate (features, label, signal, round, bucket, accepted).
__device__ void export_round(const KParams& kp, const KBatch& kb, const KOut& ko, char* slot,
                             WgState& st, char* lds) {
  int* cnt = reinterpret_cast<int*>(lds + decode_lds_cnt(kp.k_max));
  const int p = st.p, d2 = kp.d2, m0 = st.m0;
  const int64_t* ypl = reinterpret_cast<const int64_t*>(slot + kp.lay.ypl);
  const int* psort = reinterpret_cast<const int*>(slot + kp.lay.pl_sorted);
  const int64_t* ry = reg_y(kp, slot, st.sb);
  const double2* ra = reg_a(kp, slot, st.sb);
  const int* ord = reg_ord(kp, slot, st.cur);
  const int* cand = reinterpret_cast<const int*>(slot + kp.lay.cand);
  const int* acc_ok = reinterpret_cast<const int*>(slot + kp.lay.acc_ok);
  const float* ftmp = reinterpret_cast<const float*>(slot + kp.lay.feat_tmp);
  for (int h = threadIdx.x; h < p; h += kWG) cnt[h] = 0;
  __syncthreads();
  for (int j = threadIdx.x; j < st.M_pl; j += kWG) {
    const int64_t* yj = ypl + (size_t)j * d2;
    const int pos = lower_bound_rows(ry, ord, st.nR, d2, yj);
    bool present = true;
    if (pos < st.nR && lexcmp(ry + (size_t)ord[pos] * d2, yj, d2) == 0) {
      const double rx = kb.coeffs[2 * (st.off + j)] - ra[ord[pos]].x;
      const double ryy = kb.coeffs[2 * (st.off + j) + 1] - ra[ord[pos]].y;
      present = hypot(rx, ryy) >= kp.eta;
    }
    if (present) atomicAdd(&cnt[(int)pmod64(yj[m0], p)], 1);
  }
  for (int e = threadIdx.x; e < st.nR; e += kWG) {
    const int64_t* ye = ry + (size_t)ord[e] * d2;
    const int pos = lower_bound_rows(ypl, psort, st.M_pl, d2, ye);
    const bool planted = pos < st.M_pl && lexcmp(ypl + (size_t)psort[pos] * d2, ye, d2) == 0;
    if (!planted) atomicAdd(&cnt[(int)pmod64(ye[m0], p)], 1);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < st.ncand; c += kWG) {
    const unsigned long long slot_i = atomicAdd((unsigned long long*)ko.count, 1ull);
    if ((int64_t)slot_i < ko.cap) {
      for (int i = 0; i < kMlpIn; ++i) ko.feat[slot_i * kMlpIn + i] = ftmp[(size_t)c * kMlpIn + i];
      ko.label[slot_i] = cnt[cand[c]] == 1 ? 1 : 0;
      ko.meta[slot_i * 4 + 0] = st.sig;
      ko.meta[slot_i * 4 + 1] = st.i;
      ko.meta[slot_i * 4 + 2] = cand[c];
      ko.meta[slot_i * 4 + 3] = acc_ok[c];
    }
  }
  __syncthreads();
}

// ------------------------------------------------------ registry merge ------
// R[y] += a for the accepted buckets (ascending h), then prune |a| < eta.
// Entries keep their slot; the lexicographic order of y is an index array,
// merged by binary search against the accepted entries (sorted, stable).  New
// entries take the next free slots.  When the free slots run out, the live
// entries are first compacted into the other storage bank.  With the residual
// subtracted from the samples, the exponential-sum rows of new, updated and
// pruned slots are rebuilt.
template <typename T>
__device__ void merge_round(const KParams& kp, char* slot, WgState& st, char* lds,
                            int* sh_part, int P0) {
  const int d2 = kp.d2;
  const int nC = st.ncand;
  const MergeLds ml = merge_lds(kp.k_max, kp.cap);
  char* mb = merge_base(kp, slot, lds);
  int* accpos = reinterpret_cast<int*>(lds + ml.accpos);     // exscan of accept flags (LDS)
  int* ids = reinterpret_cast<int*>(mb + ml.ids);            // candidate index, sorted
  int64_t* key0 = reinterpret_cast<int64_t*>(mb + ml.key0);  // first coordinate of y
  int* runflag = reinterpret_cast<int*>(mb + ml.runflag);    // 1 matched run, 2 new run
  int* runpos = reinterpret_cast<int*>(mb + ml.runpos);      // lower_bound in R
  int* cnt = reinterpret_cast<int*>(mb + ml.cnt);            // new runs per position
  int* matchrun = reinterpret_cast<int*>(mb + ml.matchrun);  // run updating entry e
  int* keep = reinterpret_cast<int*>(mb + ml.keep);          // ranks, then prune flags
  const int64_t* acc_y = reinterpret_cast<const int64_t*>(slot + kp.lay.acc_y);
  const double2* acc_a = reinterpret_cast<const double2*>(slot + kp.lay.acc_a);
  int* dirty = reinterpret_cast<int*>(slot + kp.lay.dirty);
  const bool rows = kp.residual == 1;  // registry rows in the exponential sum to keep current
  const int nA = st.nacc;
  const int nR = st.nR;

  // compaction: live entries into slots 0..nR-1 of the other bank
  if (st.nslots + nA > kp.cap) {
    const int nb = st.sb ^ 1;
    const int64_t* y0 = reg_y(kp, slot, st.sb);
    const double2* a0 = reg_a(kp, slot, st.sb);
    int64_t* y1 = reg_y(kp, slot, nb);
    double2* a1 = reg_a(kp, slot, nb);
    int* o = reg_ord(kp, slot, st.cur);
    for (int e = threadIdx.x; e < nR; e += kWG) {
      const int src = o[e];
      for (int i = 0; i < d2; ++i) y1[(size_t)e * d2 + i] = y0[(size_t)src * d2 + i];
      a1[e] = a0[src];
      if (sizeof(T) == 4 && !rows) {
        const cpx<float>* E0 = reg_E(kp, slot, st.sb);
        cpx<float>* E1 = reg_E(kp, slot, nb);
        for (int s = 0; s < kp.S; ++s) E1[(size_t)e * kp.S + s] = E0[(size_t)src * kp.S + s];
      }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nR; e += kWG) o[e] = e;
    if (threadIdx.x == 0) {
      st.sb = nb;
      st.nslots = nR;
    }
    __syncthreads();
    if (rows) rebuild_rows<T>(kp, slot, st, P0, false);
  }
  int64_t* sy = reg_y(kp, slot, st.sb);
  double2* sa = reg_a(kp, slot, st.sb);
  const int cur = st.cur, nxt = cur ^ 1;
  const int* ord = reg_ord(kp, slot, cur);
  int* ord2 = reg_ord(kp, slot, nxt);
  const int ns0 = st.nslots;

  // accepted candidate indices in ascending h
  int N2 = 1;
  while (N2 < nA) N2 <<= 1;
  for (int c = threadIdx.x; c < nC; c += kWG) {
    const int pos = accpos[c];
    const int nextpos = (c + 1 < nC) ? accpos[c + 1] : nA;
    if (nextpos > pos) {
      ids[pos] = c;
      key0[pos] = acc_y[(size_t)c * d2];
    }
  }
  for (int q = nA + threadIdx.x; q < N2; q += kWG) {
    ids[q] = 0x7fffffff;
    key0[q] = INT64_MAX;
  }
  __syncthreads();
  // bitonic sort by (y lexicographic, candidate index); padding sorts last
  for (int size = 2; size <= N2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < N2 / 2; t += kWG) {
        const int lo_i = 2 * t - (t & (stride - 1));
        const int hi_i = lo_i + stride;
        const bool asc = ((lo_i & size) == 0);
        const int a = ids[lo_i], b = ids[hi_i];
        int cmp;
        if (key0[lo_i] != key0[hi_i]) {
          cmp = key0[lo_i] < key0[hi_i] ? -1 : 1;
        } else if (a == 0x7fffffff || b == 0x7fffffff) {
          cmp = (a == b) ? 0 : (a < b ? -1 : 1);
        } else {
          cmp = lexcmp(acc_y + (size_t)a * d2, acc_y + (size_t)b * d2, d2);
          if (cmp == 0) cmp = (a < b) ? -1 : (a > b ? 1 : 0);
        }
        if ((cmp > 0) == asc) {
          ids[lo_i] = b;
          ids[hi_i] = a;
          const int64_t k0 = key0[lo_i];
          key0[lo_i] = key0[hi_i];
          key0[hi_i] = k0;
        }
      }
      __syncthreads();
    }
  }
  // runs of equal y; lower_bound of each run in the registry order
  for (int e = threadIdx.x; e <= nR; e += kWG) cnt[e] = 0;
  for (int e = threadIdx.x; e < nR; e += kWG) matchrun[e] = -1;
  __syncthreads();
  for (int u = threadIdx.x; u < nA; u += kWG) {
    const int64_t* yu = acc_y + (size_t)ids[u] * d2;
    const bool first = (u == 0) || lexcmp(acc_y + (size_t)ids[u - 1] * d2, yu, d2) != 0;
    int flagv = 0, pos = 0;
    if (first) {
      pos = lower_bound_rows(sy, ord, nR, d2, yu);
      const bool matched = (pos < nR) && lexcmp(sy + (size_t)ord[pos] * d2, yu, d2) == 0;
      if (matched) {
        flagv = 1;
        matchrun[pos] = u;
      } else {
        flagv = 2;
        atomicAdd(&cnt[pos], 1);
      }
    }
    runflag[u] = flagv;
    runpos[u] = pos;
  }
  __syncthreads();
  // unmatched ranks (keep[] as scratch of nA ints)
  for (int u = threadIdx.x; u < nA; u += kWG) keep[u] = (runflag[u] == 2) ? 1 : 0;
  __syncthreads();
  const int nU = block_exscan(keep, nA, sh_part);
  block_exscan(cnt, nR + 1, sh_part);
  // old entries move to e + #new runs with pos <= e; matched ones add their run
  for (int e = threadIdx.x; e < nR; e += kWG) {
    const int dst = e + cnt[e + 1];
    const int se = ord[e];
    ord2[dst] = se;
    const int u0 = matchrun[e];
    if (u0 >= 0) {
      double ax = sa[se].x, ay = sa[se].y;
      const int64_t* yu = acc_y + (size_t)ids[u0] * d2;
      for (int u = u0; u < nA && lexcmp(acc_y + (size_t)ids[u] * d2, yu, d2) == 0; ++u) {
        ax += acc_a[ids[u]].x;
        ay += acc_a[ids[u]].y;
      }
      sa[se] = make_double2(ax, ay);
      if (rows) dirty[se] = 1;
    }
  }
  // new entries take slots ns0 + rank
  for (int u = threadIdx.x; u < nA; u += kWG) {
    if (runflag[u] != 2) continue;
    const int sl = ns0 + keep[u];
    const int64_t* yu = acc_y + (size_t)ids[u] * d2;
    for (int i = 0; i < d2; ++i) sy[(size_t)sl * d2 + i] = yu[i];
    double ax = 0.0, ay = 0.0;
    for (int v = u; v < nA && lexcmp(acc_y + (size_t)ids[v] * d2, yu, d2) == 0; ++v) {
      ax += acc_a[ids[v]].x;
      ay += acc_a[ids[v]].y;
    }
    sa[sl] = make_double2(ax, ay);
    if (rows) dirty[sl] = 1;
    ord2[runpos[u] + keep[u]] = sl;
  }
  __syncthreads();
  // FP32 spectrum plans: shift phases of the new slots for subtract_registry
  if (sizeof(T) == 4 && !rows) {
    cpx<float>* sE = reg_E(kp, slot, st.sb);
    // U phases per thread at a time, their coordinate loads issued together
    constexpr int U = 4;
    const int nq = nU * kp.S;
    for (int q0 = threadIdx.x; q0 < nq; q0 += U * kWG) {
      int64_t yv[U], Kv[U];
      int dst[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int q = q0 + u * kWG;
        yv[u] = 0;
        Kv[u] = 0;
        dst[u] = -1;
        if (q < nq) {
          const int sl = ns0 + q / kp.S, s = 1 + q % kp.S;
          int n0;
          shift_of(kp, s, &n0, &Kv[u]);
          yv[u] = sy[(size_t)sl * d2 + n0];
          dst[u] = sl * kp.S + s - 1;
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (dst[u] < 0) continue;
        // exp(i pi q / NB), q = K y mod 2 NB exact; the FP32 phase is what is stored
        const int64_t qq = pmod64(Kv[u] * yv[u], 2 * kp.NB);
        float sn, cs;
        sincospif((float)((double)qq / (double)kp.NB), &sn, &cs);
        sE[dst[u]] = cmk<float>(cs, sn);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) st.nslots = ns0 + nU;
  // prune |a| < eta: zero coefficient (rows rebuilt as zero), dropped from the order
  const int nM = nR + nU;
  int npr = 0;
  for (int e = threadIdx.x; e < nM; e += kWG) {
    const int se = ord2[e];
    const int k = (hypot(sa[se].x, sa[se].y) >= kp.eta) ? 1 : 0;
    if (!k) {
      sa[se] = make_double2(0.0, 0.0);
      if (rows) dirty[se] = 1;
    }
    keep[e] = k;
    npr += 1 - k;
  }
  npr = block_sum(npr, sh_part);
  if (npr == 0) {
    if (threadIdx.x == 0) {
      st.cur = nxt;
      st.nR = nM;
    }
  } else {
    const int nK = block_exscan(keep, nM, sh_part);
    int* o = reg_ord(kp, slot, cur);
    for (int e = threadIdx.x; e < nM; e += kWG) {
      const int pos = keep[e];
      const int nx = (e + 1 < nM) ? keep[e + 1] : nK;
      if (nx > pos) o[pos] = ord2[e];
    }
    if (threadIdx.x == 0) st.nR = nK;
  }
  __syncthreads();
  if (rows) rebuild_rows<T>(kp, slot, st, P0, true);
}

// ------------------------------------------------------------- output ------
// Wrap y back to w with balanced base-N digits (inverse of eq. (35), over the
// blocks and coordinate order of the partition) and write the registry in
// lexicographic order of w.
__device__ void write_output(const KParams& kp, const KOut& ko, char* slot, WgState& st,
                                    char* lds) {
  if (ko.freqs == nullptr) {  // feature export only: no recovery outputs
    __syncthreads();
    return;
  }
  const int d = kp.d, d2 = kp.d2, nR = st.nR;
  const int64_t* ry = reg_y(kp, slot, st.sb);
  const double2* ra = reg_a(kp, slot, st.sb);
  const int* ord = reg_ord(kp, slot, st.cur);
  int64_t* fo = ko.freqs + (size_t)st.sig * kp.k_max * d;
  double* co = ko.coeffs + (size_t)st.sig * kp.k_max * 2;
  const int nOut = min(nR, kp.k_max);
  const int64_t half = kp.N / 2;
  // entries in registry order first (lexicographic in y): into the output when that is
  // also the order of w, else into wtmp to be ranked
  int64_t* wo = kp.wrap_rank ? reinterpret_cast<int64_t*>(slot + kp.lay.wtmp) : fo;
  for (int e = threadIdx.x; e < nOut && kp.tilt; e += kWG) {
    // rotation back, w = U y / c^2 (exact: decode admits only such y)
    const int64_t y0 = ry[(size_t)ord[e] * 2], y1 = ry[(size_t)ord[e] * 2 + 1];
    wo[(size_t)e * 2] = (kp.tb * y0 + kp.ta * y1) / kp.tc2;
    wo[(size_t)e * 2 + 1] = (kp.tb * y1 - kp.ta * y0) / kp.tc2;
  }
  for (int e = threadIdx.x; e < nOut && !kp.tilt; e += kWG) {
    for (int q = 0; q < d2; ++q) {
      int64_t rest = ry[(size_t)ord[e] * d2 + q];
      for (int l = kp.blk[q]; l < kp.blk[q + 1]; ++l) {
        const int64_t digit = pmod64(rest + half, kp.N) - half;
        wo[(size_t)e * d + kp.perm[l]] = digit;
        rest = (rest - digit) / kp.N;
      }
    }
  }
  __syncthreads();
  if (kp.wrap_rank) {
    // rank by lexicographic order of w: a key of the leading coordinates packed into 63
    // bits (each shifted to [0, N)) decides most comparisons in LDS; equal keys compare
    // the rows themselves
    uint64_t* key = reinterpret_cast<uint64_t*>(lds);
    int* rank = reinterpret_cast<int*>(lds + 8 * (size_t)kp.k_max);
    int bits = 1;
    while ((int64_t(1) << bits) < kp.N) ++bits;
    const int nk = min(d, 63 / bits);
    for (int e = threadIdx.x; e < nOut; e += kWG) {
      uint64_t kv = 0;
      for (int i = 0; i < nk; ++i) kv = (kv << bits) | (uint64_t)(wo[(size_t)e * d + i] + half);
      key[e] = kv;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nOut; e += kWG) {
      const uint64_t ke = key[e];
      int rk = 0;
      for (int f = 0; f < nOut; ++f) {
        const uint64_t kf = key[f];
        if (kf < ke || (kf == ke && f != e &&
                        lexcmp(wo + (size_t)f * d + nk, wo + (size_t)e * d + nk, d - nk) < 0))
          ++rk;
      }
      rank[e] = rk;
    }
    __syncthreads();
    for (size_t q = threadIdx.x; q < (size_t)nOut * d; q += kWG) {
      const int e = (int)(q / d), col = (int)(q - (size_t)e * d);
      fo[(size_t)rank[e] * d + col] = wo[q];
    }
    for (int e = threadIdx.x; e < nOut; e += kWG) {
      co[2 * rank[e]] = ra[ord[e]].x;
      co[2 * rank[e] + 1] = ra[ord[e]].y;
    }
  } else {
    for (int e = threadIdx.x; e < nOut; e += kWG) {
      co[2 * e] = ra[ord[e]].x;
      co[2 * e + 1] = ra[ord[e]].y;
    }
  }
  for (int e = nOut + threadIdx.x; e < kp.k_max; e += kWG) {
    for (int i = 0; i < d; ++i) fo[(size_t)e * d + i] = 0;
    co[2 * e] = 0.0;
    co[2 * e + 1] = 0.0;
  }
  if (ko.trace) {
    int32_t* tr = ko.trace + (size_t)st.sig * kp.max_rounds * 8;
    for (int e = (st.i - 1) * 8 + threadIdx.x; e < kp.max_rounds * 8; e += kWG) tr[e] = 0;
  }
  if (threadIdx.x == 0) {
    ko.k_found[st.sig] = nOut;
    ko.status[st.sig] = st.status;
    if (ko.rounds) ko.rounds[st.sig] = st.i - 1;
    if (ko.samples) ko.samples[st.sig] = st.samples;
  }
  __syncthreads();
}

// Phase timestamp (device wall clock, 100 MHz) of the current round, when asked for.
__device__ __forceinline__ void phase_mark(const KParams& kp, const KOut& ko, const WgState& st,
                                           int ph) {
  if (ko.phase && threadIdx.x == 0 && st.i <= kp.max_rounds)
    ko.phase[((size_t)st.sig * kp.max_rounds + (st.i - 1)) * 8 + ph] = (int64_t)wall_clock64();
}

// ---------------------------------------------------------- the kernel ------
template <typename T, int RT>
__global__ void __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(2)))
recover_kernel(KParams kp, KBatch kb, KOut ko) {
  extern __shared__ __align__(16) char lds[];
  __shared__ WgState st;
  __shared__ int sh_part[kWG];
  char* slot = kp.ws + (size_t)blockIdx.x * kp.ws_slot;
  cpx<T>* V = ws_cpx<T>(slot, kp.lay.V);
  const int vstride = kp.vstride;
  for (;;) {
    if (threadIdx.x == 0) st.sig = atomicAdd(kp.queue, 1);
    __syncthreads();
    if (st.sig >= kb.B) break;
    if (threadIdx.x == 0) {
      const int sig = st.sig;
      st.off = kb.mode_off[sig];
      st.M_pl = (int)(kb.mode_off[sig + 1] - st.off);
      st.k = kb.k[sig];
      st.sigma = kb.sigma[sig];
      st.nR = 0;
      st.cur = 0;
      st.sb = 0;
      st.nslots = 0;
      st.i = 1;
      st.samples = 0;
      st.status = 0;
      st.flag = 0;
      if (st.M_pl > kp.k_max || st.M_pl < 0 || st.k < 1 || st.k > kp.k_max) st.flag = 1;
    }
    __syncthreads();
    if (st.flag) {
      if (threadIdx.x == 0 && ko.k_found) {
        ko.k_found[st.sig] = 0;
        ko.status[st.sig] = -1;  // SFFT_EINVAL
        if (ko.rounds) ko.rounds[st.sig] = 0;
        if (ko.samples) ko.samples[st.sig] = 0;
      }
      __syncthreads();
      continue;
    }
    planted_setup<T>(kp, kb, slot, st);
    const int P0 = (st.M_pl + 1) / 2;
    if constexpr (sizeof(T) == 4) {
      scatter_afrag(kp, ws_cpx<float>(slot, kp.lay.ccomp),
                    reinterpret_cast<float*>(slot + kp.lay.afrag), 0, 2 * P0);
      __syncthreads();
    }
    if (ko.feat) export_sort_planted(kp, slot, st, lds);
    if (threadIdx.x == 0) {
      st.kv = 0;
      st.verified = 0;
    }
    __syncthreads();
    while (st.i <= kp.max_rounds) {
      const bool at_k = st.nR >= st.k && st.kv == 0;
      if (at_k && (!kp.verify || st.verified)) break;
      if (threadIdx.x == 0) {
        st.kstar = at_k ? 0 : (st.nR < st.k ? st.k - st.nR : st.kv);
        st.p = prime_for_round(kp, at_k ? 1 : st.kstar, st.i);
        st.m0 = st.i % kp.d2;
        if (st.p < 2 || st.p > kp.p_max) {
          st.flag = 1;
        } else {
          int L = 1, lg = 0;
          while (L < 2 * st.p - 1) {
            L <<= 1;
            ++lg;
          }
          st.L = L;
          st.log2L = lg;
        }
      }
      __syncthreads();
      if (st.flag) {
        if (threadIdx.x == 0) st.status = -2;  // SFFT_ERANGE
        __syncthreads();
        break;
      }
      phase_mark(kp, ko, st, 0);
      if (at_k) {
        verify_round<T>(kp, kb, slot, st, lds, V, sh_part, nullptr);
        phase_mark(kp, ko, st, 6);
        if (threadIdx.x == 0) {
          st.samples += st.p;
          if (ko.trace) {
            int32_t* tr = ko.trace + ((size_t)st.sig * kp.max_rounds + (st.i - 1)) * 8;
            tr[0] = st.i;
            tr[1] = 0;
            tr[2] = st.p;
            tr[3] = 0;
            tr[4] = st.ncand;
            tr[5] = 0;
            tr[6] = st.nR;
            tr[7] = 1;
          }
          st.i += 1;
          if (st.ncand == 0) {
            st.verified = 1;
          } else {
            // the registry grows past k by at most max(16, ceil(k/8)) while repaired
            const int room = st.k + max(16, (st.k + 7) / 8) - st.nR;
            st.kv = min(min(st.ncand, st.k), room);
            if (st.kv <= 0) {
              st.kv = 0;
              st.flag = 2;  // no room: stop with RESIDUAL_NONZERO
            }
          }
        }
        __syncthreads();
        if (st.flag) break;
        continue;
      }
      sample_round<T, RT>(kp, kb, slot, st, P0, lds, V, vstride);
      phase_mark(kp, ko, st, 1);
      dft_round<T>(kp, slot, st, lds, V, vstride, kp.S1);
      phase_mark(kp, ko, st, 2);
      if (kp.residual == 0) subtract_registry<T>(kp, slot, st, lds, V, vstride, kp.S1, sh_part);
      phase_mark(kp, ko, st, 7);
      select_round<T>(kp, slot, st, lds, V, sh_part);
      phase_mark(kp, ko, st, 3);
      decode_round<T>(kp, ko, slot, st, V, vstride, lds, sh_part);
      if (ko.feat) export_round(kp, kb, ko, slot, st, lds);
      decode_finish(kp, st, lds, sh_part);
      phase_mark(kp, ko, st, 4);
      merge_round<T>(kp, slot, st, lds, sh_part, P0);
      phase_mark(kp, ko, st, 5);
      if (threadIdx.x == 0) {
        st.samples += (int64_t)kp.S1 * st.p;
        if (ko.trace) {
          int32_t* tr = ko.trace + ((size_t)st.sig * kp.max_rounds + (st.i - 1)) * 8;
          tr[0] = st.i;
          tr[1] = st.kstar;
          tr[2] = st.p;
          tr[3] = st.m0 + 1;
          tr[4] = st.ncand;
          tr[5] = st.nacc;
          tr[6] = st.nR;
          tr[7] = 0;
        }
        st.kv = 0;
        st.i += 1;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0 && st.status == 0)
      st.status = (st.nR < st.k) ? 1 : (st.nR > st.k || (kp.verify && !st.verified)) ? 2 : 0;
    __syncthreads();
    write_output(kp, ko, slot, st, lds);
  }
}

// ------------------------------------------ several work-groups per signal --
// Batches smaller than the chip (fewer signals than the device holds work-groups)
// run with ngrp work-groups per signal: split_setup_kernel (one work-group per
// signal: the per-signal set-up and the rounds up to the first ordinary one), then
// per ordinary round split_sample_kernel (ngrp work-groups per signal, group g
// sampling every ngrp-th block of column tiles, each point's sum formed as in the
// one-group sampler), for plans with much DFT work per round (split_dft_launch)
// split_dft_kernel (ngrp per signal: the noise and DFTs of every ngrp-th set or
// batch of sets), and split_post_kernel (one per signal: the noise and DFTs when
// they have no launch of their own, subtraction, selection, decode and merge, then
// the rounds up to the next ordinary one).  Verification rounds sample a single
// line and run whole in the one-group kernels.  Signal b uses workspace slot b; its round state stays
// in global memory between launches.  The outputs equal the one-kernel recovery's
// bit for bit.

// recover_kernel's round loop from the current state up to the next ordinary
// round, which is left pending (st.split = 1, prime, axis and length set);
// verification rounds run here whole; a finished signal writes its outputs
// (st.split = 2).
// What a finished verification round leaves in the state: its trace row, the sample
// count, and either the verified flag or the number of buckets to repair (thread 0
// writes; a barrier follows).
__device__ inline void verify_account(const KParams& kp, const KOut& ko, WgState& st) {
  if (threadIdx.x == 0) {
    st.samples += st.p;
    if (ko.trace) {
      int32_t* tr = ko.trace + ((size_t)st.sig * kp.max_rounds + (st.i - 1)) * 8;
      tr[0] = st.i;
      tr[1] = 0;
      tr[2] = st.p;
      tr[3] = 0;
      tr[4] = st.ncand;
      tr[5] = 0;
      tr[6] = st.nR;
      tr[7] = 1;
    }
    st.i += 1;
    if (st.ncand == 0) {
      st.verified = 1;
    } else {
      const int room = st.k + max(16, (st.k + 7) / 8) - st.nR;
      st.kv = min(min(st.ncand, st.k), room);
      if (st.kv <= 0) {
        st.kv = 0;
        st.flag = 2;  // no room: stop with RESIDUAL_NONZERO
      }
    }
  }
  __syncthreads();
}

// A verification line the sampling launch's groups sum (split = 3): FP32 lines of
// 512 to 4096 points, where every one-group form sums each point in one thread.
__host__ __device__ inline bool split_verify_line(const KParams& kp, int p) {
  return kp.precision == 1 && p > 2 * kWG && p <= 16 * kWG;
}

template <typename T>
__device__ void split_advance(const KParams& kp, const KBatch& kb, const KOut& ko, char* slot,
                              WgState& st, char* lds, cpx<T>* V, int* sh_part,
                              bool verify_summed = false) {
  if (verify_summed) {
    // the groups summed this verification line: the rest of the round, then on
    verify_round<T>(kp, kb, slot, st, lds, V, sh_part, nullptr, 2);
    phase_mark(kp, ko, st, 6);
    verify_account(kp, ko, st);
  }
  while (st.flag == 0 && st.i <= kp.max_rounds) {
    const bool at_k = st.nR >= st.k && st.kv == 0;
    if (at_k && (!kp.verify || st.verified)) break;
    if (threadIdx.x == 0) {
      st.kstar = at_k ? 0 : (st.nR < st.k ? st.k - st.nR : st.kv);
      st.p = prime_for_round(kp, at_k ? 1 : st.kstar, st.i);
      st.m0 = st.i % kp.d2;
      if (st.p < 2 || st.p > kp.p_max) {
        st.flag = 1;
      } else {
        int L = 1, lg = 0;
        while (L < 2 * st.p - 1) {
          L <<= 1;
          ++lg;
        }
        st.L = L;
        st.log2L = lg;
      }
    }
    __syncthreads();
    if (st.flag) {
      if (threadIdx.x == 0) st.status = -2;  // SFFT_ERANGE
      __syncthreads();
      break;
    }
    phase_mark(kp, ko, st, 0);
    if (!at_k || split_verify_line(kp, st.p)) {
      if (threadIdx.x == 0) st.split = at_k ? 3 : 1;
      __syncthreads();
      return;
    }
    verify_round<T>(kp, kb, slot, st, lds, V, sh_part, nullptr);
    phase_mark(kp, ko, st, 6);
    verify_account(kp, ko, st);
  }
  if (threadIdx.x == 0 && st.status == 0)
    st.status = (st.nR < st.k) ? 1 : (st.nR > st.k || (kp.verify && !st.verified)) ? 2 : 0;
  __syncthreads();
  write_output(kp, ko, slot, st, lds);
  if (threadIdx.x == 0) st.split = 2;
  __syncthreads();
}

template <typename T, int RT>
__global__ void __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(2)))
split_setup_kernel(KParams kp, KBatch kb, KOut ko, WgState* state) {
  extern __shared__ __align__(16) char lds[];
  __shared__ WgState st;
  __shared__ int sh_part[kWG];
  const int b = blockIdx.x;
  char* slot = kp.ws + (size_t)b * kp.ws_slot;
  cpx<T>* V = ws_cpx<T>(slot, kp.lay.V);
  if (threadIdx.x == 0) {
    WgState z;
    memset(&z, 0, sizeof(z));
    z.sig = b;
    z.off = kb.mode_off[b];
    z.M_pl = (int)(kb.mode_off[b + 1] - z.off);
    z.k = kb.k[b];
    z.sigma = kb.sigma[b];
    z.i = 1;
    if (z.M_pl > kp.k_max || z.M_pl < 0 || z.k < 1 || z.k > kp.k_max) z.flag = 1;
    st = z;
  }
  __syncthreads();
  if (st.flag) {
    if (threadIdx.x == 0) {
      if (ko.k_found) {
        ko.k_found[b] = 0;
        ko.status[b] = -1;  // SFFT_EINVAL
        if (ko.rounds) ko.rounds[b] = 0;
        if (ko.samples) ko.samples[b] = 0;
      }
      st.split = 2;
      state[b] = st;
    }
    return;
  }
  planted_setup<T>(kp, kb, slot, st);
  const int P0 = (st.M_pl + 1) / 2;
  if constexpr (sizeof(T) == 4) {
    scatter_afrag(kp, ws_cpx<float>(slot, kp.lay.ccomp),
                  reinterpret_cast<float*>(slot + kp.lay.afrag), 0, 2 * P0);
    __syncthreads();
  }
  if (ko.feat) export_sort_planted(kp, slot, st, lds);
  split_advance<T>(kp, kb, ko, slot, st, lds, V, sh_part);
  if (threadIdx.x == 0) state[b] = st;
}

template <typename T, int RT>
__global__ void __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(2)))
split_sample_kernel(KParams kp, KBatch kb, const WgState* state, int ngrp) {
  extern __shared__ __align__(16) char lds[];
  __shared__ WgState st;
  const int b = blockIdx.x / ngrp, g = blockIdx.x - b * ngrp;
  if (threadIdx.x == 0) st = state[b];
  __syncthreads();
  if (st.split != 1 && st.split != 3) return;  // uniform over the work-group
  char* slot = kp.ws + (size_t)b * kp.ws_slot;
  cpx<T>* V = ws_cpx<T>(slot, kp.lay.V);
  if (st.split == 3) {
    // a verification line: this group sums its share of the points
    const int chunk = (st.p + ngrp - 1) / ngrp;
    const int lo = min(st.p, g * chunk), hi = min(st.p, lo + chunk);
    verify_round<T>(kp, kb, slot, st, lds, V, nullptr, nullptr, 1, lo, hi);
    return;
  }
  if (sizeof(T) == 4 && kp.tw_half)
    sample_round<T, RT, true>(kp, kb, slot, st, (st.M_pl + 1) / 2, lds, V, kp.vstride, g, ngrp,
                              false);
  else
    sample_round<T, RT>(kp, kb, slot, st, (st.M_pl + 1) / 2, lds, V, kp.vstride, g, ngrp, false);
}

// Noise and DFTs of a round in the several-groups launches: group g of signal b adds
// the noise of, and transforms, sets g, g + ngrp, ... (batches of sets when they are
// transformed several at a time), with its own Bluestein tables and parts buffer
// (`scr`: scr_bytes per work-group).
template <typename T>
__global__ void __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(2)))
split_dft_kernel(KParams kp, KBatch kb, KOut ko, const WgState* state, int ngrp, char* scr,
                 size_t scr_bytes) {
  extern __shared__ __align__(16) char lds[];
  __shared__ WgState st;
  const int b = blockIdx.x / ngrp, g = blockIdx.x - b * ngrp;
  if (threadIdx.x == 0) st = state[b];
  __syncthreads();
  if (st.split != 1) return;  // uniform over the work-group
  char* slot = kp.ws + (size_t)b * kp.ws_slot;
  cpx<T>* V = ws_cpx<T>(slot, kp.lay.V);
  const SplitDftScratch sc = split_dft_scratch(kp);
  char* mine = scr + (size_t)blockIdx.x * scr_bytes;
  if (g == 0) phase_mark(kp, ko, st, 1);  // (the sampling launch)
  dft_sets<T>(kp, st, lds, V, kp.vstride, kp.S1, reinterpret_cast<cpx<T>*>(mine + sc.chirp),
              reinterpret_cast<cpx<T>*>(mine + sc.bhat), reinterpret_cast<cpx<T>*>(mine + sc.big),
              g, ngrp, true, kb.seed);
  if (g == 0) phase_mark(kp, ko, st, 2);
}

template <typename T, int RT>
__global__ void __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(2)))
split_post_kernel(KParams kp, KBatch kb, KOut ko, WgState* state, int dft_here) {
  extern __shared__ __align__(16) char lds[];
  __shared__ WgState st;
  __shared__ int sh_part[kWG];
  const int b = blockIdx.x;
  char* slot = kp.ws + (size_t)b * kp.ws_slot;
  cpx<T>* V = ws_cpx<T>(slot, kp.lay.V);
  const int vstride = kp.vstride;
  if (threadIdx.x == 0) st = state[b];
  __syncthreads();
  if (st.split == 3) {
    // the sampling launch summed a verification line: its noise, DFT and count, then on
    // (split_advance sets st.split again before it returns)
    split_advance<T>(kp, kb, ko, slot, st, lds, V, sh_part, true);
    if (threadIdx.x == 0) state[b] = st;
    return;
  }
  if (st.split != 1) return;
  if (dft_here) {
    add_noise<T>(V, vstride, st.p, 0, kp.S1, kb.seed, (uint64_t)st.sig, st.i, st.sigma);
    __syncthreads();
    phase_mark(kp, ko, st, 1);  // (the sampling launch and the noise)
    dft_round<T>(kp, slot, st, lds, V, vstride, kp.S1);
    phase_mark(kp, ko, st, 2);
  }  // (otherwise split_dft_kernel added the noise and transformed the sets)
  if (kp.residual == 0) subtract_registry<T>(kp, slot, st, lds, V, vstride, kp.S1, sh_part);
  phase_mark(kp, ko, st, 7);
  select_round<T>(kp, slot, st, lds, V, sh_part);
  phase_mark(kp, ko, st, 3);
  decode_round<T>(kp, ko, slot, st, V, vstride, lds, sh_part);
  if (ko.feat) export_round(kp, kb, ko, slot, st, lds);
  decode_finish(kp, st, lds, sh_part);
  phase_mark(kp, ko, st, 4);
  merge_round<T>(kp, slot, st, lds, sh_part, (st.M_pl + 1) / 2);
  phase_mark(kp, ko, st, 5);
  if (threadIdx.x == 0) {
    st.samples += (int64_t)kp.S1 * st.p;
    if (ko.trace) {
      int32_t* tr = ko.trace + ((size_t)st.sig * kp.max_rounds + (st.i - 1)) * 8;
      tr[0] = st.i;
      tr[1] = st.kstar;
      tr[2] = st.p;
      tr[3] = st.m0 + 1;
      tr[4] = st.ncand;
      tr[5] = st.nacc;
      tr[6] = st.nR;
      tr[7] = 0;
    }
    st.kv = 0;
    st.i += 1;
    st.split = 0;
  }
  __syncthreads();
  split_advance<T>(kp, kb, ko, slot, st, lds, V, sh_part);
  if (threadIdx.x == 0) state[b] = st;
}

// ------------------------------------------ caller-supplied samples ------
// A session recovers signals the library cannot evaluate itself: every round
// is one launch, the caller samples f on the lines the session asks for, and
// each signal's round state lives in global memory between launches.  The
// steps after sampling are the recovery kernel's (DFT, registry subtraction in
// the spectra, selection, decode, merge; in a verification round the registry's
// sum on the tilted line, the DFT and the bucket count).  One work-group per
// signal, slot b of the session's workspace for signal b.

// A verification round is due (the recovery kernel's test, the state after a
// round): the registry holds k entries and no repair round is pending.
__device__ __forceinline__ bool session_at_k(const WgState& st) {
  return st.nR >= st.k && st.kv == 0;
}

// The next round of a signal (thread 0): st.p = 0 once it is finished.
__device__ void session_next(const KParams& kp, WgState& st) {
  st.p = 0;
  if (st.flag) return;
  const bool at_k = session_at_k(st);
  if ((at_k && (!kp.verify || st.verified)) || st.i > kp.max_rounds) {
    st.flag = 3;
    return;
  }
  st.kstar = at_k ? 0 : (st.nR < st.k ? st.k - st.nR : st.kv);
  const int p = prime_for_round(kp, at_k ? 1 : st.kstar, st.i);
  st.m0 = st.i % kp.d2;
  if (p < 2 || p > kp.p_max) {
    st.status = -2;  // SFFT_ERANGE
    st.flag = 3;
    return;
  }
  int L = 1, lg = 0;
  while (L < 2 * p - 1) {
    L <<= 1;
    ++lg;
  }
  st.p = p;
  st.L = L;
  st.log2L = lg;
}

// The request: m >= 1 names the axis of an ordinary round; m = -q a verification
// line, v_n = q^(n-1) mod p.
__device__ __forceinline__ void session_publish(const KSess& ss, const WgState& st, int b) {
  ss.req_p[b] = st.p;
  ss.req_m[b] = (st.p > 1 && session_at_k(st)) ? -(1 + (st.i % (st.p - 1))) : st.m0 + 1;
  ss.state[b] = st;
}

template <typename T>
__global__ void __launch_bounds__(kWG) session_init_kernel(KParams kp, KSess ss) {
  __shared__ WgState st;
  const int b = blockIdx.x;
  if (threadIdx.x == 0) {
    WgState z;
    memset(&z, 0, sizeof(z));
    z.sig = b;
    z.k = ss.k[b];
    z.i = 1;
    if (z.k < 1 || z.k > kp.k_max) {
      z.status = -1;  // SFFT_EINVAL
      z.flag = 3;
    }
    st = z;
    session_next(kp, st);
    session_publish(ss, st, b);
  }
}

template <typename T>
__global__ void __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(2)))
session_feed_kernel(KParams kp, KSess ss, const void* samples) {
  extern __shared__ __align__(16) char lds[];
  __shared__ WgState st;
  __shared__ int sh_part[kWG];
  const int b = blockIdx.x;
  char* slot = kp.ws + (size_t)b * kp.ws_slot;
  cpx<T>* V = ws_cpx<T>(slot, kp.lay.V);
  const int vstride = kp.vstride;
  if (threadIdx.x == 0) st = ss.state[b];
  __syncthreads();
  if (st.p == 0) return;  // finished (uniform over the work-group)
  const int p = st.p;
  const cpx<T>* src = reinterpret_cast<const cpx<T>*>(samples) + (size_t)b * kp.S1 * kp.p_max;
  if (session_at_k(st)) {
    // verification round: f on the tilted line (set 0 of the samples) enters the
    // residual sum through the set-1 area of V
    cpx<T>* f = V + vstride;
    for (int h = threadIdx.x; h < p; h += kWG) f[h] = src[h];
    __syncthreads();
    KBatch kb;
    memset(&kb, 0, sizeof(kb));
    verify_round<T>(kp, kb, slot, st, lds, V, sh_part, f);
    if (threadIdx.x == 0) {
      st.samples += st.p;
      int32_t* tr = ss.trace + ((size_t)b * kp.max_rounds + (st.i - 1)) * 8;
      tr[0] = st.i;
      tr[1] = 0;
      tr[2] = st.p;
      tr[3] = 0;
      tr[4] = st.ncand;
      tr[5] = 0;
      tr[6] = st.nR;
      tr[7] = 1;
      st.i += 1;
      if (st.ncand == 0) {
        st.verified = 1;
      } else {
        const int room = st.k + max(16, (st.k + 7) / 8) - st.nR;
        st.kv = min(min(st.ncand, st.k), room);
        if (st.kv <= 0) {
          st.kv = 0;
          st.flag = 2;  // no room: RESIDUAL_NONZERO
        }
      }
      session_next(kp, st);
      session_publish(ss, st, b);
    }
    return;
  }
  for (int q = threadIdx.x; q < kp.S1 * p; q += kWG) {
    const int sidx = q / p, h = q - sidx * p;
    V[(size_t)sidx * vstride + h] = src[(size_t)sidx * kp.p_max + h];
  }
  __syncthreads();
  KOut ko;
  memset(&ko, 0, sizeof(ko));
  dft_round<T>(kp, slot, st, lds, V, vstride, kp.S1);
  subtract_registry<T>(kp, slot, st, lds, V, vstride, kp.S1, sh_part);
  select_round<T>(kp, slot, st, lds, V, sh_part);
  decode_round<T>(kp, ko, slot, st, V, vstride, lds, sh_part);
  decode_finish(kp, st, lds, sh_part);
  merge_round<T>(kp, slot, st, lds, sh_part, 0);
  if (threadIdx.x == 0) {
    st.samples += (int64_t)kp.S1 * st.p;
    st.kv = 0;
    int32_t* tr = ss.trace + ((size_t)b * kp.max_rounds + (st.i - 1)) * 8;
    tr[0] = st.i;
    tr[1] = st.kstar;
    tr[2] = st.p;
    tr[3] = st.m0 + 1;
    tr[4] = st.ncand;
    tr[5] = st.nacc;
    tr[6] = st.nR;
    tr[7] = 0;
    st.i += 1;
    session_next(kp, st);
    session_publish(ss, st, b);
  }
}

// Points of the requested lines: t[b][s][h][l] = (h/p) U[l][m] + eps K_s U[l][n_s]
// (eqs. (36), (41); U of the plan's partition, or of the tilt), h < p.
__global__ void __launch_bounds__(kWG) session_points_kernel(KParams kp, KSess ss, double* t) {
  // products and sums rounded one by one (no fused multiply-add), so that a
  // point is the same double however the caller forms it from the formula
#pragma clang fp contract(off)
  const int b = blockIdx.x;
  const int p = ss.req_p[b];
  if (p == 0) return;
  const int d = kp.d;
  if (ss.req_m[b] < 0) {
    // verification line t_h = (h/p) U v, v_n = q^(n-1) mod p (set 0 only)
    const int64_t q = -ss.req_m[b];
    double* out0 = t + (size_t)b * kp.S1 * kp.p_max * d;
    for (int h = threadIdx.x; h < p; h += kWG) {
      const double x = (double)h / (double)p;
      double* out = out0 + (size_t)h * d;
      for (int l = 0; l < d; ++l) out[l] = 0.0;
      int64_t v = 1;
      if (kp.tilt) {
        // U v with U = [[b, a], [-a, b]], v = (1, q)
        out[0] = x * (double)(kp.tb + kp.ta * q);
        out[1] = x * (double)(kp.tb * q - kp.ta);
      } else {
        for (int n = 0; n < kp.d2; ++n) {
          double pw = 1.0;
          for (int l = kp.blk[n]; l < kp.blk[n + 1]; ++l) {
            out[kp.perm[l]] = x * ((double)v * pw);
            pw *= (double)kp.N;
          }
          v = (v * q) % p;
        }
      }
    }
    return;
  }
  const int m0 = ss.req_m[b] - 1;
  const double eps = 1.0 / (2.0 * (double)kp.NB);
  for (int q = threadIdx.x; q < kp.S1 * p; q += kWG) {
    const int sidx = q / p, h = q - sidx * p;
    int n0 = 0;
    int64_t K = 0;
    if (sidx > 0) shift_of(kp, sidx, &n0, &K);
    const double x = (double)h / (double)p, sh = eps * (double)K;
    double* out = t + (((size_t)b * kp.S1 + sidx) * kp.p_max + h) * d;
    for (int l = 0; l < d; ++l) out[l] = 0.0;
    if (kp.tilt) {
      // columns of U = [[b, a], [-a, b]]: (b, -a) and (a, b)
      const double c0[2] = {(double)kp.tb, -(double)kp.ta}, c1[2] = {(double)kp.ta, (double)kp.tb};
      const double* cm = m0 == 0 ? c0 : c1;
      out[0] = x * cm[0];
      out[1] = x * cm[1];
      if (sidx > 0) {
        const double* cn = n0 == 0 ? c0 : c1;
        out[0] += sh * cn[0];
        out[1] += sh * cn[1];
      }
    } else {
      double pw = 1.0;
      for (int l = kp.blk[m0]; l < kp.blk[m0 + 1]; ++l) {
        out[kp.perm[l]] += x * pw;
        pw *= (double)kp.N;
      }
      if (sidx > 0) {
        pw = 1.0;
        for (int l = kp.blk[n0]; l < kp.blk[n0 + 1]; ++l) {
          out[kp.perm[l]] += sh * pw;
          pw *= (double)kp.N;
        }
      }
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kWG) session_finish_kernel(KParams kp, KSess ss, KOut ko) {
  extern __shared__ __align__(16) char lds[];
  __shared__ WgState st;
  const int b = blockIdx.x;
  char* slot = kp.ws + (size_t)b * kp.ws_slot;
  if (threadIdx.x == 0) {
    st = ss.state[b];
    if (st.status == 0)
      st.status = (st.nR < st.k) ? 1 : (st.nR > st.k || (kp.verify && !st.verified)) ? 2 : 0;
  }
  __syncthreads();
  if (ko.trace) {
    const int32_t* tr = ss.trace + (size_t)b * kp.max_rounds * 8;
    int32_t* to = ko.trace + (size_t)b * kp.max_rounds * 8;
    for (int e = threadIdx.x; e < (st.i - 1) * 8; e += kWG) to[e] = tr[e];
  }
  write_output(kp, ko, slot, st, lds);
}

// ----------------------------------------------- component: line sampler ----
template <typename T, int RT>
__global__ void __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(2))) sample_kernel(KParams kp, KBatch kb, int round, int p,
                                                     int m, const int64_t* res_off,
                                                     const int64_t* res_y, const double* res_c,
                                                     void* Vvoid) {
  cpx<T>* Vout = reinterpret_cast<cpx<T>*>(Vvoid);
  extern __shared__ __align__(16) char lds[];
  __shared__ WgState st;
  char* slot = kp.ws + (size_t)blockIdx.x * kp.ws_slot;
  for (int sig = blockIdx.x; sig < kb.B; sig += gridDim.x) {
    if (threadIdx.x == 0) {
      st.sig = sig;
      st.off = kb.mode_off[sig];
      st.M_pl = min((int)(kb.mode_off[sig + 1] - st.off), kp.k_max);
      st.sigma = kb.sigma[sig];
      st.cur = 0;
      st.sb = 0;
      st.i = round;
      st.p = p;
      st.m0 = m - 1;
      int nres = 0;
      if (res_off) nres = (int)(res_off[sig + 1] - res_off[sig]);
      st.nR = max(0, min(nres, kp.cap));
      st.nslots = st.nR;
    }
    __syncthreads();
    planted_setup<T>(kp, kb, slot, st);
    const int P0 = (st.M_pl + 1) / 2;
    // the caller's residual modes become registry slots 0..nR-1
    if (res_off) {
      int64_t* ry = reg_y(kp, slot, 0);
      double2* ra = reg_a(kp, slot, 0);
      int* ord = reg_ord(kp, slot, 0);
      const int64_t r0 = res_off[sig];
      for (int e = threadIdx.x; e < st.nR; e += kWG) {
        for (int q = 0; q < kp.d2; ++q) ry[(size_t)e * kp.d2 + q] = res_y[(r0 + e) * kp.d2 + q];
        ra[e] = make_double2(res_c[2 * (r0 + e)], res_c[2 * (r0 + e) + 1]);
        ord[e] = e;
      }
      __syncthreads();
    }
    if constexpr (sizeof(T) == 4) {
      scatter_afrag(kp, ws_cpx<float>(slot, kp.lay.ccomp),
                    reinterpret_cast<float*>(slot + kp.lay.afrag), 0, 2 * P0);
      __syncthreads();
    }
    cpx<T>* Vs = Vout + (size_t)sig * kp.S1 * p;
    if (kp.residual == 1) rebuild_rows<T>(kp, slot, st, P0, false);
    if (sizeof(T) == 4 && kp.tw_half)
      sample_round<T, RT, true>(kp, kb, slot, st, P0, lds, Vs, p);
    else
      sample_round<T, RT>(kp, kb, slot, st, P0, lds, Vs, p);
    // spectrum-mode plans subtract the registry after the DFT; here the caller
    // asked for samples: V[s][h] -= sum_e a_e exp(2 pi i y_e . t_{s,h}), FP64 per value
    if (kp.residual == 0 && st.nR > 0) {
      const int64_t* ry = reg_y(kp, slot, 0);
      const double2* ra = reg_a(kp, slot, 0);
      for (int q = threadIdx.x; q < kp.S1 * p; q += kWG) {
        const int s = q / p, h = q - s * p;
        int n0 = 0;
        int64_t K = 0;
        if (s > 0) shift_of(kp, s, &n0, &K);
        double ax = 0.0, ay = 0.0;
        for (int e = 0; e < st.nR; ++e) {
          const int64_t* y = ry + (size_t)e * kp.d2;
          // phase (h y_m / p + eps K y_n) mod 1 as an exact rational over 2 p N^d1
          const int64_t hm = (int64_t)h * pmod64(y[st.m0], p) % p;
          cpx<double> w;
          expipi(2.0 * (double)hm / (double)p, &w.x, &w.y);
          if (s > 0) w = cmul(w, shift_phase(y[n0], K, kp.NB));
          ax += ra[e].x * w.x - ra[e].y * w.y;
          ay += ra[e].x * w.y + ra[e].y * w.x;
        }
        cpx<T>* v = Vs + (size_t)s * p + h;
        *v = cmk<T>((T)((double)v->x - ax), (T)((double)v->y - ay));
      }
      __syncthreads();
    }
  }
}

// ----------------------------------------------------- component: DFT ------
template <typename T>
__global__ void __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(2))) dft_kernel(KParams kp, cpx<T>* data, int count, int p) {
  extern __shared__ __align__(16) char lds[];
  __shared__ WgState st;
  char* slot = kp.ws + (size_t)blockIdx.x * kp.ws_slot;
  if (threadIdx.x == 0) {
    int L = 1, lg = 0;
    while (L < 2 * p - 1) {
      L <<= 1;
      ++lg;
    }
    st.p = p;
    st.L = L;
    st.log2L = lg;
  }
  __syncthreads();
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(lds);
  cpx<T>* chirp = ws_cpx<T>(slot, kp.lay.chirp);
  cpx<T>* bhat = ws_cpx<T>(slot, kp.lay.bhat);
  constexpr int ML = MaxL<T>::value;
  const int R = st.L > ML ? st.L / ML : 1;
  // short lengths: several sequences per batched pass, as in a round's DFTs
  constexpr int MAXV = MaxL<T>::value / kWG;
  const int Lb = min(kp.L_max, ML);
  const bool batched = R == 1 && kp.sched_dft_batch != 1 && st.L <= MAXV * kWG &&
                       2 * st.L <= Lb;
  const BsTabs<T> tb = bs_tables<T>(st.L, st.L / R, buf + lds_padded(batched ? Lb : st.L / R));
  cpx<T>* G = ws_cpx<T>(slot, kp.lay.big);
  int cap = 1;
  if (batched) {
    cap = min(Lb, MAXV * kWG) / st.L;
    if (kp.sched_dft_batch > 1) cap = min(cap, kp.sched_dft_batch);
  }
  // the first pass computes chirp and filter, then this group's sequences: blocks of
  // cap consecutive sequences, block b = blockIdx.x, blockIdx.x + gridDim.x, ...
  bool setup = true;
  for (int q = blockIdx.x * cap; q < count && !batched;) {
    bluestein_run<T>(setup, setup ? nullptr : data + (size_t)q * p, p, st.L, R,
                     st.log2L - (R >> 1), chirp, bhat, G, buf, tb, kp.sched_fft);
    if (setup)
      setup = false;
    else
      q += gridDim.x;
  }
  if (batched) {
    bluestein_run<T>(true, nullptr, p, st.L, 1, st.log2L, chirp, bhat, G, buf, tb, kp.sched_fft);
    for (int q0 = blockIdx.x * cap; q0 < count; q0 += gridDim.x * cap) {
      const int g = min(cap, count - q0);
      bluestein_dft_batch<T, MAXV>(data + (size_t)q0 * p, p, g, p, st.L, st.log2L, chirp, bhat,
                                   buf, tb.T1M, kp.sched_fft);
    }
  }
}

__global__ void zero_queue_kernel(int* q, int64_t* count) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *q = 0;
    if (count) *count = 0;
  }
}

// ------------------------------------------------------------ launchers -----
int launch_zero_queue(const KParams& kp, int64_t* count, void* stream) {
  hipLaunchKernelGGL(zero_queue_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, kp.queue,
                     count);
  return (int)hipGetLastError();
}

#define SFFT_RT_DISPATCH(KERNEL, ...)                                              \
  switch (kp.precision == 1 ? kp.RT : 0) {                                        \
    case 1: hipLaunchKernelGGL((KERNEL<float, 1>), __VA_ARGS__); break;           \
    case 2: hipLaunchKernelGGL((KERNEL<float, 2>), __VA_ARGS__); break;           \
    case 3: hipLaunchKernelGGL((KERNEL<float, 3>), __VA_ARGS__); break;           \
    case 4: hipLaunchKernelGGL((KERNEL<float, 4>), __VA_ARGS__); break;           \
    case 5: hipLaunchKernelGGL((KERNEL<float, 5>), __VA_ARGS__); break;           \
    case 6: hipLaunchKernelGGL((KERNEL<float, 6>), __VA_ARGS__); break;           \
    case 7: hipLaunchKernelGGL((KERNEL<float, 7>), __VA_ARGS__); break;           \
    case 8: hipLaunchKernelGGL((KERNEL<float, 8>), __VA_ARGS__); break;           \
    default: hipLaunchKernelGGL((KERNEL<double, 0>), __VA_ARGS__); break;         \
  }

int launch_recover(const KParams& kp, const KBatch& kb, const KOut& ko, int grid, void* stream) {
  SFFT_RT_DISPATCH(recover_kernel, dim3(grid), dim3(kWG), kp.lds_bytes, (hipStream_t)stream, kp,
                   kb, ko);
  return (int)hipGetLastError();
}

size_t split_state_bytes() { return sizeof(WgState); }

// One set-up launch, then max_rounds (sample, post) pairs: every ordinary round
// takes one round index, so no signal has more; launches past a signal's end
// return at once.  No host synchronisation (the sequence can be captured).
int launch_recover_split(const KParams& kp, const KBatch& kb, const KOut& ko, void* state,
                         int ngrp, void* dft_scratch, void* stream) {
  hipStream_t hs = (hipStream_t)stream;
  WgState* stt = reinterpret_cast<WgState*>(state);
  const bool dft_launch = split_dft_launch(kp);
  SFFT_RT_DISPATCH(split_setup_kernel, dim3(kb.B), dim3(kWG), kp.lds_bytes, hs, kp, kb, ko, stt);
  hipError_t e = hipGetLastError();
  for (int r = 0; r < kp.max_rounds && e == hipSuccess; ++r) {
    SFFT_RT_DISPATCH(split_sample_kernel, dim3(kb.B * ngrp), dim3(kWG), kp.lds_bytes, hs, kp,
                     kb, (const WgState*)stt, ngrp);
    if (dft_launch && kp.precision == 1)
      hipLaunchKernelGGL(split_dft_kernel<float>, dim3(kb.B * ngrp), dim3(kWG), kp.lds_bytes, hs,
                         kp, kb, ko, (const WgState*)stt, ngrp, (char*)dft_scratch,
                         split_dft_scratch(kp).bytes);
    else if (dft_launch)
      hipLaunchKernelGGL(split_dft_kernel<double>, dim3(kb.B * ngrp), dim3(kWG), kp.lds_bytes,
                         hs, kp, kb, ko, (const WgState*)stt, ngrp, (char*)dft_scratch,
                         split_dft_scratch(kp).bytes);
    SFFT_RT_DISPATCH(split_post_kernel, dim3(kb.B), dim3(kWG), kp.lds_bytes, hs, kp, kb, ko, stt,
                     dft_launch ? 0 : 1);
    e = hipGetLastError();
  }
  return (int)e;
}

// ------------------------------------------------ fixed device scratch ------
// Workspace of sfft_recover_static: the work-queue counter in the first 256
// bytes, then as many workspace slots as fit.  One copy per device, held
// until the process ends; every call on a device shares it.  In host code the
// array's name is no device address: the address of each device's copy comes
// from hipGetSymbolAddress (static_scratch_setup) and only that is used.
static __device__ __align__(256) char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};  // per device, set once with that device current
}  // namespace

int static_scratch_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return (int)hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev]) return 0;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return (int)e;
  if (!ptr) return (int)hipErrorInvalidSymbol;
  g_scratch_ptr[dev] = static_cast<char*>(ptr);
  return 0;
}

int static_scratch_slots(size_t ws_slot) {
  return ws_slot ? (int)((kStaticScratchBytes - kStaticQueueBytes) / ws_slot) : 0;
}

// Zero-fills n16 16-byte words (a kernel, not hipMemsetAsync, so that the call
// can be captured in a graph).
__global__ void __launch_bounds__(256) zero_fill_kernel(uint4* p, size_t n16) {
  const uint4 z = make_uint4(0u, 0u, 0u, 0u);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = z;
}

int launch_recover_static(const KParams& kp, const KBatch& kb, const KOut& ko, int dev,
                          void* stream) {
  if (dev < 0 || dev >= kMaxDevices) return (int)hipErrorInvalidDevice;
  char* base;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    base = g_scratch_ptr[dev];
  }
  if (!base) return (int)hipErrorNotInitialized;
  const int fit = static_scratch_slots(kp.ws_slot);
  const int grid = min(kb.B, min(kp.n_slots, fit));
  if (grid < 1) return (int)hipErrorInvalidValue;
  KParams k2 = kp;
  k2.queue = reinterpret_cast<int*>(base);
  k2.ws = base + kStaticQueueBytes;
  k2.n_slots = grid;
  // the slots start as a new plan's workspace does (zeroed): another plan's
  // layout may have left anything there
  const size_t n16 = (kStaticQueueBytes + (size_t)grid * kp.ws_slot) / 16;
  // about 16 words per thread, at most 1024 work-groups
  const int zb = (int)(n16 / 4096 + 1 < 1024 ? n16 / 4096 + 1 : 1024);
  hipLaunchKernelGGL(zero_fill_kernel, dim3(zb), dim3(256), 0, (hipStream_t)stream,
                     reinterpret_cast<uint4*>(base), n16);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return (int)e;
  hipLaunchKernelGGL(zero_queue_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, k2.queue,
                     ko.count);
  e = hipGetLastError();
  if (e != hipSuccess) return (int)e;
  SFFT_RT_DISPATCH(recover_kernel, dim3(grid), dim3(kWG), kp.lds_bytes, (hipStream_t)stream, k2,
                   kb, ko);
  return (int)hipGetLastError();
}

int launch_sample_lines(const KParams& kp, const KBatch& kb, int round, int p, int m,
                        const int64_t* res_off, const int64_t* res_y, const double* res_c,
                        void* V, void* stream) {
  const int grid = min(kb.B, kp.n_slots);
  // V is passed as void* and typed inside the kernel by its precision
  SFFT_RT_DISPATCH(sample_kernel, dim3(grid), dim3(kWG), kp.lds_bytes, (hipStream_t)stream, kp,
                   kb, round, p, m, res_off, res_y, res_c, V);
  return (int)hipGetLastError();
}

int launch_dft(const KParams& kp, void* data, int count, int p, void* stream) {
  const int grid = min(count, kp.n_slots);
  if (kp.precision == 1) {
    hipLaunchKernelGGL(dft_kernel<float>, dim3(grid), dim3(kWG), kp.lds_bytes,
                       (hipStream_t)stream, kp, (cpx<float>*)data, count, p);
  } else {
    hipLaunchKernelGGL(dft_kernel<double>, dim3(grid), dim3(kWG), kp.lds_bytes,
                       (hipStream_t)stream, kp, (cpx<double>*)data, count, p);
  }
  return (int)hipGetLastError();
}

size_t session_state_bytes() { return sizeof(WgState); }

int launch_session(const KParams& kp, const KSess& ss, int what, const void* samples, double* t,
                   const KOut* ko, void* stream) {
  const dim3 grid(ss.B), block(kWG);
  hipStream_t hs = (hipStream_t)stream;
  const bool f32 = kp.precision == 1;
  switch (what) {
    case 0:
      if (f32) hipLaunchKernelGGL(session_init_kernel<float>, grid, block, 0, hs, kp, ss);
      else hipLaunchKernelGGL(session_init_kernel<double>, grid, block, 0, hs, kp, ss);
      break;
    case 1:
      if (f32)
        hipLaunchKernelGGL(session_feed_kernel<float>, grid, block, kp.lds_bytes, hs, kp, ss, samples);
      else
        hipLaunchKernelGGL(session_feed_kernel<double>, grid, block, kp.lds_bytes, hs, kp, ss, samples);
      break;
    case 2:
      hipLaunchKernelGGL(session_points_kernel, grid, block, 0, hs, kp, ss, t);
      break;
    default:
      if (f32)
        hipLaunchKernelGGL(session_finish_kernel<float>, grid, block, kp.lds_bytes, hs, kp, ss, *ko);
      else
        hipLaunchKernelGGL(session_finish_kernel<double>, grid, block, kp.lds_bytes, hs, kp, ss, *ko);
  }
  return (int)hipGetLastError();
}

int set_kernel_lds_limits(int lds_bytes) {
  hipError_t e = hipSuccess;
  const void* fns[] = {
      (const void*)recover_kernel<float, 1>, (const void*)recover_kernel<float, 2>,
      (const void*)recover_kernel<float, 3>, (const void*)recover_kernel<float, 4>,
      (const void*)recover_kernel<float, 5>, (const void*)recover_kernel<float, 6>,
      (const void*)recover_kernel<float, 7>, (const void*)recover_kernel<float, 8>,
      (const void*)recover_kernel<double, 0>, (const void*)sample_kernel<float, 1>,
      (const void*)sample_kernel<float, 2>,  (const void*)sample_kernel<float, 3>,
      (const void*)sample_kernel<float, 4>,  (const void*)sample_kernel<float, 5>,
      (const void*)sample_kernel<float, 6>,  (const void*)sample_kernel<float, 7>,
      (const void*)sample_kernel<float, 8>,  (const void*)sample_kernel<double, 0>,
      (const void*)dft_kernel<float>,        (const void*)dft_kernel<double>,
      (const void*)session_feed_kernel<float>, (const void*)session_feed_kernel<double>,
      (const void*)session_finish_kernel<float>, (const void*)session_finish_kernel<double>,
#define SFFT_SPLIT_FNS(K)                                                               \
  (const void*)K<float, 1>, (const void*)K<float, 2>, (const void*)K<float, 3>,        \
      (const void*)K<float, 4>, (const void*)K<float, 5>, (const void*)K<float, 6>,    \
      (const void*)K<float, 7>, (const void*)K<float, 8>, (const void*)K<double, 0>
      SFFT_SPLIT_FNS(split_setup_kernel), SFFT_SPLIT_FNS(split_sample_kernel),
      SFFT_SPLIT_FNS(split_post_kernel), (const void*)split_dft_kernel<float>,
      (const void*)split_dft_kernel<double>};
#undef SFFT_SPLIT_FNS
  for (const void* f : fns) {
    hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    if (r != hipSuccess) e = r;
  }
  return (int)e;
}

}  // namespace sfft
