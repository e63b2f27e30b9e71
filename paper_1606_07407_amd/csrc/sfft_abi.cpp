// Host side of the C ABI: parameter validation, plan construction (prime
// tables, DFT sizes, workspace) and the launch entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "sfft.h"
#include "sfft_internal.hpp"

using namespace sfft;

namespace {

thread_local char g_err[512] = "";

sfft_status fail(sfft_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

sfft_status hip_fail(hipError_t e, const char* what) {
  return fail(SFFT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool is_prime_host(int64_t n) {
  if (n < 2) return false;
  if (n < 4) return true;
  if (n % 2 == 0) return false;
  for (int64_t f = 3; f * f <= n; f += 2)
    if (n % f == 0) return false;
  return true;
}

bool smooth7(int64_t n) {
  if (n < 1) return false;
  for (int64_t f : {2, 3, 5, 7})
    while (n % f == 0) n /= f;
  return n == 1;
}

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

namespace sfft {
// Error text for the other host sources of the library (the autotuner).
sfft_status set_error(sfft_status st, const char* msg) { return fail(st, "%s", msg); }
}  // namespace sfft

struct sfft_plan_s {
  sfft_params prm;
  int device = 0;
  int max_batch = 0;
  KParams kp;
  int32_t* d_primes = nullptr;
  char* d_part = nullptr;
  char* d_ws = nullptr;
  int* d_queue = nullptr;
  char* d_split = nullptr;  // round states of the several-groups-per-signal launches
  char* d_split_dft = nullptr;   // their DFT groups' Bluestein tables
  size_t split_dft_bytes = 0;
  int capacity = 0;         // work-groups of this plan the device holds at once
};

// The partition of the d coordinates: block sizes and coordinate order (uniform
// blocks of d1 in the natural order unless `blocks` / `order` are given).
static sfft_status resolve_partition(const sfft_params* p, std::vector<int32_t>* blocks,
                                     std::vector<int32_t>* order) {
  if (p->d < 1) return fail(SFFT_EINVAL, "d must be >= 1");
  blocks->clear();
  if (!p->blocks) {
    if (p->n_blocks != 0) return fail(SFFT_EINVAL, "n_blocks without blocks");
    if (p->d1 < 1 || p->d % p->d1 != 0)
      return fail(SFFT_EINVAL, "d (%d) must be a positive multiple of d1 (%d)", p->d, p->d1);
    if (p->d / p->d1 > kMaxD2) return fail(SFFT_ERANGE, "d2 = d/d1 exceeds %d", kMaxD2);
    blocks->assign(p->d / p->d1, p->d1);
  } else {
    if (p->n_blocks < 1) return fail(SFFT_EINVAL, "n_blocks must be >= 1 with blocks");
    if (p->n_blocks > kMaxD2) return fail(SFFT_ERANGE, "n_blocks exceeds %d", kMaxD2);
    int64_t sum = 0;
    for (int q = 0; q < p->n_blocks; ++q) {
      if (p->blocks[q] < 1) return fail(SFFT_EINVAL, "block %d has size %d", q, p->blocks[q]);
      sum += p->blocks[q];
      blocks->push_back(p->blocks[q]);
    }
    if (sum != p->d) return fail(SFFT_EINVAL, "block sizes sum to %lld, not d = %d",
                                 (long long)sum, p->d);
  }
  order->resize(p->d);
  if (!p->order) {
    for (int l = 0; l < p->d; ++l) (*order)[l] = l;
  } else {
    std::vector<char> seen(p->d, 0);
    for (int l = 0; l < p->d; ++l) {
      const int32_t v = p->order[l];
      if (v < 0 || v >= p->d || seen[v]) return fail(SFFT_EINVAL, "order is not a permutation");
      seen[v] = 1;
      (*order)[l] = v;
    }
  }
  return SFFT_OK;
}

static int64_t gcd64(int64_t x, int64_t y) {
  while (y) {
    const int64_t t = x % y;
    x = y;
    y = t;
  }
  return x < 0 ? -x : x;
}

// The rotation of 2D tilting: the caller's triple, or the Pythagorean triple
// (a, b, c) with b > 2N and gcd(a, b) = 1 of least a + b (then least b).  Every
// primitive triple is {m^2 - n^2, 2mn} with hypotenuse m^2 + n^2 (m > n >= 1
// coprime, m - n odd).  A triple with m > sqrt(8N) + 1 has a + b >= m^2 > 8N,
// more than that of n = ceil(sqrt N), m = n + 1, so the search stops there.
static sfft_status resolve_tilt(const sfft_params* p, int64_t* a, int64_t* b, int64_t* c) {
  if (p->tilt_a || p->tilt_b || p->tilt_c) {
    *a = p->tilt_a;
    *b = p->tilt_b;
    *c = p->tilt_c;
    if (!(*a >= 1 && *a < *b && *b < *c && (*a) * (*a) + (*b) * (*b) == (*c) * (*c)))
      return fail(SFFT_EINVAL, "tilt (%lld, %lld, %lld) is not a triple with 1 <= a < b < c",
                  (long long)*a, (long long)*b, (long long)*c);
    if (gcd64(*a, *b) != 1 || *b <= 2 * p->N)
      return fail(SFFT_EINVAL, "tilt needs gcd(a, b) = 1 and b > 2N");
    return SFFT_OK;
  }
  int64_t best_sum = -1;
  const int64_t m_max = (int64_t)std::sqrt(8.0 * (double)p->N) + 2;
  for (int64_t m = 2; m <= m_max; ++m)
    for (int64_t n = 1; n < m; ++n) {
      if ((m - n) % 2 == 0 || gcd64(m, n) != 1) continue;
      const int64_t legs[2] = {m * m - n * n, 2 * m * n};
      for (int o = 0; o < 2; ++o) {
        const int64_t x = legs[o], y = legs[1 - o];  // candidate a = x, b = y
        if (y > 2 * p->N && x < y &&
            (best_sum < 0 || x + y < best_sum || (x + y == best_sum && y < *b))) {
          best_sum = x + y;
          *a = x;
          *b = y;
          *c = m * m + n * n;
        }
      }
    }
  if (best_sum < 0) return fail(SFFT_ERANGE, "no tilt found");
  return SFFT_OK;
}

static sfft_status validate_params(const sfft_params* p) {
  if (!p) return fail(SFFT_EINVAL, "params is NULL");
  std::vector<int32_t> blocks, order;
  const sfft_status ps = resolve_partition(p, &blocks, &order);
  if (ps != SFFT_OK) return ps;
  const int dmax = *std::max_element(blocks.begin(), blocks.end());
  if (p->N < 2 || p->N % 2 != 0) return fail(SFFT_EINVAL, "N must be even and >= 2");
  double nb = 1.0;
  for (int r = 0; r < dmax; ++r) nb *= (double)p->N;
  if (p->tilt != 0 && p->tilt != 1) return fail(SFFT_EINVAL, "tilt must be 0 or 1");
  if (p->tilt) {
    if (p->d != 2 || p->d1 != 1 || p->blocks || p->order)
      return fail(SFFT_EINVAL, "tilting needs d = 2, d1 = 1 and no blocks or order");
    if (p->N > (1 << 24)) return fail(SFFT_ERANGE, "N too large for tilting");
    int64_t ta = 0, tb = 0, tc = 0;
    const sfft_status ts = resolve_tilt(p, &ta, &tb, &tc);
    if (ts != SFFT_OK) return ts;
    nb = (double)(ta + tb) * (double)p->N / 2.0;
  } else if (p->tilt_a || p->tilt_b || p->tilt_c) {
    return fail(SFFT_EINVAL, "tilt_a/b/c without tilt");
  }
  if (nb > 1099511627776.0) return fail(SFFT_ERANGE, "N^d1 exceeds 2^40");
  if (p->k_max < 1) return fail(SFFT_EINVAL, "k_max must be >= 1");
  if (!(p->c > 1.0) || !std::isfinite(p->c)) return fail(SFFT_EINVAL, "c must be > 1");
  if (p->prime_rule != SFFT_PRIME_PAPER && p->prime_rule != SFFT_PRIME_SMOOTH)
    return fail(SFFT_EINVAL, "unknown prime_rule");
  if (p->p_min < 0) return fail(SFFT_EINVAL, "p_min must be >= 0");
  if (p->ladder_K < 1) return fail(SFFT_EINVAL, "ladder_K must be >= 1");
  if (p->ladder_K > 1 && (double)p->ladder_K * nb > 4.0e18)
    return fail(SFFT_ERANGE, "ladder_K * N^d1 overflows");
  if (!std::isfinite(p->tau)) return fail(SFFT_EINVAL, "tau must be finite");
  if (!(p->tau_noise >= 0.0) || !std::isfinite(p->tau_noise))
    return fail(SFFT_EINVAL, "tau_noise must be >= 0");
  if (!(p->eta > 0.0) || !std::isfinite(p->eta)) return fail(SFFT_EINVAL, "eta must be > 0");
  if (p->max_rounds < 1 || p->max_rounds > 256)
    return fail(SFFT_EINVAL, "max_rounds must be in 1..256");
  if (p->precision != SFFT_FP64 && p->precision != SFFT_FP32)
    return fail(SFFT_EINVAL, "unknown precision");
  if (p->robust != 0 && p->robust != 1) return fail(SFFT_EINVAL, "robust must be 0 or 1");
  if (p->classifier != SFFT_CLS_PLAIN && p->classifier != SFFT_CLS_MLP)
    return fail(SFFT_EINVAL, "unknown classifier");
  if (p->classifier == SFFT_CLS_MLP) {
    if (!p->mlp_weights) return fail(SFFT_EINVAL, "the learned classifier needs mlp_weights");
    if (!(p->mlp_threshold > 0.0 && p->mlp_threshold < 1.0))
      return fail(SFFT_EINVAL, "mlp_threshold must be in (0, 1)");
  }
  if (!std::isfinite(p->feature_scale)) return fail(SFFT_EINVAL, "feature_scale must be finite");
  if (p->verify != 0 && p->verify != 1) return fail(SFFT_EINVAL, "verify must be 0 or 1");
  if (!std::isfinite(p->verify_eta)) return fail(SFFT_EINVAL, "verify_eta must be finite");
  if (p->residual != SFFT_RESIDUAL_SPECTRUM && p->residual != SFFT_RESIDUAL_SAMPLES)
    return fail(SFFT_EINVAL, "unknown residual mode");
  for (int b = 0; b < kNtBands; ++b) {
    const int v = p->sched_nt[b];
    const bool ok = v == 0 || (v >= 2 && v <= (b >= 2 ? 8 : 4));
    if (!ok) return fail(SFFT_EINVAL, "sched_nt[%d] = %d is not allowed", b, v);
  }
  if (p->sched_fft < 0 || p->sched_fft > kFftRadix8Head)
    return fail(SFFT_EINVAL, "unknown sched_fft %d", p->sched_fft);
  if (p->sched_dft_batch < 0 || p->sched_dft_batch > 64)
    return fail(SFFT_EINVAL, "sched_dft_batch must be in 0..64");
  if (p->split_groups < 0 || p->split_groups > 16)
    return fail(SFFT_EINVAL, "split_groups must be in 0..16");
  return SFFT_OK;
}

// Work-groups per signal for a batch of B signals: the plan's split_groups, or
// automatically (0) as many as fill the device (at most 8) when the batch takes at
// most half of it and the rounds are large (k_max >= 256); 1 when each signal needs
// its own slot and fewer are there.  (Measured: 64 signals at d = 20, k = 4096, FP32,
// 1.9x faster with 4 groups; 100 signals at d = 100, k = 1024, FP64, 1.2x with 2.)
static int split_groups_for(const sfft_plan_s* plan, int B) {
  if (B < 1 || B > plan->kp.n_slots) return 1;
  const int want = plan->prm.split_groups;
  if (want >= 1) return want;
  if (plan->kp.tw_half) return std::max(1, std::min(8, plan->capacity / B));
  if (2 * B > plan->capacity || plan->kp.k_max < 256) return 1;
  return std::max(1, std::min(8, plan->capacity / B));
}

extern "C" {

const char* sfft_last_error(void) { return g_err; }

int32_t sfft_version(void) { return 100; }

sfft_status sfft_plan_create(const sfft_params* params, int32_t max_batch, sfft_plan* out) {
  g_err[0] = 0;
  if (!out) return fail(SFFT_EINVAL, "out is NULL");
  sfft_status st = validate_params(params);
  if (st != SFFT_OK) return st;
  if (max_batch < 1) return fail(SFFT_EINVAL, "max_batch must be >= 1");
  const sfft_params& P = *params;
  std::vector<int32_t> blocks, order;
  resolve_partition(params, &blocks, &order);  // checked by validate_params

  KParams kp;
  memset(&kp, 0, sizeof(kp));
  kp.d = P.d;
  kp.d1 = *std::max_element(blocks.begin(), blocks.end());
  kp.d2 = (int)blocks.size();
  kp.S = (P.ladder_K > 1) ? 2 * kp.d2 : kp.d2;
  kp.S1 = kp.S + 1;
  kp.RT = (2 * kp.S1 + 15) / 16;
  if (P.precision == SFFT_FP32 && kp.RT > kMaxRT)
    return fail(SFFT_ERANGE, "2 (S+1) = %d real rows exceed the %d MFMA row tiles", 2 * kp.S1,
                kMaxRT);
  kp.N = P.N;
  kp.NB = 1;
  for (int r = 0; r < kp.d1; ++r) kp.NB *= P.N;
  int64_t ta = 0, tb = 0, tc = 0;
  if (P.tilt) {
    resolve_tilt(params, &ta, &tb, &tc);  // checked by validate_params
    kp.tilt = 1;
    kp.ta = ta;
    kp.tb = tb;
    kp.tc2 = tc * tc;
    kp.NB = (ta + tb) * P.N / 2;  // every |y| <= NB, the top one below it
  }
  kp.k_max = P.k_max;
  // registry capacity: k_max, plus the repair slack of the verification round
  kp.cap = P.k_max + (P.verify ? std::max(16, (P.k_max + 7) / 8) : 0);
  kp.pairs_max = (kp.k_max + 1) / 2 + (kp.cap + 1) / 2;
  kp.m_max = 2 * kp.pairs_max;
  kp.max_rounds = P.max_rounds;
  kp.prime_rule = P.prime_rule;
  kp.p_min = P.p_min;
  kp.ladder_K = P.ladder_K;
  kp.robust = P.robust;
  kp.precision = P.precision;
  kp.c = P.c;
  kp.tau = (P.tau > 0.0) ? P.tau : 1.0 / (2.0 * (double)kp.NB);
  kp.tau_noise = P.tau_noise;
  kp.eta = P.eta;
  kp.classifier = P.classifier;
  kp.mlp_w = (const uint16_t*)P.mlp_weights;
  kp.mlp_thr = P.mlp_threshold;
  kp.feat_scale = (P.feature_scale > 0.0) ? P.feature_scale : kp.tau;
  kp.verify = P.verify;
  kp.residual = P.residual;
  for (int b = 0; b < kNtBands; ++b) kp.sched_nt[b] = P.sched_nt[b];
  kp.sched_fft = P.sched_fft ? P.sched_fft : kFftRadix24Head;
  kp.sched_dft_batch = P.sched_dft_batch;
  kp.verify_eta = (P.verify_eta > 0.0) ? P.verify_eta : P.eta;

  // Largest prime a round can use: the max_rounds-th rule prime >= max(ceil(c k_max), p_min),
  // clamped to what the DFT holds (Bluestein length 2p - 1 <= kBluesteinParts maxL: LDS
  // holds FFTs of up to maxL points, longer ones run in parts through the slot).  A round
  // that would need a larger prime (k* still near k_max after many rounds) ends its signal
  // with SFFT_ERANGE; the first round must fit.
  const int maxL = (P.precision == SFFT_FP32) ? kLdsFftMax32 : kLdsFftMax64;
  const int64_t p_lim = ((int64_t)kBluesteinParts * maxL + 1) / 2;
  const double xd = std::max(std::ceil(P.c * (double)P.k_max), (double)P.p_min);
  if (xd > 40000.0) return fail(SFFT_ERANGE, "c * k_max = %.0f is beyond the prime range", xd);
  const int64_t x = (int64_t)xd;
  std::vector<int32_t> primes;
  const bool smooth = (P.prime_rule == SFFT_PRIME_SMOOTH);
  int found = 0;
  int64_t pmax = 0;
  for (int64_t q = 2; found < P.max_rounds && q <= p_lim; ++q) {
    if (is_prime_host(q) && (!smooth || smooth7(q - 1))) {
      primes.push_back((int32_t)q);
      if (q >= x) {
        ++found;
        pmax = q;
      }
    }
  }
  if (found == 0)
    return fail(SFFT_ERANGE,
                "the first round needs a prime >= %lld; the DFT holds primes up to %lld",
                (long long)x, (long long)p_lim);
  kp.p_max = (int)pmax;
  int L = 1, lg = 0;
  while (L < 2 * kp.p_max - 1) {
    L <<= 1;
    ++lg;
  }
  kp.L_max = L;
  kp.log2_Lmax = lg;
  kp.vstride = kp.p_max;
  const size_t cs = (P.precision == SFFT_FP32) ? 8 : 16;  // complex element size

  // LDS: the largest of the per-step carve-ups.  The merge/sort arrays stay in
  // LDS unless they would be the largest; then they live in the slot.
  size_t lds = 0;
  const char* lds_step = "";
  auto need = [&](size_t bytes, const char* step) {
    if (bytes > lds) {
      lds = bytes;
      lds_step = step;
    }
  };
  {
    // FFT buffer (at most maxL points) and twiddle tables
    const int Mx = std::min(L, maxL);
    need((size_t)(lds_padded(Mx) + bs_tab_entries(L, Mx)) * cs, L > maxL ? "DFT (in parts)" : "DFT");
  }
  {
    // the sampler's twiddle table: all p points, or (FP32) p/2 + 1 when the whole table and
    // the staged A fragments do not fit
    const size_t rest = 2 * align16(2 * (size_t)(sampler_m_max(kp) + 4)) +
                        (P.precision == SFFT_FP32 ? 2 * (size_t)(kChunk + 1) * kp.RT * 256
                                                  : kF64StageBytes);
    const size_t full = align16((size_t)kp.p_max * cs) + rest;
    kp.tw_half = 0;
    if (P.precision == SFFT_FP32 && full > kLdsLimit) kp.tw_half = 1;
    need(kp.tw_half ? align16((size_t)(kp.p_max / 2 + 1) * cs) + rest : full, "sampler");
  }
  need(align16((size_t)kp.p_max * (cs / 2)) + 4 * (size_t)kp.p_max + 4 * 256 + 16, "selection");
  need(decode_lds_cnt(kp.k_max) + 4 * (size_t)kp.p_max, "decode");
  {
    size_t n2 = 1;
    while (n2 < (size_t)kp.cap) n2 <<= 1;
    need(4 * ((size_t)kp.p_max + 1 + 2 * (size_t)kp.cap), "registry subtraction");
    need(align16(4 * ((size_t)kp.p_max + 1 + n2)) + 16 * (size_t)kp.cap,
         "registry subtraction (sorted entries)");
  }
  need(12 * (size_t)kp.k_max, "output");  // rank keys and ranks
  {
    // verification rounds use the prime for k* = 1: the max_rounds-th table prime
    // >= max(ceil(c), p_min)
    const int64_t xv = std::max((int64_t)std::ceil(P.c), (int64_t)P.p_min);
    int cntv = 0;
    kp.p_vmax = 2;
    for (int32_t q : primes)
      if (q >= xv && cntv < P.max_rounds) {
        kp.p_vmax = q;
        ++cntv;
      }
    if (P.verify)
      need(align16((size_t)kp.p_vmax * cs) + align16(2 * (size_t)(kp.m_max + 4)) +
               (size_t)kp.m_max * cs + 4 * (size_t)kWG * cs,
           "verification");
  }
  // FP32 spectrum subtraction staged through LDS: as many sets per block (up to 8) as
  // fit in what the other steps already need, so that the stage never sets the size
  if (P.precision == SFFT_FP32 && P.residual == SFFT_RESIDUAL_SPECTRUM) {
    const size_t fixed = align16(4 * ((size_t)kp.p_max + 1 + kp.cap)) + 16 * (size_t)kp.cap;
    for (int cs = 8; cs >= 1; --cs)
      if (fixed + 8 * (size_t)kp.cap * cs <= lds) {
        kp.sub_cs = cs;
        break;
      }
  }
  const size_t merge_bytes = merge_lds(kp.k_max, kp.cap).bytes;
  kp.merge_global = merge_bytes > lds ? 1 : 0;
  if (!kp.merge_global) need(merge_bytes, "merge");
  lds = align16(lds);
  if (lds > kLdsLimit)
    return fail(SFFT_ERANGE, "plan needs %zu bytes of LDS per work-group (%s step, largest "
                "prime %d)", lds, lds_step, kp.p_max);
  kp.lds_bytes = (int)lds;

  // Lexicographic order of w equals that of y (the registry's order) only for blocks of
  // one coordinate in the natural order, untilted; otherwise the output is ranked.
  {
    bool natural = !kp.tilt;
    for (int q = 0; q < kp.d2; ++q)
      if (blocks[q] != 1) natural = false;
    for (int l = 0; l < P.d; ++l)
      if (order[l] != l) natural = false;
    kp.wrap_rank = natural ? 0 : 1;
  }

  // Workspace layout of one slot.
  WsLayout lay;
  size_t o = 0;
  const int d2 = kp.d2, S = kp.S, S1 = kp.S1;
  lay.ypl = o;   o = al256(o + 8 * (size_t)kp.k_max * d2);
  lay.ccomp = o; o = al256(o + cs * (size_t)(kp.m_max + 2) * S1);
  // slack: the sampler copies whole chunks of A fragments past npairs
  lay.afrag = o; o = al256(o + (P.precision == SFFT_FP32 ? 4 * (size_t)(kp.pairs_max + kChunk + 2) * kp.RT * 64 : 0));
  for (int b = 0; b < 2; ++b) {
    lay.sy[b] = o;  o = al256(o + 8 * (size_t)kp.cap * d2);
    lay.sa[b] = o;  o = al256(o + 16 * (size_t)kp.cap);
    lay.sE[b] = o;  o = al256(o + 8 * (size_t)kp.cap * S);
    lay.ord[b] = o; o = al256(o + 4 * (size_t)kp.cap);
  }
  lay.dirty = o;  o = al256(o + 4 * (size_t)(kp.cap + 1));
  lay.V = o;      o = al256(o + cs * (size_t)S1 * kp.vstride);
  lay.chirp = o;  o = al256(o + cs * (size_t)kp.p_max);
  lay.bhat = o;   o = al256(o + cs * (size_t)L);
  lay.big = o;    o = al256(o + (L > maxL ? cs * (size_t)L : 0));
  lay.cand = o;   o = al256(o + 4 * (size_t)kp.k_max);
  lay.acc_y = o;  o = al256(o + 8 * (size_t)kp.k_max * d2);
  lay.acc_a = o;  o = al256(o + 16 * (size_t)kp.k_max);
  lay.acc_ok = o; o = al256(o + 4 * (size_t)kp.k_max);
  lay.run = o;    o = al256(o + 4 * (size_t)kp.k_max);
  lay.pl_sorted = o; o = al256(o + 4 * (size_t)kp.k_max);
  lay.feat_tmp = o;  o = al256(o + 4 * 8 * (size_t)kp.k_max);
  lay.merge = o;     o = al256(o + (kp.merge_global ? merge_bytes : 0));
  lay.wtmp = o;      o = al256(o + (kp.wrap_rank ? 8 * (size_t)kp.k_max * P.d : 0));
  lay.bytes = o;
  kp.lay = lay;
  kp.ws_slot = lay.bytes;

  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  const int per_cu = (lds <= 80 * 1024) ? 2 : 1;
  const int capacity = prop.multiProcessorCount * per_cu;
  kp.n_slots = std::min(max_batch, capacity);
  if (kp.n_slots < 1) kp.n_slots = 1;

  sfft_plan plan = new (std::nothrow) sfft_plan_s();
  if (!plan) return fail(SFFT_ENOMEM, "host allocation failed");
  plan->prm = P;
  plan->prm.blocks = nullptr;  // the caller's arrays are not kept
  plan->prm.order = nullptr;
  plan->device = dev;
  plan->max_batch = max_batch;
  plan->capacity = capacity;

  const size_t ws_bytes = (size_t)kp.n_slots * kp.ws_slot;
  // partition tables: block starts [d2 + 1], coordinate order [d], bands [d2][2]
  std::vector<int32_t> blk(kp.d2 + 1, 0);
  std::vector<int64_t> band(2 * (size_t)kp.d2, 0);
  const int64_t wlo = -(P.N / 2), whi = P.N / 2 - 1;
  for (int q = 0; q < kp.d2; ++q) {
    blk[q + 1] = blk[q] + blocks[q];
    int64_t s = 0, pw = 1;
    for (int r = 0; r < blocks[q]; ++r) {
      s += pw;
      pw *= P.N;
    }
    band[2 * q] = wlo * s;
    band[2 * q + 1] = whi * s;
  }
  if (kp.tilt) {
    // y0 = b w0 - a w1, y1 = a w0 + b w1 over w in [wlo, whi]^2
    band[0] = tb * wlo - ta * whi;
    band[1] = tb * whi - ta * wlo;
    band[2] = (ta + tb) * wlo;
    band[3] = (ta + tb) * whi;
  }
  const size_t part_blk = 0, part_perm = al256(4 * (size_t)(kp.d2 + 1));
  const size_t part_band = part_perm + al256(4 * (size_t)P.d);
  const size_t part_bytes = part_band + 16 * (size_t)kp.d2;
  if ((e = hipMalloc((void**)&plan->d_primes, primes.size() * sizeof(int32_t))) != hipSuccess ||
      (e = hipMalloc((void**)&plan->d_part, part_bytes)) != hipSuccess ||
      (e = hipMalloc((void**)&plan->d_ws, ws_bytes)) != hipSuccess ||
      (e = hipMalloc((void**)&plan->d_queue, 256)) != hipSuccess ||
      (e = hipMalloc((void**)&plan->d_split, (size_t)max_batch * split_state_bytes())) !=
          hipSuccess) {
    sfft_plan_destroy(plan);
    return fail(SFFT_ENOMEM, "device allocation of %zu bytes failed: %s", ws_bytes,
                hipGetErrorString(e));
  }
  // Bluestein tables of the grouped DFT launch of the several-groups recovery: one set
  // per work-group, as many work-groups as sfft_recover can run (signals x groups: at
  // most the device's capacity automatically, n_slots x split_groups when given)
  if (split_dft_launch(kp)) {
    const size_t nwg = P.split_groups >= 1 ? (size_t)kp.n_slots * P.split_groups
                                           : (size_t)capacity;
    plan->split_dft_bytes = nwg * split_dft_scratch(kp).bytes;
    if ((e = hipMalloc((void**)&plan->d_split_dft, plan->split_dft_bytes)) != hipSuccess) {
      const size_t want_bytes = plan->split_dft_bytes;
      plan->d_split_dft = nullptr;
      sfft_plan_destroy(plan);
      return fail(SFFT_ENOMEM, "device allocation of %zu bytes failed: %s", want_bytes,
                  hipGetErrorString(e));
    }
  }
  if ((e = hipMemcpy(plan->d_primes, primes.data(), primes.size() * sizeof(int32_t),
                     hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(plan->d_part + part_blk, blk.data(), blk.size() * sizeof(int32_t),
                     hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(plan->d_part + part_perm, order.data(), order.size() * sizeof(int32_t),
                     hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(plan->d_part + part_band, band.data(), band.size() * sizeof(int64_t),
                     hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemset(plan->d_ws, 0, ws_bytes)) != hipSuccess ||
      (e = hipMemset(plan->d_queue, 0, 256)) != hipSuccess) {
    sfft_plan_destroy(plan);
    return hip_fail(e, "plan upload");
  }
  // the fixed scratch of sfft_recover_static: its address on this device, looked up once
  const int se = static_scratch_setup(dev);
  if (se != 0) {
    sfft_plan_destroy(plan);
    return hip_fail((hipError_t)se, "hipGetSymbolAddress of the fixed scratch");
  }
  const int le = set_kernel_lds_limits((int)lds);
  if (le != 0) {
    sfft_plan_destroy(plan);
    return hip_fail((hipError_t)le, "hipFuncSetAttribute");
  }
  kp.primes = plan->d_primes;
  kp.n_primes = (int)primes.size();
  kp.blk = reinterpret_cast<const int32_t*>(plan->d_part + part_blk);
  kp.perm = reinterpret_cast<const int32_t*>(plan->d_part + part_perm);
  kp.band = reinterpret_cast<const int64_t*>(plan->d_part + part_band);
  kp.ws = plan->d_ws;
  kp.queue = plan->d_queue;
  plan->kp = kp;
  *out = plan;
  return SFFT_OK;
}

sfft_status sfft_plan_destroy(sfft_plan plan) {
  if (!plan) return SFFT_OK;
  (void)hipDeviceSynchronize();
  if (plan->d_primes) (void)hipFree(plan->d_primes);
  if (plan->d_part) (void)hipFree(plan->d_part);
  if (plan->d_ws) (void)hipFree(plan->d_ws);
  if (plan->d_queue) (void)hipFree(plan->d_queue);
  if (plan->d_split) (void)hipFree(plan->d_split);
  if (plan->d_split_dft) (void)hipFree(plan->d_split_dft);
  delete plan;
  return SFFT_OK;
}

int32_t sfft_plan_max_prime(sfft_plan plan) { return plan ? plan->kp.p_max : 0; }

int32_t sfft_plan_num_sets(sfft_plan plan) { return plan ? plan->kp.S1 : 0; }

static sfft_status check_batch(sfft_plan plan, const sfft_signal_batch* b) {
  if (!plan) return fail(SFFT_EINVAL, "plan is NULL");
  if (!b) return fail(SFFT_EINVAL, "batch is NULL");
  if (b->B < 1 || b->B > plan->max_batch)
    return fail(SFFT_EINVAL, "batch size %d outside 1..%d", b->B, plan->max_batch);
  if (!b->mode_off || !b->freqs || !b->coeffs || !b->k || !b->sigma)
    return fail(SFFT_EINVAL, "batch has a NULL array");
  int dev = -1;
  (void)hipGetDevice(&dev);
  if (dev != plan->device)
    return fail(SFFT_EINVAL, "current device %d is not the plan's device %d", dev, plan->device);
  return SFFT_OK;
}

static KBatch to_kbatch(const sfft_signal_batch* b) {
  KBatch kb;
  kb.B = b->B;
  kb.mode_off = b->mode_off;
  kb.freqs = b->freqs;
  kb.coeffs = b->coeffs;
  kb.k = b->k;
  kb.sigma = b->sigma;
  kb.seed = b->seed;
  return kb;
}

sfft_status sfft_recover(sfft_plan plan, const sfft_signal_batch* batch, const sfft_outputs* out,
                         void* stream) {
  g_err[0] = 0;
  sfft_status st = check_batch(plan, batch);
  if (st != SFFT_OK) return st;
  if (!out || !out->freqs || !out->coeffs || !out->k_found || !out->status)
    return fail(SFFT_EINVAL, "outputs need freqs, coeffs, k_found and status");
  KOut ko;
  ko.freqs = out->freqs;
  ko.coeffs = out->coeffs;
  ko.k_found = out->k_found;
  ko.status = out->status;
  ko.rounds = out->rounds;
  ko.samples = out->samples;
  ko.trace = out->trace;
  const int nexp = (out->feat != nullptr) + (out->label != nullptr) + (out->feat_meta != nullptr) +
                   (out->feat_count != nullptr);
  if (nexp != 0 && nexp != 4)
    return fail(SFFT_EINVAL, "feature export needs feat, label, feat_meta and feat_count");
  if (nexp == 4 && out->feat_cap < 0) return fail(SFFT_EINVAL, "feat_cap must be >= 0");
  ko.feat = out->feat;
  ko.label = out->label;
  ko.meta = out->feat_meta;
  ko.count = out->feat_count;
  ko.cap = nexp ? out->feat_cap : 0;
  ko.phase = out->phase;
  int e = launch_zero_queue(plan->kp, out->feat_count, stream);
  if (e) return hip_fail((hipError_t)e, "queue reset launch");
  const int groups = split_groups_for(plan, batch->B);
  if (plan->kp.tw_half && batch->B > plan->kp.n_slots)
    return fail(SFFT_ERANGE, "this plan's lines run as the several-groups recovery, one "
                "workspace slot per signal: at most %d signals", plan->kp.n_slots);
  if (groups > 1 || plan->kp.tw_half) {
    // each DFT group's tables (reserved at plan creation for every batch this path takes)
    const size_t need = split_dft_launch(plan->kp)
                            ? (size_t)batch->B * groups * split_dft_scratch(plan->kp).bytes
                            : 0;
    if (need > plan->split_dft_bytes)
      return fail(SFFT_ERANGE, "%d signals x %d groups need %zu bytes of DFT tables, the plan "
                  "holds %zu", batch->B, groups, need, plan->split_dft_bytes);
    e = launch_recover_split(plan->kp, to_kbatch(batch), ko, plan->d_split, groups,
                             plan->d_split_dft, stream);
    if (e) return hip_fail((hipError_t)e, "recover launch (several groups per signal)");
    return SFFT_OK;
  }
  const int grid = std::min(batch->B, plan->kp.n_slots);
  e = launch_recover(plan->kp, to_kbatch(batch), ko, grid, stream);
  if (e) return hip_fail((hipError_t)e, "recover launch");
  return SFFT_OK;
}

sfft_status sfft_recover_static(sfft_plan plan, const sfft_signal_batch* batch,
                                const sfft_outputs* out, void* stream) {
  g_err[0] = 0;
  sfft_status st = check_batch(plan, batch);
  if (st != SFFT_OK) return st;
  if (!out || !out->freqs || !out->coeffs || !out->k_found || !out->status)
    return fail(SFFT_EINVAL, "outputs need freqs, coeffs, k_found and status");
  if (out->feat || out->label || out->feat_meta || out->feat_count)
    return fail(SFFT_EINVAL, "sfft_recover_static does not export features");
  if (plan->kp.tw_half)
    return fail(SFFT_ERANGE, "this plan's lines need the several-groups recovery (sfft_recover)");
  if (plan->kp.ws_slot + kStaticQueueBytes > kStaticScratchBytes)
    return fail(SFFT_ERANGE,
                "one workspace slot of this plan takes %zu bytes; the fixed scratch holds %zu",
                plan->kp.ws_slot, kStaticScratchBytes - kStaticQueueBytes);
  KOut ko;
  memset(&ko, 0, sizeof(ko));
  ko.freqs = out->freqs;
  ko.coeffs = out->coeffs;
  ko.k_found = out->k_found;
  ko.status = out->status;
  ko.rounds = out->rounds;
  ko.samples = out->samples;
  ko.trace = out->trace;
  ko.phase = out->phase;
  const int e = launch_recover_static(plan->kp, to_kbatch(batch), ko, plan->device, stream);
  if (e) return hip_fail((hipError_t)e, "static-scratch recover launch");
  return SFFT_OK;
}

int32_t sfft_static_scratch_slots(sfft_plan plan) {
  return plan ? static_scratch_slots(plan->kp.ws_slot) : 0;
}

sfft_status sfft_export_bucket_features(sfft_plan plan, const sfft_signal_batch* batch,
                                        float* feat, uint8_t* label, int32_t* feat_meta,
                                        int64_t feat_cap, int64_t* feat_count, void* stream) {
  g_err[0] = 0;
  sfft_status st = check_batch(plan, batch);
  if (st != SFFT_OK) return st;
  if (!feat || !label || !feat_meta || !feat_count)
    return fail(SFFT_EINVAL, "feat, label, feat_meta and feat_count are required");
  if (feat_cap < 0) return fail(SFFT_EINVAL, "feat_cap must be >= 0");
  KOut ko;
  memset(&ko, 0, sizeof(ko));  // no recovery outputs: the kernel writes only the export
  ko.feat = feat;
  ko.label = label;
  ko.meta = feat_meta;
  ko.count = feat_count;
  ko.cap = feat_cap;
  int e = launch_zero_queue(plan->kp, feat_count, stream);
  if (e) return hip_fail((hipError_t)e, "queue reset launch");
  const int grid = std::min(batch->B, plan->kp.n_slots);
  e = launch_recover(plan->kp, to_kbatch(batch), ko, grid, stream);
  if (e) return hip_fail((hipError_t)e, "recover launch");
  return SFFT_OK;
}

sfft_status sfft_sample_lines(sfft_plan plan, const sfft_signal_batch* batch, int32_t round,
                              int32_t p, int32_t m, const int64_t* res_off, const int64_t* res_y,
                              const double* res_coeffs, void* V, void* stream) {
  g_err[0] = 0;
  sfft_status st = check_batch(plan, batch);
  if (st != SFFT_OK) return st;
  if (!V) return fail(SFFT_EINVAL, "V is NULL");
  if (round < 1) return fail(SFFT_EINVAL, "round is 1-based");
  if (p < 2 || p > plan->kp.p_max || !is_prime_host(p))
    return fail(SFFT_EINVAL, "p = %d must be a prime in 2..%d", p, plan->kp.p_max);
  if (m < 1 || m > plan->kp.d2) return fail(SFFT_EINVAL, "m must be in 1..d2");
  if (res_off && (!res_y || !res_coeffs))
    return fail(SFFT_EINVAL, "res_off given without res_y / res_coeffs");
  const int e = launch_sample_lines(plan->kp, to_kbatch(batch), round, p, m, res_off, res_y,
                                    res_coeffs, V, stream);
  if (e) return hip_fail((hipError_t)e, "sampler launch");
  return SFFT_OK;
}

struct sfft_session_s {
  KParams kp;     // the plan's, with ws = the session's workspace
  KSess ss;
  char* d_ws = nullptr;
  char* d_state = nullptr;
  int32_t* d_req = nullptr;    // p [B] then m [B]
  int32_t* d_trace = nullptr;
};

sfft_status sfft_session_destroy(sfft_session s) {
  if (!s) return SFFT_OK;
  (void)hipDeviceSynchronize();
  if (s->d_ws) (void)hipFree(s->d_ws);
  if (s->d_state) (void)hipFree(s->d_state);
  if (s->d_req) (void)hipFree(s->d_req);
  if (s->d_trace) (void)hipFree(s->d_trace);
  delete s;
  return SFFT_OK;
}

sfft_status sfft_session_create(sfft_plan plan, int32_t B, const int32_t* k, void* stream,
                                sfft_session* out) {
  g_err[0] = 0;
  if (!out) return fail(SFFT_EINVAL, "out is NULL");
  *out = nullptr;
  if (!plan) return fail(SFFT_EINVAL, "plan is NULL");
  if (B < 1) return fail(SFFT_EINVAL, "B must be >= 1");
  if (!k) return fail(SFFT_EINVAL, "k is NULL");
  if (plan->kp.residual != SFFT_RESIDUAL_SPECTRUM)
    return fail(SFFT_EINVAL, "sessions need the residual subtracted in the spectra");
  sfft_session s = new (std::nothrow) sfft_session_s();
  if (!s) return fail(SFFT_ENOMEM, "host allocation failed");
  s->kp = plan->kp;
  const size_t ws = (size_t)B * s->kp.ws_slot;
  const size_t state = (size_t)B * session_state_bytes();
  const size_t trace = (size_t)B * s->kp.max_rounds * 8 * sizeof(int32_t);
  hipError_t e;
  if ((e = hipMalloc((void**)&s->d_ws, ws)) != hipSuccess ||
      (e = hipMalloc((void**)&s->d_state, state)) != hipSuccess ||
      (e = hipMalloc((void**)&s->d_req, 2 * (size_t)B * sizeof(int32_t))) != hipSuccess ||
      (e = hipMalloc((void**)&s->d_trace, trace)) != hipSuccess) {
    sfft_session_destroy(s);
    return fail(SFFT_ENOMEM, "session allocation of %zu bytes failed: %s", ws + state + trace,
                hipGetErrorString(e));
  }
  if ((e = hipMemset(s->d_ws, 0, ws)) != hipSuccess ||
      (e = hipMemset(s->d_trace, 0, trace)) != hipSuccess) {
    sfft_session_destroy(s);
    return hip_fail(e, "session set-up");
  }
  s->kp.ws = s->d_ws;
  s->ss.B = B;
  s->ss.k = k;
  s->ss.state = reinterpret_cast<WgState*>(s->d_state);
  s->ss.req_p = s->d_req;
  s->ss.req_m = s->d_req + B;
  s->ss.trace = s->d_trace;
  const int le = launch_session(s->kp, s->ss, 0, nullptr, nullptr, nullptr, stream);
  if (le) {
    sfft_session_destroy(s);
    return hip_fail((hipError_t)le, "session init launch");
  }
  *out = s;
  return SFFT_OK;
}

sfft_status sfft_session_request(sfft_session s, int32_t* p, int32_t* m, void* stream) {
  g_err[0] = 0;
  if (!s) return fail(SFFT_EINVAL, "session is NULL");
  if (!p || !m) return fail(SFFT_EINVAL, "p and m are needed");
  const size_t n = (size_t)s->ss.B * sizeof(int32_t);
  hipError_t e;
  if ((e = hipMemcpyAsync(p, s->ss.req_p, n, hipMemcpyDeviceToDevice, (hipStream_t)stream)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(m, s->ss.req_m, n, hipMemcpyDeviceToDevice, (hipStream_t)stream)) !=
          hipSuccess)
    return hip_fail(e, "session request copy");
  return SFFT_OK;
}

sfft_status sfft_session_points(sfft_session s, double* t, void* stream) {
  g_err[0] = 0;
  if (!s) return fail(SFFT_EINVAL, "session is NULL");
  if (!t) return fail(SFFT_EINVAL, "t is NULL");
  const int e = launch_session(s->kp, s->ss, 2, nullptr, t, nullptr, stream);
  if (e) return hip_fail((hipError_t)e, "session points launch");
  return SFFT_OK;
}

sfft_status sfft_session_feed(sfft_session s, const void* samples, void* stream) {
  g_err[0] = 0;
  if (!s) return fail(SFFT_EINVAL, "session is NULL");
  if (!samples) return fail(SFFT_EINVAL, "samples is NULL");
  const int e = launch_session(s->kp, s->ss, 1, samples, nullptr, nullptr, stream);
  if (e) return hip_fail((hipError_t)e, "session feed launch");
  return SFFT_OK;
}

sfft_status sfft_session_finish(sfft_session s, const sfft_outputs* out, void* stream) {
  g_err[0] = 0;
  if (!s) return fail(SFFT_EINVAL, "session is NULL");
  if (!out || !out->freqs || !out->coeffs || !out->k_found || !out->status)
    return fail(SFFT_EINVAL, "outputs need freqs, coeffs, k_found and status");
  if (out->feat || out->label || out->feat_meta || out->feat_count || out->phase)
    return fail(SFFT_EINVAL, "sessions offer no feature export or phase timestamps");
  KOut ko;
  memset(&ko, 0, sizeof(ko));
  ko.freqs = out->freqs;
  ko.coeffs = out->coeffs;
  ko.k_found = out->k_found;
  ko.status = out->status;
  ko.rounds = out->rounds;
  ko.samples = out->samples;
  ko.trace = out->trace;
  const int e = launch_session(s->kp, s->ss, 3, nullptr, nullptr, &ko, stream);
  if (e) return hip_fail((hipError_t)e, "session finish launch");
  return SFFT_OK;
}

sfft_status sfft_dft(sfft_plan plan, void* data, int32_t count, int32_t p, void* stream) {
  g_err[0] = 0;
  if (!plan) return fail(SFFT_EINVAL, "plan is NULL");
  if (!data) return fail(SFFT_EINVAL, "data is NULL");
  if (count < 1) return fail(SFFT_EINVAL, "count must be >= 1");
  if (p < 2 || p > plan->kp.p_max)
    return fail(SFFT_EINVAL, "p = %d outside 2..%d", p, plan->kp.p_max);
  const int e = launch_dft(plan->kp, data, count, p, stream);
  if (e) return hip_fail((hipError_t)e, "dft launch");
  return SFFT_OK;
}

sfft_status sfft_mlp_forward(const void* w, const float* x, int64_t n, float* prob, void* stream) {
  g_err[0] = 0;
  if (!w || !x || !prob) return fail(SFFT_EINVAL, "NULL argument");
  if (n < 1) return fail(SFFT_EINVAL, "n must be >= 1");
  const int e = launch_mlp_forward(w, x, n, prob, stream);
  if (e) return hip_fail((hipError_t)e, "mlp forward launch");
  return SFFT_OK;
}

sfft_status sfft_mlp_grad(const void* w, const float* x, const uint8_t* y, int64_t n, float* grad,
                          float* loss, void* stream) {
  g_err[0] = 0;
  if (!w || !x || !y || !grad || !loss) return fail(SFFT_EINVAL, "NULL argument");
  if (n < 1) return fail(SFFT_EINVAL, "n must be >= 1");
  float* part = nullptr;
  const size_t part_bytes = sizeof(float) * (size_t)kMlpGradGroups * kMlpPartStride;
  hipError_t he = hipMalloc((void**)&part, part_bytes);
  if (he != hipSuccess) return fail(SFFT_ENOMEM, "gradient partial sums: %s", hipGetErrorString(he));
  const int e = launch_mlp_grad(w, x, y, n, n, 0, 0, part, grad, loss, stream);
  const hipError_t se = hipStreamSynchronize((hipStream_t)stream);
  (void)hipFree(part);
  if (e) return hip_fail((hipError_t)e, "mlp grad launch");
  if (se != hipSuccess) return hip_fail(se, "mlp grad");
  return SFFT_OK;
}

sfft_status sfft_mlp_train(void* w, const float* x, const uint8_t* y, int64_t n, int32_t epochs,
                           int32_t batch, double lr, uint64_t seed, float* loss_hist,
                           void* stream) {
  g_err[0] = 0;
  if (!w || !x || !y) return fail(SFFT_EINVAL, "NULL argument");
  if (n < 1 || epochs < 1 || batch < 1) return fail(SFFT_EINVAL, "n, epochs, batch must be >= 1");
  if (!(lr > 0.0) || !std::isfinite(lr)) return fail(SFFT_EINVAL, "lr must be > 0");
  const int P = kMlpParamCount;
  float* st = nullptr;  // master, m, v, grad, loss, gradient partial sums
  hipError_t he = hipMalloc((void**)&st, sizeof(float) * (4 * (size_t)P + 64 +
                                                          (size_t)kMlpGradGroups * kMlpPartStride));
  if (he != hipSuccess) return fail(SFFT_ENOMEM, "optimiser state: %s", hipGetErrorString(he));
  float *master = st, *m = st + P, *v = st + 2 * P, *g = st + 3 * P, *loss = st + 4 * P;
  float* part = st + 4 * (size_t)P + 64;
  const uint64_t hseed = seed ? seed : 0x5DEECE66Dull;  // 0 would mean "rows in order"
  const int64_t steps = (n + batch - 1) / batch;
  int e = launch_mlp_init(w, master, m, v, stream);
  if (!e && loss_hist) e = launch_fill(loss_hist, epochs, 0.f, stream);
  double b1t = 1.0, b2t = 1.0;
  uint64_t t = 0;
  for (int ep = 0; ep < epochs && !e; ++ep) {
    for (int64_t s = 0; s < steps && !e; ++s) {
      ++t;
      b1t *= 0.9;
      b2t *= 0.999;
      e = launch_mlp_grad(w, x, y, n, batch, hseed, t, part, g, loss, stream);
      if (!e) e = launch_mlp_adam(master, m, v, g, w, (float)lr, (float)(1.0 - b1t),
                                  (float)(1.0 - b2t), stream);
      if (!e && loss_hist) e = launch_mlp_accum(loss, loss_hist + ep, 1.f / (float)steps, stream);
    }
  }
  hipError_t se = hipStreamSynchronize((hipStream_t)stream);
  (void)hipFree(st);
  if (e) return hip_fail((hipError_t)e, "mlp train launch");
  if (se != hipSuccess) return hip_fail(se, "mlp train");
  return SFFT_OK;
}

}  // extern "C"
