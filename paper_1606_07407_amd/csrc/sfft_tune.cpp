// Autotuner of the C ABI: times whole recoveries of a sample batch for
// candidate values of c and of the kernel schedules, and keeps the fastest
// candidate among those with the most exact recoveries.  Host code only; the
// measured launches are ordinary sfft_recover calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <vector>

#include "sfft.h"
#include "sfft_internal.hpp"

namespace sfft {
sfft_status set_error(sfft_status st, const char* msg);
}

namespace {

using sfft::kNtBands;

// A schedule change is kept only when it is faster by more than this fraction
// (launch-to-launch noise of a whole recovery is about 1%).
constexpr double kKeepMargin = 0.02;

sfft_status tune_fail(sfft_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
sfft_status tune_fail(sfft_status st, const char* fmt, ...) {
  char msg[400];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(msg, sizeof(msg), fmt, ap);
  va_end(ap);
  return sfft::set_error(st, msg);
}

// Device buffers of one batch's outputs and the host copies compared with the
// planted supports.
struct Work {
  int B = 0, d = 0, k_max = 0;
  std::vector<int64_t> off;     // [B + 1]
  std::vector<int64_t> truth;   // planted frequencies, rows sorted per signal
  int64_t* freqs = nullptr;
  double* coeffs = nullptr;
  int32_t* k_found = nullptr;
  int32_t* status = nullptr;
  std::vector<hipEvent_t> ev;
  std::vector<int64_t> h_freqs;
  std::vector<int32_t> h_k, h_status;

  ~Work() {
    if (freqs) (void)hipFree(freqs);
    if (coeffs) (void)hipFree(coeffs);
    if (k_found) (void)hipFree(k_found);
    if (status) (void)hipFree(status);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

sfft_status hip_err(hipError_t e, const char* what) {
  return tune_fail(SFFT_EDEVICE, "autotune: %s: %s", what, hipGetErrorString(e));
}

// Host copy of the planted frequencies, each signal's rows in lexicographic
// order (the order sfft_recover writes).
sfft_status load_truth(const sfft_signal_batch* b, Work& w) {
  w.off.resize((size_t)b->B + 1);
  hipError_t e = hipMemcpy(w.off.data(), b->mode_off, w.off.size() * sizeof(int64_t),
                           hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_err(e, "copy of mode_off");
  for (int i = 0; i < b->B; ++i)
    if (w.off[i + 1] < w.off[i] || w.off[0] != 0)
      return tune_fail(SFFT_EINVAL, "autotune: mode_off is not non-decreasing from 0");
  const size_t n = (size_t)w.off[b->B];
  std::vector<int64_t> raw(n * (size_t)w.d);
  if (n) {
    e = hipMemcpy(raw.data(), b->freqs, raw.size() * sizeof(int64_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_err(e, "copy of the planted frequencies");
  }
  w.truth.resize(raw.size());
  const int d = w.d;
  for (int s = 0; s < b->B; ++s) {
    const int64_t lo = w.off[s], hi = w.off[s + 1];
    std::vector<int64_t> idx;
    for (int64_t j = lo; j < hi; ++j) idx.push_back(j);
    std::sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) {
      return std::lexicographical_compare(&raw[x * d], &raw[x * d] + d, &raw[y * d],
                                          &raw[y * d] + d);
    });
    for (size_t r = 0; r < idx.size(); ++r)
      std::memcpy(&w.truth[(lo + r) * d], &raw[idx[r] * d], d * sizeof(int64_t));
  }
  return SFFT_OK;
}

int count_exact(Work& w) {
  int exact = 0;
  for (int s = 0; s < w.B; ++s) {
    const int64_t n = w.off[s + 1] - w.off[s];
    if (w.h_status[s] != SFFT_OK || w.h_k[s] != n) continue;
    if (std::memcmp(&w.h_freqs[(size_t)s * w.k_max * w.d], &w.truth[(size_t)w.off[s] * w.d],
                    (size_t)n * w.d * sizeof(int64_t)) == 0)
      ++exact;
  }
  return exact;
}

void fill_entry(const sfft_params& p, sfft_tune_entry* e) {
  e->c = p.c;
  for (int b = 0; b < kNtBands; ++b) e->sched_nt[b] = p.sched_nt[b];
  // the schedule as run: sched_fft 0 is the radix-2/4 head, which is what the
  // winner written back to the caller says as well
  e->sched_fft = p.sched_fft == 0 ? sfft::kFftRadix24Head : p.sched_fft;
  e->sched_dft_batch = p.sched_dft_batch;
  e->status = SFFT_OK;
  e->exact = 0;
  e->ms = std::numeric_limits<double>::infinity();
}

// One candidate: plan, warm-up and timed launches, results compared with the
// planted supports.  A plan the library refuses is recorded, not an error.
sfft_status measure(const sfft_params& cand, const sfft_signal_batch* b, int warmup, int steps,
                    hipStream_t stream, Work& w, sfft_tune_entry* e) {
  fill_entry(cand, e);
  sfft_plan plan = nullptr;
  sfft_status st = sfft_plan_create(&cand, b->B, &plan);
  if (st == SFFT_EINVAL || st == SFFT_ERANGE) {
    e->status = st;
    return SFFT_OK;
  }
  if (st != SFFT_OK) return st;
  sfft_outputs out;
  std::memset(&out, 0, sizeof(out));
  out.freqs = w.freqs;
  out.coeffs = w.coeffs;
  out.k_found = w.k_found;
  out.status = w.status;
  for (int i = 0; i < warmup && st == SFFT_OK; ++i) st = sfft_recover(plan, b, &out, stream);
  for (int i = 0; i < steps && st == SFFT_OK; ++i) {
    hipError_t he = hipEventRecord(w.ev[2 * i], stream);
    if (he != hipSuccess) {
      st = hip_err(he, "event record");
      break;
    }
    st = sfft_recover(plan, b, &out, stream);
    if (st != SFFT_OK) break;
    he = hipEventRecord(w.ev[2 * i + 1], stream);
    if (he != hipSuccess) st = hip_err(he, "event record");
  }
  if (st == SFFT_OK) {
    hipError_t he = hipStreamSynchronize(stream);
    if (he != hipSuccess) st = hip_err(he, "stream synchronisation");
  }
  std::vector<double> ms;
  for (int i = 0; i < steps && st == SFFT_OK; ++i) {
    float t = 0.f;
    hipError_t he = hipEventElapsedTime(&t, w.ev[2 * i], w.ev[2 * i + 1]);
    if (he != hipSuccess) st = hip_err(he, "event timing");
    ms.push_back(t);
  }
  if (st == SFFT_OK) {
    hipError_t he;
    if ((he = hipMemcpy(w.h_k.data(), w.k_found, w.B * sizeof(int32_t), hipMemcpyDeviceToHost)) !=
            hipSuccess ||
        (he = hipMemcpy(w.h_status.data(), w.status, w.B * sizeof(int32_t),
                        hipMemcpyDeviceToHost)) != hipSuccess ||
        (he = hipMemcpy(w.h_freqs.data(), w.freqs, w.h_freqs.size() * sizeof(int64_t),
                        hipMemcpyDeviceToHost)) != hipSuccess)
      st = hip_err(he, "copy of the results");
  }
  sfft_plan_destroy(plan);
  if (st != SFFT_OK) return st;
  std::sort(ms.begin(), ms.end());
  const size_t n = ms.size();
  e->ms = (n % 2) ? ms[n / 2] : 0.5 * (ms[n / 2 - 1] + ms[n / 2]);
  e->exact = count_exact(w);
  return SFFT_OK;
}

// a is better than b: more exact recoveries, or as many and faster by more
// than `margin` (relative).
bool better(const sfft_tune_entry& a, const sfft_tune_entry& b, double margin) {
  if (a.status != SFFT_OK) return false;
  if (b.status != SFFT_OK) return true;
  if (a.exact != b.exact) return a.exact > b.exact;
  return a.ms < b.ms * (1.0 - margin);
}

}  // namespace

extern "C" sfft_status sfft_autotune(sfft_params* params, const sfft_signal_batch* batch,
                                     const double* c_values, int32_t n_c, int32_t warmup,
                                     int32_t steps, sfft_tune_entry* log, int32_t log_cap,
                                     int32_t* n_log, void* stream) {
  if (!params || !batch || !n_log) return tune_fail(SFFT_EINVAL, "autotune: NULL argument");
  if (n_c < 0 || (n_c > 0 && !c_values))
    return tune_fail(SFFT_EINVAL, "autotune: n_c = %d without c_values", n_c);
  if (warmup < 0 || steps < 1 || steps > 1000)
    return tune_fail(SFFT_EINVAL, "autotune: warmup >= 0 and steps in 1..1000 required");
  if (log_cap < 0 || (log_cap > 0 && !log))
    return tune_fail(SFFT_EINVAL, "autotune: log_cap = %d without log", log_cap);
  if (batch->B < 1 || !batch->mode_off || !batch->freqs || !batch->coeffs || !batch->k ||
      !batch->sigma)
    return tune_fail(SFFT_EINVAL, "autotune: incomplete batch");
  *n_log = 0;
  hipStream_t hs = (hipStream_t)stream;

  // The starting point must be a valid plan (its own errors are reported as is).
  {
    sfft_plan probe = nullptr;
    sfft_status st = sfft_plan_create(params, batch->B, &probe);
    if (st != SFFT_OK) return st;
    sfft_plan_destroy(probe);
  }

  Work w;
  w.B = batch->B;
  w.d = params->d;
  w.k_max = params->k_max;
  sfft_status st = load_truth(batch, w);
  if (st != SFFT_OK) return st;
  const size_t rows = (size_t)w.B * w.k_max;
  hipError_t he;
  if ((he = hipMalloc((void**)&w.freqs, rows * w.d * sizeof(int64_t))) != hipSuccess ||
      (he = hipMalloc((void**)&w.coeffs, rows * 2 * sizeof(double))) != hipSuccess ||
      (he = hipMalloc((void**)&w.k_found, w.B * sizeof(int32_t))) != hipSuccess ||
      (he = hipMalloc((void**)&w.status, w.B * sizeof(int32_t))) != hipSuccess)
    return tune_fail(SFFT_ENOMEM, "autotune: output allocation failed: %s",
                     hipGetErrorString(he));
  w.ev.resize(2 * (size_t)steps);
  for (auto& e : w.ev) {
    if ((he = hipEventCreate(&e)) != hipSuccess) {
      e = nullptr;
      return hip_err(he, "event creation");
    }
  }
  w.h_freqs.resize(rows * w.d);
  w.h_k.resize(w.B);
  w.h_status.resize(w.B);

  std::vector<sfft_tune_entry> all;
  auto run = [&](const sfft_params& cand) -> sfft_status {
    sfft_tune_entry e;
    sfft_status s2 = measure(cand, batch, warmup, steps, hs, w, &e);
    if (s2 != SFFT_OK) return s2;
    all.push_back(e);
    return SFFT_OK;
  };

  // Stage 1: c.
  sfft_params best_p = *params;
  sfft_tune_entry best;
  fill_entry(best_p, &best);
  best.status = SFFT_EINVAL;
  std::vector<double> cs(c_values, c_values + n_c);
  if (cs.empty()) cs.push_back(params->c);
  for (double c : cs) {
    sfft_params cand = *params;
    cand.c = c;
    if ((st = run(cand)) != SFFT_OK) return st;
    if (better(all.back(), best, 0.0)) {
      best = all.back();
      best_p = cand;
    }
  }
  if (best.status != SFFT_OK)
    return tune_fail(SFFT_ERANGE, "autotune: no value of c gives a valid plan");

  // Stage 2: one schedule at a time.
  // knob(p) is the field of p being tuned
  auto try_knob = [&](auto knob, const std::vector<int>& values) -> sfft_status {
    const int cur = knob(best_p);
    for (int v : values) {
      if (v == cur) continue;
      sfft_params cand = best_p;
      knob(cand) = v;
      sfft_status s2 = run(cand);
      if (s2 != SFFT_OK) return s2;
      if (better(all.back(), best, kKeepMargin)) {
        best = all.back();
        best_p = cand;
      }
    }
    return SFFT_OK;
  };
  if (best_p.sched_fft == 0) best_p.sched_fft = sfft::kFftRadix24Head;
  st = try_knob([](sfft_params& p) -> int32_t& { return p.sched_fft; },
                {sfft::kFftRadix24Head, sfft::kFftRadix8Head});
  if (st != SFFT_OK) return st;
  if (best_p.precision == SFFT_FP32) {
    st = try_knob([](sfft_params& p) -> int32_t& { return p.sched_dft_batch; }, {0, 1, 2, 4, 8});
    if (st != SFFT_OK) return st;
    for (int b = 0; b < kNtBands; ++b) {
      const std::vector<int> vals = b < 2 ? std::vector<int>{0, 2, 4}
                                          : std::vector<int>{0, 2, 4, 8};
      st = try_knob([b](sfft_params& p) -> int32_t& { return p.sched_nt[b]; }, vals);
      if (st != SFFT_OK) return st;
    }
  }

  params->c = best_p.c;
  for (int b = 0; b < kNtBands; ++b) params->sched_nt[b] = best_p.sched_nt[b];
  params->sched_fft = best_p.sched_fft;
  params->sched_dft_batch = best_p.sched_dft_batch;
  *n_log = (int32_t)all.size();
  for (int i = 0; i < (int)all.size() && i < log_cap; ++i) log[i] = all[i];
  return SFFT_OK;
}
