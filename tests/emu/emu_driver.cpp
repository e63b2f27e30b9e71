// Runs libsfft's host code and kernels in the host emulation on one batch read
// from a file and writes the outputs to another (test infrastructure).
//
//   emu_driver IN OUT
//
// IN (little-endian, written by tests/emu/emu.py): the sfft_params struct bytes
// (pointer fields ignored), the partition arrays, the batch and the entry point
// (for sfft_dft also p, count and the sequences as FP64 pairs); OUT: the plan's
// and the call's status, then every output array of sfft_outputs (sfft_dft: the
// transformed sequences as FP64 pairs).
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "sfft.h"

namespace {
FILE* g_in;
template <typename T>
T rd() {
  T v;
  if (fread(&v, sizeof(T), 1, g_in) != 1) {
    fprintf(stderr, "[emu] short input\n");
    exit(2);
  }
  return v;
}
template <typename T>
std::vector<T> rdv(size_t n) {
  std::vector<T> v(n);
  if (n && fread(v.data(), sizeof(T), n, g_in) != n) {
    fprintf(stderr, "[emu] short input\n");
    exit(2);
  }
  return v;
}
}  // namespace

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: emu_driver IN OUT\n");
    return 2;
  }
  g_in = fopen(argv[1], "rb");
  if (!g_in) return 2;
  if (rd<int64_t>() != 0x73666674656d75LL) return 3;  // "sfftemu"
  if (rd<int64_t>() != (int64_t)sizeof(sfft_params)) {
    fprintf(stderr, "[emu] sfft_params size mismatch\n");
    return 3;
  }
  sfft_params P = rd<sfft_params>();
  const int32_t nb = rd<int32_t>();
  std::vector<int32_t> blocks = rdv<int32_t>(nb);
  const int32_t no = rd<int32_t>();
  std::vector<int32_t> order = rdv<int32_t>(no);
  P.blocks = nb ? blocks.data() : nullptr;
  P.order = no ? order.data() : nullptr;
  P.mlp_weights = nullptr;
  const int32_t B = rd<int32_t>();
  const int32_t max_batch = rd<int32_t>();
  const int32_t entry = rd<int32_t>();  // 0 sfft_recover, 1 sfft_recover_static, 2 sfft_dft
  std::vector<int64_t> mode_off = rdv<int64_t>(B + 1);
  const int64_t total = mode_off[B];
  std::vector<int64_t> freqs = rdv<int64_t>((size_t)total * P.d);
  std::vector<double> coeffs = rdv<double>((size_t)total * 2);
  std::vector<int32_t> k = rdv<int32_t>(B);
  std::vector<double> sigma = rdv<double>(B);
  const uint64_t seed = rd<uint64_t>();
  int32_t dft_p = 0, dft_count = 0;
  std::vector<double> dft_x;
  if (entry == 2) {
    dft_p = rd<int32_t>();
    dft_count = rd<int32_t>();
    dft_x = rdv<double>((size_t)2 * dft_p * dft_count);
  }
  fclose(g_in);

  sfft_plan plan = nullptr;
  sfft_status st = sfft_plan_create(&P, max_batch, &plan);
  FILE* out = fopen(argv[2], "wb");
  if (!out) return 2;
  int32_t st32 = st;
  fwrite(&st32, 4, 1, out);
  if (st != SFFT_OK) {
    fprintf(stderr, "[emu] plan: %s\n", sfft_last_error());
    fclose(out);
    return 0;
  }
  if (entry == 2) {
    // the sequences in the plan's precision, transformed in place
    const size_t n = (size_t)dft_p * dft_count;
    const bool f32 = P.precision == SFFT_FP32;
    std::vector<float> xf(f32 ? 2 * n : 0);
    for (size_t i = 0; i < xf.size(); ++i) xf[i] = (float)dft_x[i];
    st = sfft_dft(plan, f32 ? (void*)xf.data() : (void*)dft_x.data(), dft_count, dft_p, nullptr);
    st32 = st;
    fwrite(&st32, 4, 1, out);
    if (st != SFFT_OK) fprintf(stderr, "[emu] dft: %s\n", sfft_last_error());
    for (size_t i = 0; i < xf.size(); ++i) dft_x[i] = xf[i];
    fwrite(dft_x.data(), 8, dft_x.size(), out);
    fclose(out);
    sfft_plan_destroy(plan);
    return 0;
  }
  sfft_signal_batch batch = {B, mode_off.data(), freqs.data(), coeffs.data(), k.data(),
                             sigma.data(), seed};
  const size_t km = (size_t)P.k_max, R = (size_t)P.max_rounds;
  std::vector<int64_t> o_freqs(B * km * P.d);
  std::vector<double> o_coeffs(B * km * 2);
  std::vector<int32_t> o_kf(B), o_status(B), o_rounds(B), o_trace(B * R * 8);
  std::vector<int64_t> o_samples(B);
  sfft_outputs o;
  memset(&o, 0, sizeof(o));
  o.freqs = o_freqs.data();
  o.coeffs = o_coeffs.data();
  o.k_found = o_kf.data();
  o.status = o_status.data();
  o.rounds = o_rounds.data();
  o.samples = o_samples.data();
  o.trace = o_trace.data();
  st = entry == 1 ? sfft_recover_static(plan, &batch, &o, nullptr)
                  : sfft_recover(plan, &batch, &o, nullptr);
  st32 = st;
  fwrite(&st32, 4, 1, out);
  if (st != SFFT_OK) fprintf(stderr, "[emu] recover: %s\n", sfft_last_error());
  fwrite(o_freqs.data(), 8, o_freqs.size(), out);
  fwrite(o_coeffs.data(), 8, o_coeffs.size(), out);
  fwrite(o_kf.data(), 4, B, out);
  fwrite(o_status.data(), 4, B, out);
  fwrite(o_rounds.data(), 4, B, out);
  fwrite(o_samples.data(), 8, B, out);
  fwrite(o_trace.data(), 4, o_trace.size(), out);
  fclose(out);
  sfft_plan_destroy(plan);
  return 0;
}
