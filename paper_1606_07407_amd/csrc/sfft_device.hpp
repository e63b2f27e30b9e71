// Device building blocks: complex arithmetic, Philox4x64-10 noise, block
// scans, the LDS Stockham FFT used by the Bluestein prime-length DFT, and the
// exponential-sum (line sampler) kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sfft_internal.hpp"

namespace sfft {

// ----------------------------------------------------------------- complex --
template <typename T>
struct cpx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cpx<T> cmk(T a, T b) {
  cpx<T> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) {
  return cmk<T>(a.x + b.x, a.y + b.y);
}
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) {
  return cmk<T>(a.x - b.x, a.y - b.y);
}
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return cmk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__device__ __forceinline__ cpx<T> cscale(cpx<T> a, T s) {
  return cmk<T>(a.x * s, a.y * s);
}

// Largest power-of-two FFT length kept in LDS for each precision: 32 complex
// values per thread in the register-held Stockham pass (FP32 8192, FP64 4096
// points).  Longer Bluestein lengths (up to 4 times these) run in parts
// through the workspace (bluestein_run).
template <typename T>
struct MaxL;
template <>
struct MaxL<float> {
  static constexpr int value = kLdsFftMax32;
};
template <>
struct MaxL<double> {
  static constexpr int value = kLdsFftMax64;
};

// exp(i pi x) in FP64 for a dyadic/rational x given as q / den, q exact.
__device__ __forceinline__ void expipi(double q_over_den, double* c, double* s) {
  sincospi(q_over_den, s, c);
}

// ------------------------------------------------------- Philox4x64-10 -----
// Salmon, Moraes, Dror, Shaw (SC 2011): round function
// (c0,c1,c2,c3) <- (hi(M1 c2)^c1^k0, lo(M1 c2), hi(M0 c0)^c3^k1, lo(M0 c0)),
// key bumped by the Weyl constants between rounds.
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
    const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
    const uint64_t n0 = hi1 ^ c[1] ^ k0;
    const uint64_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// Complex Gaussian noise of the sample pair (2 hp, 2 hp + 1): one Philox block,
// key (seed, signal), counter (hp, set, round, 0); words 0, 1 give the even
// sample, words 2, 3 the odd one.  For words (w0, w1): u1, u2 = top 53 bits
// times 2^-53, g = sqrt(-2 ln(1 - u1)) e^{2 pi i u2}, noise = sigma/sqrt(2) g.
// The FP64 path evaluates Box-Muller in FP64; the FP32 path in FP32 from the
// exact integer 2^53 (1 - u1), which keeps the tail (u1 near 1) finite and
// accurate to FP32 rounding.
__device__ __forceinline__ void noise_pair64(uint64_t seed, uint64_t signal, uint64_t round,
                                             uint64_t set, uint64_t hp, double sigma,
                                             cpx<double>* n0, cpx<double>* n1) {
  uint64_t c[4] = {hp, set, round, 0ull};
  philox4x64_10(c, seed, signal);
  const double sc = sigma / sqrt(2.0);
  for (int e = 0; e < 2; ++e) {
    const double u1 = (double)(c[2 * e] >> 11) * 0x1p-53;
    const double u2 = (double)(c[2 * e + 1] >> 11) * 0x1p-53;
    const double rad = sqrt(-2.0 * log1p(-u1));
    const double ang = 2.0 * M_PI * u2;
    const cpx<double> g = cmk<double>(sc * (rad * cos(ang)), sc * (rad * sin(ang)));
    if (e == 0) *n0 = g; else *n1 = g;
  }
}

__device__ __forceinline__ void noise_pair32(uint64_t seed, uint64_t signal, uint64_t round,
                                             uint64_t set, uint64_t hp, float sigma,
                                             cpx<float>* n0, cpx<float>* n1) {
  uint64_t c[4] = {hp, set, round, 0ull};
  philox4x64_10(c, seed, signal);
  const float sc = sigma * 0.70710678118654752440f;
  for (int e = 0; e < 2; ++e) {
    const float v = (float)((1ull << 53) - (c[2 * e] >> 11)) * 0x1p-53f;  // 1 - u1 in (0, 1]
    const float u2 = (float)(c[2 * e + 1] >> 11) * 0x1p-53f;
    const float rad = sqrtf(-2.0f * logf(v));
    float sn, cs;
    sincospif(2.0f * u2, &sn, &cs);
    const cpx<float> g = cmk<float>(sc * (rad * cs), sc * (rad * sn));
    if (e == 0) *n0 = g; else *n1 = g;
  }
}

// ------------------------------------------------------------ block scans --
// In-place exclusive prefix sum of n ints in LDS; returns the total.  Every
// thread of the work-group must call it.  `part` is LDS scratch of kWG ints.
__device__ inline int block_exscan(int* a, int n, int* part) {
  const int tid = threadIdx.x;
  const int chunk = (n + kWG - 1) / kWG;
  const int lo = min(n, tid * chunk), hi = min(n, lo + chunk);
  int s = 0;
  for (int i = lo; i < hi; ++i) s += a[i];
  part[tid] = s;
  __syncthreads();
  for (int off = 1; off < kWG; off <<= 1) {
    const int v = (tid >= off) ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int base = (tid == 0) ? 0 : part[tid - 1];
  const int total = part[kWG - 1];
  for (int i = lo; i < hi; ++i) {
    const int v = a[i];
    a[i] = base;
    base += v;
  }
  __syncthreads();
  return total;
}

__device__ inline int block_sum(int v, int* part) {
  const int tid = threadIdx.x;
  part[tid] = v;
  __syncthreads();
  for (int off = kWG / 2; off > 0; off >>= 1) {
    if (tid < off) part[tid] += part[tid + off];
    __syncthreads();
  }
  const int r = part[0];
  __syncthreads();
  return r;
}

// ----------------------------------------------------- LDS Stockham FFT ----
// The DFT buffer in LDS holds element i at i + i / 16 (one complex of padding
// after every 16): the strided writes of the first Stockham passes (16 or 256
// elements apart) then spread over the LDS banks instead of hitting one.
__device__ __forceinline__ int lp(int i) { return i + (i >> 4); }

// One radix-R pass of the Stockham autosort FFT over L points in LDS:
// item j (k = j mod Ns) reads x_r = buf[j + r L/R], multiplies by
// w^{r k} with w = exp(-+2 pi i / (Ns R)), applies the R-point DFT and writes
// buf[(j - k) R + k + r Ns].  All items are read before any is written.
// 4-point DFT of x[0], x[s], x[2s], x[3s] in place (forward: exp(-2 pi i / 4)).
template <typename T>
__device__ __forceinline__ void dft4(cpx<T>* x, int s, bool inv) {
  const cpx<T> t0 = cadd(x[0], x[2 * s]), t1 = csub(x[0], x[2 * s]);
  const cpx<T> t2 = cadd(x[s], x[3 * s]), t3 = csub(x[s], x[3 * s]);
  const cpx<T> mi_t3 = cmk<T>(t3.y, -t3.x);  // -i * t3
  x[0] = cadd(t0, t2);
  x[2 * s] = csub(t0, t2);
  x[s] = inv ? csub(t1, mi_t3) : cadd(t1, mi_t3);
  x[3 * s] = inv ? cadd(t1, mi_t3) : csub(t1, mi_t3);
}

template <typename T, int R>
__device__ __forceinline__ void butterfly(cpx<T>* x, bool inv) {
  if (R == 16) {
    // n = 4 n1 + n2, k = k1 + 4 k2: DFT4 over n1, twiddle W16^{n2 k1}, DFT4 over n2.
    for (int n2 = 0; n2 < 4; ++n2) dft4<T>(x + n2, 4, inv);
    // x[4 k1 + n2] now holds Y[n2][k1]; multiply by W16^{n2 k1}
    const T c1 = (T)0.92387953251128675613, s1 = (T)0.38268343236508977173;
    const T h = (T)0.70710678118654752440;
    const cpx<T> w[10] = {cmk<T>(1, 0),  cmk<T>(c1, -s1), cmk<T>(h, -h),  cmk<T>(s1, -c1),
                          cmk<T>(0, -1), cmk<T>(-s1, -c1), cmk<T>(-h, -h), cmk<T>(-c1, -s1),
                          cmk<T>(-1, 0), cmk<T>(-c1, s1)};
#pragma unroll
    for (int k1 = 1; k1 < 4; ++k1)
#pragma unroll
      for (int n2 = 1; n2 < 4; ++n2) {
        cpx<T> tw = w[n2 * k1];
        if (inv) tw.y = -tw.y;
        x[4 * k1 + n2] = cmul(x[4 * k1 + n2], tw);
      }
    for (int k1 = 0; k1 < 4; ++k1) dft4<T>(x + 4 * k1, 1, inv);
    // x[4 k1 + k2] holds X[k1 + 4 k2]: transpose the 4 x 4 block
    cpx<T> y[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) y[i] = x[i];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) x[k1 + 4 * k2] = y[4 * k1 + k2];
  } else if (R == 8) {
    // n = 4 n1 + n2, k = k1 + 2 k2: DFT2 over n1, twiddle W8^{n2 k1}, DFT4 over n2.
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      const cpx<T> a = x[n2], b = x[4 + n2];
      x[n2] = cadd(a, b);
      x[4 + n2] = csub(a, b);
    }
    const T h = (T)0.70710678118654752440;
    const T sg = inv ? (T)1 : (T)-1;  // sign of the imaginary part of W8^1 and W8^2
    x[5] = cmul(x[5], cmk<T>(h, sg * h));
    x[6] = cmul(x[6], cmk<T>(0, sg));
    x[7] = cmul(x[7], cmk<T>(-h, sg * h));
    dft4<T>(x, 1, inv);
    dft4<T>(x + 4, 1, inv);
    // x[4 k1 + k2] holds X[k1 + 2 k2]
    cpx<T> y[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) y[i] = x[i];
#pragma unroll
    for (int k1 = 0; k1 < 2; ++k1)
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) x[k1 + 2 * k2] = y[4 * k1 + k2];
  } else if (R == 2) {
    const cpx<T> a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  } else {
    const cpx<T> t0 = cadd(x[0], x[2]), t1 = csub(x[0], x[2]);
    const cpx<T> t2 = cadd(x[1], x[3]), t3 = csub(x[1], x[3]);
    // -i * t3 = (t3.y, -t3.x)
    const cpx<T> mi_t3 = cmk<T>(t3.y, -t3.x);
    x[0] = cadd(t0, t2);
    x[2] = csub(t0, t2);
    if (!inv) {
      x[1] = cadd(t1, mi_t3);
      x[3] = csub(t1, mi_t3);
    } else {
      x[1] = csub(t1, mi_t3);
      x[3] = cadd(t1, mi_t3);
    }
  }
}

// Twiddle exp(-2 pi i t / L) from the two LDS tables T1[i] = exp(-2 pi i 64 i / L),
// T2[j] = exp(-2 pi i j / L): one complex product per lookup.
template <typename T>
__device__ __forceinline__ cpx<T> twiddle(const cpx<T>* T1, const cpx<T>* T2, int t) {
  return cmul(T1[t >> kTwiddleBits], T2[t & ((1 << kTwiddleBits) - 1)]);
}

// One in-place pass: every thread holds its up to MAXV items in registers
// between the read and the write phase, so L <= MAXV * kWG.
template <typename T, int R, int MAXV>
__device__ void stockham_pass(cpx<T>* buf, int L, int Ns, const cpx<T>* T1, const cpx<T>* T2,
                              bool inv) {
  constexpr int NQ = MAXV / R;
  cpx<T> v[MAXV];
  const int nitems = L / R;
  const int tw_mul = L / (Ns * R);
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int j = tid + q * kWG;
    if (j < nitems) {
      const int k = j & (Ns - 1);
      cpx<T> x[R];
#pragma unroll
      for (int r = 0; r < R; ++r) x[r] = buf[lp(j + r * nitems)];
      if (Ns > 1) {
        if (R == 16) {
          // w^r = w^{4a} w^b with w^{4a} from the table (a = 1, 2) or one product,
          // w^b from at most two products: every factor within a few ulp
          cpx<T> w1 = twiddle(T1, T2, k * tw_mul);
          cpx<T> w4 = twiddle(T1, T2, 4 * k * tw_mul);
          cpx<T> w8 = twiddle(T1, T2, 8 * k * tw_mul);
          if (inv) {
            w1.y = -w1.y;
            w4.y = -w4.y;
            w8.y = -w8.y;
          }
          const cpx<T> w2 = cmul(w1, w1), w3 = cmul(w2, w1), w12 = cmul(w8, w4);
          const cpx<T> lo[4] = {cmk<T>(1, 0), w1, w2, w3};
          const cpx<T> hi[4] = {cmk<T>(1, 0), w4, w8, w12};
#pragma unroll
          for (int r = 1; r < R; ++r) {
            const cpx<T> wr = (r & 3) == 0 ? hi[r >> 2]
                              : (r >> 2) == 0 ? lo[r & 3]
                                              : cmul(hi[r >> 2], lo[r & 3]);
            x[r] = cmul(x[r], wr);
          }
        } else {
          // w^k, then its powers by multiplication
          cpx<T> w1 = twiddle(T1, T2, k * tw_mul);
          if (inv) w1.y = -w1.y;
          cpx<T> wr = w1;
#pragma unroll
          for (int r = 1; r < R; ++r) {
            x[r] = cmul(x[r], wr);
            if (r + 1 < R) wr = cmul(wr, w1);
          }
        }
      }
      butterfly<T, R>(x, inv);
#pragma unroll
      for (int r = 0; r < R; ++r) v[q * R + r] = x[r];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int j = tid + q * kWG;
    if (j < nitems) {
      const int k = j & (Ns - 1);
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[lp(base + r * Ns)] = v[q * R + r];
    }
  }
  __syncthreads();
}

// LDS twiddle tables for length L (T1: max(1, L/64) entries, T2: min(L, 64)).
template <typename T>
__device__ void twiddle_tables(int L, cpx<T>* T1, cpx<T>* T2) {
  const int n1 = (L >> kTwiddleBits) > 0 ? (L >> kTwiddleBits) : 1;
  const int n2 = L < (1 << kTwiddleBits) ? L : (1 << kTwiddleBits);
  for (int i = threadIdx.x; i < n1 + n2; i += kWG) {
    const int t = (i < n1) ? (i << kTwiddleBits) : (i - n1);
    double c, s;
    expipi(-2.0 * (double)t / (double)L, &c, &s);
    const cpx<T> w = cmk<T>((T)c, (T)s);
    if (i < n1)
      T1[i] = w;
    else
      T2[i - n1] = w;
  }
  __syncthreads();
}

// Unnormalised power-of-two FFT of L points in LDS, forward (exp(-2 pi i ...))
// or inverse (exp(+2 pi i ...)), Stockham: log2 L = 4 a + b, radix-2 / radix-4
// passes for b, then a radix-16 passes.  MAXV = L / kWG items per thread.
template <typename T, int MAXV>
__device__ __forceinline__ void fft_lds_v(cpx<T>* buf, int L, int log2L, const cpx<T>* T1,
                                          const cpx<T>* T2, bool inv, int fs) {
  int Ns = 1;
  const int b = log2L & 3;
  if (b == 3 && fs == kFftRadix8Head) {
    stockham_pass<T, 8, MAXV>(buf, L, Ns, T1, T2, inv);
    Ns = 8;
  } else if (b & 1) {
    stockham_pass<T, 2, MAXV>(buf, L, Ns, T1, T2, inv);
    Ns = 2;
  }
  if ((b & 2) && Ns < 8) {
    stockham_pass<T, 4, MAXV>(buf, L, Ns, T1, T2, inv);
    Ns *= 4;
  }
  while (Ns < L) {
    stockham_pass<T, 16, MAXV>(buf, L, Ns, T1, T2, inv);
    Ns *= 16;
  }
}

// L <= MaxL<T>.
template <typename T>
__device__ __forceinline__ void fft_lds(cpx<T>* buf, int L, int log2L, const cpx<T>* T1,
                                        const cpx<T>* T2, bool inv, int fs) {
  fft_lds_v<T, MaxL<T>::value / kWG>(buf, L, log2L, T1, T2, inv, fs);
}

// Element-wise Bluestein steps with the global loads of U consecutive thread
// strides issued together (one memory latency per U elements instead of per
// element).  buf has n_all points of G sequences of length L (2^log2L).
constexpr int kLoadBlock = 8;

template <typename T>
__device__ __forceinline__ void bs_chirp_in(cpx<T>* buf, const cpx<T>* x0, int vstride, int n_all,
                                            int p, int L, int log2L, const cpx<T>* chirp) {
  for (int n0 = threadIdx.x; n0 < n_all; n0 += kLoadBlock * kWG) {
    cpx<T> xv[kLoadBlock], cv[kLoadBlock];
#pragma unroll
    for (int u = 0; u < kLoadBlock; ++u) {
      const int n = n0 + u * kWG;
      const int g = n >> log2L, m = n & (L - 1);
      xv[u] = cmk<T>(0, 0);
      cv[u] = cmk<T>(0, 0);
      if (n < n_all && m < p) {
        xv[u] = x0[(size_t)g * vstride + m];
        cv[u] = chirp[m];
      }
    }
#pragma unroll
    for (int u = 0; u < kLoadBlock; ++u) {
      const int n = n0 + u * kWG;
      if (n < n_all) buf[lp(n)] = cmul(xv[u], cv[u]);
    }
  }
}

template <typename T>
__device__ __forceinline__ void bs_filter(cpx<T>* buf, int n_all, int L, const cpx<T>* bhat) {
  for (int n0 = threadIdx.x; n0 < n_all; n0 += kLoadBlock * kWG) {
    cpx<T> hv[kLoadBlock];
#pragma unroll
    for (int u = 0; u < kLoadBlock; ++u) {
      const int n = n0 + u * kWG;
      hv[u] = (n < n_all) ? bhat[n & (L - 1)] : cmk<T>(0, 0);
    }
#pragma unroll
    for (int u = 0; u < kLoadBlock; ++u) {
      const int n = n0 + u * kWG;
      if (n < n_all) buf[lp(n)] = cmul(buf[lp(n)], hv[u]);
    }
  }
}

template <typename T>
__device__ __forceinline__ void bs_chirp_out(cpx<T>* x0, int vstride, int G, int p, int L,
                                             const cpx<T>* buf, const cpx<T>* chirp) {
  const T invL = (T)1 / (T)L;
  const int n_out = G * p;
  for (int n0 = threadIdx.x; n0 < n_out; n0 += kLoadBlock * kWG) {
    cpx<T> cv[kLoadBlock];
#pragma unroll
    for (int u = 0; u < kLoadBlock; ++u) {
      const int n = n0 + u * kWG;
      cv[u] = (n < n_out) ? chirp[n % p] : cmk<T>(0, 0);
    }
#pragma unroll
    for (int u = 0; u < kLoadBlock; ++u) {
      const int n = n0 + u * kWG;
      if (n < n_out) {
        const int g = n / p, m = n - g * p;
        x0[(size_t)g * vstride + m] = cscale(cmul(buf[lp(g * L + m)], cv[u]), invL);
      }
    }
  }
}

// ------------------------------------------------ Bluestein prime DFT ----
// X[h] = sum_n x[n] exp(-2 pi i h n / p) for prime p as the cyclic convolution
// X = chirp . IFFT_L(FFT_L(x . chirp) . bhat) / L with L a power of two >= 2p - 1,
// chirp[n] = exp(-i pi (n^2 mod 2p) / p) and bhat = FFT_L(b), b[n] =
// conj(chirp[|n|]) for |n| < p (indices mod L), 0 elsewhere.
//
// L-point transforms up to MaxL<T> run in LDS (R = 1).  Longer ones (L = R M,
// M = MaxL<T>, R = 2 or 4) run as R in-LDS M-point FFTs: decimation in time
// splits the forward transform into the FFTs of the points x[R m + r], kept in
// the slot buffer G (row r of M points each); one element-wise pass over k < M
// finishes it with the R-point butterflies X[k + j M] = sum_r W_R^{rj} W^{rk}
// G_r[k] (W = exp(-2 pi i / L)), multiplies by the filter spectrum and starts
// the inverse transform by decimation in frequency, a_r[k] = W^{-rk} sum_j
// W_R^{-rj} Z[k + j M]; the inverse M-point FFTs of the rows a_r are the points
// R m + r of the convolution.
template <typename T>
struct BsTabs {
  const cpx<T>* T1M;  // twiddle tables of the M-point FFT
  const cpx<T>* T2M;
  const cpx<T>* T1L;  // of the L-point butterflies (R > 1)
  const cpx<T>* T2L;
};

template <typename T>
__device__ __forceinline__ BsTabs<T> bs_tables(int L, int M, cpx<T>* tab) {
  cpx<T>* t1m = tab;
  cpx<T>* t2m = t1m + ((M >> kTwiddleBits) > 0 ? (M >> kTwiddleBits) : 1);
  cpx<T>* t1l = t2m + (1 << kTwiddleBits);
  cpx<T>* t2l = t1l + (L >> kTwiddleBits);
  twiddle_tables<T>(M, t1m, t2m);
  if (L > M) twiddle_tables<T>(L, t1l, t2l);
  BsTabs<T> tb;
  tb.T1M = t1m;
  tb.T2M = t2m;
  tb.T1L = t1l;
  tb.T2L = t2l;
  return tb;
}

// The R-point butterflies of the element-wise pass at k (R = 2 or 4): with
// filter = true the whole middle step on G (forward butterflies, filter,
// inverse butterflies); with filter = false the forward butterflies alone,
// written to out (the filter spectrum's set-up).
template <typename T, int R>
__device__ __forceinline__ void bs_middle(cpx<T>* G, int M, int k, const cpx<T>* bhat,
                                          cpx<T>* out, bool filter, const BsTabs<T>& tb) {
  cpx<T> g[R], w[R];
  w[0] = cmk<T>(1, 0);
  g[0] = G[k];
#pragma unroll
  for (int r = 1; r < R; ++r) {
    w[r] = twiddle(tb.T1L, tb.T2L, r * k);
    g[r] = cmul(G[(size_t)r * M + k], w[r]);
  }
  butterfly<T, R>(g, false);
  if (!filter) {
#pragma unroll
    for (int j = 0; j < R; ++j) out[(size_t)j * M + k] = g[j];
    return;
  }
#pragma unroll
  for (int j = 0; j < R; ++j) g[j] = cmul(g[j], bhat[(size_t)j * M + k]);
  butterfly<T, R>(g, true);
  G[k] = g[0];
#pragma unroll
  for (int r = 1; r < R; ++r) G[(size_t)r * M + k] = cmul(g[r], cmk<T>(w[r].x, -w[r].y));
}

// setup = true: writes chirp (p points) and bhat (L points); x is not used.
// setup = false: the DFT of x (p points, global) in place with them.  R = L / M
// is 1, 2 or 4; G (L points, global) is used only when R > 1.  Every FFT of the
// step goes through the one forward fft_lds call below: the inverse transforms
// run as conj(FFT(conj(.))), the conjugations folded into the loads and stores.
template <typename T>
__device__ __noinline__ void bluestein_run(bool setup, cpx<T>* x, int p, int L, int R,
                                              int log2M, cpx<T>* chirp, cpx<T>* bhat,
                                              cpx<T>* G, cpx<T>* buf, const BsTabs<T>& tb,
                                              int fs) {
  const int M = L / R;
  const int tid = threadIdx.x;
  if (setup) {
    for (int n = tid; n < p; n += kWG) {
      const int64_t q = ((int64_t)n * n) % (2 * (int64_t)p);
      double c, s;
      expipi(-(double)q / (double)p, &c, &s);
      chirp[n] = cmk<T>((T)c, (T)s);
    }
    __syncthreads();
  }
  const T invL = (T)1 / (T)L;
  const int passes = setup ? R : 2 * R;
  for (int it = 0; it < passes; ++it) {
    const bool inv = it >= R;
    const int r = it & (R - 1);
    if (R > 1 && it == R) {
      for (int k = tid; k < M; k += kWG) {
        if (R == 2)
          bs_middle<T, 2>(G, M, k, bhat, nullptr, true, tb);
        else
          bs_middle<T, 4>(G, M, k, bhat, nullptr, true, tb);
      }
      __syncthreads();
    }
    if (R > 1 || !inv) {
      // (R = 1, inverse: the filtered spectrum is already in buf)
      for (int m0 = tid; m0 < M; m0 += kLoadBlock * kWG) {
        cpx<T> v[kLoadBlock];
#pragma unroll
        for (int u = 0; u < kLoadBlock; ++u) {
          const int m = m0 + u * kWG, n = R * m + r;
          cpx<T> a = cmk<T>(0, 0);
          if (m < M) {
            if (inv) {
              a = G[(size_t)r * M + m];
              a.y = -a.y;
            } else if (setup) {
              if (n < p) a = chirp[n];
              else if (n > L - p) a = chirp[L - n];
              a.y = -a.y;
            } else if (n < p) {
              a = cmul(x[n], chirp[n]);
            }
          }
          v[u] = a;
        }
#pragma unroll
        for (int u = 0; u < kLoadBlock; ++u) {
          const int m = m0 + u * kWG;
          if (m < M) buf[lp(m)] = v[u];
        }
      }
      __syncthreads();
    }
    fft_lds<T>(buf, M, log2M, tb.T1M, tb.T2M, false, fs);
    for (int m0 = tid; m0 < M; m0 += kLoadBlock * kWG) {
      cpx<T> f[kLoadBlock];
#pragma unroll
      for (int u = 0; u < kLoadBlock; ++u) {
        const int m = m0 + u * kWG, n = R * m + r;
        f[u] = cmk<T>(0, 0);
        if (m < M) {
          if (inv) {
            if (n < p) f[u] = chirp[n];
          } else if (R == 1 && !setup) {
            f[u] = bhat[m];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < kLoadBlock; ++u) {
        const int m = m0 + u * kWG, n = R * m + r;
        if (m < M) {
          cpx<T> v = buf[lp(m)];
          if (inv) {
            v.y = -v.y;
            if (n < p) x[n] = cscale(cmul(v, f[u]), invL);
          } else if (R > 1) {
            G[(size_t)r * M + m] = v;
          } else if (setup) {
            bhat[m] = v;
          } else {
            // filtered, and conjugated for the inverse transform that follows
            v = cmul(v, f[u]);
            v.y = -v.y;
            buf[lp(m)] = v;
          }
        }
      }
    }
    __syncthreads();
  }
  if (setup && R > 1) {
    for (int k = tid; k < M; k += kWG) {
      if (R == 2)
        bs_middle<T, 2>(G, M, k, nullptr, bhat, false, tb);
      else
        bs_middle<T, 4>(G, M, k, nullptr, bhat, false, tb);
    }
    __syncthreads();
  }
}

// ---------------------------------------- batched small DFTs (FP32) ------
// G independent L-point sequences back to back in LDS (G L <= MAXV kWG), one
// Stockham radix-R pass over all of them: the later rounds' short transforms
// then keep every thread busy instead of L / R of them.
template <typename T, int R, int MAXV>
__device__ void stockham_pass_b(cpx<T>* buf, int L, int lgn, int G, int Ns, const cpx<T>* T1,
                                const cpx<T>* T2, bool inv) {
  constexpr int NQ = MAXV / R;
  cpx<T> v[MAXV];
  const int nitems = L / R;  // per sequence, 1 << lgn
  const int total = G * nitems;
  const int tw_mul = L / (Ns * R);
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int jj = tid + q * kWG;
    if (jj < total) {
      const int j = jj & (nitems - 1);
      const int b = (jj >> lgn) * L;  // first element of this sequence
      const int k = j & (Ns - 1);
      cpx<T> x[R];
#pragma unroll
      for (int r = 0; r < R; ++r) x[r] = buf[lp(b + j + r * nitems)];
      if (Ns > 1) {
        if (R == 16) {
          cpx<T> w1 = twiddle(T1, T2, k * tw_mul);
          cpx<T> w4 = twiddle(T1, T2, 4 * k * tw_mul);
          cpx<T> w8 = twiddle(T1, T2, 8 * k * tw_mul);
          if (inv) {
            w1.y = -w1.y;
            w4.y = -w4.y;
            w8.y = -w8.y;
          }
          const cpx<T> w2 = cmul(w1, w1), w3 = cmul(w2, w1), w12 = cmul(w8, w4);
          const cpx<T> lo[4] = {cmk<T>(1, 0), w1, w2, w3};
          const cpx<T> hi[4] = {cmk<T>(1, 0), w4, w8, w12};
#pragma unroll
          for (int r = 1; r < R; ++r) {
            const cpx<T> wr = (r & 3) == 0 ? hi[r >> 2]
                              : (r >> 2) == 0 ? lo[r & 3]
                                              : cmul(hi[r >> 2], lo[r & 3]);
            x[r] = cmul(x[r], wr);
          }
        } else {
          cpx<T> w1 = twiddle(T1, T2, k * tw_mul);
          if (inv) w1.y = -w1.y;
          cpx<T> wr = w1;
#pragma unroll
          for (int r = 1; r < R; ++r) {
            x[r] = cmul(x[r], wr);
            if (r + 1 < R) wr = cmul(wr, w1);
          }
        }
      }
      butterfly<T, R>(x, inv);
#pragma unroll
      for (int r = 0; r < R; ++r) v[q * R + r] = x[r];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int jj = tid + q * kWG;
    if (jj < total) {
      const int j = jj & (nitems - 1);
      const int b = (jj >> lgn) * L;
      const int k = j & (Ns - 1);
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[lp(b + base + r * Ns)] = v[q * R + r];
    }
  }
  __syncthreads();
}

template <typename T, int MAXV>
__device__ __forceinline__ void fft_lds_batch(cpx<T>* buf, int L, int log2L, int G,
                                              const cpx<T>* T1, const cpx<T>* T2, bool inv,
                                              int fs) {
  int Ns = 1;
  const int b = log2L & 3;
  if (b == 3 && fs == kFftRadix8Head) {
    stockham_pass_b<T, 8, MAXV>(buf, L, log2L - 3, G, Ns, T1, T2, inv);
    Ns = 8;
  } else if (b & 1) {
    stockham_pass_b<T, 2, MAXV>(buf, L, log2L - 1, G, Ns, T1, T2, inv);
    Ns = 2;
  }
  if ((b & 2) && Ns < 8) {
    stockham_pass_b<T, 4, MAXV>(buf, L, log2L - 2, G, Ns, T1, T2, inv);
    Ns *= 4;
  }
  while (Ns < L) {
    stockham_pass_b<T, 16, MAXV>(buf, L, log2L - 4, G, Ns, T1, T2, inv);
    Ns *= 16;
  }
}

// G sequences x_g = x0 + g vstride (length p) transformed together, in place.
template <typename T, int MAXV>
__device__ __forceinline__ void bluestein_dft_batch(cpx<T>* x0, int vstride, int G, int p, int L, int log2L,
                                    const cpx<T>* chirp, const cpx<T>* bhat, cpx<T>* buf,
                                    const cpx<T>* tab, int fs) {
  const int tid = threadIdx.x;
  const cpx<T>* T1 = tab;
  const cpx<T>* T2 = T1 + ((L >> kTwiddleBits) > 0 ? (L >> kTwiddleBits) : 1);
  const int n_all = G * L;
  (void)tid;
  bs_chirp_in<T>(buf, x0, vstride, n_all, p, L, log2L, chirp);
  __syncthreads();
  fft_lds_batch<T, MAXV>(buf, L, log2L, G, T1, T2, false, fs);
  bs_filter<T>(buf, n_all, L, bhat);
  __syncthreads();
  fft_lds_batch<T, MAXV>(buf, L, log2L, G, T1, T2, true, fs);
  bs_chirp_out<T>(x0, vstride, G, p, L, buf, chirp);
  __syncthreads();
}

// ------------------------------------------------- exponential sums -------
// (h * r) mod p exactly, for h, r < 2^16 with h * r < 2^32: the FP32 quotient
// estimate is off by at most one, fixed branch-free in each direction
// (unsigned minimum picks the in-range candidate).
__device__ __forceinline__ int mulmod(uint32_t h, uint32_t r, int p, float inv_p) {
  const uint32_t x = h * r;
  const uint32_t q = (uint32_t)(int)((float)x * inv_p);
  const uint32_t up = (uint32_t)p;
  uint32_t rem = x - q * up;
  rem = min(rem, rem + up);  // rem was negative
  rem = min(rem, rem - up);  // rem was >= p
  return (int)rem;
}

// The same with 24-bit multiplies, for p <= 2^14 and h < p + 128 (what the FP32
// sampler uses): h * r < 2^28.1, and the FP32 quotient estimate (absolute error
// below 0.01 on a quotient below 2^14 + 128) is off by at most one.
__device__ __forceinline__ uint32_t mulmod24(uint32_t h, uint32_t r, uint32_t p, float inv_p) {
  const uint32_t x = __umul24(h, r);
  const uint32_t q = (uint32_t)(int)((float)x * inv_p);
  uint32_t rem = x - __umul24(q, p);
  rem = min(rem, rem + p);
  rem = min(rem, rem - p);
  return rem;
}

typedef float floatx4 __attribute__((ext_vector_type(4)));

// FP32 line sampler on the matrix cores.  The S1 sample sets of one round
// share the points h/p along the unwrapped axis m, so
//   V[s][h] = sum_j C[j][s] * omega_p^{(h r_j) mod p},  r_j = y_{j,m} mod p,
// is a complex product C (S1 x M) times T (M x p) with T generated from the
// integer-reduced index.  As a real product, row 2s / 2s+1 hold Re / Im of set
// s and K index 2j / 2j+1 hold Re / Im of mode j; it runs as
// v_mfma_f32_16x16x4_f32 tiles: RT row tiles of 16 rows, NT column tiles of
// 16 points per wave, two modes per K step.
//
// Operands: `afrag` (global) holds A in lane order ([pair][RT][64], readable
// two pairs past npairs); `rr` (LDS) holds r_j, zero-padded two pairs past
// npairs, and `rs` the column steps (16 r_j) mod p; `tw` (LDS) holds omega_p^x;
// `abuf` (LDS, 2 x (kChunk + 1) pairs)
// stages A: the four waves share one A stream, copied cooperatively one chunk
// ahead.  Each chunk buffer also holds the first pair of the next chunk so the
// A fragments and twiddles of step pr + 1 can be read while the MFMAs of step
// pr run.
// B fragments of one K step: omega_p^{((h0 + 16 u) r) mod p} (Re or Im part
// selected by the caller's table offset) for the NT column tiles of a lane;
// `step` = (16 r) mod p.
// HALF: the table holds omega_p^x for x <= p/2 only (long lines whose full table does
// not fit in LDS); omega_p^x = conj(omega_p^(p - x)) above that, so the lanes reading
// the imaginary part (neg_im) negate it there.
template <int NT, bool HALF = false>
__device__ __forceinline__ void twiddle_column(const float* twf, uint32_t h0, uint32_t r,
                                               uint32_t step, uint32_t p, float inv_p,
                                               float* b, bool neg_im = false) {
  uint32_t idx = mulmod24(h0, r, p, inv_p);
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    if constexpr (HALF) {
      const uint32_t j = min(idx, p - idx);
      const float v = twf[2 * j];
      b[u] = (neg_im && j != idx) ? -v : v;
    } else {
      b[u] = twf[2 * idx];
    }
    const uint32_t t = idx + step;
    idx = min(t, t - p);  // t - p wraps above t when t < p
  }
}

// grp / ngrp: when ngrp work-groups share the line, this group takes the
// column-tile blocks grp, grp + ngrp, ... (block = one tile per wave); every
// point's sum is formed the same way whichever group computes it.
template <int RT, int NT, bool HALF = false, bool BLK = (RT * NT <= 12)>
__device__ void expsum_mfma(const float* __restrict__ afrag, const uint16_t* rr,
                            const uint16_t* rs,
                            const cpx<float>* tw, float* abuf, int npairs, int p, int S1,
                            cpx<float>* __restrict__ V, int vstride, int grp = 0,
                            int ngrp = 1) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  constexpr int NWAVES = kWG / 64;
  constexpr int NCOL = 16 * NT;
  constexpr int PAIR = RT * 64;                   // floats per pair
  constexpr int BUF = (kChunk + 1) * PAIR;        // floats per chunk buffer
  constexpr int CPY = (BUF + kWG - 1) / kWG;      // floats copied per thread per chunk
  const int ntiles = (p + NCOL - 1) / NCOL;
  const int passes = (ntiles + NWAVES * ngrp - 1) / (NWAVES * ngrp);
  const int nchunks = (npairs + kChunk - 1) / kChunk;
  const float inv_p = 1.0f / (float)p;
  const int kk = lane >> 4;       // K row of the B fragment
  const int col = lane & 15;      // column (point) of the B fragment
  const int jsel = kk >> 1;       // which mode of the pair
  const int tpart = kk & 1;       // Re / Im of the twiddle
  const float* twf = reinterpret_cast<const float*>(tw) + tpart;
  for (int pass = 0; pass < passes; ++pass) {
    const int tile = (pass * ngrp + grp) * NWAVES + wave;
    const bool active = tile < ntiles;
    const int hbase = tile * NCOL;
    const uint32_t h0 = (uint32_t)(hbase + col);
    // BLK: the MFMAs of one chunk (32 modes) accumulate from zero and the chunk
    // sum is then added to `tot`, so the FP32 rounding of a long sum grows with
    // the chunk sums instead of the running total (used where the registers allow)
    floatx4 acc[RT][NT], tot[RT][NT];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int u = 0; u < NT; ++u) {
        acc[t][u] = floatx4{0.f, 0.f, 0.f, 0.f};
        tot[t][u] = floatx4{0.f, 0.f, 0.f, 0.f};
      }
    // chunk 0 into buffer 0
#pragma unroll
    for (int q = 0; q < CPY; ++q) {
      const int e = threadIdx.x + q * kWG;
      if (e < BUF) abuf[e] = afrag[e];
    }
    __syncthreads();
    float a_cur[RT], b_cur[NT];
#pragma unroll
    for (int t = 0; t < RT; ++t) a_cur[t] = abuf[t * 64 + lane];
    const uint32_t up = (uint32_t)p;
    twiddle_column<NT, HALF>(twf, h0, (uint32_t)rr[jsel], (uint32_t)rs[jsel], up, inv_p, b_cur,
                             tpart == 1);
    uint32_t r1 = (uint32_t)rr[2 + jsel];       // residue of step pr + 1
    uint32_t s1 = (uint32_t)rs[2 + jsel];
    for (int c = 0; c < nchunks; ++c) {
      const float* ab = abuf + (c & 1) * BUF;
      // next chunk's A, held in registers while this chunk computes
      float stage[CPY];
      if (c + 1 < nchunks) {
        const float* src = afrag + (size_t)(c + 1) * kChunk * PAIR;
#pragma unroll
        for (int q = 0; q < CPY; ++q) {
          const int e = threadIdx.x + q * kWG;
          stage[q] = (e < BUF) ? src[e] : 0.f;
        }
      }
      const int k1 = min(kChunk, npairs - c * kChunk);
      if (active) {
        if constexpr (BLK) {
#pragma unroll
          for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int u = 0; u < NT; ++u) acc[t][u] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
        for (int q = 0; q < k1; ++q) {
          const int pr = c * kChunk + q;
          // operands of step pr + 1 (A from this chunk buffer, twiddles from the
          // residue loaded one step earlier) and the residue of step pr + 2
          float a_nxt[RT], b_nxt[NT];
          twiddle_column<NT, HALF>(twf, h0, r1, s1, up, inv_p, b_nxt, tpart == 1);
#pragma unroll
          for (int t = 0; t < RT; ++t) a_nxt[t] = ab[(q + 1) * PAIR + t * 64 + lane];
          const uint32_t r2 = (uint32_t)rr[2 * (pr + 2) + jsel];
          const uint32_t s2 = (uint32_t)rs[2 * (pr + 2) + jsel];
#pragma unroll
          for (int u = 0; u < NT; ++u)
#pragma unroll
            for (int t = 0; t < RT; ++t)
              acc[t][u] =
                  __builtin_amdgcn_mfma_f32_16x16x4f32(a_cur[t], b_cur[u], acc[t][u], 0, 0, 0);
          if constexpr (RT <= 2) {
            // one or two row tiles: interleaving LDS reads and index arithmetic
            // between the MFMAs measured faster than the compiler's own order;
            // from three row tiles on the compiler's order is faster
#pragma unroll
            for (int g = 0; g < RT * NT; ++g) {
              __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // one MFMA
              __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // one LDS read
              __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);   // three VALU
            }
          }
#pragma unroll
          for (int t = 0; t < RT; ++t) a_cur[t] = a_nxt[t];
#pragma unroll
          for (int u = 0; u < NT; ++u) b_cur[u] = b_nxt[u];
          r1 = r2;
          s1 = s2;
        }
        if constexpr (BLK) {
#pragma unroll
          for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int u = 0; u < NT; ++u) tot[t][u] += acc[t][u];
        }
      }
      if (c + 1 < nchunks) {
        float* dst = abuf + ((c + 1) & 1) * BUF;
#pragma unroll
        for (int q = 0; q < CPY; ++q) {
          const int e = threadIdx.x + q * kWG;
          if (e < BUF) dst[e] = stage[q];
        }
      }
      __syncthreads();
    }
    // D layout: lane holds rows 4*(lane/16) + i (i = 0..3) of column lane%16;
    // rows 4*kk, 4*kk+1 are Re, Im of set 2*kk (+ 8 t), rows 4*kk+2, +3 of the next set.
    if (active) {
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const int s0 = 8 * t + 2 * kk;
#pragma unroll
        for (int u = 0; u < NT; ++u) {
          const int h = hbase + 16 * u + col;
          const floatx4 r = BLK ? tot[t][u] : acc[t][u];
          if (h < p) {
            if (s0 < S1) V[(size_t)s0 * vstride + h] = cmk<float>(r[0], r[1]);
            if (s0 + 1 < S1) V[(size_t)(s0 + 1) * vstride + h] = cmk<float>(r[2], r[3]);
          }
        }
      }
    }
  }
}

// Column tiles per wave for a round with prime p: the widest tile (best reuse
// of each A fragment) that still gives every wave about the same number of
// columns; a tile pass costs about 4 column tiles' worth of fixed overhead.  Any
// width from 2 to 8 tiles: e.g. p = 323 takes 7 tiles of 48 points in two passes
// (96 points per wave) where 64-point tiles would need 128.
__host__ __device__ inline int choose_nt(int p) {
  // below 640 points the chunk-blocked accumulation (at most 4 column tiles)
  // keeps the FP32 error of the long planted sum small relative to F / p
  int best = 8;
  int best_cost = 1 << 30;
  for (int nt = (p < 640 ? 4 : 8); nt >= 2; --nt) {
    const int tiles = (p + 16 * nt - 1) / (16 * nt);
    const int passes = (tiles + 3) / 4;
    const int cost = passes * (16 * nt + 64);
    if (cost < best_cost) {
      best_cost = cost;
      best = nt;
    }
  }
  return best;
}

// Noise of the synthetic black box, added to every sample of sets s_begin ..
// s_end - 1 of the round (one Philox block per pair of points).
template <typename T>
__device__ void add_noise(cpx<T>* __restrict__ V, int vstride, int p, int s_begin, int s_end,
                          uint64_t seed, uint64_t signal, int round, double sigma) {
  if (!(sigma > 0.0)) return;
  const int np2 = (p + 1) / 2;
  for (int q = threadIdx.x; q < (s_end - s_begin) * np2; q += kWG) {
    const int s = s_begin + q / np2, hp = q - (s - s_begin) * np2;
    cpx<T>* v = V + (size_t)s * vstride + 2 * hp;
    if constexpr (sizeof(T) == 4) {
      cpx<float> n0, n1;
      noise_pair32(seed, signal, (uint64_t)round, (uint64_t)s, (uint64_t)hp, (float)sigma, &n0,
                   &n1);
      v[0] = cadd(v[0], n0);
      if (2 * hp + 1 < p) v[1] = cadd(v[1], n1);
    } else {
      cpx<double> n0, n1;
      noise_pair64(seed, signal, (uint64_t)round, (uint64_t)s, (uint64_t)hp, sigma, &n0, &n1);
      v[0] = cadd(v[0], n0);
      if (2 * hp + 1 < p) v[1] = cadd(v[1], n1);
    }
  }
}

// FP64 line sampler on the vector units, V[s][h] = sum_j C[j][s] omega_p^{(h r_j) mod p}
// (C: [M][S1] coefficient rows, global; rr: r_j, LDS; tw: omega_p^x, LDS).  A tile
// is a block of SB sets times 64 HB points; the four waves of the work-group share
// a tile, each summing a quarter of every chunk of kF64Chunk modes, whose
// coefficients for the tile's sets are first staged in LDS (`stage`, kF64StageBytes):
// per mode a wave reads SB coefficients (one address for all lanes) and HB twiddles
// (indices stepped by (64 r_j) mod p), and each lane accumulates SB x HB complex
// sums in registers.  The four partial sums are added in wave order through
// `stage`.  (grp / ngrp: several work-groups on one line, this one taking every
// ngrp-th tile.)
template <int SB, int HB>
__device__ void expsum_f64_tiled(const cpx<double>* __restrict__ C, const uint16_t* rr,
                                 const cpx<double>* tw, cpx<double>* stage, int M, int p, int S1,
                                 cpx<double>* __restrict__ V, int vstride, int grp = 0,
                                 int ngrp = 1) {
  static_assert(kF64Chunk * SB * 16 <= kF64StageBytes && SB * HB * 64 * 16 <= kF64StageBytes,
                "FP64 sampler stage");
  constexpr int NW = kWG / 64;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ngroups = (S1 + SB - 1) / SB;
  const int nchunks = (p + 64 * HB - 1) / (64 * HB);
  const float inv_p = 1.0f / (float)p;
  for (int tile = grp; tile < ngroups * nchunks; tile += ngrp) {
    const int g = tile / nchunks, hc = tile - g * nchunks;
    const int s0 = g * SB;
    const uint32_t h0 = (uint32_t)(hc * 64 * HB + lane);
    cpx<double> acc[SB][HB];
#pragma unroll
    for (int b = 0; b < SB; ++b)
#pragma unroll
      for (int u = 0; u < HB; ++u) acc[b][u] = cmk<double>(0.0, 0.0);
    for (int j0 = 0; j0 < M; j0 += kF64Chunk) {
      const int jn = min(kF64Chunk, M - j0);
      // the chunk's coefficients of the tile's sets (padding sets repeat the last)
      for (int e = threadIdx.x; e < jn * SB; e += kWG) {
        const int q = e / SB, b = e - q * SB;
        stage[e] = C[(size_t)(j0 + q) * S1 + min(s0 + b, S1 - 1)];
      }
      __syncthreads();
      const int jq = (jn + NW - 1) / NW;
      const int ja = wave * jq, jb = min(jn, ja + jq);
#pragma unroll 2
      for (int q = ja; q < jb; ++q) {
        const uint32_t r = rr[j0 + q];
        const uint32_t step = (uint32_t)mulmod(64u, r, p, inv_p);
        uint32_t idx = (uint32_t)mulmod(h0, r, p, inv_p);
        cpx<double> t[HB];
#pragma unroll
        for (int u = 0; u < HB; ++u) {
          t[u] = tw[idx];
          const uint32_t nx = idx + step;
          idx = min(nx, nx - (uint32_t)p);  // nx - p wraps above nx when nx < p
        }
        const cpx<double>* cq = stage + q * SB;
#pragma unroll
        for (int b = 0; b < SB; ++b) {
          const cpx<double> c = cq[b];
#pragma unroll
          for (int u = 0; u < HB; ++u) {
            acc[b][u].x = fma(c.x, t[u].x, fma(-c.y, t[u].y, acc[b][u].x));
            acc[b][u].y = fma(c.x, t[u].y, fma(c.y, t[u].x, acc[b][u].y));
          }
        }
      }
      __syncthreads();
    }
    // wave 0 adds the other waves' sums, in wave order
    for (int w = 1; w < NW; ++w) {
      if (wave == w) {
#pragma unroll
        for (int b = 0; b < SB; ++b)
#pragma unroll
          for (int u = 0; u < HB; ++u) stage[(b * HB + u) * 64 + lane] = acc[b][u];
      }
      __syncthreads();
      if (wave == 0) {
#pragma unroll
        for (int b = 0; b < SB; ++b)
#pragma unroll
          for (int u = 0; u < HB; ++u) acc[b][u] = cadd(acc[b][u], stage[(b * HB + u) * 64 + lane]);
      }
      __syncthreads();
    }
    if (wave == 0) {
#pragma unroll
      for (int b = 0; b < SB; ++b)
#pragma unroll
        for (int u = 0; u < HB; ++u) {
          const int s = s0 + b, h = (int)h0 + 64 * u;
          if (s < S1 && h < p) V[(size_t)s * vstride + h] = acc[b][u];
        }
    }
  }
}

// Sets per work item of the FP64 sampler: 2, 3 or 4, the fewest padding sets
// (ties to the larger block).
__host__ __device__ inline int f64_set_block(int S1) {
  int best = 4, waste = (4 - S1 % 4) % 4;
  for (int sb = 3; sb >= 2; --sb) {
    const int w = (sb - S1 % sb) % sb;
    if (w < waste) {
      waste = w;
      best = sb;
    }
  }
  return best;
}

}  // namespace sfft
