// Kernels of the full-length CQ-NSGT (Algorithms 1 and 2 at the signal
// length L, Section 3): batched power-of-two FFTs of any length up to
// kLongVals^2 (one LDS block up to kLongVals points, else a four-step FFT
// in two passes), the band gather X g_k wrapped modulo M_k (Algorithm 1) and
// the per-bin dual overlap-add (Algorithm 2).
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "common.hpp"
#include "fft_device.hpp"
#include "plan.hpp"

namespace slicq {

// e^{DIR 2 pi i m / n} for 0 <= m < n <= 2^24, from the FP64 sine and cosine
// of pi (2 m / n) (exact argument), rounded once to T.
template <class T, int DIR>
__device__ __forceinline__ C2<T> long_twiddle(int64_t m, int64_t n) {
  double s, c;
  sincospi(2.0 * (double)m / (double)n, &s, &c);
  return {(T)c, (T)(DIR > 0 ? s : -s)};
}

// Batched FFTs over a table of runs (FullRunDev): run r holds count
// sequences of length 2^logn at off (complex values, contiguous) and owns the
// blocks blk0 .. of its launch; a block finds its run by binary search. One
// launch transforms every run of a length class, whatever its length.
__device__ __forceinline__ int find_run(const FullRunDev* __restrict__ runs, int nruns, int64_t b) {
  int lo = 0, hi = nruns - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (runs[mid].blk0 <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Runs of length 2^logn <= kLongVals: a block transforms kLongVals >> logn
// sequences in LDS and writes scale * result. in may equal out (a block reads
// only what it writes).
template <class T, int DIR>
__global__ void __launch_bounds__(kLongThreads) k_long_fft(const FullRunDev* __restrict__ runs, int nruns,
                                                           const C2<T>* in, C2<T>* out, T scale,
                                                           const C2<T>* __restrict__ tw) {
  extern __shared__ unsigned char smem[];
  C2<T>* buf = reinterpret_cast<C2<T>*>(smem);
  const int tid = threadIdx.x;
  const FullRunDev R = runs[find_run(runs, nruns, blockIdx.x)];
  const int logn = R.logn;
  const int per = kLongVals >> logn;
  const int64_t s0 = (int64_t)(blockIdx.x - R.blk0) * per;
  const int ns = (int)imin64(per, R.count - s0);
  const int cnt = ns << logn;
  const int64_t g0 = R.off + (s0 << logn);
  for (int i = tid; i < cnt; i += kLongThreads) buf[pidx(i)] = in[g0 + i];
  __syncthreads();
  lds_fft<T, DIR, CONTIG, 16, 16>(buf, 0, logn, ns, 0, TwGlobal<T>{tw}, tid, kLongThreads);
  for (int i = tid; i < cnt; i += kLongThreads) out[g0 + i] = cscale(buf[pidx(i)], scale);
}

// Runs longer than kLongVals as a four-step FFT: n = n1 n2 (n1 = 2^logn1 <=
// n2 = 2^logn2 <= kLongVals, logn1 = logn / 2), element t1 n2 + t2 is row t1,
// column t2. Columns pass: each block transforms C = kLongVals / n1 adjacent
// columns over t1, multiplies element (k1, t2) by e^{DIR 2 pi i t2 k1 / n} and
// writes it to tmp[off + k1 n2 + t2] (tmp laid out like the data).
template <class T, int DIR>
__global__ void __launch_bounds__(kLongThreads) k_long_cols(const FullRunDev* __restrict__ runs, int nruns,
                                                            const C2<T>* __restrict__ in, C2<T>* __restrict__ tmp,
                                                            const C2<T>* __restrict__ tw) {
  extern __shared__ unsigned char smem[];
  C2<T>* buf = reinterpret_cast<C2<T>*>(smem);
  const int tid = threadIdx.x;
  const FullRunDev R = runs[find_run(runs, nruns, blockIdx.x)];
  const int logn1 = R.logn / 2, logn2 = R.logn - logn1;
  const int logC = kLongLog - logn1;
  const int C = 1 << logC;
  const int64_t n = int64_t(1) << R.logn;
  const int64_t lb = blockIdx.x - R.blk0;
  const int blocks_per_seq = 1 << (logn2 - logC);
  const int64_t s = lb / blocks_per_seq;
  const int t20 = (int)(lb % blocks_per_seq) << logC;
  const C2<T>* src = in + R.off + s * n + t20;
  for (int i = tid; i < kLongVals; i += kLongThreads) {
    const int c = i & (C - 1), t1 = i >> logC;
    buf[pidx((c << logn1) + t1)] = src[((int64_t)t1 << logn2) + c];
  }
  __syncthreads();
  lds_fft<T, DIR, CONTIG, 16, 16>(buf, 0, logn1, C, 0, TwGlobal<T>{tw}, tid, kLongThreads);
  C2<T>* dst = tmp + R.off + s * n + t20;
  for (int i = tid; i < kLongVals; i += kLongThreads) {
    const int c = i & (C - 1), k1 = i >> logC;
    const C2<T> v = buf[pidx((c << logn1) + k1)];
    dst[((int64_t)k1 << logn2) + c] = cmul(v, long_twiddle<T, DIR>((int64_t)(t20 + c) * k1, n));
  }
}

// Rows pass: each block transforms R = kLongVals / n2 adjacent rows k1 of
// tmp over t2 and writes scale * X[k1 + n1 k2] to out (out may be the
// columns pass's input).
template <class T, int DIR>
__global__ void __launch_bounds__(kLongThreads) k_long_rows(const FullRunDev* __restrict__ runs, int nruns,
                                                            const C2<T>* __restrict__ tmp, C2<T>* __restrict__ out,
                                                            T scale, const C2<T>* __restrict__ tw) {
  extern __shared__ unsigned char smem[];
  C2<T>* buf = reinterpret_cast<C2<T>*>(smem);
  const int tid = threadIdx.x;
  const FullRunDev Rn = runs[find_run(runs, nruns, blockIdx.x)];
  const int logn1 = Rn.logn / 2, logn2 = Rn.logn - logn1;
  const int logR = kLongLog - logn2;
  const int R = 1 << logR;
  const int64_t n = int64_t(1) << Rn.logn;
  const int64_t lb = blockIdx.x - Rn.blk0;
  const int blocks_per_seq = 1 << (logn1 - logR);
  const int64_t s = lb / blocks_per_seq;
  const int k10 = (int)(lb % blocks_per_seq) << logR;
  const C2<T>* src = tmp + Rn.off + s * n + ((int64_t)k10 << logn2);
  for (int i = tid; i < kLongVals; i += kLongThreads) buf[pidx(i)] = src[i];
  __syncthreads();
  lds_fft<T, DIR, CONTIG, 16, 16>(buf, 0, logn2, R, 0, TwGlobal<T>{tw}, tid, kLongThreads);
  C2<T>* dst = out + Rn.off + s * n + k10;
  for (int i = tid; i < kLongVals; i += kLongThreads) {
    const int r = i & (R - 1), k2 = i >> logR;
    dst[((int64_t)k2 << logn1) + r] = cscale(buf[pidx((r << logn2) + k2)], scale);
  }
}

// Algorithm 1's band step for every band at once: coefficient i of band k
// (off_k <= i < off_k + M_k, p = i - off_k) collects the bins j of J_k with
// j = p (mod M_k): out[i] = sum X[j mod L] g_k[j]. One thread per coefficient.
template <class T>
__global__ void __launch_bounds__(256) k_full_gather(const FullBandDev* __restrict__ bands, int nb,
                                                     const C2<T>* __restrict__ X, int64_t L,
                                                     const T* __restrict__ g, int64_t total,
                                                     C2<T>* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (bands[mid].off <= i) lo = mid;
    else hi = mid - 1;
  }
  const FullBandDev b = bands[lo];
  const int64_t p = i - b.off;
  int64_t d = (p - b.start) % b.M;
  if (d < 0) d += b.M;
  C2<T> acc{T(0), T(0)};
  for (int64_t t = d; t < b.len; t += b.M) {
    int64_t j = (b.start + t) % L;
    if (j < 0) j += L;
    const C2<T> x = X[j];
    const T w = g[b.goff + t];
    acc.x += x.x * w;
    acc.y += x.y * w;
  }
  out[i] = acc;
}

// Algorithm 2's overlap-add: Z[j] = sum over the bands covering bin j of
// g~_k[j] C_k[j mod M_k] (entries in increasing band order). One thread per bin.
template <class T>
__global__ void __launch_bounds__(256) k_full_ola(const int32_t* __restrict__ ent_off,
                                                  const int32_t* __restrict__ ent_idx,
                                                  const T* __restrict__ ent_w, const C2<T>* __restrict__ C,
                                                  int64_t L, C2<T>* __restrict__ Z) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= L) return;
  C2<T> acc{T(0), T(0)};
  const int e1 = ent_off[j + 1];
  for (int e = ent_off[j]; e < e1; ++e) {
    const C2<T> c = C[ent_idx[e]];
    const T w = ent_w[e];
    acc.x += c.x * w;
    acc.y += c.y * w;
  }
  Z[j] = acc;
}

// ---------------------------------------------------------------------------
// Launch sequences, on any launcher with launch(kernel, grid, block, shmem, args...).

// Workspace regions (bytes): C (band spectra, coef_count complex values),
// X / Z (L values), and the four-step scratch (max(L, coef_count) values).
struct FullWork {
  size_t c_off, x_off, t_off, total;
};

inline FullWork full_work(const FullPlan& f, int dtype) {
  const size_t cb = dtype == 0 ? 8 : 16;
  auto up = [](size_t v) { return (v + 255) & ~size_t(255); };
  FullWork w;
  w.c_off = 0;
  w.x_off = up(w.c_off + cb * (size_t)f.coef_count);
  w.t_off = up(w.x_off + cb * (size_t)f.L);
  w.total = up(w.t_off + cb * (size_t)(f.L > f.coef_count ? f.L : f.coef_count));
  return w;
}

template <class T>
constexpr size_t long_lds_bytes() { return (size_t)padded(kLongVals) * sizeof(C2<T>); }

// The transforms of one run table set (short runs, then long ones), scaled:
// short runs in one LDS block per kLongVals values, long ones as columns
// then rows through tmp.
template <class T, int DIR, class Ln>
void long_fft(Ln& ln, const char* tabs, const FullRunSet& rs, const C2<T>* in, C2<T>* out, C2<T>* tmp, T scale,
              const C2<T>* tw) {
  const auto* small = reinterpret_cast<const FullRunDev*>(tabs + rs.small);
  const auto* large = reinterpret_cast<const FullRunDev*>(tabs + rs.large);
  if (rs.nsmall)
    ln.launch(k_long_fft<T, DIR>, rs.blk_small, kLongThreads, long_lds_bytes<T>(), small, rs.nsmall, in, out, scale,
              tw);
  if (rs.nlarge) {
    ln.launch(k_long_cols<T, DIR>, rs.blk_large, kLongThreads, long_lds_bytes<T>(), large, rs.nlarge, in, tmp, tw);
    ln.launch(k_long_rows<T, DIR>, rs.blk_large, kLongThreads, long_lds_bytes<T>(), large, rs.nlarge,
              static_cast<const C2<T>*>(tmp), out, scale, tw);
  }
}

// Analysis: unitary DFT of x into X, X g_k wrapped modulo M_k into coef, the
// inverse DFTs of length M_k (unnormalised) in place.
template <class T, class Ln>
void full_analyze_launch(Ln& ln, const FullPlan& f, const char* tabs, const FullLayout& lay, const C2<T>* x,
                         C2<T>* coef, char* wk, const FullWork& w) {
  const auto* tw = reinterpret_cast<const C2<T>*>(tabs + lay.tw);
  auto* X = reinterpret_cast<C2<T>*>(wk + w.x_off);
  auto* tmp = reinterpret_cast<C2<T>*>(wk + w.t_off);
  long_fft<T, -1>(ln, tabs, lay.sig, x, X, tmp, (T)(1.0 / std::sqrt((double)f.L)), tw);
  ln.launch(k_full_gather<T>, (f.coef_count + 255) / 256, 256, 0, reinterpret_cast<const FullBandDev*>(tabs + lay.bands),
            (int)f.bands.size(), static_cast<const C2<T>*>(X), f.L, reinterpret_cast<const T*>(tabs + lay.g),
            f.coef_count, coef);
  long_fft<T, 1>(ln, tabs, lay.bandruns, static_cast<const C2<T>*>(coef), coef, tmp, T(1), tw);
}

// Synthesis: DFTs of length M_k (unnormalised) into C, the dual-weighted
// overlap-add into Z, the unitary inverse DFT into y.
template <class T, class Ln>
void full_synthesize_launch(Ln& ln, const FullPlan& f, const char* tabs, const FullLayout& lay,
                            const C2<T>* coef, C2<T>* y, char* wk, const FullWork& w) {
  const auto* tw = reinterpret_cast<const C2<T>*>(tabs + lay.tw);
  auto* C = reinterpret_cast<C2<T>*>(wk + w.c_off);
  auto* Z = reinterpret_cast<C2<T>*>(wk + w.x_off);
  auto* tmp = reinterpret_cast<C2<T>*>(wk + w.t_off);
  long_fft<T, -1>(ln, tabs, lay.bandruns, coef, C, tmp, T(1), tw);
  ln.launch(k_full_ola<T>, (f.L + 255) / 256, 256, 0, reinterpret_cast<const int32_t*>(tabs + lay.ent_off),
            reinterpret_cast<const int32_t*>(tabs + lay.ent_idx), reinterpret_cast<const T*>(tabs + lay.ent_w),
            static_cast<const C2<T>*>(C), f.L, Z);
  long_fft<T, 1>(ln, tabs, lay.sig, static_cast<const C2<T>*>(Z), y, tmp, (T)(1.0 / std::sqrt((double)f.L)), tw);
}

}  // namespace slicq
