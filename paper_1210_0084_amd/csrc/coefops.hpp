// Coefficient-domain kernels (elementwise, HBM-bound): the 2-layer view of
// Algorithm 3 and the sliCQ spectrogram (Section 4.3), dB masks and band
// transposition (Section 6), and the packing steps that build the transform
// of complex signals from two real ones.
//
// Layers: slice m's coefficients of band k sit in layer m mod 2 at positions
// (m - 1) M_k / 2 + n, n < M_k, circular modulo S M_k / 2 (Algorithm 3). A
// layer position p of band k is covered by exactly one slice of each layer:
// odd slice m = 2 (p div M_k) + 1 at n = p mod M_k, and even slice m = 2 (p'
// div M_k) at n = p' mod M_k with p' = (p + M_k / 2) mod (S M_k / 2).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"
#include "fft_device.hpp"

namespace slicq {

// Band of flat index i of a band-major array whose band k starts at R off_k
// (R = S for coefficients, S/2 for the layer grid): the largest k with
// off_k <= i div R.
__device__ __forceinline__ int band_of(const BandDev* __restrict__ bands, int nb, int64_t i, int R) {
  const int64_t key = i / R;
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (bands[mid].off <= key) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Coefficient n of slice m of band k in one signal's coefficients.
struct CoefAddr {
  int32_t slice_major, cps, S;
  __device__ __forceinline__ int64_t at(const BandDev& b, int m, int n) const {
    return slice_major ? (int64_t)m * cps + b.off + n : (int64_t)S * b.off + (int64_t)m * b.M + n;
  }
};

// Layer sum s^0 + s^1 (MODE 0, complex) or the sliCQ spectrogram |s^0 + s^1|^2
// (MODE 1, real) of every stored band; output band k at (S/2) off_k.
template <class T, int MODE>
__global__ void __launch_bounds__(256) k_layer_sum(const BandDev* __restrict__ bands, int64_t total,
                                                   int nb, CoefAddr ca, const C2<T>* __restrict__ coef,
                                                   void* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int k = band_of(bands, nb, i, ca.S / 2);
  const BandDev b = bands[k];
  const int p = (int)(i - (int64_t)(ca.S / 2) * b.off);
  const int half = b.M >> 1, nl = ca.S * half;
  int pe = p + half;
  if (pe >= nl) pe -= nl;
  const C2<T> s1 = coef[ca.at(b, 2 * (p / b.M) + 1, p % b.M)];
  const C2<T> s0 = coef[ca.at(b, 2 * (pe / b.M), pe % b.M)];
  const C2<T> s = cadd(s0, s1);
  if constexpr (MODE == 0) static_cast<C2<T>*>(out)[i] = s;
  else static_cast<T*>(out)[i] = s.x * s.x + s.y * s.y;
}

// dB mask on the layer grid (mask band k at (S/2) off_k, values in [0, 1]):
// each coefficient is scaled by 10^{5 (v - 1)} of its layer position (0 is
// -100 dB, 1 is 0 dB). In place; flat index i over the coefficients in
// band-major order.
template <class T>
__global__ void __launch_bounds__(256) k_mask_db(const BandDev* __restrict__ bands, int64_t total,
                                                 int nb, CoefAddr ca, const T* __restrict__ mask,
                                                 C2<T>* __restrict__ coef) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int k = band_of(bands, nb, i, ca.S);
  const BandDev b = bands[k];
  const int q = (int)(i - (int64_t)ca.S * b.off);
  const int m = q / b.M, n = q - m * b.M;
  const int half = b.M >> 1, nl = ca.S * half;
  int p = (m - 1) * half + n;
  if (p < 0) p += nl;
  else if (p >= nl) p -= nl;
  const T v = mask[(int64_t)(ca.S / 2) * b.off + p];
  T g;
  if constexpr (sizeof(T) == 4) g = exp10f(5.0f * (v - 1.0f));
  else g = exp10(5.0 * (v - 1.0));
  const int64_t a = ca.at(b, m, n);
  coef[a] = cscale(coef[a], g);
}

// Transposition by d bands: out band t (1 <= t <= K) takes in band t - d when
// 1 <= t - d <= K (equal M_k, checked on the host), else zero; the DC and
// Nyquist bands are zero. Flat index over the output's coefficients.
template <class T>
__global__ void __launch_bounds__(256) k_transpose(const BandDev* __restrict__ bands, int64_t total,
                                                   int nb, CoefAddr ca, int d, const C2<T>* __restrict__ in,
                                                   C2<T>* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int t = band_of(bands, nb, i, ca.S);
  const BandDev b = bands[t];
  const int q = (int)(i - (int64_t)ca.S * b.off);
  const int m = q / b.M, n = q - m * b.M;
  const int s = t - d, K = nb - 2;
  C2<T> v{T(0), T(0)};
  if (t >= 1 && t <= K && s >= 1 && s <= K) v = in[ca.at(bands[s], m, n)];
  out[ca.at(b, m, n)] = v;
}

// Complex signals from real transforms. Deinterleave: re[t], im[t] of x[t].
template <class T>
__global__ void __launch_bounds__(256) k_split_complex(const C2<T>* __restrict__ x, int64_t T_, T* __restrict__ re,
                                                       T* __restrict__ im) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T_) return;
  const C2<T> v = x[i];
  re[i] = v.x;
  im[i] = v.y;
}

template <class T>
__global__ void __launch_bounds__(256) k_join_complex(const T* __restrict__ re, const T* __restrict__ im, int64_t T_,
                                                      C2<T>* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T_) return;
  x[i] = {re[i], im[i]};
}

// Analysis of f = a + i b onto every band (band-major over bands 0..2K+1,
// mirror band 2K+2-k at off_all[...]): the transform is complex linear and a
// real signal's mirrored bands carry conjugate coefficients, so band k takes
// c_k(a) + i c_k(b) and its mirror conj c_k(a) + i conj c_k(b). coef holds
// c(a) in its stored part on entry (the same band-major layout) and the full
// result on exit; cb holds c(b). Flat index over the stored coefficients
// (band-major).
template <class T>
__global__ void __launch_bounds__(256) k_combine_complex(const BandDev* __restrict__ bands,
                                                         int64_t total, int nb, int S,
                                                         int64_t mirror_base, const C2<T>* __restrict__ cb,
                                                         C2<T>* __restrict__ coef) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int k = band_of(bands, nb, i, S);
  const C2<T> a = coef[i], b = cb[i];
  coef[i] = {a.x - b.y, a.y + b.x};                      // a + i b
  const int K = nb - 2;
  if (k >= 1 && k <= K) {
    // the mirrors follow the stored bands in the order K+2 .. 2K+1, i.e.
    // of sources K, K-1, ..., 1: the mirror of k sits after those of K .. k+1
    const int64_t mo = mirror_base + (int64_t)S * (bands[K + 1].off - bands[k + 1].off);
    coef[mo + (i - (int64_t)S * bands[k].off)] = {a.x + b.y, -a.y + b.x};   // conj a + i conj b
  }
}

// Synthesis of a complex signal from coefficients on every band: C = U + i V
// with U, V the Hermitian-symmetric sets U_k = (C_k + conj C_k')/2,
// V_k = (C_k - conj C_k')/(2i) (k' = 2K+2-k; for the self-mirrored DC and
// Nyquist bands U = Re C, V = Im C), so the synthesis is S_R(U) + i S_R(V)
// with S_R the real synthesis. Writes U and V over the stored bands.
template <class T>
__global__ void __launch_bounds__(256) k_hermitian_parts(const BandDev* __restrict__ bands,
                                                         int64_t total, int nb, int S,
                                                         int64_t mirror_base, const C2<T>* __restrict__ coef,
                                                         C2<T>* __restrict__ u, C2<T>* __restrict__ v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int k = band_of(bands, nb, i, S);
  const C2<T> c = coef[i];
  const int K = nb - 2;
  if (k >= 1 && k <= K) {
    const int64_t mo = mirror_base + (int64_t)S * (bands[K + 1].off - bands[k + 1].off);
    const C2<T> w = coef[mo + (i - (int64_t)S * bands[k].off)];   // C_k'
    // U = (c + conj w) / 2, V = (c - conj w) / (2i) = -i (c - conj w) / 2
    u[i] = {T(0.5) * (c.x + w.x), T(0.5) * (c.y - w.y)};
    v[i] = {T(0.5) * (c.y + w.y), T(-0.5) * (c.x - w.x)};
  } else {
    u[i] = {c.x, T(0)};
    v[i] = {c.y, T(0)};
  }
}

}  // namespace slicq

namespace slicq {

// Log-magnitude loss of the differentiable workload: with d = log(1 + |c|^2)
// - t (t the target's log-magnitudes), L = sum d^2 and its gradient with
// respect to c (real and imaginary parts: the convention of a real loss of a
// complex variable) dL/dc = 4 d c / (1 + |c|^2). One pass over c and t: every
// block of kLossThreads threads takes a fixed stride of elements and writes
// its partial sum (a tree in LDS, fixed order), k_loss_sum adds the partials
// in order, so the loss is the same on every run.
constexpr int kLossThreads = 256;

template <class T>
__global__ void __launch_bounds__(kLossThreads) k_logmag_loss(const C2<T>* __restrict__ c, const T* __restrict__ t,
                                                              int64_t n, C2<T>* __restrict__ grad,
                                                              T* __restrict__ partial) {
  __shared__ T red[kLossThreads];
  T acc = T(0);
  // four values per thread and round, all loads in flight before the arithmetic
  constexpr int U = 4;
  const int64_t stride = (int64_t)gridDim.x * kLossThreads;
  for (int64_t i0 = (int64_t)blockIdx.x * kLossThreads + threadIdx.x; i0 < n; i0 += U * stride) {
    C2<T> v[U];
    T tv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = imin64(i0 + u * stride, n - 1);
      v[u] = c[i];
      tv[u] = t[i];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + u * stride;
      if (i >= n) break;
      const T p = v[u].x * v[u].x + v[u].y * v[u].y;
      const T d = log1p(p) - tv[u];
      acc += d * d;
      const T s = T(4) * d / (T(1) + p);
      grad[i] = {s * v[u].x, s * v[u].y};
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kLossThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

template <class T>
__global__ void __launch_bounds__(kLossThreads) k_loss_sum(const T* __restrict__ partial, int nb, T* __restrict__ out) {
  __shared__ T red[kLossThreads];
  T acc = T(0);
  for (int i = threadIdx.x; i < nb; i += kLossThreads) acc += partial[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kLossThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

}  // namespace slicq
