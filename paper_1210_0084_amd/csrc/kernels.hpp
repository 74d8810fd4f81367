// HIP kernels of the sliCQ hot path for gfx950 (wave64, LDS, HBM-bound).
//
// Analysis of one slice m (Algorithm 3 with Algorithm 1 at length 2N):
//   fwd_pass1, fwd_pass2  window the slice (h_0), pack the 2N real samples as
//                         N complex values and take their N-point FFT in two
//                         passes (N = N1 N2, four-step), then split it into the
//                         unitary real spectrum X[0..N] of the slice;
//   band_ana              per group of bands of equal M_k: wrap X g_k at
//                         j mod M_k, inverse DFT of length M_k, store c^m_k.
// Synthesis (Algorithm 4 with Algorithm 2):
//   band_syn              per group of owned bins: DFT_{M_k} of every band that
//                         reaches them, multiply by the dual window, add (the
//                         frequency overlap-add), giving the half spectrum Z;
//   inv_passA, inv_passB  real inverse DFT of length 2N from Z[0..N] by the
//                         same four-step factorisation, multiply by h~_0 and
//                         overlap-add into the output.
// The adjoint of analysis uses the synthesis kernels with g_k and h_0.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"
#include "fft_device.hpp"

namespace slicq {

// Largest block each kernel is compiled for (its __launch_bounds__).
constexpr int kPassThreads = 256;     // k_fwd_pass1/2, k_inv_passA/B
constexpr int kAnaThreads = 256;      // k_band_ana
constexpr int kSynThreads = 512;      // k_band_syn

template <class T>
struct KArgs {
  const C2<T>* tw;        // twiddle pyramid
  const T* h0;            // analysis slice window (2N)
  const T* hsyn;          // synthesis slice window: h~_0 (synthesis) or h_0 (adjoint)
  const T* g;             // analysis band windows
  const T* gsyn;          // synthesis band windows: g~_k (synthesis) or g_k (adjoint)
  const BandDev* bands;
  const AnaGroupDev* ana;
  const SynGroupDev* syn;
  const SynRunDev* runs;
  const int32_t* bin_k0;
  const int32_t* bin_nk;
  int32_t N, Mt, K, n_ana;
  int32_t n_syn, N1, N2, logN1;
  int32_t logN2, C, logC, P;
  int32_t logP, zero_ola;   // zero_ola: band_syn zeroes the output overlaps
  int64_t ws1, ws2;       // complex values per slice in the two workspace regions
  T scale;                // (2N)^{-1/2}
  T inner_w;              // weight of bands 1..K in the frequency overlap-add
};

template <class T>
__device__ __forceinline__ T load_sample(const T* __restrict__ x, const SliceTask& tk, int64_t j) {
  int64_t idx = tk.x_start + j;
  if (idx >= tk.x_period) idx -= tk.x_period;
  return idx < tk.x_valid ? x[tk.x_base + idx] : T(0);
}

// ---------------------------------------------------------------------------
// Forward FFT of a slice, pass 1: columns. The N complex values
// z[n] = x_m[2n] + i x_m[2n+1] are indexed n = n1 + N1 n2; this item takes the
// C columns n1 in [cb C, cb C + C), transforms each over n2 (length N2),
// applies e^{-2 pi i n1 k2 / N} and stores W1[k2 N1 + n1].
template <class T>
__global__ void __launch_bounds__(256) k_fwd_pass1(KArgs<T> a, const SliceTask* __restrict__ tasks,
                                                    const T* __restrict__ x, C2<T>* __restrict__ W1) {
  extern __shared__ unsigned char smem[];
  C2<T>* buf = reinterpret_cast<C2<T>*>(smem);
  const int nCB = a.N1 >> a.logC;
  const int task = blockIdx.x / nCB, cb = blockIdx.x - task * nCB;
  const SliceTask tk = tasks[task];
  if (tk.S == 0) return;                              // unused task slot
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int total = a.C * a.N2;
  const int jlo = (a.N - a.Mt) / 2 + 1;              // first non-zero sample of h_0
  const int jhi = a.N + (a.N + a.Mt) / 2 - 1;        // last non-zero sample of h_0
  for (int e = tid; e < total; e += nthr) {
    const int c = e & (a.C - 1), n2 = e >> a.logC;
    const int n = cb * a.C + c + a.N1 * n2;
    const int j = 2 * n;
    T re = 0, im = 0;
    if (j + 1 >= jlo && j <= jhi) {
      re = load_sample(x, tk, j) * a.h0[j];
      im = load_sample(x, tk, j + 1) * a.h0[j + 1];
    }
    buf[pidx(e)] = {re, im};
  }
  __syncthreads();
  lds_fft<T, -1, INTERLEAVED>(buf, 0, a.logN2, a.C, a.logC, a.tw, tid, nthr);
  C2<T>* out = W1 + (int64_t)task * a.ws1;
  for (int e = tid; e < total; e += nthr) {
    const int c = e & (a.C - 1), k2 = e >> a.logC;
    const int n1 = cb * a.C + c;
    C2<T> v = cmul(buf[pidx(e)], twiddle<T, -1>(a.tw, a.N, (n1 * k2) & (a.N - 1)));
    out[(int64_t)k2 * a.N1 + n1] = v;
  }
}

// Rows handled by a pass-2 item rb: sequence s < P is the row rb P + s,
// sequence P + i is its mirror N2 - (rb P + i), except that the mirror of
// row 0 is taken to be row N2/2 (rows 0 and N2/2 are their own mirrors).
__device__ __forceinline__ int pass2_row(int rb, int s, int P, int N2) {
  if (s < P) return rb * P + s;
  const int i = s - P;
  if (rb == 0 && i == 0) return N2 / 2;
  return N2 - (rb * P + i);
}

// The unitary real spectrum from the packed FFT: with a = Zc[k], b = Zc[N-k],
// E = (a + conj b)/2, O = -i (a - conj b)/2: X[k] = E + w^k O and
// X[N-k] = conj(E - w^k O), w = e^{-2 pi i / 2N}.
template <class T>
__device__ __forceinline__ void real_split(C2<T> za, C2<T> zb, C2<T> w, T s, C2<T>& xk, C2<T>& xnk) {
  const C2<T> zbc = cconj(zb);
  const C2<T> E = cscale(cadd(za, zbc), T(0.5));
  const C2<T> O = mul_mi<T, -1>(cscale(csub(za, zbc), T(0.5)));
  const C2<T> wo = cmul(w, O);
  xk = cscale(cadd(E, wo), s);
  xnk = cscale(cconj(csub(E, wo)), s);
}

// Forward pass 2: rows. Each item takes P row pairs, transforms them over n1
// (length N1), giving Zc[N2 k1 + k2], and splits pairs (k, N - k) into the
// real spectrum X[0..N] of the slice (W2).
template <class T>
__global__ void __launch_bounds__(256) k_fwd_pass2(KArgs<T> a, const C2<T>* __restrict__ W1,
                                                    C2<T>* __restrict__ W2) {
  extern __shared__ unsigned char smem[];
  C2<T>* buf = reinterpret_cast<C2<T>*>(smem);
  const int nRB = (a.N2 / 2) >> a.logP;
  const int task = blockIdx.x / nRB, rb = blockIdx.x - task * nRB;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int P = a.P, twoP = 2 * a.P, logTwoP = a.logP + 1;
  const C2<T>* in = W1 + (int64_t)task * a.ws1;
  for (int e = tid; e < twoP * a.N1; e += nthr) {
    const int s = e >> a.logN1, n1 = e & (a.N1 - 1);
    const int row = pass2_row(rb, s, P, a.N2);
    buf[pidx((n1 << logTwoP) + s)] = in[(int64_t)row * a.N1 + n1];
  }
  __syncthreads();
  lds_fft<T, -1, INTERLEAVED>(buf, 0, a.logN1, twoP, logTwoP, a.tw, tid, nthr);
  C2<T>* X = W2 + (int64_t)task * a.ws2;
  const int N = a.N, N1 = a.N1, N2 = a.N2;
  for (int t = tid; t < P * N1; t += nthr) {
    const int i = t & (P - 1), k1 = t >> a.logP;
    const int row = rb * P + i;
    C2<T> xk, xnk;
    if (row != 0) {
      const int k = N2 * k1 + row;
      const C2<T> za = buf[pidx((k1 << logTwoP) + i)];
      const C2<T> zb = buf[pidx(((N1 - 1 - k1) << logTwoP) + P + i)];
      real_split(za, zb, twiddle<T, -1>(a.tw, 2 * N, k), a.scale, xk, xnk);
      X[k] = xk;
      X[N - k] = xnk;
    } else if (k1 < N1 / 2) {
      // row 0: pairs (k1, N1 - k1); k1 = 0 gives X[0], X[N] and also X[N/2]
      const int k = N2 * k1;
      const C2<T> za = buf[pidx((k1 << logTwoP))];
      const C2<T> zb = buf[pidx((((N1 - k1) & (N1 - 1)) << logTwoP))];
      real_split(za, zb, twiddle<T, -1>(a.tw, 2 * N, k), a.scale, xk, xnk);
      X[k] = xk;
      X[N - k] = xnk;
      if (k1 == 0) {
        const C2<T> zh = buf[pidx(((N1 / 2) << logTwoP))];
        real_split(zh, zh, twiddle<T, -1>(a.tw, 2 * N, N / 2), a.scale, xk, xnk);
        X[N / 2] = xk;
      }
    } else {
      // row N2/2 (sequence P): pairs (kk, N1 - 1 - kk)
      const int kk = k1 - N1 / 2;
      const int k = N2 * kk + N2 / 2;
      const C2<T> za = buf[pidx((kk << logTwoP) + P)];
      const C2<T> zb = buf[pidx(((N1 - 1 - kk) << logTwoP) + P)];
      real_split(za, zb, twiddle<T, -1>(a.tw, 2 * N, k), a.scale, xk, xnk);
      X[k] = xk;
      X[N - k] = xnk;
    }
  }
}

// Value of the full slice spectrum at signed bin j from the half spectrum.
template <class T>
__device__ __forceinline__ C2<T> spec_at(const C2<T>* __restrict__ X, int j, int N) {
  if (j < 0) return cconj(X[-j]);
  if (j > N) return cconj(X[2 * N - j]);
  return X[j];
}

// Band analysis: bands k0 .. k0 + cnt - 1 of one slice. Slot r of band k
// holds X[j] g_k[j] for the bin j of J_k with j = r (mod M_k), or 0; the
// inverse DFT of length M_k gives c^m_{n,k} (equation CQ_coeff).
template <class T, int E>
__global__ void __launch_bounds__(256) k_band_ana(KArgs<T> a, const SliceTask* __restrict__ tasks,
                                                   const C2<T>* __restrict__ W2, C2<T>* __restrict__ coef) {
  extern __shared__ unsigned char smem[];
  C2<T>* buf = reinterpret_cast<C2<T>*>(smem);
  const int task = blockIdx.x / a.n_ana, gi = blockIdx.x - task * a.n_ana;
  const AnaGroupDev G = a.ana[gi];
  const SliceTask tk = tasks[task];
  if (tk.S == 0) return;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const C2<T>* X = W2 + (int64_t)task * a.ws2;
  const int total = G.cnt << G.logM, mask = G.M - 1;
  for (int e = tid; e < total; e += nthr) {
    const int k = G.k0 + (e >> G.logM), r = e & mask;
    const BandDev B = a.bands[k];
    const int t = (r - B.start) & mask;
    C2<T> v = {0, 0};
    if (t < B.len) v = cscale(spec_at(X, B.start + t, a.N), a.g[B.goff + t]);
    buf[pidx(e)] = v;
  }
  __syncthreads();
  lds_fft<T, 1, CONTIG, E>(buf, 0, G.logM, G.cnt, 0, a.tw, tid, nthr);
  const int64_t S = tk.S;
  for (int e = tid; e < total; e += nthr) {
    const int k = G.k0 + (e >> G.logM), n = e & mask;
    const int64_t dst = tk.coef_base + S * a.bands[k].off + (int64_t)tk.m * G.M + n;
    coef[dst] = buf[pidx(e)];
  }
}

// Band synthesis: owned bins [lo, hi) of the half spectrum of one slice.
// Every band ke..kb is transformed (DFT_{M_k}), then each owned bin j sums
// w_k[j] C_k[j mod M_k] over the bands covering it, in increasing k: weight
// inner_w for bands 1..K and, for the self-mirrored DC and Nyquist bands,
// (w[j]/2)(C[j mod M] + conj C[-j mod M]) (real part of the full synthesis).
template <class T, int E>
__global__ void __launch_bounds__(512) k_band_syn(KArgs<T> a, const SliceTask* __restrict__ tasks,
                                                   const C2<T>* __restrict__ coef, C2<T>* __restrict__ W2,
                                                   T* __restrict__ y) {
  extern __shared__ unsigned char smem[];
  C2<T>* buf = reinterpret_cast<C2<T>*>(smem);
  const int task = blockIdx.x / a.n_syn, gi = blockIdx.x - task * a.n_syn;
  const SynGroupDev G = a.syn[gi];
  const SliceTask tk = tasks[task];
  if (tk.S == 0) return;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int64_t S = tk.S;
  const int base_off = a.bands[G.ke].off;
  for (int ri = 0; ri < G.nrun; ++ri) {
    const SynRunDev R = a.runs[G.run0 + ri];
    const int tot = R.cnt << R.logM;
    for (int e = tid; e < tot; e += nthr) {
      const int k = R.k0 + (e >> R.logM), n = e & (R.M - 1);
      const int64_t src = tk.coef_base + S * a.bands[k].off + (int64_t)tk.m * R.M + n;
      buf[pidx(R.lds_off + e)] = coef[src];
    }
  }
  if (gi == 0 && a.zero_ola && (tk.flags & 1)) {
    // zero the right-hand overlap of this slice in the output, which the
    // inverse pass then accumulates into from this slice and the next
    const int j0 = a.N + (a.N - a.Mt) / 2 + 1, j1 = a.N + (a.N + a.Mt) / 2;
    for (int j = j0 + tid; j < j1; j += nthr) {
      int64_t idx = tk.y_start + j;
      if (idx >= tk.y_period) idx -= tk.y_period;
      if (idx < tk.y_valid) y[tk.y_base + idx] = T(0);
    }
  }
  __syncthreads();
  for (int ri = 0; ri < G.nrun; ++ri) {
    const SynRunDev R = a.runs[G.run0 + ri];
    lds_fft<T, -1, CONTIG, E>(buf, R.lds_off, R.logM, R.cnt, 0, a.tw, tid, nthr);
  }
  C2<T>* Z = W2 + (int64_t)task * a.ws2;
  const int K1 = a.K + 1;
  for (int j = G.lo + tid; j < G.hi; j += nthr) {
    const int k0 = a.bin_k0[j], nk = a.bin_nk[j];
    C2<T> acc = {0, 0};
    for (int k = k0; k < k0 + nk; ++k) {
      const BandDev B = a.bands[k];
      const int lpos = B.off - base_off;
      const T w = a.gsyn[B.goff + (j - B.start)];
      const C2<T> c1 = buf[pidx(lpos + (j & (B.M - 1)))];
      if (k == 0 || k == K1) {
        const C2<T> c2 = buf[pidx(lpos + ((-j) & (B.M - 1)))];
        acc = cadd(acc, cscale(cadd(c1, cconj(c2)), T(0.5) * w));
      } else {
        acc = cadd(acc, cscale(c1, a.inner_w * w));
      }
    }
    Z[j] = acc;
  }
}

// Inverse pass A: rows. From the Hermitian half spectrum Z[0..N] form the
// packed spectrum Zc[k] = (Z[k] + conj Z[N-k]) + i e^{+2 pi i k/2N}(Z[k] - conj Z[N-k])
// of z[n] = y[2n] + i y[2n+1], transform over k1 (length N1, e^+), apply
// e^{+2 pi i n1 k2 / N} and store W1[k2 N1 + n1].
template <class T>
__device__ __forceinline__ void herm_pack(C2<T> a, C2<T> b, C2<T> u, C2<T>& zk, C2<T>& znk) {
  const C2<T> bc = cconj(b);
  const C2<T> Pp = cadd(a, bc);
  const C2<T> Q = cmul(u, csub(a, bc));
  zk = cadd(Pp, mul_mi<T, 1>(Q));                 // P + iQ
  znk = cconj(csub(Pp, mul_mi<T, 1>(Q)));         // conj(P - iQ)
}

template <class T>
__global__ void __launch_bounds__(256) k_inv_passA(KArgs<T> a, const C2<T>* __restrict__ W2,
                                                    C2<T>* __restrict__ W1) {
  extern __shared__ unsigned char smem[];
  C2<T>* buf = reinterpret_cast<C2<T>*>(smem);
  const int nRB = (a.N2 / 2) >> a.logP;
  const int task = blockIdx.x / nRB, rb = blockIdx.x - task * nRB;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int P = a.P, twoP = 2 * a.P, logTwoP = a.logP + 1;
  const int N = a.N, N1 = a.N1, N2 = a.N2;
  const C2<T>* Z = W2 + (int64_t)task * a.ws2;
  for (int t = tid; t < P * N1; t += nthr) {
    const int i = t & (P - 1), k1 = t >> a.logP;
    const int row = rb * P + i;
    C2<T> zk, znk;
    if (row != 0) {
      const int k = N2 * k1 + row;
      herm_pack(Z[k], Z[N - k], twiddle<T, 1>(a.tw, 2 * N, k), zk, znk);
      buf[pidx((k1 << logTwoP) + i)] = zk;
      buf[pidx(((N1 - 1 - k1) << logTwoP) + P + i)] = znk;
    } else if (k1 < N1 / 2) {
      const int k = N2 * k1;
      herm_pack(Z[k], Z[N - k], twiddle<T, 1>(a.tw, 2 * N, k), zk, znk);
      buf[pidx(k1 << logTwoP)] = zk;
      if (k1 != 0) buf[pidx(((N1 - k1) & (N1 - 1)) << logTwoP)] = znk;
      if (k1 == 0) {
        herm_pack(Z[N / 2], Z[N / 2], twiddle<T, 1>(a.tw, 2 * N, N / 2), zk, znk);
        buf[pidx((N1 / 2) << logTwoP)] = zk;
      }
    } else {
      const int kk = k1 - N1 / 2;
      const int k = N2 * kk + N2 / 2;
      herm_pack(Z[k], Z[N - k], twiddle<T, 1>(a.tw, 2 * N, k), zk, znk);
      buf[pidx((kk << logTwoP) + P)] = zk;
      buf[pidx(((N1 - 1 - kk) << logTwoP) + P)] = znk;
    }
  }
  __syncthreads();
  lds_fft<T, 1, INTERLEAVED>(buf, 0, a.logN1, twoP, logTwoP, a.tw, tid, nthr);
  C2<T>* out = W1 + (int64_t)task * a.ws1;
  for (int e = tid; e < twoP * N1; e += nthr) {
    const int s = e >> a.logN1, n1 = e & (N1 - 1);
    const int row = pass2_row(rb, s, P, N2);
    const C2<T> v = cmul(buf[pidx((n1 << logTwoP) + s)], twiddle<T, 1>(a.tw, N, (n1 * row) & (N - 1)));
    out[(int64_t)row * N1 + n1] = v;
  }
}

// Adds v at window position j of the slice into the output: plain stores where
// only this slice contributes, atomic adds on the M-1 samples shared with a
// neighbour (exactly two contributions into a zeroed sample: order-free).
template <class T>
__device__ __forceinline__ void ola_store(T* __restrict__ y, const SliceTask& tk, int j, T v, int N, int Mt) {
  int dj = j - N;
  if (dj < 0) dj = -dj;
  if (2 * dj >= N + Mt) return;
  int64_t idx = tk.y_start + j;
  if (idx >= tk.y_period) idx -= tk.y_period;
  if (idx >= tk.y_valid) return;
  T* p = y + tk.y_base + idx;
  if (2 * dj <= N - Mt) *p = v;
  else unsafeAtomicAdd(p, v);
}

// Inverse pass B: columns n1 in [cb C, cb C + C): transform over k2 (length
// N2, e^+), giving z[n1 + N1 n2] = y[2n] + i y[2n+1]; scale, multiply by the
// synthesis slice window and overlap-add (Algorithm 4).
template <class T>
__global__ void __launch_bounds__(256) k_inv_passB(KArgs<T> a, const SliceTask* __restrict__ tasks,
                                                    const C2<T>* __restrict__ W1, T* __restrict__ y) {
  extern __shared__ unsigned char smem[];
  C2<T>* buf = reinterpret_cast<C2<T>*>(smem);
  const int nCB = a.N1 >> a.logC;
  const int task = blockIdx.x / nCB, cb = blockIdx.x - task * nCB;
  const SliceTask tk = tasks[task];
  if (tk.S == 0) return;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int total = a.C * a.N2;
  const C2<T>* in = W1 + (int64_t)task * a.ws1;
  for (int e = tid; e < total; e += nthr) {
    const int c = e & (a.C - 1), k2 = e >> a.logC;
    buf[pidx(e)] = in[(int64_t)k2 * a.N1 + cb * a.C + c];
  }
  __syncthreads();
  lds_fft<T, 1, INTERLEAVED>(buf, 0, a.logN2, a.C, a.logC, a.tw, tid, nthr);
  for (int e = tid; e < total; e += nthr) {
    const int c = e & (a.C - 1), n2 = e >> a.logC;
    const int n = cb * a.C + c + a.N1 * n2;
    const C2<T> v = buf[pidx(e)];
    const int j = 2 * n;
    ola_store(y, tk, j, v.x * a.scale * a.hsyn[j], a.N, a.Mt);
    ola_store(y, tk, j + 1, v.y * a.scale * a.hsyn[j + 1], a.N, a.Mt);
  }
}

// Zeroes the right-hand output overlap of every task (used when slices are
// processed in several chunks, so that no chunk clears a sample that an
// earlier chunk has already accumulated into).
template <class T>
__global__ void __launch_bounds__(256) k_zero_overlaps(const SliceTask* __restrict__ tasks, int64_t ntasks,
                                                       int32_t N, int32_t Mt, T* __restrict__ y) {
  const int64_t per = (Mt - 1 + 255) / 256;
  const int64_t task = blockIdx.x / per;
  if (task >= ntasks) return;
  const SliceTask tk = tasks[task];
  if (tk.S == 0 || !(tk.flags & 1)) return;
  const int j = N + (N - Mt) / 2 + 1 + (int)(blockIdx.x - task * per) * 256 + threadIdx.x;
  if (j >= N + (N + Mt) / 2) return;
  int64_t idx = tk.y_start + j;
  if (idx >= tk.y_period) idx -= tk.y_period;
  if (idx < tk.y_valid) y[tk.y_base + idx] = T(0);
}

// Slices of one signal of T samples (L = 2N ceil(T/2N), S = L/N), m0.. m0+count-1.
__global__ void __launch_bounds__(256) k_tasks_plain(SliceTask* __restrict__ tasks, int64_t m0,
                                                     int64_t count, int64_t T, int64_t N, int64_t S) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int64_t m = m0 + i;
  const int64_t L = S * N;
  SliceTask t;
  t.x_base = 0;
  t.x_start = ((m - 1) * N + L) % L;
  t.x_period = L;
  t.x_valid = T;
  t.y_base = 0;
  t.y_start = t.x_start;
  t.y_period = L;
  t.y_valid = T;
  t.coef_base = 0;
  t.m = (int32_t)m;
  t.S = (int32_t)S;
  t.flags = 1;
  t.pad_ = 0;
  t.pad2_ = 0;
  tasks[i] = t;
}

// Slices of a ragged batch: signal b holds samples x_off[b] .. x_off[b+1]-1
// and its coefficients start at coef_off[b]. One block of 1024 threads first
// marks every task slot unused, then scans the slice counts
// S_b = 2 ceil(T_b / 2N) and writes the tasks of every signal in order.
// Signals whose samples or coefficients fall outside the buffers are skipped
// and flagged in status[0]; status[1] receives the number of slices.
__global__ void __launch_bounds__(1024) k_tasks_batched(SliceTask* __restrict__ tasks,
                                                        const int64_t* __restrict__ x_off,
                                                        const int64_t* __restrict__ coef_off,
                                                        int32_t nsig, int64_t N, int64_t max_tasks,
                                                        int64_t x_len, int64_t coef_len,
                                                        int64_t coefs_per_slice,
                                                        int32_t* __restrict__ status) {
  extern __shared__ unsigned char smem[];        // 1024 + 2 int64 words
  int64_t* scan = reinterpret_cast<int64_t*>(smem);
  int64_t& carry = scan[1024];
  int32_t& bad = *reinterpret_cast<int32_t*>(&scan[1025]);
  const int tid = threadIdx.x;
  for (int64_t i = tid; i < max_tasks; i += 1024) {
    SliceTask t{};
    tasks[i] = t;
  }
  if (tid == 0) {
    carry = 0;
    bad = 0;
  }
  __syncthreads();
  for (int32_t b0 = 0; b0 < nsig; b0 += 1024) {
    const int32_t b = b0 + tid;
    int64_t Tb = 0, Sb = 0;
    if (b < nsig) {
      Tb = x_off[b + 1] - x_off[b];
      if (Tb < 0) Tb = 0;
      Sb = 2 * ((Tb + 2 * N - 1) / (2 * N));
    }
    scan[tid] = Sb;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
      const int64_t v = tid >= d ? scan[tid - d] : 0;
      __syncthreads();
      scan[tid] += v;
      __syncthreads();
    }
    const int64_t first = carry + scan[tid] - Sb;
    if (b < nsig && Sb > 0) {
      const bool ok = x_off[b] >= 0 && x_off[b] + Tb <= x_len && coef_off[b] >= 0 &&
                      coef_off[b] + Sb * coefs_per_slice <= coef_len && first + Sb <= max_tasks;
      if (!ok) {
        bad = 1;
      } else {
        const int64_t L = Sb * N;
        for (int64_t m = 0; m < Sb; ++m) {
          SliceTask t{};
          t.x_base = x_off[b];
          t.x_start = ((m - 1) * N + L) % L;
          t.x_period = L;
          t.x_valid = Tb;
          t.y_base = x_off[b];
          t.y_start = t.x_start;
          t.y_period = L;
          t.y_valid = Tb;
          t.coef_base = coef_off[b];
          t.m = (int32_t)m;
          t.S = (int32_t)Sb;
          t.flags = 1;
          tasks[first + m] = t;
        }
      }
    }
    __syncthreads();
    if (tid == 1023) carry += scan[1023];
    __syncthreads();
  }
  if (tid == 0) {
    status[0] = bad;
    status[1] = (int32_t)(carry > 0x7fffffff ? 0x7fffffff : carry);
  }
}

}  // namespace slicq
