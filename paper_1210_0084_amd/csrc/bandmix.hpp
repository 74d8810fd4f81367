// Band transforms for plans whose M_k are even smooth numbers M = R P with
// R in {1, 3, 5} and P = 2^logM (equation framecond1 only asks M_k >= |J_k|;
// Algorithm 3's layers need M_k even). A length-M DFT is R interleaved
// length-P DFTs and a radix-R combination:
//   F_M x [p + P q] = sum_r e^{s 2 pi i r q / R} e^{s 2 pi i r p / M} (F_P x[R t + r])[p]
// (s = -1 forward, +1 inverse; p < P, q < R). Values sit in LDS with the R
// subsequences of each band contiguous (position b M + r P + t holds
// x[R t + r] of band b), the power-of-two FFTs run over all of them at once,
// and the combination reads the R values of one p and writes the R outputs
// back to the same R positions in natural order. Twiddles of the combination
// come from a table per (R, P) (FP64-generated, rounded once); the
// power-of-two passes read the plan's twiddle pyramid (staging split tables
// in LDS measured no faster here).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"
#include "fft_device.hpp"
#include "kernels.hpp"

namespace slicq {

constexpr int kMixThreads = 1024;      // largest block; 8 values per thread, 16 for items above 8192 values

// x / R for R in {1, 3, 5} (division by a constant: a multiply and a shift).
__device__ __forceinline__ int div_r(int x, int R) {
  return R == 3 ? x / 3 : (R == 5 ? x / 5 : x);
}

// In-place DFT of R = 3 or 5 values, e^{DIR 2 pi i r q / R}, unnormalised.
template <class T, int DIR, int R>
__device__ __forceinline__ void dft_small(C2<T>* y) {
  static_assert(R == 3 || R == 5, "radix 3 or 5");
  if constexpr (R == 3) {
    const T c = T(-0.5), s = T(DIR) * T(0.86602540378443864676);     // e^{DIR 2 pi i / 3}
    const C2<T> a = cadd(y[1], y[2]), d = csub(y[1], y[2]);
    const C2<T> m{y[0].x + c * a.x, y[0].y + c * a.y};
    const C2<T> rot{-s * d.y, s * d.x};                                // i s d
    y[0] = cadd(y[0], a);
    y[1] = cadd(m, rot);
    y[2] = csub(m, rot);
  } else {
    const T c1 = T(0.30901699437494742410), c2 = T(-0.80901699437494742410);
    const T s1 = T(DIR) * T(0.95105651629515357212), s2 = T(DIR) * T(0.58778525229247312917);
    const C2<T> a1 = cadd(y[1], y[4]), d1 = csub(y[1], y[4]);
    const C2<T> a2 = cadd(y[2], y[3]), d2 = csub(y[2], y[3]);
    const C2<T> m1{y[0].x + c1 * a1.x + c2 * a2.x, y[0].y + c1 * a1.y + c2 * a2.y};
    const C2<T> m2{y[0].x + c2 * a1.x + c1 * a2.x, y[0].y + c2 * a1.y + c1 * a2.y};
    // i (s1 d1 + s2 d2) and i (s2 d1 - s1 d2)
    const C2<T> r1{-(s1 * d1.y + s2 * d2.y), s1 * d1.x + s2 * d2.x};
    const C2<T> r2{-(s2 * d1.y - s1 * d2.y), s2 * d1.x - s1 * d2.x};
    y[0] = cadd(y[0], cadd(a1, a2));
    y[1] = cadd(m1, r1);
    y[4] = csub(m1, r1);
    y[2] = cadd(m2, r2);
    y[3] = csub(m2, r2);
  }
}

// LDS position of value m (< M) of band b inside a group of bands of length M = R P.
__device__ __forceinline__ int mix_pos(int b, int m, int M, int R, int logP) {
  const int q = div_r(m, R);
  return b * M + ((m - q * R) << logP) + q;
}

// The radix-R combination of nseq bands of length M = R 2^logP at LDS base:
// for each p, the R values p + r P (subsequence DFTs) become the outputs
// p + q P, handed to out(b, n, value) (in place in LDS, or to global memory).
template <class T, int DIR, int R, class OUT>
__device__ __forceinline__ void mix_combine(const C2<T>* buf, int base, int nseq, int M, int logP,
                                            const C2<T>* __restrict__ twmix, int mixL, int tid, int nthr, OUT out) {
  const int P = 1 << logP, units = nseq << logP;
  const C2<T>* __restrict__ tw = twmix + mix_tw_base(R, logP, mixL);   // e^{-2 pi i k / M}
  for (int u = tid; u < units; u += nthr) {
    const int b = u >> logP, p = u & (P - 1);
    const int p0 = base + b * M + p;
    C2<T> y[R], w[R];
#pragma unroll
    for (int r = 1; r < R; ++r) w[r] = tw[r * p];
#pragma unroll
    for (int r = 0; r < R; ++r) y[r] = buf[pidx(p0 + r * P)];
#pragma unroll
    for (int r = 1; r < R; ++r) {
      if constexpr (DIR > 0) w[r].y = -w[r].y;
      y[r] = cmul(y[r], w[r]);
    }
    dft_small<T, DIR, R>(y);
#pragma unroll
    for (int q = 0; q < R; ++q) out(b, p + q * P, y[q]);
  }
}

// Power-of-two FFTs of every subsequence, then the radix-R combination
// (natural order) handed to out(b, n, value); for R = 1 the caller reads the
// result from LDS. nseq bands of length M at LDS base. Returns R; ends with
// a barrier when the combination wrote LDS.
template <class T, int DIR, int E, class TW, class OUT>
__device__ __forceinline__ int mix_fft(const KArgs<T>& a, C2<T>* buf, int base, int nseq, int M, int logP,
                                       const TW& tws, int tid, int nthr, OUT out) {
  const int R = M >> logP;
  lds_fft_contig<T, DIR, E, 8>(buf, base, logP, nseq * R, tws, tid, nthr);
  __syncthreads();
  if (R == 3) mix_combine<T, DIR, 3>(buf, base, nseq, M, logP, a.twmix, a.mixL, tid, nthr, out);
  else if (R == 5) mix_combine<T, DIR, 5>(buf, base, nseq, M, logP, a.twmix, a.mixL, tid, nthr, out);
  return R;
}

// Values handled per batch of a loop over a work item: addresses first, then
// every load of the batch in flight, then the uses.
constexpr int kMixBatch = 8;

// Band analysis of a group of equal-M bands of one slice (the work items and
// grid of k_band_ana): gather X g_k wrapped modulo M (bins outside [0, N]
// through conjugate symmetry) into the subsequence layout, inverse DFT of
// length M, coefficient stores (from the combination directly when R > 1).
template <class T, int E>
__global__ void __launch_bounds__(kMixThreads) k_band_ana_mx(KArgs<T> a, const SliceTask* __restrict__ tasks,
                                                             const C2<T>* __restrict__ W2, C2<T>* __restrict__ coef,
                                                             int g0, int ng) {
  extern __shared__ unsigned char smem[];
  C2<T>* buf = reinterpret_cast<C2<T>*>(smem);
  const int task = blockIdx.x / ng, gi = g0 + (int)blockIdx.x - task * ng;
  const AnaGroupDev G = a.ana[gi];
  const SliceTask tk = tasks[task];
  if (tk.S == 0) return;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int M = G.M, logP = G.logM, R = M >> logP, total = G.cnt * M;
  const C2<T>* __restrict__ X = W2 + (int64_t)task * a.ws2;
#pragma unroll
  for (int e0 = 0; e0 < E; e0 += kMixBatch) {
    int xi[kMixBatch], wi[kMixBatch], pos[kMixBatch];
#pragma unroll
    for (int e = 0; e < kMixBatch; ++e) {
      const int i = tid + (e0 + e) * nthr;
      const int ic = imin(i, total - 1);
      const int b = div_r(ic >> logP, R), m = ic - b * M;
      const BandDev B = a.bands[G.k0 + b];
      int t = m + a.bsmod[G.k0 + b];             // (m - start) mod M
      if (t >= M) t -= M;
      const bool in = i < total && t < B.len;
      const int jb = B.start + t;                 // signed bin, -N < jb < 2N
      const int jj = jb < 0 ? -jb : (jb > a.N ? 2 * a.N - jb : jb);
      xi[e] = in ? ((jb < 0 || jb > a.N) ? ~jj : jj) : 0;   // ~jj (< 0) marks a conjugate
      wi[e] = in ? B.goff + t : -1;
      pos[e] = i < total ? mix_pos(b, m, M, R, logP) : -1;
    }
    C2<T> v[kMixBatch];
    T w[kMixBatch];
#pragma unroll
    for (int e = 0; e < kMixBatch; ++e) {
      v[e] = X[xi[e] < 0 ? ~xi[e] : xi[e]];
      w[e] = a.g[imax(wi[e], 0)];
    }
#pragma unroll
    for (int e = 0; e < kMixBatch; ++e) {
      if (pos[e] < 0) continue;
      const T g = wi[e] < 0 ? T(0) : w[e];
      buf[pidx(pos[e])] = {v[e].x * g, (xi[e] < 0 ? -v[e].y : v[e].y) * g};
    }
  }
  __syncthreads();
  C2<T>* __restrict__ cs = coef + tk.coef_base;
  const int off0 = a.bands[G.k0].off;
  const int cbase = a.slice_major ? tk.m * a.cps + off0 : tk.S * off0 + tk.m * M;
  const int bstride = a.slice_major ? M : tk.S * M;
  auto store = [&](int b, int n, C2<T> v) { cs[cbase + b * bstride + n] = v; };
  if (mix_fft<T, 1, E>(a, buf, 0, G.cnt, M, logP, TwGlobal<T>{a.tw}, tid, nthr, store) == 1) {
    for (int i = tid; i < total; i += nthr) {
      const int b = i >> logP, n = i - (b << logP);
      store(b, n, buf[pidx(i)]);
    }
  }
}

// Band synthesis of the owned bins [lo, hi) of one slice (the work items,
// runs and grid of k_band_syn): coefficient loads into the subsequence
// layout, DFTs of length M per run (natural order back in LDS), then each
// owned bin's overlap-add program (LDS positions from the plan).
template <class T, int E>
__global__ void __launch_bounds__(kMixThreads) k_band_syn_mx(KArgs<T> a, const SliceTask* __restrict__ tasks,
                                                             const C2<T>* __restrict__ coef, C2<T>* __restrict__ W2,
                                                             T* __restrict__ y, int g0, int ntask) {
  extern __shared__ unsigned char smem[];
  C2<T>* buf = reinterpret_cast<C2<T>*>(smem);
  const int task = (int)(blockIdx.z * gridDim.x + blockIdx.x), gi = g0 + (int)blockIdx.y;
  if (task >= ntask) return;
  const SynGroupDev G = a.syn[gi];
  const SliceTask tk = tasks[task];
  if (tk.S == 0) return;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const C2<T>* __restrict__ cs = coef + tk.coef_base;
  // all runs' loads as one flat range of G.total values (runs are contiguous in LDS)
#pragma unroll
  for (int e0 = 0; e0 < E; e0 += kMixBatch) {
    int src[kMixBatch], dst[kMixBatch];
#pragma unroll
    for (int e = 0; e < kMixBatch; ++e) {
      const int i = tid + (e0 + e) * nthr;
      const int ic = imin(i, G.total - 1);
      SynRunDev Rn = G.r[0];
      if (G.nrun > 1 && ic >= G.r[1].lds_off) Rn = G.r[1];
      for (int ri = 2; ri < G.nrun; ++ri) {
        const SynRunDev Q = a.runs[G.run0 + ri];
        if (ic >= Q.lds_off) Rn = Q;
      }
      const int M = Rn.M, logP = Rn.logM, R = M >> logP;
      const int q = ic - Rn.lds_off;
      const int b = div_r(q >> logP, R), n = q - b * M;
      src[e] = a.slice_major ? tk.m * a.cps + Rn.off + b * M + n : tk.S * (Rn.off + b * M) + tk.m * M + n;
      dst[e] = i < G.total ? Rn.lds_off + mix_pos(b, n, M, R, logP) : -1;
    }
    C2<T> v[kMixBatch];
#pragma unroll
    for (int e = 0; e < kMixBatch; ++e) v[e] = cs[src[e]];
#pragma unroll
    for (int e = 0; e < kMixBatch; ++e)
      if (dst[e] >= 0) buf[pidx(dst[e])] = v[e];
  }
  __syncthreads();
  for (int ri = 0; ri < G.nrun; ++ri) {
    SynRunDev Rn;
    if (ri == 0) Rn = G.r[0];
    else if (ri == 1) Rn = G.r[1];
    else Rn = a.runs[G.run0 + ri];
    int t = tid;
    asm volatile("" : "+v"(t));      // keeps each FFT length's address arithmetic inside the loop (registers)
    auto back = [&](int b, int n, C2<T> v) { buf[pidx(Rn.lds_off + b * Rn.M + n)] = v; };
    if (mix_fft<T, -1, E>(a, buf, Rn.lds_off, Rn.cnt, Rn.M, Rn.logM, TwGlobal<T>{a.tw}, t, nthr, back) > 1)
      __syncthreads();
  }
  C2<T>* Z = W2 + (int64_t)task * a.ws2;
  for (int j = G.lo + tid; j < G.hi; j += nthr) {
    const OlaRec<T> rec = a.ola2[j];
    const uint32_t y0 = rec.yy & kOlaNone, y1 = rec.yy >> 16;
    C2<T> c0 = buf[pidx(rec.xx & kOlaPosMask)], c1 = buf[pidx(rec.xx >> 16)];
    if (y0 != kOlaNone) c0 = cadd(c0, cconj(buf[pidx(y0)]));
    if (y1 != kOlaNone) c1 = cadd(c1, cconj(buf[pidx(y1)]));
    C2<T> acc = cadd(cscale(c0, rec.w0), cscale(c1, rec.w1));
    if (rec.xx & kOlaMore) {
      for (int e = a.ent_off[j]; e < a.ent_off[j + 1]; ++e) {
        const int2 pe = a.ent_pos[e];
        C2<T> c = buf[pidx(pe.x)];
        if (pe.y >= 0) c = cadd(c, cconj(buf[pidx(pe.y)]));
        acc = cadd(acc, cscale(c, a.ent_w[e]));
      }
    }
    Z[j] = acc;
  }
  (void)y;
}

}  // namespace slicq
