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
//
// Every thread owns at most E values of a work item. Global loads are issued
// for all of a thread's values before any is used (loops unrolled to E), so a
// work item waits for memory once per phase rather than once per value.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"
#include "fft_device.hpp"

namespace slicq {

// Largest block each kernel is compiled for (its __launch_bounds__).
constexpr int kPassThreads = 512;     // k_fwd_pass1/2, k_inv_passA/B (largest block)
// Band kernels: items of at most kAnaSmallValues / kSynSmallValues values run
// with kSmallE values per thread; larger ones with kBigAnaE / kBigSynE values
// per thread in blocks of up to 1024 threads, all at kSmallWaves waves per
// SIMD (FFT radix at most 8).
constexpr int kSmallE = 8;
constexpr int kBigAnaE = 8;
constexpr int kBigSynE = 16;
constexpr int kSmallWaves = 4;
template <class T>
constexpr int kSynSmallWaves = sizeof(T) == 4 ? 6 : 4;   // small synthesis items (FP32: 3 blocks of 512 per CU)
constexpr int kAnaThreads = kAnaSmallValues / kSmallE;   // k_band_ana, small items
constexpr int kAnaBigThreads = 1024;                     // k_band_ana, large items
constexpr int kSynThreads = kSynSmallValues / kSmallE;   // k_band_syn, small items
constexpr int kSynBigThreads = 1024;                     // k_band_syn, large items
static_assert(kAnaBigThreads * kBigAnaE >= 8192 && kSynBigThreads * kBigSynE >= kSynMaxValues,
              "large work items must fit one block");
constexpr int kPassE = 8;             // values per thread in the slice-FFT passes
// Waves per SIMD the slice-FFT passes are compiled for: the row passes fit
// 64 VGPRs in FP32 (4 blocks of 512 per CU); the column passes hold their
// prefetched per-output data across the transform and would spill there.
constexpr int kRowPassWavesF32 = 8;
constexpr int kColPassWaves = 4;
// Largest padded length and coefficient count of one signal: offsets inside a
// signal are 32-bit.
constexpr int64_t kMaxSignalElems = 0x7fffffffLL;

template <class T>
struct KArgs {
  const C2<T>* tw;        // twiddle pyramid
  const C2<T>* tw8;       // radix-8 twiddle rows of the band FFTs (TwBand)
  const T* h0;            // analysis slice window (2N)
  const T* hsyn;          // synthesis slice window: h~_0 (synthesis) or h_0 (adjoint)
  const T* g;             // analysis band windows
  const BandDev* bands;
  const AnaGroupDev* ana;
  const SynGroupDev* syn;
  const SynRunDev* runs;
  const OlaRec<T>* ola2;  // frequency overlap-add program: first two entries of each bin, weighted
                          // by the dual windows (synthesis) or the analysis windows (adjoint)
  const int32_t* ent_off; // further entries of each bin
  const int2* ent_pos;
  const T* ent_w;
  int32_t N, Mt, K, N1;
  int32_t N2, logN1, min_M, pad1_;  // min_M: smallest M_k of the plan
  int32_t logN2, C, logC, P;
  int32_t logP, pad2_;
  // coefficient layout: coefficient n of band k (packing offset off_k) of
  // slice m sits at S off_k + m M_k + n (band-major) or m cps + off_k + n
  // (slice-major), relative to the signal's coef_base
  int32_t slice_major, cps;
  int64_t ws1, ws2;       // complex values per slice in the two workspace regions
  // tasks [task0, task1) of the call's task table are the ones being launched
  // (the time overlap-add needs to know which neighbouring slices come first)
  int64_t task0, task1;
  T scale;                // (2N)^{-1/2}
  // fused per-slice schedule (valid when fused != 0): items, overlap-add
  // records of the synthesis items (dual or, for the adjoint, analysis weights)
  const FusedItemDev* fana;
  const FusedItemDev* fsyn;
  const FOlaRec<T>* fola;
  const int32_t* fent_off;
  const int2* fent_pos;
  const T* fent_w;
  int32_t fused, nfana, nfsyn, flogM;
  int32_t fcap, pad3_;
  // mixed-radix band transforms (plans with M_k = 3 2^a or 5 2^a)
  const C2<T>* twmix;     // combination twiddles (mix_tw_base)
  const int32_t* bsmod;   // (-start_k) mod M_k per stored band
  int32_t mixL, pad4_;    // largest logP of the twiddle table
};

// Byte offset, 16-byte aligned, just past `values` padded complex values in LDS.
template <class T>
__host__ __device__ constexpr size_t lds_tail_offset(int values) {
  return ((size_t)padded(values) * 2 * sizeof(T) + 15) & ~(size_t)15;
}

// A slice's view of its signal (or ring): xs = x + x_base, sample j of the
// slice at (start + j) mod period, zero at and beyond `valid`. Offsets within
// one signal are 32-bit (the C ABI rejects longer signals).
struct SliceIn {
  int start, period, valid, even;
};

__device__ __forceinline__ SliceIn slice_in(const SliceTask& tk) {
  return {(int)tk.x_start, (int)tk.x_period, (int)tk.x_valid,
          ((tk.x_base | tk.x_start | tk.x_period) & 1) == 0};
}

template <class T>
__device__ __forceinline__ T load_sample(const T* __restrict__ xs, const SliceIn& si, int j) {
  int idx = si.start + j;
  if (idx >= si.period) idx -= si.period;
  return idx < si.valid ? xs[idx] : T(0);
}

// Samples j and j + 1 (j even) of the slice as one complex value. With an even
// base, start and period the pair is contiguous and aligned: one vector load.
template <class T>
__device__ __forceinline__ C2<T> load_sample_pair(const T* __restrict__ xs, const SliceIn& si, int j) {
  if (si.even) {
    int idx = si.start + j;
    if (idx >= si.period) idx -= si.period;
    if (idx + 1 < si.valid) return *reinterpret_cast<const C2<T>*>(xs + idx);
    return {idx < si.valid ? xs[idx] : T(0), T(0)};
  }
  return {load_sample(xs, si, j), load_sample(xs, si, j + 1)};
}

// ---------------------------------------------------------------------------
// Dispatches a runtime FFT length 2^logn (1..10) to BODY<L>(args...).
#define SLICQ_LOGN_SWITCH(logn, CALL)                                                              \
  switch (logn) {                                                                                 \
    case 1: CALL(1); break;                                                                       \
    case 2: CALL(2); break;                                                                       \
    case 3: CALL(3); break;                                                                       \
    case 4: CALL(4); break;                                                                       \
    case 5: CALL(5); break;                                                                       \
    case 6: CALL(6); break;                                                                       \
    case 7: CALL(7); break;                                                                       \
    case 8: CALL(8); break;                                                                       \
    case 9: CALL(9); break;                                                                       \
    default: CALL(10); break;                                                                     \
  }

// Forward FFT of a slice, pass 1: columns. The N complex values
// z[n] = x_m[2n] + i x_m[2n+1] are indexed n = n1 + N1 n2; this item takes the
// C columns n1 in [cb C, cb C + C), transforms each over n2 (length N2 =
// 2^LOGN), applies e^{-2 pi i n1 k2 / N} and stores W1[k2 N1 + n1]. The first
// FFT pass reads the windowed samples directly and the last one stores to W1.
// Samples outside the support of h_0 are not read (their pair index is
// clamped into it and the window, zero there, drops them). plain (uniform):
// the whole window lies inside the valid, unwrapped part of the signal, so
// pairs are single vector loads; only the loads differ between the two cases,
// the arithmetic is one code path (a signal's result does not depend on where
// it sits in a batch).
template <class T, int LOGN, class TW>
__device__ __forceinline__ void fwd_pass1_body(const KArgs<T>& a, const SliceTask& tk, int cb, C2<T>* buf,
                                               const TW& tws, const InterTw<T>& inter, const T* __restrict__ x,
                                               C2<T>* __restrict__ out, bool plain, int tid, int nthr) {
  const int jlo = ((a.N - a.Mt) / 2) & ~1;           // first sample pair touching the support of h_0
  const int jhi = (a.N + (a.N + a.Mt) / 2 - 1) & ~1;  // last one
  const T* __restrict__ xs = x + tk.x_base;
  const SliceIn si = slice_in(tk);
  const int c0 = cb * a.C;
  // the window product is rounded by itself: the same value whichever load
  // path fed it, so both instantiations below give bitwise equal results
  auto load_plain = [&](int s, int e) -> C2<T> {
    const int j = 2 * (c0 + s + a.N1 * e);
    const int jc = imin(imax(j, jlo), jhi);
    const C2<T> x2 = *reinterpret_cast<const C2<T>*>(xs + si.start + jc);
    const C2<T> h2 = *reinterpret_cast<const C2<T>*>(a.h0 + j);
    return {mul_rn(x2.x, h2.x), mul_rn(x2.y, h2.y)};
  };
  auto load_any = [&](int s, int e) -> C2<T> {
    const int j = 2 * (c0 + s + a.N1 * e);
    const int jc = imin(imax(j, jlo), jhi);
    const C2<T> x2 = load_sample_pair(xs, si, jc);
    const C2<T> h2 = *reinterpret_cast<const C2<T>*>(a.h0 + j);
    return {mul_rn(x2.x, h2.x), mul_rn(x2.y, h2.y)};
  };
  auto store = [&](int, int, int s, int e, C2<T> v) {
    out[e * a.N1 + c0 + s] = cmul(v, inter.template get<-1>(((c0 + s) * e) & (a.N - 1)));
  };
  // one branch per block: a per-load choice made the compiler wait for every
  // load before issuing the next
  if (plain) fft_ci_fused<T, -1, kPassE, LOGN, true, true, false>(buf, a.logC, tws, tid, nthr, load_plain, store);
  else fft_ci_fused<T, -1, kPassE, LOGN, true, true, false>(buf, a.logC, tws, tid, nthr, load_any, store);
}

// TWL stages the FFT twiddles in LDS. LDS: values (padded) | FFT twiddles (N2)
// | four-step tables (N1 + N2).
template <class T, bool TWL>
__global__ void __launch_bounds__(kPassThreads) __attribute__((amdgpu_waves_per_eu(kColPassWaves)))
k_fwd_pass1(KArgs<T> a, const SliceTask* __restrict__ tasks, const T* __restrict__ x, C2<T>* __restrict__ W1) {
  extern __shared__ unsigned char smem[];
  C2<T>* buf = reinterpret_cast<C2<T>*>(smem);
  const int nCB = a.N1 >> a.logC;
  const int task = blockIdx.x / nCB, cb = blockIdx.x - task * nCB;
  const SliceTask tk = tasks[task];
  if (tk.S == 0) return;                              // unused task slot
  const int tid = threadIdx.x, nthr = blockDim.x;
  C2<T>* twl = buf + padded(a.C * a.N2);
  const InterTw<T> inter{twl + a.N2, twl + a.N2 + a.N1, a.logN2};
  stage_inter(twl + a.N2, twl + a.N2 + a.N1, a.tw, a.N, a.N1, a.N2, tid, nthr);
  if constexpr (TWL) stage_twiddles(twl, a.tw, a.N2, tid, nthr);
  const SliceIn si = slice_in(tk);
  const bool plain = si.even && si.start >= 0 && si.start + 2 * a.N <= imin(si.valid, si.period);
  C2<T>* out = W1 + (int64_t)task * a.ws1;
  const TwLds<T> tl{twl};
  const TwGlobal<T> tg{a.tw};
#define SLICQ_P1(L)                                                                             \
  if constexpr (TWL) fwd_pass1_body<T, L>(a, tk, cb, buf, tl, inter, x, out, plain, tid, nthr);  \
  else fwd_pass1_body<T, L>(a, tk, cb, buf, tg, inter, x, out, plain, tid, nthr);
  SLICQ_LOGN_SWITCH(a.logN2, SLICQ_P1)
#undef SLICQ_P1
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

// The pair (k, N - k) of packed-spectrum bins a pass-2 unit t handles, and
// where the two values sit in LDS (sequence-interleaved rows). Row 0 pairs k1
// with N1 - k1 (k1 < N1/2; unit k1 = 0 also yields bin N/2 at la2); row N2/2
// pairs k1 with N1 - 1 - k1.
struct PairIdx {
  int k, la, lb, la2;
};

__device__ __forceinline__ PairIdx pass2_pair(int t, int rb, int P, int logP, int N1, int N2, int logTwoP) {
  const int i = t & (P - 1), k1 = t >> logP;
  const int row = rb * P + i;
  PairIdx q;
  q.la2 = -1;
  if (row != 0) {
    q.k = N2 * k1 + row;
    q.la = (k1 << logTwoP) + i;
    q.lb = ((N1 - 1 - k1) << logTwoP) + P + i;
  } else if (k1 < N1 / 2) {
    q.k = N2 * k1;
    q.la = k1 << logTwoP;
    q.lb = ((N1 - k1) & (N1 - 1)) << logTwoP;
    if (k1 == 0) q.la2 = (N1 / 2) << logTwoP;
  } else {
    const int kk = k1 - N1 / 2;
    q.k = N2 * kk + N2 / 2;
    q.la = (kk << logTwoP) + P;
    q.lb = ((N1 - 1 - kk) << logTwoP) + P;
  }
  return q;
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
// (length N1 = 2^LOGN), giving Zc[N2 k1 + k2], and splits pairs (k, N - k)
// into the real spectrum X[0..N] of the slice (W2). The rows are read in
// natural order (coalesced) into LDS first: a fused first pass would read
// them coalesced only in an order whose LDS writes conflict on one bank.
template <class T, int LOGN, class TW>
__device__ __forceinline__ void fwd_pass2_fft(int logTwoP, C2<T>* buf, const TW& tws, int tid, int nthr) {
  auto none_ld = [](int, int) { return C2<T>{T(0), T(0)}; };
  auto none_st = [](int, int, int, int, C2<T>) {};
  fft_ci_fused<T, -1, kPassE, LOGN, false, false, false>(buf, logTwoP, tws, tid, nthr, none_ld, none_st);
}

// TWL stages the FFT twiddles in LDS. LDS: values (padded) | twiddles.
template <class T, bool TWL>
__global__ void __launch_bounds__(kPassThreads) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? kRowPassWavesF32 : 4)))
k_fwd_pass2(KArgs<T> a, const C2<T>* __restrict__ W1, C2<T>* __restrict__ W2) {
  extern __shared__ unsigned char smem[];
  C2<T>* buf = reinterpret_cast<C2<T>*>(smem);
  const int nRB = (a.N2 / 2) >> a.logP;
  const int task = blockIdx.x / nRB, rb = blockIdx.x - task * nRB;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int P = a.P, twoP = 2 * a.P, logTwoP = a.logP + 1;
  const int total = twoP * a.N1, N = a.N, units = P * a.N1;
  C2<T>* twl = buf + padded(total);
  const C2<T>* in = W1 + (int64_t)task * a.ws1;
  constexpr int U = kPassE / 2;
  C2<T> w[U];
#pragma unroll
  for (int i = 0; i < U; ++i) {
    const PairIdx q = pass2_pair(imin(tid + i * nthr, units - 1), rb, P, a.logP, a.N1, a.N2, logTwoP);
    w[i] = twiddle<T, -1>(a.tw, 2 * N, q.k);
  }
  const C2<T> w2 = twiddle<T, -1>(a.tw, 2 * N, N / 2);
  C2<T> v[kPassE];
#pragma unroll
  for (int i = 0; i < kPassE; ++i) {
    const int e = imin(tid + i * nthr, total - 1);
    v[i] = in[pass2_row(rb, e >> a.logN1, P, a.N2) * a.N1 + (e & (a.N1 - 1))];
  }
  if constexpr (TWL) stage_twiddles(twl, a.tw, a.N1, tid, nthr);
#pragma unroll
  for (int i = 0; i < kPassE; ++i) {
    const int e = tid + i * nthr;
    if (e < total) buf[pidx(((e & (a.N1 - 1)) << logTwoP) + (e >> a.logN1))] = v[i];
  }
  __syncthreads();
  const TwLds<T> tl{twl};
  const TwGlobal<T> tg{a.tw};
#define SLICQ_P2(L)                                                   \
  if constexpr (TWL) fwd_pass2_fft<T, L>(logTwoP, buf, tl, tid, nthr); \
  else fwd_pass2_fft<T, L>(logTwoP, buf, tg, tid, nthr);
  SLICQ_LOGN_SWITCH(a.logN1, SLICQ_P2)
#undef SLICQ_P2
  C2<T>* X = W2 + (int64_t)task * a.ws2;
#pragma unroll
  for (int i = 0; i < U; ++i) {
    const int t = tid + i * nthr;
    if (t < units) {
      const PairIdx q = pass2_pair(t, rb, P, a.logP, a.N1, a.N2, logTwoP);
      C2<T> xk, xnk;
      real_split(buf[pidx(q.la)], buf[pidx(q.lb)], w[i], a.scale, xk, xnk);
      X[q.k] = xk;
      X[N - q.k] = xnk;
      if (q.la2 >= 0) {
        const C2<T> zh = buf[pidx(q.la2)];
        real_split(zh, zh, w2, a.scale, xk, xnk);
        X[N / 2] = xk;
      }
    }
  }
}

// Stages the TwLds table for FFT lengths up to n (n - 1 entries) at twl:
// one entry per thread when the block covers the table, else each thread
// issues up to 8 loads before writing any of them.
template <class T>
__device__ __forceinline__ void stage_twiddles(C2<T>* twl, const C2<T>* __restrict__ tw, int n, int tid, int nthr) {
  if (n - 1 <= nthr) {
    if (tid < n - 1) twl[tid] = tw_stage_value(tw, tid);
    return;
  }
  for (int b = tid; b < n - 1; b += 8 * nthr) {
    C2<T> v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = tw_stage_value(tw, imin(b + q * nthr, n - 2));
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (b + q * nthr < n - 1) twl[b + q * nthr] = v[q];
  }
}

// The TwBand tables for transforms up to 2^L: split hi levels, split lo
// levels, then (P8) the radix-8 rows.
template <bool P8, class T>
__device__ __forceinline__ void stage_band(C2<T>* t, const C2<T>* __restrict__ tw, const C2<T>* __restrict__ tw8,
                                           int L, int tid, int nthr) {
  const int nh = 1 << (L - (L >> 1)), nl = 1 << (L >> 1), ns = nh + nl;
  for (int i = tid; i < band_tw_entries(L, P8); i += nthr)
    t[i] = i < nh ? tw[nh + i] : i < ns ? tw[(1 << L) + i - nh] : tw8[i - ns];
}

template <bool P8, class T>
__device__ __forceinline__ TwBand<T, P8> band_tw(const C2<T>* t, int L) {
  return TwBand<T, P8>{t, L, t + split_tw_entries(L)};
}

// Stages the four-step twiddle tables of InterTw: hi[q] = e^{-2 pi i q / N1}
// (level N1 of the pyramid) and lo[r] = e^{-2 pi i r / N} for r < N2 (one
// entry per thread when the block covers both).
template <class T>
__device__ __forceinline__ void stage_inter(C2<T>* hi, C2<T>* lo, const C2<T>* __restrict__ tw, int N, int N1,
                                            int N2, int tid, int nthr) {
  if (N1 + N2 <= nthr) {
    if (tid < N1) hi[tid] = tw[N1 + tid];
    else if (tid < N1 + N2) lo[tid - N1] = tw[N + tid - N1];
    return;
  }
  for (int b = tid; b < N1 + N2; b += 8 * nthr) {
    C2<T> v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int i = imin(b + q * nthr, N1 + N2 - 1);
      v[q] = i < N1 ? tw[N1 + i] : tw[N + i - N1];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int i = b + q * nthr;
      if (i < N1) hi[i] = v[q];
      else if (i < N1 + N2) lo[i - N1] = v[q];
    }
  }
}

// Band analysis of one work item with M_k = 2^LOGN (bands k0 .. k0 + cnt - 1).
// The first FFT pass is fused with the gather: a thread takes the R values of
// one first-pass butterfly (all in one band), forms X[j] g_k[j] for them,
// transforms in registers and writes LDS. Middle passes run in LDS. The last
// pass stores its outputs straight to the coefficients. DIR = +1 (e^{+}).
template <class T, int E, int LOGN, class TW>
__device__ __forceinline__ void band_ana_fft(const KArgs<T>& a, const SliceTask& tk, const AnaGroupDev& G,
                                             const C2<T>* __restrict__ X, C2<T>* __restrict__ cs, C2<T>* buf,
                                             const TW& tws, int tid, int nthr) {
  constexpr int M = 1 << LOGN, MASK = M - 1;
  constexpr int LR1 = pass_log_radix(LOGN, 0, 8), R1 = 1 << LR1, U1 = E / R1;
  constexpr int LU1 = LOGN - LR1;               // log2 first-pass units per band
  constexpr int LAST = last_pass_logns(LOGN, 8);
  const int units1 = G.cnt << LU1;
  // gather in first-pass order: unit u of band s holds slots j + r 2^LU1
  int xi[U1][R1], wi[U1][R1];
#pragma unroll
  for (int i = 0; i < U1; ++i) {
    const int u = imin(tid + i * nthr, units1 - 1);
    const int sb = u >> LU1, j = u & ((1 << LU1) - 1);
    const BandDev B = a.bands[G.k0 + sb];
    const bool live = tid + i * nthr < units1;
#pragma unroll
    for (int r = 0; r < R1; ++r) {
      const int slot = j + (r << LU1);
      const int t = (slot - B.start) & MASK;
      const int jb = B.start + t;                 // signed bin, -N < jb < 2N
      const bool in = live && t < B.len;
      const int jj = jb < 0 ? -jb : (jb > a.N ? 2 * a.N - jb : jb);
      const bool cj = jb < 0 || jb > a.N;
      xi[i][r] = in ? (cj ? ~jj : jj) : 0;          // ~jj (< 0) marks a conjugate
      wi[i][r] = in ? B.goff + t : -1;
    }
  }
  C2<T> v[U1][R1];
  T gv[U1][R1];
#pragma unroll
  for (int i = 0; i < U1; ++i) {
#pragma unroll
    for (int r = 0; r < R1; ++r) {
      v[i][r] = X[xi[i][r] < 0 ? ~xi[i][r] : xi[i][r]];
      gv[i][r] = a.g[imax(wi[i][r], 0)];
    }
  }
#pragma unroll
  for (int i = 0; i < U1; ++i) {
#pragma unroll
    for (int r = 0; r < R1; ++r) {
      const T w = wi[i][r] < 0 ? T(0) : gv[i][r];
      v[i][r] = {v[i][r].x * w, (xi[i][r] < 0 ? -v[i][r].y : v[i][r].y) * w};
    }
    dft_reg<T, R1, 1>(v[i]);
  }
  // band-major: c(k0 + s, m, n) at S off_{k0+s} + m M + n; slice-major: m cps + off_{k0+s} + n
  const int off0 = a.bands[G.k0].off;
  const int cbase = a.slice_major ? tk.m * a.cps + off0 : tk.S * off0 + tk.m * M;
  const int bstride = a.slice_major ? M : tk.S * M;   // band k0 + s starts s bstride later
  if constexpr (LAST == 0) {
    // a single pass: outputs n = r of unit j = 0
#pragma unroll
    for (int i = 0; i < U1; ++i) {
      const int u = tid + i * nthr;
      if (u < units1) {
#pragma unroll
        for (int r = 0; r < R1; ++r) cs[cbase + u * bstride + r] = v[i][r];
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < U1; ++i) {
      const int u = tid + i * nthr;
      if (u < units1) {
        const int sb = u >> LU1, j = u & ((1 << LU1) - 1);
        const int p0 = (sb << LOGN) + (j << LR1);
#pragma unroll
        for (int r = 0; r < R1; ++r) buf[pidx(p0 + r)] = v[i][r];
      }
    }
    __syncthreads();
    lds_fft_c<T, 1, E, 8, LOGN, LR1, TW, LAST>(buf, 0, G.cnt, tws, tid, nthr);
    // last pass: LDS -> registers -> coefficients
    constexpr int LRL = LOGN - LAST, RL = 1 << LRL, UL = E / RL, NS = 1 << LAST;
    constexpr int LUL = LOGN - LRL;
    const int unitsL = G.cnt << LUL;
    C2<T> q[UL][RL];
#pragma unroll
    for (int i = 0; i < UL; ++i) {
      const int u = imin(tid + i * nthr, unitsL - 1);
      const int sb = u >> LUL, j = u & ((1 << LUL) - 1);
      const int p0 = (sb << LOGN) + j;
      const int pb = pidx(p0);
#pragma unroll
      for (int r = 0; r < RL; ++r) q[i][r] = buf[pidx_step<(1 << LUL)>(pb, p0, r)];
    }
#pragma unroll
    for (int i = 0; i < UL; ++i) {
      const int u = imin(tid + i * nthr, unitsL - 1);
      C2<T> w[RL];
      pass_twiddles<T, 1, RL, NS>(tws, u & (NS - 1), w);
#pragma unroll
      for (int r = 1; r < RL; ++r) q[i][r] = cmul(q[i][r], w[r]);
      dft_reg<T, RL, 1>(q[i]);
    }
#pragma unroll
    for (int i = 0; i < UL; ++i) {
      const int u = tid + i * nthr;
      if (u < unitsL) {
        // LAST + LRL = LOGN: unit j < NS writes outputs n = j + r NS of its band
        const int sb = u >> LUL, j = u & ((1 << LUL) - 1);
#pragma unroll
        for (int r = 0; r < RL; ++r) cs[cbase + sb * bstride + j + r * NS] = q[i][r];
      }
    }
  }
}

// Band analysis: bands k0 .. k0 + cnt - 1 of one slice. Slot r of band k
// holds X[j] g_k[j] for the bin j of J_k with j = r (mod M_k), or 0; the
// inverse DFT of length M_k gives c^m_{n,k} (equation CQ_coeff). Bins
// outside [0, N] read the half spectrum by conjugate symmetry.
// Block b takes work item g0 + b mod ng of task b / ng (the items of one
// slice run together: their spectrum reads overlap). TWL stages the
// twiddles of lengths up to M in LDS, otherwise the TwBand tables.
// LDS: values (padded) | twiddles.
template <class T, int E, int NT, int WPE, bool TWL>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE)))
k_band_ana(KArgs<T> a, const SliceTask* __restrict__ tasks, const C2<T>* __restrict__ W2, C2<T>* __restrict__ coef,
           int g0, int ng) {
  extern __shared__ unsigned char smem[];
  C2<T>* buf = reinterpret_cast<C2<T>*>(smem);
  const int task = blockIdx.x / ng, gi = g0 + (int)blockIdx.x - task * ng;
  const AnaGroupDev G = a.ana[gi];
  const SliceTask tk = tasks[task];
  if (tk.S == 0) return;
  const int tid = threadIdx.x, nthr = blockDim.x;
  C2<T>* twl = reinterpret_cast<C2<T>*>(smem + lds_tail_offset<T>(G.cnt << G.logM));
  if constexpr (TWL) stage_twiddles(twl, a.tw, G.M, tid, nthr);
  else stage_band<false>(twl, a.tw, a.tw8, G.logM, tid, nthr);   // the radix-8 rows cost more than they save here
  const C2<T>* __restrict__ X = W2 + (int64_t)task * a.ws2;
  C2<T>* __restrict__ cs = coef + tk.coef_base;
  const TwLds<T> tws{twl};
#define SLICQ_ANA_CASE(L)                                                                  \
  case L:                                                                                  \
    if constexpr (TWL) band_ana_fft<T, E, L>(a, tk, G, X, cs, buf, tws, tid, nthr);        \
    else band_ana_fft<T, E, L>(a, tk, G, X, cs, buf, band_tw<false>(twl, L), tid, nthr);   \
    break;
  switch (G.logM) {
    SLICQ_ANA_CASE(1) SLICQ_ANA_CASE(2) SLICQ_ANA_CASE(3) SLICQ_ANA_CASE(4) SLICQ_ANA_CASE(5)
    SLICQ_ANA_CASE(6) SLICQ_ANA_CASE(7) SLICQ_ANA_CASE(8) SLICQ_ANA_CASE(9) SLICQ_ANA_CASE(10)
    SLICQ_ANA_CASE(11) SLICQ_ANA_CASE(12)
    default:
      if constexpr (TWL) band_ana_fft<T, E, 13>(a, tk, G, X, cs, buf, tws, tid, nthr);
      else band_ana_fft<T, E, 13>(a, tk, G, X, cs, buf, band_tw<false>(twl, 13), tid, nthr);
      break;
  }
#undef SLICQ_ANA_CASE
}

// Element index of LDS position p of a synthesis item inside run R: band
// k0 + q / M, coefficient q mod M, q = p - lds_off (band-major layout).
__device__ __forceinline__ int run_coef_index(const SliceTask& tk, const SynRunDev& R, int p) {
  const int q = p - R.lds_off;
  return tk.S * (R.off + (q >> R.logM) * R.M) + tk.m * R.M + (q & (R.M - 1));
}

// Band synthesis: owned bins [lo, hi) of the half spectrum of one slice.
// Every band ke..kb is transformed (DFT_{M_k}, runs of equal M_k), then each
// owned bin runs its overlap-add program: the sum over the bands covering it,
// in increasing k, of weight * C_k[j mod M_k] (for the self-mirrored DC and
// Nyquist bands weight * (C[j mod M] + conj C[-j mod M]), the real part of the
// full synthesis). Block (x, y, z) takes work item g0 + y of task
// z gridDim.x + x: one item of a tile of consecutive slices runs together
// (they read the same overlap-add records and twiddles; tiles keep the band
// an item shares with its neighbour in cache until the neighbour reads it). TWL stages the twiddles of lengths up to the item's largest
// M in LDS, otherwise the TwBand tables. LDS: values (padded) | twiddles.
template <class T, int E, int NT, int WPE, bool TWL>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE)))
k_band_syn(KArgs<T> a, const SliceTask* __restrict__ tasks, const C2<T>* __restrict__ coef, C2<T>* __restrict__ W2,
           T* __restrict__ y, int g0, int ntask) {
  extern __shared__ unsigned char smem[];
  C2<T>* buf = reinterpret_cast<C2<T>*>(smem);
  const int task = (int)(blockIdx.z * gridDim.x + blockIdx.x), gi = g0 + (int)blockIdx.y;
  if (task >= ntask) return;                   // padding of the last tile
  const SynGroupDev G = a.syn[gi];
  const SliceTask tk = tasks[task];
  if (tk.S == 0) return;
  const int tid = threadIdx.x, nthr = blockDim.x;
  C2<T>* twl = reinterpret_cast<C2<T>*>(smem + lds_tail_offset<T>(G.total));
  const int Lmax = 31 - __builtin_clz((unsigned)G.maxM);
  const C2<T>* __restrict__ cs = coef + tk.coef_base;
  if ((E == 8 || E == 16) && a.min_M >= 8) {
    // first radix-8 pass fused with the loads: unit u (all runs flattened,
    // u = p / 8) takes slots j + r M/8 of one band, r = 0..7
    const int units = G.total >> 3;
#pragma unroll
    for (int i = 0; i < E / 8; ++i) {
      const bool live = wave_has(tid + i * nthr, units);   // idle waves skip loads and arithmetic
      const int u = imin(tid + i * nthr, units - 1);
      const int p = u << 3;
      int lds_off = G.r[0].lds_off, off = G.r[0].off, M = G.r[0].M, logM = G.r[0].logM;
      for (int r = 1; r < G.nrun; ++r) {
        SynRunDev R;
        if (r == 1) R = G.r[1];
        else R = a.runs[G.run0 + r];
        if (p >= R.lds_off) { lds_off = R.lds_off; off = R.off; M = R.M; logM = R.logM; }
      }
      const int lu = logM - 3, q = (p - lds_off) >> 3;
      const int sb = q >> lu, j = q & ((1 << lu) - 1);
      const int cbase = a.slice_major ? tk.m * a.cps + off + sb * M + j : tk.S * (off + sb * M) + tk.m * M + j;
      C2<T> v[8];
      if (live) {
#pragma unroll
        for (int r = 0; r < 8; ++r) v[r] = cs[cbase + (r << lu)];
      }
      if (i == 0) {
        if constexpr (TWL) stage_twiddles(twl, a.tw, G.maxM, tid, nthr);
        else stage_band<true>(twl, a.tw, a.tw8, Lmax, tid, nthr);
      }
      if (live) {
        dft_reg<T, 8, -1>(v);
        if (tid + i * nthr < units) {
          const int p0 = lds_off + (sb << logM) + (j << 3);
#pragma unroll
          for (int r = 0; r < 8; ++r) buf[pidx(p0 + r)] = v[r];
        }
      }
    }
    __syncthreads();
    for (int ri = 0; ri < G.nrun; ++ri) {
      SynRunDev R;
      if (ri == 0) R = G.r[0];
      else if (ri == 1) R = G.r[1];
      else R = a.runs[G.run0 + ri];
      // an opaque copy of the thread index: keeps the compiler from hoisting
      // the address arithmetic of every FFT length out of this loop (registers)
      int t = tid;
      asm volatile("" : "+v"(t));
      if constexpr (TWL) lds_fft_contig_after8<T, -1, E>(buf, R.lds_off, R.logM, R.cnt, TwLds<T>{twl}, t, nthr);
      else lds_fft_contig_after8<T, -1, E>(buf, R.lds_off, R.logM, R.cnt, band_tw<true>(twl, Lmax), t, nthr);
    }
  } else {
    // coefficient addresses of a batch of values (no branches), then every load
    // of the batch; batches of 8 values per thread bound the registers
    const SynRunDev R0 = G.r[0];
    constexpr int EB = E < 8 ? E : 8;
#pragma unroll
    for (int c = 0; c < E; c += EB) {
      int idx[EB];
      if (a.slice_major) {
#pragma unroll
        for (int i = 0; i < EB; ++i) idx[i] = tk.m * a.cps + R0.off + imin(tid + (c + i) * nthr, G.total - 1);
      } else {
#pragma unroll
        for (int i = 0; i < EB; ++i) idx[i] = run_coef_index(tk, R0, imin(tid + (c + i) * nthr, G.total - 1));
        for (int r = 1; r < G.nrun; ++r) {
          SynRunDev R;
          if (r == 1) R = G.r[1];
          else R = a.runs[G.run0 + r];
#pragma unroll
          for (int i = 0; i < EB; ++i) {
            const int p = imin(tid + (c + i) * nthr, G.total - 1);
            if (p >= R.lds_off) idx[i] = run_coef_index(tk, R, p);
          }
        }
      }
      C2<T> v[EB];
#pragma unroll
      for (int i = 0; i < EB; ++i) v[i] = cs[idx[i]];
      if (c == 0) {
        if constexpr (TWL) stage_twiddles(twl, a.tw, G.maxM, tid, nthr);
        else stage_band<true>(twl, a.tw, a.tw8, Lmax, tid, nthr);
      }
#pragma unroll
      for (int i = 0; i < EB; ++i) {
        const int p = tid + (c + i) * nthr;
        if (p < G.total) buf[pidx(p)] = v[i];
      }
    }
    __syncthreads();
    for (int ri = 0; ri < G.nrun; ++ri) {
      SynRunDev R;
      if (ri == 0) R = G.r[0];
      else if (ri == 1) R = G.r[1];
      else R = a.runs[G.run0 + ri];
      int t = tid;
      asm volatile("" : "+v"(t));
      if constexpr (TWL) lds_fft_contig<T, -1, E, 8>(buf, R.lds_off, R.logM, R.cnt, TwLds<T>{twl}, t, nthr);
      else lds_fft_contig<T, -1, E, 8>(buf, R.lds_off, R.logM, R.cnt, band_tw<true>(twl, Lmax), t, nthr);
    }
  }
  C2<T>* Z = W2 + (int64_t)task * a.ws2;
  constexpr int QB = 2;                         // owned bins per thread per round
  for (int j0 = G.lo + tid; j0 < G.hi; j0 += QB * nthr) {
    OlaRec<T> rec[QB];
#pragma unroll
    for (int q = 0; q < QB; ++q) rec[q] = a.ola2[imin(j0 + q * nthr, G.hi - 1)];
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int j = j0 + q * nthr;
      if (j >= G.hi) continue;
      const uint32_t y0 = rec[q].yy & kOlaNone, y1 = rec[q].yy >> 16;
      C2<T> c0 = buf[pidx(rec[q].xx & kOlaPosMask)], c1 = buf[pidx(rec[q].xx >> 16)];
      // mirror entries only in the bins of the DC and Nyquist bands
      if (y0 != kOlaNone) c0 = cadd(c0, cconj(buf[pidx(y0)]));
      if (y1 != kOlaNone) c1 = cadd(c1, cconj(buf[pidx(y1)]));
      C2<T> acc = cadd(cscale(c0, rec[q].w0), cscale(c1, rec[q].w1));
      if (rec[q].xx & kOlaMore) {                 // bins covered by more than two bands
        for (int e = a.ent_off[j]; e < a.ent_off[j + 1]; ++e) {
          const int2 pe = a.ent_pos[e];
          C2<T> c = buf[pidx(pe.x)];
          if (pe.y >= 0) c = cadd(c, cconj(buf[pidx(pe.y)]));
          acc = cadd(acc, cscale(c, a.ent_w[e]));
        }
      }
      Z[j] = acc;
    }
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

// Row IFFTs of inverse pass A (length N1 = 2^LOGN) from the packed spectrum in
// LDS; the last FFT pass applies e^{+2 pi i n1 k2 / N} and stores W1.
template <class T, int LOGN, class TW>
__device__ __forceinline__ void inv_passA_fft(const KArgs<T>& a, int rb, int logTwoP, C2<T>* buf, const TW& tws,
                                              const InterTw<T>& inter, C2<T>* __restrict__ out, int tid, int nthr) {
  auto none = [](int, int) { return C2<T>{T(0), T(0)}; };
  auto store = [&](int, int, int s, int e, C2<T> v) {
    const int row = pass2_row(rb, s, a.P, a.N2);
    out[row * a.N1 + e] = cmul(v, inter.template get<1>((e * row) & (a.N - 1)));
  };
  fft_ci_fused<T, 1, kPassE, LOGN, false, true, true>(buf, logTwoP, tws, tid, nthr, none, store);
}

// TWL stages the FFT twiddles in LDS. LDS: values (padded) | FFT twiddles (N1)
// | four-step tables (N1 + N2).
template <class T, bool TWL>
__global__ void __launch_bounds__(kPassThreads) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? kRowPassWavesF32 : 4)))
k_inv_passA(KArgs<T> a, const C2<T>* __restrict__ W2, C2<T>* __restrict__ W1) {
  extern __shared__ unsigned char smem[];
  C2<T>* buf = reinterpret_cast<C2<T>*>(smem);
  const int nRB = (a.N2 / 2) >> a.logP;
  const int task = blockIdx.x / nRB, rb = blockIdx.x - task * nRB;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int P = a.P, twoP = 2 * a.P, logTwoP = a.logP + 1;
  const int N = a.N, N1 = a.N1, N2 = a.N2;
  const int units = P * N1, total = twoP * N1;
  C2<T>* twl = buf + padded(total);
  const InterTw<T> inter{twl + N1, twl + 2 * N1, a.logN2};
  const C2<T>* Z = W2 + (int64_t)task * a.ws2;
  constexpr int U = kPassE / 2;
  // every load first: spectrum pairs and their twiddles
  C2<T> za[U], zb[U], w[U];
#pragma unroll
  for (int i = 0; i < U; ++i) {
    const PairIdx q = pass2_pair(imin(tid + i * nthr, units - 1), rb, P, a.logP, N1, N2, logTwoP);
    za[i] = Z[q.k];
    zb[i] = Z[N - q.k];
    w[i] = twiddle<T, 1>(a.tw, 2 * N, q.k);
  }
  const C2<T> zh = Z[N / 2], wh = twiddle<T, 1>(a.tw, 2 * N, N / 2);
  stage_inter(twl + N1, twl + 2 * N1, a.tw, N, N1, N2, tid, nthr);
  if constexpr (TWL) stage_twiddles(twl, a.tw, N1, tid, nthr);
#pragma unroll
  for (int i = 0; i < U; ++i) {
    const int t = tid + i * nthr;
    if (t < units) {
      const PairIdx q = pass2_pair(t, rb, P, a.logP, N1, N2, logTwoP);
      C2<T> zk, znk;
      herm_pack(za[i], zb[i], w[i], zk, znk);
      buf[pidx(q.la)] = zk;
      if (q.k != 0) buf[pidx(q.lb)] = znk;     // bin 0 has no partner in [0, N)
      if (q.la2 >= 0) {
        herm_pack(zh, zh, wh, zk, znk);
        buf[pidx(q.la2)] = zk;
      }
    }
  }
  __syncthreads();
  C2<T>* out = W1 + (int64_t)task * a.ws1;
  const TwLds<T> tl{twl};
  const TwGlobal<T> tg{a.tw};
#define SLICQ_PA(L)                                                                 \
  if constexpr (TWL) inv_passA_fft<T, L>(a, rb, logTwoP, buf, tl, inter, out, tid, nthr); \
  else inv_passA_fft<T, L>(a, rb, logTwoP, buf, tg, inter, out, tid, nthr);
  SLICQ_LOGN_SWITCH(a.logN1, SLICQ_PA)
#undef SLICQ_PA
}

// Time overlap-add (Algorithm 4) without atomics. Window position j of a
// slice (0 <= j < 2N, output sample start + j) is its own when
// 2|j - N| <= N - Mt and is shared with the left (j < N) or right neighbour
// slice when N - Mt < 2|j - N| < N + Mt: the two overlaps of nov samples,
// |j - N| = ola_d0 .. ola_d0 + nov - 1. Of the two contributions to a shared
// sample, the one written first is stored into y; the other is stored into
// the slice's overlap buffer (left side at 0, right side at Mt) and added by
// k_ola_fix after the inverse pass. One rounding either way (a + b = b + a).
__host__ __device__ constexpr int ola_d0(int N, int Mt) { return (N - Mt) / 2 + 1; }
__host__ __device__ constexpr int ola_count(int N, int Mt) { return (N + Mt - 1) / 2 - (N - Mt) / 2; }

// Which sides of task gi (slice m of S; tasks of one signal are consecutive
// in m, neighbours circular) are written second: the left side when the left
// neighbour was launched in an earlier batch of tasks or is in this one, the
// right side when the right neighbour was launched in an earlier batch. With
// a single batch: every left side, no right side. Single-slice tasks (stream
// rings) take their neighbours from earlier and later calls.
__device__ __forceinline__ void ola_sides(const SliceTask& tk, int64_t gi, int64_t t0, int64_t t1, bool& add_l,
                                          bool& add_r) {
  if (tk.S <= 1) {
    add_l = true;
    add_r = false;
    return;
  }
  const int64_t iL = tk.m >= 1 ? gi - 1 : gi + tk.S - 1;
  const int64_t iR = tk.m <= tk.S - 2 ? gi + 1 : gi - (tk.S - 1);
  add_l = iL < t1;
  add_r = iR < t0;
}

// Stores v at window position j of a slice: into the output, or into the
// overlap buffer ov for a shared sample written second.
template <class T>
__device__ __forceinline__ void ola_store(T* __restrict__ ys, T* __restrict__ ov, int ystart, int yperiod,
                                          int yvalid, int j, T v, int N, int Mt, bool add_l, bool add_r) {
  const bool right = j > N;
  const int dj = right ? j - N : N - j;
  if (2 * dj >= N + Mt) return;
  int idx = ystart + j;
  if (idx >= yperiod) idx -= yperiod;
  if (idx >= yvalid) return;
  if (2 * dj > N - Mt && (right ? add_r : add_l)) ov[(right ? Mt : 0) + dj - ola_d0(N, Mt)] = v;
  else ys[idx] = v;
}

// Inverse pass B: columns n1 in [cb C, cb C + C): transform over k2 (length
// N2 = 2^LOGN, e^+; the first FFT pass reads W1 directly), giving
// z[n1 + N1 n2] = y[2n] + i y[2n+1]; the last pass scales, multiplies by the
// synthesis slice window and overlap-adds into the output (Algorithm 4) or
// the overlap buffer ov.
template <class T, int LOGN, class TW>
__device__ __forceinline__ void inv_passB_body(const KArgs<T>& a, const SliceTask& tk, int cb, C2<T>* buf,
                                               const TW& tws, const C2<T>* __restrict__ in, T* __restrict__ y,
                                               T* __restrict__ ov, bool add_l, bool add_r, int tid, int nthr) {
  constexpr int LAST = last_pass_logns(LOGN, 8), RL = 1 << (LOGN - LAST), UL = kPassE / RL, NS = 1 << LAST;
  const int c0 = cb * a.C, smask = a.C - 1, unitsL = 1 << (a.logC + LAST);
  // synthesis window at this thread's outputs, fetched before the transform
  C2<T> h[UL][RL];
#pragma unroll
  for (int i = 0; i < UL; ++i) {
    const int u = imin(tid + i * nthr, unitsL - 1);
    const int n1 = c0 + (u & smask), j = u >> a.logC;
#pragma unroll
    for (int r = 0; r < RL; ++r) h[i][r] = *reinterpret_cast<const C2<T>*>(a.hsyn + 2 * (n1 + a.N1 * (j + r * NS)));
  }
  T* __restrict__ ys = y + tk.y_base;
  const int ys0 = (int)tk.y_start, yper = (int)tk.y_period, yval = (int)tk.y_valid;
  auto load = [&](int s, int e) -> C2<T> { return in[e * a.N1 + c0 + s]; };
  auto store = [&](int i, int r, int s, int e, C2<T> z) {
    const int j = 2 * (c0 + s + a.N1 * e);
    ola_store(ys, ov, ys0, yper, yval, j, z.x * a.scale * h[i][r].x, a.N, a.Mt, add_l, add_r);
    ola_store(ys, ov, ys0, yper, yval, j + 1, z.y * a.scale * h[i][r].y, a.N, a.Mt, add_l, add_r);
  };
  fft_ci_fused<T, 1, kPassE, LOGN, true, true, false>(buf, a.logC, tws, tid, nthr, load, store);
}

// TWL stages the FFT twiddles in LDS. LDS: values (padded) | twiddles. The
// overlap buffer of a task is its W2 region (free once pass A has read it).
template <class T, bool TWL>
__global__ void __launch_bounds__(kPassThreads) __attribute__((amdgpu_waves_per_eu(kColPassWaves)))
k_inv_passB(KArgs<T> a, const SliceTask* __restrict__ tasks, const C2<T>* __restrict__ W1, C2<T>* __restrict__ W2,
            T* __restrict__ y) {
  extern __shared__ unsigned char smem[];
  C2<T>* buf = reinterpret_cast<C2<T>*>(smem);
  const int nCB = a.N1 >> a.logC;
  const int task = blockIdx.x / nCB, cb = blockIdx.x - task * nCB;
  const SliceTask tk = tasks[task];
  if (tk.S == 0) return;
  const int tid = threadIdx.x, nthr = blockDim.x;
  C2<T>* twl = buf + padded(a.C * a.N2);
  if constexpr (TWL) stage_twiddles(twl, a.tw, a.N2, tid, nthr);
  const C2<T>* in = W1 + (int64_t)task * a.ws1;
  T* ov = reinterpret_cast<T*>(W2 + (int64_t)task * a.ws2);
  bool add_l, add_r;
  ola_sides(tk, a.task0 + task, a.task0, a.task1, add_l, add_r);
  const TwLds<T> tl{twl};
  const TwGlobal<T> tg{a.tw};
#define SLICQ_PB(L)                                                                                 \
  if constexpr (TWL) inv_passB_body<T, L>(a, tk, cb, buf, tl, in, y, ov, add_l, add_r, tid, nthr); \
  else inv_passB_body<T, L>(a, tk, cb, buf, tg, in, y, ov, add_l, add_r, tid, nthr);
  SLICQ_LOGN_SWITCH(a.logN2, SLICQ_PB)
#undef SLICQ_PB
}

// Second contributions of the shared output samples: block b adds the
// buffered samples r*kOlaFixRun .. of side b % 2 (left, right) of task
// b / (2 * runs) into the output, for the sides written second (see
// ola_sides); each thread moves kOlaFixPer samples 256 apart.
constexpr int kOlaFixPer = 8, kOlaFixRun = 256 * kOlaFixPer;
template <class T>
__global__ void __launch_bounds__(256) k_ola_fix(KArgs<T> a, const SliceTask* __restrict__ tasks,
                                                 const C2<T>* __restrict__ W2, T* __restrict__ y) {
  const int nov = ola_count(a.N, a.Mt);
  const int runs = (nov + kOlaFixRun - 1) / kOlaFixRun;
  const int64_t task = blockIdx.x / (2 * runs);
  const int rest = (int)(blockIdx.x - task * 2 * runs);
  const bool right = rest & 1;
  const SliceTask tk = tasks[task];
  if (tk.S == 0) return;
  bool add_l, add_r;
  ola_sides(tk, a.task0 + task, a.task0, a.task1, add_l, add_r);
  if (!(right ? add_r : add_l)) return;
  const T* __restrict__ ov = reinterpret_cast<const T*>(W2 + task * a.ws2) + (right ? a.Mt : 0);
  T* __restrict__ ys = y + tk.y_base;
  const int d0 = ola_d0(a.N, a.Mt);
  const int q0 = (rest >> 1) * kOlaFixRun + (int)threadIdx.x;
  int64_t idx[kOlaFixPer];
  T v[kOlaFixPer], w[kOlaFixPer];
#pragma unroll
  for (int i = 0; i < kOlaFixPer; ++i) {
    const int q = imin(q0 + 256 * i, nov - 1);
    const int dj = d0 + q;
    int64_t t = tk.y_start + (right ? a.N + dj : a.N - dj);
    if (t >= tk.y_period) t -= tk.y_period;
    idx[i] = imin64(t, tk.y_valid - 1);
  }
#pragma unroll
  for (int i = 0; i < kOlaFixPer; ++i) {
    v[i] = ov[imin(q0 + 256 * i, nov - 1)];
    w[i] = ys[idx[i]];
  }
#pragma unroll
  for (int i = 0; i < kOlaFixPer; ++i) {
    const int q = q0 + 256 * i;
    if (q >= nov) break;
    const int dj = d0 + q;
    int64_t t = tk.y_start + (right ? a.N + dj : a.N - dj);
    if (t >= tk.y_period) t -= tk.y_period;
    if (t < tk.y_valid) ys[t] = w[i] + v[i];
  }
}

// Streaming ring traffic: block b moves descriptor b's samples from the packed
// staging buffer into the ring (to_ring) or from the ring into staging.
// R is a power of two.
template <class T>
__global__ void __launch_bounds__(256) k_ring_copy(const RingCopy* __restrict__ d, T* __restrict__ staging,
                                                   T* __restrict__ rings, int64_t R, int32_t to_ring) {
  const RingCopy c = d[blockIdx.x];
  T* ring = rings + (int64_t)c.slot * R;
  for (int i = threadIdx.x; i < c.count; i += blockDim.x) {
    const int64_t r = (c.pos + i) & (R - 1);
    if (to_ring) ring[r] = staging[c.off + i];
    else staging[c.off + i] = ring[r];
  }
}

// Zeroes `n` values starting at p.
template <class T>
__global__ void __launch_bounds__(256) k_fill_zero(T* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = T(0);
}

// Slices of one signal of T samples (L = 2N ceil(T/2N), S = L/N), m0.. m0+count-1.
__global__ void __launch_bounds__(256) k_tasks_plain(SliceTask* __restrict__ tasks, int64_t m0,
                                                     int64_t count, int64_t T, int64_t N, int64_t S) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int64_t m = m0 + i;
  const int64_t L = S * N;
  SliceTask t{};
  t.x_base = 0;
  t.x_start = m == 0 ? L - N : (m - 1) * N;
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
  tasks[i] = t;
}

// Slices of a ragged batch: signal b holds samples x_off[b] .. x_off[b+1]-1
// and its coefficients start at coef_off[b]. One block of 1024 threads scans
// the slice counts S_b = 2 ceil(T_b / 2N) of 1024 signals at a time and then
// fills that chunk's tasks in parallel (each thread finds its signal by binary
// search in the scan). Signals whose samples or coefficients fall outside the
// buffers get unused task slots and set status[0]; slots past the last task
// are marked unused; status[1] receives the number of slices.
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
  if (tid == 0) {
    carry = 0;
    bad = 0;
  }
  __syncthreads();
  for (int32_t b0 = 0; b0 < nsig; b0 += 1024) {
    const int32_t b = b0 + tid;
    int64_t Sb = 0;
    if (b < nsig) {
      int64_t Tb = x_off[b + 1] - x_off[b];
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
    const int64_t chunk = scan[1023], base = carry;
    for (int64_t i = tid; i < chunk; i += 1024) {
      const int64_t g = base + i;
      if (g >= max_tasks) {
        bad = 1;
        break;
      }
      int lo = 0, hi = 1023;                     // first s with scan[s] > i
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (scan[mid] > i) hi = mid;
        else lo = mid + 1;
      }
      const int32_t sb = b0 + lo;
      const int64_t m = i - (lo ? scan[lo - 1] : 0);
      const int64_t Tb = x_off[sb + 1] - x_off[sb];
      const int64_t S = 2 * ((Tb + 2 * N - 1) / (2 * N));
      const int64_t L = S * N;
      const bool ok = x_off[sb] >= 0 && x_off[sb + 1] <= x_len && coef_off[sb] >= 0 &&
                      coef_off[sb] + S * coefs_per_slice <= coef_len && L <= kMaxSignalElems &&
                      S * coefs_per_slice <= kMaxSignalElems;
      SliceTask t{};
      if (ok) {
        t.x_base = x_off[sb];
        t.x_start = m == 0 ? L - N : (m - 1) * N;
        t.x_period = L;
        t.x_valid = Tb;
        t.y_base = x_off[sb];
        t.y_start = t.x_start;
        t.y_period = L;
        t.y_valid = Tb;
        t.coef_base = coef_off[sb];
        t.m = (int32_t)m;
        t.S = (int32_t)S;
        t.flags = 1;
      } else {
        bad = 1;
      }
      tasks[g] = t;
    }
    __syncthreads();
    if (tid == 0) carry = base + chunk;
    __syncthreads();
  }
  for (int64_t i = carry + tid; i < max_tasks; i += 1024) {
    SliceTask t{};
    tasks[i] = t;
  }
  if (tid == 0) {
    status[0] = bad;
    status[1] = (int32_t)(carry > 0x7fffffff ? 0x7fffffff : carry);
  }
}

}  // namespace slicq
