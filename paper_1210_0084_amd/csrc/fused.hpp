// One workgroup per slice: the whole analysis (or synthesis) of a slice in a
// single kernel, for plans whose half spectrum fits in one workgroup's LDS
// (2N <= 32768 in FP32, 2N <= 8192 in FP64). Nothing but the signal and the
// coefficients crosses HBM (plus the overlap buffers of the time
// overlap-add): the slice FFT, the half spectrum and every band transform stay
// in LDS.
//
// LDS holds an index space [0, fcap) (padded as in fft_device.hpp) and two
// split twiddle tables. Indices 0..N hold the half spectrum X (analysis) or Z
// (synthesis). The plan orders the band work items and places each one's
// transform either past the spectrum or over spectrum bins that are dead:
//   analysis (Algorithm 3 with Algorithm 1 per slice), items in increasing k:
//     windowed sample pairs -> N-point FFT -> real split into X[0..N] ->
//     per item: gather X g_k at j mod M_k (Hermitian reads for the DC and
//     Nyquist bands), inverse DFT of length M_k, store c^m_k;
//     an item may overwrite bins below every bin it and later items read;
//   synthesis (Algorithm 4 with Algorithm 2 per slice), items in decreasing k:
//     per item: load c^m_k, DFT of length M_k, add dual-window-weighted values
//     into Z (the first item to reach a bin sets it) -> Hermitian packing ->
//     N-point inverse FFT -> h~_0 and overlap-add as in the pipeline;
//     an item may overwrite bins below every bin it and earlier items wrote.
// The adjoint runs the synthesis kernel with the analysis weights and h_0.
#pragma once
#include "kernels.hpp"

namespace slicq {

// Values per thread of the slice FFT of 2^LOGN points.
template <int LOGN>
constexpr int kSliceE = LOGN >= 14 ? 16 : 8;

// Global data of one thread for the first FFT pass of a fused analysis item
// (bands k0 .. k0 + cnt - 1, M >= 8: unit tid takes slots j + r M/8 of band
// k0 + sb), loaded one item ahead so that the loads overlap the current
// item's transform: spectrum index of each value (~index marks a conjugate),
// the window value as loaded, and a bit per value that holds one.
template <class T>
struct AnaPrefetch {
  int xi[8];
  T gv[8];
  int live;
};

template <class T>
__device__ __forceinline__ AnaPrefetch<T> ana_prefetch(const KArgs<T>& a, const FusedItemDev& G, int tid) {
  AnaPrefetch<T> f;
  const int lu = G.logM - 3, units = G.cnt << lu, mask = G.M - 1, N = a.N;
  const int u = imin(tid, units - 1);
  const int sb = u >> lu, j = u & ((1 << lu) - 1);
  const BandDev B = a.bands[G.k0 + sb];
  f.live = 0;
  int wi[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int t = (j + (r << lu) - B.start) & mask;
    const int jb = B.start + t;                 // signed bin, -N < jb < 2N
    const bool in = tid < units && t < B.len;
    const int jj = jb < 0 ? -jb : (jb > N ? 2 * N - jb : jb);
    f.xi[r] = (jb < 0 || jb > N) ? ~jj : jj;
    wi[r] = in ? B.goff + t : 0;
    f.live |= in ? (1 << r) : 0;
  }
#pragma unroll
  for (int r = 0; r < 8; ++r) f.gv[r] = a.g[wi[r]];
  return f;
}

// Analysis of one fused item with M = 2^LOGM: the first FFT pass takes the
// prefetched gather (M >= 8; smaller M gather here), the last one stores the
// coefficients. DIR = +1 (e^{+}). Ends with a barrier.
template <class T, int LOGM, class TW>
__device__ __forceinline__ void fused_ana_item(const KArgs<T>& a, const SliceTask& tk, const FusedItemDev& G,
                                               const AnaPrefetch<T>& pf, C2<T>* buf, C2<T>* __restrict__ cs,
                                               const TW& tws, int tid, int nthr) {
  constexpr int E = kFusedE;
  constexpr int M = 1 << LOGM, MASK = M - 1;
  constexpr int LR1 = pass_log_radix(LOGM, 0, 8), R1 = 1 << LR1, U1 = E / R1;
  constexpr int LU1 = LOGM - LR1;               // log2 first-pass units per band
  constexpr int LAST = last_pass_logns(LOGM, 8);
  const int base = G.lds, N = a.N;
  const int units1 = G.cnt << LU1;
  const int off0 = a.bands[G.k0].off;
  const int cbase = a.slice_major ? tk.m * a.cps + off0 : tk.S * off0 + tk.m * M;
  const int bstride = a.slice_major ? M : tk.S * M;   // band k0 + s starts s bstride later
  C2<T> v[U1][R1];
  if constexpr (R1 == 8) {
    // U1 = 1: unit tid, its gather prefetched with the item
    if (wave_has(tid, units1)) {
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int x = pf.xi[r];
        const C2<T> xv = buf[pidx(x < 0 ? ~x : x)];
        const T w = ((pf.live >> r) & 1) ? pf.gv[r] : T(0);
        v[0][r] = {xv.x * w, (x < 0 ? -xv.y : xv.y) * w};
      }
      dft_reg<T, 8, 1>(v[0]);
    }
  } else {
#pragma unroll
    for (int i = 0; i < U1; ++i) {
      if (!wave_has(tid + i * nthr, units1)) continue;   // idle waves skip the gather
      const int u = imin(tid + i * nthr, units1 - 1);
      const int sb = u >> LU1, j = u & ((1 << LU1) - 1);
      const BandDev B = a.bands[G.k0 + sb];
      const bool live = tid + i * nthr < units1;
      int xi[R1], wi[R1];
#pragma unroll
      for (int r = 0; r < R1; ++r) {
        const int slot = j + (r << LU1);
        const int t = (slot - B.start) & MASK;
        const int jb = B.start + t;
        const bool in = live && t < B.len;
        const int jj = jb < 0 ? -jb : (jb > N ? 2 * N - jb : jb);
        xi[r] = in ? ((jb < 0 || jb > N) ? ~jj : jj) : 0;
        wi[r] = in ? B.goff + t : -1;
      }
      T gv[R1];
#pragma unroll
      for (int r = 0; r < R1; ++r) gv[r] = a.g[imax(wi[r], 0)];
#pragma unroll
      for (int r = 0; r < R1; ++r) {
        const C2<T> xv = buf[pidx(xi[r] < 0 ? ~xi[r] : xi[r])];
        const T w = wi[r] < 0 ? T(0) : gv[r];
        v[i][r] = {xv.x * w, (xi[r] < 0 ? -xv.y : xv.y) * w};
      }
      dft_reg<T, R1, 1>(v[i]);
    }
  }
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
        const int p0 = base + (sb << LOGM) + (j << LR1);
#pragma unroll
        for (int r = 0; r < R1; ++r) buf[pidx(p0 + r)] = v[i][r];
      }
    }
    __syncthreads();
    lds_fft_c<T, 1, E, 8, LOGM, LR1, TW, LAST, true>(buf, base, G.cnt, tws, tid, nthr);
    // last pass: LDS -> registers -> coefficients
    constexpr int LRL = LOGM - LAST, RL = 1 << LRL, UL = E / RL, NS = 1 << LAST;
    constexpr int LUL = LOGM - LRL;
    const int unitsL = G.cnt << LUL;
#pragma unroll
    for (int i = 0; i < UL; ++i) {
      if (!wave_has(tid + i * nthr, unitsL)) continue;
      const int u = imin(tid + i * nthr, unitsL - 1);
      const int sb = u >> LUL, j = u & ((1 << LUL) - 1);
      const int p0 = base + (sb << LOGM) + j;
      const int pb = pidx(p0);
      C2<T> q[RL];
#pragma unroll
      for (int r = 0; r < RL; ++r) q[r] = buf[pidx_step<(1 << LUL)>(pb, p0, r)];
      C2<T> w[RL];
      pass_twiddles<T, 1, RL, NS>(tws, u & (NS - 1), w);
#pragma unroll
      for (int r = 1; r < RL; ++r) q[r] = cmul(q[r], w[r]);
      dft_reg<T, RL, 1>(q);
      if (tid + i * nthr < unitsL) {
        // LAST + LRL = LOGM: unit j < NS writes outputs n = j + r NS of its band
#pragma unroll
        for (int r = 0; r < RL; ++r) cs[cbase + sb * bstride + j + r * NS] = q[r];
      }
    }
  }
  __syncthreads();    // the next item may overwrite this item's indices
}

// Global data of one thread for a fused synthesis item, loaded one item ahead:
// the eight coefficients of its first-pass unit (M >= 8: unit tid takes
// coefficients j + r M/8 of band k0 + s) and the overlap-add records of its
// first kSynPre bins (olo + tid + q nthr; fewer in FP64, whose records and
// values take twice the registers).
template <class T>
constexpr int kSynPre = sizeof(T) == 4 ? 2 : 1;
// FP32 loads the next item's data during the current item; FP64 (the check
// path, twice the registers per value) loads each item's data at its start.
template <class T>
constexpr bool kAhead = sizeof(T) == 4;

template <class T>
struct SynPrefetch {
  C2<T> v[8];
  FOlaRec<T> rec[kSynPre<T>];
};

template <class T>
__device__ __forceinline__ SynPrefetch<T> syn_prefetch(const KArgs<T>& a, const SliceTask& tk,
                                                       const FusedItemDev& G, const C2<T>* __restrict__ cs, int tid,
                                                       int nthr) {
  SynPrefetch<T> f;
  if (G.logM >= 3) {
    const int lu = G.logM - 3, units = G.cnt << lu;
    const int u = imin(tid, units - 1);
    const int s = u >> lu, j = u & ((1 << lu) - 1);
    const int off0 = a.bands[G.k0].off;
    const int cb0 = a.slice_major ? tk.m * a.cps + off0 : tk.S * off0 + tk.m * G.M;
    const int bstride = a.slice_major ? G.M : tk.S * G.M;
#pragma unroll
    for (int r = 0; r < 8; ++r) f.v[r] = cs[cb0 + s * bstride + j + (r << lu)];
  }
#pragma unroll
  for (int q = 0; q < kSynPre<T>; ++q) f.rec[q] = a.fola[G.rec0 + imin(tid + q * nthr, G.ohi - G.olo)];
  return f;
}

// Band transforms of one fused synthesis item: DFT of length M = 2^LOGM
// (e^{-}) of bands k0 .. k0 + cnt - 1 at LDS indices lds .. lds + cnt M - 1,
// the first radix-8 pass on the prefetched coefficients. Ends with a barrier.
template <class T, int LOGM, class TW>
__device__ __forceinline__ void fused_syn_item(const KArgs<T>& a, const SliceTask& tk, const FusedItemDev& G,
                                               const SynPrefetch<T>& pf, C2<T>* buf, const C2<T>* __restrict__ cs,
                                               const TW& tws, int tid, int nthr) {
  constexpr int M = 1 << LOGM;
  const int base = G.lds;
  if constexpr (LOGM >= 3) {
    constexpr int LU = LOGM - 3;
    const int units = G.cnt << LU;
    if (wave_has(tid, units)) {
      C2<T> v[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) v[r] = pf.v[r];
      dft_reg<T, 8, -1>(v);
      if (tid < units) {
        const int s = tid >> LU, j = tid & ((1 << LU) - 1);
        const int p0 = base + (s << LOGM) + (j << 3);
#pragma unroll
        for (int r = 0; r < 8; ++r) buf[pidx(p0 + r)] = v[r];
      }
    }
    __syncthreads();
    lds_fft_c<T, -1, kFusedE, 8, LOGM, 3, TW, LOGM, true>(buf, base, G.cnt, tws, tid, nthr);
  } else {
    const int off0 = a.bands[G.k0].off;
    const int cb0 = a.slice_major ? tk.m * a.cps + off0 : tk.S * off0 + tk.m * M;
    const int bstride = a.slice_major ? M : tk.S * M;
    const int total = G.cnt << LOGM;
    for (int p = tid; p < total; p += nthr) buf[pidx(base + p)] = cs[cb0 + (p >> LOGM) * bstride + (p & (M - 1))];
    __syncthreads();
    lds_fft_c<T, -1, kFusedE, 8, LOGM, 0, TW, LOGM, true>(buf, base, G.cnt, tws, tid, nthr);
  }
}

// Frequency overlap-add of one bin j of a fused synthesis item from its record
// (rec index ri): Z[j] = (first writer ? 0 : Z[j]) + sum of the item's entries.
template <class T>
__device__ __forceinline__ void fused_ola_bin(const KArgs<T>& a, C2<T>* buf, int j, int ri, const FOlaRec<T>& rec) {
  const uint32_t y0 = rec.yy & 0xffffu, y1 = rec.yy >> 16;
  C2<T> c0 = buf[pidx(rec.xx & kFPos)], c1 = buf[pidx((rec.xx >> 16) & kFPos)];
  if (y0 != 0xffffu) c0 = cadd(c0, cconj(buf[pidx(y0)]));
  if (y1 != 0xffffu) c1 = cadd(c1, cconj(buf[pidx(y1)]));
  C2<T> acc = cadd(cscale(c0, rec.w0), cscale(c1, rec.w1));
  if (rec.xx & kFMore) {
    for (int e = a.fent_off[ri]; e < a.fent_off[ri + 1]; ++e) {
      const int2 pe = a.fent_pos[e];
      C2<T> c = buf[pidx(pe.x)];
      if (pe.y >= 0) c = cadd(c, cconj(buf[pidx(pe.y)]));
      acc = cadd(acc, cscale(c, a.fent_w[e]));
    }
  }
  if (!(rec.xx & kFInit)) acc = cadd(buf[pidx(j)], acc);
  buf[pidx(j)] = acc;
}

// Dispatches a fused item's band length 2^logM (1 <= logM <= MAXL) to BODY<L>.
#define SLICQ_FUSED_SWITCH(logM, MAXL, CALL)                                                       \
  switch (logM) {                                                                                \
    case 1: CALL(1); break;                                                                      \
    case 2: if constexpr (MAXL >= 2) CALL(2); break;                                             \
    case 3: if constexpr (MAXL >= 3) CALL(3); break;                                             \
    case 4: if constexpr (MAXL >= 4) CALL(4); break;                                             \
    case 5: if constexpr (MAXL >= 5) CALL(5); break;                                             \
    case 6: if constexpr (MAXL >= 6) CALL(6); break;                                             \
    case 7: if constexpr (MAXL >= 7) CALL(7); break;                                             \
    case 8: if constexpr (MAXL >= 8) CALL(8); break;                                             \
    case 9: if constexpr (MAXL >= 9) CALL(9); break;                                             \
    case 10: if constexpr (MAXL >= 10) CALL(10); break;                                          \
    case 11: if constexpr (MAXL >= 11) CALL(11); break;                                          \
    case 12: if constexpr (MAXL >= 12) CALL(12); break;                                          \
    default: if constexpr (MAXL >= 13) CALL(13); break;                                          \
  }

// Fused analysis: block b runs slice task b (Algorithm 3 with Algorithm 1).
// N = 2^LOGN. LDS: index space (fcap, padded) | slice twiddles | band twiddles.
template <class T, int LOGN>
__global__ void __launch_bounds__(kFusedThreads)
k_ana_fused(KArgs<T> a, const SliceTask* __restrict__ tasks, const T* __restrict__ x, C2<T>* __restrict__ coef) {
  extern __shared__ unsigned char smem[];
  C2<T>* buf = reinterpret_cast<C2<T>*>(smem);
  const SliceTask tk = tasks[blockIdx.x];
  if (tk.S == 0) return;                              // unused task slot
  constexpr int N = 1 << LOGN, ES = kSliceE<LOGN>, RS = ES >= 16 ? 16 : 8;
  constexpr int MAXL = LOGN + 1 < 13 ? LOGN + 1 : 13;  // M_k <= 2N
  const int tid = threadIdx.x, nthr = blockDim.x;
  C2<T>* twN = reinterpret_cast<C2<T>*>(smem + lds_tail_offset<T>(a.fcap));
  C2<T>* twB = twN + split_tw_entries(LOGN);
  stage_band<false>(twN, a.tw, a.tw8, LOGN, tid, nthr);
  stage_band<false>(twB, a.tw, a.tw8, a.flogM, tid, nthr);
  // windowed sample pairs z[n] = x_m[2n] h_0 + i x_m[2n+1] h_0; samples outside
  // the support of h_0 are not read (the index is clamped into it and the
  // window, zero there, drops them); the product is rounded by itself so
  // both load paths give the same values
  const int jlo = ((N - a.Mt) / 2) & ~1;
  const int jhi = (N + (N + a.Mt) / 2 - 1) & ~1;
  const T* __restrict__ xs = x + tk.x_base;
  const SliceIn si = slice_in(tk);
  const bool plain = si.even && si.start >= 0 && si.start + 2 * N <= imin(si.valid, si.period);
  C2<T> v[ES];
  if (plain) {
#pragma unroll
    for (int i = 0; i < ES; ++i) {
      const int j = 2 * imin(tid + i * nthr, N - 1);
      const C2<T> x2 = *reinterpret_cast<const C2<T>*>(xs + si.start + imin(imax(j, jlo), jhi));
      const C2<T> h2 = *reinterpret_cast<const C2<T>*>(a.h0 + j);
      v[i] = {mul_rn(x2.x, h2.x), mul_rn(x2.y, h2.y)};
    }
  } else {
#pragma unroll
    for (int i = 0; i < ES; ++i) {
      const int j = 2 * imin(tid + i * nthr, N - 1);
      const C2<T> x2 = load_sample_pair(xs, si, imin(imax(j, jlo), jhi));
      const C2<T> h2 = *reinterpret_cast<const C2<T>*>(a.h0 + j);
      v[i] = {mul_rn(x2.x, h2.x), mul_rn(x2.y, h2.y)};
    }
  }
#pragma unroll
  for (int i = 0; i < ES; ++i)
    if (tid + i * nthr < N) buf[pidx(tid + i * nthr)] = v[i];
  __syncthreads();
  lds_fft_c<T, -1, ES, RS, LOGN, 0, TwBand<T, false>, LOGN, true>(buf, 0, 1, band_tw<false>(twN, LOGN), tid, nthr);
  // real split: X[k], X[N - k] from the packed pair (k, N - k); X[N] at index N
  for (int k = tid; k <= N / 2; k += nthr) {
    const C2<T> za = buf[pidx(k)], zb = buf[pidx((N - k) & (N - 1))];
    C2<T> xk, xnk;
    real_split(za, zb, twiddle<T, -1>(a.tw, 2 * N, k), a.scale, xk, xnk);
    buf[pidx(k)] = xk;
    if (k == 0) buf[pidx(N)] = xnk;
    else if (2 * k != N) buf[pidx(N - k)] = xnk;
  }
  __syncthreads();
  C2<T>* __restrict__ cs = coef + tk.coef_base;
  const TwBand<T, false> tb = band_tw<false>(twB, a.flogM);
  // each item's global gather data is loaded while the previous item transforms
  FusedItemDev Gn = a.fana[0];
  AnaPrefetch<T> pn{};
  if constexpr (kAhead<T>) {
    if (Gn.logM >= 3) pn = ana_prefetch(a, Gn, tid);
  }
  for (int it = 0; it < a.nfana; ++it) {
    const FusedItemDev G = Gn;
    AnaPrefetch<T> pf{};
    if constexpr (kAhead<T>) {
      pf = pn;
      if (it + 1 < a.nfana) {
        Gn = a.fana[it + 1];
        if (Gn.logM >= 3) pn = ana_prefetch(a, Gn, tid);
      }
    } else {
      if (G.logM >= 3) pf = ana_prefetch(a, G, tid);
      if (it + 1 < a.nfana) Gn = a.fana[it + 1];
    }
    // an opaque copy of the thread index keeps each length's address
    // arithmetic inside the loop (registers)
    int t = tid;
    asm volatile("" : "+v"(t));
#define SLICQ_FA(L) fused_ana_item<T, L>(a, tk, G, pf, buf, cs, tb, t, nthr)
    SLICQ_FUSED_SWITCH(G.logM, MAXL, SLICQ_FA)
#undef SLICQ_FA
  }
}

// Fused synthesis (or adjoint): block b runs slice task b (Algorithm 4 with
// Algorithm 2), then the same time overlap-add as inverse pass B (the second
// contribution of a shared sample goes to the task's overlap buffer for
// k_ola_fix).
template <class T, int LOGN>
__global__ void __launch_bounds__(kFusedThreads)
k_syn_fused(KArgs<T> a, const SliceTask* __restrict__ tasks, const C2<T>* __restrict__ coef, C2<T>* __restrict__ W2,
            T* __restrict__ y) {
  extern __shared__ unsigned char smem[];
  C2<T>* buf = reinterpret_cast<C2<T>*>(smem);
  const int task = blockIdx.x;
  const SliceTask tk = tasks[task];
  if (tk.S == 0) return;
  constexpr int N = 1 << LOGN, ES = kSliceE<LOGN>, RS = ES >= 16 ? 16 : 8;
  constexpr int MAXL = LOGN + 1 < 13 ? LOGN + 1 : 13;
  const int tid = threadIdx.x, nthr = blockDim.x;
  C2<T>* twN = reinterpret_cast<C2<T>*>(smem + lds_tail_offset<T>(a.fcap));
  C2<T>* twB = twN + split_tw_entries(LOGN);
  stage_band<false>(twN, a.tw, a.tw8, LOGN, tid, nthr);
  stage_band<false>(twB, a.tw, a.tw8, a.flogM, tid, nthr);
  __syncthreads();
  const C2<T>* __restrict__ cs = coef + tk.coef_base;
  const TwBand<T, false> tb = band_tw<false>(twB, a.flogM);
  // each item's coefficients and first overlap-add records are loaded while
  // the previous item transforms
  FusedItemDev Gn = a.fsyn[0];
  SynPrefetch<T> pn;
  if constexpr (kAhead<T>) pn = syn_prefetch(a, tk, Gn, cs, tid, nthr);
  for (int it = 0; it < a.nfsyn; ++it) {
    const FusedItemDev G = Gn;
    SynPrefetch<T> pf;
    if constexpr (kAhead<T>) {
      pf = pn;
      if (it + 1 < a.nfsyn) {
        Gn = a.fsyn[it + 1];
        pn = syn_prefetch(a, tk, Gn, cs, tid, nthr);
      }
    } else {
      pf = syn_prefetch(a, tk, G, cs, tid, nthr);
      if (it + 1 < a.nfsyn) Gn = a.fsyn[it + 1];
    }
    int t = tid;
    asm volatile("" : "+v"(t));
#define SLICQ_FS(L) fused_syn_item<T, L>(a, tk, G, pf, buf, cs, tb, t, nthr)
    SLICQ_FUSED_SWITCH(G.logM, MAXL, SLICQ_FS)
#undef SLICQ_FS
    // frequency overlap-add of this item's bands into Z[olo..ohi]
    const int nbin = G.ohi - G.olo + 1;
#pragma unroll
    for (int q = 0; q < kSynPre<T>; ++q) {
      const int d = tid + q * nthr;
      if (d < nbin) fused_ola_bin(a, buf, G.olo + d, G.rec0 + d, pf.rec[q]);
    }
    for (int d = tid + kSynPre<T> * nthr; d < nbin; d += nthr)
      fused_ola_bin(a, buf, G.olo + d, G.rec0 + d, a.fola[G.rec0 + d]);
    __syncthreads();
  }
  // Hermitian packing of Z[0..N] into the N-point spectrum of y[2n] + i y[2n+1]
  for (int k = tid; k <= N / 2; k += nthr) {
    const C2<T> za = buf[pidx(k)], zb = buf[pidx(N - k)];
    C2<T> zk, znk;
    herm_pack(za, zb, twiddle<T, 1>(a.tw, 2 * N, k), zk, znk);
    buf[pidx(k)] = zk;
    if (k != 0 && 2 * k != N) buf[pidx(N - k)] = znk;
  }
  __syncthreads();
  lds_fft_c<T, 1, ES, RS, LOGN, 0, TwBand<T, false>, LOGN, true>(buf, 0, 1, band_tw<false>(twN, LOGN), tid, nthr);
  // scale, synthesis window, overlap-add
  T* __restrict__ ys = y + tk.y_base;
  T* __restrict__ ov = reinterpret_cast<T*>(W2 + (int64_t)task * a.ws2);
  bool add_l, add_r;
  ola_sides(tk, a.task0 + task, a.task0, a.task1, add_l, add_r);
  const int ys0 = (int)tk.y_start, yper = (int)tk.y_period, yval = (int)tk.y_valid;
  C2<T> h[ES];
#pragma unroll
  for (int i = 0; i < ES; ++i) h[i] = *reinterpret_cast<const C2<T>*>(a.hsyn + 2 * imin(tid + i * nthr, N - 1));
#pragma unroll
  for (int i = 0; i < ES; ++i) {
    const int n = tid + i * nthr;
    if (n < N) {
      const C2<T> z = buf[pidx(n)];
      ola_store(ys, ov, ys0, yper, yval, 2 * n, z.x * a.scale * h[i].x, N, a.Mt, add_l, add_r);
      ola_store(ys, ov, ys0, yper, yval, 2 * n + 1, z.y * a.scale * h[i].y, N, a.Mt, add_l, add_r);
    }
  }
}

}  // namespace slicq
