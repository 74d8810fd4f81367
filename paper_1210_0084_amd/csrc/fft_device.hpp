// Device building blocks for the sliCQ kernels on gfx950: complex values,
// radix-2/4/8/16 DFTs in registers, and batched power-of-two FFTs in LDS
// (Stockham autosort, in place, every thread holding at most E values).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"

namespace slicq {

template <class T>
struct alignas(2 * sizeof(T)) C2 {
  T x, y;
};

template <class T>
__device__ __forceinline__ C2<T> cadd(C2<T> a, C2<T> b) { return {a.x + b.x, a.y + b.y}; }
template <class T>
__device__ __forceinline__ C2<T> csub(C2<T> a, C2<T> b) { return {a.x - b.x, a.y - b.y}; }
template <class T>
__device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <class T>
__device__ __forceinline__ C2<T> cconj(C2<T> a) { return {a.x, -a.y}; }
// a * b rounded by itself: the compiler cannot contract it into a following
// add, so the value does not depend on how the surrounding code is compiled.
template <class T>
__device__ __forceinline__ T mul_rn(T a, T b) {
  if constexpr (sizeof(T) == 4) return __builtin_fmaf(a, b, 0.0f);
  else return __builtin_fma(a, b, 0.0);
}
template <class T>
__device__ __forceinline__ C2<T> cscale(C2<T> a, T s) { return {a.x * s, a.y * s}; }
// multiply by -i (forward) or +i (inverse)
template <class T, int DIR>
__device__ __forceinline__ C2<T> mul_mi(C2<T> a) {
  if constexpr (DIR < 0) return {a.y, -a.x};
  else return {-a.y, a.x};
}

__device__ __forceinline__ int imin(int a, int b) { return a < b ? a : b; }
__device__ __forceinline__ int64_t imin64(int64_t a, int64_t b) { return a < b ? a : b; }
__device__ __forceinline__ int imax(int a, int b) { return a > b ? a : b; }

// LDS index with one pad slot every 2^kPadShift complex values (kPadShift
// and padded() in common.hpp).
__device__ __forceinline__ int pidx(int i) { return i + (i >> kPadShift); }

// Lanes per wavefront (CDNA): blocks are one-dimensional, so the lanes of a
// wave are threads (tid & ~(kWave - 1)) .. + kWave - 1.
constexpr int kWave = 64;

// True for every lane of a wave that holds at least one index below n:
// lets a whole idle wave branch around work it would only repeat (clamped).
// The wave base is read from the first lane, so the test is a scalar branch.
__device__ __forceinline__ bool wave_has(int tid, int n) {
  return __builtin_amdgcn_readfirstlane(tid & ~(kWave - 1)) < n;
}

// e^{DIR 2 pi i k / R} for small constant R, as constants.
template <class T, int R, int DIR>
__device__ __forceinline__ C2<T> wconst(int k) {
  // cos(2 pi k / 16) for k = 0..4
  constexpr double c16[5] = {1.0, 0.92387953251128675613, 0.70710678118654752440,
                             0.38268343236508977173, 0.0};
  int q = k * (16 / R);            // angle in sixteenths of a turn, q in [0, 16)
  // cos and sin of 2 pi q / 16
  int qc = q & 15;
  double c, s;
  int m = qc & 3, quad = qc >> 2;
  double cc = c16[m], ss = c16[4 - m];
  switch (quad) {
    case 0: c = cc; s = ss; break;
    case 1: c = -ss; s = cc; break;
    case 2: c = -cc; s = -ss; break;
    default: c = ss; s = -cc; break;
  }
  return {(T)c, (T)(DIR < 0 ? -s : s)};
}

// In-register DFT of size R (power of two <= 16), natural order in and out.
// DIR < 0: e^{-2 pi i jk/R} (forward), DIR > 0: e^{+} (inverse), unnormalised.
template <class T, int R, int DIR>
__device__ __forceinline__ void dft_reg(C2<T>* v) {
  // radix-2 decimation in frequency, output in bit-reversed order
#pragma unroll
  for (int span = R / 2; span >= 1; span >>= 1) {
#pragma unroll
    for (int b = 0; b < R; b += 2 * span) {
#pragma unroll
      for (int q = 0; q < span; ++q) {
        C2<T> a = v[b + q], c = v[b + q + span];
        v[b + q] = cadd(a, c);
        C2<T> d = csub(a, c);
        // twiddle e^{DIR 2 pi i q / (2 span)} = w_R^{q R / (2 span)}
        const int e = q * (R / (2 * span));
        if (e == 0) {
          v[b + q + span] = d;
        } else if (4 * e == R) {
          v[b + q + span] = mul_mi<T, DIR>(d);    // e^{DIR i pi/2}: -i forward, +i inverse
        } else {
          v[b + q + span] = cmul(d, wconst<T, R, DIR>(e));
        }
      }
    }
  }
  // undo the bit reversal (register renaming once unrolled)
  C2<T> t[R];
#pragma unroll
  for (int i = 0; i < R; ++i) t[i] = v[i];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    int r = 0;
#pragma unroll
    for (int bit = 1, rb = R / 2; bit < R; bit <<= 1, rb >>= 1)
      if (i & bit) r |= rb;
    v[r] = t[i];
  }
}

// Twiddle e^{DIR 2 pi i k / n} from the pyramid (entry n + k holds e^{-2 pi i k / n}).
template <class T, int DIR>
__device__ __forceinline__ C2<T> twiddle(const C2<T>* __restrict__ tw, int n, int k) {
  C2<T> w = tw[(unsigned)(n + k)];
  if constexpr (DIR > 0) w.y = -w.y;
  return w;
}

// Twiddle sources for the LDS FFT; get(n, k) returns e^{-2 pi i k / n} for
// 0 <= k < n/2. TwGlobal reads the pyramid in global memory; TwLds reads the
// lower halves of its levels 2, 4, ..., n_max staged in LDS, level n at
// entries n/2 - 1 .. n - 2 (n_max - 1 entries in all, contiguous per level).
template <class T>
struct TwGlobal {
  const C2<T>* __restrict__ tw;
  __device__ __forceinline__ C2<T> get(int n, int k) const { return tw[(unsigned)(n + k)]; }
};

template <class T>
struct TwLds {
  const C2<T>* tw;
  __device__ __forceinline__ C2<T> get(int n, int k) const { return tw[(n >> 1) - 1 + k]; }
};

// Twiddles of the band FFTs, from small LDS tables. get(n, k) gives
// e^{-2 pi i k / n} for n = 2^l <= 2^L as a product: with
// m = k 2^(L - l) = hi 2^(L/2) + lo, it is e^{-2 pi i hi / 2^(L - L/2)} (t[hi])
// times e^{-2 pi i lo / 2^L} (t[2^(L - L/2) + lo]). That needs 2^(L - L/2) +
// 2^(L/2) entries instead of every level up to 2^L, with the error of one
// more rounding.
// With P8, the radix-8 passes at Ns = 8 and Ns = 64 read their seven powers
// directly instead (pow8): row r = 1..7 of pass Ns holds
// e^{-2 pi i r k / (8 Ns)}, for k < Ns, contiguous in k (p8: the Ns = 8 rows,
// then the Ns = 64 rows). That saves the index arithmetic and products, and
// costs kPow8Entries more entries to stage.
template <class T, bool P8>
struct TwBand {
  const C2<T>* t;
  int L;
  const C2<T>* p8;
  static constexpr bool kPow8 = P8;
  __device__ __forceinline__ C2<T> get(int n, int k) const {
    const int LL = L >> 1;
    const int m = k << (L - (31 - __builtin_clz((unsigned)n)));
    return cmul(t[m >> LL], t[(1 << (L - LL)) + (m & ((1 << LL) - 1))]);
  }
  template <int DIR, int NS>
  __device__ __forceinline__ void pow8(int k, C2<T>* w) const {
    const C2<T>* row = p8 + (NS == 8 ? 0 : 7 * 8) + k;
#pragma unroll
    for (int r = 1; r < 8; ++r) {
      w[r] = row[(r - 1) * NS];
      if constexpr (DIR > 0) w[r].y = -w[r].y;
    }
  }
};

// Entries of the TwBand tables for transforms up to 2^L (the split tables,
// then, with P8, the radix-8 rows).
__host__ __device__ constexpr int band_tw_entries(int L, bool p8) {
  return split_tw_entries(L) + (p8 ? kPow8Entries : 0);
}

// Four-step twiddles e^{DIR 2 pi i m / N}, 0 <= m < N = N1 N2, as the product
// of e^{-2 pi i (m >> log N2) / N1} (hi, N1 entries) and e^{-2 pi i (m mod N2) / N}
// (lo, N2 entries), both staged in LDS: two small tables instead of gathers
// from the N-entry level of the pyramid (error within one more rounding).
template <class T>
struct InterTw {
  const C2<T>* hi;
  const C2<T>* lo;
  int logN2;
  template <int DIR>
  __device__ __forceinline__ C2<T> get(int m) const {
    C2<T> w = cmul(hi[m >> logN2], lo[m & ((1 << logN2) - 1)]);
    if constexpr (DIR > 0) w.y = -w.y;
    return w;
  }
};

// Entry i of the TwLds table for levels up to n_max: level n = 2^(floor(log2(i + 1)) + 1),
// k = i + 1 - n/2, read from the pyramid.
template <class T>
__device__ __forceinline__ C2<T> tw_stage_value(const C2<T>* __restrict__ tw, int i) {
  const int n = 2 << (31 - __builtin_clz((unsigned)(i + 1)));
  return tw[(unsigned)(n + i + 1 - (n >> 1))];
}

// Powers w^r, r = 1..R-1, of w = e^{DIR 2 pi i k / n}, k < n / R: w^1, w^2,
// w^4, w^8 are read (w^r = e^{-2 pi i k / (n/r)}, contiguous in k within a
// level), every other power is a product of at most three of them.
template <class T, int DIR, int R, class TW>
__device__ __forceinline__ void twiddle_powers(const TW& src, int n, int k, C2<T>* w) {
  auto rd = [&](int m) {
    C2<T> v = src.get(m, k);
    if constexpr (DIR > 0) v.y = -v.y;
    return v;
  };
  w[1] = rd(n);
  if constexpr (R > 2) {
    w[2] = rd(n >> 1);
    w[3] = cmul(w[1], w[2]);
  }
  if constexpr (R > 4) {
    w[4] = rd(n >> 2);
    w[5] = cmul(w[4], w[1]);
    w[6] = cmul(w[4], w[2]);
    w[7] = cmul(w[4], w[3]);
  }
  if constexpr (R > 8) {
    w[8] = rd(n >> 3);
#pragma unroll
    for (int r = 9; r < 16; ++r) w[r] = cmul(w[8], w[r - 8]);
  }
}

// Twiddles w^1 .. w^(R-1) of a pass at Ns = NS (w = e^{DIR 2 pi i k / (NS R)}):
// the direct radix-8 rows where the source has them, else twiddle_powers.
template <class TW, class = void>
struct HasPow8 {
  static constexpr bool value = false;
};
template <class TW>
struct HasPow8<TW, decltype((void)TW::kPow8)> {
  static constexpr bool value = TW::kPow8;
};

template <class T, int DIR, int R, int NS, class TW>
__device__ __forceinline__ void pass_twiddles(const TW& src, int k, C2<T>* w) {
  if constexpr (R == 8 && (NS == 8 || NS == 64) && HasPow8<TW>::value) src.template pow8<DIR, NS>(k, w);
  else twiddle_powers<T, DIR, R>(src, NS * R, k, w);
}

// Batch layouts of `nseq` sequences of length n in LDS (padded indices):
// CONTIG puts element i of sequence s at s*n + i, INTERLEAVED at i*nseq + s.
enum Layout { CONTIG = 0, INTERLEAVED = 1 };

// One in-place Stockham pass of radix R. Ns is the product of the radices of
// earlier passes. Every thread reads all of its units into registers, the
// block synchronises, then every thread writes back.
template <class T, int DIR, int R, int LAY, int E, class TW>
__device__ __forceinline__ void stockham_pass(C2<T>* buf, int base, int logn, int Ns, int logNs,
                                              int nseq, int lognseq, const TW& tws,
                                              int tid, int nthr) {
  constexpr int U = E / R;
  constexpr int LR = (R == 2) ? 1 : (R == 4) ? 2 : (R == 8) ? 3 : 4;
  C2<T> v[U][R];
  const int lunits = logn - LR;            // log2 of units per sequence
  const int total = (LAY == CONTIG) ? (nseq << lunits) : (1 << (lognseq + lunits));
  // Threads past the last unit repeat it (no branch around the reads, so the
  // reads of all units are in flight together); only real units write back.
#pragma unroll
  for (int i = 0; i < U; ++i) {
    const int u = imin(tid + i * nthr, total - 1);
    int s, j;
    if constexpr (LAY == CONTIG) { s = u >> lunits; j = u & ((1 << lunits) - 1); }
    else { s = u & ((1 << lognseq) - 1); j = u >> lognseq; }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int e = j + (r << lunits);
      const int pos = (LAY == CONTIG) ? (s << logn) + e : (e << lognseq) + s;
      v[i][r] = buf[pidx(base + pos)];
    }
  }
#pragma unroll
  for (int i = 0; i < U; ++i) {
    if (Ns > 1) {
      const int u = imin(tid + i * nthr, total - 1);
      const int j = (LAY == CONTIG) ? (u & ((1 << lunits) - 1)) : (u >> lognseq);
      C2<T> w[R];
      twiddle_powers<T, DIR, R>(tws, Ns * R, j & (Ns - 1), w);
#pragma unroll
      for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], w[r]);
    }
    dft_reg<T, R, DIR>(v[i]);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < U; ++i) {
    const int u = tid + i * nthr;
    if (u < total) {
      int s, j;
      if constexpr (LAY == CONTIG) { s = u >> lunits; j = u & ((1 << lunits) - 1); }
      else { s = u & ((1 << lognseq) - 1); j = u >> lognseq; }
      const int idxD = ((j >> logNs) << (logNs + LR)) + (j & (Ns - 1));
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int e = idxD + r * Ns;
        const int pos = (LAY == CONTIG) ? (s << logn) + e : (e << lognseq) + s;
        buf[pidx(base + pos)] = v[i][r];
      }
    }
  }
  __syncthreads();
}

// Batched FFT of `nseq` sequences of length 2^logn held in LDS at padded
// positions pidx(base + pos); INTERLEAVED needs nseq = 2^lognseq. Needs
// nseq * n <= E * nthr. Passes have radix at most RMAX (each thread holds E
// values, E / R butterflies of radix R). Unnormalised, DIR < 0 forward (e^-), DIR > 0
// inverse (e^+). The caller synchronises the data in; the routine ends with a
// barrier.
template <class T, int DIR, int LAY, int E = 16, int RMAX = (E < 16 ? E : 16), class TW>
__device__ __forceinline__ void lds_fft(C2<T>* buf, int base, int logn, int nseq, int lognseq,
                        const TW& tw, int tid, int nthr) {
  static_assert(E >= 2 && (E & (E - 1)) == 0, "E must be a power of two");
  static_assert(RMAX >= 2 && RMAX <= E && RMAX <= 16, "largest radix must fit E");
  int Ns = 1, logNs = 0, rem = logn;
  while (rem > 0) {
    if constexpr (RMAX >= 16) {
      if (rem >= 4) {
        stockham_pass<T, DIR, 16, LAY, E, TW>(buf, base, logn, Ns, logNs, nseq, lognseq, tw, tid, nthr);
        Ns <<= 4; logNs += 4; rem -= 4;
        continue;
      }
    }
    if constexpr (RMAX >= 8) {
      if (rem >= 3) {
        stockham_pass<T, DIR, 8, LAY, E, TW>(buf, base, logn, Ns, logNs, nseq, lognseq, tw, tid, nthr);
        Ns <<= 3; logNs += 3; rem -= 3;
        continue;
      }
    }
    if (RMAX >= 4 && rem >= 2) {
      stockham_pass<T, DIR, (RMAX >= 4 ? 4 : 2), LAY, E, TW>(buf, base, logn, Ns, logNs, nseq, lognseq, tw, tid, nthr);
      Ns <<= 2; logNs += 2; rem -= 2;
    } else {
      stockham_pass<T, DIR, 2, LAY, E, TW>(buf, base, logn, Ns, logNs, nseq, lognseq, tw, tid, nthr);
      Ns <<= 1; logNs += 1; rem -= 1;
    }
  }
}

// ---------------------------------------------------------------------------
// The same Stockham FFT for the CONTIG layout with the length fixed at compile
// time (n = 2^LOGN): every stride is a constant, so the padded LDS addresses of
// a butterfly are one computed base plus immediate offsets.

// Padded position of base + r * S for a constant stride S: for S a multiple of
// the pad run the pad count grows by S >> kPadShift per step.
template <int S>
__device__ __forceinline__ int pidx_step(int pb, int p0, int r) {
  if constexpr (S % (1 << kPadShift) == 0) {
    return pb + r * (S + (S >> kPadShift));
  } else if constexpr (S == (1 << kPadShift) / 2) {
    // half a pad run: the pad count grows by (r + c) / 2 with c the bit of p0
    // below the run length, so even r sit at constant offsets from pb and odd
    // r at constant offsets from pb + c
    return pb + r * S + (r >> 1) + ((r & 1) ? ((p0 >> (kPadShift - 1)) & 1) : 0);
  } else {
    return pidx(p0 + r * S);
  }
}

// SKIP: waves without a unit branch around the reads and the arithmetic (for
// callers whose batches leave whole waves idle; it costs a few instructions).
template <class T, int DIR, int R, int E, int LOGN, int LOGNS, class TW, bool SKIP = false>
__device__ __forceinline__ void stockham_pass_c(C2<T>* buf, int base, int nseq, const TW& tws, int tid, int nthr) {
  constexpr int U = E / R;
  constexpr int LR = (R == 2) ? 1 : (R == 4) ? 2 : (R == 8) ? 3 : 4;
  constexpr int LUNITS = LOGN - LR;           // log2 of units per sequence
  constexpr int NS = 1 << LOGNS;
  constexpr int SREAD = 1 << LUNITS;          // read stride of a unit's values
  const int total = nseq << LUNITS;
  C2<T> v[U][R];
  if (!SKIP || wave_has(tid, total)) {
#pragma unroll
    for (int i = 0; i < U; ++i) {
      const int u = imin(tid + i * nthr, total - 1);
      const int s = u >> LUNITS, j = u & (SREAD - 1);
      const int p0 = base + (s << LOGN) + j;
      const int pb = pidx(p0);
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = buf[pidx_step<SREAD>(pb, p0, r)];
    }
    // a thread's units lie nthr apart: with nthr a multiple of NS they share
    // the twiddle index, so the powers are computed once (lanes past the end
    // are clamped and never written back)
    const bool share = U > 1 && (nthr & (NS - 1)) == 0;
    C2<T> w0[R];
#pragma unroll
    for (int i = 0; i < U; ++i) {
      if constexpr (NS > 1) {
        C2<T> w[R];
        if (i > 0 && share) {
#pragma unroll
          for (int r = 1; r < R; ++r) w[r] = w0[r];
        } else {
          const int u = imin(tid + i * nthr, total - 1);
          pass_twiddles<T, DIR, R, NS>(tws, u & (NS - 1), w);
          if (i == 0) {
#pragma unroll
            for (int r = 1; r < R; ++r) w0[r] = w[r];
          }
        }
#pragma unroll
        for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], w[r]);
      }
      dft_reg<T, R, DIR>(v[i]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < U; ++i) {
    const int u = tid + i * nthr;
    if (u < total) {
      const int s = u >> LUNITS, j = u & (SREAD - 1);
      const int p0 = base + (s << LOGN) + ((j >> LOGNS) << (LOGNS + LR)) + (j & (NS - 1));
      const int pb = pidx(p0);
#pragma unroll
      for (int r = 0; r < R; ++r) buf[pidx_step<NS>(pb, p0, r)] = v[i][r];
    }
  }
  __syncthreads();
}

// log2 of the radix of the pass that starts at Ns = 2^logns (greedy, largest first).
__host__ __device__ constexpr int pass_log_radix(int logn, int logns, int rmax) {
  return (rmax >= 16 && logn - logns >= 4) ? 4 : (rmax >= 8 && logn - logns >= 3) ? 3
         : (rmax >= 4 && logn - logns >= 2) ? 2 : 1;
}

// log2 Ns of the last pass of a length-2^logn FFT.
__host__ __device__ constexpr int last_pass_logns(int logn, int rmax) {
  int ns = 0;
  while (ns + pass_log_radix(logn, ns, rmax) < logn) ns += pass_log_radix(logn, ns, rmax);
  return ns;
}

// Passes of the CONTIG FFT from Ns = 2^LOGNS while Ns < 2^STOP (the whole
// transform with the defaults).
template <class T, int DIR, int E, int RMAX, int LOGN, int LOGNS, class TW, int STOP = LOGN, bool SKIP = false>
__device__ __forceinline__ void lds_fft_c(C2<T>* buf, int base, int nseq, const TW& tw, int tid, int nthr) {
  if constexpr (LOGNS < LOGN && LOGNS < STOP) {
    constexpr int REM = LOGN - LOGNS;
    constexpr int LR = (RMAX >= 16 && REM >= 4) ? 4 : (RMAX >= 8 && REM >= 3) ? 3 : (RMAX >= 4 && REM >= 2) ? 2 : 1;
    stockham_pass_c<T, DIR, (1 << LR), E, LOGN, LOGNS, TW, SKIP>(buf, base, nseq, tw, tid, nthr);
    lds_fft_c<T, DIR, E, RMAX, LOGN, LOGNS + LR, TW, STOP, SKIP>(buf, base, nseq, tw, tid, nthr);
  }
}

// INTERLEAVED layout with the length fixed at compile time: element e of
// sequence s at e * nseq + s (nseq = 2^lognseq at run time). Strides that are
// multiples of the pad run use one base plus offsets.
__device__ __forceinline__ int pidx_run(int pb, int p0, int r, int S) {
  return (S & ((1 << kPadShift) - 1)) == 0 ? pb + r * (S + (S >> kPadShift)) : pidx(p0 + r * S);
}

template <class T, int DIR, int R, int E, int LOGN, int LOGNS, class TW>
__device__ __forceinline__ void stockham_pass_ci(C2<T>* buf, int lognseq, const TW& tws, int tid, int nthr) {
  constexpr int U = E / R;
  constexpr int LR = (R == 2) ? 1 : (R == 4) ? 2 : (R == 8) ? 3 : 4;
  constexpr int LUNITS = LOGN - LR;
  constexpr int NS = 1 << LOGNS;
  const int total = 1 << (lognseq + LUNITS);
  const int sread = 1 << (LUNITS + lognseq), swrite = NS << lognseq;
  const int smask = (1 << lognseq) - 1;
  C2<T> v[U][R];
#pragma unroll
  for (int i = 0; i < U; ++i) {
    const int u = imin(tid + i * nthr, total - 1);
    const int s = u & smask, j = u >> lognseq;
    const int p0 = (j << lognseq) + s;
    const int pb = pidx(p0);
#pragma unroll
    for (int r = 0; r < R; ++r) v[i][r] = buf[pidx_run(pb, p0, r, sread)];
  }
#pragma unroll
  for (int i = 0; i < U; ++i) {
    if constexpr (NS > 1) {
      const int u = imin(tid + i * nthr, total - 1);
      C2<T> w[R];
      twiddle_powers<T, DIR, R>(tws, NS * R, (u >> lognseq) & (NS - 1), w);
#pragma unroll
      for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], w[r]);
    }
    dft_reg<T, R, DIR>(v[i]);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < U; ++i) {
    const int u = tid + i * nthr;
    if (u < total) {
      const int s = u & smask, j = u >> lognseq;
      const int e0 = ((j >> LOGNS) << (LOGNS + LR)) + (j & (NS - 1));
      const int p0 = (e0 << lognseq) + s;
      const int pb = pidx(p0);
#pragma unroll
      for (int r = 0; r < R; ++r) buf[pidx_run(pb, p0, r, swrite)] = v[i][r];
    }
  }
  __syncthreads();
}

template <class T, int DIR, int E, int RMAX, int LOGN, int LOGNS, class TW, int STOP = LOGN>
__device__ __forceinline__ void lds_fft_ci(C2<T>* buf, int lognseq, const TW& tw, int tid, int nthr) {
  if constexpr (LOGNS < LOGN && LOGNS < STOP) {
    constexpr int REM = LOGN - LOGNS;
    constexpr int LR = (RMAX >= 16 && REM >= 4) ? 4 : (RMAX >= 8 && REM >= 3) ? 3 : (RMAX >= 4 && REM >= 2) ? 2 : 1;
    stockham_pass_ci<T, DIR, (1 << LR), E, LOGN, LOGNS, TW>(buf, lognseq, tw, tid, nthr);
    lds_fft_ci<T, DIR, E, RMAX, LOGN, LOGNS + LR, TW, STOP>(buf, lognseq, tw, tid, nthr);
  }
}

// Unit u of a pass with 2^logj units per sequence over 2^lognseq sequences:
// sequence-fastest (s = u mod 2^lognseq) or, with JF, unit-fastest
// (j = u mod 2^logj), which makes global accesses of one sequence coalesce.
template <bool JF>
__device__ __forceinline__ void ci_unit(int u, int lognseq, int logj, int& s, int& j) {
  if constexpr (JF) { j = u & ((1 << logj) - 1); s = u >> logj; }
  else { s = u & ((1 << lognseq) - 1); j = u >> lognseq; }
}

// FFT of length 2^LOGN over 2^lognseq sequences (INTERLEAVED in LDS between
// passes, radix <= 8) whose first pass takes its inputs from load(s, e)
// (element e of sequence s) and whose last pass gives its outputs to
// store(i, r, s, e, value) instead of LDS: FIRST and LAST select which of the
// two are fused (an unfused first pass reads LDS, an unfused last pass writes
// LDS). Output e of the last pass is held by unit u = tid + i nthr with
// (s, j) = ci_unit<JF>(u, lognseq, L), e = j + r 2^L, L = last_pass_logns,
// so a caller can fetch per-output data before the transform. JF orders the
// fused passes' units unit-fastest (coalesced when a sequence is contiguous
// in global memory). The caller synchronises after an unfused last pass; a
// fused first pass needs no synchronisation before it; LDS the block wrote
// before the call is visible to store (there is a barrier before it).
template <class T, int DIR, int E, int LOGN, bool FIRST, bool LASTF, bool JF, class TW, class LD, class ST>
__device__ __forceinline__ void fft_ci_fused(C2<T>* buf, int lognseq, const TW& tw, int tid, int nthr, LD load,
                                             ST store) {
  constexpr int LR1 = pass_log_radix(LOGN, 0, 8), R1 = 1 << LR1, U1 = E / R1;
  constexpr int LAST = last_pass_logns(LOGN, 8);
  if constexpr (FIRST) {
    const int units = 1 << (lognseq + LOGN - LR1);
    C2<T> v[U1][R1];
#pragma unroll
    for (int i = 0; i < U1; ++i) {
      int s, j;
      ci_unit<JF>(imin(tid + i * nthr, units - 1), lognseq, LOGN - LR1, s, j);
#pragma unroll
      for (int r = 0; r < R1; ++r) v[i][r] = load(s, j + (r << (LOGN - LR1)));
    }
#pragma unroll
    for (int i = 0; i < U1; ++i) dft_reg<T, R1, DIR>(v[i]);
    if constexpr (LASTF && LAST == 0) {
      __syncthreads();                  // a store may read LDS tables the block staged before the call
#pragma unroll
      for (int i = 0; i < U1; ++i) {
        const int u = tid + i * nthr;
        if (u < units) {
          int s, j;
          ci_unit<JF>(u, lognseq, 0, s, j);
#pragma unroll
          for (int r = 0; r < R1; ++r) store(i, r, s, j + r, v[i][r]);
        }
      }
      return;
    }
#pragma unroll
    for (int i = 0; i < U1; ++i) {
      const int u = tid + i * nthr;
      if (u < units) {
        int s, j;
        ci_unit<JF>(u, lognseq, LOGN - LR1, s, j);
        const int p0 = ((j << LR1) << lognseq) + s;
#pragma unroll
        for (int r = 0; r < R1; ++r) buf[pidx(p0 + (r << lognseq))] = v[i][r];
      }
    }
    __syncthreads();
  }
  if constexpr (LASTF) {
    if constexpr (FIRST) lds_fft_ci<T, DIR, E, 8, LOGN, LR1, TW, LAST>(buf, lognseq, tw, tid, nthr);
    else lds_fft_ci<T, DIR, E, 8, LOGN, 0, TW, LAST>(buf, lognseq, tw, tid, nthr);
    constexpr int LRL = LOGN - LAST, RL = 1 << LRL, UL = E / RL, NS = 1 << LAST;
    const int units = 1 << (lognseq + LAST);
    C2<T> q[UL][RL];
#pragma unroll
    for (int i = 0; i < UL; ++i) {
      int s, j;
      ci_unit<JF>(imin(tid + i * nthr, units - 1), lognseq, LAST, s, j);
      const int p0 = (j << lognseq) + s;
      const int pb = pidx(p0);
#pragma unroll
      for (int r = 0; r < RL; ++r) q[i][r] = buf[pidx_run(pb, p0, r, NS << lognseq)];
    }
#pragma unroll
    for (int i = 0; i < UL; ++i) {
      if constexpr (NS > 1) {
        int s, j;
        ci_unit<JF>(imin(tid + i * nthr, units - 1), lognseq, LAST, s, j);
        C2<T> w[RL];
        twiddle_powers<T, DIR, RL>(tw, NS * RL, j, w);
#pragma unroll
        for (int r = 1; r < RL; ++r) q[i][r] = cmul(q[i][r], w[r]);
      }
      dft_reg<T, RL, DIR>(q[i]);
    }
#pragma unroll
    for (int i = 0; i < UL; ++i) {
      const int u = tid + i * nthr;
      if (u < units) {
        int s, j;
        ci_unit<JF>(u, lognseq, LAST, s, j);
#pragma unroll
        for (int r = 0; r < RL; ++r) store(i, r, s, j + r * NS, q[i][r]);
      }
    }
  } else {
    if constexpr (FIRST) lds_fft_ci<T, DIR, E, 8, LOGN, LR1, TW>(buf, lognseq, tw, tid, nthr);
    else lds_fft_ci<T, DIR, E, 8, LOGN, 0, TW>(buf, lognseq, tw, tid, nthr);
  }
}

// Batched INTERLEAVED FFT (2^lognseq sequences of length 2^logn, 1 <= logn
// <= 10, at LDS base 0), dispatched to the compile-time variant.
template <class T, int DIR, int E, int RMAX, class TW>
__device__ __forceinline__ void lds_fft_interleaved(C2<T>* buf, int logn, int lognseq, const TW& tw, int tid,
                                                    int nthr) {
  switch (logn) {
    case 1: lds_fft_ci<T, DIR, E, RMAX, 1, 0, TW>(buf, lognseq, tw, tid, nthr); break;
    case 2: lds_fft_ci<T, DIR, E, RMAX, 2, 0, TW>(buf, lognseq, tw, tid, nthr); break;
    case 3: lds_fft_ci<T, DIR, E, RMAX, 3, 0, TW>(buf, lognseq, tw, tid, nthr); break;
    case 4: lds_fft_ci<T, DIR, E, RMAX, 4, 0, TW>(buf, lognseq, tw, tid, nthr); break;
    case 5: lds_fft_ci<T, DIR, E, RMAX, 5, 0, TW>(buf, lognseq, tw, tid, nthr); break;
    case 6: lds_fft_ci<T, DIR, E, RMAX, 6, 0, TW>(buf, lognseq, tw, tid, nthr); break;
    case 7: lds_fft_ci<T, DIR, E, RMAX, 7, 0, TW>(buf, lognseq, tw, tid, nthr); break;
    case 8: lds_fft_ci<T, DIR, E, RMAX, 8, 0, TW>(buf, lognseq, tw, tid, nthr); break;
    case 9: lds_fft_ci<T, DIR, E, RMAX, 9, 0, TW>(buf, lognseq, tw, tid, nthr); break;
    default: lds_fft_ci<T, DIR, E, RMAX, 10, 0, TW>(buf, lognseq, tw, tid, nthr); break;
  }
}

// The passes after a first radix-8 pass done by the caller (3 <= logn <= 13).
// Waves without a unit skip each pass (a batch may fill only part of the block).
template <class T, int DIR, int E, class TW>
__device__ __forceinline__ void lds_fft_contig_after8(C2<T>* buf, int base, int logn, int nseq, const TW& tw,
                                                      int tid, int nthr) {
  switch (logn) {
    case 3: break;
    case 4: lds_fft_c<T, DIR, E, 8, 4, 3, TW, 4, true>(buf, base, nseq, tw, tid, nthr); break;
    case 5: lds_fft_c<T, DIR, E, 8, 5, 3, TW, 5, true>(buf, base, nseq, tw, tid, nthr); break;
    case 6: lds_fft_c<T, DIR, E, 8, 6, 3, TW, 6, true>(buf, base, nseq, tw, tid, nthr); break;
    case 7: lds_fft_c<T, DIR, E, 8, 7, 3, TW, 7, true>(buf, base, nseq, tw, tid, nthr); break;
    case 8: lds_fft_c<T, DIR, E, 8, 8, 3, TW, 8, true>(buf, base, nseq, tw, tid, nthr); break;
    case 9: lds_fft_c<T, DIR, E, 8, 9, 3, TW, 9, true>(buf, base, nseq, tw, tid, nthr); break;
    case 10: lds_fft_c<T, DIR, E, 8, 10, 3, TW, 10, true>(buf, base, nseq, tw, tid, nthr); break;
    case 11: lds_fft_c<T, DIR, E, 8, 11, 3, TW, 11, true>(buf, base, nseq, tw, tid, nthr); break;
    case 12: lds_fft_c<T, DIR, E, 8, 12, 3, TW, 12, true>(buf, base, nseq, tw, tid, nthr); break;
    default: lds_fft_c<T, DIR, E, 8, 13, 3, TW, 13, true>(buf, base, nseq, tw, tid, nthr); break;
  }
}

// Batched CONTIG FFT of nseq sequences of length 2^logn, 1 <= logn <= 13,
// dispatched to the compile-time variant (same contract as lds_fft); waves
// without a unit skip each pass.
template <class T, int DIR, int E, int RMAX, class TW>
__device__ __forceinline__ void lds_fft_contig(C2<T>* buf, int base, int logn, int nseq, const TW& tw, int tid,
                                               int nthr) {
  switch (logn) {
    case 1: lds_fft_c<T, DIR, E, RMAX, 1, 0, TW, 1, true>(buf, base, nseq, tw, tid, nthr); break;
    case 2: lds_fft_c<T, DIR, E, RMAX, 2, 0, TW, 2, true>(buf, base, nseq, tw, tid, nthr); break;
    case 3: lds_fft_c<T, DIR, E, RMAX, 3, 0, TW, 3, true>(buf, base, nseq, tw, tid, nthr); break;
    case 4: lds_fft_c<T, DIR, E, RMAX, 4, 0, TW, 4, true>(buf, base, nseq, tw, tid, nthr); break;
    case 5: lds_fft_c<T, DIR, E, RMAX, 5, 0, TW, 5, true>(buf, base, nseq, tw, tid, nthr); break;
    case 6: lds_fft_c<T, DIR, E, RMAX, 6, 0, TW, 6, true>(buf, base, nseq, tw, tid, nthr); break;
    case 7: lds_fft_c<T, DIR, E, RMAX, 7, 0, TW, 7, true>(buf, base, nseq, tw, tid, nthr); break;
    case 8: lds_fft_c<T, DIR, E, RMAX, 8, 0, TW, 8, true>(buf, base, nseq, tw, tid, nthr); break;
    case 9: lds_fft_c<T, DIR, E, RMAX, 9, 0, TW, 9, true>(buf, base, nseq, tw, tid, nthr); break;
    case 10: lds_fft_c<T, DIR, E, RMAX, 10, 0, TW, 10, true>(buf, base, nseq, tw, tid, nthr); break;
    case 11: lds_fft_c<T, DIR, E, RMAX, 11, 0, TW, 11, true>(buf, base, nseq, tw, tid, nthr); break;
    case 12: lds_fft_c<T, DIR, E, RMAX, 12, 0, TW, 12, true>(buf, base, nseq, tw, tid, nthr); break;
    default: lds_fft_c<T, DIR, E, RMAX, 13, 0, TW, 13, true>(buf, base, nseq, tw, tid, nthr); break;
  }
}

}  // namespace slicq
