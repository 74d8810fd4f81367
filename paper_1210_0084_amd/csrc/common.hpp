// Plain-old-data records shared by the host plan and the HIP kernels.
#pragma once
#include <cstdint>

namespace slicq {

// LDS arrays of the kernels hold one pad slot every 2^kPadShift complex
// values (bank spreading for the strided Stockham stores; one pad per 8
// values measured no faster than one per 16): padded(n) slots hold n values.
constexpr int kPadShift = 4;
constexpr int padded(int n) { return n + (n >> kPadShift) + 1; }

// Entries of the split twiddle tables for transforms up to 2^L (two levels
// of the pyramid, 2^(L - L/2) and 2^L: every e^{-2 pi i k / 2^l}, l <= L, is
// a product of one entry of each).
constexpr int split_tw_entries(int L) { return (1 << (L - (L >> 1))) + (1 << (L >> 1)); }

// One slice to process: where its 2N input samples come from, where its
// coefficients go and where its overlap-added output goes. Sample j of the
// slice (j < 2N, window position t = j - N) reads x[x_base + idx] with
// idx = (x_start + j) mod x_period, and reads zero when idx >= x_valid.
// The output side uses the same addressing. Coefficient n of band k lands at
// coef_base + S * off_k + m * M_k + n (band-major layout).
struct alignas(16) SliceTask {
  int64_t x_base, x_start, x_period, x_valid;
  int64_t y_base, y_start, y_period, y_valid;
  int64_t coef_base;
  int32_t m, S;
  int32_t flags;      // reserved (set to 1 by the task builders)
  int32_t pad_;
  int64_t pad2_;
};
static_assert(sizeof(SliceTask) == 96, "SliceTask layout");

// Per stored band k (0..K+1): support J_k = {start, ..., start + len - 1}
// (signed bins, circular), M_k coefficients per slice, packing offset off_k,
// offset goff of its window values, half-spectrum coverage [hlo, hhi].
struct alignas(16) BandDev {
  int32_t start, len, M, logM;
  int32_t off, goff, hlo, hhi;
};

// Four 32-bit integers (one 16-byte load).
struct alignas(16) I4 {
  int32_t x, y, z, w;
};

// Largest work item (complex values) of the kernels for small items; larger
// items (a wide DC or Nyquist plateau band) go to kernels with more threads
// or more values per thread.
constexpr int kAnaSmallValues = 4096;
constexpr int kSynSmallValues = 8192;
constexpr int kSynMaxValues = 16384;    // largest synthesis work item
// Most bands one work item may span (an analysis item stages their
// descriptors in LDS).
constexpr int kMaxGroupBands = 256;

// Analysis work item: bands k0 .. k0 + cnt - 1, all with M_k = M.
struct alignas(16) AnaGroupDev {
  int32_t k0, cnt, M, logM;
};

// A run: bands k0 .. k0 + cnt - 1 with M_k = M, packed from offset off of the
// slice's coefficients, held at LDS position lds_off of the work item.
struct alignas(16) SynRunDev {
  int32_t k0, cnt, M, logM;
  int32_t lds_off, off, pad0_, pad1_;
};

// Synthesis work item: bins [lo, hi) of the half spectrum, built from bands
// ke .. kb whose coefficients are transformed in runs of equal M_k (at most
// kMaxRuns runs, runs[run0 ..]); maxM is the largest M_k among them. The
// first two runs are repeated inline (read with the item, no second lookup).
struct alignas(16) SynGroupDev {
  int32_t ke, kb, lo, hi;
  int32_t run0, nrun, total, maxM;
  SynRunDev r[2];
};

constexpr int kMaxRuns = 8;

// Streaming: `count` samples move between position `pos` (mod R) of the ring
// of stream slot `slot` and offset `off` of a packed staging buffer.
struct alignas(16) RingCopy {
  int32_t slot, count;
  int64_t pos, off;
};

// Byte offsets of the device tables inside one uploaded blob. The frequency
// overlap-add of synthesis is a per-bin program over the bands covering bin
// j (0..N) in increasing k; an entry reads the transformed coefficient at LDS
// position x of the owning work item (and, for the self-mirrored DC and
// Nyquist bands, adds the conjugate of the one at position y, else y = -1)
// times a weight: the dual window (synthesis) or the analysis window
// (adjoint). The first two entries of bin j sit in one record, ola_syn[j] or
// ola_adj[j] (weight 0 and x = 0 for a missing entry); any further entries
// are ent_off[j] .. ent_off[j+1]-1 of ent_pos (pairs x, y) and ent_w*.
// Entries of the radix-8 twiddle rows of the band FFTs (passes at Ns = 8 and
// Ns = 64, seven rows each).
constexpr int kPow8Entries = 7 * 8 + 7 * 64;

struct TableLayout {
  uint64_t tw, tw8, h0, hd, g, gd, gdw, bands, ana, syn, runs;
  uint64_t ola_syn, ola_adj, ent_off, ent_pos, ent_wsyn, ent_wadj;
  uint64_t fana, fsyn, fola_syn, fola_adj, fent_off, fent_pos, fent_wsyn, fent_wadj;
  uint64_t twmix, bsmod;     // mixed-radix plans: combination twiddles, (-start_k) mod M_k per band
  uint64_t total;
};

// Fused per-slice work item, for plans whose half spectrum fits in one
// workgroup's LDS: one block runs the whole analysis (or synthesis) of a
// slice, its LDS holding an index space [0, cap) whose indices 0..N hold the
// half spectrum. Item: bands k0 .. k0 + cnt - 1 (equal M_k) transformed at
// indices lds .. lds + cnt M - 1, either past the spectrum (lds = N + 1) or
// over spectrum bins no later item reads (analysis, in increasing k) or
// writes before it (synthesis, in decreasing k). Synthesis items add their
// bands into bins [olo, ohi] through records rec0 .. rec0 + ohi - olo.
struct alignas(16) FusedItemDev {
  int32_t k0, cnt, M, logM;
  int32_t lds, olo, ohi, rec0;
};

// Frequency overlap-add record of one bin of a fused synthesis item: LDS
// indices x0 | x1 << 16 of the first two entries (bit 15: further entries
// follow in the overflow table; bit 31: this item is the first to write the
// bin, which it sets instead of adding to), mirror indices y0 | y1 << 16
// (0xffff: none) and the two weights.
template <class T>
struct alignas(16) FOlaRec {
  uint32_t xx, yy;
  T w0, w1;
};
constexpr uint32_t kFMore = 0x8000u, kFInit = 0x80000000u, kFPos = 0x7fffu;
constexpr int kFusedThreads = 1024;     // block of the fused kernels
constexpr int kFusedE = 8;              // values per thread of a fused item's band FFT
constexpr int kFusedMaxItem = kFusedThreads * kFusedE;

// The first two overlap-add entries of a bin, read with one load: positions
// x0 | x1 << 16 (bit 15 set when the bin has further entries), mirror
// positions y0 | y1 << 16 (0xffff: none), weights w0, w1. Positions are below
// kSynMaxValues, so 14 bits hold them.
template <class T>
struct alignas(16) OlaRec {
  uint32_t xx, yy;
  T w0, w1;
};
constexpr uint32_t kOlaMore = 0x8000u, kOlaPosMask = 0x3fffu, kOlaNone = 0xffffu;
static_assert(kSynMaxValues <= 0x4000, "overlap-add positions must fit 14 bits");

// Full-length CQ-NSGT (Algorithms 1 and 2 at the signal length L): band k
// over J^L_k = {start, ..., start + len - 1} (signed bins, circular modulo
// L), M^L_k coefficients at offset off, window values at goff.
struct alignas(16) FullBandDev {
  int64_t start, off, goff;
  int32_t len, M;
};

// A run of count transforms of length 2^logn at off (complex values) that
// owns blocks blk0 .. of its launch.
struct alignas(16) FullRunDev {
  int64_t off, blk0;
  int32_t count, logn;
  int64_t pad_;
};

// Run tables of one set of transforms (byte offsets in the blob): runs of at
// most kLongVals points (one LDS block each per kLongVals values) and longer
// runs (four-step, kLongVals values per block and pass).
struct FullRunSet {
  size_t small = 0, large = 0;
  int32_t nsmall = 0, nlarge = 0;
  int64_t blk_small = 0, blk_large = 0;
};

// Device tables of a full-length plan (byte offsets in one blob); sig is the
// one transform of the signal, bandruns the band transforms.
struct FullLayout {
  size_t bands = 0, g = 0, ent_off = 0, ent_idx = 0, ent_w = 0, tw = 0, total = 0;
  FullRunSet sig, bandruns;
};

// Mixed-radix twiddle table: for R = 3 then R = 5, for logP = 1 .. L,
// e^{-2 pi i k / M} for k < M = R 2^logP (entries from R (2^logP - 2) of the
// R block; the R = 5 block starts after the 3 (2^(L+1) - 2) entries of R = 3).
constexpr int64_t mix_tw_base(int R, int logP, int L) {
  return (R == 3 ? 0 : 3 * ((int64_t(2) << L) - 2)) + R * ((int64_t(1) << logP) - 2);
}

// Complex values one block of the long-transform kernels holds in LDS (16
// per thread of 256): transforms up to this length run in one block, longer
// ones (up to kLongVals^2) as two passes of a four-step FFT.
constexpr int kLongVals = 4096;
constexpr int kLongLog = 12;
constexpr int kLongThreads = 256;

}  // namespace slicq
