// Plain-old-data records shared by the host plan and the HIP kernels.
#pragma once
#include <cstdint>

namespace slicq {

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
  int32_t flags;      // bit 0: zero the right-hand overlap of the output first
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
// (adjoint). The first two entries of bin j sit at fixed places, ent2_pos[j]
// = (x0, y0, x1, y1) and ent2_w*[2j], ent2_w*[2j + 1] (weight 0 and x = 0
// for a missing entry); any further entries are ent_off[j] .. ent_off[j+1]-1
// of ent_pos (pairs x, y) and ent_w*.
struct TableLayout {
  uint64_t tw, h0, hd, g, gd, bands, ana, syn, runs;
  uint64_t ent2_pos, ent2_wsyn, ent2_wadj, ent_off, ent_pos, ent_wsyn, ent_wadj, total;
};

}  // namespace slicq
