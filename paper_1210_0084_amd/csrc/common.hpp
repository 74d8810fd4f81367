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

// Analysis work item: bands k0 .. k0 + cnt - 1, all with M_k = M.
struct alignas(16) AnaGroupDev {
  int32_t k0, cnt, M, logM;
};

// Synthesis work item: bins [lo, hi) of the half spectrum, built from bands
// ke .. kb whose coefficients are transformed in runs of equal M_k.
struct alignas(16) SynGroupDev {
  int32_t ke, kb, lo, hi;
  int32_t run0, nrun, total, pad_;
};

struct alignas(16) SynRunDev {
  int32_t k0, cnt, M, logM;
  int32_t lds_off, pad0_, pad1_, pad2_;
};

// Streaming: `count` samples move between position `pos` (mod R) of the ring
// of stream slot `slot` and offset `off` of a packed staging buffer.
struct alignas(16) RingCopy {
  int32_t slot, count;
  int64_t pos, off;
};

// Byte offsets of the device tables inside one uploaded blob. The frequency
// overlap-add of synthesis is a per-bin program: bin j (0..N) sums entries
// ent_off[j] .. ent_off[j+1]-1, entry e reading the transformed coefficient at
// LDS position ent_pos[e].x (and, for the self-mirrored DC and Nyquist bands,
// the conjugate of the one at ent_pos[e].y, else y = -1) times ent_wsyn[e]
// (synthesis, dual windows) or ent_wadj[e] (adjoint, analysis windows).
struct TableLayout {
  uint64_t tw, h0, hd, g, gd, bands, ana, syn, runs, ent_off, ent_pos, ent_wsyn, ent_wadj, total;
};

}  // namespace slicq
