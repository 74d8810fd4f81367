// FP64 host plan of the constant-Q painless NSG frame and the Tukey slicing
// windows, and the work schedule of the HIP kernels.
#pragma once
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

namespace slicq {

struct PlanParams {
  double fs = 0, fmin = 0, fmax = 0;
  int32_t bins_per_octave = 0;
  int64_t slice_len = 0;        // 2N
  int64_t transition = 0;       // M of the Tukey window
  double min_win = 16.0;        // minimal filter length in bins
  int32_t dual_kind = 0;        // 0: canonical dual slice window, 1: indicator of supp h_0
  int32_t group_cap = 2048;     // coefficients per analysis work item
  int32_t lds_cap = 4096;       // target complex values per synthesis work item
  int32_t pass_cap = 4096;      // complex values per four-step FFT work item
  int32_t coef_layout = 0;      // 0: band-major, 1: slice-major
  int32_t fused = 0;            // 1: one workgroup per slice where the half spectrum fits in LDS, 0: never
  int32_t window = 0;           // band window: 0 Hann, 1 Blackman-Harris (4 terms)
  int32_t scale = 0;            // centres: 0 constant-Q (geometric), 1 mel, 2 Bark
  int32_t slicing = 0;          // 0 Tukey (sum_m h_m = 1), 1 square root of Tukey (sum_m h_m^2 = 1)
  int32_t m_policy = 0;         // 0 smallest power of two >= |J_k|, 1 one M for every band (rectangular),
                                // 2 smallest even 2^a, 3 2^a or 5 2^a >= |J_k|
};

// The fused per-slice schedule of one dtype (see FusedItemDev).
struct FusedPlan {
  bool ok = false;
  int32_t cap = 0;              // LDS indices used (spectrum, scratch)
  int32_t nthr = 0;             // threads per block
  int32_t logM = 0;             // log2 of the largest M_k (band twiddle tables)
  size_t lds_bytes = 0;         // dynamic LDS per block
  std::vector<FusedItemDev> ana, syn;
  // overlap-add records of the synthesis items (positions and both weight sets)
  std::vector<uint32_t> rec_xx, rec_yy;
  std::vector<double> rec_ws, rec_wa;   // two per record
  std::vector<int32_t> ent_off;         // per record, then the end
  std::vector<int32_t> ent_pos;         // pairs (x, y)
  std::vector<double> ent_ws, ent_wa;
};

struct BandInfo {
  int32_t k = 0;
  int64_t start = 0;   // signed first bin of J_k
  int32_t len = 0;     // |J_k|
  int32_t M = 0;       // M_k = 2N / a_k
  int32_t logM = 0;    // M_k = R 2^logM with R in {1, 3, 5}
  int64_t off = 0;     // sum_{k' < k} M_k'
  int64_t goff = 0;    // offset in the concatenated window tables
  int32_t hlo = 0, hhi = 0;   // bins of J_k inside [0, N]
  double xi = 0, omega = 0;   // centre and bandwidth in Hz
};

struct Plan {
  PlanParams prm;
  double Q = 0;
  int64_t two_n = 0, N = 0, Mt = 0;
  int32_t K0 = 0, K = 0, nb = 0;
  std::vector<BandInfo> bands;          // stored bands 0..K+1
  std::vector<double> g, gd;            // windows over each J_k, concatenated
  std::vector<double> D;                // frame-operator diagonal, 2N bins
  std::vector<double> h0, hd;           // slicing window and dual, index j = t + N
  std::vector<int32_t> bin_k0, bin_nk;  // bands covering each bin of [0, N]
  // frequency overlap-add program (see TableLayout): two fixed entries per
  // bin, then the rest of each bin's entries
  std::vector<int32_t> ent2_pos;        // (x0, y0, x1, y1) per bin
  std::vector<double> ent2_wsyn, ent2_wadj;
  std::vector<int32_t> ent_off;
  std::vector<int32_t> ent_pos;         // pairs (x, y)
  std::vector<double> ent_wsyn, ent_wadj;
  int64_t coefs_per_slice = 0;
  int32_t max_M = 0;
  bool mixed = false;                   // some M_k = 3 2^a or 5 2^a: band kernels for mixed radix
  int32_t mix_L = 0;                    // largest logM among bands with M_k = 3 2^a or 5 2^a

  // kernel schedule
  std::vector<AnaGroupDev> ana;
  std::vector<SynGroupDev> syn;
  std::vector<SynRunDev> runs;
  int32_t ana_cap = 0, syn_cap = 0;     // largest work item, complex values
  int32_t syn_bands = 0;                // most bands in one synthesis work item
  // Work items are ordered small first: ana[0, ana_small) hold at most
  // kAnaSmallValues values, the rest more (likewise syn / kSynSmallValues).
  // The two classes launch as separate kernels sized for each.
  int32_t ana_small = 0, syn_small = 0;
  int32_t ana_cap_small = 0, ana_cap_big = 0, syn_cap_small = 0, syn_cap_big = 0;
  int32_t ana_maxM_small = 0, syn_maxM_small = 0;   // largest M_k in the small items
  int32_t N1 = 0, N2 = 0, logN1 = 0, logN2 = 0;
  int32_t C = 0, P = 0;                 // columns per pass-1 item, row pairs per pass-2 item
  FusedPlan fused[2];                   // per dtype (0: f32, 1: f64)

  // device tables, per dtype (0: f32, 1: f64); owned by the caller
  std::mutex mu;
  void* dev[2] = {nullptr, nullptr};
  size_t dev_bytes[2] = {0, 0};
  TableLayout layout[2] = {};
};

// Full-length CQ-NSGT of a complex signal of length L (Algorithms 1 and 2 at
// length L, Section 3) on the band windows of a sliCQ plan sampled on the
// L-point grid (g_k[j] = g^L_k[j L / 2N], Proposition 4), all 2K+2 bands:
// 0..K+1, then the mirrors of K..1. Lattice 0 keeps the sliCQ hops
// (M^L_k = M_k L / 2N), lattice 1 takes the smallest power of two >= |J^L_k|
// (the painless case of Proposition 2).
struct FullRun {
  int64_t off;          // first coefficient of the run
  int32_t count;        // consecutive bands with equal M^L_k
  int32_t logn;         // log2 M^L_k
};

struct FullPlan {
  int64_t L = 0, two_n = 0;
  int32_t logL = 0, lattice = 0, nb = 0;
  bool painless = false;               // every band has M^L_k >= |J^L_k|
  std::vector<FullBandDev> bands;
  std::vector<double> g;               // windows over each J^L_k, concatenated
  std::vector<double> D;               // frame-operator diagonal, L bins
  // synthesis gather: bin j takes entries [ent_off[j], ent_off[j + 1]) of
  // (coefficient index, dual weight), bands in increasing order
  std::vector<int32_t> ent_off, ent_idx;
  std::vector<double> ent_w;
  std::vector<FullRun> runs;
  int64_t coef_count = 0, max_M = 0;

  // device tables, per dtype; owned by the caller
  std::mutex mu;
  void* dev[2] = {nullptr, nullptr};
  size_t dev_bytes[2] = {0, 0};
  FullLayout layout[2] = {};
};

// Builds the full-length plan of p at length L; returns 0 or a negative
// status with a message in err.
int build_full(const Plan& p, int64_t L, int lattice, FullPlan& out, std::string& err);

// Packs a full-length plan's device tables for dtype into a host byte vector.
void pack_full_tables(const FullPlan& f, int dtype, std::vector<unsigned char>& blob, FullLayout& lay);

// Builds the plan; returns 0 or a negative status with a message in err.
int build_plan(const PlanParams& p, Plan& out, std::string& err);

// Packs the device tables for dtype (0 f32, 1 f64) into a host byte vector.
void pack_tables(const Plan& p, int dtype, std::vector<unsigned char>& blob, TableLayout& lay);

}  // namespace slicq
