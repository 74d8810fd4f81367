// Host orchestration of the sliCQ kernels: argument packing, workspace
// layout, launch geometry and the per-call launch sequences. Templated on the
// launcher so the same sequence drives the device (hipLaunchKernelGGL).
#pragma once
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>

#include "bandmix.hpp"
#include "fused.hpp"
#include "kernels.hpp"
#include "plan.hpp"

namespace slicq {

inline int threads_for(int64_t values, int E = 16) {
  int64_t t = (values + E - 1) / E;
  t = (t + 63) / 64 * 64;
  return (int)std::min<int64_t>(1024, std::max<int64_t>(64, t));
}

inline int ilog2i(int64_t n) {
  int l = 0;
  while ((int64_t(1) << l) < n) ++l;
  return l;
}

inline size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

constexpr size_t kMaxLdsBytes = 160 * 1024;   // LDS of one gfx950 workgroup

// Workspace: [slice tasks][status words][W1: chunk x N][W2: chunk x (N + 64)]
struct WorkLayout {
  size_t tasks_off = 0, status_off = 0, w1_off = 0, w2_off = 0, total = 0;
  int64_t chunk = 0;
};

inline int64_t ws1_len(const Plan& p) { return p.N; }
inline int64_t ws2_len(const Plan& p) { return p.N + 64; }

inline size_t slice_scratch_bytes(const Plan& p, int dtype) {
  const size_t cb = dtype ? 16 : 8;
  return (size_t)(ws1_len(p) + ws2_len(p)) * cb;
}

inline size_t tasks_bytes(int64_t ntasks) { return align256((size_t)std::max<int64_t>(ntasks, 1) * sizeof(SliceTask)); }

inline size_t workspace_bytes(const Plan& p, int dtype, int64_t ntasks) {
  return tasks_bytes(ntasks) + 256 + 2 * 256 + (size_t)std::max<int64_t>(ntasks, 1) * slice_scratch_bytes(p, dtype);
}

// Lays out `bytes` of workspace for ntasks slices; chunk = slices per pass.
inline bool work_layout(const Plan& p, int dtype, int64_t ntasks, size_t bytes, WorkLayout& w) {
  const size_t cb = dtype ? 16 : 8;
  w.tasks_off = 0;
  w.status_off = tasks_bytes(ntasks);
  const size_t fixed = w.status_off + 256;
  const size_t per = slice_scratch_bytes(p, dtype);
  if (bytes < fixed + 2 * 256 + per) return false;
  int64_t chunk = (int64_t)((bytes - fixed - 2 * 256) / per);
  chunk = std::min<int64_t>(chunk, std::max<int64_t>(ntasks, 1));
  w.chunk = chunk;
  w.w1_off = fixed;
  w.w2_off = align256(w.w1_off + (size_t)chunk * ws1_len(p) * cb);
  w.total = align256(w.w2_off + (size_t)chunk * ws2_len(p) * cb);
  return w.total <= bytes;
}

// Kernel arguments. adjoint: the synthesis kernels with the analysis windows
// (adjoint of analysis); dual: the analysis kernels with the dual windows
// h~_0 and w_k g~_k (adjoint of synthesis, w_k = 2 on bands 1..K).
template <class T>
KArgs<T> make_args(const Plan& p, int dtype, bool adjoint, bool dual = false) {
  const TableLayout& L = p.layout[dtype];
  const char* base = static_cast<const char*>(p.dev[dtype]);
  KArgs<T> a{};
  a.tw = reinterpret_cast<const C2<T>*>(base + L.tw);
  a.h0 = reinterpret_cast<const T*>(base + (dual ? L.hd : L.h0));
  a.hsyn = reinterpret_cast<const T*>(base + (adjoint ? L.h0 : L.hd));
  a.g = reinterpret_cast<const T*>(base + (dual ? L.gdw : L.g));
  a.bands = reinterpret_cast<const BandDev*>(base + L.bands);
  a.ana = reinterpret_cast<const AnaGroupDev*>(base + L.ana);
  a.syn = reinterpret_cast<const SynGroupDev*>(base + L.syn);
  a.runs = reinterpret_cast<const SynRunDev*>(base + L.runs);
  a.ola2 = reinterpret_cast<const OlaRec<T>*>(base + (adjoint ? L.ola_adj : L.ola_syn));
  a.tw8 = reinterpret_cast<const C2<T>*>(base + L.tw8);
  a.ent_off = reinterpret_cast<const int32_t*>(base + L.ent_off);
  a.ent_pos = reinterpret_cast<const int2*>(base + L.ent_pos);
  a.ent_w = reinterpret_cast<const T*>(base + (adjoint ? L.ent_wadj : L.ent_wsyn));
  a.N = (int32_t)p.N;
  a.min_M = 1 << 30;
  for (const BandInfo& b : p.bands) a.min_M = std::min<int32_t>(a.min_M, b.M);
  a.Mt = (int32_t)p.Mt;
  a.K = p.K;
  a.N1 = p.N1;
  a.N2 = p.N2;
  a.logN1 = p.logN1;
  a.logN2 = p.logN2;
  a.C = p.C;
  a.logC = ilog2i(p.C);
  a.P = p.P;
  a.logP = ilog2i(p.P);
  a.ws1 = ws1_len(p);
  a.ws2 = ws2_len(p);
  a.scale = (T)(1.0 / std::sqrt((double)p.two_n));
  a.slice_major = p.prm.coef_layout;
  a.cps = (int32_t)p.coefs_per_slice;
  const FusedPlan& f = p.fused[dtype];
  a.fused = f.ok ? 1 : 0;
  a.fana = reinterpret_cast<const FusedItemDev*>(base + L.fana);
  a.fsyn = reinterpret_cast<const FusedItemDev*>(base + L.fsyn);
  a.fola = reinterpret_cast<const FOlaRec<T>*>(base + (adjoint ? L.fola_adj : L.fola_syn));
  a.fent_off = reinterpret_cast<const int32_t*>(base + L.fent_off);
  a.fent_pos = reinterpret_cast<const int2*>(base + L.fent_pos);
  a.fent_w = reinterpret_cast<const T*>(base + (adjoint ? L.fent_wadj : L.fent_wsyn));
  a.nfana = (int32_t)f.ana.size();
  a.nfsyn = (int32_t)f.syn.size();
  a.flogM = f.logM;
  a.twmix = reinterpret_cast<const C2<T>*>(base + L.twmix);
  a.bsmod = reinterpret_cast<const int32_t*>(base + L.bsmod);
  a.mixL = p.mix_L;
  a.fcap = f.cap;
  return a;
}

template <class T>
struct Geometry {
  int g1, b1; size_t s1;      // forward pass 1 / inverse pass B: items per slice, threads, LDS bytes
  int g2, b2; size_t s2;      // forward pass 2 / inverse pass A
  // band analysis: small items [0, ga) with ba threads, E = kSmallE (kernel
  // bound kAnaThreads); large items [ga, ga + gab) with bab threads,
  // E = kBigAnaE (bound kAnaBigThreads). Items stage small twiddle tables
  // (TwBand) in LDS; every level up to M (tab, tsb) only for large items and
  // only where that costs no resident block per CU.
  int ga, ba; size_t sa;
  int gab, bab; size_t sab; bool tab;
  // band synthesis: small items [0, gs), bs threads, E = kSmallE (bound
  // kSynThreads); large items [gs, gs + gsb), bsb threads, E = kBigSynE
  // (bound kSynBigThreads)
  int gs, bs; size_t ss;
  int gsb, bsb; size_t ssb; bool tsb;
  // plans with some M_k = 3 2^a or 5 2^a: every band item runs the
  // mixed-radix kernels (bandmix.hpp), analysis items with bxa threads and
  // exa values per thread, synthesis items with bxs threads and exs values
  bool mixed;
  int gxa, bxa, exa; size_t sxa;
  int gxs, bxs, exs; size_t sxs;
  bool ok;                    // every block fits its kernel's launch bound
};

// An LDS copy of the twiddles (tw bytes) for blocks of lds bytes only where it
// costs no resident block per CU (measured: the copy does not pay for lost
// residency).
inline bool lds_twiddles_pay(size_t lds, size_t tw) {
  return lds + tw <= kMaxLdsBytes && kMaxLdsBytes / (lds + tw) >= kMaxLdsBytes / std::max<size_t>(lds, 1);
}

template <class T>
Geometry<T> geometry(const Plan& p) {
  Geometry<T> g{};
  const size_t cb = sizeof(C2<T>);
  auto split_bytes = [&](int32_t maxM, bool p8) {   // TwBand tables for lengths up to maxM
    int L = 0;
    while ((1 << L) < maxM) ++L;
    return (size_t)band_tw_entries(L, p8) * cb;
  };
  g.g1 = p.N1 / p.C;
  g.b1 = threads_for((int64_t)p.C * p.N2, kPassE);
  g.s1 = (padded(p.C * p.N2) + p.N2 + p.N1 + p.N2) * cb;   // values, FFT twiddles, four-step tables
  g.g2 = (p.N2 / 2) / p.P;
  g.b2 = threads_for((int64_t)2 * p.P * p.N1, kPassE);
  g.s2 = (padded(2 * p.P * p.N1) + p.N1 + p.N1 + p.N2) * cb;   // values, FFT twiddles, four-step tables
  g.ga = p.ana_small;
  g.ba = threads_for(std::max(p.ana_cap_small, 1), kSmallE);
  g.sa = lds_tail_offset<T>(p.ana_cap_small) + split_bytes(p.ana_maxM_small, false);
  g.gab = (int)p.ana.size() - p.ana_small;
  g.bab = threads_for(std::max(p.ana_cap_big, 1), kBigAnaE);
  g.sab = lds_tail_offset<T>(p.ana_cap_big);
  int32_t big_ana_M = 0;
  for (int i = p.ana_small; i < (int)p.ana.size(); ++i) big_ana_M = std::max(big_ana_M, p.ana[i].M);
  g.tab = lds_twiddles_pay(g.sab, (size_t)big_ana_M * cb);
  g.sab += g.tab ? (size_t)big_ana_M * cb : split_bytes(big_ana_M, false);
  g.gs = p.syn_small;
  g.bs = threads_for(std::max(p.syn_cap_small, 1), kSmallE);
  g.ss = lds_tail_offset<T>(p.syn_cap_small) + split_bytes(p.syn_maxM_small, true);
  g.gsb = (int)p.syn.size() - p.syn_small;
  g.bsb = threads_for(std::max(p.syn_cap_big, 1), kBigSynE);
  g.ssb = lds_tail_offset<T>(p.syn_cap_big);
  int32_t big_maxM = 0;
  for (int i = p.syn_small; i < (int)p.syn.size(); ++i) big_maxM = std::max(big_maxM, p.syn[i].maxM);
  g.tsb = lds_twiddles_pay(g.ssb, (size_t)big_maxM * cb);
  g.ssb += g.tsb ? (size_t)big_maxM * cb : split_bytes(big_maxM, true);
  g.mixed = p.mixed;
  if (p.mixed) {
    int32_t syn_max = 0;
    for (const SynGroupDev& G : p.syn) syn_max = std::max(syn_max, G.total);
    g.gxa = (int)p.ana.size();
    g.exa = p.ana_cap <= 8 * kMixThreads ? 8 : 16;
    g.bxa = threads_for(std::max(p.ana_cap, 1), g.exa);
    g.sxa = lds_tail_offset<T>(p.ana_cap);
    g.gxs = (int)p.syn.size();
    g.exs = syn_max <= 8 * kMixThreads ? 8 : 16;
    g.bxs = threads_for(std::max(syn_max, 1), g.exs);
    g.sxs = lds_tail_offset<T>(syn_max);
    g.ok = g.b1 <= kPassThreads && g.b2 <= kPassThreads && (int64_t)p.C * p.N2 <= (int64_t)kPassE * g.b1 &&
           2LL * p.P * p.N1 <= (int64_t)kPassE * g.b2 && p.ana_cap <= g.exa * g.bxa && syn_max <= g.exs * g.bxs &&
           g.gxs <= 65535 && std::max(std::max(g.s1, g.s2), std::max(g.sxa, g.sxs)) <= kMaxLdsBytes;
    return g;
  }
  size_t lds = std::max(std::max(g.s1, g.s2), std::max(g.sa, g.ss));
  if (g.gab) lds = std::max(lds, g.sab);
  if (g.gsb) lds = std::max(lds, g.ssb);
  g.ok = g.b1 <= kPassThreads && g.b2 <= kPassThreads && (int64_t)p.C * p.N2 <= (int64_t)kPassE * g.b1 &&
         2LL * p.P * p.N1 <= (int64_t)kPassE * g.b2 &&
         g.ba <= kAnaThreads && p.ana_cap_small <= kSmallE * g.ba &&
         (g.gab == 0 || (g.bab <= kAnaBigThreads && p.ana_cap_big <= kBigAnaE * g.bab)) &&
         g.bs <= kSynThreads && p.syn_cap_small <= kSmallE * g.bs &&
         (g.gsb == 0 || (g.bsb <= kSynBigThreads && p.syn_cap_big <= kBigSynE * g.bsb)) &&
         g.gs + g.gsb <= 65535 && lds <= kMaxLdsBytes;   // synthesis items per slice: grid y
  return g;
}

// Band analysis of cnt tasks: one launch per work-item class.
template <class T, class Launch>
void launch_band_ana(const KArgs<T>& a, const Geometry<T>& g, const SliceTask* tasks, int64_t cnt,
                     const C2<T>* W2, C2<T>* coef, Launch& L) {
  if (g.mixed) {
    if (g.exa == 8) L.launch(k_band_ana_mx<T, 8>, cnt * g.gxa, g.bxa, g.sxa, a, tasks, W2, coef, 0, g.gxa);
    else L.launch(k_band_ana_mx<T, 16>, cnt * g.gxa, g.bxa, g.sxa, a, tasks, W2, coef, 0, g.gxa);
    return;
  }
  if (g.ga)
    L.launch(k_band_ana<T, kSmallE, kAnaThreads, kSmallWaves, false>, cnt * g.ga, g.ba, g.sa, a, tasks, W2, coef, 0,
             g.ga);
  if (g.gab) {
    if (g.tab)
      L.launch(k_band_ana<T, kBigAnaE, kAnaBigThreads, kSmallWaves, true>, cnt * g.gab, g.bab, g.sab, a, tasks, W2,
               coef, g.ga, g.gab);
    else
      L.launch(k_band_ana<T, kBigAnaE, kAnaBigThreads, kSmallWaves, false>, cnt * g.gab, g.bab, g.sab, a, tasks, W2,
               coef, g.ga, g.gab);
  }
}

// Band synthesis (dual or adjoint) of cnt tasks: one launch per work-item
// class, on a grid of (slices of a tile, items, tiles); balanced tiles of at
// most kSynTile slices (more when 65535 tiles do not cover cnt).
constexpr int64_t kSynTile = 128;

template <class T, class Launch>
void launch_band_syn(const KArgs<T>& a, const Geometry<T>& g, const SliceTask* tasks, int64_t cnt,
                     const C2<T>* coef, C2<T>* W2, T* y, Launch& L) {
  const int64_t tiles = std::min<int64_t>((cnt + kSynTile - 1) / kSynTile, 65535);
  const int64_t tx = tiles ? (cnt + tiles - 1) / tiles : 0;
  const int n = (int)cnt;
  if (g.mixed) {
    if (g.exs == 8) L.launch_xyz(k_band_syn_mx<T, 8>, tx, g.gxs, (int)tiles, g.bxs, g.sxs, a, tasks, coef, W2, y, 0, n);
    else L.launch_xyz(k_band_syn_mx<T, 16>, tx, g.gxs, (int)tiles, g.bxs, g.sxs, a, tasks, coef, W2, y, 0, n);
    return;
  }
  if (g.gs)
    L.launch_xyz(k_band_syn<T, kSmallE, kSynThreads, kSynSmallWaves<T>, false>, tx, g.gs, (int)tiles, g.bs, g.ss, a,
                 tasks, coef, W2, y, 0, n);
  if (g.gsb) {
    if (g.tsb)
      L.launch_xyz(k_band_syn<T, kBigSynE, kSynBigThreads, kSmallWaves, true>, tx, g.gsb, (int)tiles, g.bsb, g.ssb, a,
                   tasks, coef, W2, y, g.gs, n);
    else
      L.launch_xyz(k_band_syn<T, kBigSynE, kSynBigThreads, kSmallWaves, false>, tx, g.gsb, (int)tiles, g.bsb, g.ssb, a,
                   tasks, coef, W2, y, g.gs, n);
  }
}

// One workgroup per slice (fused.hpp): analysis of cnt tasks.
template <class T, class Launch>
void launch_ana_fused(const Plan& p, const KArgs<T>& a, const SliceTask* tasks, int64_t cnt, const T* x, C2<T>* coef,
                      Launch& L) {
  const FusedPlan& f = p.fused[sizeof(T) == 8 ? 1 : 0];
  switch (ilog2i(p.N)) {
    case 5: L.launch(k_ana_fused<T, 5>, cnt, f.nthr, f.lds_bytes, a, tasks, x, coef); break;
    case 6: L.launch(k_ana_fused<T, 6>, cnt, f.nthr, f.lds_bytes, a, tasks, x, coef); break;
    case 12: L.launch(k_ana_fused<T, 12>, cnt, f.nthr, f.lds_bytes, a, tasks, x, coef); break;
    case 13: L.launch(k_ana_fused<T, 13>, cnt, f.nthr, f.lds_bytes, a, tasks, x, coef); break;
    default: L.launch(k_ana_fused<T, 14>, cnt, f.nthr, f.lds_bytes, a, tasks, x, coef); break;
  }
}

// One workgroup per slice: synthesis (or adjoint) of cnt tasks, before the overlap fix-up.
template <class T, class Launch>
void launch_syn_fused(const Plan& p, const KArgs<T>& a, const SliceTask* tasks, int64_t cnt, const C2<T>* coef,
                      C2<T>* W2, T* y, Launch& L) {
  const FusedPlan& f = p.fused[sizeof(T) == 8 ? 1 : 0];
  switch (ilog2i(p.N)) {
    case 5: L.launch(k_syn_fused<T, 5>, cnt, f.nthr, f.lds_bytes, a, tasks, coef, W2, y); break;
    case 6: L.launch(k_syn_fused<T, 6>, cnt, f.nthr, f.lds_bytes, a, tasks, coef, W2, y); break;
    case 12: L.launch(k_syn_fused<T, 12>, cnt, f.nthr, f.lds_bytes, a, tasks, coef, W2, y); break;
    case 13: L.launch(k_syn_fused<T, 13>, cnt, f.nthr, f.lds_bytes, a, tasks, coef, W2, y); break;
    default: L.launch(k_syn_fused<T, 14>, cnt, f.nthr, f.lds_bytes, a, tasks, coef, W2, y); break;
  }
}

// Analysis of tasks [t0, t0 + cnt) (Algorithm 3): slice FFT, band transforms.
template <class T, class Launch>
void launch_analysis(const Plan& p, const KArgs<T>& a, const Geometry<T>& g, const SliceTask* tasks,
                     int64_t cnt, const T* x, C2<T>* coef, C2<T>* W1, C2<T>* W2, Launch& L) {
  if (a.fused) {
    launch_ana_fused(p, a, tasks, cnt, x, coef, L);
    return;
  }
  L.launch(k_fwd_pass1<T, true>, cnt * g.g1, g.b1, g.s1, a, tasks, x, W1);
  L.launch(k_fwd_pass2<T, true>, cnt * g.g2, g.b2, g.s2, a, (const C2<T>*)W1, W2);
  launch_band_ana(a, g, tasks, cnt, (const C2<T>*)W2, coef, L);
}

// Inverse pass B of tasks [t0, t0 + cnt) of the call's task table (tasks
// points at task t0), then the second contributions of the shared samples.
template <class T, class Launch>
void launch_ola_fix(const KArgs<T>& a, const SliceTask* tasks, int64_t cnt, const C2<T>* W2, T* y, Launch& L) {
  const int nov = ola_count(a.N, a.Mt);
  if (nov > 0) L.launch(k_ola_fix<T>, cnt * 2 * ((nov + kOlaFixRun - 1) / kOlaFixRun), 256, 0, a, tasks, W2, y);
}

template <class T, class Launch>
void launch_inv_passB(const KArgs<T>& a0, const Geometry<T>& g, const SliceTask* tasks, int64_t t0, int64_t cnt,
                      C2<T>* W1, C2<T>* W2, T* y, Launch& L) {
  KArgs<T> a = a0;
  a.task0 = t0;
  a.task1 = t0 + cnt;
  if (a.fused) {
    launch_ola_fix(a, tasks, cnt, (const C2<T>*)W2, y, L);     // the fused synthesis wrote the overlap buffers
    return;
  }
  L.launch(k_inv_passB<T, true>, cnt * g.g1, g.b1, g.s1, a, tasks, (const C2<T>*)W1, W2, y);
  launch_ola_fix(a, tasks, cnt, (const C2<T>*)W2, y, L);
}

// Synthesis (or adjoint) of tasks [t0, t0 + cnt) (Algorithm 4); tasks points at task t0.
template <class T, class Launch>
void launch_synthesis(const Plan& p, const KArgs<T>& a0, const Geometry<T>& g, const SliceTask* tasks, int64_t t0,
                      int64_t cnt, const C2<T>* coef, T* y, C2<T>* W1, C2<T>* W2, Launch& L) {
  if (a0.fused) {
    KArgs<T> a = a0;
    a.task0 = t0;
    a.task1 = t0 + cnt;
    launch_syn_fused(p, a, tasks, cnt, coef, W2, y, L);
    launch_ola_fix(a, tasks, cnt, (const C2<T>*)W2, y, L);
    return;
  }
  launch_band_syn(a0, g, tasks, cnt, coef, W2, y, L);
  L.launch(k_inv_passA<T, true>, cnt * g.g2, g.b2, g.s2, a0, (const C2<T>*)W2, W1);
  launch_inv_passB(a0, g, tasks, t0, cnt, W1, W2, y, L);
}

}  // namespace slicq
