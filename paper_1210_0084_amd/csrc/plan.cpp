// FP64 plan: constant-Q band design (Section 3, Table 1), lattice M_k = L/a_k
// (equation framecond1), diagonal frame operator and canonical dual windows
// (Proposition 2), Tukey slicing window and its dual (Section 4.3, equations
// BUPU and dualwincond), and the kernel work schedule.
//
// Readings where the paper is silent: Hann H; bandwidths widened to a
// minimal filter length (Section 5.3); K reduced until xi_K + Omega_K/2 stays
// below Nyquist; plateau DC/Nyquist bands with raised-cosine flanks of width
// Omega_1/2 and Omega_K/2 measured in whole bins from 0 and N; M_k the
// smallest power of two >= |J_k| (and >= 2); canonical slice dual
// h_0 / sum_m T_{mN} h_0^2.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

namespace slicq {

namespace {

constexpr size_t kMaxLdsBytesPlan = 160 * 1024;   // LDS of one gfx950 workgroup

int64_t next_pow2(int64_t n) {
  int64_t p = 1;
  while (p < n) p <<= 1;
  return p;
}

int ilog2(int64_t n) {
  int l = 0;
  while ((int64_t(1) << l) < n) ++l;
  return l;
}

// log2 of the largest power of two dividing n > 0.
int pow2_part_log(int64_t n) {
  int l = 0;
  while (!(n & 1)) {
    n >>= 1;
    ++l;
  }
  return l;
}

// The smallest even number 2^a, 3 2^a or 5 2^a (a >= 1) that is >= n.
int64_t smooth_even(int64_t n) {
  int64_t best = 0;
  for (int64_t r : {1, 3, 5}) {
    int64_t m = 2 * r;
    while (m < n) m *= 2;
    if (!best || m < best) best = m;
  }
  return best;
}

struct RawBand {
  int64_t start = 0;
  std::vector<double> g;
  int64_t M = 0;
  double xi = 0, omega = 0;
};

// Window shape on |x| < 1/2 (x in bandwidths from the centre).
double shape(int window, double x) {
  const double c1 = std::cos(2.0 * M_PI * x);
  if (window == 0) return 0.5 + 0.5 * c1;
  return 0.35875 + 0.48829 * c1 + 0.14128 * std::cos(4.0 * M_PI * x) + 0.01168 * std::cos(6.0 * M_PI * x);
}

// Band with centre xi and bandwidth om (Hz): the bins j whose frequency lies
// strictly inside (xi - om/2, xi + om/2). The end bins come from the closed
// form of that interval, then each end is moved by at most a bin until the
// window argument computed for the table itself decides it.
RawBand cq_band(int window, double fs, int64_t two_n, double xi, double om) {
  const double bin = fs / (double)two_n;
  auto x_of = [&](int64_t j) { return ((double)j * bin - xi) / om; };
  auto inside = [&](int64_t j) {
    const double x = x_of(j);
    return x > -0.5 && x < 0.5;
  };
  RawBand r;
  r.xi = xi;
  r.omega = om;
  int64_t a = (int64_t)std::floor((xi - om / 2) / bin) + 1;   // first bin above the lower edge
  int64_t b = (int64_t)std::ceil((xi + om / 2) / bin) - 1;    // last bin below the upper edge
  if (!inside(a) && inside(a + 1)) ++a;
  else if (inside(a - 1)) --a;
  if (!inside(b) && inside(b - 1)) --b;
  else if (inside(b + 1)) ++b;
  if (b < a || !inside(a) || !inside(b)) {
    r.M = 2;
    return r;
  }
  r.start = a;
  for (int64_t j = a; j <= b; ++j) r.g.push_back(shape(window, x_of(j)));
  r.M = std::max<int64_t>(2, next_pow2(b - a + 1));
  return r;
}

// Frequency scales for the centres: u(f) and its inverse.
double scale_fwd(int scale, double f) {
  return scale == 1 ? 2595.0 * std::log10(1.0 + f / 700.0) : 26.81 * f / (1960.0 + f) - 0.53;
}
double scale_inv(int scale, double u) {
  return scale == 1 ? 700.0 * (std::pow(10.0, u / 2595.0) - 1.0) : 1960.0 * (u + 0.53) / (26.28 - u);
}

// Plateau P(d; R, w) in the distance d (Hz) from centre_bin.
RawBand plateau_band(double fs, int64_t two_n, int64_t centre_bin, double R, double w,
                     double xi, double om) {
  RawBand r;
  r.xi = xi;
  r.omega = om;
  int64_t e = 0;
  while ((double)(e + 1) * fs / (double)two_n < R) ++e;
  r.start = centre_bin - e;
  for (int64_t j = centre_bin - e; j <= centre_bin + e; ++j) {
    int64_t dj = j - centre_bin;
    if (dj < 0) dj = -dj;
    double d = (double)dj * fs / (double)two_n;
    r.g.push_back(d <= R - w ? 1.0 : 0.5 + 0.5 * std::cos(M_PI * (d - R + w) / w));
  }
  r.M = std::max<int64_t>(2, next_pow2(2 * e + 1));
  return r;
}

template <class T>
size_t append(std::vector<unsigned char>& blob, const T* data, size_t n) {
  size_t off = (blob.size() + 255) & ~size_t(255);
  blob.resize(off + n * sizeof(T));
  if (n) std::memcpy(blob.data() + off, data, n * sizeof(T));
  return off;
}

// The per-bin records of the first two overlap-add entries (weights w: two per bin).
template <class T>
std::vector<OlaRec<T>> ola_records(const Plan& p, const std::vector<double>& w) {
  const size_t nb = p.ent2_pos.size() / 4;
  std::vector<OlaRec<T>> r(nb);
  auto y16 = [](int32_t y) { return y < 0 ? kOlaNone : (uint32_t)y; };
  for (size_t j = 0; j < nb; ++j) {
    const int32_t* e = &p.ent2_pos[4 * j];
    const bool more = p.ent_off[j + 1] > p.ent_off[j];
    r[j].xx = (uint32_t)e[0] | ((uint32_t)e[2] << 16) | (more ? kOlaMore : 0u);
    r[j].yy = y16(e[1]) | (y16(e[3]) << 16);
    r[j].w0 = (T)w[2 * j];
    r[j].w1 = (T)w[2 * j + 1];
  }
  return r;
}

// Fused per-slice schedule for one dtype (cb bytes per complex value): the
// half spectrum X[0..N] at LDS indices 0..N, band items in increasing k
// (analysis) and decreasing k (synthesis), each placed at index 0 when it
// fits below every bin its item and the items after it touch (the spectrum
// bins there are dead in analysis and not yet written in synthesis), else
// past the spectrum. ok stays false when the spectrum and the largest item do
// not fit one workgroup's LDS.
void build_fused(const Plan& p, int dtype, FusedPlan& f) {
  f = FusedPlan();
  const int64_t N = p.N;
  const int logN = ilog2(N);
  if (!p.prm.fused || N < 32 || N > 16384) return;
  if (!(logN == 5 || logN == 6 || (logN >= 12 && logN <= 14))) return;   // compiled slice lengths
  if (p.mixed) return;                         // the per-slice kernels transform powers of two only
  const size_t cb = dtype ? 16 : 8;
  const int nb = (int)p.bands.size();
  f.logM = ilog2(p.max_M);
  const size_t tw_bytes = (size_t)(split_tw_entries(logN) + split_tw_entries(std::max(f.logM, 1))) * cb;
  if (tw_bytes + 64 >= kMaxLdsBytesPlan) return;
  // largest index space whose padded array fits beside the twiddle tables
  int64_t cap = (int64_t)((kMaxLdsBytesPlan - tw_bytes - 64) / cb);
  while (cap > 0 && (size_t)padded((int)cap) * cb + tw_bytes + 64 > kMaxLdsBytesPlan) --cap;
  if (cap < N + 1) return;
  const int64_t tail = cap - (N + 1);
  // lowest half-spectrum bin read (analysis) or written (synthesis) by bands >= k
  std::vector<int64_t> sufmin(nb + 1, N + 1);
  for (int k = nb - 1; k >= 0; --k) sufmin[k] = std::min<int64_t>(sufmin[k + 1], p.bands[k].hlo);
  int64_t used = N + 1;
  auto room = [&](int64_t bottom) { return std::min<int64_t>(kFusedMaxItem, std::max(bottom, tail)); };
  // analysis: increasing k
  for (int k = 0; k < nb;) {
    const int32_t M = p.bands[k].M;
    const int64_t r = room(sufmin[k]);
    if (M > r) return;
    int cnt = 1;
    while (k + cnt < nb && p.bands[k + cnt].M == M && (int64_t)(cnt + 1) * M <= r && cnt < kMaxGroupBands) ++cnt;
    FusedItemDev it{};
    it.k0 = k;
    it.cnt = cnt;
    it.M = M;
    it.logM = p.bands[k].logM;
    it.lds = (int64_t)cnt * M <= sufmin[k] ? 0 : (int32_t)(N + 1);
    used = std::max<int64_t>(used, it.lds + (int64_t)cnt * M);
    f.ana.push_back(it);
    k += cnt;
  }
  // synthesis: decreasing k; the bound of an item is set by its lowest band
  std::vector<char> written(N + 1, 0);
  f.ent_off.clear();
  for (int k = nb - 1; k >= 0;) {
    const int32_t M = p.bands[k].M;
    if (M > room(sufmin[k])) return;
    int cnt = 1;
    while (k - cnt >= 0 && p.bands[k - cnt].M == M && (int64_t)(cnt + 1) * M <= room(sufmin[k - cnt]) &&
           cnt < kMaxGroupBands)
      ++cnt;
    const int kl = k - cnt + 1;
    FusedItemDev it{};
    it.k0 = kl;
    it.cnt = cnt;
    it.M = M;
    it.logM = p.bands[kl].logM;
    it.lds = (int64_t)cnt * M <= sufmin[kl] ? 0 : (int32_t)(N + 1);
    used = std::max<int64_t>(used, it.lds + (int64_t)cnt * M);
    int32_t olo = (int32_t)N, ohi = 0;
    for (int b = kl; b <= k; ++b) {
      olo = std::min(olo, p.bands[b].hlo);
      ohi = std::max(ohi, p.bands[b].hhi);
    }
    it.olo = olo;
    it.ohi = ohi;
    it.rec0 = (int32_t)f.rec_xx.size();
    for (int64_t j = olo; j <= ohi; ++j) {
      struct E { int32_t x, y; double ws, wa; };
      std::vector<E> ent;
      for (int b = kl; b <= k; ++b) {            // increasing k: a fixed summation order
        const BandInfo& bi = p.bands[b];
        if (j < bi.hlo || j > bi.hhi) continue;
        const int64_t pos = it.lds + (int64_t)(b - kl) * M;
        const bool selfmirror = (b == 0 || b == p.K + 1);
        const int64_t t = j - bi.start;
        E e;
        e.x = (int32_t)(pos + (j & (M - 1)));
        e.y = selfmirror ? (int32_t)(pos + ((-j) & (M - 1))) : -1;
        e.ws = (selfmirror ? 0.5 : 1.0) * p.gd[bi.goff + t];
        e.wa = 0.5 * p.g[bi.goff + t];
        ent.push_back(e);
      }
      const bool init = !written[j];
      written[j] = 1;
      const int32_t x0 = ent.empty() ? (int32_t)it.lds : ent[0].x;
      const int32_t x1 = ent.size() > 1 ? ent[1].x : x0;
      auto y16 = [](int32_t y) { return y < 0 ? 0xffffu : (uint32_t)y; };
      f.rec_xx.push_back((uint32_t)x0 | ((uint32_t)x1 << 16) | (ent.size() > 2 ? kFMore : 0u) | (init ? kFInit : 0u));
      f.rec_yy.push_back(y16(ent.empty() ? -1 : ent[0].y) | (y16(ent.size() > 1 ? ent[1].y : -1) << 16));
      f.rec_ws.push_back(ent.empty() ? 0.0 : ent[0].ws);
      f.rec_ws.push_back(ent.size() > 1 ? ent[1].ws : 0.0);
      f.rec_wa.push_back(ent.empty() ? 0.0 : ent[0].wa);
      f.rec_wa.push_back(ent.size() > 1 ? ent[1].wa : 0.0);
      f.ent_off.push_back((int32_t)f.ent_ws.size());
      for (size_t q = 2; q < ent.size(); ++q) {
        f.ent_pos.push_back(ent[q].x);
        f.ent_pos.push_back(ent[q].y);
        f.ent_ws.push_back(ent[q].ws);
        f.ent_wa.push_back(ent[q].wa);
      }
    }
    f.syn.push_back(it);
    k = kl - 1;
  }
  f.ent_off.push_back((int32_t)f.ent_ws.size());
  for (int64_t j = 0; j <= N; ++j)
    if (!written[j]) return;                  // every bin must be set by some item
  if (used > kFPos) return;                   // LDS indices must fit the records' 15 bits
  f.cap = (int32_t)used;
  int64_t need = N / (logN >= 14 ? 16 : 8);    // slice FFT: 16 values per thread at 2^14 points, else 8
  for (const FusedItemDev& it : f.ana) need = std::max<int64_t>(need, ((int64_t)it.cnt * it.M + kFusedE - 1) / kFusedE);
  for (const FusedItemDev& it : f.syn) need = std::max<int64_t>(need, ((int64_t)it.cnt * it.M + kFusedE - 1) / kFusedE);
  f.nthr = (int32_t)std::min<int64_t>(kFusedThreads, std::max<int64_t>(64, (need + 63) / 64 * 64));
  f.lds_bytes = ((size_t)padded(f.cap) * cb + 15) / 16 * 16 + tw_bytes;
  f.ok = f.lds_bytes <= kMaxLdsBytesPlan;
}

}  // namespace

int build_plan(const PlanParams& p, Plan& out, std::string& err) {
  const double fs = p.fs, fmin = p.fmin, fmax = p.fmax;
  const int B = p.bins_per_octave;
  const int64_t two_n = p.slice_len, Mt = p.transition;
  char msg[256];
  if (!(fs > 0 && fmin > 0 && fmin < fmax && fmin < fs / 2 && B >= 1)) {
    err = "need fs > 0, 0 < fmin < fmax, fmin < fs/2 and bins_per_octave >= 1";
    return -1;
  }
  if (two_n < 16 || two_n > (int64_t(1) << 20) || (two_n & (two_n - 1))) {
    err = "slice length 2N must be a power of two in [16, 2^20]";
    return -1;
  }
  const int64_t N = two_n / 2;
  if (!(Mt > 0 && Mt < N) || ((N - Mt) & 1)) {
    err = "transition length M needs 0 < M < N and N - M even";
    return -1;
  }
  if (!(p.min_win >= 0) || p.dual_kind < 0 || p.dual_kind > 1 || p.coef_layout < 0 || p.coef_layout > 1) {
    err = "min_win must be >= 0, dual_kind and coef_layout 0 or 1";
    return -1;
  }
  if (p.window < 0 || p.window > 1 || p.scale < 0 || p.scale > 2 || p.slicing < 0 || p.slicing > 1 ||
      p.m_policy < 0 || p.m_policy > 2) {
    err = "window (0 Hann, 1 Blackman-Harris), scale (0 cq, 1 mel, 2 Bark), slicing (0 Tukey, 1 root "
          "Tukey) or m_policy (0 power of two, 1 rectangular, 2 even smooth number) out of range";
    return -1;
  }
  if (p.group_cap < 16 || p.group_cap > 4096 || p.lds_cap < 64 || p.lds_cap > kSynMaxValues ||
      p.pass_cap < 64 || p.pass_cap > 4096 ||
      (p.group_cap & (p.group_cap - 1)) || (p.pass_cap & (p.pass_cap - 1))) {
    err = "group_cap and pass_cap must be powers of two in [16, 4096] and [64, 4096], "
          "lds_cap in [64, 16384]";
    return -1;
  }
  out.prm = p;
  out.two_n = two_n;
  out.N = N;
  out.Mt = Mt;
  const double Q = 1.0 / (std::pow(2.0, 1.0 / B) - std::pow(2.0, -1.0 / B));
  out.Q = Q;

  // centres and bandwidths (Table 1)
  const int K0 = 1 + (int)std::ceil((double)B * std::log2(fmax / fmin) - 1e-12);
  const double bw_min = p.min_win * fs / (double)two_n;
  std::vector<double> xi(K0), om(K0);
  if (p.scale == 0) {
    for (int k = 1; k <= K0; ++k) {
      xi[k - 1] = fmin * std::pow(2.0, (double)(k - 1) / (double)B);
      om[k - 1] = std::max(xi[k - 1] / Q, bw_min);
    }
  } else {
    // K0 centres equally spaced on the mel or Bark scale from fmin to fmax;
    // bandwidth = distance of the two neighbouring centres (xi_k / Q for constant Q)
    const double u0 = scale_fwd(p.scale, fmin), du = (scale_fwd(p.scale, fmax) - u0) / std::max(K0 - 1, 1);
    auto centre = [&](int k) { return scale_inv(p.scale, u0 + (double)(k - 1) * du); };
    for (int k = 1; k <= K0; ++k) {
      xi[k - 1] = centre(k);
      om[k - 1] = std::max(centre(k + 1) - centre(k - 1), bw_min);
    }
  }
  int K = K0;
  while (K >= 1 && !(xi[K - 1] + om[K - 1] / 2 < fs / 2)) --K;
  if (K < 1) {
    err = "no constant-Q band fits below Nyquist";
    return -1;
  }
  out.K0 = K0;
  out.K = K;
  out.nb = K + 2;

  std::vector<RawBand> raw;
  {
    const double R0 = xi[0];
    const double w0 = std::min(om[0] / 2, R0);
    raw.push_back(plateau_band(fs, two_n, 0, R0, w0, 0.0, 2.0 * xi[0]));
    for (int k = 1; k <= K; ++k) raw.push_back(cq_band(p.window, fs, two_n, xi[k - 1], om[k - 1]));
    const double RN = fs / 2 - xi[K - 1];
    const double wN = std::min(om[K - 1] / 2, RN);
    raw.push_back(plateau_band(fs, two_n, N, RN, wN, fs / 2, fs - 2 * xi[K - 1]));
  }
  if (p.m_policy == 1) {       // rectangular: every band takes the largest M
    int64_t Mr = 0;
    for (const RawBand& r : raw) Mr = std::max(Mr, r.M);
    for (RawBand& r : raw) r.M = Mr;
  } else if (p.m_policy == 2) {   // M_k >= |J_k| (equation framecond1), even for Algorithm 3's layers
    for (RawBand& r : raw) r.M = smooth_even(std::max<int64_t>(2, (int64_t)r.g.size()));
  }
  for (int k = 0; k < K + 2; ++k) {
    if (raw[k].g.empty()) {
      std::snprintf(msg, sizeof msg, "band %d has empty support; raise min_win", k);
      err = msg;
      return -1;
    }
  }
  for (int k = 1; k <= K; ++k) {
    const RawBand& r = raw[k];
    if (r.start < 1 || r.start + (int64_t)r.g.size() - 1 > N - 1) {
      err = "a constant-Q band reaches bin 0 or bin N; raise fmin or lower min_win";
      return -1;
    }
  }

  // frame-operator diagonal over all 2K+2 bands (mirrors g_{2K+2-k}[j] = g_k[2N-j])
  out.D.assign(two_n, 0.0);
  auto add_band = [&](int64_t start, const std::vector<double>& g, int64_t M, bool mirror) {
    const int64_t len = (int64_t)g.size();
    for (int64_t t = 0; t < len; ++t) {
      int64_t j, src;
      if (!mirror) {
        j = start + t;
        src = t;
      } else {
        j = -(start + len - 1) + t;
        src = len - 1 - t;
      }
      j %= two_n;
      if (j < 0) j += two_n;
      out.D[j] += (double)M * g[src] * g[src];
    }
  };
  for (int k = 0; k < K + 2; ++k) add_band(raw[k].start, raw[k].g, raw[k].M, false);
  for (int k = K + 2; k < 2 * K + 2; ++k) {
    const RawBand& s = raw[2 * K + 2 - k];
    add_band(s.start, s.g, s.M, true);
  }
  for (int64_t j = 0; j < two_n; ++j) {
    if (!(out.D[j] > 0)) {
      err = "frame condition fails: the frame-operator diagonal has a zero (Proposition 2)";
      return -1;
    }
  }

  // stored bands, windows and duals
  out.bands.clear();
  out.g.clear();
  out.gd.clear();
  int64_t off = 0, goff = 0;
  out.max_M = 0;
  for (int k = 0; k < K + 2; ++k) {
    const RawBand& r = raw[k];
    BandInfo b;
    b.k = k;
    b.start = r.start;
    b.len = (int32_t)r.g.size();
    b.M = (int32_t)r.M;
    b.logM = pow2_part_log(r.M);          // M_k = R 2^logM, R in {1, 3, 5}
    b.off = off;
    b.goff = goff;
    b.xi = r.xi;
    b.omega = r.omega;
    b.hlo = (int32_t)std::max<int64_t>(0, r.start);
    b.hhi = (int32_t)std::min<int64_t>(N, r.start + b.len - 1);
    off += r.M;
    goff += b.len;
    out.max_M = std::max(out.max_M, b.M);
    for (int64_t t = 0; t < b.len; ++t) {
      int64_t j = (r.start + t) % two_n;
      if (j < 0) j += two_n;
      out.g.push_back(r.g[t]);
      out.gd.push_back(r.g[t] / out.D[j]);
    }
    out.bands.push_back(b);
  }
  out.coefs_per_slice = off;
  out.mixed = false;
  out.mix_L = 1;
  for (const BandInfo& b : out.bands)
    if (b.M & (b.M - 1)) {
      out.mixed = true;
      out.mix_L = std::max(out.mix_L, b.logM);
    }
  if (out.max_M > 8192) {
    std::snprintf(msg, sizeof msg, "a band needs M_k = %d coefficients per slice; "
                  "the single-workgroup band transforms support up to 8192", out.max_M);
    err = msg;
    return -1;
  }

  // half-spectrum coverage must be monotone in k for the per-bin gather
  for (int k = 1; k < K + 2; ++k) {
    if (out.bands[k].hlo < out.bands[k - 1].hlo || out.bands[k].hhi < out.bands[k - 1].hhi) {
      err = "band supports are not ordered by frequency";
      return -1;
    }
  }
  out.bin_k0.assign(N + 1, 0);
  out.bin_nk.assign(N + 1, 0);
  {
    int kfirst = 0;
    for (int64_t j = 0; j <= N; ++j) {
      while (kfirst < K + 2 && out.bands[kfirst].hhi < j) ++kfirst;
      int k = kfirst, n = 0;
      while (k + n < K + 2 && out.bands[k + n].hlo <= j) ++n;
      out.bin_k0[j] = k;
      out.bin_nk[j] = n;
      if (n == 0) {
        err = "a bin of [0, N] is covered by no band";
        return -1;
      }
    }
  }

  // Tukey slicing window on t in [-N, N), index j = t + N
  out.h0.assign(two_n, 0.0);
  out.hd.assign(two_n, 0.0);
  const int64_t flat = (N - Mt) / 2;
  for (int64_t j = 0; j < two_n; ++j) {
    int64_t a = j - N;
    if (a < 0) a = -a;
    double h = 0.0;
    if (a <= flat) h = 1.0;
    else if ((double)a < (double)(N + Mt) / 2) h = 0.5 + 0.5 * std::cos(M_PI * (double)(a - flat) / (double)Mt);
    out.h0[j] = p.slicing == 1 ? std::sqrt(h) : h;   // sum_m h_m^2 = 1 for the square root
  }
  for (int64_t j = 0; j < two_n; ++j) {
    const double h = out.h0[j];
    if (h == 0.0) continue;
    if (p.dual_kind == 1) {
      out.hd[j] = 1.0;
    } else {
      double den = h * h;
      if (j >= N) den += out.h0[j - N] * out.h0[j - N];
      else den += out.h0[j + N] * out.h0[j + N];
      out.hd[j] = h / den;
    }
  }

  // four-step factorisation of the N-point complex FFT of a slice
  out.logN1 = ilog2(N) / 2;
  out.logN2 = ilog2(N) - out.logN1;
  out.N1 = 1 << out.logN1;
  out.N2 = 1 << out.logN2;
  out.C = (int32_t)std::min<int64_t>(out.N1, std::max<int64_t>(1, p.pass_cap / out.N2));
  out.P = (int32_t)std::min<int64_t>(out.N2 / 2, std::max<int64_t>(1, p.pass_cap / (2 * out.N1)));

  // analysis work items: consecutive bands of equal M_k, at most group_cap values
  out.ana.clear();
  out.ana_cap = 0;
  for (int k = 0; k < K + 2;) {
    AnaGroupDev gdv{};
    gdv.k0 = k;
    gdv.M = out.bands[k].M;
    gdv.logM = out.bands[k].logM;
    int cnt = 1;
    while (k + cnt < K + 2 && out.bands[k + cnt].M == gdv.M && (cnt + 1) * gdv.M <= p.group_cap &&
           cnt < kMaxGroupBands)
      ++cnt;
    gdv.cnt = cnt;
    out.ana.push_back(gdv);
    out.ana_cap = std::max(out.ana_cap, cnt * gdv.M);
    k += cnt;
  }

  // synthesis work items: own bands ka..kb (equal M_k), owned bins [lo, hi),
  // plus the earlier bands ke..ka-1 that reach into [lo, hi)
  out.syn.clear();
  out.runs.clear();
  out.syn_cap = 0;
  {
    std::vector<std::pair<int, int>> own;   // (ka, kb)
    for (int k = 0; k < K + 2;) {
      const int lo = (k == 0) ? 0 : out.bands[k].hlo;
      int ke = k;
      while (ke > 0 && out.bands[ke - 1].hhi >= lo) --ke;
      int64_t extra = out.bands[k].off - out.bands[ke].off;
      int cnt = 1;
      const int M = out.bands[k].M;
      // own bands are added while the item stays within lds_cap values; the
      // first one is always taken (its item may exceed lds_cap up to kSynMaxValues)
      while (k + cnt < K + 2 && out.bands[k + cnt].M == M &&
             extra + (int64_t)(cnt + 1) * M <= p.lds_cap && k + cnt - ke < kMaxGroupBands)
        ++cnt;
      if (extra + (int64_t)cnt * M > kSynMaxValues || k + cnt - ke > kMaxGroupBands) {
        std::snprintf(msg, sizeof msg, "bins near band %d need more than %d coefficients or %d bands in "
                      "one synthesis work item", k, kSynMaxValues, kMaxGroupBands);
        err = msg;
        return -1;
      }
      own.push_back({k, k + cnt - 1});
      k += cnt;
    }
    for (size_t i = 0; i < own.size(); ++i) {
      const int ka = own[i].first, kb = own[i].second;
      SynGroupDev s{};
      s.lo = (i == 0) ? 0 : out.bands[ka].hlo;
      s.hi = (i + 1 < own.size()) ? out.bands[own[i + 1].first].hlo : (int32_t)(N + 1);
      int ke = ka;
      while (ke > 0 && out.bands[ke - 1].hhi >= s.lo) --ke;
      s.ke = ke;
      s.kb = kb;
      s.run0 = (int32_t)out.runs.size();
      for (int k = ke; k <= kb;) {
        SynRunDev r{};
        r.k0 = k;
        r.M = out.bands[k].M;
        r.logM = out.bands[k].logM;
        r.lds_off = (int32_t)(out.bands[k].off - out.bands[ke].off);
        r.off = (int32_t)out.bands[k].off;
        int c = 1;
        while (k + c <= kb && out.bands[k + c].M == r.M) ++c;
        r.cnt = c;
        out.runs.push_back(r);
        k += c;
      }
      s.nrun = (int32_t)out.runs.size() - s.run0;
      if (s.nrun > kMaxRuns) {
        std::snprintf(msg, sizeof msg, "bins near band %d span %d different M_k (at most %d)", ka, s.nrun,
                      kMaxRuns);
        err = msg;
        return -1;
      }
      s.maxM = 0;
      for (int r = s.run0; r < s.run0 + s.nrun; ++r) s.maxM = std::max(s.maxM, out.runs[r].M);
      for (int r = 0; r < 2; ++r) s.r[r] = r < s.nrun ? out.runs[s.run0 + r] : SynRunDev{};
      s.total = (int32_t)(out.bands[kb].off + out.bands[kb].M - out.bands[ke].off);
      out.syn_cap = std::max(out.syn_cap, s.total);
      out.syn_bands = std::max(out.syn_bands, kb - ke + 1);
      out.syn.push_back(s);
    }
  }

  // small work items first, then the large ones (each class is one launch)
  {
    auto ana_big = [](const AnaGroupDev& G) { return G.cnt * G.M > kAnaSmallValues; };
    auto syn_big = [](const SynGroupDev& G) { return G.total > kSynSmallValues; };
    std::stable_partition(out.ana.begin(), out.ana.end(), [&](const AnaGroupDev& G) { return !ana_big(G); });
    std::stable_partition(out.syn.begin(), out.syn.end(), [&](const SynGroupDev& G) { return !syn_big(G); });
    out.ana_small = out.syn_small = 0;
    out.ana_cap_small = out.ana_cap_big = out.syn_cap_small = out.syn_cap_big = 0;
    out.ana_maxM_small = out.syn_maxM_small = 0;
    for (const AnaGroupDev& G : out.ana) {
      const int32_t v = G.cnt * G.M;
      if (ana_big(G)) {
        out.ana_cap_big = std::max(out.ana_cap_big, v);
      } else {
        ++out.ana_small;
        out.ana_cap_small = std::max(out.ana_cap_small, v);
        out.ana_maxM_small = std::max(out.ana_maxM_small, G.M);
      }
    }
    for (const SynGroupDev& G : out.syn) {
      if (syn_big(G)) {
        out.syn_cap_big = std::max(out.syn_cap_big, G.total);
      } else {
        ++out.syn_small;
        out.syn_cap_small = std::max(out.syn_cap_small, G.total);
        out.syn_maxM_small = std::max(out.syn_maxM_small, G.maxM);
      }
    }
  }

  // frequency overlap-add program: for every bin j of [0, N], in increasing k,
  // the bands covering it with their LDS position inside the owning work item
  out.ent_off.assign(N + 2, 0);
  out.ent_pos.clear();
  out.ent_wsyn.clear();
  out.ent_wadj.clear();
  out.ent2_pos.assign(4 * (N + 1), 0);
  out.ent2_wsyn.assign(2 * (N + 1), 0.0);
  out.ent2_wadj.assign(2 * (N + 1), 0.0);
  for (int64_t j = 0; j <= N; ++j) out.ent2_pos[4 * j + 1] = out.ent2_pos[4 * j + 3] = -1;
  for (const SynGroupDev& G : out.syn) {
    const int64_t base = out.bands[G.ke].off;
    for (int64_t j = G.lo; j < G.hi; ++j) {
      out.ent_off[j] = (int32_t)out.ent_wsyn.size();
      int slot = 0;
      for (int k = out.bin_k0[j]; k < out.bin_k0[j] + out.bin_nk[j]; ++k, ++slot) {
        const BandInfo& b = out.bands[k];
        if (k < G.ke || k > G.kb) {
          err = "synthesis work item misses a band covering one of its bins";
          return -1;
        }
        const int64_t lds = b.off - base;
        const int64_t t = j - b.start;
        const bool selfmirror = (k == 0 || k == K + 1);
        // slot of bin j and, for the self-mirrored bands, of its mirror: the
        // signed bins of J_k, -j around DC and 2N - j around Nyquist (the same
        // slot modulo M_k when M_k divides 2N)
        const int64_t jm = k == 0 ? -j : 2 * N - j;
        const int32_t px = (int32_t)(lds + ((j % b.M) + b.M) % b.M);
        const int32_t py = selfmirror ? (int32_t)(lds + ((jm % b.M) + b.M) % b.M) : -1;
        const double ws = (selfmirror ? 0.5 : 1.0) * out.gd[b.goff + t], wa = 0.5 * out.g[b.goff + t];
        if (slot < 2) {
          out.ent2_pos[4 * j + 2 * slot] = px;
          out.ent2_pos[4 * j + 2 * slot + 1] = py;
          out.ent2_wsyn[2 * j + slot] = ws;
          out.ent2_wadj[2 * j + slot] = wa;
        } else {
          out.ent_pos.push_back(px);
          out.ent_pos.push_back(py);
          out.ent_wsyn.push_back(ws);
          out.ent_wadj.push_back(wa);
        }
      }
    }
  }
  out.ent_off[N + 1] = (int32_t)out.ent_wsyn.size();
  build_fused(out, 0, out.fused[0]);
  build_fused(out, 1, out.fused[1]);
  return 0;
}

void pack_tables(const Plan& p, int dtype, std::vector<unsigned char>& blob, TableLayout& lay) {
  blob.clear();
  const int64_t two_n = p.two_n;
  // twiddle pyramid: entry n + k holds e^{-2 pi i k / n} for n = 1, 2, 4, ..., 2N
  std::vector<double> tw(2 * 2 * two_n, 0.0);
  for (int64_t n = 1; n <= two_n; n <<= 1) {
    for (int64_t k = 0; k < n; ++k) {
      // reduce the angle exactly to the first octant before calling cos/sin
      const double a = 2.0 * M_PI * (double)k / (double)n;
      double c = std::cos(a), s = -std::sin(a);
      if (4 * k == n) { c = 0.0; s = -1.0; }
      if (2 * k == n) { c = -1.0; s = 0.0; }
      if (4 * k == 3 * n) { c = 0.0; s = 1.0; }
      if (8 * k == n) { c = std::sqrt(0.5); s = -std::sqrt(0.5); }
      tw[2 * (n + k)] = c;
      tw[2 * (n + k) + 1] = s;
    }
  }
  // radix-8 rows of the band FFTs: row r of pass Ns holds e^{-2 pi i r k / (8 Ns)}
  // (entry r k of pyramid level 8 Ns), k < Ns
  std::vector<double> tw8;
  for (int64_t ns : {8, 64})
    for (int64_t r = 1; r < 8; ++r)
      for (int64_t k = 0; k < ns; ++k) {
        const int64_t e = 8 * ns + r * k;
        tw8.push_back(8 * ns <= two_n ? tw[2 * e] : 1.0);
        tw8.push_back(8 * ns <= two_n ? tw[2 * e + 1] : 0.0);
      }
  // dual windows weighted for the adjoint of synthesis: 2 g~_k on bands 1..K
  // (each synthesises also through its mirror), g~_k on the DC and Nyquist bands
  std::vector<double> gdw_d(p.gd);
  for (const BandInfo& b : p.bands)
    if (b.k >= 1 && b.k <= p.K)
      for (int32_t t = 0; t < b.len; ++t) gdw_d[b.goff + t] *= 2.0;
  std::vector<BandDev> bd;
  for (const BandInfo& b : p.bands) {
    BandDev d{};
    d.start = (int32_t)b.start;
    d.len = b.len;
    d.M = b.M;
    d.logM = b.logM;
    d.off = (int32_t)b.off;
    d.goff = (int32_t)b.goff;
    d.hlo = b.hlo;
    d.hhi = b.hhi;
    bd.push_back(d);
  }
  if (dtype == 0) {
    auto cvt = [](const std::vector<double>& v) {
      std::vector<float> f(v.size());
      for (size_t i = 0; i < v.size(); ++i) f[i] = (float)v[i];
      return f;
    };
    std::vector<float> twf = cvt(tw), h0 = cvt(p.h0), hd = cvt(p.hd), g = cvt(p.g), gd = cvt(p.gd), gdw = cvt(gdw_d);
    lay.tw = append(blob, twf.data(), twf.size());
    const std::vector<float> tw8f = cvt(tw8);
    lay.tw8 = append(blob, tw8f.data(), tw8f.size());
    lay.h0 = append(blob, h0.data(), h0.size());
    lay.hd = append(blob, hd.data(), hd.size());
    lay.g = append(blob, g.data(), g.size());
    lay.gd = append(blob, gd.data(), gd.size());
    lay.gdw = append(blob, gdw.data(), gdw.size());
  } else {
    lay.tw = append(blob, tw.data(), tw.size());
    lay.tw8 = append(blob, tw8.data(), tw8.size());
    lay.h0 = append(blob, p.h0.data(), p.h0.size());
    lay.hd = append(blob, p.hd.data(), p.hd.size());
    lay.g = append(blob, p.g.data(), p.g.size());
    lay.gd = append(blob, p.gd.data(), p.gd.size());
    lay.gdw = append(blob, gdw_d.data(), gdw_d.size());
  }
  lay.bands = append(blob, bd.data(), bd.size());
  lay.ana = append(blob, p.ana.data(), p.ana.size());
  lay.syn = append(blob, p.syn.data(), p.syn.size());
  lay.runs = append(blob, p.runs.data(), p.runs.size());
  lay.ent_off = append(blob, p.ent_off.data(), p.ent_off.size());
  // overflow entries: keep at least one element so every table has an address
  std::vector<int32_t> epos = p.ent_pos;
  std::vector<double> ews = p.ent_wsyn, ewa = p.ent_wadj;
  if (ews.empty()) { epos = {0, -1}; ews = {0.0}; ewa = {0.0}; }
  lay.ent_pos = append(blob, epos.data(), epos.size());
  if (dtype == 0) {
    std::vector<float> ws(ews.begin(), ews.end()), wa(ewa.begin(), ewa.end());
    const std::vector<OlaRec<float>> rs = ola_records<float>(p, p.ent2_wsyn), ra = ola_records<float>(p, p.ent2_wadj);
    lay.ola_syn = append(blob, rs.data(), rs.size());
    lay.ola_adj = append(blob, ra.data(), ra.size());
    lay.ent_wsyn = append(blob, ws.data(), ws.size());
    lay.ent_wadj = append(blob, wa.data(), wa.size());
  } else {
    const std::vector<OlaRec<double>> rs = ola_records<double>(p, p.ent2_wsyn), ra = ola_records<double>(p, p.ent2_wadj);
    lay.ola_syn = append(blob, rs.data(), rs.size());
    lay.ola_adj = append(blob, ra.data(), ra.size());
    lay.ent_wsyn = append(blob, ews.data(), ews.size());
    lay.ent_wadj = append(blob, ewa.data(), ewa.size());
  }
  // fused per-slice schedule of this dtype (tables with at least one element each)
  {
    const FusedPlan& f = p.fused[dtype];
    std::vector<FusedItemDev> fa = f.ana, fs = f.syn;
    if (fa.empty()) fa.resize(1);
    if (fs.empty()) fs.resize(1);
    lay.fana = append(blob, fa.data(), fa.size());
    lay.fsyn = append(blob, fs.data(), fs.size());
    std::vector<int32_t> eo = f.ent_off, ep = f.ent_pos;
    std::vector<double> ws = f.ent_ws, wa = f.ent_wa;
    if (eo.empty()) eo = {0};
    if (ws.empty()) { ep = {0, -1}; ws = {0.0}; wa = {0.0}; }
    lay.fent_off = append(blob, eo.data(), eo.size());
    lay.fent_pos = append(blob, ep.data(), ep.size());
    const size_t nrec = std::max<size_t>(f.rec_xx.size(), 1);
    auto recs = [&](const std::vector<double>& w, auto tag) {
      using T = decltype(tag);
      std::vector<FOlaRec<T>> r(nrec);
      for (size_t i = 0; i < f.rec_xx.size(); ++i) r[i] = {f.rec_xx[i], f.rec_yy[i], (T)w[2 * i], (T)w[2 * i + 1]};
      return r;
    };
    if (dtype == 0) {
      const std::vector<FOlaRec<float>> rs = recs(f.rec_ws, 0.0f), ra = recs(f.rec_wa, 0.0f);
      lay.fola_syn = append(blob, rs.data(), rs.size());
      lay.fola_adj = append(blob, ra.data(), ra.size());
      std::vector<float> wsf(ws.begin(), ws.end()), waf(wa.begin(), wa.end());
      lay.fent_wsyn = append(blob, wsf.data(), wsf.size());
      lay.fent_wadj = append(blob, waf.data(), waf.size());
    } else {
      const std::vector<FOlaRec<double>> rs = recs(f.rec_ws, 0.0), ra = recs(f.rec_wa, 0.0);
      lay.fola_syn = append(blob, rs.data(), rs.size());
      lay.fola_adj = append(blob, ra.data(), ra.size());
      lay.fent_wsyn = append(blob, ws.data(), ws.size());
      lay.fent_wadj = append(blob, wa.data(), wa.size());
    }
  }
  // mixed-radix tables: combination twiddles e^{-2 pi i k / M}, M = R 2^l,
  // and (-start_k) mod M_k per band
  {
    const int L = p.mix_L;
    std::vector<double> tm(2 * (size_t)mix_tw_base(5, L + 1, L), 0.0);
    if (p.mixed)
      for (int R : {3, 5})
        for (int l = 1; l <= L; ++l) {
          const int64_t M = (int64_t)R << l, b0 = mix_tw_base(R, l, L);
          for (int64_t k = 0; k < M; ++k) {
            const double a = 2.0 * M_PI * (double)k / (double)M;
            tm[2 * (b0 + k)] = std::cos(a);
            tm[2 * (b0 + k) + 1] = -std::sin(a);
          }
        }
    std::vector<int32_t> sm;
    for (const BandInfo& b : p.bands) sm.push_back((int32_t)(((-b.start) % b.M + b.M) % b.M));
    if (dtype == 0) {
      std::vector<float> tf(tm.begin(), tm.end());
      lay.twmix = append(blob, tf.data(), tf.size());
    } else {
      lay.twmix = append(blob, tm.data(), tm.size());
    }
    lay.bsmod = append(blob, sm.data(), sm.size());
  }
  blob.resize((blob.size() + 255) & ~size_t(255));
  lay.total = blob.size();
}

int build_full(const Plan& p, int64_t L, int lattice, FullPlan& out, std::string& err) {
  const double fs = p.prm.fs;
  if (lattice < 0 || lattice > 1) {
    err = "lattice must be 0 (sliCQ hops) or 1 (painless)";
    return -1;
  }
  if (L < p.two_n || (L & (L - 1)) || L > (int64_t(1) << (2 * kLongLog))) {
    err = "L must be a power of two, at least the slice length 2N and at most 2^24";
    return -1;
  }
  if (lattice == 0 && p.mixed) {
    err = "the sliCQ lattice of a plan with M_k = 3 2^a or 5 2^a needs mixed-radix transforms of length L; "
          "use the painless lattice";
    return -1;
  }
  const int64_t r = L / p.two_n;
  const int K = p.K;
  out.L = L;
  out.two_n = p.two_n;
  out.logL = ilog2(L);
  out.lattice = lattice;
  out.nb = 2 * K + 2;
  // the slice plan's bands (centres, bandwidths after widening, plateau
  // radii and flanks in Hz) sampled on the L-point grid
  std::vector<RawBand> raw;
  {
    const double R0 = p.bands[1].xi, w0 = std::min(p.bands[1].omega / 2, R0);
    raw.push_back(plateau_band(fs, L, 0, R0, w0, 0.0, 2.0 * R0));
    for (int k = 1; k <= K; ++k) raw.push_back(cq_band(p.prm.window, fs, L, p.bands[k].xi, p.bands[k].omega));
    const double RN = fs / 2 - p.bands[K].xi, wN = std::min(p.bands[K].omega / 2, RN);
    raw.push_back(plateau_band(fs, L, L / 2, RN, wN, fs / 2, fs - 2 * p.bands[K].xi));
  }
  for (int k = 0; k < K + 2; ++k) {
    if (raw[k].g.empty()) {
      err = "a band has no bin on the L-point grid";
      return -1;
    }
    if (lattice == 0) raw[k].M = (int64_t)p.bands[k].M * r;
  }
  if (lattice == 1 && p.prm.m_policy == 1) {
    int64_t Mr = 0;
    for (const RawBand& b : raw) Mr = std::max(Mr, b.M);
    for (RawBand& b : raw) b.M = Mr;
  }
  // mirrors K+2 .. 2K+1 of bands K .. 1: reversed supports, reversed windows
  for (int k = K + 2; k < 2 * K + 2; ++k) {
    const RawBand& s = raw[2 * K + 2 - k];
    RawBand m;
    m.start = -(s.start + (int64_t)s.g.size() - 1);
    m.g.assign(s.g.rbegin(), s.g.rend());
    m.M = s.M;
    raw.push_back(m);
  }
  auto wrap = [L](int64_t j) {
    j %= L;
    return j < 0 ? j + L : j;
  };
  out.D.assign(L, 0.0);
  out.painless = true;
  out.max_M = 0;
  for (const RawBand& b : raw) {
    for (size_t t = 0; t < b.g.size(); ++t) out.D[wrap(b.start + (int64_t)t)] += (double)b.M * b.g[t] * b.g[t];
    if ((int64_t)b.g.size() > b.M) out.painless = false;
    if (b.M > (int64_t(1) << (2 * kLongLog))) {
      err = "a band's coefficient count exceeds 2^24";
      return -1;
    }
    out.max_M = std::max(out.max_M, b.M);
  }
  for (int64_t j = 0; j < L; ++j)
    if (!(out.D[j] > 0)) {
      err = "frame condition fails on the L-point grid: the frame-operator diagonal has a zero";
      return -1;
    }
  out.bands.clear();
  out.g.clear();
  out.runs.clear();
  int64_t off = 0, goff = 0;
  for (size_t k = 0; k < raw.size(); ++k) {
    const RawBand& b = raw[k];
    FullBandDev d{};
    d.start = b.start;
    d.off = off;
    d.goff = goff;
    d.len = (int32_t)b.g.size();
    d.M = (int32_t)b.M;
    out.bands.push_back(d);
    out.g.insert(out.g.end(), b.g.begin(), b.g.end());
    if (!out.runs.empty() && (int64_t(1) << out.runs.back().logn) == b.M) ++out.runs.back().count;
    else out.runs.push_back(FullRun{off, 1, ilog2(b.M)});
    off += b.M;
    goff += d.len;
  }
  out.coef_count = off;
  if (off >= (int64_t(1) << 31) || goff >= (int64_t(1) << 31)) {
    err = "coefficient count or synthesis entries reach 2^31";
    return -1;
  }
  // synthesis entries sorted by bin (counting sort), bands in increasing order
  out.ent_off.assign(L + 1, 0);
  for (const FullBandDev& b : out.bands)
    for (int32_t t = 0; t < b.len; ++t) ++out.ent_off[wrap(b.start + t) + 1];
  for (int64_t j = 0; j < L; ++j) out.ent_off[j + 1] += out.ent_off[j];
  out.ent_idx.assign(goff, 0);
  out.ent_w.assign(goff, 0.0);
  std::vector<int32_t> fill(out.ent_off.begin(), out.ent_off.end() - 1);
  for (const FullBandDev& b : out.bands)
    for (int32_t t = 0; t < b.len; ++t) {
      const int64_t j = wrap(b.start + t);
      int64_t q = (b.start + t) % b.M;
      if (q < 0) q += b.M;
      const int32_t e = fill[j]++;
      out.ent_idx[e] = (int32_t)(b.off + q);
      out.ent_w[e] = out.g[b.goff + t] / out.D[j];
    }
  return 0;
}

void pack_full_tables(const FullPlan& f, int dtype, std::vector<unsigned char>& blob, FullLayout& lay) {
  blob.clear();
  // twiddle pyramid of the one-block transforms: entry n + k holds e^{-2 pi i k / n}, n <= kLongVals
  std::vector<double> tw(4 * kLongVals, 0.0);
  for (int64_t n = 1; n <= kLongVals; n <<= 1)
    for (int64_t k = 0; k < n; ++k) {
      const double a = 2.0 * M_PI * (double)k / (double)n;
      double c = std::cos(a), s = -std::sin(a);
      if (4 * k == n) { c = 0.0; s = -1.0; }
      if (2 * k == n) { c = -1.0; s = 0.0; }
      if (4 * k == 3 * n) { c = 0.0; s = 1.0; }
      if (8 * k == n) { c = std::sqrt(0.5); s = -std::sqrt(0.5); }
      tw[2 * (n + k)] = c;
      tw[2 * (n + k) + 1] = s;
    }
  lay.bands = append(blob, f.bands.data(), f.bands.size());
  // run tables: the signal (one transform of length L), then the band runs,
  // each split into short and long runs with their blocks numbered
  auto runset = [&](const std::vector<FullRun>& runs) {
    std::vector<FullRunDev> sm, lg;
    FullRunSet rs;
    for (const FullRun& r : runs) {
      FullRunDev d{};
      d.off = r.off;
      d.count = r.count;
      d.logn = r.logn;
      if (r.logn <= kLongLog) {
        const int64_t per = kLongVals >> r.logn;
        d.blk0 = rs.blk_small;
        rs.blk_small += (r.count + per - 1) / per;
        sm.push_back(d);
      } else {
        d.blk0 = rs.blk_large;
        rs.blk_large += (int64_t)r.count << (r.logn - kLongLog);
        lg.push_back(d);
      }
    }
    rs.nsmall = (int32_t)sm.size();
    rs.nlarge = (int32_t)lg.size();
    if (sm.empty()) sm.resize(1);
    if (lg.empty()) lg.resize(1);
    rs.small = append(blob, sm.data(), sm.size());
    rs.large = append(blob, lg.data(), lg.size());
    return rs;
  };
  lay.sig = runset({FullRun{0, 1, f.logL}});
  lay.bandruns = runset(f.runs);
  lay.ent_off = append(blob, f.ent_off.data(), f.ent_off.size());
  lay.ent_idx = append(blob, f.ent_idx.data(), f.ent_idx.size());
  if (dtype == 0) {
    auto cvt = [](const std::vector<double>& v) {
      std::vector<float> o(v.size());
      for (size_t i = 0; i < v.size(); ++i) o[i] = (float)v[i];
      return o;
    };
    const std::vector<float> g = cvt(f.g), w = cvt(f.ent_w), t = cvt(tw);
    lay.g = append(blob, g.data(), g.size());
    lay.ent_w = append(blob, w.data(), w.size());
    lay.tw = append(blob, t.data(), t.size());
  } else {
    lay.g = append(blob, f.g.data(), f.g.size());
    lay.ent_w = append(blob, f.ent_w.data(), f.ent_w.size());
    lay.tw = append(blob, tw.data(), tw.size());
  }
  blob.resize((blob.size() + 255) & ~size_t(255));
  lay.total = blob.size();
}

}  // namespace slicq
