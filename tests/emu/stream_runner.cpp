// CPU emulation runner for the streaming server (test harness only): the
// library's StreamServer scheduler and kernels driven by a host backend
// (heap buffers, memcpy, thread-per-lane kernel emulation).
//
// usage: stream_runner DTYPE fs fmin fmax B 2N M min_win max_streams max_batch budget hop mode IN OUT
//   IN : n_streams, lengths[n], then each stream's samples (float64)
//   mode 0: every stream in the mix; mode k > 0: only stream k-1, alone
//   OUT: each selected stream's first T output samples (float64), then stats
//        (admitted, rejected, slices, ticks)
// Scenario: per round, every stream pushes its next hop, one tick runs, every
// stream polls. After the input, zeros flush the tail. Stream 0 also takes a
// snapshot at round 3 and the run checks that restoring it into a new stream
// and replaying the rest reproduces stream 0's output bit for bit.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "stream_server.hpp"

thread_local dim3 threadIdx, blockIdx, blockDim, gridDim;
thread_local std::barrier<>* emu_barrier = nullptr;

namespace slicq {
constexpr size_t EMU_LDS = 1 << 20;
alignas(64) unsigned char smem[EMU_LDS];
}  // namespace slicq

namespace {

struct EmuBackend {
  void* dmalloc(size_t n) { return std::calloc(n + 64, 1); }
  void dfree(void* p) { std::free(p); }
  void* hmalloc(size_t n) { return std::calloc(n + 64, 1); }
  void hfree(void* p) { std::free(p); }
  void h2d(void* d, const void* h, size_t n) { std::memcpy(d, h, n); }
  void d2h(void* h, const void* d, size_t n) { std::memcpy(h, d, n); }
  template <class K, class... A>
  void launch(K kernel, int64_t grid, int block, size_t shmem, A... args) {
    launch_xyz(kernel, grid, 1, 1, block, shmem, args...);
  }
  template <class K, class... A>
  void launch_xyz(K kernel, int64_t gx, int gy, int gz, int block, size_t shmem, A... args) {
    if (gx <= 0 || gy <= 0 || gz <= 0) return;
    if (shmem > slicq::EMU_LDS || block <= 0 || block > 1024) std::exit(3);
    for (int64_t b = 0; b < gx * gy * gz; ++b) {
      std::memset(slicq::smem, 0xff, slicq::EMU_LDS);
      std::barrier<> bar(block);
      std::vector<std::thread> th;
      for (int t = 0; t < block; ++t) {
        th.emplace_back([&, t] {
          threadIdx = dim3((unsigned)t);
          blockIdx = dim3((unsigned)(b % gx), (unsigned)(b / gx % gy), (unsigned)(b / (gx * gy)));
          blockDim = dim3((unsigned)block);
          gridDim = dim3((unsigned)gx, (unsigned)gy, (unsigned)gz);
          emu_barrier = &bar;
          kernel(args...);
        });
      }
      for (auto& x : th) x.join();
    }
  }
  bool sync() { return true; }
};

template <class T>
int run(slicq::Plan& plan, int dt, int max_streams, int max_batch, size_t budget, int64_t hop, int mode,
        const std::vector<double>& in, const char* outpath) {
  using namespace slicq;
  std::vector<unsigned char> blob;
  pack_tables(plan, dt, blob, plan.layout[dt]);
  plan.dev[dt] = blob.data();
  EmuBackend be;
  StreamServer<T, EmuBackend> srv(plan, dt, be, max_streams, max_batch, budget);
  std::string err;
  if (!srv.init(err)) {
    std::fprintf(stderr, "init: %s\n", err.c_str());
    return 10;
  }
  size_t pos = 0;
  const int ns = (int)in[pos++];
  std::vector<int64_t> len(ns);
  for (int i = 0; i < ns; ++i) len[i] = (int64_t)in[pos++];
  std::vector<std::vector<T>> x(ns);
  for (int i = 0; i < ns; ++i) {
    for (int64_t t = 0; t < len[i]; ++t) x[i].push_back((T)in[pos++]);
  }
  std::vector<int> sel;
  for (int i = 0; i < ns; ++i)
    if (mode == 0 || mode - 1 == i) sel.push_back(i);
  std::vector<int> id(ns, -1);
  for (int i : sel) {
    id[i] = srv.open();
    if (id[i] < 0) {
      std::fprintf(stderr, "admission refused for stream %d\n", i);
      return 11;
    }
  }
  const int64_t flush = plan.N + plan.Mt;
  std::vector<std::vector<T>> y(ns);
  std::vector<int64_t> fed(ns, 0);
  std::vector<unsigned char> snap;
  int64_t snap_fed = -1, min_out8 = -1;
  bool more = true;
  for (int round = 0; more; ++round) {
    more = false;
    for (int i : sel) {
      const int64_t total = len[i] + flush;
      if (fed[i] >= total) continue;
      const int64_t n = std::min(hop, total - fed[i]);
      std::vector<T> h(n, T(0));
      for (int64_t t = 0; t < n; ++t)
        if (fed[i] + t < len[i]) h[t] = x[i][fed[i] + t];
      srv.push(id[i], h.data(), n);
      fed[i] += n;
      more = more || fed[i] < total;
    }
    if (srv.tick() < 0) return 12;
    for (int i : sel) {
      std::vector<T> buf(1 << 16);
      int64_t got;
      while ((got = srv.poll(id[i], buf.data(), (int64_t)buf.size())) > 0) y[i].insert(y[i].end(), buf.begin(), buf.begin() + got);
    }
    if (round == 3 && id[sel[0]] >= 0) {
      if (!srv.snapshot(id[sel[0]], snap)) return 13;
      snap_fed = fed[sel[0]];
    }
    if (round == 8) {                       // progress of the least served stream so far
      min_out8 = (int64_t)1 << 62;
      for (int i : sel) min_out8 = std::min<int64_t>(min_out8, (int64_t)y[i].size());
    }
  }
  // drain: slices still queued when max_batch was below the arrival rate
  for (int64_t n = 1; n > 0;) {
    n = srv.tick();
    if (n < 0) return 12;
    for (int i : sel) {
      std::vector<T> buf(1 << 16);
      int64_t got;
      while ((got = srv.poll(id[i], buf.data(), (int64_t)buf.size())) > 0) y[i].insert(y[i].end(), buf.begin(), buf.begin() + got);
    }
  }
  // replay stream sel[0] from its snapshot in a fresh slot and compare the rest
  if (snap_fed >= 0) {
    const int i = sel[0];
    const int rid = srv.open();
    if (rid < 0) return 14;
    if (!srv.restore(rid, snap.data(), snap.size())) return 15;
    std::vector<T> ry;
    int64_t f = snap_fed;
    const int64_t total = len[i] + flush;
    while (f < total) {
      const int64_t n = std::min(hop, total - f);
      std::vector<T> h(n, T(0));
      for (int64_t t = 0; t < n; ++t)
        if (f + t < len[i]) h[t] = x[i][f + t];
      srv.push(rid, h.data(), n);
      f += n;
      if (srv.tick() < 0) return 12;
      std::vector<T> buf(1 << 16);
      int64_t got;
      while ((got = srv.poll(rid, buf.data(), (int64_t)buf.size())) > 0) ry.insert(ry.end(), buf.begin(), buf.begin() + got);
    }
    // the restored stream resumes with the original's queued output; compare tails
    if (ry.size() > y[i].size()) return 16;
    const size_t off = y[i].size() - ry.size();
    if (std::memcmp(ry.data(), y[i].data() + off, ry.size() * sizeof(T)) != 0) {
      std::fprintf(stderr, "restored stream diverged\n");
      return 17;
    }
    srv.close(rid);
  }
  FILE* f = std::fopen(outpath, "wb");
  for (int i : sel) {
    if ((int64_t)y[i].size() < len[i]) {
      std::fprintf(stderr, "stream %d produced %zu of %lld samples\n", i, y[i].size(), (long long)len[i]);
      return 18;
    }
    for (int64_t t = 0; t < len[i]; ++t) {
      double v = (double)y[i][t];
      std::fwrite(&v, sizeof v, 1, f);
    }
  }
  const StreamStats st = srv.stats();
  double stv[5] = {(double)st.admitted, (double)st.rejected, (double)st.slices, (double)st.ticks, (double)min_out8};
  std::fwrite(stv, sizeof stv, 1, f);
  std::fclose(f);
  return 0;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 16) {
    std::fprintf(stderr, "usage: %s DTYPE fs fmin fmax B 2N M min_win max_streams max_batch budget hop mode IN OUT\n",
                 argv[0]);
    return 2;
  }
  const int dt = std::atoi(argv[1]);
  slicq::PlanParams pp;
  pp.fs = std::atof(argv[2]);
  pp.fmin = std::atof(argv[3]);
  pp.fmax = std::atof(argv[4]);
  pp.bins_per_octave = std::atoi(argv[5]);
  pp.slice_len = std::atoll(argv[6]);
  pp.transition = std::atoll(argv[7]);
  pp.min_win = std::atof(argv[8]);
  slicq::Plan plan;
  std::string err;
  if (slicq::build_plan(pp, plan, err)) {
    std::fprintf(stderr, "plan: %s\n", err.c_str());
    return 8;
  }
  std::vector<double> in;
  {
    FILE* f = std::fopen(argv[14], "rb");
    double d;
    while (std::fread(&d, sizeof d, 1, f) == 1) in.push_back(d);
    std::fclose(f);
  }
  const int ms = std::atoi(argv[9]), mb = std::atoi(argv[10]);
  const size_t budget = (size_t)std::atoll(argv[11]);
  const int64_t hop = std::atoll(argv[12]);
  const int mode = std::atoi(argv[13]);
  return dt == 0 ? run<float>(plan, dt, ms, mb, budget, hop, mode, in, argv[15])
                 : run<double>(plan, dt, ms, mb, budget, hop, mode, in, argv[15]);
}
