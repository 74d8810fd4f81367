// CPU emulation runner for the sliCQ kernels (test harness only).
//
// Compiles the library's own kernel and pipeline headers against the
// thread-per-lane stand-in in tests/emu/include and runs one transform on
// host memory, so the CPU tests can check the kernels' index arithmetic and
// results against the FP64 oracle without a GPU. Global buffers are exact-size
// heap allocations (AddressSanitizer catches out-of-bounds accesses); the
// emulated LDS is filled with NaN before every block and its bytes past the
// launch's dynamic size are checked after every block.
//
// usage: emu_runner OP DTYPE fs fmin fmax B 2N M min_win dual group_cap lds_cap pass_cap chunk layout fused m_policy IN OUT
//   OP: ana | syn | adj       IN: T then T doubles (ana) / S*C complex doubles (syn, adj)
//       bana | bsyn | badj    IN: nsig, lengths[nsig], then samples or coefficients, packed
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "pipeline.hpp"

thread_local dim3 threadIdx, blockIdx, blockDim, gridDim;
thread_local std::barrier<>* emu_barrier = nullptr;

namespace slicq {
constexpr size_t EMU_LDS = 1 << 20;
alignas(64) unsigned char smem[EMU_LDS];
}  // namespace slicq

namespace {

struct EmuLaunch {
  template <class K, class... A>
  void launch(K kernel, int64_t grid, int block, size_t shmem, A... args) {
    launch_xyz(kernel, grid, 1, 1, block, shmem, args...);
  }
  template <class K, class... A>
  void launch_xyz(K kernel, int64_t gx, int gy, int gz, int block, size_t shmem, A... args) {
    if (gx <= 0 || gy <= 0 || gz <= 0) return;
    if (shmem > slicq::EMU_LDS || block <= 0 || block > 1024) {
      std::fprintf(stderr, "bad launch: block %d shmem %zu\n", block, shmem);
      std::exit(3);
    }
    for (int64_t b = 0; b < gx * gy * gz; ++b) {
      std::memset(slicq::smem, 0xff, slicq::EMU_LDS);
      std::barrier<> bar(block);
      std::vector<std::thread> th;
      th.reserve(block);
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
      for (size_t i = shmem; i < slicq::EMU_LDS; ++i) {
        if (slicq::smem[i] != 0xff) {
          std::fprintf(stderr, "LDS write past the %zu-byte allocation at byte %zu (block %lld)\n", shmem, i,
                       (long long)b);
          std::exit(4);
        }
      }
    }
  }
};

std::vector<double> read_all(const char* path) {
  FILE* f = std::fopen(path, "rb");
  if (!f) std::exit(5);
  std::vector<double> v;
  double d;
  while (std::fread(&d, sizeof d, 1, f) == 1) v.push_back(d);
  std::fclose(f);
  return v;
}

template <class T>
int run(const std::string& op, slicq::Plan& p, int dt, int64_t chunk_req, const std::vector<double>& in,
        const char* outpath) {
  using namespace slicq;
  std::vector<unsigned char> blob;
  pack_tables(p, dt, blob, p.layout[dt]);
  std::vector<unsigned char> tables(blob);          // exact-size "device" copy
  p.dev[dt] = tables.data();
  const bool batched = op[0] == 'b';
  const std::string kind = batched ? op.substr(1) : op;
  const int64_t cps = p.coefs_per_slice;

  // signal lengths and offsets
  std::vector<int64_t> lens;
  size_t pos = 0;
  if (batched) {
    const int64_t nsig = (int64_t)in[pos++];
    for (int64_t b = 0; b < nsig; ++b) lens.push_back((int64_t)in[pos++]);
  } else {
    lens.push_back((int64_t)in[pos++]);
  }
  const int32_t nsig = (int32_t)lens.size();
  std::vector<int64_t> x_off(nsig + 1, 0), c_off(nsig, 0);
  int64_t total = 0, ccount = 0;
  for (int32_t b = 0; b < nsig; ++b) {
    const int64_t S = lens[b] > 0 ? 2 * ((lens[b] + p.two_n - 1) / p.two_n) : 0;
    x_off[b + 1] = x_off[b] + lens[b];
    c_off[b] = ccount;
    ccount += S * cps;
    total += S;
  }
  const int64_t xlen = x_off[nsig];
  std::vector<T> x(std::max<int64_t>(xlen, 1), T(0));
  std::vector<C2<T>> coef(std::max<int64_t>(ccount, 1));
  if (kind == "ana") {
    for (int64_t i = 0; i < xlen; ++i) x[i] = (T)in[pos + i];
  } else {
    for (int64_t i = 0; i < ccount; ++i) coef[i] = {(T)in[pos + 2 * i], (T)in[pos + 2 * i + 1]};
    for (int64_t i = 0; i < xlen; ++i) x[i] = (T)12345.0;   // synthesis must overwrite all of y
  }
  if (total == 0) {
    FILE* f = std::fopen(outpath, "wb");
    std::fclose(f);
    return 0;
  }
  const int64_t chunk = chunk_req > 0 ? std::min(chunk_req, total) : total;
  size_t wbytes = tasks_bytes(total) + 256 + 2 * 256 + (size_t)chunk * slice_scratch_bytes(p, dt);
  std::vector<unsigned char> work(wbytes);
  WorkLayout w;
  if (!work_layout(p, dt, total, wbytes, w)) return 6;
  auto* tasks = reinterpret_cast<SliceTask*>(work.data() + w.tasks_off);
  auto* status = reinterpret_cast<int32_t*>(work.data() + w.status_off);
  EmuLaunch L;
  if (batched) {
    L.launch(k_tasks_batched, 1, 1024, 1026 * sizeof(int64_t), tasks, (const int64_t*)x_off.data(),
             (const int64_t*)c_off.data(), nsig, (int64_t)p.N, total, xlen, ccount, cps, status);
    if (status[0] != 0 || status[1] != total) {
      std::fprintf(stderr, "task builder status %d %d (expected 0 %lld)\n", status[0], status[1], (long long)total);
      return 7;
    }
  } else {
    L.launch(k_tasks_plain, (total + 255) / 256, 256, 0, tasks, (int64_t)0, total, lens[0], (int64_t)p.N, total);
  }
  C2<T>* W1 = reinterpret_cast<C2<T>*>(work.data() + w.w1_off);
  C2<T>* W2 = reinterpret_cast<C2<T>*>(work.data() + w.w2_off);
  const Geometry<T> g = geometry<T>(p);
  if (!g.ok) {
    std::fprintf(stderr, "work items exceed the kernels' block limits\n");
    return 9;
  }
  if (kind == "ana") {
    KArgs<T> a = make_args<T>(p, dt, false);
    for (int64_t t0 = 0; t0 < total; t0 += w.chunk)
      launch_analysis<T>(p, a, g, tasks + t0, std::min(w.chunk, total - t0), x.data(), coef.data(), W1, W2, L);
    FILE* f = std::fopen(outpath, "wb");
    for (int64_t i = 0; i < ccount; ++i) {
      double v[2] = {(double)coef[i].x, (double)coef[i].y};
      std::fwrite(v, sizeof v, 1, f);
    }
    std::fclose(f);
  } else {
    KArgs<T> a = make_args<T>(p, dt, kind == "adj");
    for (int64_t t0 = 0; t0 < total; t0 += w.chunk)
      launch_synthesis<T>(p, a, g, tasks + t0, t0, std::min(w.chunk, total - t0), (const C2<T>*)coef.data(),
                          x.data(), W1, W2, L);
    FILE* f = std::fopen(outpath, "wb");
    for (int64_t i = 0; i < xlen; ++i) {
      double v = (double)x[i];
      std::fwrite(&v, sizeof v, 1, f);
    }
    std::fclose(f);
  }
  return 0;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 20) {
    std::fprintf(stderr, "usage: %s OP DTYPE fs fmin fmax B 2N M min_win dual group_cap lds_cap pass_cap chunk layout fused "
                 "m_policy IN OUT\n",
                 argv[0]);
    return 2;
  }
  const std::string op = argv[1];
  const int dt = std::atoi(argv[2]);
  slicq::PlanParams pp;
  pp.fs = std::atof(argv[3]);
  pp.fmin = std::atof(argv[4]);
  pp.fmax = std::atof(argv[5]);
  pp.bins_per_octave = std::atoi(argv[6]);
  pp.slice_len = std::atoll(argv[7]);
  pp.transition = std::atoll(argv[8]);
  pp.min_win = std::atof(argv[9]);
  pp.dual_kind = std::atoi(argv[10]);
  if (std::atoi(argv[11])) pp.group_cap = std::atoi(argv[11]);
  if (std::atoi(argv[12])) pp.lds_cap = std::atoi(argv[12]);
  if (std::atoi(argv[13])) pp.pass_cap = std::atoi(argv[13]);
  const int64_t chunk = std::atoll(argv[14]);
  pp.coef_layout = std::atoi(argv[15]);
  pp.fused = std::atoi(argv[16]);
  pp.m_policy = std::atoi(argv[17]);
  slicq::Plan plan;
  std::string err;
  if (slicq::build_plan(pp, plan, err)) {
    std::fprintf(stderr, "plan: %s\n", err.c_str());
    return 8;
  }
  if (pp.fused && !plan.fused[dt].ok) {
    std::fprintf(stderr, "the fused schedule was asked for but does not fit this plan and dtype\n");
    return 19;
  }
  const std::vector<double> in = read_all(argv[18]);
  return dt == 0 ? run<float>(op, plan, dt, chunk, in, argv[19]) : run<double>(op, plan, dt, chunk, in, argv[19]);
}
