// CPU emulation runner for the full-length CQ-NSGT kernels (test harness
// only): compiles the library's fullnsgt.hpp against the thread-per-lane
// stand-in in tests/emu/include and runs one analysis or synthesis on host
// memory (exact-size heap buffers for AddressSanitizer; the emulated LDS is
// filled with NaN before every block and checked past the launch's size).
//
// usage: full_runner OP DTYPE fs fmin fmax B 2N M min_win window L lattice IN OUT
//   OP: ana (IN: L complex doubles) | syn (IN: coef_count complex doubles)
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "fullnsgt.hpp"

thread_local dim3 threadIdx, blockIdx, blockDim, gridDim;
thread_local std::barrier<>* emu_barrier = nullptr;

namespace slicq {
constexpr size_t EMU_LDS = 1 << 18;
alignas(64) unsigned char smem[EMU_LDS];
}  // namespace slicq

namespace {

struct EmuLaunch {
  template <class K, class... A>
  void launch(K kernel, int64_t grid, int block, size_t shmem, A... args) {
    if (grid <= 0) return;
    if (shmem > slicq::EMU_LDS || block <= 0 || block > 1024) {
      std::fprintf(stderr, "bad launch: block %d shmem %zu\n", block, shmem);
      std::exit(3);
    }
    for (int64_t b = 0; b < grid; ++b) {
      std::memset(slicq::smem, 0xff, slicq::EMU_LDS);
      std::barrier<> bar(block);
      std::vector<std::thread> th;
      th.reserve(block);
      for (int t = 0; t < block; ++t) {
        th.emplace_back([&, t] {
          threadIdx = dim3((unsigned)t);
          blockIdx = dim3((unsigned)b);
          blockDim = dim3((unsigned)block);
          gridDim = dim3((unsigned)grid);
          emu_barrier = &bar;
          kernel(args...);
        });
      }
      for (auto& x : th) x.join();
      for (size_t i = shmem; i < slicq::EMU_LDS; ++i)
        if (slicq::smem[i] != 0xff) {
          std::fprintf(stderr, "LDS write past the %zu-byte allocation at byte %zu\n", shmem, i);
          std::exit(4);
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
int run(const std::string& op, slicq::FullPlan& f, int dt, const std::vector<double>& in, const char* outpath) {
  using namespace slicq;
  std::vector<unsigned char> blob;
  pack_full_tables(f, dt, blob, f.layout[dt]);
  const FullWork w = full_work(f, dt);
  std::vector<unsigned char> work(w.total);
  for (size_t i = 0; i < work.size(); ++i) work[i] = 0xff;     // NaN: every value read must be written first
  const int64_t nin = op == "ana" ? f.L : f.coef_count, nout = op == "ana" ? f.coef_count : f.L;
  if ((int64_t)in.size() != 2 * nin) {
    std::fprintf(stderr, "input holds %zu doubles, expected %lld\n", in.size(), (long long)(2 * nin));
    return 6;
  }
  std::vector<C2<T>> x(nin), y(nout);
  for (int64_t i = 0; i < nin; ++i) x[i] = {(T)in[2 * i], (T)in[2 * i + 1]};
  EmuLaunch ln;
  if (op == "ana") full_analyze_launch<T>(ln, f, (const char*)blob.data(), f.layout[dt], x.data(), y.data(),
                                          (char*)work.data(), w);
  else full_synthesize_launch<T>(ln, f, (const char*)blob.data(), f.layout[dt], x.data(), y.data(),
                                 (char*)work.data(), w);
  FILE* fo = std::fopen(outpath, "wb");
  for (int64_t i = 0; i < nout; ++i) {
    double v[2] = {(double)y[i].x, (double)y[i].y};
    std::fwrite(v, sizeof v, 1, fo);
  }
  std::fclose(fo);
  return 0;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 15) {
    std::fprintf(stderr, "usage: %s OP DTYPE fs fmin fmax B 2N M min_win window L lattice IN OUT\n", argv[0]);
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
  pp.window = std::atoi(argv[10]);
  slicq::Plan plan;
  std::string err;
  if (slicq::build_plan(pp, plan, err)) {
    std::fprintf(stderr, "plan: %s\n", err.c_str());
    return 8;
  }
  slicq::FullPlan f;
  if (slicq::build_full(plan, std::atoll(argv[11]), std::atoi(argv[12]), f, err)) {
    std::fprintf(stderr, "full plan: %s\n", err.c_str());
    return 9;
  }
  if (op == "syn" && !f.painless) {
    std::fprintf(stderr, "synthesis needs a painless lattice\n");
    return 10;
  }
  const std::vector<double> in = read_all(argv[13]);
  return dt == 0 ? run<float>(op, f, dt, in, argv[14]) : run<double>(op, f, dt, in, argv[14]);
}
