// C ABI of the sliCQ library (include/slicq.h): plan management, table
// upload and the enqueue-only transform calls.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <new>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/slicq.h"
#include "coefops.hpp"
#include "fullnsgt.hpp"
#include "pipeline.hpp"
#include "stream_server.hpp"

// Scratch of slicq_analyze_static: the slice task table and the two slice
// workspace regions, in a file-scope device array (each device that runs the
// library holds its own copy until the process ends). Host code uses the
// address hipGetSymbolAddress returns on each device, never this name.
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

struct slicq_plan_s {
  slicq::Plan p;
  std::vector<unsigned char> blob[2];   // packed tables, kept alive for async uploads
};

struct slicq_full_s {
  slicq::FullPlan f;
  std::vector<unsigned char> blob[2];   // packed tables, kept alive for async uploads
};

// A prepared ragged batch: its task table (caller-owned device memory) and
// the bounds the tasks were validated against.
struct slicq_batch_s {
  slicq_plan plan;
  slicq::SliceTask* tasks;
  int64_t total, x_len, coef_len;
};

namespace {

thread_local std::string g_err;
constexpr size_t kMaxLdsBytesAbi = slicq::kMaxLdsBytes;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  char b[256];
  std::snprintf(b, sizeof b, "%s: %s", what, hipGetErrorString(e));
  return fail(SLICQ_EHIP, b);
}

// Raises a kernel's dynamic-LDS limit once (not per launch, so that launches
// recorded into a graph contain nothing but the kernels).
void allow_lds(const void* kernel, size_t bytes) {
  static std::mutex mu;
  static std::unordered_map<const void*, size_t> done;
  std::lock_guard<std::mutex> lk(mu);
  size_t& cur = done[kernel];
  if (bytes > cur) {
    (void)hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLdsBytesAbi);
    cur = kMaxLdsBytesAbi;
  }
}

struct HipLaunch {
  hipStream_t st;
  template <class K, class... A>
  void launch(K kernel, int64_t grid, int block, size_t shmem, A... args) {
    if (grid <= 0) return;
    if (shmem > 65536) allow_lds(reinterpret_cast<const void*>(kernel), shmem);
    hipLaunchKernelGGL(kernel, dim3((unsigned)grid), dim3((unsigned)block), shmem, st, args...);
  }
  // gx x gy x gz blocks (gy, gz <= 65535)
  template <class K, class... A>
  void launch_xyz(K kernel, int64_t gx, int gy, int gz, int block, size_t shmem, A... args) {
    if (gx <= 0 || gy <= 0 || gz <= 0) return;
    if (shmem > 65536) allow_lds(reinterpret_cast<const void*>(kernel), shmem);
    hipLaunchKernelGGL(kernel, dim3((unsigned)gx, (unsigned)gy, (unsigned)gz), dim3((unsigned)block), shmem, st,
                       args...);
  }
};

int check_geometry(const slicq::Plan& p, int dt);

int check_plan(slicq_plan plan, slicq_dtype dt) {
  if (!plan) return fail(SLICQ_EINVAL, "null plan");
  if (dt != SLICQ_F32 && dt != SLICQ_F64) return fail(SLICQ_EINVAL, "dtype must be SLICQ_F32 or SLICQ_F64");
  if (!plan->p.dev[dt]) return fail(SLICQ_ESTATE, "plan tables not uploaded for this dtype (nsgt_plan_upload)");
  return check_geometry(plan->p, dt);
}

int check_geometry(const slicq::Plan& p, int dt) {
  const bool ok = dt == SLICQ_F32 ? slicq::geometry<float>(p).ok : slicq::geometry<double>(p).ok;
  return ok ? SLICQ_OK : fail(SLICQ_EINVAL, "plan work items exceed the kernels' block limits");
}

int64_t slices_of(const slicq::Plan& p, int64_t T) {
  if (T <= 0) return 0;
  return 2 * ((T + p.two_n - 1) / p.two_n);
}

// One signal must keep its padded length and coefficient count below 2^31.
int check_signal_size(const slicq::Plan& p, int64_t T) {
  const int64_t S = slices_of(p, T);
  if (S * p.N > slicq::kMaxSignalElems || S * p.coefs_per_slice > slicq::kMaxSignalElems)
    return fail(SLICQ_EINVAL, "signal too long for one call: split it (padded length and coefficient count "
                              "must stay below 2^31)");
  return SLICQ_OK;
}

int layout_or_fail(const slicq::Plan& p, int dt, int64_t ntasks, size_t bytes, slicq::WorkLayout& w) {
  if (!slicq::work_layout(p, dt, ntasks, bytes, w)) {
    char b[200];
    const size_t need = slicq::tasks_bytes(ntasks) + 256 + 2 * 256 + slicq::slice_scratch_bytes(p, dt);
    std::snprintf(b, sizeof b, "workspace of %zu bytes is below the minimum %zu for %lld slices", bytes, need,
                  (long long)ntasks);
    return fail(SLICQ_ESIZE, b);
  }
  return SLICQ_OK;
}

template <class T>
int run_analysis(slicq::Plan& p, int dt, const slicq::SliceTask* tasks, int64_t ntasks, const void* x,
                 void* coef, const slicq::WorkLayout& w, char* work, hipStream_t st, bool dual = false) {
  using namespace slicq;
  KArgs<T> a = make_args<T>(p, dt, false, dual);
  const Geometry<T> g = geometry<T>(p);
  HipLaunch L{st};
  C2<T>* W1 = reinterpret_cast<C2<T>*>(work + w.w1_off);
  C2<T>* W2 = reinterpret_cast<C2<T>*>(work + w.w2_off);
  for (int64_t t0 = 0; t0 < ntasks; t0 += w.chunk) {
    const int64_t cnt = std::min<int64_t>(w.chunk, ntasks - t0);
    launch_analysis<T>(p, a, g, tasks + t0, cnt, static_cast<const T*>(x), static_cast<C2<T>*>(coef), W1, W2, L);
  }
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? SLICQ_OK : hip_fail(e, "analysis launch");
}

template <class T>
int run_synthesis(slicq::Plan& p, int dt, bool adjoint, const slicq::SliceTask* tasks, int64_t ntasks,
                  const void* coef, void* y, const slicq::WorkLayout& w, char* work, hipStream_t st) {
  using namespace slicq;
  KArgs<T> a = make_args<T>(p, dt, adjoint);
  const Geometry<T> g = geometry<T>(p);
  HipLaunch L{st};
  C2<T>* W1 = reinterpret_cast<C2<T>*>(work + w.w1_off);
  C2<T>* W2 = reinterpret_cast<C2<T>*>(work + w.w2_off);
  for (int64_t t0 = 0; t0 < ntasks; t0 += w.chunk) {
    const int64_t cnt = std::min<int64_t>(w.chunk, ntasks - t0);
    launch_synthesis<T>(p, a, g, tasks + t0, t0, cnt, static_cast<const C2<T>*>(coef), static_cast<T*>(y), W1, W2,
                        L);
  }
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? SLICQ_OK : hip_fail(e, adjoint ? "adjoint launch" : "synthesis launch");
}

int plain_tasks(const slicq::Plan& p, int64_t T, int64_t S, slicq::SliceTask* tasks, hipStream_t st) {
  HipLaunch L{st};
  L.launch(slicq::k_tasks_plain, (S + 255) / 256, 256, 0, tasks, (int64_t)0, S, T, (int64_t)p.N, S);
  return SLICQ_OK;
}

int synth_common(slicq_plan plan, slicq_dtype dt, bool adjoint, const void* coef, int64_t coef_count, void* y,
                 int64_t T, void* work, size_t work_bytes, void* stream) {
  int rc = check_plan(plan, dt);
  if (rc) return rc;
  slicq::Plan& p = plan->p;
  if (T < 0) return fail(SLICQ_EINVAL, "T must be >= 0");
  const int64_t S = slices_of(p, T);
  if (S == 0) return SLICQ_OK;
  if ((rc = check_signal_size(p, T))) return rc;
  if (!coef || !y || !work) return fail(SLICQ_EINVAL, "null buffer");
  if (coef_count < S * p.coefs_per_slice) return fail(SLICQ_ESIZE, "coef_count < S * coefs_per_slice");
  slicq::WorkLayout w;
  if ((rc = layout_or_fail(p, dt, S, work_bytes, w))) return rc;
  char* wk = static_cast<char*>(work);
  auto* tasks = reinterpret_cast<slicq::SliceTask*>(wk + w.tasks_off);
  hipStream_t st = static_cast<hipStream_t>(stream);
  plain_tasks(p, T, S, tasks, st);
  return dt == SLICQ_F32 ? run_synthesis<float>(p, dt, adjoint, tasks, S, coef, y, w, wk, st)
                         : run_synthesis<double>(p, dt, adjoint, tasks, S, coef, y, w, wk, st);
}

int batched_tasks(const slicq::Plan& p, const int64_t* x_off, int32_t nsig, int64_t total, int64_t x_len,
                  const int64_t* coef_off, int64_t coef_len, slicq::SliceTask* tasks, int32_t* status,
                  hipStream_t st) {
  HipLaunch L{st};
  L.launch(slicq::k_tasks_batched, 1, 1024, 1026 * sizeof(int64_t), tasks, x_off, coef_off, nsig, (int64_t)p.N, total, x_len,
           coef_len, (int64_t)p.coefs_per_slice, status);
  return SLICQ_OK;
}

int synth_batched_common(slicq_plan plan, slicq_dtype dt, bool adjoint, const void* coef, int64_t coef_len,
                         const int64_t* coef_off, void* y, int64_t y_len, const int64_t* y_off, int32_t nsig,
                         int64_t total, void* work, size_t work_bytes, void* stream) {
  int rc = check_plan(plan, dt);
  if (rc) return rc;
  slicq::Plan& p = plan->p;
  if (nsig < 0 || total < 0) return fail(SLICQ_EINVAL, "nsig and total_slices must be >= 0");
  if (nsig == 0 || total == 0) return SLICQ_OK;
  if (!coef || !coef_off || !y || !y_off || !work) return fail(SLICQ_EINVAL, "null buffer");
  slicq::WorkLayout w;
  if ((rc = layout_or_fail(p, dt, total, work_bytes, w))) return rc;
  char* wk = static_cast<char*>(work);
  auto* tasks = reinterpret_cast<slicq::SliceTask*>(wk + w.tasks_off);
  hipStream_t st = static_cast<hipStream_t>(stream);
  batched_tasks(p, y_off, nsig, total, y_len, coef_off, coef_len, tasks,
                reinterpret_cast<int32_t*>(wk + w.status_off), st);
  return dt == SLICQ_F32 ? run_synthesis<float>(p, dt, adjoint, tasks, total, coef, y, w, wk, st)
                         : run_synthesis<double>(p, dt, adjoint, tasks, total, coef, y, w, wk, st);
}

// Device backend of the streaming server: its own non-blocking stream (default
// priority), hipMalloc'd device buffers, hipHostMalloc'd staging.
struct HipBackend {
  hipStream_t st = nullptr;
  void* dmalloc(size_t n) {
    void* p = nullptr;
    return hipMalloc(&p, n) == hipSuccess ? p : nullptr;
  }
  void dfree(void* p) {
    if (p) (void)hipFree(p);
  }
  void* hmalloc(size_t n) {
    void* p = nullptr;
    return hipHostMalloc(&p, n, hipHostMallocDefault) == hipSuccess ? p : nullptr;
  }
  void hfree(void* p) {
    if (p) (void)hipHostFree(p);
  }
  void h2d(void* d, const void* h, size_t n) { (void)hipMemcpyAsync(d, h, n, hipMemcpyHostToDevice, st); }
  void d2h(void* h, const void* d, size_t n) { (void)hipMemcpyAsync(h, d, n, hipMemcpyDeviceToHost, st); }
  template <class K, class... A>
  void launch(K kernel, int64_t grid, int block, size_t shmem, A... args) {
    HipLaunch L{st};
    L.launch(kernel, grid, block, shmem, args...);
  }
  template <class K, class... A>
  void launch_xyz(K kernel, int64_t gx, int gy, int gz, int block, size_t shmem, A... args) {
    HipLaunch L{st};
    L.launch_xyz(kernel, gx, gy, gz, block, shmem, args...);
  }
  bool sync() { return hipStreamSynchronize(st) == hipSuccess && hipGetLastError() == hipSuccess; }
};

}  // namespace

struct slicq_stream_server_s {
  HipBackend be;
  slicq::StreamServer<float, HipBackend>* f = nullptr;
  slicq::StreamServer<double, HipBackend>* d = nullptr;
  int dt = 0;
  ~slicq_stream_server_s() {
    delete f;
    delete d;
    if (be.st) (void)hipStreamDestroy(be.st);
  }
};

namespace {

template <class F>
int with_server(slicq_stream_server s, F&& fn) {
  if (!s) return fail(SLICQ_EINVAL, "null server");
  if ((s->f && s->f->fenced()) || (s->d && s->d->fenced()))
    return fail(SLICQ_EHIP, "the server hit a device error and is fenced; destroy it");
  return s->dt == SLICQ_F32 ? fn(*s->f) : fn(*s->d);
}

}  // namespace

namespace {

// Device address of `scratch` on the current device, looked up once per device.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int static_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(SLICQ_EINVAL, "device index out of range for the static scratch");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return SLICQ_OK;
}

}  // namespace

extern "C" {

int slicq_stream_server_create(slicq_plan plan, slicq_dtype dt, int32_t max_streams, int32_t max_batch,
                               size_t hbm_budget_bytes, slicq_stream_server* out) {
  int rc = check_plan(plan, dt);
  if (rc) return rc;
  if (!out || max_streams <= 0 || max_batch <= 0) return fail(SLICQ_EINVAL, "bad server arguments");
  *out = nullptr;
  auto* s = new (std::nothrow) slicq_stream_server_s;
  if (!s) return fail(SLICQ_ENOMEM, "out of host memory");
  s->dt = dt;
  hipError_t e = hipStreamCreateWithFlags(&s->be.st, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete s;
    return hip_fail(e, "stream creation");
  }
  std::string err;
  bool ok;
  if (dt == SLICQ_F32) {
    s->f = new slicq::StreamServer<float, HipBackend>(plan->p, dt, s->be, max_streams, max_batch, hbm_budget_bytes);
    ok = s->f->init(err);
  } else {
    s->d = new slicq::StreamServer<double, HipBackend>(plan->p, dt, s->be, max_streams, max_batch, hbm_budget_bytes);
    ok = s->d->init(err);
  }
  if (!ok) {
    delete s;
    return fail(err.find("budget") != std::string::npos ? SLICQ_EBUSY : SLICQ_ENOMEM, err);
  }
  *out = s;
  return SLICQ_OK;
}

void slicq_stream_server_destroy(slicq_stream_server s) { delete s; }

int slicq_stream_open(slicq_stream_server s, int32_t* id) {
  if (!id) return fail(SLICQ_EINVAL, "null id");
  return with_server(s, [&](auto& srv) -> int {
    const int r = srv.open();
    *id = r;
    return r >= 0 ? SLICQ_OK : fail(SLICQ_EBUSY, "no free stream slot within the memory budget");
  });
}

int slicq_stream_push(slicq_stream_server s, int32_t id, const void* samples, int64_t n) {
  return with_server(s, [&](auto& srv) -> int {
    using T = std::remove_pointer_t<decltype(srv.ring_type())>;
    if (!srv.valid(id)) return fail(SLICQ_ESTATE, "stream is not open");
    if (n < 0 || (n > 0 && !samples)) return fail(SLICQ_EINVAL, "bad samples");
    srv.push(id, static_cast<const T*>(samples), n);
    return SLICQ_OK;
  });
}

int slicq_stream_push_many(slicq_stream_server s, int32_t n_ids, const int32_t* ids, const void* samples,
                           const int64_t* counts) {
  return with_server(s, [&](auto& srv) -> int {
    using T = std::remove_pointer_t<decltype(srv.ring_type())>;
    if (n_ids < 0 || (n_ids > 0 && (!ids || !counts))) return fail(SLICQ_EINVAL, "bad id list");
    int64_t total = 0;
    for (int32_t i = 0; i < n_ids; ++i) {
      if (!srv.valid(ids[i])) return fail(SLICQ_ESTATE, "stream is not open");
      if (counts[i] < 0) return fail(SLICQ_EINVAL, "bad count");
      total += counts[i];
    }
    if (total > 0 && !samples) return fail(SLICQ_EINVAL, "bad samples");
    const T* x = static_cast<const T*>(samples);
    for (int32_t i = 0; i < n_ids; ++i) {
      srv.push(ids[i], x, counts[i]);
      x += counts[i];
    }
    return SLICQ_OK;
  });
}

int slicq_stream_push_gap(slicq_stream_server s, int32_t id, int64_t n) {
  return with_server(s, [&](auto& srv) -> int {
    if (!srv.valid(id)) return fail(SLICQ_ESTATE, "stream is not open");
    if (n < 0) return fail(SLICQ_EINVAL, "bad count");
    srv.push_gap(id, n);
    return SLICQ_OK;
  });
}

int slicq_stream_tick(slicq_stream_server s, int64_t* n_slices) {
  return with_server(s, [&](auto& srv) -> int {
    const int64_t r = srv.tick();
    if (n_slices) *n_slices = r < 0 ? 0 : r;
    return r >= 0 ? SLICQ_OK : fail(SLICQ_EHIP, "device error in a streaming tick");
  });
}

int slicq_stream_poll(slicq_stream_server s, int32_t id, void* out, int64_t max, int64_t* n) {
  return with_server(s, [&](auto& srv) -> int {
    using T = std::remove_pointer_t<decltype(srv.ring_type())>;
    if (!srv.valid(id)) return fail(SLICQ_ESTATE, "stream is not open");
    if (!n || max < 0 || (max > 0 && !out)) return fail(SLICQ_EINVAL, "bad output buffer");
    *n = srv.poll(id, static_cast<T*>(out), max);
    return SLICQ_OK;
  });
}

int slicq_stream_poll_many(slicq_stream_server s, int32_t n_ids, const int32_t* ids, void* out, int64_t cap,
                           int64_t* counts) {
  return with_server(s, [&](auto& srv) -> int {
    using T = std::remove_pointer_t<decltype(srv.ring_type())>;
    if (n_ids < 0 || (n_ids > 0 && (!ids || !counts))) return fail(SLICQ_EINVAL, "bad id list");
    if (cap < 0 || (cap > 0 && !out)) return fail(SLICQ_EINVAL, "bad output buffer");
    for (int32_t i = 0; i < n_ids; ++i)
      if (!srv.valid(ids[i])) return fail(SLICQ_ESTATE, "stream is not open");
    T* y = static_cast<T*>(out);
    int64_t left = cap;
    for (int32_t i = 0; i < n_ids; ++i) {
      const int64_t got = left > 0 ? srv.poll(ids[i], y, left) : 0;
      counts[i] = got;
      y += got;
      left -= got;
    }
    return SLICQ_OK;
  });
}

int slicq_stream_close(slicq_stream_server s, int32_t id) {
  return with_server(s, [&](auto& srv) -> int {
    if (!srv.valid(id)) return fail(SLICQ_ESTATE, "stream is not open");
    srv.close(id);
    return SLICQ_OK;
  });
}

int slicq_stream_stats_get(slicq_stream_server s, slicq_stream_stats* out) {
  if (!out) return fail(SLICQ_EINVAL, "null stats");
  return with_server(s, [&](auto& srv) -> int {
    const slicq::StreamStats t = srv.stats();
    std::memset(out, 0, sizeof *out);
    out->ticks = t.ticks;
    out->slices = t.slices;
    out->samples_in = t.samples_in;
    out->samples_out = t.samples_out;
    out->admitted = t.admitted;
    out->rejected = t.rejected;
    out->closed = t.closed;
    out->gap_samples = t.gaps;
    out->latency_p50_s = t.latency_p50;
    out->latency_p99_s = t.latency_p99;
    out->latency_max_s = t.latency_max;
    out->latency_count = t.latency_count;
    out->busy_s = t.busy_seconds;
    out->slots = srv.slots();
    out->ring_len = srv.ring();
    out->bytes_per_stream = (int64_t)srv.per_stream_bytes();
    out->fixed_bytes = (int64_t)srv.fixed_bytes();
    return SLICQ_OK;
  });
}

int slicq_stream_coefs(slicq_stream_server s, int32_t id, void* out, int64_t cap, int64_t* m) {
  if (!m) return fail(SLICQ_EINVAL, "null m");
  return with_server(s, [&](auto& srv) -> int {
    using T = std::remove_pointer_t<decltype(srv.ring_type())>;
    if (!srv.valid(id)) return fail(SLICQ_ESTATE, "stream is not open");
    if (!out || cap < srv.coefs_per_slice()) return fail(SLICQ_ESIZE, "buffer below coefs_per_slice");
    *m = srv.last_coefs(id, static_cast<slicq::C2<T>*>(out));
    return SLICQ_OK;
  });
}

int slicq_stream_stats_reset(slicq_stream_server s) {
  return with_server(s, [&](auto& srv) -> int {
    srv.reset_stats();
    return SLICQ_OK;
  });
}

int slicq_stream_snapshot(slicq_stream_server s, int32_t id, void* buf, size_t cap, size_t* bytes) {
  if (!bytes) return fail(SLICQ_EINVAL, "null size");
  return with_server(s, [&](auto& srv) -> int {
    if (!srv.valid(id)) return fail(SLICQ_ESTATE, "stream is not open");
    std::vector<unsigned char> blob;
    if (!srv.snapshot(id, blob)) return fail(SLICQ_EHIP, "device error while reading the stream state");
    *bytes = blob.size();
    if (!buf) return SLICQ_OK;
    if (cap < blob.size()) return fail(SLICQ_ESIZE, "snapshot buffer too small");
    std::memcpy(buf, blob.data(), blob.size());
    return SLICQ_OK;
  });
}

int slicq_stream_restore(slicq_stream_server s, int32_t id, const void* buf, size_t bytes) {
  return with_server(s, [&](auto& srv) -> int {
    if (!srv.valid(id)) return fail(SLICQ_ESTATE, "stream is not open");
    if (!buf) return fail(SLICQ_EINVAL, "null snapshot");
    if (!srv.restore(id, static_cast<const unsigned char*>(buf), bytes))
      return fail(SLICQ_EINVAL, "snapshot does not match this server (plan, dtype or size)");
    return SLICQ_OK;
  });
}


int nsgt_plan_ex(const slicq_plan_opts* o, slicq_plan* out) {
  if (!o || !out) return fail(SLICQ_EINVAL, "null argument");
  *out = nullptr;
  slicq::PlanParams pp;
  pp.fs = o->fs;
  pp.fmin = o->fmin;
  pp.fmax = o->fmax;
  pp.bins_per_octave = o->bins_per_octave;
  pp.slice_len = o->slice_len;
  pp.transition = o->transition_len;
  pp.min_win = o->min_win;
  pp.dual_kind = o->dual_slice;
  if (o->group_cap) pp.group_cap = o->group_cap;
  if (o->lds_cap) pp.lds_cap = o->lds_cap;
  if (o->pass_cap) pp.pass_cap = o->pass_cap;
  pp.coef_layout = o->coef_layout;
  pp.fused = o->fused ? 1 : 0;
  pp.window = o->window;
  pp.scale = o->scale;
  pp.slicing = o->slicing;
  pp.m_policy = o->m_policy;
  slicq_plan h = new (std::nothrow) slicq_plan_s;
  if (!h) return fail(SLICQ_ENOMEM, "out of host memory");
  std::string err;
  int rc;
  try {
    rc = slicq::build_plan(pp, h->p, err);
  } catch (const std::bad_alloc&) {
    delete h;
    return fail(SLICQ_ENOMEM, "out of host memory");
  }
  if (rc) {
    delete h;
    return fail(SLICQ_EINVAL, err);
  }
  *out = h;
  return SLICQ_OK;
}

int nsgt_plan(double fs, double fmin, double fmax, int bins_per_octave, int64_t slice_len_2N,
              int64_t transition_len, slicq_plan* out) {
  slicq_plan_opts o{};
  o.fs = fs;
  o.fmin = fmin;
  o.fmax = fmax;
  o.bins_per_octave = bins_per_octave;
  o.slice_len = slice_len_2N;
  o.transition_len = transition_len;
  o.min_win = 16.0;
  o.dual_slice = 0;
  return nsgt_plan_ex(&o, out);
}

void nsgt_plan_destroy(slicq_plan plan) { delete plan; }

int nsgt_plan_info(slicq_plan plan, slicq_plan_info* info) {
  if (!plan || !info) return fail(SLICQ_EINVAL, "null argument");
  const slicq::Plan& p = plan->p;
  std::memset(info, 0, sizeof *info);
  info->K = p.K;
  info->nbands = p.nb;
  info->slice_len = p.two_n;
  info->transition_len = p.Mt;
  info->coefs_per_slice = p.coefs_per_slice;
  info->Q = p.Q;
  info->max_M = p.max_M;
  info->n_ana_items = (int32_t)p.ana.size();
  info->n_syn_items = (int32_t)p.syn.size();
  info->coef_layout = p.prm.coef_layout;
  info->fused = (p.fused[0].ok ? 1 : 0) | (p.fused[1].ok ? 2 : 0);
  info->coefs_per_slice_all = p.coefs_per_slice;
  for (int k = 1; k <= p.K; ++k) info->coefs_per_slice_all += p.bands[k].M;
  return SLICQ_OK;
}

int nsgt_plan_bands(slicq_plan plan, int32_t* M, int64_t* off, int64_t* start, int32_t* len, double* fc_hz,
                    double* bw_hz) {
  if (!plan) return fail(SLICQ_EINVAL, "null plan");
  const auto& b = plan->p.bands;
  for (size_t k = 0; k < b.size(); ++k) {
    if (M) M[k] = b[k].M;
    if (off) off[k] = b[k].off;
    if (start) start[k] = b[k].start;
    if (len) len[k] = b[k].len;
    if (fc_hz) fc_hz[k] = b[k].xi;
    if (bw_hz) bw_hz[k] = b[k].omega;
  }
  return SLICQ_OK;
}

int nsgt_plan_windows(slicq_plan plan, double* g, double* gd, double* h0, double* hd, double* D) {
  if (!plan) return fail(SLICQ_EINVAL, "null plan");
  const slicq::Plan& p = plan->p;
  if (g) std::memcpy(g, p.g.data(), p.g.size() * sizeof(double));
  if (gd) std::memcpy(gd, p.gd.data(), p.gd.size() * sizeof(double));
  if (h0) std::memcpy(h0, p.h0.data(), p.h0.size() * sizeof(double));
  if (hd) std::memcpy(hd, p.hd.data(), p.hd.size() * sizeof(double));
  if (D) std::memcpy(D, p.D.data(), p.D.size() * sizeof(double));
  return SLICQ_OK;
}

int nsgt_plan_table_bytes(slicq_plan plan, slicq_dtype dt, size_t* bytes) {
  if (!plan || !bytes) return fail(SLICQ_EINVAL, "null argument");
  if (dt != SLICQ_F32 && dt != SLICQ_F64) return fail(SLICQ_EINVAL, "bad dtype");
  std::lock_guard<std::mutex> lk(plan->p.mu);
  if (plan->blob[dt].empty()) slicq::pack_tables(plan->p, dt, plan->blob[dt], plan->p.layout[dt]);
  *bytes = plan->blob[dt].size();
  return SLICQ_OK;
}

int nsgt_plan_upload(slicq_plan plan, slicq_dtype dt, void* dev, size_t bytes, void* stream) {
  size_t need = 0;
  int rc = nsgt_plan_table_bytes(plan, dt, &need);
  if (rc) return rc;
  if (!dev) return fail(SLICQ_EINVAL, "null device pointer");
  if (reinterpret_cast<uintptr_t>(dev) & 255) return fail(SLICQ_EINVAL, "device tables must be 256-byte aligned");
  if (bytes < need) return fail(SLICQ_ESIZE, "device table buffer too small");
  std::lock_guard<std::mutex> lk(plan->p.mu);
  hipError_t e = hipMemcpyAsync(dev, plan->blob[dt].data(), need, hipMemcpyHostToDevice,
                                static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "table upload");
  plan->p.dev[dt] = dev;
  plan->p.dev_bytes[dt] = bytes;
  return SLICQ_OK;
}

int64_t slicq_num_slices(slicq_plan plan, int64_t T) {
  if (!plan) return fail(SLICQ_EINVAL, "null plan");
  return slices_of(plan->p, T);
}

int slicq_workspace_size(slicq_plan plan, slicq_dtype dt, int64_t n_slices, size_t* bytes) {
  if (!plan || !bytes) return fail(SLICQ_EINVAL, "null argument");
  if (dt != SLICQ_F32 && dt != SLICQ_F64) return fail(SLICQ_EINVAL, "bad dtype");
  if (n_slices < 0) return fail(SLICQ_EINVAL, "n_slices must be >= 0");
  *bytes = slicq::workspace_bytes(plan->p, dt, n_slices);
  return SLICQ_OK;
}

// Analysis-shaped calls on one signal (plain task table): analysis, or with
// dual the adjoint of synthesis (dual windows, doubled weights on bands 1..K).
static int analyze_common(slicq_plan plan, slicq_dtype dt, const void* x, int64_t T, void* coef, int64_t coef_count,
                          void* work, size_t work_bytes, void* stream, bool dual) {
  int rc = check_plan(plan, dt);
  if (rc) return rc;
  slicq::Plan& p = plan->p;
  if (T < 0) return fail(SLICQ_EINVAL, "T must be >= 0");
  const int64_t S = slices_of(p, T);
  if (S == 0) return SLICQ_OK;
  if ((rc = check_signal_size(p, T))) return rc;
  if (!x || !coef || !work) return fail(SLICQ_EINVAL, "null buffer");
  if (coef_count < S * p.coefs_per_slice) return fail(SLICQ_ESIZE, "coef_count < S * coefs_per_slice");
  slicq::WorkLayout w;
  if ((rc = layout_or_fail(p, dt, S, work_bytes, w))) return rc;
  char* wk = static_cast<char*>(work);
  auto* tasks = reinterpret_cast<slicq::SliceTask*>(wk + w.tasks_off);
  hipStream_t st = static_cast<hipStream_t>(stream);
  plain_tasks(p, T, S, tasks, st);
  return dt == SLICQ_F32 ? run_analysis<float>(p, dt, tasks, S, x, coef, w, wk, st, dual)
                         : run_analysis<double>(p, dt, tasks, S, x, coef, w, wk, st, dual);
}

int slicq_synthesize_adjoint(slicq_plan plan, slicq_dtype dt, const void* y, int64_t T, void* coef,
                             int64_t coef_count, void* work, size_t work_bytes, void* stream) {
  return analyze_common(plan, dt, y, T, coef, coef_count, work, work_bytes, stream, true);
}

}  // extern "C"

namespace {

// Workspace of the complex-signal calls: the real workspace, then two real
// sample arrays of T and two coefficient sets of the stored bands.
struct ComplexLayout {
  size_t real_bytes = 0, re_off = 0, im_off = 0, ca_off = 0, cb_off = 0, total = 0;
};

ComplexLayout complex_layout(const slicq::Plan& p, int dt, int64_t T) {
  using slicq::align256;
  ComplexLayout c;
  const int64_t S = slices_of(p, T);
  const size_t b = dt ? 8 : 4;
  c.real_bytes = slicq::workspace_bytes(p, dt, S);
  c.re_off = align256(c.real_bytes);
  c.im_off = align256(c.re_off + (size_t)T * b);
  c.ca_off = align256(c.im_off + (size_t)T * b);
  c.cb_off = align256(c.ca_off + (size_t)S * p.coefs_per_slice * 2 * b);
  c.total = align256(c.cb_off + (size_t)S * p.coefs_per_slice * 2 * b);
  return c;
}

int64_t coefs_all(const slicq::Plan& p) {
  int64_t n = p.coefs_per_slice;
  for (int k = 1; k <= p.K; ++k) n += p.bands[k].M;
  return n;
}

int check_complex(slicq_plan plan, slicq_dtype dt, int64_t T) {
  int rc = check_plan(plan, dt);
  if (rc) return rc;
  if (plan->p.prm.coef_layout != 0) return fail(SLICQ_EINVAL, "complex-signal calls need the band-major layout");
  if (T < 0) return fail(SLICQ_EINVAL, "T must be >= 0");
  return check_signal_size(plan->p, T);
}

template <class T, class K, class... A>
void launch_flat(hipStream_t st, K kernel, int64_t n, A... args) {
  if (n <= 0) return;
  hipLaunchKernelGGL(kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, args...);
}

const slicq::BandDev* dev_bands(const slicq::Plan& p, int dt) {
  return reinterpret_cast<const slicq::BandDev*>(static_cast<const char*>(p.dev[dt]) + p.layout[dt].bands);
}

}  // namespace

extern "C" {

int slicq_complex_workspace_size(slicq_plan plan, slicq_dtype dt, int64_t T, size_t* bytes) {
  if (!plan || !bytes) return fail(SLICQ_EINVAL, "null argument");
  if (dt != SLICQ_F32 && dt != SLICQ_F64) return fail(SLICQ_EINVAL, "bad dtype");
  if (T < 0) return fail(SLICQ_EINVAL, "T must be >= 0");
  *bytes = complex_layout(plan->p, dt, T).total;
  return SLICQ_OK;
}

int slicq_analyze_complex(slicq_plan plan, slicq_dtype dt, const void* x, int64_t T, void* coef, int64_t coef_count,
                          void* work, size_t work_bytes, void* stream) {
  int rc = check_complex(plan, dt, T);
  if (rc) return rc;
  slicq::Plan& p = plan->p;
  const int64_t S = slices_of(p, T);
  if (S == 0) return SLICQ_OK;
  if (!x || !coef || !work) return fail(SLICQ_EINVAL, "null buffer");
  if (coef_count < S * coefs_all(p)) return fail(SLICQ_ESIZE, "coef_count < S * coefs_per_slice_all");
  const ComplexLayout cl = complex_layout(p, dt, T);
  if (work_bytes < cl.total) return fail(SLICQ_ESIZE, "workspace below slicq_complex_workspace_size");
  char* wk = static_cast<char*>(work);
  hipStream_t st = static_cast<hipStream_t>(stream);
  auto go = [&](auto tag) -> int {
    using F = decltype(tag);
    using namespace slicq;
    F* re = reinterpret_cast<F*>(wk + cl.re_off);
    F* im = reinterpret_cast<F*>(wk + cl.im_off);
    C2<F>* cb = reinterpret_cast<C2<F>*>(wk + cl.cb_off);
    launch_flat<F>(st, k_split_complex<F>, T, static_cast<const C2<F>*>(x), T, re, im);
    int r = analyze_common(plan, dt, re, T, coef, S * p.coefs_per_slice, wk, cl.real_bytes, stream, false);
    if (!r) r = analyze_common(plan, dt, im, T, cb, S * p.coefs_per_slice, wk, cl.real_bytes, stream, false);
    if (r) return r;
    launch_flat<F>(st, k_combine_complex<F>, S * p.coefs_per_slice, dev_bands(p, dt), S * p.coefs_per_slice,
                   p.nb, (int)S, S * p.coefs_per_slice, (const C2<F>*)cb, static_cast<C2<F>*>(coef));
    return SLICQ_OK;
  };
  rc = dt == SLICQ_F32 ? go(float{}) : go(double{});
  if (rc) return rc;
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? SLICQ_OK : hip_fail(e, "complex analysis launch");
}

int slicq_synthesize_complex(slicq_plan plan, slicq_dtype dt, const void* coef, int64_t coef_count, void* y,
                             int64_t T, void* work, size_t work_bytes, void* stream) {
  int rc = check_complex(plan, dt, T);
  if (rc) return rc;
  slicq::Plan& p = plan->p;
  const int64_t S = slices_of(p, T);
  if (S == 0) return SLICQ_OK;
  if (!y || !coef || !work) return fail(SLICQ_EINVAL, "null buffer");
  if (coef_count < S * coefs_all(p)) return fail(SLICQ_ESIZE, "coef_count < S * coefs_per_slice_all");
  const ComplexLayout cl = complex_layout(p, dt, T);
  if (work_bytes < cl.total) return fail(SLICQ_ESIZE, "workspace below slicq_complex_workspace_size");
  char* wk = static_cast<char*>(work);
  hipStream_t st = static_cast<hipStream_t>(stream);
  auto go = [&](auto tag) -> int {
    using F = decltype(tag);
    using namespace slicq;
    F* re = reinterpret_cast<F*>(wk + cl.re_off);
    F* im = reinterpret_cast<F*>(wk + cl.im_off);
    C2<F>* u = reinterpret_cast<C2<F>*>(wk + cl.ca_off);
    C2<F>* v = reinterpret_cast<C2<F>*>(wk + cl.cb_off);
    launch_flat<F>(st, k_hermitian_parts<F>, S * p.coefs_per_slice, dev_bands(p, dt), S * p.coefs_per_slice,
                   p.nb, (int)S, S * p.coefs_per_slice, static_cast<const C2<F>*>(coef), u, v);
    int r = synth_common(plan, dt, false, u, S * p.coefs_per_slice, re, T, wk, cl.real_bytes, stream);
    if (!r) r = synth_common(plan, dt, false, v, S * p.coefs_per_slice, im, T, wk, cl.real_bytes, stream);
    if (r) return r;
    launch_flat<F>(st, k_join_complex<F>, T, (const F*)re, (const F*)im, T, static_cast<C2<F>*>(y));
    return SLICQ_OK;
  };
  rc = dt == SLICQ_F32 ? go(float{}) : go(double{});
  if (rc) return rc;
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? SLICQ_OK : hip_fail(e, "complex synthesis launch");
}

int slicq_layers(slicq_plan plan, slicq_dtype dt, const void* coef, int64_t S, int mode, void* out,
                 int64_t out_count, void* stream) {
  int rc = check_plan(plan, dt);
  if (rc) return rc;
  slicq::Plan& p = plan->p;
  if (S < 0 || (S & 1)) return fail(SLICQ_EINVAL, "S must be an even slice count >= 0");
  if (mode != 0 && mode != 1) return fail(SLICQ_EINVAL, "mode is 0 (layer sum) or 1 (spectrogram)");
  if (S == 0) return SLICQ_OK;
  if (!coef || !out) return fail(SLICQ_EINVAL, "null buffer");
  const int64_t n = (S / 2) * p.coefs_per_slice;
  if (out_count < n) return fail(SLICQ_ESIZE, "out_count < (S / 2) * coefs_per_slice");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const slicq::CoefAddr ca{p.prm.coef_layout, (int32_t)p.coefs_per_slice, (int32_t)S};
  if (dt == SLICQ_F32) {
    if (mode == 0) launch_flat<float>(st, slicq::k_layer_sum<float, 0>, n, dev_bands(p, dt), n, p.nb, ca,
                                      static_cast<const slicq::C2<float>*>(coef), out);
    else launch_flat<float>(st, slicq::k_layer_sum<float, 1>, n, dev_bands(p, dt), n, p.nb, ca,
                            static_cast<const slicq::C2<float>*>(coef), out);
  } else {
    if (mode == 0) launch_flat<double>(st, slicq::k_layer_sum<double, 0>, n, dev_bands(p, dt), n, p.nb, ca,
                                       static_cast<const slicq::C2<double>*>(coef), out);
    else launch_flat<double>(st, slicq::k_layer_sum<double, 1>, n, dev_bands(p, dt), n, p.nb, ca,
                             static_cast<const slicq::C2<double>*>(coef), out);
  }
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? SLICQ_OK : hip_fail(e, "layer launch");
}

int slicq_mask_db(slicq_plan plan, slicq_dtype dt, void* coef, int64_t S, const void* mask, int64_t mask_count,
                  void* stream) {
  int rc = check_plan(plan, dt);
  if (rc) return rc;
  slicq::Plan& p = plan->p;
  if (S < 0 || (S & 1)) return fail(SLICQ_EINVAL, "S must be an even slice count >= 0");
  if (S == 0) return SLICQ_OK;
  if (!coef || !mask) return fail(SLICQ_EINVAL, "null buffer");
  if (mask_count < (S / 2) * p.coefs_per_slice) return fail(SLICQ_ESIZE, "mask_count < (S / 2) * coefs_per_slice");
  const int64_t n = S * p.coefs_per_slice;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const slicq::CoefAddr ca{p.prm.coef_layout, (int32_t)p.coefs_per_slice, (int32_t)S};
  if (dt == SLICQ_F32)
    launch_flat<float>(st, slicq::k_mask_db<float>, n, dev_bands(p, dt), n, p.nb, ca, static_cast<const float*>(mask),
                       static_cast<slicq::C2<float>*>(coef));
  else
    launch_flat<double>(st, slicq::k_mask_db<double>, n, dev_bands(p, dt), n, p.nb, ca,
                        static_cast<const double*>(mask), static_cast<slicq::C2<double>*>(coef));
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? SLICQ_OK : hip_fail(e, "mask launch");
}

int slicq_transpose(slicq_plan plan, slicq_dtype dt, const void* in, void* out, int64_t S, int32_t d, void* stream) {
  int rc = check_plan(plan, dt);
  if (rc) return rc;
  slicq::Plan& p = plan->p;
  if (S < 0) return fail(SLICQ_EINVAL, "S must be >= 0");
  if (S == 0) return SLICQ_OK;
  if (!in || !out || in == out) return fail(SLICQ_EINVAL, "null or aliased buffers");
  for (int t = 1; t <= p.K; ++t) {
    const int s = t - d;
    if (s >= 1 && s <= p.K && p.bands[s].M != p.bands[t].M)
      return fail(SLICQ_EINVAL, "transposition moves a band onto one with a different M_k (use m_policy 1, "
                                "the rectangular representation, or a shift inside a run of equal M_k)");
  }
  const int64_t n = S * p.coefs_per_slice;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const slicq::CoefAddr ca{p.prm.coef_layout, (int32_t)p.coefs_per_slice, (int32_t)S};
  if (dt == SLICQ_F32)
    launch_flat<float>(st, slicq::k_transpose<float>, n, dev_bands(p, dt), n, p.nb, ca, (int)d,
                       static_cast<const slicq::C2<float>*>(in), static_cast<slicq::C2<float>*>(out));
  else
    launch_flat<double>(st, slicq::k_transpose<double>, n, dev_bands(p, dt), n, p.nb, ca, (int)d,
                        static_cast<const slicq::C2<double>*>(in), static_cast<slicq::C2<double>*>(out));
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? SLICQ_OK : hip_fail(e, "transpose launch");
}

int slicq_analyze(slicq_plan plan, slicq_dtype dt, const void* x, int64_t T, void* coef, int64_t coef_count,
                  void* work, size_t work_bytes, void* stream) {
  return analyze_common(plan, dt, x, T, coef, coef_count, work, work_bytes, stream, false);
}


size_t slicq_static_scratch_bytes(void) { return kStaticScratchBytes; }

int slicq_analyze_static(slicq_plan plan, slicq_dtype dt, const void* x, int64_t T, void* coef, int64_t coef_count,
                         void* stream) {
  int rc = check_plan(plan, dt);
  if (rc) return rc;
  slicq::Plan& p = plan->p;
  if (T < 0) return fail(SLICQ_EINVAL, "T must be >= 0");
  const int64_t S = slices_of(p, T);
  if (S == 0) return SLICQ_OK;
  if ((rc = check_signal_size(p, T))) return rc;
  if (!x || !coef) return fail(SLICQ_EINVAL, "null buffer");
  if (coef_count < S * p.coefs_per_slice) return fail(SLICQ_ESIZE, "coef_count < S * coefs_per_slice");
  // the task table of all S slices and the scratch of at least one slice must fit
  slicq::WorkLayout w;
  if (!slicq::work_layout(p, dt, S, kStaticScratchBytes, w)) {
    char b[200];
    std::snprintf(b, sizeof b, "the static scratch (%zu bytes) cannot hold the tasks of %lld slices and one slice's "
                  "workspace; use slicq_analyze with a caller workspace", kStaticScratchBytes, (long long)S);
    return fail(SLICQ_ESIZE, b);
  }
  void* base = nullptr;
  if ((rc = static_scratch(&base))) return rc;
  char* wk = static_cast<char*>(base);
  auto* tasks = reinterpret_cast<slicq::SliceTask*>(wk + w.tasks_off);
  hipStream_t st = static_cast<hipStream_t>(stream);
  plain_tasks(p, T, S, tasks, st);
  return dt == SLICQ_F32 ? run_analysis<float>(p, dt, tasks, S, x, coef, w, wk, st)
                         : run_analysis<double>(p, dt, tasks, S, x, coef, w, wk, st);
}

int64_t slicq_logmag_loss_partials(int64_t n) {
  if (n <= 0) return 1;
  return std::min<int64_t>(4096, (n + 4 * slicq::kLossThreads - 1) / (4 * slicq::kLossThreads));
}

int slicq_logmag_loss(slicq_dtype dt, const void* coef, const void* target, int64_t n, void* grad, void* partial,
                      int64_t partial_count, void* loss, void* stream) {
  if (dt != SLICQ_F32 && dt != SLICQ_F64) return fail(SLICQ_EINVAL, "bad dtype");
  if (n < 0) return fail(SLICQ_EINVAL, "n must be >= 0");
  if (!coef || !target || !grad || !partial || !loss) return fail(SLICQ_EINVAL, "null buffer");
  const int64_t nb = slicq_logmag_loss_partials(n);
  if (partial_count < nb) return fail(SLICQ_ESIZE, "partial_count < slicq_logmag_loss_partials(n)");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dt == SLICQ_F32) {
    hipLaunchKernelGGL(slicq::k_logmag_loss<float>, dim3((unsigned)nb), dim3(slicq::kLossThreads), 0, st,
                       static_cast<const slicq::C2<float>*>(coef), static_cast<const float*>(target), n,
                       static_cast<slicq::C2<float>*>(grad), static_cast<float*>(partial));
    hipLaunchKernelGGL(slicq::k_loss_sum<float>, dim3(1), dim3(slicq::kLossThreads), 0, st,
                       static_cast<const float*>(partial), (int)nb, static_cast<float*>(loss));
  } else {
    hipLaunchKernelGGL(slicq::k_logmag_loss<double>, dim3((unsigned)nb), dim3(slicq::kLossThreads), 0, st,
                       static_cast<const slicq::C2<double>*>(coef), static_cast<const double*>(target), n,
                       static_cast<slicq::C2<double>*>(grad), static_cast<double*>(partial));
    hipLaunchKernelGGL(slicq::k_loss_sum<double>, dim3(1), dim3(slicq::kLossThreads), 0, st,
                       static_cast<const double*>(partial), (int)nb, static_cast<double*>(loss));
  }
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? SLICQ_OK : hip_fail(e, "loss launch");
}

int slicq_synthesize(slicq_plan plan, slicq_dtype dt, const void* coef, int64_t coef_count, void* y, int64_t T,
                     void* work, size_t work_bytes, void* stream) {
  return synth_common(plan, dt, false, coef, coef_count, y, T, work, work_bytes, stream);
}

int slicq_adjoint(slicq_plan plan, slicq_dtype dt, const void* coef, int64_t coef_count, void* y, int64_t T,
                  void* work, size_t work_bytes, void* stream) {
  return synth_common(plan, dt, true, coef, coef_count, y, T, work, work_bytes, stream);
}

int slicq_analyze_batched(slicq_plan plan, slicq_dtype dt, const void* x, int64_t x_len, const int64_t* x_off,
                          int32_t nsig, int64_t total, void* coef, int64_t coef_len, const int64_t* coef_off,
                          void* work, size_t work_bytes, void* stream) {
  int rc = check_plan(plan, dt);
  if (rc) return rc;
  slicq::Plan& p = plan->p;
  if (nsig < 0 || total < 0) return fail(SLICQ_EINVAL, "nsig and total_slices must be >= 0");
  if (nsig == 0 || total == 0) return SLICQ_OK;
  if (!x || !x_off || !coef || !coef_off || !work) return fail(SLICQ_EINVAL, "null buffer");
  slicq::WorkLayout w;
  if ((rc = layout_or_fail(p, dt, total, work_bytes, w))) return rc;
  char* wk = static_cast<char*>(work);
  auto* tasks = reinterpret_cast<slicq::SliceTask*>(wk + w.tasks_off);
  hipStream_t st = static_cast<hipStream_t>(stream);
  batched_tasks(p, x_off, nsig, total, x_len, coef_off, coef_len, tasks,
                reinterpret_cast<int32_t*>(wk + w.status_off), st);
  return dt == SLICQ_F32 ? run_analysis<float>(p, dt, tasks, total, x, coef, w, wk, st)
                         : run_analysis<double>(p, dt, tasks, total, x, coef, w, wk, st);
}

int slicq_synthesize_batched(slicq_plan plan, slicq_dtype dt, const void* coef, int64_t coef_len,
                             const int64_t* coef_off, void* y, int64_t y_len, const int64_t* y_off, int32_t nsig,
                             int64_t total, void* work, size_t work_bytes, void* stream) {
  return synth_batched_common(plan, dt, false, coef, coef_len, coef_off, y, y_len, y_off, nsig, total, work,
                              work_bytes, stream);
}

int slicq_adjoint_batched(slicq_plan plan, slicq_dtype dt, const void* coef, int64_t coef_len,
                          const int64_t* coef_off, void* y, int64_t y_len, const int64_t* y_off, int32_t nsig,
                          int64_t total, void* work, size_t work_bytes, void* stream) {
  return synth_batched_common(plan, dt, true, coef, coef_len, coef_off, y, y_len, y_off, nsig, total, work,
                              work_bytes, stream);
}

int slicq_batched_status(slicq_plan plan, slicq_dtype dt, int64_t total, const void* work, size_t work_bytes,
                         int32_t* bad, int64_t* slices, void* stream) {
  if (!plan || !work || !bad) return fail(SLICQ_EINVAL, "null argument");
  if (dt != SLICQ_F32 && dt != SLICQ_F64) return fail(SLICQ_EINVAL, "bad dtype");
  if (total <= 0) return fail(SLICQ_EINVAL, "total_slices must be > 0");
  slicq::WorkLayout w;
  int rc = layout_or_fail(plan->p, dt, total, work_bytes, w);
  if (rc) return rc;
  int32_t hs[2] = {0, 0};
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(hs, static_cast<const char*>(work) + w.status_off, sizeof hs, hipMemcpyDeviceToHost,
                                st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "status read");
  *bad = hs[0] != 0 ? 1 : 0;
  if (slices) *slices = hs[1];
  return *bad ? fail(SLICQ_ESIZE, "the last batched call skipped a signal outside its buffers") : SLICQ_OK;
}

size_t slicq_batch_tasks_bytes(int64_t total_slices) {
  return total_slices < 0 ? 0 : slicq::tasks_bytes(total_slices) + 256;   // tasks, then two status words
}

int slicq_batch_create(slicq_plan plan, const int64_t* x_off, const int64_t* coef_off, int32_t nsig,
                       int64_t total, int64_t x_len, int64_t coef_len, void* tasks, size_t tasks_bytes,
                       void* stream, slicq_batch* out) {
  if (!out) return fail(SLICQ_EINVAL, "null output handle");
  *out = nullptr;
  if (!plan) return fail(SLICQ_EINVAL, "null plan");
  if (nsig <= 0 || total <= 0) return fail(SLICQ_EINVAL, "a prepared batch needs nsig > 0 and total_slices > 0");
  if (x_len < 0 || coef_len < 0) return fail(SLICQ_EINVAL, "x_len and coef_len must be >= 0");
  if (!x_off || !coef_off || !tasks) return fail(SLICQ_EINVAL, "null buffer");
  if (tasks_bytes < slicq_batch_tasks_bytes(total)) return fail(SLICQ_ESIZE, "tasks buffer too small");
  slicq::Plan& p = plan->p;
  auto* t = static_cast<slicq::SliceTask*>(tasks);
  auto* status = reinterpret_cast<int32_t*>(static_cast<char*>(tasks) + slicq::tasks_bytes(total));
  hipStream_t st = static_cast<hipStream_t>(stream);
  batched_tasks(p, x_off, nsig, total, x_len, coef_off, coef_len, t, status, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "task table launch");
  // one wait per prepared batch: a table with skipped signals is refused here
  int32_t hs[2] = {0, 0};
  e = hipMemcpyAsync(hs, status, sizeof hs, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "task table check");
  if (hs[0] != 0)
    return fail(SLICQ_ESIZE, "a signal's samples or coefficients fall outside x_len / coef_len, or the slices "
                             "exceed total_slices");
  if ((int64_t)hs[1] != total) {
    char b[160];
    std::snprintf(b, sizeof b, "the offsets describe %d slices, not total_slices = %lld", hs[1], (long long)total);
    return fail(SLICQ_ESIZE, b);
  }
  *out = new (std::nothrow) slicq_batch_s{plan, t, total, x_len, coef_len};
  return *out ? SLICQ_OK : fail(SLICQ_ENOMEM, "out of host memory");
}

void slicq_batch_destroy(slicq_batch batch) { delete batch; }

int slicq_analyze_batch(slicq_batch b, slicq_dtype dt, const void* x, int64_t x_len, void* coef, int64_t coef_len,
                        void* work, size_t work_bytes, void* stream) {
  if (!b) return fail(SLICQ_EINVAL, "null batch");
  int rc = check_plan(b->plan, dt);
  if (rc) return rc;
  if (!x || !coef || !work) return fail(SLICQ_EINVAL, "null buffer");
  if (x_len < b->x_len || coef_len < b->coef_len)
    return fail(SLICQ_ESIZE, "buffers are shorter than the batch was prepared for");
  slicq::Plan& p = b->plan->p;
  slicq::WorkLayout w;
  if ((rc = layout_or_fail(p, dt, b->total, work_bytes, w))) return rc;
  char* wk = static_cast<char*>(work);
  hipStream_t st = static_cast<hipStream_t>(stream);
  return dt == SLICQ_F32 ? run_analysis<float>(p, dt, b->tasks, b->total, x, coef, w, wk, st)
                         : run_analysis<double>(p, dt, b->tasks, b->total, x, coef, w, wk, st);
}

static int synth_batch_common(slicq_batch b, slicq_dtype dt, bool adjoint, const void* coef, int64_t coef_len,
                              void* y, int64_t y_len, void* work, size_t work_bytes, void* stream) {
  if (!b) return fail(SLICQ_EINVAL, "null batch");
  int rc = check_plan(b->plan, dt);
  if (rc) return rc;
  if (!coef || !y || !work) return fail(SLICQ_EINVAL, "null buffer");
  if (y_len < b->x_len || coef_len < b->coef_len)
    return fail(SLICQ_ESIZE, "buffers are shorter than the batch was prepared for");
  slicq::Plan& p = b->plan->p;
  slicq::WorkLayout w;
  if ((rc = layout_or_fail(p, dt, b->total, work_bytes, w))) return rc;
  char* wk = static_cast<char*>(work);
  hipStream_t st = static_cast<hipStream_t>(stream);
  return dt == SLICQ_F32 ? run_synthesis<float>(p, dt, adjoint, b->tasks, b->total, coef, y, w, wk, st)
                         : run_synthesis<double>(p, dt, adjoint, b->tasks, b->total, coef, y, w, wk, st);
}

int slicq_synthesize_batch(slicq_batch b, slicq_dtype dt, const void* coef, int64_t coef_len, void* y, int64_t y_len,
                           void* work, size_t work_bytes, void* stream) {
  return synth_batch_common(b, dt, false, coef, coef_len, y, y_len, work, work_bytes, stream);
}

int slicq_adjoint_batch(slicq_batch b, slicq_dtype dt, const void* coef, int64_t coef_len, void* y, int64_t y_len,
                        void* work, size_t work_bytes, void* stream) {
  return synth_batch_common(b, dt, true, coef, coef_len, y, y_len, work, work_bytes, stream);
}

static int profile_stage_impl(slicq::Plan& p, slicq_dtype dt, int stage, int64_t n_slices,
                              const slicq::SliceTask* tasks, const void* x, void* coef, void* y,
                              const slicq::WorkLayout& w, char* wk, hipStream_t st) {
  HipLaunch L{st};
  auto go = [&](auto tag) {
    using T = decltype(tag);
    using namespace slicq;
    KArgs<T> a = make_args<T>(p, dt, false);
    const Geometry<T> g = geometry<T>(p);
    C2<T>* W1 = reinterpret_cast<C2<T>*>(wk + w.w1_off);
    C2<T>* W2 = reinterpret_cast<C2<T>*>(wk + w.w2_off);
    const int64_t n = n_slices;
    if (a.fused) {
      // one workgroup per slice: stage 0 runs the fused analysis, 3 the fused
      // synthesis (whole slices), 5 the overlap fix-up; the others are empty
      a.task0 = 0;
      a.task1 = n;
      if (stage == 0) launch_ana_fused(p, a, tasks, n, static_cast<const T*>(x), static_cast<C2<T>*>(coef), L);
      else if (stage == 3) launch_syn_fused(p, a, tasks, n, (const C2<T>*)coef, W2, static_cast<T*>(y), L);
      else if (stage == 5) launch_ola_fix(a, tasks, n, (const C2<T>*)W2, static_cast<T*>(y), L);
      return;
    }
    switch (stage) {
      case 0: L.launch(k_fwd_pass1<T, true>, n * g.g1, g.b1, g.s1, a, tasks, static_cast<const T*>(x), W1); break;
      case 1: L.launch(k_fwd_pass2<T, true>, n * g.g2, g.b2, g.s2, a, (const C2<T>*)W1, W2); break;
      case 2:
        launch_band_ana(a, g, tasks, n, (const C2<T>*)W2, static_cast<C2<T>*>(coef), L);
        break;
      case 3:
        launch_band_syn(a, g, tasks, n, (const C2<T>*)coef, W2, static_cast<T*>(y), L);
        break;
      case 4: L.launch(k_inv_passA<T, true>, n * g.g2, g.b2, g.s2, a, (const C2<T>*)W2, W1); break;
      default: launch_inv_passB(a, g, tasks, 0, n, W1, W2, static_cast<T*>(y), L); break;
    }
  };
  if (dt == SLICQ_F32) go(float{});
  else go(double{});
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? SLICQ_OK : hip_fail(e, "stage launch");
}

int slicq_profile_stage(slicq_plan plan, slicq_dtype dt, int stage, int64_t n_slices, const void* x, void* coef,
                        void* y, void* work, size_t work_bytes, void* stream) {
  int rc = check_plan(plan, dt);
  if (rc) return rc;
  slicq::Plan& p = plan->p;
  if (stage < 0 || stage > 5) return fail(SLICQ_EINVAL, "stage must be in 0..5");
  if (n_slices <= 0 || !x || !coef || !y || !work) return fail(SLICQ_EINVAL, "bad argument");
  slicq::WorkLayout w;
  if ((rc = layout_or_fail(p, dt, n_slices, work_bytes, w))) return rc;
  if (w.chunk < n_slices) return fail(SLICQ_ESIZE, "profiling needs a workspace for all slices at once");
  char* wk = static_cast<char*>(work);
  const auto* tasks = reinterpret_cast<const slicq::SliceTask*>(wk + w.tasks_off);
  return profile_stage_impl(p, dt, stage, n_slices, tasks, x, coef, y, w, wk, static_cast<hipStream_t>(stream));
}

int slicq_profile_stage_batch(slicq_batch b, slicq_dtype dt, int stage, const void* x, int64_t x_len, void* coef,
                              int64_t coef_len, void* y, int64_t y_len, void* work, size_t work_bytes, void* stream) {
  if (!b) return fail(SLICQ_EINVAL, "null batch");
  int rc = check_plan(b->plan, dt);
  if (rc) return rc;
  slicq::Plan& p = b->plan->p;
  if (stage < 0 || stage > 5) return fail(SLICQ_EINVAL, "stage must be in 0..5");
  if (!x || !coef || !y || !work) return fail(SLICQ_EINVAL, "null buffer");
  if (x_len < b->x_len || y_len < b->x_len || coef_len < b->coef_len)
    return fail(SLICQ_ESIZE, "buffers are shorter than the batch was prepared for");
  slicq::WorkLayout w;
  if ((rc = layout_or_fail(p, dt, b->total, work_bytes, w))) return rc;
  if (w.chunk < b->total) return fail(SLICQ_ESIZE, "profiling needs a workspace for all slices at once");
  return profile_stage_impl(p, dt, stage, b->total, b->tasks, x, coef, y, w, static_cast<char*>(work),
                            static_cast<hipStream_t>(stream));
}

const char* slicq_last_error(void) { return g_err.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------
// Full-length CQ-NSGT (Algorithms 1 and 2 at the signal length L)

namespace {

int check_full(slicq_full full, slicq_dtype dt) {
  if (!full) return fail(SLICQ_EINVAL, "null full-length plan");
  if (dt != SLICQ_F32 && dt != SLICQ_F64) return fail(SLICQ_EINVAL, "dtype must be SLICQ_F32 or SLICQ_F64");
  if (!full->f.dev[dt]) return fail(SLICQ_ESTATE, "full-length tables not uploaded for this dtype (nsgt_full_upload)");
  return SLICQ_OK;
}

}  // namespace

extern "C" {

int nsgt_full_plan(slicq_plan plan, int64_t L, int32_t lattice, slicq_full* out) {
  if (!plan || !out) return fail(SLICQ_EINVAL, "null argument");
  *out = nullptr;
  auto* h = new (std::nothrow) slicq_full_s();
  if (!h) return fail(SLICQ_ENOMEM, "out of host memory");
  std::string err;
  if (slicq::build_full(plan->p, L, lattice, h->f, err) != 0) {
    delete h;
    return fail(SLICQ_EINVAL, err);
  }
  *out = h;
  return SLICQ_OK;
}

void nsgt_full_destroy(slicq_full full) { delete full; }

int nsgt_full_info(slicq_full full, slicq_full_info* info) {
  if (!full || !info) return fail(SLICQ_EINVAL, "null argument");
  const slicq::FullPlan& f = full->f;
  std::memset(info, 0, sizeof *info);
  info->L = f.L;
  info->nbands = f.nb;
  info->lattice = f.lattice;
  info->painless = f.painless ? 1 : 0;
  info->coef_count = f.coef_count;
  info->max_M = f.max_M;
  info->entries = (int64_t)f.ent_idx.size();
  return SLICQ_OK;
}

int nsgt_full_bands(slicq_full full, int64_t* start, int32_t* len, int32_t* M, int64_t* off) {
  if (!full) return fail(SLICQ_EINVAL, "null full-length plan");
  const auto& b = full->f.bands;
  for (size_t k = 0; k < b.size(); ++k) {
    if (start) start[k] = b[k].start;
    if (len) len[k] = b[k].len;
    if (M) M[k] = b[k].M;
    if (off) off[k] = b[k].off;
  }
  return SLICQ_OK;
}

int nsgt_full_windows(slicq_full full, double* g, double* gd) {
  if (!full) return fail(SLICQ_EINVAL, "null full-length plan");
  const slicq::FullPlan& f = full->f;
  if (g) std::memcpy(g, f.g.data(), f.g.size() * sizeof(double));
  if (gd)
    for (const auto& b : f.bands)
      for (int32_t t = 0; t < b.len; ++t) {
        int64_t j = (b.start + t) % f.L;
        if (j < 0) j += f.L;
        gd[b.goff + t] = f.g[b.goff + t] / f.D[j];
      }
  return SLICQ_OK;
}

int nsgt_full_table_bytes(slicq_full full, slicq_dtype dt, size_t* bytes) {
  if (!full || !bytes) return fail(SLICQ_EINVAL, "null argument");
  if (dt != SLICQ_F32 && dt != SLICQ_F64) return fail(SLICQ_EINVAL, "bad dtype");
  std::lock_guard<std::mutex> lk(full->f.mu);
  if (full->blob[dt].empty()) slicq::pack_full_tables(full->f, dt, full->blob[dt], full->f.layout[dt]);
  *bytes = full->blob[dt].size();
  return SLICQ_OK;
}

int nsgt_full_upload(slicq_full full, slicq_dtype dt, void* dev, size_t bytes, void* stream) {
  size_t need = 0;
  int rc = nsgt_full_table_bytes(full, dt, &need);
  if (rc) return rc;
  if (!dev) return fail(SLICQ_EINVAL, "null device pointer");
  if (reinterpret_cast<uintptr_t>(dev) & 255) return fail(SLICQ_EINVAL, "device tables must be 256-byte aligned");
  if (bytes < need) return fail(SLICQ_ESIZE, "device table buffer too small");
  std::lock_guard<std::mutex> lk(full->f.mu);
  hipError_t e = hipMemcpyAsync(dev, full->blob[dt].data(), need, hipMemcpyHostToDevice,
                                static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "table upload");
  full->f.dev[dt] = dev;
  full->f.dev_bytes[dt] = bytes;
  return SLICQ_OK;
}

int nsgt_full_workspace_size(slicq_full full, slicq_dtype dt, size_t* bytes) {
  if (!full || !bytes) return fail(SLICQ_EINVAL, "null argument");
  if (dt != SLICQ_F32 && dt != SLICQ_F64) return fail(SLICQ_EINVAL, "bad dtype");
  *bytes = slicq::full_work(full->f, dt).total;
  return SLICQ_OK;
}

int nsgt_full_analyze(slicq_full full, slicq_dtype dt, const void* x, void* coef, int64_t coef_count, void* work,
                      size_t work_bytes, void* stream) {
  int rc = check_full(full, dt);
  if (rc) return rc;
  const slicq::FullPlan& f = full->f;
  if (!x || !coef || !work) return fail(SLICQ_EINVAL, "null buffer");
  if (coef_count < f.coef_count) return fail(SLICQ_ESIZE, "coef_count below the plan's coefficient count");
  const slicq::FullWork w = slicq::full_work(f, dt);
  if (work_bytes < w.total) return fail(SLICQ_ESIZE, "workspace smaller than nsgt_full_workspace_size");
  const char* tabs = static_cast<const char*>(f.dev[dt]);
  HipLaunch ln{static_cast<hipStream_t>(stream)};
  if (dt == SLICQ_F32)
    slicq::full_analyze_launch<float>(ln, f, tabs, f.layout[dt], static_cast<const slicq::C2<float>*>(x),
                                      static_cast<slicq::C2<float>*>(coef), static_cast<char*>(work), w);
  else
    slicq::full_analyze_launch<double>(ln, f, tabs, f.layout[dt], static_cast<const slicq::C2<double>*>(x),
                                       static_cast<slicq::C2<double>*>(coef), static_cast<char*>(work), w);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? SLICQ_OK : hip_fail(e, "full-length analysis launch");
}

int nsgt_full_synthesize(slicq_full full, slicq_dtype dt, const void* coef, int64_t coef_count, void* y, void* work,
                         size_t work_bytes, void* stream) {
  int rc = check_full(full, dt);
  if (rc) return rc;
  const slicq::FullPlan& f = full->f;
  if (!f.painless)
    return fail(SLICQ_EINVAL, "synthesis needs M_k >= |J_k| on every band (painless lattice, Proposition 2); "
                              "this plan's lattice aliases some band");
  if (!y || !coef || !work) return fail(SLICQ_EINVAL, "null buffer");
  if (coef_count < f.coef_count) return fail(SLICQ_ESIZE, "coef_count below the plan's coefficient count");
  const slicq::FullWork w = slicq::full_work(f, dt);
  if (work_bytes < w.total) return fail(SLICQ_ESIZE, "workspace smaller than nsgt_full_workspace_size");
  const char* tabs = static_cast<const char*>(f.dev[dt]);
  HipLaunch ln{static_cast<hipStream_t>(stream)};
  if (dt == SLICQ_F32)
    slicq::full_synthesize_launch<float>(ln, f, tabs, f.layout[dt], static_cast<const slicq::C2<float>*>(coef),
                                         static_cast<slicq::C2<float>*>(y), static_cast<char*>(work), w);
  else
    slicq::full_synthesize_launch<double>(ln, f, tabs, f.layout[dt], static_cast<const slicq::C2<double>*>(coef),
                                          static_cast<slicq::C2<double>*>(y), static_cast<char*>(work), w);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? SLICQ_OK : hip_fail(e, "full-length synthesis launch");
}

}  // extern "C"
