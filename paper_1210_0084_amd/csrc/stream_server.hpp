// Streaming sliCQ service: many real-time audio streams, continuously batched.
//
// Each admitted stream owns a slot with an input ring and an output ring of
// R = 4N samples in device memory. A stream is the linear (non-circular)
// sliCQ of an unbounded signal that is zero before sample 0: slice m is
// centred on sample mN (Algorithm 3) and needs samples up to
// mN + (N+M)/2 - 1, so it becomes ready once that many samples have been
// pushed. Each tick
//   1. packs the newly pushed samples of every stream into one staging buffer
//      and scatters them into the input rings (one copy, one kernel);
//   2. runs analysis and synthesis (Algorithms 3-4) for every ready slice of
//      every stream in one launch sequence;
//   3. gathers the output samples that became final (all of sample t's slices
//      processed, t <= mN + (N-M)/2 after slice m) into one staging buffer
//      and copies them to the host.
// Pushes and polls from other threads proceed while a tick's work is on the
// device; what arrives meanwhile joins the next tick (continuous batching).
// Admission is bounded by a device-memory budget (slots are preallocated).
//
// Templated on the device backend (allocation, copies, launches, waits) so
// that the same scheduler can be run on the host by the test harness.
#pragma once
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <vector>

#include "pipeline.hpp"

namespace slicq {

struct StreamStats {
  int64_t ticks = 0, slices = 0, samples_in = 0, samples_out = 0;
  int64_t admitted = 0, rejected = 0, closed = 0, gaps = 0;
  double latency_p50 = 0, latency_p99 = 0, latency_max = 0;   // seconds
  int64_t latency_count = 0;
  double busy_seconds = 0;                                    // host time inside ticks
};

// FIFO of samples in one contiguous vector with a read offset (bulk append
// and bulk read with memcpy; the consumed front is dropped once it is the
// larger half).
template <class T>
class SampleFifo {
 public:
  int64_t size() const { return (int64_t)(buf_.size() - head_); }
  const T* data() const { return buf_.data() + head_; }
  void append(const T* x, int64_t n) {
    if (n > 0) buf_.insert(buf_.end(), x, x + n);
  }
  // Moves the first n (<= size()) samples to y.
  void read(T* y, int64_t n) {
    if (n <= 0) return;
    std::memcpy(y, buf_.data() + head_, (size_t)n * sizeof(T));
    head_ += (size_t)n;
    if (head_ == buf_.size()) {
      buf_.clear();
      head_ = 0;
    } else if (head_ >= 4096 && 2 * head_ >= buf_.size()) {
      buf_.erase(buf_.begin(), buf_.begin() + (std::ptrdiff_t)head_);
      head_ = 0;
    }
  }
  void assign(const T* x, int64_t n) {
    buf_.assign(x, x + n);
    head_ = 0;
  }

 private:
  std::vector<T> buf_;
  size_t head_ = 0;
};

template <class T, class Backend>
class StreamServer {
 public:
  struct Stream {
    bool active = false;
    int64_t pushed = 0;        // samples pushed by the producer
    int64_t on_device = 0;     // samples moved into the device input ring
    int64_t next_slice = 0;    // m of the next slice to process
    int64_t released = 0;      // output samples moved to `out`
    SampleFifo<T> pending;     // pushed, not yet on the device
    SampleFifo<T> out;         // final output samples, not yet polled
    std::deque<std::pair<int64_t, double>> arrivals;   // (pushed after a push, time)
    int64_t last_m = -1;       // most recent processed slice
    int64_t last_task = -1;    // its index in the last tick's coefficient buffer
  };

  StreamServer(Plan& plan, int dtype, Backend& be, int max_streams, int max_batch, size_t budget_bytes)
      : p_(plan), dt_(dtype), be_(be) {
    N_ = p_.N;
    R_ = 4 * p_.N;
    cps_ = p_.coefs_per_slice;
    max_batch_ = std::max(max_batch, 1);
    // device bytes: per slot two rings, its share of the staging buffer and
    // two copy records; fixed: the workspace and coefficients of max_batch
    // slices and the spare copy records
    per_stream_ = 3 * (size_t)R_ * sizeof(T) + 2 * sizeof(RingCopy);
    fixed_ = workspace_bytes(p_, dt_, max_batch_) + (size_t)max_batch_ * cps_ * sizeof(C2<T>) + 2 * sizeof(RingCopy);
    int64_t cap = max_streams;
    if (budget_bytes > 0)
      cap = budget_bytes > fixed_ ? std::min<int64_t>(cap, (int64_t)((budget_bytes - fixed_) / per_stream_)) : 0;
    slots_ = (int)std::max<int64_t>(cap, 0);
    streams_.resize(slots_);
  }

  ~StreamServer() { release(); }

  // Allocates every device and pinned buffer; false on failure.
  bool init(std::string& err) {
    if (slots_ <= 0) {
      err = "memory budget admits no stream";
      return false;
    }
    const size_t ring_bytes = (size_t)slots_ * R_ * sizeof(T);
    work_bytes_ = workspace_bytes(p_, dt_, max_batch_);   // counted in fixed_
    staging_cap_ = (int64_t)slots_ * R_;
    xring_ = (T*)be_.dmalloc(ring_bytes);
    yring_ = (T*)be_.dmalloc(ring_bytes);
    coef_ = (C2<T>*)be_.dmalloc((size_t)max_batch_ * cps_ * sizeof(C2<T>));
    work_ = (char*)be_.dmalloc(work_bytes_);
    stage_d_ = (T*)be_.dmalloc((size_t)staging_cap_ * sizeof(T));
    copies_d_ = (RingCopy*)be_.dmalloc((size_t)2 * (slots_ + 1) * sizeof(RingCopy));
    stage_h_ = (T*)be_.hmalloc((size_t)staging_cap_ * sizeof(T));
    tasks_h_ = (SliceTask*)be_.hmalloc((size_t)max_batch_ * sizeof(SliceTask));
    if (!xring_ || !yring_ || !coef_ || !work_ || !stage_d_ || !copies_d_ || !stage_h_ || !tasks_h_) {
      err = "allocation of the stream buffers failed";
      return false;
    }
    if (!work_layout(p_, dt_, max_batch_, work_bytes_, wl_) || wl_.chunk < max_batch_) {
      err = "workspace layout failed";
      return false;
    }
    geo_ = geometry<T>(p_);
    if (!geo_.ok) {
      err = "plan work items exceed the kernels' block limits";
      return false;
    }
    zero(xring_, (int64_t)slots_ * R_);
    zero(yring_, (int64_t)slots_ * R_);
    if (!be_.sync()) {
      err = "device error while clearing the rings";
      return false;
    }
    return true;
  }

  static T* ring_type() { return nullptr; }   // names the sample type for generic callers
  int slots() const { return slots_; }
  int64_t ring() const { return R_; }
  int64_t coefs_per_slice() const { return cps_; }
  size_t per_stream_bytes() const { return per_stream_; }
  size_t fixed_bytes() const { return fixed_; }

  // Admission: returns a slot id >= 0, or -1 if every slot is taken.
  int open() {
    std::lock_guard<std::mutex> lk(mu_);
    for (int s = 0; s < slots_; ++s) {
      if (!streams_[s].active && !dirty(s)) {
        streams_[s] = Stream();
        streams_[s].active = true;
        ++st_.admitted;
        return s;
      }
    }
    ++st_.rejected;
    return -1;
  }

  bool valid(int id) const { return id >= 0 && id < slots_ && streams_[id].active; }

  // Appends n samples (host memory) to stream id.
  void push(int id, const T* x, int64_t n) {
    const double t = now();
    std::lock_guard<std::mutex> lk(mu_);
    Stream& s = streams_[id];
    s.pending.append(x, n);
    s.pushed += n;
    s.arrivals.emplace_back(s.pushed, t);
    st_.samples_in += n;
  }

  // A hop that never arrived: n zero samples, counted as a gap.
  void push_gap(int id, int64_t n) {
    std::vector<T> z((size_t)n, T(0));
    push(id, z.data(), n);
    std::lock_guard<std::mutex> lk(mu_);
    st_.gaps += n;
  }

  // Copies up to max final output samples of stream id into y; returns the count.
  int64_t poll(int id, T* y, int64_t max) {
    std::lock_guard<std::mutex> lk(mu_);
    Stream& s = streams_[id];
    const int64_t n = std::min<int64_t>(max, s.out.size());
    s.out.read(y, n);
    return n;
  }

  // Ends stream id; its slot is cleared on the device before reuse.
  void close(int id) {
    std::lock_guard<std::mutex> lk(mu_);
    streams_[id] = Stream();
    to_clear_.push_back(id);
    ++st_.closed;
  }

  // One batch: move samples, process every ready slice (up to max_batch),
  // release final output. Returns the number of slices, or -1 on a device error.
  int64_t tick() {
    std::lock_guard<std::mutex> tick_lk(tick_mu_);
    if (fenced_) return -1;
    const double t0 = now();
    std::vector<RingCopy> in_copies, out_copies;
    std::vector<std::pair<int, int64_t>> done;        // (slot, m) processed this tick
    std::vector<int> clear;
    int64_t staged = 0, ntask = 0;
    {
      std::lock_guard<std::mutex> lk(mu_);
      clear.swap(to_clear_);
      for (int id = 0; id < slots_; ++id) {
        Stream& s = streams_[id];
        if (!s.active) continue;
        // input ring holds samples [(next_slice - 1) N, (next_slice - 1) N + R)
        const int64_t limit = (s.next_slice - 1) * N_ + R_;
        const int64_t n = std::min<int64_t>(s.pending.size(), limit - s.on_device);
        if (n > 0 && staged + n <= staging_cap_) {
          s.pending.read(stage_h_ + staged, n);
          in_copies.push_back({id, (int32_t)n, s.on_device & (R_ - 1), staged});
          staged += n;
          s.on_device += n;
        }
      }
      // round robin: start with the stream the previous tick's batch could not
      // take (a stream holds at most R/N ready slices, so every stream is
      // served within a bounded number of ticks)
      const int start = rr_;
      bool full = false;
      for (int i = 0; i < slots_ && !full; ++i) {
        const int id = (start + i) % slots_;
        Stream& s = streams_[id];
        while (s.active && s.on_device >= s.next_slice * N_ + (N_ + p_.Mt) / 2) {
          if (ntask == max_batch_) {       // full: this stream is served first next tick
            rr_ = id;
            full = true;
            break;
          }
          const int64_t m = s.next_slice++;
          SliceTask tk{};
          tk.x_base = (int64_t)id * R_;
          tk.x_start = ((m - 1) * N_) & (R_ - 1);
          tk.x_period = R_;
          tk.x_valid = R_;
          tk.y_base = (int64_t)id * R_;
          tk.y_start = tk.x_start;
          tk.y_period = R_;
          tk.y_valid = R_;
          tk.coef_base = ntask * cps_;
          tk.m = 0;
          tk.S = 1;
          tk.flags = 1;
          s.last_m = m;
          s.last_task = ntask;
          tasks_h_[ntask++] = tk;
          done.emplace_back(id, m);
        }
      }
    }
    // device work (no host lock held: pushes and polls continue meanwhile)
    {
      // coefficients of earlier ticks are overwritten by this one
      std::lock_guard<std::mutex> lk(mu_);
      for (int id = 0; id < slots_; ++id) {
        bool here = false;
        for (auto& dm : done) here = here || dm.first == id;
        if (!here) streams_[id].last_task = -1;
      }
    }
    for (int id : clear) {
      zero(xring_ + (int64_t)id * R_, R_);
      zero(yring_ + (int64_t)id * R_, R_);
    }
    if (!in_copies.empty()) {
      be_.h2d(stage_d_, stage_h_, (size_t)staged * sizeof(T));
      be_.h2d(copies_d_, in_copies.data(), in_copies.size() * sizeof(RingCopy));
      be_.launch(k_ring_copy<T>, (int64_t)in_copies.size(), 256, 0, (const RingCopy*)copies_d_, stage_d_, xring_,
                 R_, (int32_t)1);
    }
    if (ntask > 0) {
      SliceTask* tasks_d = reinterpret_cast<SliceTask*>(work_ + wl_.tasks_off);
      be_.h2d(tasks_d, tasks_h_, (size_t)ntask * sizeof(SliceTask));
      C2<T>* W1 = reinterpret_cast<C2<T>*>(work_ + wl_.w1_off);
      C2<T>* W2 = reinterpret_cast<C2<T>*>(work_ + wl_.w2_off);
      KArgs<T> a = make_args<T>(p_, dt_, false);
      launch_analysis<T>(p_, a, geo_, tasks_d, ntask, xring_, coef_, W1, W2, be_);
      launch_synthesis<T>(p_, a, geo_, tasks_d, 0, ntask, coef_, yring_, W1, W2, be_);
    }
    // release output made final by this tick's slices
    int64_t gathered = 0;
    std::vector<int64_t> rel_upto(slots_, -1);
    {
      std::lock_guard<std::mutex> lk(mu_);
      for (auto& dm : done) {
        const int64_t fin = dm.second * N_ + (N_ - p_.Mt) / 2 + 1;   // samples < fin are final
        rel_upto[dm.first] = std::max(rel_upto[dm.first], fin);
      }
      for (int id = 0; id < slots_; ++id) {
        if (rel_upto[id] < 0 || !streams_[id].active) continue;
        Stream& s = streams_[id];
        const int64_t n = rel_upto[id] - s.released;
        if (n <= 0) continue;
        out_copies.push_back({id, (int32_t)n, s.released & (R_ - 1), gathered});
        gathered += n;
      }
    }
    if (!out_copies.empty()) {
      RingCopy* out_d = copies_d_ + (slots_ + 1);
      be_.h2d(out_d, out_copies.data(), out_copies.size() * sizeof(RingCopy));
      be_.launch(k_ring_copy<T>, (int64_t)out_copies.size(), 256, 0, (const RingCopy*)out_d, stage_d_, yring_,
                 R_, (int32_t)0);
      be_.d2h(stage_h_, stage_d_, (size_t)gathered * sizeof(T));
    }
    if (!be_.sync()) return fence();
    const double t1 = now();
    {
      std::lock_guard<std::mutex> lk(mu_);
      for (const RingCopy& c : out_copies) {
        Stream& s = streams_[c.slot];
        if (!s.active) continue;
        s.out.append(stage_h_ + c.off, c.count);
        s.released += c.count;
        st_.samples_out += c.count;
      }
      for (auto& dm : done) {
        Stream& s = streams_[dm.first];
        const int64_t thr = dm.second * N_ + (N_ + p_.Mt) / 2;   // samples the slice needs
        double tr = -1;
        for (auto& a : s.arrivals) {
          if (a.first >= thr) {
            tr = a.second;
            break;
          }
        }
        if (tr >= 0) record_latency(t1 - tr);
        while (s.arrivals.size() > 1 && s.arrivals[1].first <= thr) s.arrivals.pop_front();
      }
      st_.ticks += 1;
      st_.slices += ntask;
      st_.busy_seconds += t1 - t0;
    }
    return ntask;
  }

  StreamStats stats() {
    std::lock_guard<std::mutex> lk(mu_);
    StreamStats s = st_;
    if (!lat_.empty()) {
      std::vector<double> v(lat_);
      std::sort(v.begin(), v.end());
      auto pct = [&](double q) { return v[std::min(v.size() - 1, (size_t)std::floor(q * (v.size() - 1) + 0.5))]; };
      s.latency_p50 = pct(0.50);
      s.latency_p99 = pct(0.99);
      s.latency_max = v.back();
      s.latency_count = (int64_t)v.size();
    }
    return s;
  }

  void reset_stats() {
    std::lock_guard<std::mutex> lk(mu_);
    st_ = StreamStats();
    lat_.clear();
  }

  // Snapshot of stream id: counters, host queues and both device rings.
  bool snapshot(int id, std::vector<unsigned char>& blob) {
    std::lock_guard<std::mutex> tick_lk(tick_mu_);
    std::lock_guard<std::mutex> lk(mu_);
    const Stream& s = streams_[id];
    std::vector<T> xr(R_), yr(R_);
    be_.d2h(xr.data(), xring_ + (int64_t)id * R_, R_ * sizeof(T));
    be_.d2h(yr.data(), yring_ + (int64_t)id * R_, R_ * sizeof(T));
    if (!be_.sync()) return false;
    int64_t hdr[8] = {0x51494c53, R_, (int64_t)sizeof(T), s.pushed, s.on_device, s.next_slice, s.released,
                      s.pending.size()};
    const int64_t nout = s.out.size();
    blob.clear();
    auto put = [&](const void* p, size_t n) {
      if (n == 0) return;
      const size_t o = blob.size();
      blob.resize(o + n);
      std::memcpy(blob.data() + o, p, n);
    };
    put(hdr, sizeof hdr);
    put(&nout, sizeof nout);
    put(xr.data(), R_ * sizeof(T));
    put(yr.data(), R_ * sizeof(T));
    put(s.pending.data(), (size_t)s.pending.size() * sizeof(T));
    put(s.out.data(), (size_t)nout * sizeof(T));
    return true;
  }

  // Restores a snapshot into the open stream id; false if the blob does not fit.
  bool restore(int id, const unsigned char* blob, size_t bytes) {
    std::lock_guard<std::mutex> tick_lk(tick_mu_);
    std::lock_guard<std::mutex> lk(mu_);
    int64_t hdr[8], nout;
    if (bytes < sizeof hdr + sizeof nout) return false;
    std::memcpy(hdr, blob, sizeof hdr);
    std::memcpy(&nout, blob + sizeof hdr, sizeof nout);
    if (hdr[0] != 0x51494c53 || hdr[1] != R_ || hdr[2] != (int64_t)sizeof(T)) return false;
    const size_t need = sizeof hdr + sizeof nout + 2 * R_ * sizeof(T) + (size_t)(hdr[7] + nout) * sizeof(T);
    if (bytes != need) return false;
    const unsigned char* p = blob + sizeof hdr + sizeof nout;
    std::vector<T> xr(R_), yr(R_);
    std::memcpy(xr.data(), p, R_ * sizeof(T));
    std::memcpy(yr.data(), p + R_ * sizeof(T), R_ * sizeof(T));
    p += 2 * R_ * sizeof(T);
    be_.h2d(xring_ + (int64_t)id * R_, xr.data(), R_ * sizeof(T));
    be_.h2d(yring_ + (int64_t)id * R_, yr.data(), R_ * sizeof(T));
    if (!be_.sync()) return false;
    Stream& s = streams_[id];
    s = Stream();
    s.active = true;
    s.pushed = hdr[3];
    s.on_device = hdr[4];
    s.next_slice = hdr[5];
    s.released = hdr[6];
    const T* q = reinterpret_cast<const T*>(p);
    s.pending.assign(q, hdr[7]);
    s.out.assign(q + hdr[7], nout);
    s.arrivals.emplace_back(s.pushed, now());
    return true;
  }

  bool fenced() const { return fenced_; }

  // Coefficients (slice-major c^m, coefs_per_slice values) of stream id's most
  // recent slice if the last tick processed it; returns its m or -1.
  int64_t last_coefs(int id, C2<T>* out) {
    std::lock_guard<std::mutex> tick_lk(tick_mu_);
    int64_t task, m;
    {
      std::lock_guard<std::mutex> lk(mu_);
      task = streams_[id].last_task;
      m = streams_[id].last_m;
    }
    if (task < 0) return -1;
    be_.d2h(out, coef_ + task * cps_, (size_t)cps_ * sizeof(C2<T>));
    if (!be_.sync()) return -1;
    return m;
  }

 private:
  bool dirty(int s) const { return std::find(to_clear_.begin(), to_clear_.end(), s) != to_clear_.end(); }

  void zero(T* ptr, int64_t n) {
    if (n > 0) be_.launch(k_fill_zero<T>, (n + 255) / 256, 256, 0, ptr, n);
  }

  int64_t fence() {
    fenced_ = true;
    return -1;
  }

  void record_latency(double s) {
    if (lat_.size() >= kMaxLatencies) lat_.erase(lat_.begin(), lat_.begin() + kMaxLatencies / 2);
    lat_.push_back(s);
  }

  static double now() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
  }

  void release() {
    be_.dfree(xring_);
    be_.dfree(yring_);
    be_.dfree(coef_);
    be_.dfree(work_);
    be_.dfree(stage_d_);
    be_.dfree(copies_d_);
    be_.hfree(stage_h_);
    be_.hfree(tasks_h_);
    xring_ = yring_ = stage_d_ = stage_h_ = nullptr;
  }

  static constexpr size_t kMaxLatencies = 1 << 20;

  Plan& p_;
  int dt_;
  Backend& be_;
  int64_t N_ = 0, R_ = 0, cps_ = 0, staging_cap_ = 0;
  size_t per_stream_ = 0, fixed_ = 0, work_bytes_ = 0;
  int slots_ = 0, max_batch_ = 0, rr_ = 0;
  std::vector<Stream> streams_;
  std::vector<int> to_clear_;
  std::vector<double> lat_;
  StreamStats st_;
  std::mutex mu_, tick_mu_;
  bool fenced_ = false;
  WorkLayout wl_{};
  Geometry<T> geo_{};
  T *xring_ = nullptr, *yring_ = nullptr, *stage_d_ = nullptr, *stage_h_ = nullptr;
  C2<T>* coef_ = nullptr;
  char* work_ = nullptr;
  RingCopy* copies_d_ = nullptr;
  SliceTask* tasks_h_ = nullptr;
};

}  // namespace slicq
