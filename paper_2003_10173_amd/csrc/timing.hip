// Launch timing of selected kernels for roofline reporting: while enabled,
// each timed launch is bracketed by HIP events recorded on the stream it is
// launched on, together with the algorithmic work it performs (flops or
// bytes, computed on the host from the shapes; optionally times a count the
// kernel writes to device memory, such as the number of Jacobi sweeps).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>

#include "internal.h"
#include "timing.h"

namespace h2 {

h2_status guarded_status(const std::function<void()>& f);

namespace {
struct Rec {
  std::string name;
  hipEvent_t e0, e1;
  double work, work_per_count;
  int slot;  // pinned count slot, -1: none
};
struct State {
  std::mutex mu;
  bool on = false;
  std::vector<Rec> recs;
  int* pinned = nullptr;  // count slots (host-mapped pinned memory)
  int nslots = 0, used = 0;
  struct Sum { int64_t launches = 0; double ms = 0, work = 0; };
  std::map<std::string, Sum> sums;
};
State& st() {
  static State s;
  return s;
}

void drain(State& s) {
  for (auto& r : s.recs) {
    H2_HIP(hipEventSynchronize(r.e1));
    float ms = 0;
    H2_HIP(hipEventElapsedTime(&ms, r.e0, r.e1));
    auto& sum = s.sums[r.name];
    sum.launches += 1;
    sum.ms += ms;
    sum.work += r.work + (r.slot >= 0 ? r.work_per_count * s.pinned[r.slot] : 0.0);
    (void)hipEventDestroy(r.e0);
    (void)hipEventDestroy(r.e1);
  }
  s.recs.clear();
  s.used = 0;
}
}  // namespace

bool timing_on() { return st().on; }

int timing_begin(hipStream_t s) {
  State& S = st();
  if (!S.on) return -1;
  std::lock_guard<std::mutex> g(S.mu);
  Rec r{};
  H2_HIP(hipEventCreate(&r.e0));
  H2_HIP(hipEventCreate(&r.e1));
  H2_HIP(hipEventRecord(r.e0, s));
  r.slot = -1;
  S.recs.push_back(r);
  return (int)S.recs.size() - 1;
}

void timing_end(int token, const char* name, hipStream_t s, double work, const int* dev_count,
                double work_per_count) {
  State& S = st();
  if (token < 0 || !S.on) return;
  std::lock_guard<std::mutex> g(S.mu);
  Rec& r = S.recs.at(token);
  H2_HIP(hipEventRecord(r.e1, s));
  r.name = name;
  r.work = work;
  r.work_per_count = work_per_count;
  if (dev_count) {
    if (S.used < S.nslots) {
      r.slot = S.used++;
      H2_HIP(hipMemcpyAsync(S.pinned + r.slot, dev_count, sizeof(int), hipMemcpyDeviceToHost, s));
    } else {
      r.work = std::nan("");  // count slots exhausted before a read: work unknown
    }
  }
}

// plain streaming copy (the reference kernel for scaling HBM byte counters)
__global__ void k_stream_copy(const double* __restrict__ src, double* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

}  // namespace h2

using namespace h2;

extern "C" {

h2_status h2_timing_enable(int on) {
  return h2::guarded_status([&] {
    State& S = st();
    std::lock_guard<std::mutex> g(S.mu);
    if (S.on) drain(S);
    S.sums.clear();
    if (on && !S.pinned) {
      S.nslots = 1 << 16;
      H2_HIP(hipHostMalloc((void**)&S.pinned, S.nslots * sizeof(int), hipHostMallocDefault));
      std::memset(S.pinned, 0, S.nslots * sizeof(int));
    }
    S.on = on != 0;
  });
}

h2_status h2_stream_copy(const double* src, double* dst, int64_t n, hipStream_t stream) {
  return h2::guarded_status([&] {
    H2_CHECK(n >= 0 && (n == 0 || (src && dst)), H2_EINVAL, "bad copy arguments");
    if (n == 0) return;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
    k_stream_copy<<<(unsigned)blocks, 256, 0, stream>>>(src, dst, n);
    H2_LAUNCH_CHECK();
  });
}

h2_status h2_timing_read(const char* kernel, int64_t* launches, double* total_ms, double* work) {
  return h2::guarded_status([&] {
    H2_CHECK(kernel && launches && total_ms && work, H2_EINVAL, "null argument");
    State& S = st();
    std::lock_guard<std::mutex> g(S.mu);
    drain(S);
    auto it = S.sums.find(kernel);
    *launches = it == S.sums.end() ? 0 : it->second.launches;
    *total_ms = it == S.sums.end() ? 0 : it->second.ms;
    *work = it == S.sums.end() ? 0 : it->second.work;
  });
}

}  // extern "C"
