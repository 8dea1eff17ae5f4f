// CPU stand-in for the HIP runtime and for the library's device launchers,
// for the host lifetime harness (see hip/hip_runtime.h for the semantics).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <mutex>
#include <vector>

#include "../../paper_1605_03228_amd/csrc/internal.hpp"
#include "stub_control.hpp"

namespace {

typedef std::function<void()> Op;

struct StreamState {
  std::deque<Op> queue;
  bool capturing = false;
  std::vector<Op> captured;
};

std::mutex g_mu;                          // guards every stream's state
std::map<hipStream_t, StreamState> g_st;  // keyed by handle (nullptr = default stream)
thread_local long t_calls = 0;
thread_local long t_fail_at = -1;
thread_local long t_failed_at = -1;       // call index of the injected failure, -1 = none yet
thread_local hipError_t t_last = hipSuccess;
double g_decay = 1.0;                     // norms written by the stubs fall geometrically

bool inject() {
  ++t_calls;
  if (t_calls == t_fail_at) {
    t_failed_at = t_calls;
    return true;
  }
  return false;
}

hipError_t fail_with(hipError_t e) {
  t_last = e;
  return e;
}

// queue an operation (or record it while the stream is being captured)
hipError_t enqueue(hipStream_t s, Op op, hipError_t err = hipErrorLaunchFailure) {
  if (inject()) return fail_with(err);
  std::lock_guard<std::mutex> g(g_mu);
  StreamState& st = g_st[s];
  if (st.capturing) st.captured.push_back(std::move(op));
  else st.queue.push_back(std::move(op));
  return hipSuccess;
}

void run_queue(hipStream_t s) {
  std::deque<Op> q;
  {
    std::lock_guard<std::mutex> g(g_mu);
    q.swap(g_st[s].queue);
  }
  for (Op& op : q) op();
}

double next_norm() {
  std::lock_guard<std::mutex> g(g_mu);
  g_decay *= 0.5;
  if (g_decay < 1e-30) g_decay = 1.0;
  return g_decay;
}

thread_local bool g_rec = false;
thread_local std::vector<StubRec> g_recs;

void rec(int kind, bool fp32, const void* in, const void* out) {
  if (g_rec) g_recs.push_back({kind, fp32, in, out});
}

}  // namespace

void stub_record(bool on) {
  g_rec = on;
  if (on) g_recs.clear();
}
std::vector<StubRec> stub_records() { return g_recs; }

struct ihipEvent_t {
  hipStream_t s;
};
struct ihipGraph {
  std::vector<Op> ops;
};
struct hipGraphExec {
  std::vector<Op> ops;
};

// ---- harness controls ----
void stub_set_fail_at(long n) {
  t_calls = 0;
  t_fail_at = n;
  t_failed_at = -1;
}
long stub_calls() { return t_calls; }
long stub_failed_at() { return t_failed_at; }
void stub_drain(hipStream_t s) { run_queue(s); }
size_t stub_pending(hipStream_t s) {
  std::lock_guard<std::mutex> g(g_mu);
  return g_st[s].queue.size();
}

// ---- runtime ----
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t s) {
  return enqueue(s, [=] { std::memcpy(dst, src, bytes); }, hipErrorInvalidValue);
}
hipError_t hipMemsetAsync(void* dst, int v, size_t bytes, hipStream_t s) {
  return enqueue(s, [=] { std::memset(dst, v, bytes); }, hipErrorInvalidValue);
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  if (inject()) return fail_with(hipErrorUnknown);  // the queue stays pending
  {
    std::lock_guard<std::mutex> g(g_mu);
    if (g_st[s].capturing) return fail_with(hipErrorStreamCaptureInvalidated);
  }
  run_queue(s);
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) {
  if (inject()) return fail_with(hipErrorUnknown);
  *e = new ihipEvent_t{nullptr};
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  if (inject()) return fail_with(hipErrorUnknown);
  e->s = s;
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) { return hipStreamSynchronize(e->s); }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  if (inject()) return fail_with(hipErrorUnknown);
  *ms = 1.0f;
  return hipSuccess;
}
hipError_t hipGetLastError() {
  hipError_t e = t_last;
  t_last = hipSuccess;
  return e;
}
const char* hipGetErrorString(hipError_t) { return "stub error"; }
const char* hipGetErrorName(hipError_t) { return "hipErrorStub"; }
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  if (inject()) return fail_with(hipErrorUnknown);
  std::lock_guard<std::mutex> g(g_mu);
  g_st[s].capturing = true;
  g_st[s].captured.clear();
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* out) {
  std::vector<Op> ops;
  {
    std::lock_guard<std::mutex> g(g_mu);
    ops.swap(g_st[s].captured);
    g_st[s].capturing = false;
  }
  if (inject()) return fail_with(hipErrorStreamCaptureInvalidated);
  *out = new ihipGraph{std::move(ops)};
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* exec, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  if (inject()) return fail_with(hipErrorUnknown);
  *exec = new hipGraphExec{g->ops};
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  delete g;
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t g) {
  delete g;
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t g, hipStream_t s) {
  std::vector<Op> ops = g->ops;
  return enqueue(s, [ops] {
    for (const Op& op : ops) op();
  });
}

// ---- the library's device launchers: queued no-ops, except the ones whose
// outputs the host reads back (norms, dot products, flags) ----
namespace ihdg {

static hipError_t nop(hipStream_t s) {
  return enqueue(s, [] {});
}
static hipError_t fill(double* out, int n, hipStream_t s) {
  if (!out) return nop(s);
  return enqueue(s, [=] {
    const double v = next_norm();
    for (int i = 0; i < n; ++i) out[i] = v;
  });
}

hipError_t launch_setup(const SetupArgs&, hipStream_t s) { return nop(s); }
size_t cd_consts_doubles(int np, int n_in) { return (size_t)7 * np * np + (size_t)3 * np * n_in; }
hipError_t launch_cd_consts(const SetupArgs&, hipStream_t s) { return nop(s); }
hipError_t launch_shared_c(const SetupArgs&, hipStream_t s) { return nop(s); }
hipError_t launch_maps(const SetupArgs&, int*, hipStream_t s) { return nop(s); }
hipError_t launch_time_operator(const SetupArgs&, double*, hipStream_t s) { return nop(s); }
hipError_t launch_time_rhs(double*, const double*, const double*, const double*, const double*, int, int64_t,
                           double, double, double, hipStream_t s) {
  return nop(s);
}
hipError_t launch_node_points(const MeshInfo&, const RefTab&, double*, hipStream_t s) { return nop(s); }
hipError_t launch_quad_points(const MeshInfo&, const RefTab&, double*, double*, hipStream_t s) { return nop(s); }
hipError_t launch_sweep_transport(int, int, bool fp32, bool, int, const SweepArgs& a, hipStream_t s) {
  rec(0, fp32, a.uin, a.uout);
  return nop(s);
}
hipError_t launch_sweep_sw(int, bool fp32, bool, int, const SweepArgs& a, hipStream_t s) {
  rec(0, fp32, a.uin, a.uout);
  return nop(s);
}
hipError_t launch_sweep_cd(int, bool fp32, bool, int, const SweepArgs& a, hipStream_t s) {
  rec(0, fp32, a.uin, a.uout);
  return nop(s);
}
bool direct_supported(int, int) { return true; }
bool gemm_supported(int, int) { return true; }
bool own_supported(int, int) { return true; }
hipError_t launch_own(int, int, bool, const SweepArgs&, hipStream_t s) { return nop(s); }
hipError_t launch_own_batched(int, int, bool, const BatchDesc*, const int*, int64_t, int, hipStream_t s) {
  return nop(s);
}
hipError_t noalloc_scratch(hipStream_t, void** out) {
  static void* buf = std::malloc(kNoAllocScratchBytes);
  if (inject()) return fail_with(hipErrorUnknown);
  *out = buf;
  return hipSuccess;
}
bool direct_cd_supported(int) { return true; }
hipError_t launch_sweep_batched_transport(int, int, bool, bool, int, const BatchDesc*, const int*, int64_t, int,
                                          hipStream_t s) {
  return nop(s);
}
hipError_t launch_sweep_batched_sw(int, bool, bool, int, const BatchDesc*, const int*, int64_t, int, hipStream_t s) {
  return nop(s);
}
hipError_t launch_sweep_batched_cd(int, bool, bool, int, const BatchDesc*, const int*, int64_t, int, hipStream_t s) {
  return nop(s);
}
hipError_t launch_reduce_partials(const double*, int64_t, double* out2, hipStream_t s) {
  return enqueue(s, [=] {
    out2[0] = next_norm();
    out2[1] = 1.0;
  });
}
hipError_t launch_diff_to_f32(const double*, const double*, float*, int64_t, hipStream_t s) { return nop(s); }
hipError_t launch_add_f32_to_f64(double*, const float*, int64_t, hipStream_t s) { return nop(s); }
hipError_t launch_fill_zero_f32(float* p, int64_t, hipStream_t s) {
  rec(1, true, nullptr, p);
  return nop(s);
}
hipError_t launch_fill_zero_f64(double* p, int64_t, hipStream_t s) {
  rec(1, false, nullptr, p);
  return nop(s);
}
hipError_t launch_to_user(const double*, double*, int64_t, int, hipStream_t s) { return nop(s); }
hipError_t launch_from_user(const double*, double*, int64_t, int, hipStream_t s) { return nop(s); }
hipError_t launch_axpby(double*, double, const double*, double, int64_t, hipStream_t s) { return nop(s); }
hipError_t launch_multi_axpy(double*, const double*, const double*, int, int64_t, hipStream_t s) { return nop(s); }
hipError_t launch_multi_axpy(float*, const float*, const double*, int, int64_t, hipStream_t s) { return nop(s); }
hipError_t launch_multi_axpy(double*, const float*, const double*, int, int64_t, hipStream_t s) { return nop(s); }
hipError_t launch_reduce_batched(const BatchDesc*, int n, double* norms, hipStream_t s) {
  return enqueue(s, [=] {
    const double v = next_norm();
    for (int i = 0; i < n; ++i) {
      norms[2 * i] = v;
      norms[2 * i + 1] = 1.0;
    }
  });
}
int kdot_groups(int64_t) { return 4; }
hipError_t launch_kdots(const double*, const double*, int64_t, int k, const double*, int, double*, double* out,
                        double* acc, int, hipStream_t s) {
  return enqueue(s, [=] {
    const double v = next_norm();
    for (int j = 0; j < k; ++j) {
      if (out) out[j] = v;
      if (acc) acc[j] = v;
    }
  });
}
hipError_t launch_kdots(const float*, const float*, int64_t, int k, const double*, int, double*, double* out,
                        double* acc, int, hipStream_t s) {
  return enqueue(s, [=] {
    const double v = next_norm();
    for (int j = 0; j < k; ++j) {
      if (out) out[j] = v;
      if (acc) acc[j] = v;
    }
  });
}
hipError_t launch_knormalize(double*, int64_t, const double*, double* hn, hipStream_t s) { return fill(hn, 1, s); }
hipError_t launch_knormalize(float*, int64_t, const double*, double* hn, hipStream_t s) { return fill(hn, 1, s); }
hipError_t launch_kapply(double*, const double*, const double*, int64_t, hipStream_t s) { return nop(s); }
hipError_t launch_kapply_linear(float*, const float*, int64_t, hipStream_t s) { return nop(s); }
hipError_t launch_scale_to_f32(float*, const double*, double, int64_t, hipStream_t s) { return nop(s); }
hipError_t launch_bicg_p(double*, const double*, const double*, double*, const double*, int, int, int64_t,
                         hipStream_t s) {
  return nop(s);
}
hipError_t launch_bicg_s(double*, const double*, const double*, double*, const double*, int, int64_t, hipStream_t s) {
  return nop(s);
}
hipError_t launch_bicg_apply_dot1(double*, const double*, const double*, const double*, const double*, int, int64_t,
                                  double*, hipStream_t s) {
  return nop(s);
}
hipError_t launch_bicg_apply_dot2(double*, const double*, const double*, const double*, int, int64_t, double*,
                                  hipStream_t s) {
  return nop(s);
}
hipError_t launch_bicg_xr_dot(double*, double*, const double*, const double*, const double*, const double*, double*,
                              const double*, int, int64_t, const double*, double*, hipStream_t s) {
  return nop(s);
}
hipError_t launch_kdots_final(const double*, int64_t, int k, double* out, hipStream_t s) { return fill(out, k, s); }

}  // namespace ihdg
