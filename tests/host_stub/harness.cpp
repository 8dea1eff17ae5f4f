// Host lifetime harness for the library's C ABI.
//
// The host layer (ihdg_api.cpp) is built with the host compiler under
// AddressSanitizer and UBSan against a CPU stand-in of the HIP runtime
// (hip_stub.cpp) that defers every asynchronous copy until its stream is
// synchronised and can make any runtime call or launch fail.  Each scenario
// drives one entry point (setup, the solve drivers, the batch) and is repeated
// with a failure injected at its 1st, 2nd, ... call.  After each run the
// deferred operations are completed (stub_drain), as a DMA engine would
// complete them after the caller had moved on, and only then are the caller's
// buffers released.  A host staging buffer that the library gives up while a
// copy into or out of it is still queued then shows up as an ASan
// use-after-free or stack-use-after-return.  Several threads run the
// scenarios at once on separate contexts and streams.
//
// Usage: harness [threads]   (exit status 0: every run returned a status
// and no sanitizer fired; ASan aborts the process otherwise)
//        harness tune        (the autotuner's buffer use, below)
#include <algorithm>
#include <atomic>
#include <functional>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ihdg.h"
#include "stub_control.hpp"

namespace {

struct DevMem {  // "device" buffers of one run, released after the drain
  std::vector<void*> bufs;
  void* get(size_t n) {
    n = (n + 255) & ~(size_t)255;
    void* p = std::aligned_alloc(256, n ? n : 256);
    std::memset(p, 0, n ? n : 256);
    bufs.push_back(p);
    return p;
  }
  ~DevMem() {
    for (void* p : bufs) std::free(p);
  }
};

struct Problem {
  ihdg_mesh mesh;
  int order;
  ihdg_pde pde;
  ihdg_coeffs cf;
  ihdg_options opt;
};

Problem make(int pde, bool per_element, int prec, int krylov, int kmethod, bool graph, bool tstep) {
  Problem p{};
  p.mesh.dim = 2;
  p.mesh.n[0] = p.mesh.n[1] = 9;  // two 64-element blocks, the second ragged
  p.mesh.n[2] = 1;
  p.mesh.hi[0] = p.mesh.hi[1] = p.mesh.hi[2] = 1.0;
  p.order = 2;
  p.pde = (ihdg_pde)pde;
  static double dummy[64];  // never read by the stand-in launchers
  if (per_element) p.cf.beta_q = dummy;
  p.cf.beta_const[0] = 1.0;
  p.cf.beta_const[1] = 0.5;
  p.cf.sigma_const = 1.0;
  p.cf.kappa = 1e-2;
  p.cf.nu = 1.0;
  p.cf.Phi = 1.0;
  p.cf.mass_coef = 20.0;
  p.opt.prec = (ihdg_precision)prec;
  p.opt.check_every = 4;
  p.opt.max_iters = 64;
  p.opt.krylov_restart = krylov;
  p.opt.krylov_method = kmethod;
  p.opt.use_graph = graph ? 1 : 0;
  p.opt.block_waves = 0;  // the autotuner runs too
  p.opt.time_stepping = tstep ? 1 : 0;
  return p;
}

// One context through setup and `work`; returns false if a call returned a
// value that is not a status.
template <typename F>
bool run_ctx(const Problem& pr, hipStream_t st, DevMem& dm, ihdg_ctx** out, F work) {
  size_t pb = 0, sb = 0;
  if (ihdg_footprint(&pr.mesh, pr.order, pr.pde, &pr.cf, &pr.opt, &pb, &sb) != IHDG_OK) return false;
  void* ws = dm.get(pb);
  void* sc = dm.get(sb);
  ihdg_ctx* c = nullptr;
  ihdg_status s = ihdg_setup(&pr.mesh, pr.order, pr.pde, &pr.cf, &pr.opt, ws, pb, sc, sb, st, &c);
  if (s != IHDG_OK) {
    if (c) return false;  // no context on failure
    *out = nullptr;
    return s >= 0 && s <= IHDG_ERR_MAXITER;
  }
  *out = c;
  return work(c);
}

bool solve_once(ihdg_ctx* c) {
  int32_t it = 0;
  double inc = 0, dfc = 0;
  ihdg_status s = ihdg_solve(c, 1e-8, &it, &inc, &dfc);
  return s >= 0 && s <= IHDG_ERR_MAXITER;
}

struct Scenario {
  const char* name;
  std::function<bool(hipStream_t, DevMem&, std::vector<ihdg_ctx*>&, hipStream_t)> run;
};

std::vector<Scenario> scenarios() {
  std::vector<Scenario> v;
  auto single = [](Problem pr, bool extra) {
    return [pr, extra](hipStream_t st, DevMem& dm, std::vector<ihdg_ctx*>& ctxs, hipStream_t) {
      ihdg_ctx* c = nullptr;
      bool ok = run_ctx(pr, st, dm, &c, [&](ihdg_ctx* cc) {
        bool r = solve_once(cc);
        if (extra) {
          double nrm[2];
          ihdg_status s = ihdg_sweep(cc, 3, nrm);
          r = r && s >= 0 && s <= IHDG_ERR_MAXITER;
          s = ihdg_residual(cc, nrm);
          r = r && s >= 0 && s <= IHDG_ERR_MAXITER;
          if (pr.opt.time_stepping) {
            s = ihdg_time_step(cc, 1);
            r = r && s >= 0 && s <= IHDG_ERR_MAXITER;
            r = r && solve_once(cc);
          }
        }
        return r;
      });
      if (c) ctxs.push_back(c);
      return ok;
    };
  };
  v.push_back({"transport per-element fp64", single(make(0, true, 0, 0, 0, false, false), true)});
  v.push_back({"transport per-element mixed", single(make(0, true, 1, 0, 0, false, false), false)});
  v.push_back({"transport shared fp64 graphs", single(make(0, false, 0, 0, 0, true, false), true)});
  v.push_back({"shallow water time steps", single(make(1, false, 0, 0, 0, true, true), true)});
  v.push_back({"conv.-diff. gmres fp64", single(make(2, true, 0, 8, 0, false, false), false)});
  v.push_back({"conv.-diff. gmres mixed", single(make(2, true, 1, 8, 0, false, false), false)});
  v.push_back({"conv.-diff. bicgstab", single(make(2, true, 0, 8, 1, false, false), false)});
  auto batch = [](bool graphs) {
    return [graphs](hipStream_t st, DevMem& dm, std::vector<ihdg_ctx*>& ctxs, hipStream_t bst) {
      const Problem prs[3] = {make(0, true, 0, 0, 0, false, false), make(0, true, 1, 0, 0, false, false),
                              make(1, false, 1, 0, 0, false, false)};
      size_t bb = 0;
      if (ihdg_batch_footprint(8, 64, &bb) != IHDG_OK) return false;
      void* bws = dm.get(bb);
      ihdg_batch* b = nullptr;
      ihdg_status s = ihdg_batch_create(8, 64, bws, bb, bst, &b);
      if (s != IHDG_OK) return s >= 0 && s <= IHDG_ERR_MAXITER && !b;
      ihdg_batch_use_graphs(b, graphs ? 1 : 0);
      bool ok = true;
      for (int i = 0; i < 3; ++i) {
        ihdg_ctx* c = nullptr;
        ok = ok && run_ctx(prs[i], st, dm, &c, [&](ihdg_ctx* cc) {
          ihdg_status r = ihdg_batch_add(b, cc, 1e-8, i);
          return r >= 0 && r <= IHDG_ERR_MAXITER;
        });
        if (c) ctxs.push_back(c);
      }
      for (int round = 0; round < 12 && ok; ++round) {
        int32_t n = 0;
        s = ihdg_batch_round(b, 4, &n);
        ok = s >= 0 && s <= IHDG_ERR_MAXITER;
        if (s != IHDG_OK || n == 0) break;
      }
      ihdg_batch_result res[8];
      int32_t nout = 0;
      s = ihdg_batch_poll(b, res, 8, &nout);
      ok = ok && s == IHDG_OK;
      ihdg_batch_destroy(b);
      return ok;
    };
  };
  v.push_back({"batch, direct launches", batch(false)});
  v.push_back({"batch, graph replay", batch(true)});
  return v;
}

std::atomic<long> g_runs{0}, g_bad{0};

void worker(int tid) {
  hipStream_t st = (hipStream_t)(uintptr_t)(0x1000 + 16 * tid);
  hipStream_t bst = (hipStream_t)(uintptr_t)(0x1008 + 16 * tid);
  for (const Scenario& sc : scenarios()) {
    // calls of a clean run bound the failure positions to try
    long n_clean = 0;
    {
      DevMem dm;
      std::vector<ihdg_ctx*> ctxs;
      stub_set_fail_at(-1);
      if (!sc.run(st, dm, ctxs, bst)) {
        std::fprintf(stderr, "[t%d] %s: clean run returned a non-status\n", tid, sc.name);
        ++g_bad;
      }
      n_clean = stub_calls();
      stub_drain(st);
      stub_drain(bst);
      for (ihdg_ctx* c : ctxs) ihdg_destroy(c);
    }
    for (long k = 1; k <= n_clean; ++k) {
      DevMem dm;
      std::vector<ihdg_ctx*> ctxs;
      stub_set_fail_at(k);
      const bool ok = sc.run(st, dm, ctxs, bst);
      stub_set_fail_at(-1);
      // the caller has its statuses; whatever is still queued completes now
      stub_drain(st);
      stub_drain(bst);
      for (ihdg_ctx* c : ctxs) ihdg_destroy(c);
      stub_drain(st);
      stub_drain(bst);
      ++g_runs;
      if (!ok) {
        std::fprintf(stderr, "[t%d] %s: failure at call %ld gave a non-status\n", tid, sc.name, k);
        ++g_bad;
      }
    }
    std::printf("[t%d] %s: %ld calls, every failure position tried\n", tid, sc.name, n_clean);
    std::fflush(stdout);
  }
}

// The autotuner at setup times its candidate launches on two scratch
// iterates per precision: each launch reads one and writes the other, both
// are zeroed after the last one, and neither is the iterate a solve starts
// from.
int tune_check() {
  hipStream_t st = (hipStream_t)(uintptr_t)0x2000;
  DevMem dm;
  stub_set_fail_at(-1);
  ihdg_ctx* c = nullptr;
  stub_record(true);
  const bool ok = run_ctx(make(0, false, 1, 0, 0, false, false), st, dm, &c, [](ihdg_ctx*) { return true; });
  const std::vector<StubRec> tune = stub_records();
  if (!ok || !c) {
    std::printf("tune: setup failed\n");
    return 1;
  }
  stub_record(true);
  ihdg_status s = ihdg_sweep(c, 1, nullptr);
  const std::vector<StubRec> first = stub_records();
  stub_record(false);
  stub_drain(st);
  int bad = 0;
  if (s != IHDG_OK || first.empty() || first[0].kind != 0) {
    std::printf("tune: no sweep recorded after setup\n");
    bad = 1;
  }
  for (int fp32 = 0; fp32 < 2 && !bad; ++fp32) {
    std::vector<const void*> bufs;
    size_t last = 0, n = 0;
    for (size_t i = 0; i < tune.size(); ++i) {
      const StubRec& r = tune[i];
      if (r.kind != 0 || r.fp32 != (fp32 == 1)) continue;
      ++n;
      last = i;
      for (const void* b : {r.in, r.out})
        if (std::find(bufs.begin(), bufs.end(), b) == bufs.end()) bufs.push_back(b);
      if (r.in == r.out) bad = 1;
    }
    bool zeroed[2] = {false, false};
    for (size_t i = last + 1; i < tune.size() && bufs.size() == 2; ++i)
      for (int k = 0; k < 2; ++k)
        if (tune[i].kind == 1 && tune[i].out == bufs[k]) zeroed[k] = true;
    const bool cur_untouched = fp32 || std::find(bufs.begin(), bufs.end(), first[0].in) == bufs.end();
    std::printf("tune: %s %zu launches on %zu buffers, zeroed %d %d, current iterate untouched %d\n",
                fp32 ? "fp32" : "fp64", n, bufs.size(), (int)zeroed[0], (int)zeroed[1], (int)cur_untouched);
    if (n < 4 || bufs.size() != 2 || !zeroed[0] || !zeroed[1] || !cur_untouched) bad = 1;
  }
  ihdg_destroy(c);
  std::printf(bad ? "tune: FAILED\n" : "tune ok\n");
  return bad;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc > 1 && std::strcmp(argv[1], "tune") == 0) return tune_check();
  const int nt = argc > 1 ? std::atoi(argv[1]) : 4;
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t) th.emplace_back(worker, t);
  for (auto& t : th) t.join();
  std::printf("runs %ld, bad %ld\n", g_runs.load(), g_bad.load());
  return g_bad.load() ? 1 : 0;
}
