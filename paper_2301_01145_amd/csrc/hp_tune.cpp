// Plan-time autotuner (hp_autotune).
//
// Every pass of a plan carries a signature of its geometry (PassArgs.tune_key).
// For each distinct signature the tuner times, on the plan's stream, the
// configurations the kernels are built for:
//   * general kernels: every radix order of the transform length over the
//     radices 2, 3, 4, 5 and 8 (the power-of-two part split into 8s, at most
//     three 4s and at most one 2; each split in descending and ascending
//     order), tile widths of half, one and two times the planner's default,
//     and both register budgets;
//   * wavefront passes: tile widths of 8 and 16 pencils and, for the x and
//     backward-y passes, both output-tile schemes;
//   * batched plans: the persistent kernel's tile bodies (wavefront or general
//     passes) and 1, 2, 4 or 8 tiles per work item.
// A configuration replaces the planner's default only when it is at least 3%
// faster, and the choices are kept only when the whole solve is faster with
// them (batched plans: the combination of pass configurations and work-item
// size is chosen by timing the whole batch).  The tuned plan is then checked against the default on the same
// pseudo-random input: every output must agree to rounding (relative L2
// difference below 1e-5 in FP32 and 1e-12 in FP64), or the tuning is
// discarded and an error returned.  Tuning runs on scratch buffers it
// allocates and frees, so the caller's bound arrays are left untouched.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <random>
#include <set>
#include <string>
#include <vector>

#include "hp_plan.hpp"

#define HP_TRY_T(expr)                  \
  do {                                  \
    const hp_status st_ = (expr);       \
    if (st_ != HP_OK) return st_;       \
  } while (0)

namespace hp {
namespace {

size_t elems(const int* n, int nd) {
  size_t c = 1;
  for (int a = 0; a < nd; ++a) c *= (size_t)n[a];
  return c;
}

// Radix orders of L = 2^a 3^b 5^c that the general kernels run (none for
// lengths with a larger prime factor: those keep the planner's order).
std::vector<std::vector<int>> radix_orders(int L) {
  int a = 0, b = 0, c = 0, r = L;
  while (r % 2 == 0) { r /= 2; ++a; }
  while (r % 3 == 0) { r /= 3; ++b; }
  while (r % 5 == 0) { r /= 5; ++c; }
  std::vector<std::vector<int>> out;
  if (r != 1) return out;
  for (int n8 = a / 3; n8 >= 0; --n8) {
    for (int n4 = 0; n4 <= 3; ++n4) {
      const int n2 = a - 3 * n8 - 2 * n4;
      if (n2 < 0 || n2 > 1) continue;
      std::vector<int> m;
      m.insert(m.end(), n8, 8);
      m.insert(m.end(), n4, 4);
      m.insert(m.end(), n2, 2);
      m.insert(m.end(), b, 3);
      m.insert(m.end(), c, 5);
      if (m.empty() || (int)m.size() > kMaxStages) continue;
      const std::vector<int> asc(m.rbegin(), m.rend());
      for (const auto& o : {m, asc})
        if (std::find(out.begin(), out.end(), o) == out.end()) out.push_back(o);
    }
  }
  return out;
}

struct Tuner {
  hp_plan p;
  int reps;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  std::vector<void*> scratch;

  ~Tuner() {
    (void)hipStreamSynchronize(p->stream);
    for (void* q : scratch) (void)hipFree(q);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }

  hp_status alloc(size_t bytes, void** out) {
    if (hipMalloc(out, bytes ? bytes : 16) != hipSuccess) {
      (void)hipGetLastError();
      *out = nullptr;
      return plan_fail(p, HP_E_NOMEM, "autotune scratch allocation of " + std::to_string(bytes) + " bytes failed");
    }
    scratch.push_back(*out);
    return hipMemset(*out, 0, bytes ? bytes : 16) == hipSuccess
               ? HP_OK
               : plan_fail(p, HP_E_DEVICE, "autotune scratch clear failed");
  }

  // Device array of `n` pseudo-random values in [-1, 1) (plan precision).
  hp_status random_input(size_t n, unsigned seed, void** out) {
    HP_TRY_T(alloc(n * p->es, out));
    std::mt19937_64 g(seed);
    std::uniform_real_distribution<double> u(-1.0, 1.0);
    if (p->prec == 0) {
      std::vector<float> h(n);
      for (auto& v : h) v = (float)u(g);
      if (hipMemcpy(*out, h.data(), n * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        return plan_fail(p, HP_E_DEVICE, "autotune input upload failed");
    } else {
      std::vector<double> h(n);
      for (auto& v : h) v = u(g);
      if (hipMemcpy(*out, h.data(), n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
        return plan_fail(p, HP_E_DEVICE, "autotune input upload failed");
    }
    return HP_OK;
  }

  // Mean milliseconds of `reps` runs of `run` after one warm-up run (best of two
  // such measurements); negative when a launch fails.
  template <class F>
  double time(F run) {
    double best = -1.0;
    if (run() != HP_OK) { (void)hipGetLastError(); return -1.0; }
    for (int m = 0; m < 2; ++m) {
      if (hipEventRecord(e0, p->stream) != hipSuccess) return -1.0;
      for (int i = 0; i < reps; ++i)
        if (run() != HP_OK) { (void)hipGetLastError(); return -1.0; }
      if (hipEventRecord(e1, p->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
        return -1.0;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.0;
      const double t = (double)ms / reps;
      if (best < 0.0 || t < best) best = t;
    }
    return best;
  }

  static bool applied(const PassArgs& a, const Tune& t) {
    if (a.P != t.P) return false;
    if (t.fast != FAST_NONE) return a.fast == t.fast && a.emit_dbl == t.emit_dbl;
    if (a.fast != FAST_NONE || a.big != t.big || a.nstage != t.nstage) return false;
    for (int s = 0; s < t.nstage; ++s)
      if (a.radix[s] != t.radix[s]) return false;
    return true;
  }

  std::vector<Tune> candidates(const PassArgs& a) const {
    std::vector<Tune> c;
    if (a.fast == FAST_NONE) {
      std::vector<int> widths;
      for (int w : {a.P / 2, a.P, a.P * 2})
        if (w >= 1 && std::find(widths.begin(), widths.end(), w) == widths.end()) widths.push_back(w);
      // a batched plan runs every pass in one kernel whose register budget
      // and LDS are the largest of its passes: stay within those
      const int big0 = p->batched ? p->batch_big : 0, big1 = p->batched ? p->batch_big : 1;
      for (const auto& o : radix_orders(a.L))
        for (int w : widths)
          for (int big = big0; big <= big1; ++big) {
            Tune t;
            t.P = w;
            t.big = big;
            t.nstage = (int)o.size();
            for (int s = 0; s < t.nstage; ++s) t.radix[s] = o[s];
            c.push_back(t);
          }
    } else if (a.fast >= FAST_R2C && a.fast <= FAST_INV_Y) {
      const bool two = a.fast == FAST_SANDWICH || a.fast == FAST_INV_Y;
      for (int w : {8, 16}) {
        if (!fast_tile_ok(a.fast, a.L, w, p->prec)) continue;
        for (int dbl = 0; dbl < (two ? 2 : 1); ++dbl) {
          Tune t;
          t.fast = a.fast;
          t.P = w;
          t.emit_dbl = two ? dbl : a.emit_dbl;
          c.push_back(t);
        }
      }
    }
    return c;
  }

  // Tune every pass signature of problem Q's forward pass list.
  hp_status tune_list(Problem& Q, std::set<unsigned long long>& done) {
    std::vector<PassRec> base;
    HP_TRY_T(passes_for(p, Q, false, base));
    for (size_t i = 0; i < base.size(); ++i) {
      const PassArgs& a0 = base[i].a;
      const unsigned long long key = a0.tune_key;
      if (key == 0 || done.count(key)) continue;
      done.insert(key);
      const std::vector<Tune> cands = candidates(a0);
      if (cands.size() < 2) continue;
      const double t_def = time([&] { return launch_rec(p, base[i]); });
      if (t_def < 0.0) return plan_fail(p, HP_E_DEVICE, "autotune: default pass launch failed");
      double best = t_def;
      Tune best_t;
      bool have = false;
      for (const Tune& t : cands) {
        p->tuned[key] = t;
        std::vector<PassRec> ls;
        const hp_status s = passes_for(p, Q, false, ls);
        p->tuned.erase(key);
        if (s != HP_OK) return s;
        if (ls.size() != base.size() || !applied(ls[i].a, t)) continue;
        if (p->batched && ls[i].a.lds_bytes > p->batch_lds) continue;
        const double ms = time([&] { return launch_rec(p, ls[i]); });
        if (ms >= 0.0 && ms < best) {
          best = ms;
          best_t = t;
          have = true;
        }
      }
      if (have && best < 0.97 * t_def) {
        p->tuned[key] = best_t;
        ++p->tuned_passes;
      }
    }
    return HP_OK;
  }

  // Every output of the plan (all problems) copied to the host.
  hp_status outputs(std::vector<std::vector<double>>& out) {
    out.clear();
    if (hipStreamSynchronize(p->stream) != hipSuccess)
      return plan_fail(p, HP_E_DEVICE, "autotune: solve failed");
    for (auto& P : p->probs) {
      const size_t n = elems(P.nout, P.nd);
      std::vector<void*> f;
      for (int c = 0; c < P.ncomp; ++c) f.push_back(P.out[c]);
      for (int c = 0; c < P.nder; ++c) f.push_back(P.der[c]);
      for (void* d : f) {
        std::vector<double> h(n);
        if (p->prec == 0) {
          std::vector<float> t(n);
          if (hipMemcpy(t.data(), d, n * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
            return plan_fail(p, HP_E_DEVICE, "autotune: output copy failed");
          for (size_t i = 0; i < n; ++i) h[i] = t[i];
        } else if (hipMemcpy(h.data(), d, n * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
          return plan_fail(p, HP_E_DEVICE, "autotune: output copy failed");
        }
        out.push_back(std::move(h));
      }
    }
    return HP_OK;
  }

  // One solve of every problem with the current configuration (scratch bindings).
  hp_status solve_all() {
    if (p->batched) return batched_solve(p);
    std::vector<PassRec> ls;
    HP_TRY_T(passes_for(p, p->probs[0], false, ls));
    for (auto& r : ls) HP_TRY_T(launch_rec(p, r));
    return HP_OK;
  }

  hp_status run() {
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
      return plan_fail(p, HP_E_DEVICE, "autotune: event creation failed");
    p->tuned.clear();
    p->tuned_passes = 0;
    p->tune_default_ms = p->tune_best_ms = 0.0;
    p->batch_tiles = 0;
    p->batch_mode = -1;
    // scratch bindings: pseudo-random sources, zeroed outputs; the caller's
    // bindings are restored on every exit path
    struct Saved {
      const void* in[kMaxFields];
      void* out[3];
      void* der[3];
    };
    std::vector<Saved> saved(p->probs.size());
    for (size_t q = 0; q < p->probs.size(); ++q) {
      Problem& P = p->probs[q];
      std::memcpy(saved[q].in, P.in, sizeof(P.in));
      std::memcpy(saved[q].out, P.out, sizeof(P.out));
      std::memcpy(saved[q].der, P.der, sizeof(P.der));
    }
    auto restore = [&] {
      for (size_t q = 0; q < p->probs.size(); ++q) {
        Problem& P = p->probs[q];
        std::memcpy(P.in, saved[q].in, sizeof(P.in));
        std::memcpy(P.out, saved[q].out, sizeof(P.out));
        std::memcpy(P.der, saved[q].der, sizeof(P.der));
      }
    };
    hp_status s = tune_bound();
    restore();
    if (s != HP_OK) {
      p->tuned.clear();
      p->tuned_passes = 0;
      p->batch_tiles = 0;
      p->batch_mode = -1;
      if (p->batched) (void)batched_setup(p);
    }
    return s;
  }

  hp_status tune_bound() {
    for (size_t q = 0; q < p->probs.size(); ++q) {
      Problem& P = p->probs[q];
      const size_t nin = elems(P.n, P.nd), nout = elems(P.nout, P.nd);
      for (int c = 0; c < P.ncomp; ++c) {
        void* d;
        HP_TRY_T(random_input(nin, 0x5eed0000u + 7u * (unsigned)q + (unsigned)c, &d));
        P.in[c] = d;
        HP_TRY_T(alloc(nout * p->es, &P.out[c]));
      }
      for (int c = 0; c < P.nder; ++c) HP_TRY_T(alloc(nout * p->es, &P.der[c]));
    }
    // reference result and solve time with the planner's defaults
    if (p->batched) HP_TRY_T(batched_setup(p));
    HP_TRY_T(solve_all());
    std::vector<std::vector<double>> ref;
    HP_TRY_T(outputs(ref));
    const double t_def = time([&] { return solve_all(); });
    if (t_def < 0.0) return plan_fail(p, HP_E_DEVICE, "autotune: default solve failed");
    p->tune_default_ms = p->tune_best_ms = t_def;
    // per-pass configurations, timed pass by pass
    std::set<unsigned long long> done;
    for (auto& P : p->probs) HP_TRY_T(tune_list(P, done));
    if (p->batched) {
      // whole-batch timing decides between the kernels of the persistent
      // launch (wavefront tile bodies where the batch allows them; the general
      // passes with default or tuned configurations) and its work-item size
      const std::map<unsigned long long, Tune> per_pass = p->tuned;
      const int npass = p->tuned_passes;
      const int def_mode = p->batch_wf;
      double best = t_def;
      int best_tiles = 0, best_use = 0, best_mode = -1;
      for (int mode : {1, 2, 0}) {
        p->batch_mode = mode;
        p->tuned.clear();
        HP_TRY_T(batched_setup(p));
        if (mode != 0 && !p->batch_wf) continue;  // no wavefront form of this batch
        const int uses = (mode != 0 || per_pass.empty()) ? 1 : 2;
        for (int use = 0; use < uses; ++use) {
          p->tuned = use ? per_pass : std::map<unsigned long long, Tune>{};
          for (int tiles : {1, 2, 4, 8}) {
            p->batch_tiles = tiles;
            HP_TRY_T(batched_setup(p));
            const double ms = time([&] { return batched_solve(p); });
            if (ms >= 0.0 && ms < 0.97 * best) {
              best = ms;
              best_tiles = tiles;
              best_use = use;
              best_mode = mode;
            }
          }
        }
      }
      // nothing 3% faster: the planner's default kernel and work-item size
      p->batch_mode = best_mode < 0 ? (def_mode ? -1 : 0) : best_mode;
      p->tuned = best_use ? per_pass : std::map<unsigned long long, Tune>{};
      p->tuned_passes = best_use ? npass : 0;
      p->batch_tiles = best_tiles;
      p->tune_best_ms = best;
      HP_TRY_T(batched_setup(p));
    } else if (!p->tuned.empty()) {
      // keep the per-pass choices only when the whole solve gains as well
      const double ms = time([&] { return solve_all(); });
      if (ms >= 0.0 && ms < 0.97 * t_def) {
        p->tune_best_ms = ms;
      } else {
        p->tuned.clear();
        p->tuned_passes = 0;
      }
    }
    // the tuned plan must reproduce the default result to rounding
    HP_TRY_T(solve_all());
    std::vector<std::vector<double>> got;
    HP_TRY_T(outputs(got));
    const double tol = p->prec == 0 ? 1e-5 : 1e-12;
    for (size_t f = 0; f < ref.size(); ++f) {
      double num = 0.0, den = 0.0;
      bool finite = true;
      for (size_t i = 0; i < ref[f].size(); ++i) {
        const double d = got[f][i] - ref[f][i];
        finite &= std::isfinite(got[f][i]) || !std::isfinite(ref[f][i]);
        num += d * d;
        den += ref[f][i] * ref[f][i];
      }
      const double rel = std::sqrt(num / (den > 0.0 ? den : 1.0));
      if (!finite || !(rel <= tol))
        return plan_fail(p, HP_E_DEVICE,
                         "autotune: tuned configuration disagrees with the default (output " +
                             std::to_string(f) + ", relative L2 difference " + std::to_string(rel) +
                             "); tuning discarded");
    }
    return HP_OK;
  }
};

}  // namespace
}  // namespace hp

extern "C" hp_status hp_autotune(hp_plan plan, int reps) {
  if (!plan) return HP_E_ARG;
  if (reps < 1) reps = 5;
  if (reps > 100) reps = 100;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(plan->stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
    return hp::plan_fail(plan, HP_E_STATE, "autotune during stream capture");
  if (hipStreamSynchronize(plan->stream) != hipSuccess)
    return hp::plan_fail(plan, HP_E_DEVICE, "stream synchronisation failed");
  hp::Tuner t{plan, reps};
  return t.run();
}
