// Host-side plan state shared by the C-ABI and the batched solver.
#pragma once

#include <map>
#include <string>
#include <vector>

#include "hipoisson.h"
#include "hp_internal.hpp"

namespace hp {

// Configuration the autotuner chose for every pass with one signature
// (PassArgs.tune_key): general kernels take the radix order, tile width and
// register budget; wavefront passes the tile width and output-tile scheme.
struct Tune {
  int fast = 0;  // FastKind of the pass (FAST_NONE: general kernel)
  int P = 0, big = 0, emit_dbl = 0;
  int nstage = 0;
  int radix[kMaxStages] = {};
};

struct PassRec {
  PassArgs a;
  int grid_y;
  double bytes = -1.0;  // algorithmic bytes when set by the planner
};

struct Problem {
  hp_desc d{};
  int nd = 0, ncomp = 1, nder = 0;
  int n[3] = {1, 1, 1};     // unknowns
  int nout[3] = {1, 1, 1};  // output points
  int M[3] = {1, 1, 1};     // doubled sizes (unbounded)
  double h[3] = {1, 1, 1}, len[3] = {1, 1, 1};
  // bindings (device pointers); slot c < ncomp for f / psi, derivative d
  const void* in[kMaxFields] = {};
  void* out[3] = {};
  void* der[3] = {};
  const void* face[3][2][3] = {};
  // plan-owned device memory backing unbound slots
  void* own_in[kMaxFields] = {};
  void* own_out[3] = {};
  void* own_der[3] = {};
  void* grad_s = nullptr;  // Dirichlet / Neumann gradient: transformed source
  void* dtmp[3] = {};      // Dirichlet / Neumann DIV / CURL: second derivative terms
  void* own_face[3][2][3] = {};
  std::vector<void*> a1, b2, c2, c1;  // unbounded / periodic workspaces
  double* lam[3] = {};        // eigenvalue tables (bounded)
  void* kvec[3] = {};         // wavenumber tables
  void* green = nullptr;      // Ghat octant
  void* green_odd = nullptr;  // semi-unbounded derivative: odd-kernel rows
  long long g_s[3] = {0, 0, 0};  // octant strides of i0, i1, k2
  double norm = 1.0;
  std::vector<std::pair<int, int>> slabs;  // kz (first, count) of the free-space y / x passes
  bool fast_periodic = false;  // periodic plan on the wavefront passes (M = n)
  int free_axis = -1;          // semi-unbounded plan: the free axis (M[free_axis] = 2 n)
};

}  // namespace hp

namespace hp {
// the event pair recorded around pass `pass` of one solve (hp_set_timing)
struct PassEvents {
  int pass;
  hipEvent_t e0, e1;
};
}  // namespace hp

struct hp_plan_s {
  hipStream_t stream = nullptr;
  int prec = 0;
  size_t es = 4;  // real element size
  bool batched = false;
  bool solved = false;
  std::vector<hp::Problem> probs;
  std::vector<void*> allocs;
  std::map<int, void*> tw;   // L -> W_L table
  std::map<int, void*> qtw;  // n -> exp(-i pi j / 2n)
  std::map<int, void*> ftw;  // L -> per-stage wavefront-FFT twiddles
  std::string err;
  size_t ws_bytes = 0;
  int alloc_count = 0;
  int fail_alloc_at = -1;
  // batched persistent-kernel state
  void* batch_probs = nullptr;
  void* batch_items = nullptr;
  unsigned* batch_counters = nullptr;
  int batch_nitems = 0, batch_ncounters = 0, batch_grid = 0, batch_lds = 0;
  int batch_big = 0;  // register budget of the persistent kernel (PassArgs.big)
  // kernels of the batched solve: 0 = general passes in one persistent launch
  // (k_batched); 1 = wavefront tile bodies in one persistent launch
  // (k_batched_wf, forward type batch_xf); 2 = the wavefront tile bodies as
  // one launch per pass level (k_batched_level).  batch_mode -1 = the
  // planner's choice (1 where every pass allows it, else 0); 0, 1, 2 chosen
  // by the autotuner (1 and 2 fall back to 0 where not allowed)
  int batch_wf = 0, batch_xf = 0, batch_mode = -1;
  std::vector<hp::BatchGroup> batch_groups;  // mode 2: launches (level, length) in order
  // mode 2 under stream capture: the groups of one level run on forked
  // streams (default priority), joined by events before the next level; fork
  // event and join events per level, created at setup
  std::vector<hipStream_t> batch_aux;
  std::vector<hipEvent_t> batch_ev;
  bool batch_fork = true;
  std::vector<hp::PassRec> batch_passes;
  int batch_tiles = 0;  // tiles per work item (0: the default)
  double* zm_partial = nullptr;  // per-block partial sums of the zero-mode query
  // autotuning (hp_autotune): chosen configurations by pass signature, the
  // number of signatures that left the default, and the summed per-pass
  // times of the default and chosen configurations measured while tuning
  std::map<unsigned long long, hp::Tune> tuned;
  int tuned_passes = 0;
  double tune_default_ms = 0.0, tune_best_ms = 0.0;
  std::vector<unsigned char> batch_uploaded;  // pass table last copied to the device
  // per-pass timing
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::vector<hp::PassEvents>> ev_solves;
  int timing_pass = -1;  // -1: every pass; else only this pass index
  size_t ev_used = 0;
  std::vector<double> pass_bytes;
  std::vector<const char*> pass_names;
};

namespace hp {
// implemented in hp_api.cpp
hp_status plan_fail(hp_plan p, hp_status s, const std::string& msg);
hp_status plan_alloc(hp_plan p, size_t bytes, void** out);
void plan_free(hp_plan p, void* ptr);
hp_status launch_rec(hp_plan p, const PassRec& r);
bool radix_ok(int L, const int* radix, int nstage);
hp_status plan_outputs(hp_plan p, Problem& P);
hp_status plan_fast_twiddles(hp_plan p, int L, const void** out);
hp_status passes_for(hp_plan p, Problem& P, bool adjoint, std::vector<PassRec>& out);
double passes_model_bytes(hp_plan p, const std::vector<PassRec>& ps);
// implemented in hp_batched.cpp
hp_status batched_setup(hp_plan p);
hp_status batched_solve(hp_plan p);
int batch_tiles_of(hp_plan p);  // tiles per work item in effect
}  // namespace hp
