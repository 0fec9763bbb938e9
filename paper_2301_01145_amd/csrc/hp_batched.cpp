// Batched persistent solve: many independent bounded problems of different
// sizes in one launch.  The pass list of every problem is the one of the
// single-problem path (all passes in place in the problem's output array); the
// persistent kernel walks a global item list (one item = consecutive tiles of
// one pass) ordered pass level by pass level, with per-pass completion
// counters as the only dependencies between workgroups.  Where every pass of
// every problem has a wavefront FFT (FP32, lengths 64, 96, 128, 192, 256) the
// kernel runs the wavefront tile bodies (k_batched_wf); otherwise the general
// pass code (k_batched).
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "hp_plan.hpp"

namespace hp {

namespace {

// Pass lists of every problem with the current bindings (placeholders for
// unbound slots so that the geometry can be built at plan time).
hp_status build_all(hp_plan p, bool placeholders, std::vector<std::vector<PassRec>>& lists) {
  static char dummy[16];
  lists.clear();
  for (auto& P : p->probs) {
    Problem Q = P;
    if (placeholders) {
      if (!Q.in[0]) Q.in[0] = dummy;
      if (!Q.out[0]) Q.out[0] = dummy;
    }
    std::vector<PassRec> ps;
    hp_status s = passes_for(p, Q, false, ps);
    if (s != HP_OK) return s;
    lists.push_back(std::move(ps));
  }
  return HP_OK;
}

int tiles_of(const PassArgs& a) { return ((a.Np + a.P - 1) / a.P) * a.No; }

// Transform pair of a batch on the wavefront kernels: every pass a
// real-to-real one-way or sandwich pass of the pair (xf, Table 1 partner) with
// a length of batched_wf_length, FP32, no boundary terms.  Returns xf, or 0.
int wf_family(hp_plan p, const std::vector<std::vector<PassRec>>& lists) {
  if (p->prec != 0 || std::getenv("HP_GENERIC")) return 0;
  int xf = 0;
  for (auto& l : lists)
    for (auto& r : l)
      if (r.a.kind == PK_SANDWICH) xf = r.a.xf;
  const int xb = xf == X_DCT2 ? X_DCT3 : (xf == X_DST2 ? X_DST3 : xf);
  if (xf != X_DCT2 && xf != X_DST2 && xf != X_DCT1) return 0;
  for (auto& l : lists)
    for (auto& r : l) {
      const PassArgs& a = r.a;
      if (a.fast != FAST_NONE || !batched_wf_length(a.L) || a.n > a.L / 2 + 1) return 0;
      if (a.kind == PK_SANDWICH ? (a.xf != xf || a.xb != xb) : (a.xf != xf && a.xf != xb)) return 0;
      for (int ax = 0; ax < 3; ++ax)
        if (a.face[ax][0] || a.face[ax][1]) return 0;
    }
  return xf;
}

// The pass on the wavefront tile bodies of k_batched_wf (same descriptor).
hp_status to_wf(hp_plan p, PassArgs& a) {
  const bool contig = a.kind == PK_ONEWAY && a.in_jfast && a.out_jfast;
  a.fast = a.kind == PK_SANDWICH ? FAST_R2R_SW : (contig ? FAST_R2R_C : FAST_R2R_S);
  const void* tw;
  hp_status s = plan_fast_twiddles(p, a.L, &tw);
  if (s != HP_OK) return s;
  a.tw = tw;
  a.P = 32;
  a.lds_bytes = batched_wf_lds(a.fast, a.L);
  return HP_OK;
}

// Kind of a wavefront pass in the level launches (BatchGroup.kind); general
// passes are all kind 0 (they are never launched by level).
int pass_kind(const PassArgs& a, int xf) {
  if (a.fast == FAST_R2R_SW) return 4;
  if (a.fast == FAST_R2R_C) return a.xf == xf ? 0 : 1;
  if (a.fast == FAST_R2R_S) return a.xf == xf ? 2 : 3;
  return 0;
}

// Tiles of a pass in the kernel of the plan's mode.
int mode_tiles(hp_plan p, const PassArgs& a) { return p->batch_wf ? batched_wf_tiles(a) : tiles_of(a); }

int batch_tiles_per_item() {
  if (const char* e = std::getenv("HP_BATCH_TILES")) {
    const int v = std::atoi(e);
    if (v >= 1 && v <= 64) return v;
  }
  return 4;
}
const int kBatchTilesPerItem = batch_tiles_per_item();

}  // namespace

int batch_tiles_of(hp_plan p) { return p->batch_tiles > 0 ? p->batch_tiles : kBatchTilesPerItem; }

hp_status batched_setup(hp_plan p) {
  for (auto& P : p->probs) {
    if (P.d.bc == HP_DIRICHLET && P.d.grid == HP_REGULAR)
      return plan_fail(p, HP_E_UNSUPPORTED, "batched plans take grids without boundary nodes");
    if (P.ncomp != 1) return plan_fail(p, HP_E_UNSUPPORTED, "batched plans take scalar problems");
  }
  std::vector<std::vector<PassRec>> lists;
  hp_status s = build_all(p, true, lists);
  if (s != HP_OK) return s;
  // wavefront tile bodies where every pass allows them (unless the autotuner
  // chose the general passes)
  const int xf = p->batch_mode == 0 ? 0 : wf_family(p, lists);
  // HP_BATCH_LEVELS=1: the level-launch form by default (as the autotuner may choose)
  const char* lv = std::getenv("HP_BATCH_LEVELS");
  const bool levels = p->batch_mode == 2 || (p->batch_mode < 0 && lv && std::atoi(lv) == 1);
  p->batch_wf = xf == 0 ? 0 : (levels ? 2 : 1);
  p->batch_xf = xf;
  if (p->batch_wf) {
    p->tuned.clear();  // per-pass configurations are those of the general kernels
    for (auto& l : lists)
      for (auto& r : l) {
        s = to_wf(p, r.a);
        if (s != HP_OK) return s;
      }
  }
  // items: pass level by pass level, problems in order, tiles in order
  std::vector<int> first(lists.size(), 0);
  int npass = 0, maxlev = 0, lds = 0, big = 0;
  for (size_t q = 0; q < lists.size(); ++q) {
    first[q] = npass;
    npass += (int)lists[q].size();
    maxlev = std::max(maxlev, (int)lists[q].size());
    for (auto& r : lists[q]) {
      lds = std::max(lds, r.a.lds_bytes);
      big = std::max(big, r.a.big);
    }
  }
  p->batch_big = big;
  const int per_item = batch_tiles_of(p);
  std::vector<BatchItem> items;
  p->batch_groups.clear();
  for (int lev = 0; lev < maxlev; ++lev) {
    // within a level, the problems' passes grouped by transform length and
    // kind (the level launches run one kernel instance per group; the
    // persistent kernels take any order within a level)
    std::vector<std::pair<int, int>> keys;
    for (size_t q = 0; q < lists.size(); ++q)
      if (lev < (int)lists[q].size()) keys.push_back({lists[q][lev].a.L, pass_kind(lists[q][lev].a, xf)});
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    for (auto key : keys) {
      BatchGroup grp{(int)items.size(), 0, key.first, key.second, 0, lev};
      for (size_t q = 0; q < lists.size(); ++q) {
        if (lev >= (int)lists[q].size() || lists[q][lev].a.L != key.first ||
            pass_kind(lists[q][lev].a, xf) != key.second)
          continue;
        grp.lds = std::max(grp.lds, lists[q][lev].a.lds_bytes);
        const int gp = first[q] + lev;
        const int dep = lev > 0 ? gp - 1 : -1;
        const int need = lev > 0 ? mode_tiles(p, lists[q][lev - 1].a) : 0;
        // consecutive tiles of a pass share one item (one queue step, one
        // dependency check and one release per item); a wavefront strided item
        // holds one tile per group of wavefronts for every step
        const PassArgs& a = lists[q][lev].a;
        const int nt = mode_tiles(p, a);
        const int step = per_item * (p->batch_wf ? batched_wf_group(a) : 1);
        for (int t = 0; t < nt; t += step)
          items.push_back({gp, t, std::min(step, nt - t), dep, need});
      }
      grp.count = (int)items.size() - grp.first;
      p->batch_groups.push_back(grp);
    }
  }
  p->batch_nitems = (int)items.size();
  p->batch_ncounters = 1 + npass;
  p->batch_lds = lds;
  // a second setup (after autotuning) replaces the tables of the first
  (void)hipStreamSynchronize(p->stream);
  plan_free(p, p->batch_items);
  plan_free(p, p->batch_counters);
  plan_free(p, p->batch_probs);
  p->batch_items = p->batch_probs = nullptr;
  p->batch_counters = nullptr;
  p->batch_uploaded.clear();
  void* d;
  s = plan_alloc(p, items.size() * sizeof(BatchItem), &d);
  if (s != HP_OK) return s;
  p->batch_items = d;
  if (hipMemcpy(d, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice) != hipSuccess)
    return plan_fail(p, HP_E_DEVICE, "upload of the batched work list failed");
  s = plan_alloc(p, (size_t)p->batch_ncounters * sizeof(unsigned) + 64, &d);
  if (s != HP_OK) return s;
  p->batch_counters = (unsigned*)d;
  s = plan_alloc(p, (size_t)npass * sizeof(PassArgs), &d);
  if (s != HP_OK) return s;
  p->batch_probs = d;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return plan_fail(p, HP_E_DEVICE, "device query failed");
  const int per_cu = p->batch_wf ? batched_wf_blocks_per_cu(xf, lds) : batched_blocks_per_cu(lds, p->prec, big);
  p->batch_grid = std::max(1, std::min(p->batch_nitems, per_cu * cus));
  // level form: streams and events for the groups of a level (the most
  // groups in one level - 1 forked streams; a fork and the joins per level)
  if (p->batch_wf == 2) {
    const char* fk = std::getenv("HP_BATCH_FORK");
    p->batch_fork = !(fk && std::atoi(fk) == 0);
    int most = 0;
    for (size_t k = 0; k < p->batch_groups.size();) {
      size_t e = k;
      while (e < p->batch_groups.size() && p->batch_groups[e].level == p->batch_groups[k].level) ++e;
      most = std::max(most, (int)(e - k));
      k = e;
    }
    const size_t nev = (size_t)maxlev * (size_t)std::max(most, 1);
    while ((int)p->batch_aux.size() < most - 1) {
      hipStream_t st;
      if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
        return plan_fail(p, HP_E_DEVICE, "batched: stream creation failed");
      p->batch_aux.push_back(st);
    }
    while (p->batch_ev.size() < nev) {
      hipEvent_t ev;
      if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
        return plan_fail(p, HP_E_DEVICE, "batched: event creation failed");
      p->batch_ev.push_back(ev);
    }
  }
  // keep the pass list (placeholder pointers) for the byte model
  p->batch_passes.clear();
  for (auto& l : lists)
    for (auto& r : l) p->batch_passes.push_back(r);
  return HP_OK;
}

// The level form: one launch per (level, length, kind) group.  The groups of
// one level are independent (each problem has one pass per level).  While the
// plan's stream is being captured, all but the first group of a level run on
// forked streams that wait for the level's start on the plan's stream, and
// the plan's stream waits for all of them before the next level: the fork and
// the joins become graph edges, and the replayed graph runs a level's groups
// concurrently (64 Neumann problems: 0.51 -> 0.44 ms).  Eager solves launch
// the groups in order on the plan's stream, where the event calls of a fork
// cost more than the overlap gains.
hipError_t launch_levels(hp_plan p) {
  const PassArgs* passes = (const PassArgs*)p->batch_probs;
  const BatchItem* items = (const BatchItem*)p->batch_items;
  int* err = (int*)(p->batch_counters + p->batch_ncounters);
  const std::vector<BatchGroup>& gs = p->batch_groups;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  const bool capturing =
      hipStreamIsCapturing(p->stream, &cs) == hipSuccess && cs == hipStreamCaptureStatusActive;
  size_t ev = 0;
  for (size_t k = 0; k < gs.size();) {
    size_t e = k;
    while (e < gs.size() && gs[e].level == gs[k].level) ++e;
    const bool fork = p->batch_fork && capturing && e - k > 1;
    hipError_t r;
    if (fork) {
      const hipEvent_t start = p->batch_ev[ev++];
      if ((r = hipEventRecord(start, p->stream)) != hipSuccess) return r;
      for (size_t g = k + 1; g < e; ++g)
        if ((r = hipStreamWaitEvent(p->batch_aux[g - k - 1], start, 0)) != hipSuccess) return r;
    }
    for (size_t g = k; g < e; ++g) {
      const hipStream_t s = (fork && g > k) ? p->batch_aux[g - k - 1] : p->stream;
      if ((r = launch_batched_group(p->batch_xf, passes, items, gs[g], g == 0 ? err : nullptr, s)) != hipSuccess)
        return r;
    }
    if (fork) {
      for (size_t g = k + 1; g < e; ++g) {
        const hipEvent_t done = p->batch_ev[ev++];
        if ((r = hipEventRecord(done, p->batch_aux[g - k - 1])) != hipSuccess) return r;
        if ((r = hipStreamWaitEvent(p->stream, done, 0)) != hipSuccess) return r;
      }
    }
    k = e;
  }
  return hipSuccess;
}

hp_status batched_solve(hp_plan p) {
  for (size_t q = 0; q < p->probs.size(); ++q) {
    Problem& P = p->probs[q];
    if (!P.in[0]) return plan_fail(p, HP_E_STATE, "input of problem " + std::to_string(q) + " not set");
    if (!P.out[0]) {
      if (!P.own_out[0]) {
        size_t cnt = 1;
        for (int a = 0; a < P.nd; ++a) cnt *= (size_t)P.nout[a];
        hp_status s = plan_alloc(p, cnt * p->es, &P.own_out[0]);
        if (s != HP_OK) return s;
      }
      P.out[0] = P.own_out[0];
    }
  }
  std::vector<std::vector<PassRec>> lists;
  hp_status s = build_all(p, false, lists);
  if (s != HP_OK) return s;
  std::vector<PassArgs> flat;
  for (auto& l : lists)
    for (auto& r : l) {
      if (p->batch_wf) {
        s = to_wf(p, r.a);
        if (s != HP_OK) return s;
      }
      flat.push_back(r.a);
    }
  // the pass table holds the bound pointers: upload when they changed
  const size_t bytes = flat.size() * sizeof(PassArgs);
  std::vector<unsigned char> img(bytes);
  std::memcpy(img.data(), flat.data(), bytes);
  if (p->batch_uploaded != img) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(p->stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
      return plan_fail(p, HP_E_STATE,
                       "bindings changed during stream capture: run one solve before capturing");
    if (hipMemcpyAsync(p->batch_probs, img.data(), bytes, hipMemcpyHostToDevice, p->stream) != hipSuccess ||
        hipStreamSynchronize(p->stream) != hipSuccess)
      return plan_fail(p, HP_E_DEVICE, "upload of the batched pass table failed");
    p->batch_uploaded = img;
  }
  hipError_t e =
      p->batch_wf == 2
          ? launch_levels(p)
      : p->batch_wf
          ? launch_batched_wf(p->batch_xf, (const PassArgs*)p->batch_probs,
                              (const BatchItem*)p->batch_items, p->batch_nitems, p->batch_counters,
                              p->batch_ncounters, (int*)(p->batch_counters + p->batch_ncounters),
                              p->batch_grid, p->batch_lds, p->stream)
          : launch_batched((const PassArgs*)p->batch_probs, (const BatchItem*)p->batch_items,
                           p->batch_nitems, p->batch_counters, p->batch_ncounters,
                           (int*)(p->batch_counters + p->batch_ncounters), p->batch_grid,
                           p->batch_lds, p->prec, p->batch_big, p->stream);
  if (e != hipSuccess)
    return plan_fail(p, HP_E_DEVICE, std::string("batched launch: ") + hipGetErrorString(e));
  p->solved = true;
  return HP_OK;
}

}  // namespace hp
