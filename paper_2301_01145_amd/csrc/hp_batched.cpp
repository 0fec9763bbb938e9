// Batched persistent solve: many independent bounded problems of different
// sizes in one launch.  The pass list of every problem is the one of the
// single-problem path (all passes in place in the problem's output array); the
// persistent kernel walks a global item list (one item = one tile of one pass)
// ordered pass level by pass level, with per-pass completion counters as the
// only dependencies between workgroups.
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
  for (int lev = 0; lev < maxlev; ++lev) {
    for (size_t q = 0; q < lists.size(); ++q) {
      if (lev >= (int)lists[q].size()) continue;
      const int gp = first[q] + lev;
      const int dep = lev > 0 ? gp - 1 : -1;
      const int need = lev > 0 ? tiles_of(lists[q][lev - 1].a) : 0;
      // consecutive tiles of a pass share one item (one queue step, one
      // dependency check and one release per item)
      const int nt = tiles_of(lists[q][lev].a);
      for (int t = 0; t < nt; t += per_item)
        items.push_back({gp, t, std::min(per_item, nt - t), dep, need});
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
  const int per_cu = batched_blocks_per_cu(lds, p->prec, big);
  p->batch_grid = std::max(1, std::min(p->batch_nitems, per_cu * cus));
  // keep the pass list (placeholder pointers) for the byte model
  p->batch_passes.clear();
  for (auto& l : lists)
    for (auto& r : l) p->batch_passes.push_back(r);
  return HP_OK;
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
    for (auto& r : l) flat.push_back(r.a);
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
  hipError_t e = launch_batched((const PassArgs*)p->batch_probs, (const BatchItem*)p->batch_items,
                                p->batch_nitems, p->batch_counters, p->batch_ncounters,
                                (int*)(p->batch_counters + p->batch_ncounters), p->batch_grid,
                                p->batch_lds, p->prec, p->batch_big, p->stream);
  if (e != hipSuccess)
    return plan_fail(p, HP_E_DEVICE, std::string("batched launch: ") + hipGetErrorString(e));
  p->solved = true;
  return HP_OK;
}

}  // namespace hp
