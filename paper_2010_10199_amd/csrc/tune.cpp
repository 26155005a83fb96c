// Measured launch choices of a plan, and the plan's own graphs of a transform's launches.
//
// Several launch forms compute the same transform (they differ in rounding order only): the
// forward gather of each order (GT_GATHER_SORTED / CELL / POLY), the resident wavefronts per
// compute unit of the order-2 tile spread, whether order 1 runs on the plan's second stream,
// and whether gt_plan_trafo / gt_plan_adjoint replay a captured graph instead of launching
// eagerly.  gt_plan_tune times the candidates on the plan's own nodes with HIP events and keeps
// the fastest; the choice is cached per device and problem signature, so that later plans of
// the same signature (other node draws of one workload) start from it without timing.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "gt_internal.h"

namespace gt {
namespace {

struct TuneKey {
  int dev;
  int32_t d, ds, R, dtype, basis, ragged, nterms;
  int32_t N[kMaxOrder + 1], m[kMaxOrder + 1], n[kMaxOrder + 1];
  int64_t Mtot;
  uint64_t terms_hash;
  bool operator==(const TuneKey &o) const { return memcmp(this, &o, sizeof(TuneKey)) == 0; }
};

struct TuneChoice {
  int32_t path[kMaxOrder + 1];
  int32_t adj[kMaxOrder + 1];
  int32_t waves_cu;
  bool use_side, use_graph, use_fused;
  std::string report;
};

std::mutex g_tune_mu;
std::vector<std::pair<TuneKey, TuneChoice>> g_tune;

TuneKey key_of(const gt_plan *pl) {
  TuneKey k;
  memset(&k, 0, sizeof(k));   // padding bytes take part in the comparison
  (void)hipGetDevice(&k.dev);
  k.d = pl->d;
  k.ds = pl->ds;
  k.R = pl->R;
  k.dtype = pl->dtype;
  k.basis = pl->basis;
  k.ragged = pl->ragged ? 1 : 0;
  k.nterms = pl->nterms;
  for (int t = 1; t <= pl->ds; ++t) {
    k.N[t] = pl->ord[t].N;
    k.m[t] = pl->ord[t].m;
    k.n[t] = pl->ord[t].n;
  }
  k.Mtot = pl->Mtot;
  uint64_t h = 1469598103934665603ull;   // FNV-1a over the terms' coordinate lists
  for (const DevTerm &dt : pl->terms) {
    const int32_t v[4] = {dt.t, dt.c0, dt.c1, dt.c2};
    for (int i = 0; i < 4; ++i) {
      h ^= (uint64_t)(uint32_t)v[i];
      h *= 1099511628211ull;
    }
  }
  k.terms_hash = h;
  return k;
}

const char *path_name(int p) {
  return p == GT_GATHER_DIRECT ? "direct" : p == GT_GATHER_POLY ? "poly" : p == GT_GATHER_CELL ? "cell" : "sorted";
}

int eager(gt_plan *pl, int dir, const void *in, void *out, hipStream_t s) {
  if (pl->dtype == GT_C64)
    return dir == 0 ? launch_forward<float>(pl, in, nullptr, out, s) : launch_adjoint<float>(pl, in, nullptr, out, s);
  return dir == 0 ? launch_forward<double>(pl, in, nullptr, out, s) : launch_adjoint<double>(pl, in, nullptr, out, s);
}

// Buffers of the timing runs (contents irrelevant to the timing; cleared once).
struct TuneBufs {
  void *fhat = nullptr, *f = nullptr;
  ~TuneBufs() {
    dev_free(fhat, nullptr);
    dev_free(f, nullptr);
  }
};

// Mean milliseconds per call of `dirs` (bit 0 forward, bit 1 adjoint): one timed call; when
// it took less than 20 ms (a first call may include loading code), one more untimed call and
// then enough timed calls for about 20 ms of work (2 to 50).
int time_calls(gt_plan *pl, int dirs, const TuneBufs &b, hipStream_t s, hipEvent_t e0, hipEvent_t e1, double *ms) {
  auto one = [&]() -> int {
    if (dirs & 1)
      if (int rc = run_plan_call(pl, 0, b.fhat, b.f, s)) return rc;
    if (dirs & 2)
      if (int rc = run_plan_call(pl, 1, b.f, b.fhat, s)) return rc;
    return GT_OK;
  };
  GT_HIP(hipEventRecord(e0, s));
  if (int rc = one()) return rc;
  GT_HIP(hipEventRecord(e1, s));
  GT_HIP(hipEventSynchronize(e1));
  float t1 = 0;
  GT_HIP(hipEventElapsedTime(&t1, e0, e1));
  if (t1 >= 20.0f) {
    *ms = (double)t1;
    return GT_OK;
  }
  if (int rc = one()) return rc;
  const int reps = std::max(2, std::min(50, (int)(20.0 / std::max(1e-3, (double)t1))));
  GT_HIP(hipEventRecord(e0, s));
  for (int i = 0; i < reps; ++i)
    if (int rc = one()) return rc;
  GT_HIP(hipEventRecord(e1, s));
  GT_HIP(hipEventSynchronize(e1));
  float tr = 0;
  GT_HIP(hipEventElapsedTime(&tr, e0, e1));
  *ms = (double)tr / reps;
  return GT_OK;
}

// Milliseconds per call of the kernels of order t in direction dir (0 forward, 1 adjoint):
// the calls launch eagerly on one stream with an event pair per launch, and the launches whose
// names end in "_<t>d" are summed (pack, gather or direct sums; spread, fold, adjoint DFT or
// direct sums).  One call; when the order took less than 5 ms, one untimed call (left out when
// the whole call took over 100 ms) and then enough calls for about 20 ms of the order's work
// (2 to 20), but no more than about 200 ms of whole calls: every call runs all orders, and on
// large plans a fast order's repetitions would otherwise cost seconds of the other orders' work.
int time_order(gt_plan *pl, int dir, int t, const TuneBufs &b, hipStream_t s, double *ms) {
  char suffix[8];
  snprintf(suffix, sizeof(suffix), "_%dd", t);
  const bool was = prof_set(true);
  auto calls = [&](int n, double *out) -> int {
    const size_t mark = prof_mark();
    for (int i = 0; i < n; ++i) {
      const int rc = dir == 0 ? run_plan_call(pl, 0, b.fhat, b.f, s) : run_plan_call(pl, 1, b.f, b.fhat, s);
      if (rc != GT_OK) {
        (void)prof_take_since(mark, suffix);
        return rc;
      }
    }
    *out = prof_take_since(mark, suffix) / n;
    return GT_OK;
  };
  double t1 = 0;
  const auto w0 = std::chrono::steady_clock::now();
  int rc = calls(1, &t1);
  const double wall = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - w0).count();
  if (rc == GT_OK && t1 < 5.0) {
    double warm = 0;
    if (wall <= 100.0) rc = calls(1, &warm);
    const int reps = std::min(std::min(20, (int)(20.0 / std::max(1e-3, t1))), (int)(200.0 / std::max(1e-3, wall)));
    if (rc == GT_OK) rc = calls(std::max(2, reps), &t1);
  }
  prof_set(was);
  *ms = t1;
  return rc;
}

// Frees what the forms an order did not keep were built with: the polynomial buffer unless the
// order keeps the polynomial gather, the cell items when it keeps the sorted gather.
void drop_unused(gt_plan *pl, int t) {
  OrderHost &o = pl->ord[t];
  if (o.path != GT_GATHER_POLY && o.d_kpoly) {
    dev_free(o.d_kpoly, nullptr);
    o.d_kpoly = nullptr;
  }
  if ((o.path == GT_GATHER_SORTED || o.path == GT_GATHER_DIRECT) && o.d_citems) {
    dev_free(o.d_citems, nullptr);
    o.d_citems = nullptr;
    o.citems.clear();
    o.citem_begin.clear();
  }
}

// A cached choice on a new plan; a form this plan cannot take (no cell items for its nodes)
// leaves the plan's default for that order.
void apply(gt_plan *pl, const TuneChoice &c) {
  for (int t = 1; t <= pl->ds; ++t) {
    if (pl->ord[t].term_end == pl->ord[t].term_begin || pl->ord[t].path == c.path[t]) continue;
    if (set_gather_path(pl, t, c.path[t]) == GT_OK)
      drop_unused(pl, t);
    else
      set_error("");
  }
  if (pl->ds >= 2 && pl->ord[2].waves_cu != c.waves_cu && set_tile_waves(pl, c.waves_cu) != GT_OK) {
    set_error("");
    (void)set_tile_waves(pl, kTileWavesPerCU);
  }
  for (int t = 1; t <= pl->ds; ++t) {
    if (pl->ord[t].term_end == pl->ord[t].term_begin || pl->ord[t].adj_form == c.adj[t]) continue;
    if (set_adjoint_form(pl, t, c.adj[t]) != GT_OK) set_error("");
  }
  pl->use_side = c.use_side;
  pl->use_graph = c.use_graph;
  pl->use_fused = c.use_fused && fused_available(pl);
}

}  // namespace

// (a graph may still run on the stream it was launched on, which the caller may since have
// destroyed: wait for the device before destroying them)
void drop_graphs(gt_plan *pl) {
  if (pl->graphs.empty()) return;
  (void)hipDeviceSynchronize();
  for (auto &g : pl->graphs) (void)hipGraphExecDestroy(g.exec);
  pl->graphs.clear();
}

void clear_tuning_cache() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
}

// A new plan takes the cached choice of its signature, if any (no timing).
int apply_cached_tuning(gt_plan *pl) {
  const TuneKey k = key_of(pl);
  TuneChoice c;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = std::find_if(g_tune.begin(), g_tune.end(), [&](const auto &e) { return e.first == k; });
    if (it == g_tune.end()) return GT_OK;
    c = it->second;
  }
  apply(pl, c);
  pl->tuning = c.report;
  return GT_OK;
}

// One transform through the plan's graph (captured on first use for these buffers) or eagerly.
// A graph is not used on the legacy default stream, nor while the caller's stream is itself
// being captured (then the caller's graph records the launches).
int run_plan_call(gt_plan *pl, int dir, const void *in, void *out, hipStream_t s) {
  if (!pl->use_graph || s == nullptr || prof_enabled()) return eager(pl, dir, in, out, s);
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  GT_HIP(hipStreamIsCapturing(s, &cs));
  if (cs != hipStreamCaptureStatusNone) return eager(pl, dir, in, out, s);
  for (auto &g : pl->graphs)
    if (g.dir == dir && g.in == in && g.out == out) {
      GT_HIP(hipGraphLaunch(g.exec, s));
      return GT_OK;
    }
  constexpr size_t kMaxGraphs = 8;
  if (pl->graphs.size() >= kMaxGraphs) {
    (void)hipDeviceSynchronize();
    (void)hipGraphExecDestroy(pl->graphs.front().exec);
    pl->graphs.erase(pl->graphs.begin());
  }
  GT_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
  const int rc = eager(pl, dir, in, out, s);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &graph);
  if (rc != GT_OK || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc != GT_OK ? rc : hip_fail(e, "hipStreamEndCapture");
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) return hip_fail(ei, "hipGraphInstantiate");
  pl->graphs.push_back({dir, in, out, s, exec});
  GT_HIP(hipGraphLaunch(exec, s));
  return GT_OK;
}

int tune_plan(gt_plan *pl, hipStream_t s) {
  const size_t csz = 2 * pl->rsize;
  TuneBufs b;
  if (int rc = dev_alloc(&b.fhat, (size_t)pl->R * pl->ncoef * csz, nullptr)) return rc;
  if (int rc = dev_alloc(&b.f, (size_t)pl->Vtot * csz, nullptr)) return rc;
  GT_HIP(hipMemsetAsync(b.fhat, 0, (size_t)pl->R * pl->ncoef * csz, s));
  GT_HIP(hipMemsetAsync(b.f, 0, (size_t)pl->Vtot * csz, s));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  GT_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(GT_EHIP, "hipEventCreate");
  }
  drop_graphs(pl);
  pl->use_graph = false;
  pl->use_fused = false;   // the per-order timings need the separate launches
  std::string js = "{\"cached\": false";
  char tmp[160];
  int rc = GT_OK;
  double fwd_ms = 0, adj_ms = 0, both_ms = 0;
  // 1. forward gather per order (coordinate descent, order by order, the highest first: its
  //    slow forms then run only while it is being timed, not in every call of the lower orders)
  js += ", \"gather\": {";
  bool firstg = true;
  for (int t = pl->ds; t >= 1 && rc == GT_OK; --t) {
    OrderHost &o = pl->ord[t];
    if (o.term_end == o.term_begin) continue;
    const int keep = o.path;
    int best = keep;
    double best_ms = 1e300;
    snprintf(tmp, sizeof(tmp), "%s\"%d\": {", firstg ? "" : ", ", t);
    js += tmp;
    firstg = false;
    bool first = true;
    for (int p = GT_GATHER_SORTED; p <= GT_GATHER_DIRECT && rc == GT_OK; ++p) {
      if (p == GT_GATHER_POLY && t != 2) continue;
      if (set_gather_path(pl, t, p) != GT_OK) {
        set_error("");
        continue;
      }
      double ms = 0;
      rc = time_order(pl, 0, t, b, s, &ms);
      if (rc != GT_OK) break;
      snprintf(tmp, sizeof(tmp), "%s\"%s\": %.4f", first ? "" : ", ", path_name(p), ms);
      js += tmp;
      first = false;
      if (ms < best_ms) {
        best_ms = ms;
        best = p;
      }
    }
    if (rc == GT_OK) rc = set_gather_path(pl, t, best);
    if (rc == GT_OK) drop_unused(pl, t);
    snprintf(tmp, sizeof(tmp), ", \"chosen\": \"%s\"}", path_name(best));
    js += tmp;
  }
  js += "}";
  // 2. order-2 tile spread: resident wavefronts per compute unit (adjoint)
  if (rc == GT_OK && pl->ds >= 2 && pl->ord[2].term_end > pl->ord[2].term_begin) {
    OrderHost &o = pl->ord[2];
    int best = o.waves_cu;
    double best_ms = 1e300;
    js += ", \"tile_waves_cu\": {";
    bool first = true;
    std::vector<int> tried_wg;   // workgroups per compute unit already timed
    // coarse 12, 20, 28; then the neighbours 4 apart of the best
    auto trial = [&](int w) -> int {
      if (w < 8 || w > 32) return GT_OK;
      if (int r2 = set_tile_waves(pl, w)) return r2;
      if (std::find(tried_wg.begin(), tried_wg.end(), o.tile_wg_cu) != tried_wg.end()) return GT_OK;
      tried_wg.push_back(o.tile_wg_cu);   // (the staging LDS may allow no more workgroups)
      double ms = 0;
      if (int r2 = time_order(pl, 1, 2, b, s, &ms)) return r2;
      snprintf(tmp, sizeof(tmp), "%s\"%d\": %.4f", first ? "" : ", ", w, ms);
      js += tmp;
      first = false;
      if (ms < best_ms) {
        best_ms = ms;
        best = w;
      }
      return GT_OK;
    };
    for (int w : {12, 20, 28})
      if (rc == GT_OK) rc = trial(w);
    const int coarse = best;
    if (rc == GT_OK) rc = trial(coarse - 4);
    if (rc == GT_OK) rc = trial(coarse + 4);
    if (rc == GT_OK) rc = set_tile_waves(pl, best);
    snprintf(tmp, sizeof(tmp), ", \"chosen\": %d}", best);
    js += tmp;
  }
  // 2b. adjoint form per order (window or direct sums)
  if (rc == GT_OK) {
    js += ", \"adjoint\": {";
    bool firsto = true;
    for (int t = pl->ds; t >= 1 && rc == GT_OK; --t) {   // the highest first, as above
      OrderHost &o = pl->ord[t];
      if (o.term_end == o.term_begin || !direct_adj_ok(pl, t)) continue;
      double ms[2] = {0, 0};
      for (int f = GT_ADJ_WINDOW; f <= GT_ADJ_DIRECT && rc == GT_OK; ++f) {
        if ((rc = set_adjoint_form(pl, t, f)) != GT_OK) break;
        rc = time_order(pl, 1, t, b, s, &ms[f]);
      }
      if (rc != GT_OK) break;
      const int best = ms[GT_ADJ_DIRECT] < ms[GT_ADJ_WINDOW] ? GT_ADJ_DIRECT : GT_ADJ_WINDOW;
      rc = set_adjoint_form(pl, t, best);
      if (best == GT_ADJ_WINDOW && o.d_dpart) {
        dev_free(o.d_dpart, nullptr);
        o.d_dpart = nullptr;
        o.dir_nslice = 0;
      }
      snprintf(tmp, sizeof(tmp), "%s\"%d\": {\"window\": %.4f, \"direct\": %.4f, \"chosen\": \"%s\"}",
               firsto ? "" : ", ", t, ms[0], ms[1], best == GT_ADJ_DIRECT ? "direct" : "window");
      js += tmp;
      firsto = false;
    }
    js += "}";
  }
  // 3. second stream for order 1 on or off (forward + adjoint).  Streams share the device's
  //    few hardware queues; a second stream that landed on the caller's queue runs nothing
  //    beside it, so when the second stream does not pay, up to three fresh ones are tried
  //    and the fastest kept.
  if (rc == GT_OK && pl->side && pl->ds >= 2) {
    double on = 0, off = 0;
    pl->use_side = true;
    rc = time_calls(pl, 3, b, s, e0, e1, &on);
    if (rc == GT_OK) {
      pl->use_side = false;
      rc = time_calls(pl, 3, b, s, e0, e1, &off);
    }
    int renewed = 0;
    for (int k = 0; k < 3 && rc == GT_OK && on > 0.95 * off; ++k) {
      hipStream_t fresh = nullptr;
      if (hipStreamCreateWithFlags(&fresh, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        break;
      }
      hipStream_t old = pl->side;
      pl->side = fresh;
      pl->use_side = true;
      double t = 0;
      rc = time_calls(pl, 3, b, s, e0, e1, &t);
      (void)hipStreamSynchronize(old);
      (void)hipStreamSynchronize(fresh);
      if (rc == GT_OK && t < on) {
        on = t;
        (void)hipStreamDestroy(old);
        ++renewed;
      } else {
        pl->side = old;
        (void)hipStreamDestroy(fresh);
      }
    }
    pl->use_side = on <= off;
    if (renewed) {
      snprintf(tmp, sizeof(tmp), ", \"side_stream_renewed\": %d", renewed);
      js += tmp;
    }
    snprintf(tmp, sizeof(tmp), ", \"side_stream\": {\"on\": %.4f, \"off\": %.4f, \"chosen\": %s}", on, off,
             pl->use_side ? "true" : "false");
    js += tmp;
    //    then both orders in shared launches against the better of those
    if (rc == GT_OK && fused_available(pl)) {
      double fu = 0;
      pl->use_fused = true;
      rc = time_calls(pl, 3, b, s, e0, e1, &fu);
      pl->use_fused = rc == GT_OK && fu < 0.95 * std::min(on, off);   // only a clear gain
      snprintf(tmp, sizeof(tmp), ", \"fused\": {\"on\": %.4f, \"off\": %.4f, \"chosen\": %s}", fu,
               std::min(on, off), pl->use_fused ? "true" : "false");
      js += tmp;
    }
  }
  // 4. graph replay against eager launches (forward + adjoint); not on the legacy default
  //    stream, where the plan does not capture
  if (rc == GT_OK && s == nullptr) {
    pl->use_graph = false;
    js += ", \"graph\": \"not on the default stream\"";
  } else if (rc == GT_OK) {
    double eg = 0, gr = 0;
    pl->use_graph = false;
    rc = time_calls(pl, 3, b, s, e0, e1, &eg);
    if (rc == GT_OK) {
      pl->use_graph = true;
      rc = time_calls(pl, 3, b, s, e0, e1, &gr);
    }
    pl->use_graph = rc == GT_OK && gr < eg;
    drop_graphs(pl);   // the timing buffers' graphs
    snprintf(tmp, sizeof(tmp), ", \"graph\": {\"eager\": %.4f, \"replay\": %.4f, \"chosen\": %s}", eg, gr,
             pl->use_graph ? "true" : "false");
    js += tmp;
    both_ms = std::min(eg, rc == GT_OK ? gr : eg);
  }
  if (rc == GT_OK) rc = time_calls(pl, 1, b, s, e0, e1, &fwd_ms);
  if (rc == GT_OK) rc = time_calls(pl, 2, b, s, e0, e1, &adj_ms);
  drop_graphs(pl);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != GT_OK) return rc;
  if (both_ms == 0) both_ms = fwd_ms + adj_ms;
  snprintf(tmp, sizeof(tmp), ", \"forward_ms\": %.4f, \"adjoint_ms\": %.4f, \"step_ms\": %.4f}", fwd_ms, adj_ms, both_ms);
  js += tmp;
  TuneChoice c;
  for (int t = 0; t <= kMaxOrder; ++t) {
    c.path[t] = t <= pl->ds ? pl->ord[t].path : GT_GATHER_SORTED;
    c.adj[t] = t <= pl->ds ? pl->ord[t].adj_form : GT_ADJ_WINDOW;
  }
  c.waves_cu = pl->ds >= 2 ? pl->ord[2].waves_cu : kTileWavesPerCU;
  c.use_side = pl->use_side;
  c.use_graph = pl->use_graph;
  c.use_fused = pl->use_fused;
  pl->tuning = js;
  c.report = js;
  c.report.replace(0, strlen("{\"cached\": false"), "{\"cached\": true");
  const TuneKey k = key_of(pl);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = std::find_if(g_tune.begin(), g_tune.end(), [&](const auto &e) { return e.first == k; });
  if (it != g_tune.end())
    it->second = c;
  else
    g_tune.push_back({k, c});
  return GT_OK;
}

}  // namespace gt
