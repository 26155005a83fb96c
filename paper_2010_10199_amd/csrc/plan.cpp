// Host runtime: index set, Kaiser-Bessel window tables, plans, C ABI entry points.
//
// Index set (Sec. 2): U_{d_s} (eq. pizmosch), groups I_N^{u,d} with (N-1)^{|u|} members
// (eq. metallica, Remark rem:cardinality), grouped set = disjoint union (eq. groupedset).
//
// Fast transform of one term (eq. somafm): the paper delegates the |u|-dimensional
// nonequispaced FFT to the NFFT literature it cites.  This library uses the textbook
// three-step form with a Kaiser-Bessel window Phi of half-width m on an oversampled grid of
// n = sigma N points per axis (window in grid units tau = n x - l):
//   Phi(tau) = m sinh(b sqrt(m^2 - tau^2)) / (sqrt(m^2 - tau^2) sinh(b m)),  |tau| < m,
//   b = pi (2 - 1/sigma),
//   Phi_hat(k) = int_{-m}^{m} Phi(tau) e^{-2 pi i k tau / n} dtau   (Gauss-Legendre, long double),
// forward: scale coefficients by (-1)^k / Phi_hat(k) per axis, inverse DFT onto the grid,
// gather with the window; adjoint: spread with the window, forward DFT, same scaling.
// The (-1)^k places grid index 0 at x = -1/2.  The window is evaluated on the GPU from
// per-window-point polynomials in the fractional node offset (Chebyshev interpolation of
// Phi converted to monomials), so the device never calls sinh or sqrt.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "gt_internal.h"

namespace gt {

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int code, const std::string &msg) {
  set_error(msg);
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? GT_ENOMEM : GT_EHIP;
}

// ------------------------------------------------------------------ profiling
struct ProfRec {
  const char *name;
  hipEvent_t a, b;
};
static std::mutex g_prof_mu;
static bool g_prof_on = false;
static std::vector<ProfRec> g_prof;
static thread_local int g_prof_open = -1;

bool prof_enabled() { return g_prof_on; }

void prof_begin(hipStream_t s, const char *name) {
  if (!g_prof_on) return;
  ProfRec r{name, nullptr, nullptr};
  if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return;
  (void)hipEventRecord(r.a, s);
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof.push_back(r);
  g_prof_open = (int)g_prof.size() - 1;
}

void prof_end(hipStream_t s) {
  if (!g_prof_on || g_prof_open < 0) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  (void)hipEventRecord(g_prof[g_prof_open].b, s);
  g_prof_open = -1;
}

bool prof_set(bool on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  const bool was = g_prof_on;
  g_prof_on = on;
  return was;
}

size_t prof_mark() {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  return g_prof.size();
}

// Milliseconds of the records made since `mark` whose names end in `suffix` (waits for them),
// and removes those records.
double prof_take_since(size_t mark, const char *suffix) {
  std::vector<ProfRec> recs;
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (mark < g_prof.size()) {
      recs.assign(g_prof.begin() + (std::ptrdiff_t)mark, g_prof.end());
      g_prof.resize(mark);
    }
  }
  const size_t ls = strlen(suffix);
  double ms = 0;
  for (auto &r : recs) {
    float t = 0;
    const size_t ln = strlen(r.name);
    if (ln >= ls && strcmp(r.name + ln - ls, suffix) == 0 && hipEventSynchronize(r.b) == hipSuccess &&
        hipEventElapsedTime(&t, r.a, r.b) == hipSuccess)
      ms += t;
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  return ms;
}

// ------------------------------------------------------------------ device allocation
// Allocation-failure hook (gt_debug_fail_alloc): when armed with k >= 1, the k-th device
// allocation from then on fails with GT_ENOMEM as if the device were out of memory.
static std::mutex g_alloc_mu;
static int64_t g_alloc_count = 0;    // device allocations since the last gt_debug_fail_alloc
static int64_t g_alloc_fail_at = 0;  // 0: hook off

int dev_alloc(void **p, size_t bytes, hipStream_t) {
  *p = nullptr;
  if (bytes == 0) return GT_OK;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    ++g_alloc_count;
    if (g_alloc_fail_at > 0 && g_alloc_count == g_alloc_fail_at)
      return fail(GT_ENOMEM, "device allocation failed (allocation-failure hook)");
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return hip_fail(e, "hipMalloc");
  }
  return GT_OK;
}

void dev_free(void *p, hipStream_t) {
  if (p) (void)hipFree(p);
}

// ------------------------------------------------------------------ live plans
static std::mutex g_plans_mu;
static std::vector<gt_plan *> g_plans;

static void plan_register(gt_plan *pl) {
  std::lock_guard<std::mutex> lk(g_plans_mu);
  g_plans.push_back(pl);
}

// Removes pl from the live set; false when it is not a live plan.
static bool plan_unregister(gt_plan *pl) {
  std::lock_guard<std::mutex> lk(g_plans_mu);
  auto it = std::find(g_plans.begin(), g_plans.end(), pl);
  if (it == g_plans.end()) return false;
  g_plans.erase(it);
  return true;
}

bool plan_is_live(const gt_plan *pl) {
  std::lock_guard<std::mutex> lk(g_plans_mu);
  return pl && std::find(g_plans.begin(), g_plans.end(), pl) != g_plans.end();
}

// ------------------------------------------------------------------ index set
// Terms of U_{d_s} in coefficient order (by order, then the sorted coordinates
// lexicographically), fn(ci, t, c) for each with its index ci in this enumeration (the index
// of a term mask) and its coordinates c[0..t-1].
template <typename F>
static void for_each_term(int d, int ds, F fn) {
  int64_t ci = 0;
  for (int t = 0; t <= ds; ++t) {
    int c[3] = {0, 1, 2};
    while (true) {
      fn(ci++, t, (const int *)c);
      if (t == 0) break;
      int i = t - 1;
      while (i >= 0 && c[i] == d - t + i) --i;
      if (i < 0) break;
      ++c[i];
      for (int k = i + 1; k < t; ++k) c[k] = c[k - 1] + 1;
    }
  }
}

static int64_t binom(int n, int k) {
  if (k < 0 || k > n) return 0;
  int64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

int validate_problem(const gt_problem *p) {
  if (!p) return fail(GT_EINVAL, "problem is NULL");
  if (p->d < 1) return fail(GT_EINVAL, "d must be >= 1");
  if (p->ds < 0 || p->ds > p->d) return fail(GT_EINVAL, "need 0 <= ds <= d");
  if (p->ds > kMaxOrder) return fail(GT_EUNSUPPORTED, "terms of order > 3 are not implemented on the GPU path");
  if (p->basis != GT_BASIS_EXP && p->basis != GT_BASIS_COS) return fail(GT_EINVAL, "basis must be GT_BASIS_EXP or GT_BASIS_COS");
  for (int t = 1; t <= p->ds; ++t) {
    int N = p->N[t - 1];
    if (N < 2 || (N % 2)) return fail(GT_EINVAL, "bandwidths must be even and >= 2");
    if (N > (p->basis == GT_BASIS_COS ? 2048 : 4096)) return fail(GT_EUNSUPPORTED, "bandwidth above 4096 (cosine: 2048)");
  }
  if (p->R < 1) return fail(GT_EINVAL, "R must be >= 1");
  if (p->dtype != GT_C64 && p->dtype != GT_C128) return fail(GT_EINVAL, "dtype must be GT_C64 or GT_C128");
  if (p->m != 0 && (p->m < kMinM || p->m > kMaxM)) return fail(GT_EUNSUPPORTED, "window half-width m must be 2..8 (or 0)");
  if (p->sigma != 0.0 && !(p->sigma >= 1.5 && p->sigma <= 8.0)) return fail(GT_EINVAL, "sigma must be in [1.5, 8] (or 0)");
  if (p->offsets) {
    if (p->offsets[0] != 0) return fail(GT_EINVAL, "offsets[0] must be 0");
    for (int b = 0; b < p->R; ++b)
      if (p->offsets[b + 1] < p->offsets[b]) return fail(GT_EINVAL, "offsets must be non-decreasing");
    if (p->offsets[p->R] <= 0) return fail(GT_EINVAL, "ragged node total must be > 0");
  } else if (p->M <= 0) {
    return fail(GT_EINVAL, "M must be > 0");
  }
  return GT_OK;
}

// Smallest m with the Kaiser-Bessel error model 2.3 exp(-2 pi m sqrt(1 - 1/sigma)) below
// the precision's target (1e-6 for FP32 bulk arithmetic, 1e-14 for FP64, which leaves a
// wide margin below the 1e-12 relative error the FP64 path is held to).
int choose_m(int dtype, double sigma) {
  const double target = dtype == GT_C64 ? 1e-6 : 1e-14;
  const double rate = 2.0 * M_PI * std::sqrt(1.0 - 1.0 / sigma);
  int m = (int)std::ceil(std::log(2.3 / target) / rate);
  return std::min(kMaxM, std::max(kMinM, m));
}

// ------------------------------------------------------------------ window maths (long double)
static long double kb_phi(long double tau, int m, long double b) {
  long double s2 = (long double)m * m - tau * tau;
  if (s2 < 0) return 0.0L;
  long double s = std::sqrt(s2);
  long double bs = b * s;
  long double ratio = bs < 1e-4L ? b * (1.0L + bs * bs / 6.0L) : std::sinh(bs) / s;
  return ratio * (long double)m / std::sinh(b * (long double)m);
}

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_q.
static void gauss_legendre(int q, std::vector<long double> &x, std::vector<long double> &w) {
  x.assign(q, 0);
  w.assign(q, 0);
  for (int i = 0; i < q; ++i) {
    long double z = std::cos(M_PIl * (i + 0.75L) / (q + 0.5L));
    long double dp = 0;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1, p1 = z;
      for (int k = 2; k <= q; ++k) {
        long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = q * (z * p1 - p0) / (z * z - 1);
      long double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-19L) break;
    }
    x[i] = z;
    w[i] = 2.0L / ((1 - z * z) * dp * dp);
  }
}

// Phi_hat(k) = 2 int_0^m Phi(tau) cos(2 pi k tau / n) dtau (Phi is even and analytic on [0, m]).
static long double kb_phihat(int k, int m, long double b, int n) {
  static std::vector<long double> gx, gw;
  static std::once_flag once;
  std::call_once(once, [] { gauss_legendre(96, gx, gw); });
  long double acc = 0;
  for (size_t i = 0; i < gx.size(); ++i) {
    long double tau = 0.5L * m * (gx[i] + 1.0L);
    acc += gw[i] * kb_phi(tau, m, b) * std::cos(2.0L * M_PIl * k * tau / n);
  }
  return acc * (long double)m;   // 2 * (m/2) * sum
}

// Monomial coefficients (in z in [-1, 1]) of the degree-D Chebyshev interpolant of
// z -> Phi(m - 1 + (z + 1)/2 - j) for window point j (tau for fractional offset (z+1)/2).
static void window_poly(int m, long double b, int D, std::vector<double> &out) {
  const int W = 2 * m;
  out.assign((size_t)W * (D + 1), 0.0);
  std::vector<long double> zi(D + 1), fi(D + 1), c(D + 1), mono(D + 1), Tkm1(D + 1), Tk(D + 1), Tkp1(D + 1);
  for (int i = 0; i <= D; ++i) zi[i] = std::cos(M_PIl * (i + 0.5L) / (D + 1));
  for (int j = 0; j < W; ++j) {
    for (int i = 0; i <= D; ++i) fi[i] = kb_phi((long double)(m - 1) + 0.5L * (zi[i] + 1.0L) - j, m, b);
    for (int k = 0; k <= D; ++k) {
      long double s = 0;
      for (int i = 0; i <= D; ++i) s += fi[i] * std::cos(M_PIl * k * (i + 0.5L) / (D + 1));
      c[k] = s * 2.0L / (D + 1);
    }
    c[0] *= 0.5L;
    // sum_k c_k T_k(z) in monomials: T_0 = 1, T_1 = z, T_{k+1} = 2 z T_k - T_{k-1}
    std::fill(mono.begin(), mono.end(), 0.0L);
    std::fill(Tkm1.begin(), Tkm1.end(), 0.0L);
    std::fill(Tk.begin(), Tk.end(), 0.0L);
    Tkm1[0] = 1;
    mono[0] += c[0];
    if (D >= 1) {
      Tk[1] = 1;
      mono[1] += c[1];
    }
    for (int k = 1; k < D; ++k) {
      std::fill(Tkp1.begin(), Tkp1.end(), 0.0L);
      for (int q = 0; q <= D; ++q) {
        if (q + 1 <= D) Tkp1[q + 1] += 2 * Tk[q];
        Tkp1[q] -= Tkm1[q];
      }
      for (int q = 0; q <= D; ++q) mono[q] += c[k + 1] * Tkp1[q];
      Tkm1 = Tk;
      Tk = Tkp1;
    }
    for (int q = 0; q <= D; ++q) out[(size_t)j * (D + 1) + q] = (double)mono[q];
  }
  // Phi is even: point 2m-1-j at offset fr equals point j at 1 - fr, i.e. at -z.  Mirror the
  // coefficients so that the pair is exactly symmetric (the kernels evaluate pairs together).
  for (int j = 0; j < m; ++j)
    for (int q = 0; q <= D; ++q)
      out[(size_t)(W - 1 - j) * (D + 1) + q] = (q & 1) ? -out[(size_t)j * (D + 1) + q] : out[(size_t)j * (D + 1) + q];
}

}  // namespace gt

using namespace gt;

// ------------------------------------------------------------------ plan build
namespace {

template <typename T>
int upload(const std::vector<double> &h, void **d) {
  std::vector<T> tmp(h.begin(), h.end());
  int rc = dev_alloc(d, tmp.size() * sizeof(T), nullptr);
  if (rc) return rc;
  GT_HIP(hipMemcpy(*d, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice));
  return GT_OK;
}

template <typename V>
int upload_raw(const std::vector<V> &h, V **d) {
  int rc = dev_alloc((void **)d, h.size() * sizeof(V), nullptr);
  if (rc) return rc;
  if (!h.empty()) GT_HIP(hipMemcpy(*d, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice));
  return GT_OK;
}

// Idle side streams per device, reused by later plans: creating a stream takes about 0.7 ms
// on this runtime and every plan takes one, so a plan returns its stream here when it is
// destroyed (after the stream has drained) and the next plan on that device takes it.
static std::mutex g_side_mu;
static std::vector<std::pair<int, hipStream_t>> g_side_pool;
constexpr size_t kSidePoolMax = 64;

static hipStream_t take_side(int dev) {
  {
    std::lock_guard<std::mutex> lk(g_side_mu);
    for (size_t i = g_side_pool.size(); i-- > 0;)
      if (g_side_pool[i].first == dev) {
        const hipStream_t st = g_side_pool[i].second;
        g_side_pool.erase(g_side_pool.begin() + (std::ptrdiff_t)i);
        return st;
      }
  }
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return st;
}

static void give_side(hipStream_t st) {
  if (!st) return;
  (void)hipStreamSynchronize(st);
  int dev = -1;
  if (hipStreamGetDevice(st, &dev) == hipSuccess) {
    std::lock_guard<std::mutex> lk(g_side_mu);
    if (g_side_pool.size() < kSidePoolMax) {
      g_side_pool.emplace_back(dev, st);
      return;
    }
  }
  (void)hipGetLastError();
  (void)hipStreamDestroy(st);
}

static void drain_side_pool() {
  std::vector<std::pair<int, hipStream_t>> all;
  {
    std::lock_guard<std::mutex> lk(g_side_mu);
    all.swap(g_side_pool);
  }
  for (auto &e : all) (void)hipStreamDestroy(e.second);
}

void free_plan(gt_plan *pl) {
  if (!pl) return;
  if (pl->stream) (void)hipStreamSynchronize(pl->stream);
  drop_graphs(pl);
  if (pl->side) {
    give_side(pl->side);
    pl->side = nullptr;
  }
  if (pl->ev_fork) (void)hipEventDestroy(pl->ev_fork);
  if (pl->ev_join) (void)hipEventDestroy(pl->ev_join);
  pl->ev_fork = pl->ev_join = nullptr;
  dev_free(pl->d_terms, nullptr);
  dev_free(pl->d_x, nullptr);
  dev_free(pl->d_grid, nullptr);
  dev_free(pl->d_gitems, nullptr);
  dev_free(pl->d_gitem_begin, nullptr);
  dev_free(pl->d_fpart, nullptr);
  dev_free(pl->d_ysum, nullptr);
  dev_free(pl->d_flag, nullptr);
  dev_free(pl->d_gxp, nullptr);
  dev_free(pl->d_cterms, nullptr);
  dev_free(pl->d_gcos, nullptr);
  for (auto &o : pl->ord) {
    dev_free(o.d_deconv, nullptr);
    dev_free(o.d_roots, nullptr);
    dev_free(o.d_poly, nullptr);
    dev_free(o.d_gitems, nullptr);
    dev_free(o.d_citems, nullptr);
    dev_free(o.d_kpoly, nullptr);
    dev_free(o.d_sitems, nullptr);
    dev_free(o.d_sitem_begin, nullptr);
    dev_free(o.d_gpart, nullptr);
    dev_free(o.d_perm, nullptr);
    dev_free(o.d_gsum, nullptr);
    dev_free(o.d_cstart, nullptr);
    dev_free(o.d_xs, nullptr);
    dev_free(o.d_waves2, nullptr);
    dev_free(o.d_tileseg, nullptr);
    dev_free(o.d_patch, nullptr);
    dev_free(o.d_tsum, nullptr);
    dev_free(o.d_dpart, nullptr);
  }
  dev_free(pl->rebin.kin, nullptr);
  dev_free(pl->rebin.kout, nullptr);
  dev_free(pl->rebin.vin, nullptr);
  dev_free(pl->rebin.tmp, nullptr);
  dev_free(pl->rebin.offs, nullptr);
  dev_free(pl->rebin.seg, nullptr);
  dev_free(pl->rebin.segcnt, nullptr);
  delete pl;
}


// The binning's cell starts of order t on the host (nt x B x nkey + 1 positions), copied
// once per plan for both setups below.
static int fetch_cell_starts(gt_plan *pl, int t, hipStream_t s, std::vector<int64_t> &cs) {
  const OrderHost &o = pl->ord[t];
  const int B = pl->ragged ? pl->R : 1;
  const int64_t nkeys = (int64_t)(o.term_end - o.term_begin) * B * o.nkey + 1;
  cs.resize(nkeys);
  hipError_t e = hipMemcpyAsync(cs.data(), o.d_cstart, nkeys * sizeof(int64_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? GT_OK : hip_fail(e, "cell boundaries");
}

// Work list of the order-2 tile spread (needs the binning's tile boundaries on the host).
// The wavefronts of all right-hand sides make one resident round of tile_wg_cu workgroups
// per compute unit (as many as the staging LDS allows, at most kTileWavesPerCU / kTileWaves);
// the launch pads the LDS so that no compute unit takes more, since a few compute units
// with an extra workgroup would finish last.  Each (term, dataset) gets its share of the
// wavefronts, rounded down (at least one, at least 256 nodes each), over equal runs of its
// sorted positions.  A wavefront writes one 16 x 16 patch per tile it meets, in
// tile order, so its segments are numbered consecutively from its first segment; the
// segments of one tile are consecutive too (waves follow the sorted order), which gives the
// fold its per-tile segment ranges.
static int setup_tile_spread(gt_plan *pl, const std::vector<int64_t> &cs) {
  OrderHost &o = pl->ord[2];
  const int nt = o.term_end - o.term_begin;
  if (nt == 0) return GT_OK;
  const int B = pl->ragged ? pl->R : 1;
  const int TS = o.ts, TT = TS * TS;
  const int64_t ntiles = (int64_t)o.ntile * o.ntile;
  const int64_t total = (int64_t)nt * pl->Mtot;
  const int reff = pl->ragged ? 1 : pl->R;
  // (the LDS of a compute unit equals the per-workgroup limit on this GPU)
  const size_t lds2 = kTileWaves * tile_lds_wave(pl->rsize);
  o.tile_wg_cu = (int32_t)std::max<size_t>(1, std::min<size_t>(o.waves_cu / kTileWaves, pl->lds_limit / lds2));
  const int64_t want_waves = std::max<int64_t>(1, (int64_t)pl->num_cu * kTileWaves * o.tile_wg_cu / reff);
  std::vector<int32_t> waves;
  std::vector<int32_t> tileseg((size_t)nt * B * ntiles + 1, 0);
  int64_t nseg = 0;
  for (int tl = 0; tl < nt; ++tl) {
    for (int b = 0; b < B; ++b) {
      const int64_t key0 = ((int64_t)tl * B + b) * o.nkey;
      const int64_t tb0 = ((int64_t)tl * B + b) * ntiles;
      const int64_t P0 = cs[key0], P1 = cs[key0 + ntiles * TT];
      const int64_t Mb = P1 - P0;
      const int64_t nw = Mb > 0 ? std::max<int64_t>(1, std::min<int64_t>((Mb + 255) / 256, Mb * want_waves / total)) : 0;
      std::vector<int32_t> tfirst(ntiles, -1);
      int64_t tile = 0;
      for (int64_t w = 0; w < nw; ++w) {
        const int64_t qa = P0 + Mb * w / nw, qb = P0 + Mb * (w + 1) / nw;
        waves.push_back((int32_t)qa);
        waves.push_back((int32_t)qb);
        waves.push_back((int32_t)nseg);
        waves.push_back(b);
        while (tile < ntiles && cs[key0 + (tile + 1) * TT] <= qa) ++tile;   // first tile ending after qa
        for (int64_t t = tile; t < ntiles && cs[key0 + t * TT] < qb; ++t) {
          if (cs[key0 + (t + 1) * TT] <= cs[key0 + t * TT]) continue;        // empty tile
          if (tfirst[t] < 0) tfirst[t] = (int32_t)nseg;
          ++nseg;
        }
      }
      // per-tile first segment (a tile without nodes gets an empty range)
      int32_t next = (int32_t)nseg;
      for (int64_t t = ntiles - 1; t >= 0; --t) {
        if (tfirst[t] >= 0) next = tfirst[t];
        tileseg[tb0 + t] = next;
      }
    }
  }
  tileseg[(size_t)nt * B * ntiles] = (int32_t)nseg;
  if (nseg >= (int64_t(1) << 31) / 256) return fail(GT_EUNSUPPORTED, "too many tile patches");
  o.nwaves2 = (int32_t)(waves.size() / 4);
  o.nseg2 = nseg;
  int rc;
  if ((rc = upload_raw(waves, &o.d_waves2)) || (rc = upload_raw(tileseg, &o.d_tileseg))) return rc;
  const size_t csz = 2 * pl->rsize;
  if ((rc = dev_alloc(&o.d_patch, (size_t)reff * std::max<int64_t>(1, nseg) * 256 * csz, nullptr))) return rc;
  if ((rc = dev_alloc(&o.d_tsum, (size_t)pl->R * nt * o.ntile * 16 * o.n * csz, nullptr))) return rc;
  return GT_OK;
}

// Cell gather items (k_gather_cell, k_gather_poly2): runs of at most 64 sorted positions inside
// one grid cell of one term and dataset, from the binning's cell starts of order t (host copy).
// Returns the lane fill of the items in *fill; builds them only when `force` or when they fill
// at least kCellGatherFill of the lanes they occupy (otherwise the order keeps
// k_gather_sorted, whose workgroups take any 1024 consecutive positions).
static int build_cell_items(gt_plan *pl, int t, bool force, double *fill_out) {
  OrderHost &o = pl->ord[t];
  if (fill_out) *fill_out = 0.0;
  if (!o.citems.empty()) return GT_OK;   // built before
  const int nt = o.term_end - o.term_begin;
  if (nt == 0 || (int64_t)nt * pl->Mtot >= (int64_t(1) << 31)) return GT_OK;
  if (o.cstart_host.empty())             // (dropped by a node update)
    if (int rc = fetch_cell_starts(pl, t, pl->stream, o.cstart_host)) return rc;
  const int B = pl->ragged ? pl->R : 1;
  const std::vector<int64_t> &cs = o.cstart_host;
  // lane fill of the items (runs of <= 64 nodes of one cell), decided before building them
  int64_t nitems = 0;
  for (size_t k = 0; k + 1 < cs.size(); ++k) nitems += (cs[k + 1] - cs[k] + 63) / 64;
  const double fill = nitems == 0 ? 0.0 : (double)((int64_t)nt * pl->Mtot) / (64.0 * (double)nitems);
  if (fill_out) *fill_out = fill;
  if ((!force && fill < kCellGatherFill) || nitems == 0 || nitems >= (int64_t(1) << 31)) return GT_OK;
  std::vector<CellItem> items;
  items.reserve((size_t)nitems);
  std::vector<int32_t> begin(nt + 1, 0);
  for (int tl = 0; tl < nt; ++tl) {
    begin[tl] = (int32_t)items.size();
    for (int b = 0; b < B; ++b) {
      const int64_t key0 = ((int64_t)tl * B + b) * o.nkey;
      for (int64_t k = 0; k < o.nkey; ++k) {
        const int64_t c0 = cs[key0 + k], c1 = cs[key0 + k + 1];
        if (c1 <= c0) continue;
        // the cell of binning key k (order 2 numbers cells tile-major, see the binning)
        int32_t cell[3] = {0, 0, 0};
        if (t == 1) {
          cell[0] = (int32_t)k;
        } else if (t == 2) {
          const int64_t TT = (int64_t)o.ts * o.ts, tile = k / TT, rem = k - tile * TT;
          cell[0] = (int32_t)((tile / o.ntile) * o.ts + rem / o.ts);
          cell[1] = (int32_t)((tile % o.ntile) * o.ts + rem % o.ts);
        } else {
          cell[0] = (int32_t)(k / ((int64_t)o.n * o.n));
          cell[1] = (int32_t)((k / o.n) % o.n);
          cell[2] = (int32_t)(k % o.n);
        }
        for (int64_t q = c0; q < c1; q += 64) {
          CellItem ci{};
          ci.q0 = (int32_t)q;
          ci.count = (int32_t)std::min<int64_t>(64, c1 - q);
          ci.tl = tl;
          ci.r = pl->ragged ? b : 0;
          ci.cell[0] = cell[0];
          ci.cell[1] = cell[1];
          ci.cell[2] = cell[2];
          items.push_back(ci);
        }
      }
    }
  }
  begin[nt] = (int32_t)items.size();
  o.citems.swap(items);
  o.citem_begin.swap(begin);
  return upload_raw(o.citems, &o.d_citems);
}

// Order 2, FP32: the gather can evaluate per-cell polynomials (k_pack_poly2 / k_gather_poly2)
// when their coefficients take at most kPolyMaxBytes and the pack's arrays fit in LDS (needs
// the cell items).  Allocates the coefficient buffer; false when the form is not available.
static int build_poly(gt_plan *pl, bool *ok) {
  OrderHost &o = pl->ord[2];
  *ok = false;
  if (o.d_kpoly) {
    *ok = true;
    return GT_OK;
  }
  if (pl->dtype != GT_C64 || o.citems.empty()) return GT_OK;
  constexpr int NQ = Deg<float>::value + 1;
  const int nt = o.term_end - o.term_begin;
  const size_t bytes = (size_t)pl->R * nt * o.n * o.n * NQ * NQ * 2 * sizeof(float);
  if (bytes > kPolyMaxBytes || poly_pack_lds(o) > pl->lds_limit) return GT_OK;
  if (int rc = dev_alloc(&o.d_kpoly, bytes, nullptr)) return rc;
  *ok = true;
  return GT_OK;
}

// The default forward form per order: the polynomial gather when available, else the cell
// gather when its items fill the lanes, else the sorted gather.
static int setup_cell_gather(gt_plan *pl) {
  for (int t = 1; t <= pl->ds; ++t) {
    OrderHost &o = pl->ord[t];
    o.path = GT_GATHER_SORTED;
    if (o.term_end == o.term_begin) continue;
    if (int rc = build_cell_items(pl, t, false, nullptr)) return rc;
    if (o.citems.empty()) continue;
    o.path = GT_GATHER_CELL;
    if (t == 2) {
      bool ok = false;
      if (int rc = build_poly(pl, &ok)) return rc;
      if (ok) o.path = GT_GATHER_POLY;
    }
  }
  return GT_OK;
}

}  // namespace

// Selects a forward form for order t (building what it needs); GT_EUNSUPPORTED when the form
// is not available for this plan.
// Direct sums (direct.h): shared nodes, at most 16 right-hand sides (the columns of the
// contraction).  Forward LDS: the coefficients as B rows ((G + 1) x (16 CT + 1) reals) and
// the phase tables of the workgroup's 64 rtw nodes (two versions of the first axis's K phases
// plus a zero row, the G / K products of the other axes rounded up to even, and for order 3
// the two per-axis tables, rows padded by 16); adjoint: |I_u| <= 256 (rows 2 G in at most 8
// row tiles per wavefront), samples (2 x 16 x 65 reals) and the phase tables of 64 nodes
// (three versions of the first axis and a zero row, the products of the others, order 3's
// per-axis tables, rows of 68).
static int64_t group_size(const gt_plan *pl, int t) {
  int64_t G = 1;
  for (int a = 0; a < t; ++a) G *= pl->ord[t].N - 1;
  return G;
}
static size_t direct_fwd_lds(const gt_plan *pl, int t, int rtw) {
  const size_t CT = pl->R <= 8 ? 1 : 2;
  const size_t K = (size_t)(pl->ord[t].N - 1), G = (size_t)group_size(pl, t), rows = 64 * (size_t)rtw + 16;
  const size_t KR2 = G / K + ((G / K) & 1);
  const size_t breals = ((G + 1) * (16 * CT + 1) + 3) & ~(size_t)3;
  return breals * pl->rsize + (2 * (K + 1) + (t >= 2 ? KR2 : 0) + (t == 3 ? 2 * K : 0)) * rows * 2 * pl->rsize +
         (size_t)t * 64 * rtw * pl->rsize;
}
// row tiles per wavefront: the most (4, 2, 1) that leave room for three workgroups per
// compute unit, else one (measured on the d = 20 workload's order 3: one and two row tiles
// alike, four 11 % slower)
int gt::direct_fwd_rtw(const gt_plan *pl, int t) {
  for (int rtw : {4, 2})
    if (direct_fwd_lds(pl, t, rtw) <= pl->lds_limit / 3) return rtw;
  return 1;
}
bool gt::direct_fwd_ok(const gt_plan *pl, int t) {
  return !pl->ragged && pl->R <= 16 && t >= 1 && t <= pl->ds && pl->ord[t].term_end > pl->ord[t].term_begin &&
         direct_fwd_lds(pl, t, 1) <= pl->lds_limit;
}
int gt::direct_adj_rtw(const gt_plan *pl, int t) {
  const int64_t rows = 2 * group_size(pl, t);
  return rows <= 64 ? 1 : rows <= 128 ? 2 : rows <= 256 ? 4 : rows <= 512 ? 8 : 0;
}
bool gt::direct_adj_ok(const gt_plan *pl, int t) {
  if (pl->ragged || pl->R > 16 || t < 1 || t > pl->ds || pl->ord[t].term_end == pl->ord[t].term_begin) return false;
  const size_t K = (size_t)(pl->ord[t].N - 1), G = (size_t)group_size(pl, t);
  const size_t lds = (size_t)(2 * 16 * 65 + 3 * 64) * pl->rsize +
                     (3 * K + 1 + (t >= 2 ? G / K : 0) + (t == 3 ? 2 * K : 0)) * 68 * 2 * pl->rsize;
  return direct_adj_rtw(pl, t) > 0 && lds <= pl->lds_limit;
}

int gt::spread1_copies(const gt_plan *pl) {
  if (pl->ds < 1) return 1;
  return (size_t)kSpreadWaves * pl->ord[1].gsize * 16 <= pl->lds_limit ? kSpreadWaves : 1;
}

bool gt::fused_available(const gt_plan *pl) {
  if (pl->ds != 2 || pl->gitems.empty()) return false;
  const OrderHost &o1 = pl->ord[1], &o2 = pl->ord[2];
  const int nt1 = o1.term_end - o1.term_begin, nt2 = o2.term_end - o2.term_begin;
  if (nt1 == 0 || nt2 == 0 || o1.m != o2.m) return false;
  if (o1.path == GT_GATHER_DIRECT || o2.path == GT_GATHER_DIRECT) return false;
  if (o1.adj_form != GT_ADJ_WINDOW || o2.adj_form != GT_ADJ_WINDOW) return false;
  if (pl->nslots < nt1 + nt2) return false;   // every window term's slot in one block
  // the order-2 fold in its tile-sum form, four wavefronts' tile sums per workgroup, beside
  // the order-1 fold's 4 KiB
  if (o2.P > 2 * o2.n || o2.ntile > 32) return false;
  if (spread1_copies(pl) != kSpreadWaves) return false;   // order 1 in the fixed summation order
  return (size_t)4 * o2.ntile * 64 * 2 * pl->rsize + 4096 + 64 <= pl->lds_limit;
}

int gt::set_adjoint_form(gt_plan *pl, int t, int form) {
  OrderHost &o = pl->ord[t];
  drop_graphs(pl);
  if (form == GT_ADJ_WINDOW) {
    o.adj_form = form;
    return GT_OK;
  }
  if (!direct_adj_ok(pl, t)) return fail(GT_EUNSUPPORTED, "the direct adjoint is not available for this order");
  if (!o.d_dpart) {
    // node slices: about eight rounds of resident workgroups over the order's terms, at least
    // 1024 nodes per slice, partials within 512 MiB
    const int64_t nt = o.term_end - o.term_begin;
    const int64_t rows = 64 * direct_adj_rtw(pl, t);
    const int64_t per_slice = nt * rows * 16 * (int64_t)pl->rsize;
    int64_t S = (8 * 8 * (int64_t)pl->num_cu + nt - 1) / nt;
    S = std::min<int64_t>(S, std::max<int64_t>(1, pl->M / 1024));
    S = std::min<int64_t>(S, std::max<int64_t>(1, (int64_t(512) << 20) / per_slice));
    S = std::max<int64_t>(1, std::min<int64_t>(S, 65535));
    if (int rc = dev_alloc(&o.d_dpart, (size_t)(per_slice * S), nullptr)) return rc;
    o.dir_nslice = (int32_t)S;
  }
  o.adj_form = form;
  return GT_OK;
}

int gt::set_gather_path(gt_plan *pl, int t, int path) {
  OrderHost &o = pl->ord[t];
  drop_graphs(pl);
  if (path == GT_GATHER_SORTED) {
    o.path = path;
    return GT_OK;
  }
  if (path == GT_GATHER_DIRECT) {
    if (!direct_fwd_ok(pl, t)) return fail(GT_EUNSUPPORTED, "the direct forward is not available for this order");
    o.path = path;
    return GT_OK;
  }
  if (int rc = build_cell_items(pl, t, true, nullptr)) return rc;
  if (o.citems.empty()) return fail(GT_EUNSUPPORTED, "no cell items for this order");
  if (path == GT_GATHER_POLY) {
    bool ok = false;
    if (t != 2) return fail(GT_EUNSUPPORTED, "the polynomial gather is for order 2");
    if (int rc = build_poly(pl, &ok)) return rc;
    if (!ok) return fail(GT_EUNSUPPORTED, "the polynomial gather is not available for this plan");
  }
  o.path = path;
  return GT_OK;
}

// Rebuilds the order-2 tile spread's work list for `waves_cu` resident wavefronts per compute
// unit (the tuner's trials).
int gt::set_tile_waves(gt_plan *pl, int waves_cu) {
  OrderHost &o = pl->ord[2];
  if (pl->ds < 2 || o.term_end == o.term_begin) return GT_OK;
  drop_graphs(pl);
  dev_free(o.d_waves2, nullptr);
  dev_free(o.d_tileseg, nullptr);
  dev_free(o.d_patch, nullptr);
  dev_free(o.d_tsum, nullptr);
  o.d_waves2 = o.d_tileseg = nullptr;
  o.d_patch = o.d_tsum = nullptr;
  o.waves_cu = waves_cu;
  if (o.cstart_host.empty())             // (dropped by a node update)
    if (int rc = fetch_cell_starts(pl, 2, pl->stream, o.cstart_host)) return rc;
  return setup_tile_spread(pl, o.cstart_host);
}

namespace {

// Deconvolution factors, roots of unity and window polynomials of an order depend only on
// (N, n, m, polynomial degree) (the shape b follows from N and n); their long-double
// evaluation costs about a millisecond, so plans share them through this process-wide
// cache (bounded; cleared when full).
struct OrderTables {
  std::vector<double> deconv, roots, poly;
};
static std::mutex g_tab_mu;
static std::map<std::array<int, 4>, OrderTables> g_tab;

static bool cached_tables(int N, int n, int m, int D, OrderHost &o) {
  std::lock_guard<std::mutex> lk(g_tab_mu);
  auto it = g_tab.find({N, n, m, D});
  if (it == g_tab.end()) return false;
  o.deconv = it->second.deconv;
  o.roots = it->second.roots;
  o.poly = it->second.poly;
  return true;
}

static void cache_tables(int N, int n, int m, int D, const OrderHost &o) {
  std::lock_guard<std::mutex> lk(g_tab_mu);
  if (g_tab.size() >= 64) g_tab.clear();
  g_tab[{N, n, m, D}] = OrderTables{o.deconv, o.roots, o.poly};
}

int build_plan(const gt_problem *p, const void *x, hipStream_t s, gt_plan **out) {
  *out = nullptr;
  int rc = validate_problem(p);
  if (rc) return rc;
  if (!x) return fail(GT_EINVAL, "node array is NULL");
  gt_plan *pl = new (std::nothrow) gt_plan();
  if (!pl) return fail(GT_ENOMEM, "host allocation");
  pl->prob = *p;
  pl->prob.offsets = nullptr;
  pl->basis = p->basis;
  pl->node_scale = p->basis == GT_BASIS_COS ? 0.5 : 1.0;
  pl->dtype = p->dtype;
  pl->rsize = p->dtype == GT_C64 ? sizeof(float) : sizeof(double);
  pl->d = p->d;
  pl->ds = p->ds;
  pl->R = p->R;
  pl->stream = s;
  if (p->offsets) {
    pl->ragged = true;
    pl->offs.assign(p->offsets, p->offsets + p->R + 1);
    pl->Mtot = pl->offs.back();
    pl->Vtot = pl->Mtot;
    pl->M = 0;
  } else {
    pl->M = p->M;
    pl->Mtot = p->M;
    pl->Vtot = p->M * p->R;
  }
  const double sigma = p->sigma == 0.0 ? 2.0 : p->sigma;
  int dev = 0;
  (void)hipGetDevice(&dev);
  int lds = 65536;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && lds > 0)
    pl->lds_limit = (size_t)lds;
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
    pl->num_cu = ncu;
  // The fork/join events order two streams of this device only, so they skip the
  // system-scope fence (an L2 write-back that would make the data visible to the host):
  // kernels release their results at device scope when they end, which is what the other
  // stream's kernels need.
  constexpr unsigned kSyncEventFlags = hipEventDisableTiming | hipEventDisableSystemFence;
  // side stream for independent per-order kernels (non-blocking, default priority); without
  // it everything runs on the caller's stream
  pl->side = take_side(dev);
  if (!pl->side || hipEventCreateWithFlags(&pl->ev_fork, kSyncEventFlags) != hipSuccess ||
      hipEventCreateWithFlags(&pl->ev_join, kSyncEventFlags) != hipSuccess) {
    (void)hipGetLastError();
    give_side(pl->side);
    if (pl->ev_fork) (void)hipEventDestroy(pl->ev_fork);
    pl->side = nullptr;
    pl->ev_fork = pl->ev_join = nullptr;
  }

  // ---- terms in coefficient order (ci: index in the unmasked enumeration, for the term mask);
  //      coef: offsets of the index set the kernels run on, coef_ext: of the caller's vectors
  int64_t coef = 0, coef_ext = 0, grid = 0, ci = 0;
  for (int t = 0; t <= p->ds; ++t) {
    OrderHost &o = pl->ord[t];
    o.term_begin = (int32_t)pl->terms.size();
    if (t > 0) {
      // the cosine basis runs on the exponential groups of twice the bandwidth (see the
      // cosine kernels), so every grid size and table below is the exponential one's
      o.N = p->N[t - 1] * (p->basis == GT_BASIS_COS ? 2 : 1);
      o.n = 2 * (int)std::ceil(sigma * o.N / 2.0);
      if (o.n < o.N + 2) o.n = o.N + 2;
      o.m = p->m ? p->m : choose_m(p->dtype, (double)o.n / o.N);
      o.P = o.n + 2 * o.m - 1;
      o.gsize = t == 1 ? o.P : (t == 2 ? o.n * o.P : o.n * o.n * o.P);
      o.b = M_PI * (2.0 - (double)o.N / o.n);
    }
    std::vector<int> c(t);
    for (int i = 0; i < t; ++i) c[i] = i;
    int64_t gsz = 1, gsz_ext = 1;
    for (int k = 0; k < t; ++k) {
      gsz *= (o.N - 1);
      gsz_ext *= (p->N[t - 1] - 1);
    }
    while (true) {
      const bool keep = t == 0 || !p->term_mask || p->term_mask[ci];
      ++ci;
      if (keep && (t == 0 || c[t - 1] < p->d)) {
        DevTerm dt{};
        dt.t = t;
        dt.c0 = t > 0 ? c[0] : -1;
        dt.c1 = t > 1 ? c[1] : -1;
        dt.c2 = t > 2 ? c[2] : -1;
        dt.coef_off = coef;
        dt.grid_off = t > 0 ? grid : 0;
        coef += t > 0 ? gsz : 1;
        pl->ext_off.push_back(coef_ext);
        coef_ext += t > 0 ? gsz_ext : 1;
        if (t > 0) grid += o.gsize;
        pl->terms.push_back(dt);
      }
      if (t == 0) break;
      // next combination
      int i = t - 1;
      while (i >= 0 && c[i] == p->d - t + i) --i;
      if (i < 0) break;
      ++c[i];
      for (int k = i + 1; k < t; ++k) c[k] = c[k - 1] + 1;
    }
    o.term_end = (int32_t)pl->terms.size();
  }
  pl->nterms = (int32_t)pl->terms.size();
  pl->ncoef = coef_ext;
  pl->ncoef_int = coef;
  pl->grid_total = grid;

  // ---- per-order tables, LDS checks
  const size_t csz = 2 * pl->rsize;
  for (int t = 1; t <= p->ds; ++t) {
    OrderHost &o = pl->ord[t];
    const int K = o.N - 1;
    size_t lds_gather = (size_t)o.gsize * 16;   // spread accumulates in FP64
    size_t lds_pack = (size_t)csz * (t == 1 ? K : t == 2 ? (size_t)K * K + (size_t)K * o.n
                                                         : (size_t)K * K * K + (size_t)K * K * o.n + (size_t)K * o.n * o.n);
    size_t lds_adj = (size_t)csz * (t == 1 ? o.n : t == 2 ? (size_t)o.n * o.n + (size_t)o.n * K
                                                         : (size_t)o.n * o.n * o.n + (size_t)o.n * o.n * K + (size_t)o.n * K * K);
    lds_pack += 2 * (size_t)o.n * pl->rsize;   // roots of unity staged in LDS
    lds_adj += 2 * (size_t)o.n * pl->rsize;
    size_t need = std::max(lds_gather, std::max(lds_pack, lds_adj));
    if (need > pl->lds_limit) {
      free_plan(pl);
      return fail(GT_EUNSUPPORTED, "grid of order " + std::to_string(t) + " needs " + std::to_string(need) +
                                       " bytes of LDS (limit " + std::to_string(pl->lds_limit) + ")");
    }
    const int D = p->dtype == GT_C64 ? Deg<float>::value : Deg<double>::value;
    if (!cached_tables(o.N, o.n, o.m, D, o)) {
      o.deconv.resize(K);
      for (int a = 0; a < K; ++a) {
        int k = a - o.N / 2 + (a >= o.N / 2 ? 1 : 0);
        long double ph = kb_phihat(k, o.m, (long double)o.b, o.n);
        o.deconv[a] = (double)(((k & 1) ? -1.0L : 1.0L) / ph);
      }
      o.roots.resize(2 * o.n);
      for (int j = 0; j < o.n; ++j) {
        long double a = 2.0L * M_PIl * j / o.n;
        o.roots[2 * j] = (double)std::cos(a);
        o.roots[2 * j + 1] = (double)std::sin(a);
      }
      window_poly(o.m, (long double)o.b, D, o.poly);
      cache_tables(o.N, o.n, o.m, D, o);
    }
    // one table at a time, stopping at the first failure (so the status and message agree)
    int rt = p->dtype == GT_C64 ? upload<float>(o.deconv, &o.d_deconv) : upload<double>(o.deconv, &o.d_deconv);
    if (!rt) rt = p->dtype == GT_C64 ? upload<float>(o.roots, &o.d_roots) : upload<double>(o.roots, &o.d_roots);
    if (!rt) rt = p->dtype == GT_C64 ? upload<float>(o.poly, &o.d_poly) : upload<double>(o.poly, &o.d_poly);
    if (rt) {
      free_plan(pl);
      return rt;
    }
  }

  // ---- gather work items: kGatherBS virtual nodes each, grouped by right-hand side
  auto add_items = [&](std::vector<WorkItem> &items, std::vector<int32_t> &begin, int64_t chunk) {
    items.clear();
    begin.assign(pl->R + 1, 0);
    for (int r = 0; r < pl->R; ++r) {
      begin[r] = (int32_t)items.size();
      int64_t lo = pl->ragged ? pl->offs[r] : 0, hi = pl->ragged ? pl->offs[r + 1] : pl->M;
      int64_t vbase = pl->ragged ? 0 : (int64_t)r * pl->M;
      for (int64_t a = lo; a < hi; a += chunk) {
        WorkItem w{};
        w.v0 = vbase + a;
        w.x0 = a;
        w.count = (int32_t)std::min<int64_t>(chunk, hi - a);
        w.r = r;
        items.push_back(w);
      }
      if (hi == lo) {   // an empty dataset keeps one empty item: its per-side results are still written
        WorkItem w{};
        w.v0 = vbase + lo;
        w.x0 = lo;
        w.count = 0;
        w.r = r;
        items.push_back(w);
      }
    }
    begin[pl->R] = (int32_t)items.size();
  };
  add_items(pl->gitems, pl->gitem_begin, kGatherBS);
  const int64_t ngi = (int64_t)pl->gitems.size();

  // ---- gather work items per order: runs of sorted positions of one term and right-hand
  //      side (the binning sorts each term's nodes by cell, dataset by dataset)
  for (int t = 1; t <= p->ds; ++t) {
    OrderHost &o = pl->ord[t];
    const int nt = o.term_end - o.term_begin;
    const int64_t chunk = (int64_t)kGatherBS * kGatherNodes;
    o.gitems.clear();
    o.gitem_begin.assign(nt + 1, 0);
    for (int tl = 0; tl < nt; ++tl) {
      o.gitem_begin[tl] = (int32_t)o.gitems.size();
      for (int r = 0; r < pl->R; ++r) {
        const int64_t lo = pl->ragged ? pl->offs[r] : 0, hi = pl->ragged ? pl->offs[r + 1] : pl->M;
        for (int64_t a = lo; a < hi; a += chunk) {
          GatherItem gi{};
          gi.q0 = (int64_t)tl * pl->Mtot + a;
          gi.count = (int32_t)std::min<int64_t>(chunk, hi - a);
          gi.tl = tl;
          gi.r = r;
          o.gitems.push_back(gi);
        }
      }
    }
    o.gitem_begin[nt] = (int32_t)o.gitems.size();
  }
  // forward output slots: one per term of a block, about 512 MiB at most
  {
    const int64_t per_slot = std::max<int64_t>(1, pl->Vtot * (int64_t)csz);
    const int64_t cap = std::max<int64_t>(1, (int64_t(512) << 20) / per_slot);
    pl->nslots = (int32_t)std::max<int64_t>(1, std::min<int64_t>(cap, std::max(1, pl->nterms - 1)));
  }

  // ---- spread work items per order: ranges of cells (orders 1, 3) or tiles (order 2) per
  //      right-hand side; partial-grid memory bounded to about 1 GiB
  for (int t = 1; t <= p->ds; ++t) {
    OrderHost &o = pl->ord[t];
    const int64_t nt = o.term_end - o.term_begin;
    int64_t ncell = 1;
    for (int k = 0; k < t; ++k) ncell *= o.n;
    o.ncell = ncell;
    o.ts = t == 2 ? tile_side(o.m) : 1;
    o.ntile = (o.n + o.ts - 1) / o.ts;
    o.nkey = t == 2 ? (int64_t)o.ntile * o.ntile * o.ts * o.ts : ncell;
    const int64_t per_item = std::max<int64_t>(1, nt * o.gsize * (int64_t)csz);
    const int64_t mem_items = std::max<int64_t>(1, ((int64_t(1) << 30) / per_item) / pl->R);
    const int64_t pairs = std::max<int64_t>(1, nt * pl->R);
    int64_t units, chunks;
    if (t == 2) {
      units = 0;   // the tile spread takes its work list from setup_tile_spread
      chunks = 0;
    } else {
      // about 8192 wavefronts in total, at least one cell per wavefront of a workgroup
      units = ncell;
      const int64_t want = std::max<int64_t>(1, (8192 / kSpreadWaves + pairs - 1) / pairs);
      const int64_t cell_cap = std::max<int64_t>(1, ncell / kSpreadWaves);
      chunks = std::max<int64_t>(1, std::min<int64_t>(want, std::min<int64_t>(cell_cap, mem_items)));
    }
    o.sitems.clear();
    o.sitem_begin.assign(pl->R + 1, 0);
    for (int r = 0; r < pl->R; ++r) {
      o.sitem_begin[r] = (int32_t)o.sitems.size();
      for (int64_t ch = 0; ch < chunks; ++ch) {
        SpreadItem si{};
        si.r = r;
        si.b = pl->ragged ? r : 0;
        si.c0 = (int32_t)(units * ch / chunks);
        si.c1 = (int32_t)(units * (ch + 1) / chunks);
        if (si.c1 > si.c0) o.sitems.push_back(si);
      }
    }
    o.sitem_begin[pl->R] = (int32_t)o.sitems.size();
    o.gpart_stride = 0;
    for (int i = o.term_begin; i < o.term_end; ++i) {
      pl->terms[i].gpart_off = o.gpart_stride;
      o.gpart_stride += o.gsize;
    }
  }

  // ---- device memory
  const int64_t nx = (int64_t)pl->d * pl->Mtot;
  if ((rc = upload_raw(pl->terms, &pl->d_terms)) || (rc = dev_alloc(&pl->d_x, (size_t)nx * pl->rsize, s)) ||
      (rc = dev_alloc(&pl->d_grid, (size_t)pl->R * pl->grid_total * csz, s)) ||
      (rc = upload_raw(pl->gitems, &pl->d_gitems)) || (rc = upload_raw(pl->gitem_begin, &pl->d_gitem_begin)) ||
      (rc = dev_alloc(&pl->d_fpart, (size_t)std::max(1, pl->nslots) * pl->Vtot * csz, s)) ||
      (rc = dev_alloc((void **)&pl->d_ysum, (size_t)ngi * 2 * sizeof(double), s)) ||
      (rc = dev_alloc((void **)&pl->d_flag, sizeof(int32_t), s))) {
    free_plan(pl);
    return rc;
  }
  for (int t = 1; t <= p->ds; ++t) {
    OrderHost &o = pl->ord[t];
    if ((rc = upload_raw(o.gitems, &o.d_gitems)) || (rc = upload_raw(o.sitems, &o.d_sitems)) ||
        (rc = upload_raw(o.sitem_begin, &o.d_sitem_begin)) ||
        (rc = dev_alloc(&o.d_gpart, (size_t)o.sitems.size() * o.gpart_stride * csz, s)) ||
        (rc = dev_alloc(&o.d_gsum, t == 2 ? 0 : (size_t)pl->R * (o.term_end - o.term_begin) * (size_t)o.ncell * csz,
                        s))) {
      free_plan(pl);
      return rc;
    }
  }

  // ---- cosine basis: per-term table of the coefficient conversion, exponential coefficients
  if (pl->basis == GT_BASIS_COS) {
    std::vector<CosTerm> ct;
    for (int i = 1; i < pl->nterms; ++i) {
      const DevTerm &dt = pl->terms[i];
      ct.push_back(CosTerm{dt.t, p->N[dt.t - 1], dt.coef_off, pl->ext_off[i]});
    }
    if (ct.empty()) ct.push_back(CosTerm{0, 2, 0, 0});   // (unused; keeps the table non-empty)
    if ((rc = upload_raw(ct, &pl->d_cterms)) ||
        (rc = dev_alloc(&pl->d_gcos, (size_t)pl->R * pl->ncoef_int * csz, s))) {
      free_plan(pl);
      return rc;
    }
  }

  // ---- nodes: wrap, transpose, validate (one synchronisation)
  rc = p->dtype == GT_C64 ? launch_prepare_nodes<float>(pl, x, s) : launch_prepare_nodes<double>(pl, x, s);
  if (rc) {
    free_plan(pl);
    return rc;
  }
  int32_t flag = 0;
  hipError_t e = hipMemcpyAsync(&flag, pl->d_flag, sizeof(flag), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    free_plan(pl);
    return hip_fail(e, "node validation");
  }
  if (flag) {
    free_plan(pl);
    return fail(GT_EINVAL, "nodes contain NaN or Inf");
  }
  // ---- node binning for the spread (per term, by cell)
  rc = p->dtype == GT_C64 ? launch_binning<float>(pl, s) : launch_binning<double>(pl, s);
  if (rc == GT_OK) {
    hipError_t e2 = hipStreamSynchronize(s);
    if (e2 != hipSuccess) rc = hip_fail(e2, "node binning");
  }
  for (int t = 1; rc == GT_OK && t <= p->ds; ++t)
    if (pl->ord[t].term_end > pl->ord[t].term_begin) rc = fetch_cell_starts(pl, t, s, pl->ord[t].cstart_host);
  if (rc == GT_OK && p->ds >= 2 && pl->ord[2].term_end > pl->ord[2].term_begin)
    rc = setup_tile_spread(pl, pl->ord[2].cstart_host);
  if (rc == GT_OK && p->ds >= 1) rc = setup_cell_gather(pl);
  if (rc == GT_OK) rc = apply_cached_tuning(pl);
  if (rc) {
    free_plan(pl);
    return rc;
  }
  plan_register(pl);
  *out = pl;
  return GT_OK;
}

// Plans made and released inside one call (the one-shot entry points) are never exposed.
static void release_plan(gt_plan *pl) {
  if (pl && plan_unregister(pl)) free_plan(pl);
}

}  // namespace

// ------------------------------------------------------------------ C ABI
extern "C" {

const char *gt_version(void) { return "grouped-nfft-gfx950 1.0"; }

const char *gt_last_error(void) { return g_last_error.c_str(); }

int gt_prof_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on != 0;
  return GT_OK;
}

int64_t gt_prof_report(char *buf, int64_t len) {
  std::vector<ProfRec> recs;
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    recs.swap(g_prof);
  }
  std::vector<std::pair<std::string, std::pair<int64_t, double>>> agg;
  for (auto &r : recs) {
    float ms = 0;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      auto it = std::find_if(agg.begin(), agg.end(), [&](auto &a) { return a.first == r.name; });
      if (it == agg.end()) {
        agg.push_back({r.name, {1, (double)ms}});
      } else {
        it->second.first += 1;
        it->second.second += ms;
      }
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  std::string js = "{";
  for (size_t i = 0; i < agg.size(); ++i) {
    char tmp[256];
    snprintf(tmp, sizeof(tmp), "%s\"%s\": [%lld, %.6f]", i ? ", " : "", agg[i].first.c_str(),
             (long long)agg[i].second.first, agg[i].second.second);
    js += tmp;
  }
  js += "}";
  if (buf && len > 0) {
    size_t nc = std::min<size_t>((size_t)len - 1, js.size());
    memcpy(buf, js.data(), nc);
    buf[nc] = 0;
  }
  return (int64_t)js.size() + 1;
}

int64_t gt_num_terms(int32_t d, int32_t ds) {
  if (d < 1 || ds < 0 || ds > d) return -1;
  int64_t s = 0;
  for (int t = 0; t <= ds; ++t) s += binom(d, t);
  return s;
}

int64_t gt_num_coeffs(int32_t d, int32_t ds, const int32_t *N) {
  if (d < 1 || ds < 0 || ds > d || (ds > 0 && !N)) return -1;
  int64_t s = 1;
  for (int t = 1; t <= ds; ++t) {
    if (N[t - 1] < 2 || N[t - 1] % 2) return -1;
    int64_t g = 1;
    for (int i = 0; i < t; ++i) g *= (N[t - 1] - 1);
    s += binom(d, t) * g;
  }
  return s;
}

int gt_term_table(const gt_problem *p, int32_t *coords, int64_t *offsets) {
  if (!p) return fail(GT_EINVAL, "problem is NULL");
  if (p->d < 1 || p->ds < 0 || p->ds > p->d) return fail(GT_EINVAL, "need d >= 1 and 0 <= ds <= d");
  if (p->ds > kMaxOrder) return fail(GT_EUNSUPPORTED, "terms of order > 3 are not implemented");
  for (int t = 1; t <= p->ds; ++t)
    if (p->N[t - 1] < 2 || p->N[t - 1] % 2) return fail(GT_EINVAL, "bandwidths must be even and >= 2");
  int64_t i = 0, off = 0;
  for_each_term(p->d, p->ds, [&](int64_t ci, int t, const int *c) {
    if (t > 0 && p->term_mask && !p->term_mask[ci]) return;
    int64_t g = 1;
    for (int k = 0; k < t; ++k) g *= (p->N[t - 1] - 1);
    if (coords)
      for (int k = 0; k < 3; ++k) coords[i * 3 + k] = k < t ? c[k] : -1;
    if (offsets) offsets[i] = off;
    off += g;
    ++i;
  });
  if (offsets) offsets[i] = off;
  return GT_OK;
}

int gt_problem_size(const gt_problem *p, int64_t *nterms, int64_t *ncoeffs) {
  if (!p) return fail(GT_EINVAL, "problem is NULL");
  if (p->d < 1 || p->ds < 0 || p->ds > p->d) return fail(GT_EINVAL, "need d >= 1 and 0 <= ds <= d");
  if (p->ds > kMaxOrder) return fail(GT_EUNSUPPORTED, "terms of order > 3 are not implemented");
  for (int t = 1; t <= p->ds; ++t)
    if (p->N[t - 1] < 2 || p->N[t - 1] % 2) return fail(GT_EINVAL, "bandwidths must be even and >= 2");
  int64_t nu = 0, ni = 0;
  for_each_term(p->d, p->ds, [&](int64_t ci, int t, const int *) {
    if (t > 0 && p->term_mask && !p->term_mask[ci]) return;
    int64_t g = 1;
    for (int k = 0; k < t; ++k) g *= (p->N[t - 1] - 1);
    ++nu;
    ni += g;
  });
  if (nterms) *nterms = nu;
  if (ncoeffs) *ncoeffs = ni;
  return GT_OK;
}

int gt_active_set(const gt_problem *p, const double *rho, const double *eps, uint8_t *mask, int64_t *nactive) {
  if (!rho || !mask || (!eps && p && p->ds > 0)) return fail(GT_EINVAL, "NULL argument");
  int64_t nu = 0;
  if (int rc = gt_problem_size(p, &nu, nullptr)) return rc;
  int64_t k = 0, na = 0;   // k: index among the problem's terms (rho's index)
  for_each_term(p->d, p->ds, [&](int64_t ci, int t, const int *) {
    const bool kept = t == 0 || !p->term_mask || p->term_mask[ci];
    bool act = false;
    if (kept) {
      act = t == 0 || rho[k] > eps[t - 1];
      ++k;
    }
    mask[ci] = act ? 1 : 0;
    na += act;
  });
  if (nactive) *nactive = na;
  return GT_OK;
}

int gt_sensitivity(const gt_problem *p, const void *fhat, double *rho, void *stream) {
  if (!fhat || !rho) return fail(GT_EINVAL, "NULL argument");
  if (int rc = validate_problem(p)) return rc;
  int64_t nu = 0;
  if (int rc = gt_problem_size(p, &nu, nullptr)) return rc;
  std::vector<int64_t> offs(nu + 1);
  if (int rc = gt_term_table(p, nullptr, offs.data())) return rc;
  const hipStream_t s = (hipStream_t)stream;
  int64_t *d_offs = nullptr;
  if (int rc = dev_alloc((void **)&d_offs, offs.size() * sizeof(int64_t), s)) return rc;
  hipError_t e = hipMemcpyAsync(d_offs, offs.data(), offs.size() * sizeof(int64_t), hipMemcpyHostToDevice, s);
  int rc = e == hipSuccess ? GT_OK : hip_fail(e, "term offsets");
  if (rc == GT_OK)
    rc = p->dtype == GT_C64 ? run_sensitivity<float>(d_offs, (int)nu, offs[nu], p->R, fhat, rho, s)
                            : run_sensitivity<double>(d_offs, (int)nu, offs[nu], p->R, fhat, rho, s);
  e = hipStreamSynchronize(s);
  if (rc == GT_OK && e != hipSuccess) rc = hip_fail(e, "sensitivity indices");
  dev_free(d_offs, s);
  return rc;
}

int gt_plan_create(const gt_problem *p, const void *x, void *stream, gt_plan **out) {
  if (!out) return fail(GT_EINVAL, "out is NULL");
  return build_plan(p, x, (hipStream_t)stream, out);
}

int gt_plan_destroy(gt_plan *plan) {
  if (!plan) return GT_OK;
  if (!plan_unregister(plan)) return fail(GT_EINVAL, "not a live plan (destroyed or released)");
  free_plan(plan);
  return GT_OK;
}

int gt_release_all(void) {
  std::vector<gt_plan *> all;
  {
    std::lock_guard<std::mutex> lk(g_plans_mu);
    all.swap(g_plans);
  }
  for (gt_plan *pl : all) free_plan(pl);
  drain_side_pool();
  {
    std::lock_guard<std::mutex> lk(g_tab_mu);
    g_tab.clear();
  }
  clear_tuning_cache();
  return GT_OK;
}

int gt_debug_fail_alloc(int64_t k) {
  if (k < 0) return fail(GT_EINVAL, "k must be >= 0");
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_alloc_fail_at = k;
  g_alloc_count = 0;
  return GT_OK;
}

int64_t gt_debug_alloc_count(void) {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  return g_alloc_count;
}

#define GT_LIVE(plan)                                                                 \
  do {                                                                                \
    if (!plan_is_live(plan)) return fail(GT_EINVAL, "not a live plan (destroyed or released)"); \
  } while (0)

int gt_plan_order_info(const gt_plan *plan, int32_t t, int32_t *m, int32_t *n) {
  GT_LIVE(plan);
  if (t < 1 || t > plan->ds) return fail(GT_EINVAL, "no such order in plan");
  if (m) *m = plan->ord[t].m;
  if (n) *n = plan->ord[t].n;
  return GT_OK;
}

int gt_plan_gather_path(const gt_plan *plan, int32_t t, int32_t *path) {
  GT_LIVE(plan);
  if (t < 1 || t > plan->ds) return fail(GT_EINVAL, "no such order in plan");
  const OrderHost &o = plan->ord[t];
  if (path) *path = o.path;
  return GT_OK;
}

int gt_plan_trafo(gt_plan *plan, const void *fhat, void *f, void *stream) {
  GT_LIVE(plan);
  if (!fhat || !f) return fail(GT_EINVAL, "NULL argument");
  plan->stream = (hipStream_t)stream;
  return run_plan_call(plan, 0, fhat, f, (hipStream_t)stream);
}

int gt_plan_adjoint(gt_plan *plan, const void *y, void *fhat, void *stream) {
  GT_LIVE(plan);
  if (!fhat || !y) return fail(GT_EINVAL, "NULL argument");
  plan->stream = (hipStream_t)stream;
  return run_plan_call(plan, 1, y, fhat, (hipStream_t)stream);
}

int gt_plan_update_nodes(gt_plan *plan, const void *x, void *stream) {
  GT_LIVE(plan);
  if (!x) return fail(GT_EINVAL, "NULL argument");
  const hipStream_t s = (hipStream_t)stream;
  plan->stream = s;
  drop_graphs(plan);
  const size_t csz = 2 * plan->rsize;
  // forward forms whose work items follow the node positions on the host take the sorted gather
  for (int t = 1; t <= plan->ds; ++t) {
    OrderHost &o = plan->ord[t];
    o.cstart_host.clear();
    if (o.path == GT_GATHER_CELL || o.path == GT_GATHER_POLY) o.path = GT_GATHER_SORTED;
    if (o.d_citems || o.d_kpoly) {
      GT_HIP(hipStreamSynchronize(s));
      dev_free(o.d_citems, nullptr);
      dev_free(o.d_kpoly, nullptr);
      o.d_citems = nullptr;
      o.d_kpoly = nullptr;
      o.citems.clear();
      o.citem_begin.clear();
    }
  }
  // order-2 tile spread: patches for the most segments any node positions can give
  OrderHost &o2 = plan->ord[2];
  if (plan->ds >= 2 && o2.term_end > o2.term_begin && o2.nwaves2 > 0) {
    const int B = plan->ragged ? plan->R : 1;
    const int64_t bound = (int64_t)o2.nwaves2 + (int64_t)(o2.term_end - o2.term_begin) * B * o2.ntile * o2.ntile;
    if (bound >= (int64_t(1) << 31) / 256) return fail(GT_EUNSUPPORTED, "too many tile patches");
    const int reff = plan->ragged ? 1 : plan->R;
    if (bound > o2.nseg2) {
      GT_HIP(hipStreamSynchronize(s));
      dev_free(o2.d_patch, nullptr);
      o2.d_patch = nullptr;
      if (int rc = dev_alloc(&o2.d_patch, (size_t)reff * bound * 256 * csz, nullptr)) return rc;
      o2.nseg2 = bound;
    }
    if (plan->rebin.segcnt_cap < o2.nwaves2) {
      GT_HIP(hipStreamSynchronize(s));
      dev_free(plan->rebin.segcnt, nullptr);
      plan->rebin.segcnt = nullptr;
      plan->rebin.segcnt_cap = 0;
      if (int rc = dev_alloc((void **)&plan->rebin.segcnt, (size_t)o2.nwaves2 * sizeof(int32_t), nullptr)) return rc;
      plan->rebin.segcnt_cap = o2.nwaves2;
    }
  }
  // nodes: wrap, transpose, validate (one synchronisation), then the binning on the device
  int rc = plan->dtype == GT_C64 ? launch_prepare_nodes<float>(plan, x, s) : launch_prepare_nodes<double>(plan, x, s);
  if (rc) return rc;
  int32_t flag = 0;
  GT_HIP(hipMemcpyAsync(&flag, plan->d_flag, sizeof(flag), hipMemcpyDeviceToHost, s));
  GT_HIP(hipStreamSynchronize(s));
  if (flag) return fail(GT_EINVAL, "nodes contain NaN or Inf (the plan's nodes are now undefined)");
  rc = plan->dtype == GT_C64 ? launch_rebin<float>(plan, s) : launch_rebin<double>(plan, s);
  if (rc == GT_OK) rc = launch_tile_relist(plan, s);
  if (rc == GT_OK) ++plan->node_version;
  return rc;
}

int gt_plan_tune(gt_plan *plan, void *stream) {
  GT_LIVE(plan);
  plan->stream = (hipStream_t)stream;
  return tune_plan(plan, (hipStream_t)stream);
}

int64_t gt_plan_tuning(const gt_plan *plan, char *buf, int64_t len) {
  if (!plan_is_live(plan)) return fail(GT_EINVAL, "not a live plan (destroyed or released)");
  const std::string &js = plan->tuning.empty() ? std::string("{}") : plan->tuning;
  if (buf && len > 0) {
    const size_t nc = std::min<size_t>((size_t)len - 1, js.size());
    memcpy(buf, js.data(), nc);
    buf[nc] = 0;
  }
  return (int64_t)js.size() + 1;
}

int gt_plan_set_graph(gt_plan *plan, int32_t on) {
  GT_LIVE(plan);
  if (plan->stream) {
    hipError_t e = hipStreamSynchronize(plan->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  }
  drop_graphs(plan);
  plan->use_graph = on != 0;
  return GT_OK;
}

int gt_plan_set_fused(gt_plan *plan, int32_t on) {
  GT_LIVE(plan);
  if (on && !gt::fused_available(plan))
    return fail(GT_EUNSUPPORTED, "shared launches need orders 1 and 2 only, window forms and one window width");
  if (plan->stream) {
    hipError_t e = hipStreamSynchronize(plan->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  }
  drop_graphs(plan);
  plan->use_fused = on != 0;
  return GT_OK;
}

int gt_plan_adjoint_form(const gt_plan *plan, int32_t t, int32_t *form) {
  GT_LIVE(plan);
  if (t < 1 || t > plan->ds) return fail(GT_EINVAL, "no such order in plan");
  if (form) *form = plan->ord[t].adj_form;
  return GT_OK;
}

int gt_plan_set_adjoint_form(gt_plan *plan, int32_t t, int32_t form) {
  GT_LIVE(plan);
  if (t < 1 || t > plan->ds) return fail(GT_EINVAL, "no such order in plan");
  if (form != GT_ADJ_WINDOW && form != GT_ADJ_DIRECT) return fail(GT_EINVAL, "unknown adjoint form");
  if (plan->ord[t].term_end == plan->ord[t].term_begin) return fail(GT_EINVAL, "the order has no terms");
  if (plan->stream) {
    hipError_t e = hipStreamSynchronize(plan->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  }
  return set_adjoint_form(plan, t, form);
}

int gt_plan_set_gather_path(gt_plan *plan, int32_t t, int32_t path) {
  GT_LIVE(plan);
  if (t < 1 || t > plan->ds) return fail(GT_EINVAL, "no such order in plan");
  if (path < GT_GATHER_SORTED || path > GT_GATHER_DIRECT) return fail(GT_EINVAL, "unknown gather form");
  if (plan->ord[t].term_end == plan->ord[t].term_begin) return fail(GT_EINVAL, "the order has no terms");
  if (plan->stream) {
    hipError_t e = hipStreamSynchronize(plan->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  }
  return set_gather_path(plan, t, path);
}

int gt_plan_node_grad(gt_plan *plan, const void *fhat, const void *g, void *gx, void *stream) {
  GT_LIVE(plan);
  if (!fhat || !g || !gx) return fail(GT_EINVAL, "NULL argument");
  plan->stream = (hipStream_t)stream;
  return plan->dtype == GT_C64 ? launch_node_grad<float>(plan, fhat, g, gx, (hipStream_t)stream)
                               : launch_node_grad<double>(plan, fhat, g, gx, (hipStream_t)stream);
}

int gt_plan_norm_estimate(gt_plan *plan, int32_t iters, double *out, void *stream) {
  GT_LIVE(plan);
  if (!out || iters < 1) return fail(GT_EINVAL, "invalid argument");
  plan->stream = (hipStream_t)stream;
  return plan->dtype == GT_C64 ? run_norm_estimate<float>(plan, iters, out, (hipStream_t)stream)
                               : run_norm_estimate<double>(plan, iters, out, (hipStream_t)stream);
}

int gt_plan_norm_estimate_noalloc(gt_plan *plan, int32_t iters, double *out, void *stream) {
  GT_LIVE(plan);
  if (!out || iters < 1) return fail(GT_EINVAL, "invalid argument");
  plan->stream = (hipStream_t)stream;
  return run_norm_estimate_noalloc(plan, iters, out, (hipStream_t)stream);
}

int grouped_trafo(const gt_problem *p, const void *x, const void *fhat, void *f, void *stream) {
  gt_plan *pl = nullptr;
  int rc = build_plan(p, x, (hipStream_t)stream, &pl);
  if (rc) return rc;
  rc = gt_plan_trafo(pl, fhat, f, stream);
  release_plan(pl);
  return rc;
}

int grouped_adjoint(const gt_problem *p, const void *x, const void *y, void *fhat, void *stream) {
  gt_plan *pl = nullptr;
  int rc = build_plan(p, x, (hipStream_t)stream, &pl);
  if (rc) return rc;
  rc = gt_plan_adjoint(pl, y, fhat, stream);
  release_plan(pl);
  return rc;
}

static int check_lambda(int R, const double *lambda, bool positive) {
  for (int r = 0; r < R; ++r) {
    const double l = lambda[r];
    if (!std::isfinite(l) || (positive ? !(l > 0.0) : !(l >= 0.0)))
      return fail(GT_EINVAL, positive ? "lambda must be finite and > 0" : "lambda must be finite and >= 0");
  }
  return GT_OK;
}

int gt_plan_lsqr(gt_plan *plan, const void *y, const double *lambda, const double *omega, int32_t max_iter,
                 double tol, void *fhat, gt_solve_info *info, void *stream) {
  GT_LIVE(plan);
  if (!y || !lambda || !fhat || !info) return fail(GT_EINVAL, "NULL argument");
  if (max_iter < 1) return fail(GT_EINVAL, "max_iter must be >= 1");
  if (int rc = check_lambda(plan->R, lambda, false)) return rc;
  plan->stream = (hipStream_t)stream;
  return plan->dtype == GT_C64
             ? run_lsqr<float>(plan, y, lambda, omega, max_iter, tol, fhat, info, (hipStream_t)stream)
             : run_lsqr<double>(plan, y, lambda, omega, max_iter, tol, fhat, info, (hipStream_t)stream);
}

int gt_plan_fista(gt_plan *plan, const void *y, const double *lambda, const double *omega, int32_t max_iter,
                  double L, double eta, double tol, void *fhat, gt_solve_info *info, void *stream) {
  GT_LIVE(plan);
  if (!y || !lambda || !fhat || !info) return fail(GT_EINVAL, "NULL argument");
  if (max_iter < 1) return fail(GT_EINVAL, "max_iter must be >= 1");
  if (!std::isfinite(L) || !std::isfinite(eta)) return fail(GT_EINVAL, "L and eta must be finite");
  if (int rc = check_lambda(plan->R, lambda, true)) return rc;
  plan->stream = (hipStream_t)stream;
  return plan->dtype == GT_C64
             ? run_fista<float>(plan, y, lambda, omega, max_iter, L, eta, tol, fhat, info, (hipStream_t)stream)
             : run_fista<double>(plan, y, lambda, omega, max_iter, L, eta, tol, fhat, info, (hipStream_t)stream);
}

int lsqr_solve(const gt_problem *p, const void *x, const void *y, const double *lambda, const double *omega,
               int32_t max_iter, double tol, void *fhat, gt_solve_info *info, void *stream) {
  if (!y || !lambda || !fhat || !info) return fail(GT_EINVAL, "NULL argument");
  if (max_iter < 1) return fail(GT_EINVAL, "max_iter must be >= 1");
  if (p && p->R >= 1)
    if (int rc = check_lambda(p->R, lambda, false)) return rc;
  gt_plan *pl = nullptr;
  int rc = build_plan(p, x, (hipStream_t)stream, &pl);
  if (rc) return rc;
  rc = gt_plan_lsqr(pl, y, lambda, omega, max_iter, tol, fhat, info, stream);
  release_plan(pl);
  return rc;
}

int fista_group_lasso(const gt_problem *p, const void *x, const void *y, const double *lambda, const double *omega,
                      int32_t max_iter, double L, double eta, double tol, void *fhat, gt_solve_info *info,
                      void *stream) {
  if (!y || !lambda || !fhat || !info) return fail(GT_EINVAL, "NULL argument");
  if (max_iter < 1) return fail(GT_EINVAL, "max_iter must be >= 1");
  if (!std::isfinite(L) || !std::isfinite(eta)) return fail(GT_EINVAL, "L and eta must be finite");
  if (p && p->R >= 1)
    if (int rc = check_lambda(p->R, lambda, true)) return rc;
  gt_plan *pl = nullptr;
  int rc = build_plan(p, x, (hipStream_t)stream, &pl);
  if (rc) return rc;
  rc = gt_plan_fista(pl, y, lambda, omega, max_iter, L, eta, tol, fhat, info, stream);
  release_plan(pl);
  return rc;
}

int gt_plan_lsqr_path(gt_plan *plan, const void *y, int32_t nlambda, const double *lambda, const double *omega,
                      int32_t max_iter, double tol, void *fhat_path, gt_solve_info *info, void *stream) {
  GT_LIVE(plan);
  if (!y || !lambda || !fhat_path || !info) return fail(GT_EINVAL, "NULL argument");
  if (nlambda < 1) return fail(GT_EINVAL, "nlambda must be >= 1");
  if (max_iter < 1) return fail(GT_EINVAL, "max_iter must be >= 1");
  if (int rc = check_lambda(nlambda, lambda, false)) return rc;
  plan->stream = (hipStream_t)stream;
  return plan->dtype == GT_C64
             ? run_lsqr_path<float>(plan, y, nlambda, lambda, omega, max_iter, tol, fhat_path, info, (hipStream_t)stream)
             : run_lsqr_path<double>(plan, y, nlambda, lambda, omega, max_iter, tol, fhat_path, info,
                                     (hipStream_t)stream);
}

int lsqr_solve_path(const gt_problem *p, const void *x, const void *y, int32_t nlambda, const double *lambda,
                    const double *omega, int32_t max_iter, double tol, void *fhat_path, gt_solve_info *info,
                    void *stream) {
  if (!y || !lambda || !fhat_path || !info) return fail(GT_EINVAL, "NULL argument");
  if (nlambda < 1) return fail(GT_EINVAL, "nlambda must be >= 1");
  if (max_iter < 1) return fail(GT_EINVAL, "max_iter must be >= 1");
  if (int rc = check_lambda(nlambda, lambda, false)) return rc;
  gt_plan *pl = nullptr;
  int rc = build_plan(p, x, (hipStream_t)stream, &pl);
  if (rc) return rc;
  rc = gt_plan_lsqr_path(pl, y, nlambda, lambda, omega, max_iter, tol, fhat_path, info, stream);
  release_plan(pl);
  return rc;
}

int fista_group_lasso_path(const gt_problem *p, const void *x, const void *y, int32_t nlambda, const double *lambda,
                           const double *omega, int32_t max_iter, double L, double eta, double tol,
                           const void *fhat0, void *fhat_path, gt_solve_info *info, void *stream) {
  if (!y || !lambda || !fhat_path || !info) return fail(GT_EINVAL, "NULL argument");
  if (nlambda < 1) return fail(GT_EINVAL, "nlambda must be >= 1");
  if (max_iter < 1) return fail(GT_EINVAL, "max_iter must be >= 1");
  if (!std::isfinite(L) || !std::isfinite(eta)) return fail(GT_EINVAL, "L and eta must be finite");
  if (int rc = check_lambda(nlambda, lambda, true)) return rc;
  gt_plan *pl = nullptr;
  int rc = build_plan(p, x, (hipStream_t)stream, &pl);
  if (rc) return rc;
  pl->stream = (hipStream_t)stream;
  rc = pl->dtype == GT_C64
           ? run_fista_path<float>(pl, y, nlambda, lambda, omega, max_iter, L, eta, tol, fhat0, fhat_path, info,
                                   (hipStream_t)stream)
           : run_fista_path<double>(pl, y, nlambda, lambda, omega, max_iter, L, eta, tol, fhat0, fhat_path, info,
                                    (hipStream_t)stream);
  release_plan(pl);
  return rc;
}

}  // extern "C"
