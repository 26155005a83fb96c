// Internal declarations of the grouped Fourier transform library (not part of the ABI).
//
// Data layout in HBM (per plan):
//   xT     d x Mtot real       nodes wrapped into [-1/2, 1/2), coordinate-major so that a
//                              wavefront reads one coordinate of 64 consecutive nodes coalesced
//   grids  R x grid_total      forward FFT grids of all terms, complex; a term of order t with
//                              grid size n and window half-width m occupies
//                              t=1: [P], t=2: [n][P], t=3: [n][n][P] with P = n + 2m - 1:
//                              the innermost axis carries a periodic halo so that a window of
//                              2m points never wraps there; outer axes wrap by index
//   gpart  per order: items x (sum of that order's term grid sizes)   adjoint partial grids,
//                              one region per node chunk (spread work item)
//   fpart  blocks x Vtot       forward partial sums per term block (Vtot = R*M or sum M_b)
//
// "Virtual node" v runs over Vtot = R * M (right-hand side r = v / M on node v % M) or over
// the concatenated ragged datasets; f, y and fpart are indexed by v.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/grouped.h"

namespace gt {

constexpr int kMaxOrder = 3;
constexpr int kMinM = 2;
constexpr int kMaxM = 8;
constexpr int kGatherBS = 256;    // threads per gather workgroup
constexpr int kGatherNodes = 4;   // sorted nodes per gather thread
constexpr int kSpreadWaves = 8;   // wavefronts per spread workgroup
constexpr int kTileBatch = 32;    // nodes per batch of the order-2 tile spread
constexpr int kTileWaves = 4;     // wavefronts per workgroup of the order-2 tile spread
constexpr int kTileWavesPerCU = 20;   // order-2 tile spread: at most this many wavefronts per compute unit
constexpr int kTileRow = 17;      // padded staging row (elements) of the order-2 tile spread
constexpr double kCellGatherFill = 0.6;   // smallest lane fill of the cell gather's work items
constexpr size_t kPolyMaxBytes = size_t(1) << 30;   // largest coefficient buffer of the order-2 polynomial gather
constexpr int kPolyRows = 3;       // cell rows per workgroup of k_pack_poly2

// Order-2 spread tiles: TS x TS grid cells whose nodes' windows all fall into one 16 x 16
// patch (TS + 2m - 1 = 16).
constexpr int tile_side(int m) { return 17 - 2 * m; }
constexpr int kPackBS = 512;   // threads of the pack and adjoint-DFT workgroups
constexpr int kVecBS = 256;

// Block coordinates of a kernel body: the grid's when the body runs as its own kernel, or
// the part's own numbering inside a launch that runs several bodies side by side.
struct Blk {
  int x, y;
};

template <typename T> struct Deg;                   // window polynomial degree per precision
template <> struct Deg<float> { static constexpr int value = 7; };
template <> struct Deg<double> { static constexpr int value = 14; };

// LDS of one wavefront of the order-2 tile spread (reals of `rsize` bytes): the window rows of
// a batch along both axes (kTileBatch x kTileRow each), the batch's samples and, in FP64, the
// window polynomial coefficients of points 0..m-1 (at most kMaxM x 15 values, more than the
// scalar registers hold).
constexpr size_t tile_lds_wave(size_t rsize) {
  return ((size_t)2 * kTileBatch * kTileRow + (size_t)2 * kTileBatch +
          (rsize == sizeof(double) ? (size_t)kMaxM * (Deg<double>::value + 1) : 0)) *
         rsize;
}

template <typename T> struct Cx;
template <> struct Cx<float> { using type = float2; };
template <> struct Cx<double> { using type = double2; };
template <typename T> using cx_t = typename Cx<T>::type;

struct DevTerm {
  int32_t t, c0, c1, c2;
  int64_t coef_off;    // offset of the group in the coefficient vector
  int64_t grid_off;    // offset of the term's grid inside one right-hand side's grid block
  int64_t gpart_off;   // offset inside one spread item's partial-grid block of its order
};

struct GatherItem {    // a run of sorted positions of one term and right-hand side
  int64_t q0;          // first position in the order's perm array
  int32_t count;
  int32_t tl;          // term index within the order
  int32_t r;           // right-hand side (dataset when ragged)
  int32_t pad;
};

struct CellItem {       // up to 64 sorted positions of one grid cell of one term (and dataset)
  int32_t q0;          // first position in the order's perm array
  int32_t count;       // 1..64
  int32_t tl;          // term index within the order
  int32_t r;           // dataset when ragged, else 0 (the launch adds the right-hand side)
  int32_t cell[3];     // the cell's grid indices along the term's axes (unused axes 0)
  int32_t pad;
};

struct SpreadItem {    // a range of grid cells of one right-hand side (dataset b of the binning)
  int32_t r, b, c0, c1;
};

struct WorkItem {      // a contiguous run of virtual nodes of one right-hand side
  int64_t v0;          // first virtual node
  int64_t x0;          // node index of v0 in xT
  int32_t count;
  int32_t r;
};

template <typename T> struct OrderParams {
  int32_t N, n, P, m, gsize, nfreq;   // nfreq = N - 1
  int32_t term_begin, term_end;
  const T *deconv;   // nfreq: (-1)^k / Phi_hat(k) for k = -N/2..-1, 1..N/2-1
  const T *roots;    // 2n: cos, sin of 2 pi j / n
  const T *poly;     // 2m x (Deg+1): window polynomial per window point, monomial in z
};

struct OrderHost {
  int32_t N = 0, n = 0, P = 0, m = 0, gsize = 0;
  int32_t term_begin = 0, term_end = 0;
  double b = 0;                       // Kaiser-Bessel shape parameter
  std::vector<double> deconv, roots, poly;
  void *d_deconv = nullptr, *d_roots = nullptr, *d_poly = nullptr;
  // gather work items of this order (runs of sorted nodes), grouped by term
  std::vector<struct GatherItem> gitems;
  struct GatherItem *d_gitems = nullptr;
  std::vector<int32_t> gitem_begin;   // per term of the order, +1
  int32_t path = GT_GATHER_SORTED;    // forward form of this order (GT_GATHER_*)
  int32_t adj_form = GT_ADJ_WINDOW;   // adjoint form of this order (GT_ADJ_*)
  int32_t dir_nslice = 0;             // GT_ADJ_DIRECT: node slices of the adjoint's direct sums
  void *d_dpart = nullptr;            // GT_ADJ_DIRECT: slice partials, terms x slices x 64 rtw x 16 reals
  int32_t waves_cu = kTileWavesPerCU; // order 2: resident wavefronts per compute unit of the tile spread
  std::vector<int64_t> cstart_host;   // the binning's cell starts (host copy, for work lists and the tuner)
  std::vector<CellItem> citems;       // cell gather work items (empty: k_gather_sorted is used)
  CellItem *d_citems = nullptr;
  void *d_kpoly = nullptr;            // order 2 FP32: per-cell window-polynomial coefficients of the grids (k_pack_poly2)
  std::vector<int32_t> citem_begin;   // per term of the order, +1
  // node binning of this order (per term, by cell) and spread work items
  int64_t ncell = 0;                  // n^order
  int32_t ts = 1;                     // cells per tile side of the binning order (order 2: tile_side(m))
  int32_t ntile = 0;                  // tiles per axis, ceil(n / ts)
  int64_t nkey = 0;                   // binning keys per (term, dataset): ntile^order * ts^order
  int32_t *d_perm = nullptr;          // terms x Mtot sorted node indices
  void *d_xs = nullptr;               // order 2: terms x Mtot x 2 coordinates of the term's axes, sorted order
  // order 2 tile spread: wavefront work list and tile patches (built after the binning)
  int32_t nwaves2 = 0;                // wavefronts (per right-hand side when nodes are shared)
  int32_t tile_wg_cu = 1;             // workgroups of the tile spread resident per compute unit
  int64_t nseg2 = 0;                  // (wavefront, tile) segments = patches per right-hand side
  int32_t *d_waves2 = nullptr;        // nwaves2 x 4: first position, end position, first segment, dataset
  int32_t *d_tileseg = nullptr;       // (terms x datasets x ntile^2) + 1: first segment of each tile
  void *d_patch = nullptr;            // (R or 1) x nseg2 x 16 x 16 complex
  void *d_tsum = nullptr;             // R x terms x ntile x 16 x n complex: patches folded along columns
  int64_t *d_cstart = nullptr;        // (terms x datasets x nkey) + 1 start positions
  std::vector<SpreadItem> sitems;
  SpreadItem *d_sitems = nullptr;
  std::vector<int32_t> sitem_begin;   // per right-hand side, R+1
  int32_t *d_sitem_begin = nullptr;
  int64_t gpart_stride = 0;           // complex elements per spread item
  void *d_gpart = nullptr;
  void *d_gsum = nullptr;             // folded spread grids: R x terms x n^order
};

// LDS bytes of k_pack_poly2 (order 2, FP32), all complex: first-pass array H (HR x n x (NQ + 1)),
// grid rows (HR x P), deconvolved coefficients (K x K), first DFT stage (K x n) and the DFT
// factors (K x n); HR = kPolyRows + 2m - 1, NQ = Deg<float> + 1, K = N - 1.
inline size_t poly_pack_lds(const OrderHost &o) {
  const size_t HR = (size_t)(kPolyRows + 2 * o.m - 1), NQ = Deg<float>::value + 1, K = (size_t)(o.N - 1);
  return (HR * o.n * (NQ + 1) + HR * o.P + K * K + 2 * K * o.n) * 2 * sizeof(float);
}

}  // namespace gt

namespace gt {
// Scratch of gt_plan_update_nodes, allocated on a plan's first update and kept: the radix
// sort's key/value batch and temporary storage, the ragged offsets on the device, and the
// per-wavefront segment counts of the order-2 tile list.
struct RebinScratch {
  bool ready = false;
  uint32_t *kin = nullptr, *kout = nullptr;
  int32_t *vin = nullptr;
  void *tmp = nullptr;
  size_t tmp_bytes = 0;
  int64_t *offs = nullptr;
  int32_t *seg = nullptr;      // ragged plans: (term, dataset) segment starts of a key batch
  int32_t *segcnt = nullptr;
  int32_t segcnt_cap = 0;
};

struct CosTerm {      // cosine basis, one non-empty term: order, bandwidth, internal/external offsets
  int32_t t, N;
  int64_t int_off, ext_off;
};
}  // namespace gt

struct gt_plan {
  gt_problem prob{};
  int basis = GT_BASIS_EXP;           // GT_BASIS_COS: exponential groups of bandwidth 2N at nodes x / 2
  double node_scale = 1.0;            // node map t = node_scale * x (1/2 for the cosine basis)
  int64_t ncoef_int = 0;              // coefficients of the exponential index set the kernels run on
  std::vector<int64_t> ext_off;       // per term: offset in the caller's coefficient vector
  gt::CosTerm *d_cterms = nullptr;    // cosine basis: per non-empty term order, bandwidth, offsets
  void *d_gcos = nullptr;             // cosine basis: R x ncoef_int exponential coefficients
  std::vector<int64_t> offs;          // ragged offsets (R+1) or empty
  bool ragged = false;
  int dtype = GT_C64;
  size_t rsize = 4;                   // sizeof real
  int32_t d = 0, ds = 0, R = 1;
  int64_t M = 0, Mtot = 0, Vtot = 0;
  int32_t nterms = 0;
  int64_t ncoef = 0;
  std::vector<gt::DevTerm> terms;
  gt::DevTerm *d_terms = nullptr;
  gt::OrderHost ord[gt::kMaxOrder + 1];
  int64_t grid_total = 0;
  void *d_x = nullptr;
  void *d_grid = nullptr;
  std::vector<gt::WorkItem> gitems;   // gather work items (kGatherBS virtual nodes each)
  gt::WorkItem *d_gitems = nullptr;
  std::vector<int32_t> gitem_begin;   // per right-hand side, R+1
  int32_t *d_gitem_begin = nullptr;
  int32_t nslots = 0;                 // gather output slots (terms per forward block)
  void *d_fpart = nullptr;            // nslots x Vtot
  double *d_ysum = nullptr;           // per gather item: partial sums (re, im) for the empty set
  int32_t *d_flag = nullptr;          // node validation flag
  void *d_gxp = nullptr;              // node-gradient partials (orders x Vtot x d), allocated on first use
  hipStream_t stream = nullptr;
  hipStream_t side = nullptr;         // second stream (default priority) for the order-1 kernels
  bool use_side = true;               // fork order 1 onto the side stream (a tuning choice)
  bool use_graph = false;             // gt_plan_trafo / gt_plan_adjoint replay a captured graph (a tuning choice)
  bool use_fused = false;             // orders 1 and 2 in shared launches (a tuning choice; fused_available)
  struct GraphEntry {
    int dir;                          // 0 forward, 1 adjoint
    const void *in;
    void *out;
    hipStream_t stream;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;     // captured launch sequences, most recent last
  std::string tuning;                 // report of the last gt_plan_tune (JSON)
  gt::RebinScratch rebin;             // gt_plan_update_nodes
  int64_t node_version = 0;           // updates of the nodes so far
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  size_t lds_limit = 65536;           // LDS per workgroup
  int num_cu = 256;                   // compute units of the device
};

namespace gt {

// ---- error handling (thread-local message) ----
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);
#define GT_HIP(call)                                              \
  do {                                                            \
    hipError_t _e = (call);                                       \
    if (_e != hipSuccess) return ::gt::hip_fail(_e, #call);       \
  } while (0)

// ---- profiling of launches ----
bool prof_enabled();
// Whether the plan's transforms can run in the shared launches of both orders (orders 1 and
// 2 only, both with window forms and one window width, all gather slots in one block, the
// order-2 fold in its tile-sum form within the LDS limit).
bool fused_available(const gt_plan *pl);

// Grid copies of the order-1 binned spread: kSpreadWaves (sums in a fixed order) when they
// fit in LDS, else 1 (one shared grid, atomic adds).
int spread1_copies(const gt_plan *pl);

void prof_begin(hipStream_t s, const char *name);
void prof_end(hipStream_t s);
bool prof_set(bool on);                                   // returns the previous state
size_t prof_mark();                                       // records so far
double prof_take_since(size_t mark, const char *suffix);  // ms of later records named *suffix; drops them

// ---- plan construction helpers (plan.cpp) ----
int validate_problem(const gt_problem *p);
int choose_m(int dtype, double sigma);

// ---- kernel launchers (kernels_f32.hip / kernels_f64.hip) ----
template <typename T> int launch_forward(gt_plan *pl, const void *fhat, const T *colscale, void *f, hipStream_t s);
template <typename T> int launch_adjoint(gt_plan *pl, const void *y, const T *colscale, void *fhat, hipStream_t s);
template <typename T> int launch_node_grad(gt_plan *pl, const void *fhat, const void *g, void *gx, hipStream_t s);
template <typename T> int launch_prepare_nodes(gt_plan *pl, const void *x, hipStream_t s);
template <typename T> int launch_binning(gt_plan *pl, hipStream_t s);   // binning.hip
template <typename T> int launch_rebin(gt_plan *pl, hipStream_t s);     // binning.hip, kept scratch
int launch_tile_relist(gt_plan *pl, hipStream_t s);                      // binning.hip

// ---- solver drivers (solvers.hip) ----
// Sensitivity indices (eq. gsi) from term offsets goff (device, nterms + 1): rho[r][u].
template <typename T> int run_sensitivity(const int64_t *goff, int nterms, int64_t ncoef, int R, const void *fhat,
                                          double *rho, hipStream_t s);
template <typename T> int run_lsqr(gt_plan *pl, const void *y, const double *lambda, const double *omega,
                                   int max_iter, double tol, void *fhat, gt_solve_info *info, hipStream_t s);
template <typename T> int run_lsqr_path(gt_plan *pl, const void *y, int nlam, const double *lambda,
                                        const double *omega, int max_iter, double tol, void *path,
                                        gt_solve_info *info, hipStream_t s);
template <typename T> int run_fista(gt_plan *pl, const void *y, const double *lambda, const double *omega,
                                    int max_iter, double L, double eta, double tol, void *fhat,
                                    gt_solve_info *info, hipStream_t s);
template <typename T> int run_fista_path(gt_plan *pl, const void *y, int nlam, const double *lambda,
                                         const double *omega, int max_iter, double L, double eta, double tol,
                                         const void *f0, void *path, gt_solve_info *info, hipStream_t s);
template <typename T> int run_norm_estimate(gt_plan *pl, int iters, double *out, hipStream_t s);
// gt_plan_norm_estimate_noalloc: the estimate with its work buffers in the fixed device array
// (kNoAllocScratchBytes per device, looked up once per device).
constexpr size_t kNoAllocScratchBytes = size_t(16) << 20;
constexpr int kMaxDevices = 64;
int run_norm_estimate_noalloc(gt_plan *pl, int iters, double *out, hipStream_t s);
template <typename T> int run_norm_estimate_region(gt_plan *pl, int iters, void *region, size_t cap, size_t *need,
                                                   double *out, hipStream_t s);

// device allocation (fails with GT_ENOMEM when the allocation-failure hook says so)
int dev_alloc(void **p, size_t bytes, hipStream_t s);
void dev_free(void *p, hipStream_t s);

// live plans (gt_release_all, and the check that a handle is one)
bool plan_is_live(const gt_plan *pl);

// tuning (tune.cpp / plan.cpp)
int set_gather_path(gt_plan *pl, int t, int path);
int set_adjoint_form(gt_plan *pl, int t, int form);
// direct sums (direct.h): availability per order and direction, and the adjoint's row tiles
// per wavefront (rows 2 |I_u| padded to 64 rtw; 0 when |I_u| > 256)
bool direct_fwd_ok(const gt_plan *pl, int t);
bool direct_adj_ok(const gt_plan *pl, int t);
int direct_adj_rtw(const gt_plan *pl, int t);
int direct_fwd_rtw(const gt_plan *pl, int t);
int set_tile_waves(gt_plan *pl, int waves_cu);
int apply_cached_tuning(gt_plan *pl);
void clear_tuning_cache();
void drop_graphs(gt_plan *pl);
int run_plan_call(gt_plan *pl, int dir, const void *in, void *out, hipStream_t s);
int tune_plan(gt_plan *pl, hipStream_t s);

}  // namespace gt
