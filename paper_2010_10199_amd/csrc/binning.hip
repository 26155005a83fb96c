// Node binning for the spread and gather: per term, a stable sort of the nodes by the grid
// cell that holds their first window point, grouped by dataset.
//
// For order t a node's cell is (fl_0, ..., fl_{t-1}), fl_j = floor(n x_j + n/2) clamped to
// [0, n), i.e. the same rounding the transform kernels use.  Orders 1 and 3 number the
// cells row-major; order 2 numbers them tile-major: tiles of ts x ts cells in row-major
// order, then the cells of a tile row-major, so that a tile's nodes are contiguous.  Keys are
//   key = (term_local * B + dataset) * nkey + cell number
// and the sort is a stable LSD radix sort (hipCUB), so nodes of one cell keep their index
// order and every plan built from the same nodes gets the same order.  Output per order:
//   perm[term_local * Mtot + pos]  node index in sorted order (term-major blocks of Mtot)
//   cstart[key]                    first sorted position of key (absolute), cstart[K] = end
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <vector>

#include "gt_internal.h"

namespace gt {

namespace {

template <typename T>
__device__ __forceinline__ int cell_of(T x, int n) {
  int f = (int)floor(fma((T)n, x, (T)(n / 2)));
  return f < 0 ? 0 : (f > n - 1 ? n - 1 : f);
}

template <typename T>
__global__ void k_bin_keys(const T *__restrict__ xT, int64_t Mtot, const DevTerm *__restrict__ terms, int term_begin,
                           int tl0, int tl1, int order, int n, int ts, int ntile, int64_t nkey, int B,
                           const int64_t *__restrict__ offs, int cell_only, uint32_t *__restrict__ keys,
                           int32_t *__restrict__ vals) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)(tl1 - tl0) * Mtot;
  if (idx >= total) return;
  const int tl = tl0 + (int)(idx / Mtot);
  const int64_t i = idx - (int64_t)(tl - tl0) * Mtot;
  const DevTerm tm = terms[term_begin + tl];
  const int f0 = cell_of<T>(xT[(int64_t)tm.c0 * Mtot + i], n);
  const int f1 = order >= 2 ? cell_of<T>(xT[(int64_t)tm.c1 * Mtot + i], n) : 0;
  const int f2 = order >= 3 ? cell_of<T>(xT[(int64_t)tm.c2 * Mtot + i], n) : 0;
  int64_t cell;
  if (order == 1) {
    cell = f0;
  } else if (order == 2) {
    const int t0 = f0 / ts, t1 = f1 / ts;
    cell = ((int64_t)t0 * ntile + t1) * ts * ts + (f0 - t0 * ts) * ts + (f1 - t1 * ts);
  } else {
    cell = ((int64_t)f0 * n + f1) * n + f2;
  }
  int b = 0;
  if (offs && !cell_only) {   // dataset of node i: last b with offs[b] <= i
    int lo = 0, hi = B;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (offs[mid] <= i) lo = mid; else hi = mid;
    }
    b = lo;
  }
  keys[idx] = cell_only ? (uint32_t)cell : (uint32_t)(((int64_t)tl * B + b) * nkey + cell);
  vals[idx] = (int32_t)i;
}

// cstart[k] for keys k in [k0, k1]: base + (first position in sorted keys with key >= k).
__global__ void k_bin_starts(const uint32_t *__restrict__ skeys, int64_t count, uint32_t k0, uint32_t k1, int64_t base,
                             int64_t *__restrict__ cstart) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j > (int64_t)k1 - k0) return;
  const uint32_t key = k0 + (uint32_t)j;
  int64_t lo = 0, hi = count;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (skeys[mid] < key) lo = mid + 1; else hi = mid;
  }
  cstart[k0 + j] = base + lo;
}

// The same after a segmented sort whose keys are the cell numbers alone, each (term, dataset)
// segment of the batch sorted on its own (segment i spans [seg[i], seg[i + 1]) of the batch):
// key k = (segment) nkey + cell starts at the first position of its segment whose cell is
// >= cell, which is where the full keys' sort puts it.
__global__ void k_bin_starts_seg(const uint32_t *__restrict__ scell, int64_t count, uint32_t k0, uint32_t k1,
                                 int64_t nkey, const int32_t *__restrict__ seg, int nseg, int64_t base,
                                 int64_t *__restrict__ cstart) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j > (int64_t)k1 - k0) return;
  const int64_t sg = j / nkey;
  if (sg >= nseg) {   // the end key: the batch's end
    cstart[k0 + j] = base + count;
    return;
  }
  const uint32_t cell = (uint32_t)(j - sg * nkey);
  int64_t lo = seg[sg], hi = seg[sg + 1];
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (scell[mid] < cell) lo = mid + 1; else hi = mid;
  }
  cstart[k0 + j] = base + lo;
}

// Order 2: the coordinates of each term's two axes in the term's sorted node order, so the
// spread streams them instead of gathering them through the node index.
template <typename T>
__global__ void k_sorted_coords(const T *__restrict__ xT, int64_t Mtot, const DevTerm *__restrict__ terms,
                                int term_begin, int nt, const int32_t *__restrict__ perm, T *__restrict__ xs) {
  const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pos >= (int64_t)nt * Mtot) return;
  const int tl = (int)(pos / Mtot);
  const DevTerm tm = terms[term_begin + tl];
  const int32_t node = perm[pos];
  xs[2 * pos] = xT[(int64_t)tm.c0 * Mtot + node];
  xs[2 * pos + 1] = xT[(int64_t)tm.c1 * Mtot + node];
}

// Order-2 tile spread work list after a re-binning (gt_plan_update_nodes).  The wavefronts
// keep their runs [qa, qb) of sorted positions, which depend only on the node counts per
// (term, dataset); what moves with the nodes is which tiles a run meets.  Four launches:
//   1. k_relist_count, a thread per wavefront: the non-empty tiles its run meets (the tiles
//      ending after qa and starting before qb), counted into segcnt; every tileseg entry -1;
//   2. k_relist_scan, one workgroup: an exclusive scan of the counts gives each wavefront's
//      first patch segment (waves[4w + 2]); the total closes tileseg;
//   3. k_relist_first, a thread per wavefront: it numbers its tiles' segments again and
//      enters, for the tiles whose first position lies in its run (it is the first wavefront
//      to meet them), the tile's first segment into tileseg;
//   4. k_relist_fill, one workgroup: tiles without nodes (still -1) take the first segment of
//      the next tile that has nodes (over all terms and datasets in order, the total after
//      the last): a backward fill in 1024 chunks, the carry into each chunk from a suffix scan
//      of the chunks' first set entries.
// waves: nwaves x {qa, qb, first segment, dataset}; cstart absolute positions per key (term
// tl's keys start at (tl B + b) nkey; tile t of a (term, dataset) spans keys t TT ..).
struct RelistArgs {
  int32_t *waves;
  int nwaves;
  const int64_t *cstart;
  int64_t Mtot;
  int B;
  int64_t nkey;
  int ntiles, TT;
  int64_t ntiles_all;
  int32_t *segcnt, *tileseg;
};

// Wavefront w's run [qa, qb), its (term, dataset)'s first key and the first tile ending after qa.
__device__ __forceinline__ void relist_tiles_of(const RelistArgs &a, int w, int64_t &key0, int &t0, int64_t &qa,
                                                int64_t &qb) {
  qa = a.waves[4 * w];
  qb = a.waves[4 * w + 1];
  const int b = a.waves[4 * w + 3];
  const int64_t tl = qa / a.Mtot;
  key0 = (tl * a.B + b) * a.nkey;
  int lo = 0, hi = a.ntiles;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a.cstart[key0 + (int64_t)(mid + 1) * a.TT] <= qa) lo = mid + 1; else hi = mid;
  }
  t0 = lo;
}

__global__ __launch_bounds__(256) void k_relist_count(RelistArgs a) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < a.ntiles_all) a.tileseg[i] = -1;
  if (i >= a.nwaves) return;
  const int w = (int)i;
  int64_t key0, qa, qb;
  int t0;
  relist_tiles_of(a, w, key0, t0, qa, qb);
  int c = 0;
  for (int t = t0; t < a.ntiles && a.cstart[key0 + (int64_t)t * a.TT] < qb; ++t)
    if (a.cstart[key0 + (int64_t)(t + 1) * a.TT] > a.cstart[key0 + (int64_t)t * a.TT]) ++c;
  a.segcnt[w] = c;
}

__global__ __launch_bounds__(1024) void k_relist_scan(RelistArgs a) {
  __shared__ int32_t part[1024];
  const int tid = threadIdx.x, nwaves = a.nwaves;
  // chunk sums, a scan of the 1024 sums in LDS, then the chunks
  const int per = (nwaves + 1023) / 1024;
  const int w0 = tid * per, w1 = min(nwaves, w0 + per);
  int32_t sum = 0;
  for (int w = w0; w < w1; ++w) sum += a.segcnt[w];
  part[tid] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int32_t v = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int32_t run = part[tid] - sum;   // exclusive prefix of this chunk
  for (int w = w0; w < w1; ++w) {
    a.waves[4 * w + 2] = run;
    run += a.segcnt[w];
  }
  if (tid == 1023) a.tileseg[a.ntiles_all] = part[1023];
}

__global__ __launch_bounds__(256) void k_relist_first(RelistArgs a) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= a.nwaves) return;
  const int w = (int)i;
  int64_t key0, qa, qb;
  int t0;
  relist_tiles_of(a, w, key0, t0, qa, qb);
  int32_t seg = a.waves[4 * w + 2];
  const int64_t tb0 = key0 / a.TT;   // (tl B + b) ntiles
  for (int t = t0; t < a.ntiles && a.cstart[key0 + (int64_t)t * a.TT] < qb; ++t) {
    const int64_t c0 = a.cstart[key0 + (int64_t)t * a.TT];
    if (a.cstart[key0 + (int64_t)(t + 1) * a.TT] <= c0) continue;   // no nodes
    if (c0 >= qa) a.tileseg[tb0 + t] = seg;
    ++seg;
  }
}

__global__ __launch_bounds__(1024) void k_relist_fill(RelistArgs a) {
  __shared__ int32_t part[1024];
  const int tid = threadIdx.x;
  int32_t *tileseg = a.tileseg;
  const int64_t per2 = (a.ntiles_all + 1023) / 1024;   // chunk tid holds entries [tid per2, (tid + 1) per2)
  const int64_t a0 = tid * per2, a1 = min(a.ntiles_all, a0 + per2);
  int32_t first = -1;   // first set entry of the chunk
  for (int64_t i = a0; i < a1; ++i)
    if (tileseg[i] >= 0) {
      first = tileseg[i];
      break;
    }
  part[tid] = first;
  __syncthreads();
  // suffix scan with "the left operand if set, else the right one": part[c] becomes the first
  // set entry among chunks c, c + 1, ..
  for (int off = 1; off < 1024; off <<= 1) {
    const int32_t r = tid + off < 1024 ? part[tid + off] : -1;
    __syncthreads();
    if (part[tid] < 0) part[tid] = r;
    __syncthreads();
  }
  const int32_t total = tileseg[a.ntiles_all];
  int32_t next = tid + 1 < 1024 && part[tid + 1] >= 0 ? part[tid + 1] : total;   // carry from the right
  for (int64_t i = a1 - 1; i >= a0; --i) {
    if (tileseg[i] < 0)
      tileseg[i] = next;
    else
      next = tileseg[i];
  }
}

}  // namespace

int launch_tile_relist(gt_plan *pl, hipStream_t s) {
  OrderHost &o = pl->ord[2];
  if (pl->ds < 2 || o.term_end == o.term_begin || o.nwaves2 == 0) return GT_OK;
  const int B = pl->ragged ? pl->R : 1;
  RelistArgs a;
  a.waves = o.d_waves2;
  a.nwaves = o.nwaves2;
  a.cstart = (const int64_t *)o.d_cstart;
  a.Mtot = pl->Mtot;
  a.B = B;
  a.nkey = o.nkey;
  a.ntiles = o.ntile * o.ntile;
  a.TT = o.ts * o.ts;
  a.ntiles_all = (int64_t)(o.term_end - o.term_begin) * B * o.ntile * o.ntile;
  a.segcnt = pl->rebin.segcnt;
  a.tileseg = o.d_tileseg;
  const int64_t n1 = std::max<int64_t>(a.nwaves, a.ntiles_all);
  hipLaunchKernelGGL(k_relist_count, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_relist_scan, dim3(1), dim3(1024), 0, s, a);
  hipLaunchKernelGGL(k_relist_first, dim3((unsigned)((a.nwaves + 255) / 256)), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_relist_fill, dim3(1), dim3(1024), 0, s, a);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? GT_OK : hip_fail(e, "tile relist");
}

// Key batches of one order: terms in batches bounded to ~2^26 (term, node) pairs.
static int bin_batch_terms(const gt_plan *pl, int t) {
  const int nt = pl->ord[t].term_end - pl->ord[t].term_begin;
  return (int)std::max<int64_t>(1, std::min<int64_t>(nt, (int64_t(1) << 26) / std::max<int64_t>(1, pl->Mtot)));
}

static int bin_end_bit(const gt_plan *pl, int t) {
  const OrderHost &o = pl->ord[t];
  const int B = pl->ragged ? pl->R : 1;
  const int64_t K = (int64_t)(o.term_end - o.term_begin) * B * o.nkey;
  int end_bit = 1;
  while ((int64_t(1) << end_bit) <= K) ++end_bit;
  return end_bit;
}

// The launches of one order's binning into o.d_perm, o.d_cstart (and o.d_xs for order 2),
// given key/value scratch for one batch and the sort's temporary storage (no allocation, no
// synchronisation).
// Segmented form (seg != nullptr, ragged plans after a node update): the input is already
// grouped by (term, dataset), so each segment is sorted on its own by the cell number alone
// (ceil(log2 nkey) key bits instead of the full key's), stably, which gives the same order.
static int cell_bits(int64_t nkey) {
  int b = 1;
  while ((int64_t(1) << b) < nkey) ++b;
  return b;
}

template <typename T>
static int bin_order(gt_plan *pl, int t, hipStream_t s, const int64_t *d_offs, uint32_t *kin, uint32_t *kout,
                     int32_t *vin, void *tmp, size_t tmp_bytes, const int32_t *seg = nullptr) {
  OrderHost &o = pl->ord[t];
  const int B = pl->ragged ? pl->R : 1;
  const int nt = o.term_end - o.term_begin;
  const int64_t Mtot = pl->Mtot, nkey = o.nkey;
  const int tpb = bin_batch_terms(pl, t), end_bit = bin_end_bit(pl, t);
  for (int tl0 = 0; tl0 < nt; tl0 += tpb) {
    const int tl1 = std::min(nt, tl0 + tpb);
    const int64_t cnt = (int64_t)(tl1 - tl0) * Mtot;
    hipLaunchKernelGGL((k_bin_keys<T>), dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, (const T *)pl->d_x,
                       Mtot, pl->d_terms, o.term_begin, tl0, tl1, t, o.n, o.ts, o.ntile, nkey, B, d_offs,
                       seg ? 1 : 0, kin, vin);
    size_t tb = tmp_bytes;
    const int nseg = (tl1 - tl0) * B;
    hipError_t e = seg ? hipcub::DeviceSegmentedRadixSort::SortPairs(tmp, tb, kin, kout, vin,
                                                                      o.d_perm + (int64_t)tl0 * Mtot, (int)cnt, nseg,
                                                                      seg, seg + 1, 0, cell_bits(nkey), s)
                       : hipcub::DeviceRadixSort::SortPairs(tmp, tb, kin, kout, vin, o.d_perm + (int64_t)tl0 * Mtot,
                                                            (int)cnt, 0, end_bit, s);
    if (e != hipSuccess) return hip_fail(e, "radix sort");
    const uint32_t k0 = (uint32_t)((int64_t)tl0 * B * nkey);
    const uint32_t k1 = (uint32_t)((int64_t)tl1 * B * nkey);   // inclusive end key (start of next batch)
    const int64_t nk = (int64_t)k1 - k0 + 1;
    if (seg)
      hipLaunchKernelGGL(k_bin_starts_seg, dim3((unsigned)((nk + 255) / 256)), dim3(256), 0, s, kout, cnt, k0, k1,
                         nkey, seg, nseg, (int64_t)tl0 * Mtot, o.d_cstart);
    else
      hipLaunchKernelGGL(k_bin_starts, dim3((unsigned)((nk + 255) / 256)), dim3(256), 0, s, kout, cnt, k0, k1,
                         (int64_t)tl0 * Mtot, o.d_cstart);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "binning kernels");
  }
  if (t == 2) {
    const int64_t cnt = (int64_t)nt * Mtot;
    hipLaunchKernelGGL((k_sorted_coords<T>), dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s,
                       (const T *)pl->d_x, Mtot, pl->d_terms, o.term_begin, nt, o.d_perm, (T *)o.d_xs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "sorted coordinates");
  }
  return GT_OK;
}

template <typename T>
int launch_binning(gt_plan *pl, hipStream_t s) {
  const int B = pl->ragged ? pl->R : 1;
  int64_t *d_offs = nullptr;
  int rc = GT_OK;
  if (pl->ragged) {
    if ((rc = dev_alloc((void **)&d_offs, pl->offs.size() * sizeof(int64_t), s))) return rc;
    hipError_t e = hipMemcpyAsync(d_offs, pl->offs.data(), pl->offs.size() * sizeof(int64_t), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
      dev_free(d_offs, s);
      return hip_fail(e, "binning offsets");
    }
  }
  const int64_t Mtot = pl->Mtot;
  // one set of key/value scratch and sort storage for all orders (sized for the largest batch)
  int64_t cap = 1;
  size_t tmp_bytes = 0;
  for (int t = 1; t <= pl->ds && rc == GT_OK; ++t) {
    const OrderHost &o = pl->ord[t];
    if (o.term_end == o.term_begin) continue;
    const int64_t c = (int64_t)bin_batch_terms(pl, t) * Mtot;
    cap = std::max(cap, c);
    size_t tb = 0;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, tb, (uint32_t *)nullptr, (uint32_t *)nullptr,
                                                       (int32_t *)nullptr, (int32_t *)nullptr, (int)c, 0,
                                                       bin_end_bit(pl, t), s);
    if (e != hipSuccess) rc = hip_fail(e, "radix sort sizing");
    tmp_bytes = std::max(tmp_bytes, tb);
  }
  uint32_t *kin = nullptr, *kout = nullptr;
  int32_t *vin = nullptr;
  void *tmp = nullptr;
  if (rc == GT_OK) rc = dev_alloc((void **)&kin, cap * sizeof(uint32_t), s);
  if (rc == GT_OK) rc = dev_alloc((void **)&kout, cap * sizeof(uint32_t), s);
  if (rc == GT_OK) rc = dev_alloc((void **)&vin, cap * sizeof(int32_t), s);
  if (rc == GT_OK) rc = dev_alloc(&tmp, std::max<size_t>(tmp_bytes, 1), s);
  for (int t = 1; t <= pl->ds && rc == GT_OK; ++t) {
    OrderHost &o = pl->ord[t];
    const int nt = o.term_end - o.term_begin;
    if (nt == 0) continue;
    const int64_t K = (int64_t)nt * B * o.nkey;
    if (K >= (int64_t(1) << 32) - 1 || (int64_t)nt * Mtot >= (int64_t(1) << 31)) {
      rc = fail(GT_EUNSUPPORTED, "too many terms x nodes for 32-bit binning keys");
      break;
    }
    if ((rc = dev_alloc((void **)&o.d_perm, (size_t)nt * Mtot * sizeof(int32_t), s))) break;
    if ((rc = dev_alloc((void **)&o.d_cstart, (size_t)(K + 1) * sizeof(int64_t), s))) break;
    if (t == 2 && (rc = dev_alloc(&o.d_xs, (size_t)nt * Mtot * 2 * sizeof(T), s))) break;
    rc = bin_order<T>(pl, t, s, d_offs, kin, kout, vin, tmp, tmp_bytes);
  }
  // keep the buffers alive until the stream has used them
  (void)hipStreamSynchronize(s);
  dev_free(tmp, s);
  dev_free(kin, s);
  dev_free(kout, s);
  dev_free(vin, s);
  if (d_offs) {
    (void)hipStreamSynchronize(s);
    dev_free(d_offs, s);
  }
  return rc;
}

// Re-binning after gt_plan_update_nodes: the same launches into the plan's existing perm,
// cell starts and sorted coordinates, with scratch kept by the plan from its first update on
// (allocated then, sized for the largest order's key batch); no synchronisation.
template <typename T>
int launch_rebin(gt_plan *pl, hipStream_t s) {
  RebinScratch &sc = pl->rebin;
  if (!sc.ready) {
    int64_t cap = 1;
    size_t tmp_bytes = 0;
    int maxtpb = 1;
    for (int t = 1; t <= pl->ds; ++t) {
      const OrderHost &o = pl->ord[t];
      if (o.term_end == o.term_begin) continue;
      const int64_t c = (int64_t)bin_batch_terms(pl, t) * pl->Mtot;
      cap = std::max(cap, c);
      maxtpb = std::max(maxtpb, bin_batch_terms(pl, t));
      size_t tb = 0;
      hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, tb, (uint32_t *)nullptr, (uint32_t *)nullptr,
                                                         (int32_t *)nullptr, (int32_t *)nullptr, (int)c, 0,
                                                         bin_end_bit(pl, t), s);
      if (e != hipSuccess) return hip_fail(e, "radix sort sizing");
      tmp_bytes = std::max(tmp_bytes, tb);
      if (pl->ragged) {
        const int nseg = bin_batch_terms(pl, t) * pl->R;
        e = hipcub::DeviceSegmentedRadixSort::SortPairs(nullptr, tb, (uint32_t *)nullptr, (uint32_t *)nullptr,
                                                        (int32_t *)nullptr, (int32_t *)nullptr, (int)c, nseg,
                                                        (const int32_t *)nullptr, (const int32_t *)nullptr, 0,
                                                        cell_bits(o.nkey), s);
        if (e != hipSuccess) return hip_fail(e, "segmented radix sort sizing");
        tmp_bytes = std::max(tmp_bytes, tb);
      }
    }
    int rc;
    if ((rc = dev_alloc((void **)&sc.kin, cap * sizeof(uint32_t), s)) ||
        (rc = dev_alloc((void **)&sc.kout, cap * sizeof(uint32_t), s)) ||
        (rc = dev_alloc((void **)&sc.vin, cap * sizeof(int32_t), s)) || (rc = dev_alloc(&sc.tmp, tmp_bytes, s)))
      return rc;
    if (pl->ragged) {
      if ((rc = dev_alloc((void **)&sc.offs, pl->offs.size() * sizeof(int64_t), s))) return rc;
      hipError_t e = hipMemcpy(sc.offs, pl->offs.data(), pl->offs.size() * sizeof(int64_t), hipMemcpyHostToDevice);
      if (e != hipSuccess) return hip_fail(e, "binning offsets");
      // segment i = (term tl, dataset b) = (i / R, i % R) of a batch starts at tl Mtot + offs[b]
      std::vector<int32_t> sg((size_t)maxtpb * pl->R + 1);
      for (int tl = 0; tl < maxtpb; ++tl)
        for (int b = 0; b < pl->R; ++b) sg[(size_t)tl * pl->R + b] = (int32_t)(tl * pl->Mtot + pl->offs[b]);
      sg[(size_t)maxtpb * pl->R] = (int32_t)(maxtpb * pl->Mtot);
      if ((rc = dev_alloc((void **)&sc.seg, sg.size() * sizeof(int32_t), s))) return rc;
      e = hipMemcpy(sc.seg, sg.data(), sg.size() * sizeof(int32_t), hipMemcpyHostToDevice);
      if (e != hipSuccess) return hip_fail(e, "segment offsets");
    }
    sc.tmp_bytes = tmp_bytes;
    sc.ready = true;
  }
  for (int t = 1; t <= pl->ds; ++t) {
    if (pl->ord[t].term_end == pl->ord[t].term_begin) continue;
    if (int rc = bin_order<T>(pl, t, s, sc.offs, sc.kin, sc.kout, sc.vin, sc.tmp, sc.tmp_bytes, sc.seg)) return rc;
  }
  return GT_OK;
}

template int launch_binning<float>(gt_plan *, hipStream_t);
template int launch_binning<double>(gt_plan *, hipStream_t);
template int launch_rebin<float>(gt_plan *, hipStream_t);
template int launch_rebin<double>(gt_plan *, hipStream_t);

}  // namespace gt
