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
                           const int64_t *__restrict__ offs, uint32_t *__restrict__ keys, int32_t *__restrict__ vals) {
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
  if (offs) {   // dataset of node i: last b with offs[b] <= i
    int lo = 0, hi = B;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (offs[mid] <= i) lo = mid; else hi = mid;
    }
    b = lo;
  }
  keys[idx] = (uint32_t)(((int64_t)tl * B + b) * nkey + cell);
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

}  // namespace

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
  for (int t = 1; t <= pl->ds && rc == GT_OK; ++t) {
    OrderHost &o = pl->ord[t];
    const int nt = o.term_end - o.term_begin;
    if (nt == 0) continue;
    const int64_t nkey = o.nkey;
    const int64_t K = (int64_t)nt * B * nkey;
    if (K >= (int64_t(1) << 32) - 1 || (int64_t)nt * Mtot >= (int64_t(1) << 31)) {
      rc = fail(GT_EUNSUPPORTED, "too many terms x nodes for 32-bit binning keys");
      break;
    }
    if ((rc = dev_alloc((void **)&o.d_perm, (size_t)nt * Mtot * sizeof(int32_t), s))) break;
    if ((rc = dev_alloc((void **)&o.d_cstart, (size_t)(K + 1) * sizeof(int64_t), s))) break;
    int end_bit = 1;
    while ((int64_t(1) << end_bit) <= K) ++end_bit;
    // batches of terms bounded to ~2^26 pairs
    const int tpb = (int)std::max<int64_t>(1, std::min<int64_t>(nt, (int64_t(1) << 26) / std::max<int64_t>(1, Mtot)));
    const int64_t cap = (int64_t)tpb * Mtot;
    uint32_t *kin = nullptr, *kout = nullptr;
    int32_t *vin = nullptr;
    void *tmp = nullptr;
    size_t tmp_bytes = 0;
    if ((rc = dev_alloc((void **)&kin, cap * sizeof(uint32_t), s)) ||
        (rc = dev_alloc((void **)&kout, cap * sizeof(uint32_t), s)) ||
        (rc = dev_alloc((void **)&vin, cap * sizeof(int32_t), s))) {
      dev_free(kin, s);
      dev_free(kout, s);
      dev_free(vin, s);
      break;
    }
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, kin, kout, vin, o.d_perm, (int)cap, 0,
                                                       end_bit, s);
    if (e == hipSuccess) rc = dev_alloc(&tmp, tmp_bytes, s);
    else rc = hip_fail(e, "radix sort sizing");
    for (int tl0 = 0; tl0 < nt && rc == GT_OK; tl0 += tpb) {
      const int tl1 = std::min(nt, tl0 + tpb);
      const int64_t cnt = (int64_t)(tl1 - tl0) * Mtot;
      hipLaunchKernelGGL((k_bin_keys<T>), dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, (const T *)pl->d_x,
                         Mtot, pl->d_terms, o.term_begin, tl0, tl1, t, o.n, o.ts, o.ntile, nkey, B,
                         (const int64_t *)d_offs, kin, vin);
      size_t tb = tmp_bytes;
      e = hipcub::DeviceRadixSort::SortPairs(tmp, tb, kin, kout, vin, o.d_perm + (int64_t)tl0 * Mtot, (int)cnt, 0,
                                             end_bit, s);
      if (e != hipSuccess) {
        rc = hip_fail(e, "radix sort");
        break;
      }
      const uint32_t k0 = (uint32_t)((int64_t)tl0 * B * nkey);
      const uint32_t k1 = (uint32_t)((int64_t)tl1 * B * nkey);   // inclusive end key (start of next batch)
      const int64_t nk = (int64_t)k1 - k0 + 1;
      hipLaunchKernelGGL(k_bin_starts, dim3((unsigned)((nk + 255) / 256)), dim3(256), 0, s, kout, cnt, k0, k1,
                         (int64_t)tl0 * Mtot, o.d_cstart);
      e = hipGetLastError();
      if (e != hipSuccess) rc = hip_fail(e, "binning kernels");
    }
    if (rc == GT_OK && t == 2) {
      if ((rc = dev_alloc(&o.d_xs, (size_t)nt * Mtot * 2 * sizeof(T), s)) == GT_OK) {
        const int64_t cnt = (int64_t)nt * Mtot;
        hipLaunchKernelGGL((k_sorted_coords<T>), dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s,
                           (const T *)pl->d_x, Mtot, pl->d_terms, o.term_begin, nt, o.d_perm, (T *)o.d_xs);
        e = hipGetLastError();
        if (e != hipSuccess) rc = hip_fail(e, "sorted coordinates");
      }
    }
    // keep the buffers alive until the stream has used them
    (void)hipStreamSynchronize(s);
    dev_free(tmp, s);
    dev_free(kin, s);
    dev_free(kout, s);
    dev_free(vin, s);
  }
  if (d_offs) {
    (void)hipStreamSynchronize(s);
    dev_free(d_offs, s);
  }
  return rc;
}

template int launch_binning<float>(gt_plan *, hipStream_t);
template int launch_binning<double>(gt_plan *, hipStream_t);

}  // namespace gt
