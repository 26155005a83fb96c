// Device-resident LSQR and FISTA over the grouped transform (batched over right-hand sides).
//
// LSQR (Sec. 4.1, eq. new_min_prob; method of Paige & Saunders, cited by the paper): Golub-
// Kahan bidiagonalisation of A = F W^{-1/2} from b = y; the damping sqrt(2 lambda) is removed
// by one plane rotation per step, then the subdiagonal by a second one; x and w are updated
// from the rotation coefficients; fhat = W^{-1/2} x.  Bulk vectors are in the precision of
// the plan; alpha, beta, all norms, rotations and the convergence estimates are FP64.
//
// FISTA (Sec. 4.2, Algorithm algo:fista, eq. projection, Theorem theorem:projection): each
// iteration evaluates F h by linearity from the two latest forward products,
// F h^{k+1} = (1 + beta_k) F f^k - beta_k F f^{k-1}, beta_k = (t_k - 1)/t_{k+1}, so the
// constant-step variant costs one forward and one adjoint transform per iteration.  The
// group norms, the proximal scale (closed form for omega = 1, bisection + Newton for xi
// otherwise) and t_k are FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "gt_internal.h"

namespace gt {

namespace {

template <typename T>
__device__ __forceinline__ cx_t<T> mk(T a, T b) {
  cx_t<T> c;
  c.x = a;
  c.y = b;
  return c;
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// Sum over the block, result broadcast to every thread.  sh: >= BS/64 + 1 doubles.
__device__ double block_sum_all(double v, double *sh) {
  v = wsum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0;
    for (int i = 0; i < nw; ++i) s += sh[i];
    sh[nw] = s;
  }
  __syncthreads();
  return sh[nw];
}

constexpr int kCoefChunk = 4096;   // coefficient-space elements per reduction workgroup

// ---------------------------------------------------------------- vector kernels
// y-space (virtual nodes): items of right-hand side r are contiguous.
template <typename T>
__global__ __launch_bounds__(kVecBS) void k_v_axpby_norm(const WorkItem *__restrict__ items, const cx_t<T> *__restrict__ a,
                                                         const double *__restrict__ ca, const cx_t<T> *__restrict__ b,
                                                         const double *__restrict__ cb, cx_t<T> *__restrict__ out,
                                                         double *__restrict__ part) {
  // out = a * ca[r] + b * cb[r] (ca or cb NULL = 1, b NULL = 0); part[item] = ||out||^2 over the item
  __shared__ double sh[kVecBS / 64 + 1];
  const WorkItem it = items[blockIdx.x];
  double s = 0;
  for (int i = threadIdx.x; i < it.count; i += kVecBS) {
    const int64_t v = it.v0 + i;
    const cx_t<T> x = a[v];
    const double fa = ca ? ca[it.r] : 1.0;
    double re = fa * (double)x.x, im = fa * (double)x.y;
    if (b) {
      const cx_t<T> z = b[v];
      const double fb = cb ? cb[it.r] : 1.0;
      re += fb * (double)z.x;
      im += fb * (double)z.y;
    }
    const cx_t<T> o = mk<T>((T)re, (T)im);
    out[v] = o;
    s += (double)o.x * o.x + (double)o.y * o.y;
  }
  s = block_sum_all(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Coefficient space: grid (chunks, R).
template <typename T>
__global__ __launch_bounds__(kVecBS) void k_c_axpby_norm(int64_t n, const cx_t<T> *__restrict__ a,
                                                         const double *__restrict__ ca, const cx_t<T> *__restrict__ b,
                                                         const double *__restrict__ cb, cx_t<T> *__restrict__ out,
                                                         double *__restrict__ part) {
  __shared__ double sh[kVecBS / 64 + 1];
  const int r = blockIdx.y;
  const int64_t lo = (int64_t)blockIdx.x * kCoefChunk, hi = min(n, lo + kCoefChunk);
  const double fa = ca ? ca[r] : 1.0, fb = cb ? cb[r] : 1.0;
  double s = 0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kVecBS) {
    const int64_t k = (int64_t)r * n + i;
    const cx_t<T> x = a[k];
    double re = fa * (double)x.x, im = fa * (double)x.y;
    if (b) {
      const cx_t<T> z = b[k];
      re += fb * (double)z.x;
      im += fb * (double)z.y;
    }
    const cx_t<T> o = mk<T>((T)re, (T)im);
    out[k] = o;
    s += (double)o.x * o.x + (double)o.y * o.y;
  }
  s = block_sum_all(s, sh);
  if (threadIdx.x == 0) part[(int64_t)r * gridDim.x + blockIdx.x] = s;
}

// Re<a, b> per right-hand side in coefficient space (partials).
template <typename T>
__global__ __launch_bounds__(kVecBS) void k_c_dot(int64_t n, const cx_t<T> *__restrict__ a, const cx_t<T> *__restrict__ b,
                                                  double *__restrict__ part) {
  __shared__ double sh[kVecBS / 64 + 1];
  const int r = blockIdx.y;
  const int64_t lo = (int64_t)blockIdx.x * kCoefChunk, hi = min(n, lo + kCoefChunk);
  double s = 0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kVecBS) {
    const int64_t k = (int64_t)r * n + i;
    const cx_t<T> x = a[k], z = b[k];
    s += (double)x.x * z.x + (double)x.y * z.y;
  }
  s = block_sum_all(s, sh);
  if (threadIdx.x == 0) part[(int64_t)r * gridDim.x + blockIdx.x] = s;
}

// out[r] = sum of partials [begin[r], begin[r+1]) (begin NULL: fixed count per r).
__global__ void k_finalize(const double *__restrict__ part, const int32_t *__restrict__ begin, int per_r, int R,
                           double *__restrict__ out, double *__restrict__ sq, double *__restrict__ inv) {
  __shared__ double sh[kVecBS / 64 + 1];
  const int r = blockIdx.x;
  const int lo = begin ? begin[r] : r * per_r, hi = begin ? begin[r + 1] : (r + 1) * per_r;
  double s = 0;
  for (int i = lo + threadIdx.x; i < hi; i += blockDim.x) s += part[i];
  s = block_sum_all(s, sh);
  if (threadIdx.x == 0) {
    if (out) out[r] = s;
    const double q = sqrt(fmax(s, 0.0));
    if (sq) sq[r] = q;
    if (inv) inv[r] = q > 0 ? 1.0 / q : 0.0;
  }
}

template <typename T>
__global__ __launch_bounds__(kVecBS) void k_v_scale(const WorkItem *__restrict__ items, const double *__restrict__ sc,
                                                    cx_t<T> *__restrict__ u) {
  const WorkItem it = items[blockIdx.x];
  const double f = sc[it.r];
  for (int i = threadIdx.x; i < it.count; i += kVecBS) {
    const int64_t v = it.v0 + i;
    const cx_t<T> x = u[v];
    u[v] = mk<T>((T)(f * x.x), (T)(f * x.y));
  }
}

template <typename T>
__global__ __launch_bounds__(kVecBS) void k_c_scale(int64_t n, const double *__restrict__ sc, cx_t<T> *__restrict__ v) {
  const int r = blockIdx.y;
  const double f = sc[r];
  const int64_t lo = (int64_t)blockIdx.x * kCoefChunk, hi = min(n, lo + kCoefChunk);
  for (int64_t i = lo + threadIdx.x; i < hi; i += kVecBS) {
    const int64_t k = (int64_t)r * n + i;
    const cx_t<T> x = v[k];
    v[k] = mk<T>((T)(f * x.x), (T)(f * x.y));
  }
}

template <typename T>
__global__ __launch_bounds__(kVecBS) void k_c_fill(int64_t total, cx_t<T> *__restrict__ v) {
  const int64_t i = (int64_t)blockIdx.x * kVecBS + threadIdx.x;
  if (i < total) v[i] = mk<T>(0, 0);
}

template <typename T>
__global__ __launch_bounds__(kVecBS) void k_c_fill_value(int64_t total, T val, cx_t<T> *__restrict__ v) {
  const int64_t i = (int64_t)blockIdx.x * kVecBS + threadIdx.x;
  if (i < total) v[i] = mk<T>(val, 0);
}

template <typename T>
__global__ __launch_bounds__(kVecBS) void k_copy(int64_t total, const cx_t<T> *__restrict__ a, cx_t<T> *__restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * kVecBS + threadIdx.x;
  if (i < total) b[i] = a[i];
}

// ---------------------------------------------------------------- LSQR scalars
struct LsqrState {
  double alpha, beta, rhobar, phibar, normal, normal0;
  double cx, cw;     // x += cx w ; w = v + cw w
  int32_t done;      // breakdown seen: x frozen
  int32_t iters;
};

__global__ void k_lsqr_init(int R, const double *__restrict__ alpha, const double *__restrict__ beta,
                            LsqrState *__restrict__ st) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  LsqrState s{};
  s.alpha = alpha[r];
  s.beta = beta[r];
  s.rhobar = s.alpha;
  s.phibar = s.beta;
  s.normal = fabs(s.alpha * s.beta);
  s.normal0 = s.normal;
  s.done = (s.alpha == 0.0 || s.beta == 0.0) ? 1 : 0;
  s.iters = 0;
  st[r] = s;
}

__global__ void k_lsqr_step(int R, const double *__restrict__ lambda, const double *__restrict__ alpha,
                            const double *__restrict__ beta, LsqrState *__restrict__ st) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  LsqrState s = st[r];
  if (s.done) {
    s.cx = 0;
    s.cw = 0;
    st[r] = s;
    return;
  }
  const double a = alpha[r], b = beta[r];
  const double damp = sqrt(2.0 * lambda[r]);
  const double rhobar1 = hypot(s.rhobar, damp);
  const double c1 = s.rhobar / rhobar1;
  s.phibar = c1 * s.phibar;
  const double rho = hypot(rhobar1, b);
  const double c = rhobar1 / rho, sn = b / rho;
  const double theta = sn * a;
  s.rhobar = -c * a;
  const double phi = c * s.phibar;
  s.phibar = sn * s.phibar;
  s.cx = phi / rho;
  s.cw = -theta / rho;
  s.normal = fabs(s.phibar) * a * fabs(c);   // phibar carries a sign
  s.alpha = a;
  s.beta = b;
  s.iters += 1;
  if (a == 0.0 || b == 0.0) s.done = 1;
  st[r] = s;
}

template <typename T>
__global__ __launch_bounds__(kVecBS) void k_lsqr_xw(int64_t n, const LsqrState *__restrict__ st,
                                                    const cx_t<T> *__restrict__ v, cx_t<T> *__restrict__ w,
                                                    cx_t<T> *__restrict__ x) {
  const int r = blockIdx.y;
  const double cx = st[r].cx, cw = st[r].cw;
  if (cx == 0.0 && cw == 0.0) return;
  const int64_t lo = (int64_t)blockIdx.x * kCoefChunk, hi = min(n, lo + kCoefChunk);
  for (int64_t i = lo + threadIdx.x; i < hi; i += kVecBS) {
    const int64_t k = (int64_t)r * n + i;
    const cx_t<T> wv = w[k], xv = x[k], vv = v[k];
    x[k] = mk<T>((T)(xv.x + cx * wv.x), (T)(xv.y + cx * wv.y));
    w[k] = mk<T>((T)(vv.x + cw * wv.x), (T)(vv.y + cw * wv.y));
  }
}

template <typename T>
__global__ __launch_bounds__(kVecBS) void k_colscale(int64_t ncoef, const T *__restrict__ omega, T *__restrict__ cs,
                                                     int32_t *__restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * kVecBS + threadIdx.x;
  if (i >= ncoef) return;
  const T w = omega[i];
  if (!(w > (T)0) || !isfinite(w)) {
    atomicOr(bad, 1);
    cs[i] = (T)1;
  } else {
    cs[i] = (T)(1.0 / sqrt((double)w));
  }
}

template <typename T>
__global__ __launch_bounds__(kVecBS) void k_c_mul_colscale(int64_t n, const T *__restrict__ cs, const cx_t<T> *__restrict__ a,
                                                           cx_t<T> *__restrict__ out) {
  const int r = blockIdx.y;
  const int64_t lo = (int64_t)blockIdx.x * kCoefChunk, hi = min(n, lo + kCoefChunk);
  for (int64_t i = lo + threadIdx.x; i < hi; i += kVecBS) {
    const int64_t k = (int64_t)r * n + i;
    const cx_t<T> x = a[k];
    const T c = cs ? cs[i] : (T)1;
    out[k] = mk<T>(x.x * c, x.y * c);
  }
}

// ---------------------------------------------------------------- FISTA kernels
// res = (1 + beta) Fcur - beta Fold - y   (beta = 0: res = Fcur - y)
template <typename T>
__global__ __launch_bounds__(kVecBS) void k_fista_resid(int64_t V, double beta, const cx_t<T> *__restrict__ Fcur,
                                                        const cx_t<T> *__restrict__ Fold, const cx_t<T> *__restrict__ y,
                                                        cx_t<T> *__restrict__ res) {
  const int64_t i = (int64_t)blockIdx.x * kVecBS + threadIdx.x;
  if (i >= V) return;
  const cx_t<T> a = Fcur[i], c = y[i];
  double re = (1.0 + beta) * (double)a.x - (double)c.x, im = (1.0 + beta) * (double)a.y - (double)c.y;
  if (beta != 0.0) {
    const cx_t<T> b = Fold[i];
    re -= beta * (double)b.x;
    im -= beta * (double)b.y;
  }
  res[i] = mk<T>((T)re, (T)im);
}

// t(xi) = sum_k w_k a_k xi^2 / (1 + xi w_k)^2 and its derivative (a_k = |z_k|^2).
struct GroupView {
  int64_t off, size;
};

// Proximal step on one (group, right-hand side): z = h - g / L_r, f_new = prox(z, lambda_r / L_r).
// stats[(r * ngroups + group) * 2 + {0,1}] = ||f_new - f_cur||^2, ||f_new||^2 over the group.
template <typename T>
__global__ __launch_bounds__(kVecBS) void k_fista_prox(int64_t ncoef, const int64_t *__restrict__ goff, int ngroups,
                                                       const double *__restrict__ lambda, const double *__restrict__ Lr,
                                                       const T *__restrict__ omega, const cx_t<T> *__restrict__ h,
                                                       const cx_t<T> *__restrict__ g, const cx_t<T> *__restrict__ fcur,
                                                       cx_t<T> *__restrict__ fnew, double *__restrict__ stats) {
  __shared__ double sh[kVecBS / 64 + 1];
  const int grp = blockIdx.x, r = blockIdx.y;
  const int64_t lo = goff[grp], hi = goff[grp + 1];
  const int64_t base = (int64_t)r * ncoef;
  const double L = Lr[r];
  const double tau = lambda[r] / L;
  const double invL = 1.0 / L;
  auto zval = [&](int64_t k, double &zr, double &zi) {
    const cx_t<T> hv = h[base + k], gv = g[base + k];
    zr = (double)hv.x - invL * (double)gv.x;
    zi = (double)hv.y - invL * (double)gv.y;
  };
  // zero level ||(z_k / omega_k)||_W = (sum |z_k|^2 / omega_k)^{1/2}  (Lemma (iii))
  double s = 0;
  for (int64_t k = lo + threadIdx.x; k < hi; k += kVecBS) {
    double zr, zi;
    zval(k, zr, zi);
    const double w = omega ? (double)omega[k] : 1.0;
    s += (zr * zr + zi * zi) / w;
  }
  const double zero_level = sqrt(block_sum_all(s, sh));
  double xi = 0.0, scale = 0.0;
  const bool zero = tau >= zero_level;
  if (!zero && !omega) {
    scale = 1.0 - tau / zero_level;   // block soft-thresholding (omega = 1)
  } else if (!zero) {
    const double target = tau * tau;
    auto t_of = [&](double xv) {       // sum w a xv^2 / (1 + xv w)^2
      double acc = 0;
      for (int64_t k = lo + threadIdx.x; k < hi; k += kVecBS) {
        double zr, zi;
        zval(k, zr, zi);
        const double w = (double)omega[k], a = zr * zr + zi * zi;
        const double den = 1.0 + xv * w;
        acc += w * a * xv * xv / (den * den);
      }
      return block_sum_all(acc, sh);
    };
    auto t_of_zeta = [&](double zeta) {   // t(1/zeta) = sum w a / (zeta + w)^2
      double acc = 0;
      for (int64_t k = lo + threadIdx.x; k < hi; k += kVecBS) {
        double zr, zi;
        zval(k, zr, zi);
        const double w = (double)omega[k], a = zr * zr + zi * zi;
        const double den = zeta + w;
        acc += w * a / (den * den);
      }
      return block_sum_all(acc, sh);
    };
    if (t_of(1.0) >= target) {
      double a = 0.0, b = 1.0;
      for (int it = 0; it < 60; ++it) {
        const double mid = 0.5 * (a + b);
        if (mid > 0 && t_of(mid) < target) a = mid; else b = mid;
      }
      xi = 0.5 * (a + b);
    } else {
      double a = 0.0, b = 1.0;
      for (int it = 0; it < 60; ++it) {
        const double mid = 0.5 * (a + b);
        if (t_of_zeta(mid) > target) a = mid; else b = mid;
      }
      xi = 1.0 / (0.5 * (a + b));
    }
    for (int it = 0; it < 20; ++it) {
      double v = 0, dv = 0;
      for (int64_t k = lo + threadIdx.x; k < hi; k += kVecBS) {
        double zr, zi;
        zval(k, zr, zi);
        const double w = (double)omega[k], a = zr * zr + zi * zi;
        const double den = 1.0 + xi * w;
        v += w * a * xi * xi / (den * den);
        dv += w * a * 2.0 * xi / (den * den * den);
      }
      v = block_sum_all(v, sh) - target;
      dv = block_sum_all(dv, sh);
      if (fabs(v) <= 1e-15 * target || dv <= 0) break;
      const double nx = xi - v / dv;
      xi = nx > 0 ? nx : 0.5 * xi;
    }
  }
  double dd = 0, nn = 0;
  for (int64_t k = lo + threadIdx.x; k < hi; k += kVecBS) {
    double zr, zi;
    zval(k, zr, zi);
    double fr = 0, fi = 0;
    if (!zero) {
      const double sc = omega ? 1.0 / (1.0 + xi * (double)omega[k]) : scale;
      fr = sc * zr;
      fi = sc * zi;
    }
    const cx_t<T> o = mk<T>((T)fr, (T)fi);
    fnew[base + k] = o;
    const cx_t<T> c = fcur[base + k];
    const double er = (double)o.x - c.x, ei = (double)o.y - c.y;
    dd += er * er + ei * ei;
    nn += (double)o.x * o.x + (double)o.y * o.y;
  }
  dd = block_sum_all(dd, sh);
  nn = block_sum_all(nn, sh);
  if (threadIdx.x == 0) {
    stats[((int64_t)r * ngroups + grp) * 2] = dd;
    stats[((int64_t)r * ngroups + grp) * 2 + 1] = nn;
  }
}

// h = f_new + beta (f_new - f_cur)
template <typename T>
__global__ __launch_bounds__(kVecBS) void k_fista_momentum(int64_t total, double beta, const cx_t<T> *__restrict__ fnew,
                                                           const cx_t<T> *__restrict__ fcur, cx_t<T> *__restrict__ h) {
  const int64_t i = (int64_t)blockIdx.x * kVecBS + threadIdx.x;
  if (i >= total) return;
  const cx_t<T> a = fnew[i], b = fcur[i];
  h[i] = mk<T>((T)((double)a.x + beta * ((double)a.x - b.x)), (T)((double)a.y + beta * ((double)a.y - b.y)));
}

// d = a - b
template <typename T>
__global__ __launch_bounds__(kVecBS) void k_sub(int64_t total, const cx_t<T> *__restrict__ a, const cx_t<T> *__restrict__ b,
                                                cx_t<T> *__restrict__ d) {
  const int64_t i = (int64_t)blockIdx.x * kVecBS + threadIdx.x;
  if (i >= total) return;
  const cx_t<T> x = a[i], z = b[i];
  d[i] = mk<T>(x.x - z.x, x.y - z.y);
}

__global__ void k_neg(int R, const double *__restrict__ a, double *__restrict__ na) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < R) na[r] = -a[r];
}

unsigned nblk(int64_t total) { return (unsigned)((total + kVecBS - 1) / kVecBS); }

int check(const char *what) {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? GT_OK : hip_fail(e, what);
}

// Scratch owned by one solver call.
struct Scratch {
  std::vector<void *> ptrs;
  ~Scratch() {
    for (void *p : ptrs) dev_free(p, nullptr);
  }
  template <typename P>
  int get(P **p, size_t bytes) {
    void *q = nullptr;
    int rc = dev_alloc(&q, std::max<size_t>(bytes, 16), nullptr);
    if (rc) return rc;
    ptrs.push_back(q);
    *p = (P *)q;
    return GT_OK;
  }
};

// ||.||^2 helpers -----------------------------------------------------------
template <typename T>
struct Norms {
  gt_plan *pl;
  double *partV = nullptr, *partC = nullptr;
  int nchunk = 1;
  int init(Scratch &sc) {
    nchunk = (int)((pl->ncoef + kCoefChunk - 1) / kCoefChunk);
    if (int rc = sc.get(&partV, sizeof(double) * std::max<size_t>(1, pl->gitems.size()))) return rc;
    return sc.get(&partC, sizeof(double) * (size_t)nchunk * pl->R);
  }
  // out = a*ca + b*cb in y-space, then sq[r] = ||out_r||, inv[r] = 1/sq[r]
  int v_axpby(const cx_t<T> *a, const double *ca, const cx_t<T> *b, const double *cb, cx_t<T> *out, double *sq,
              double *inv, hipStream_t s) {
    const unsigned ngi = (unsigned)pl->gitems.size();
    hipLaunchKernelGGL((k_v_axpby_norm<T>), dim3(ngi), dim3(kVecBS), 0, s, pl->d_gitems, a, ca, b, cb, out, partV);
    hipLaunchKernelGGL(k_finalize, dim3(pl->R), dim3(kVecBS), 0, s, partV, pl->d_gitem_begin, 0, pl->R, nullptr, sq,
                       inv);
    return check("y-space update");
  }
  int c_axpby(const cx_t<T> *a, const double *ca, const cx_t<T> *b, const double *cb, cx_t<T> *out, double *sq,
              double *inv, hipStream_t s, double *sum = nullptr) {
    hipLaunchKernelGGL((k_c_axpby_norm<T>), dim3(nchunk, pl->R), dim3(kVecBS), 0, s, pl->ncoef, a, ca, b, cb, out,
                       partC);
    hipLaunchKernelGGL(k_finalize, dim3(pl->R), dim3(kVecBS), 0, s, partC, nullptr, nchunk, pl->R, sum, sq, inv);
    return check("coefficient update");
  }
};

}  // namespace

// ================================================================== LSQR
template <typename T>
int run_lsqr(gt_plan *pl, const void *y, const double *lambda, const void *omega, int max_iter, double tol, void *fhat,
             gt_solve_info *info, hipStream_t s) {
  using C = cx_t<T>;
  const int R = pl->R;
  const int64_t V = pl->Vtot, n = pl->ncoef;
  Scratch sc;
  C *u, *v, *w, *x, *tV, *tI;
  double *alpha, *beta, *ialpha, *ibeta, *dlam;
  LsqrState *st;
  T *cs = nullptr;
  int32_t *bad;
  int rc;
  if ((rc = sc.get(&u, V * sizeof(C))) || (rc = sc.get(&tV, V * sizeof(C))) || (rc = sc.get(&v, n * R * sizeof(C))) ||
      (rc = sc.get(&w, n * R * sizeof(C))) || (rc = sc.get(&x, n * R * sizeof(C))) ||
      (rc = sc.get(&tI, n * R * sizeof(C))) || (rc = sc.get(&alpha, R * sizeof(double))) ||
      (rc = sc.get(&beta, R * sizeof(double))) || (rc = sc.get(&ialpha, R * sizeof(double))) ||
      (rc = sc.get(&ibeta, R * sizeof(double))) || (rc = sc.get(&dlam, R * sizeof(double))) ||
      (rc = sc.get(&st, R * sizeof(LsqrState))) || (rc = sc.get(&bad, sizeof(int32_t))))
    return rc;
  Norms<T> nm{pl};
  if ((rc = nm.init(sc))) return rc;
  GT_HIP(hipMemcpyAsync(dlam, lambda, R * sizeof(double), hipMemcpyHostToDevice, s));
  if (omega) {
    if ((rc = sc.get(&cs, n * sizeof(T)))) return rc;
    int32_t zero = 0;
    GT_HIP(hipMemcpyAsync(bad, &zero, sizeof(zero), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL((k_colscale<T>), dim3(nblk(n)), dim3(kVecBS), 0, s, n, (const T *)omega, cs, bad);
    int32_t hbad = 0;
    GT_HIP(hipMemcpyAsync(&hbad, bad, sizeof(hbad), hipMemcpyDeviceToHost, s));
    GT_HIP(hipStreamSynchronize(s));
    if (hbad) return fail(GT_EINVAL, "weights must be finite and > 0");
  }
  const unsigned nchunk = (unsigned)nm.nchunk;
  // beta_1 u_1 = y
  if ((rc = nm.v_axpby((const C *)y, nullptr, nullptr, nullptr, u, beta, ibeta, s))) return rc;
  hipLaunchKernelGGL((k_v_scale<T>), dim3((unsigned)pl->gitems.size()), dim3(kVecBS), 0, s, pl->d_gitems, ibeta, u);
  // alpha_1 v_1 = A^H u_1
  if ((rc = launch_adjoint<T>(pl, u, cs, v, s))) return rc;
  if ((rc = nm.c_axpby(v, nullptr, nullptr, nullptr, v, alpha, ialpha, s))) return rc;
  hipLaunchKernelGGL((k_c_scale<T>), dim3(nchunk, R), dim3(kVecBS), 0, s, n, ialpha, v);
  hipLaunchKernelGGL((k_copy<T>), dim3(nblk(n * R)), dim3(kVecBS), 0, s, n * R, v, w);
  hipLaunchKernelGGL((k_c_fill<T>), dim3(nblk(n * R)), dim3(kVecBS), 0, s, n * R, x);
  hipLaunchKernelGGL(k_lsqr_init, dim3((R + 63) / 64), dim3(64), 0, s, R, alpha, beta, st);
  if ((rc = check("lsqr init"))) return rc;
  // -alpha and -beta for the axpby kernels
  double *nalpha, *nbeta;
  if ((rc = sc.get(&nalpha, R * sizeof(double))) || (rc = sc.get(&nbeta, R * sizeof(double)))) return rc;
  std::vector<LsqrState> hst(R);
  int it = 0;
  bool converged = false;
  for (it = 1; it <= max_iter; ++it) {
    // u = A v - alpha u
    if ((rc = launch_forward<T>(pl, v, cs, tV, s))) return rc;
    hipLaunchKernelGGL(k_neg, dim3((R + 63) / 64), dim3(64), 0, s, R, (const double *)alpha, nalpha);
    if ((rc = nm.v_axpby(tV, nullptr, u, nalpha, u, beta, ibeta, s))) return rc;
    hipLaunchKernelGGL((k_v_scale<T>), dim3((unsigned)pl->gitems.size()), dim3(kVecBS), 0, s, pl->d_gitems, ibeta, u);
    // v = A^H u - beta v
    if ((rc = launch_adjoint<T>(pl, u, cs, tI, s))) return rc;
    hipLaunchKernelGGL(k_neg, dim3((R + 63) / 64), dim3(64), 0, s, R, (const double *)beta, nbeta);
    if ((rc = nm.c_axpby(tI, nullptr, v, nbeta, v, alpha, ialpha, s))) return rc;
    hipLaunchKernelGGL((k_c_scale<T>), dim3(nchunk, R), dim3(kVecBS), 0, s, n, ialpha, v);
    // rotations, x and w
    hipLaunchKernelGGL(k_lsqr_step, dim3((R + 63) / 64), dim3(64), 0, s, R, dlam, alpha, beta, st);
    hipLaunchKernelGGL((k_lsqr_xw<T>), dim3(nchunk, R), dim3(kVecBS), 0, s, n, st, v, w, x);
    if ((rc = check("lsqr iteration"))) return rc;
    if (tol > 0 && (it % 8 == 0 || it == max_iter)) {
      GT_HIP(hipMemcpyAsync(hst.data(), st, R * sizeof(LsqrState), hipMemcpyDeviceToHost, s));
      GT_HIP(hipStreamSynchronize(s));
      bool all = true;
      for (int r = 0; r < R; ++r)
        if (!(hst[r].done || hst[r].normal <= tol * hst[r].normal0)) all = false;
      if (all) {
        converged = true;
        break;
      }
    }
  }
  // fhat = W^{-1/2} x
  hipLaunchKernelGGL((k_c_mul_colscale<T>), dim3(nchunk, R), dim3(kVecBS), 0, s, n, (const T *)cs, x, (C *)fhat);
  if ((rc = check("lsqr output"))) return rc;
  GT_HIP(hipMemcpyAsync(hst.data(), st, R * sizeof(LsqrState), hipMemcpyDeviceToHost, s));
  GT_HIP(hipStreamSynchronize(s));
  for (int r = 0; r < R; ++r) {
    info[r].iters = hst[r].iters;
    info[r].resid = hst[r].normal;
    info[r].t_k = hst[r].phibar;
    info[r].L = 0;
    int32_t fl = 0;
    if (hst[r].done) fl |= GT_SOLVE_BREAKDOWN;
    if (tol > 0 && (hst[r].done || hst[r].normal <= tol * hst[r].normal0)) fl |= GT_SOLVE_CONVERGED;
    if (!converged && it > max_iter) fl |= GT_SOLVE_MAX_ITER;
    info[r].flags = fl;
  }
  return GT_OK;
}

// ================================================================== power iteration
template <typename T>
static int power_iter(gt_plan *pl, int iters, Scratch &sc, double *est_host, hipStream_t s) {
  using C = cx_t<T>;
  const int R = pl->R;
  const int64_t V = pl->Vtot, n = pl->ncoef;
  C *v, *wv, *tV;
  double *nrm, *inv, *dot, *partC;
  int rc;
  if ((rc = sc.get(&v, n * R * sizeof(C))) || (rc = sc.get(&wv, n * R * sizeof(C))) ||
      (rc = sc.get(&tV, V * sizeof(C))) || (rc = sc.get(&nrm, R * sizeof(double))) ||
      (rc = sc.get(&inv, R * sizeof(double))) || (rc = sc.get(&dot, R * sizeof(double))))
    return rc;
  Norms<T> nm{pl};
  if ((rc = nm.init(sc))) return rc;
  partC = nm.partC;
  const unsigned nchunk = (unsigned)nm.nchunk;
  // v = ones / sqrt(n)
  hipLaunchKernelGGL((k_c_fill_value<T>), dim3(nblk(n * R)), dim3(kVecBS), 0, s, n * R, (T)(1.0 / std::sqrt((double)n)),
                     v);
  for (int k = 0; k < iters; ++k) {
    if ((rc = launch_forward<T>(pl, v, nullptr, tV, s))) return rc;
    if ((rc = launch_adjoint<T>(pl, tV, nullptr, wv, s))) return rc;
    hipLaunchKernelGGL((k_c_dot<T>), dim3(nchunk, R), dim3(kVecBS), 0, s, n, v, wv, partC);
    hipLaunchKernelGGL(k_finalize, dim3(R), dim3(kVecBS), 0, s, partC, nullptr, (int)nchunk, R, dot, nullptr, nullptr);
    if ((rc = nm.c_axpby(wv, nullptr, nullptr, nullptr, wv, nrm, inv, s))) return rc;
    hipLaunchKernelGGL((k_c_scale<T>), dim3(nchunk, R), dim3(kVecBS), 0, s, n, inv, wv);
    std::swap(v, wv);
    if ((rc = check("power iteration"))) return rc;
  }
  GT_HIP(hipMemcpyAsync(est_host, dot, R * sizeof(double), hipMemcpyDeviceToHost, s));
  GT_HIP(hipStreamSynchronize(s));
  return GT_OK;
}

template <typename T>
int run_norm_estimate(gt_plan *pl, int iters, double *out, hipStream_t s) {
  Scratch sc;
  std::vector<double> est(pl->R);
  int rc = power_iter<T>(pl, iters, sc, est.data(), s);
  if (rc) return rc;
  *out = est[0];
  return GT_OK;
}

// ================================================================== FISTA
template <typename T>
int run_fista(gt_plan *pl, const void *y, const double *lambda, const void *omega, int max_iter, double L, double eta,
              double tol, void *fhat, gt_solve_info *info, hipStream_t s) {
  using C = cx_t<T>;
  const int R = pl->R;
  const int64_t V = pl->Vtot, n = pl->ncoef;
  const int ngroups = pl->nterms;
  Scratch sc;
  C *fa, *fb, *h, *g, *Fcur, *Fold, *res;
  double *dlam, *dL, *stats;
  int64_t *goff;
  int32_t *bad;
  int rc;
  if ((rc = sc.get(&fa, n * R * sizeof(C))) || (rc = sc.get(&fb, n * R * sizeof(C))) ||
      (rc = sc.get(&h, n * R * sizeof(C))) || (rc = sc.get(&g, n * R * sizeof(C))) ||
      (rc = sc.get(&Fcur, V * sizeof(C))) || (rc = sc.get(&Fold, V * sizeof(C))) || (rc = sc.get(&res, V * sizeof(C))) ||
      (rc = sc.get(&dlam, R * sizeof(double))) || (rc = sc.get(&dL, R * sizeof(double))) ||
      (rc = sc.get(&stats, (size_t)R * ngroups * 2 * sizeof(double))) ||
      (rc = sc.get(&goff, (size_t)(ngroups + 1) * sizeof(int64_t))) || (rc = sc.get(&bad, sizeof(int32_t))))
    return rc;
  if (omega) {
    T *tmp = nullptr;
    if ((rc = sc.get(&tmp, n * sizeof(T)))) return rc;
    int32_t zero = 0;
    GT_HIP(hipMemcpyAsync(bad, &zero, sizeof(zero), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL((k_colscale<T>), dim3(nblk(n)), dim3(kVecBS), 0, s, n, (const T *)omega, tmp, bad);
    int32_t hbad = 0;
    GT_HIP(hipMemcpyAsync(&hbad, bad, sizeof(hbad), hipMemcpyDeviceToHost, s));
    GT_HIP(hipStreamSynchronize(s));
    if (hbad) return fail(GT_EINVAL, "weights must be finite and > 0");
  }
  std::vector<int64_t> hoff(ngroups + 1);
  for (int i = 0; i < ngroups; ++i) hoff[i] = pl->terms[i].coef_off;
  hoff[ngroups] = n;
  GT_HIP(hipMemcpyAsync(goff, hoff.data(), hoff.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
  GT_HIP(hipMemcpyAsync(dlam, lambda, R * sizeof(double), hipMemcpyHostToDevice, s));
  std::vector<double> hL(R, L);
  if (!(L > 0)) {
    std::vector<double> est(R);
    if ((rc = power_iter<T>(pl, 50, sc, est.data(), s))) return rc;
    for (int r = 0; r < R; ++r) hL[r] = 1.05 * est[r];
  }
  for (int r = 0; r < R; ++r)
    if (!(hL[r] > 0) || !std::isfinite(hL[r])) return fail(GT_EINVAL, "step constant L must be > 0");
  GT_HIP(hipMemcpyAsync(dL, hL.data(), R * sizeof(double), hipMemcpyHostToDevice, s));
  const bool backtrack = eta > 1.0;
  C *delta = nullptr, *Fd = nullptr;
  double *partC = nullptr, *partV = nullptr, *nd = nullptr, *nFd = nullptr;
  Norms<T> nm{pl};
  if ((rc = nm.init(sc))) return rc;
  if (backtrack) {
    if ((rc = sc.get(&delta, n * R * sizeof(C))) || (rc = sc.get(&Fd, V * sizeof(C))) ||
        (rc = sc.get(&nd, R * sizeof(double))) || (rc = sc.get(&nFd, R * sizeof(double))))
      return rc;
    partC = nm.partC;
    partV = nm.partV;
  }
  const unsigned nchunk = (unsigned)nm.nchunk;
  // f_0 from fhat, h_1 = f_0, t_1 = 1, Fcur = F f_0
  hipLaunchKernelGGL((k_copy<T>), dim3(nblk(n * R)), dim3(kVecBS), 0, s, n * R, (const C *)fhat, fa);
  hipLaunchKernelGGL((k_copy<T>), dim3(nblk(n * R)), dim3(kVecBS), 0, s, n * R, (const C *)fhat, h);
  if ((rc = launch_forward<T>(pl, fa, nullptr, Fcur, s))) return rc;
  double t = 1.0, beta_prev = 0.0;
  std::vector<double> hstats((size_t)R * ngroups * 2);
  std::vector<double> rel(R, 0.0);
  std::vector<int32_t> capped(R, 0);
  int it = 0;
  bool converged = false;
  for (it = 1; it <= max_iter; ++it) {
    // gradient at h: F^H (F h - y)
    hipLaunchKernelGGL((k_fista_resid<T>), dim3(nblk(V)), dim3(kVecBS), 0, s, V, beta_prev, Fcur, Fold, (const C *)y,
                       res);
    if ((rc = launch_adjoint<T>(pl, res, nullptr, g, s))) return rc;
    hipLaunchKernelGGL((k_fista_prox<T>), dim3(ngroups, R), dim3(kVecBS), 0, s, n, goff, ngroups, dlam, dL,
                       (const T *)omega, h, g, fa, fb, stats);
    if ((rc = check("fista prox"))) return rc;
    if (backtrack) {
      // accept when ||F(f - h)||^2 <= L ||f - h||^2 (exact equivalent of the algorithm's test)
      for (int trial = 0;; ++trial) {
        hipLaunchKernelGGL((k_sub<T>), dim3(nblk(n * R)), dim3(kVecBS), 0, s, n * R, fb, h, delta);
        if ((rc = nm.c_axpby(delta, nullptr, nullptr, nullptr, delta, nullptr, nullptr, s, nd))) return rc;
        if ((rc = launch_forward<T>(pl, delta, nullptr, Fd, s))) return rc;
        if ((rc = nm.v_axpby(Fd, nullptr, nullptr, nullptr, Fd, nullptr, nullptr, s))) return rc;
        hipLaunchKernelGGL(k_finalize, dim3(R), dim3(kVecBS), 0, s, partV, pl->d_gitem_begin, 0, R, nFd, nullptr,
                           nullptr);
        std::vector<double> a(R), b(R);
        GT_HIP(hipMemcpyAsync(a.data(), nFd, R * sizeof(double), hipMemcpyDeviceToHost, s));
        GT_HIP(hipMemcpyAsync(b.data(), nd, R * sizeof(double), hipMemcpyDeviceToHost, s));
        GT_HIP(hipStreamSynchronize(s));
        bool all = true;
        for (int r = 0; r < R; ++r)
          if (a[r] > hL[r] * b[r]) {
            all = false;
            if (trial < 30) hL[r] *= eta;
          }
        if (all) break;
        if (trial >= 30) {
          for (int r = 0; r < R; ++r) capped[r] = 1;
          break;
        }
        GT_HIP(hipMemcpyAsync(dL, hL.data(), R * sizeof(double), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL((k_fista_prox<T>), dim3(ngroups, R), dim3(kVecBS), 0, s, n, goff, ngroups, dlam, dL,
                           (const T *)omega, h, g, fa, fb, stats);
        if ((rc = check("fista prox"))) return rc;
      }
    }
    const double t_next = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
    const double beta = (t - 1.0) / t_next;
    hipLaunchKernelGGL((k_fista_momentum<T>), dim3(nblk(n * R)), dim3(kVecBS), 0, s, n * R, beta, fb, fa, h);
    // F f^k into Fold, then it becomes the current product
    if ((rc = launch_forward<T>(pl, fb, nullptr, Fold, s))) return rc;
    std::swap(Fcur, Fold);
    std::swap(fa, fb);
    t = t_next;
    beta_prev = beta;
    if ((rc = check("fista iteration"))) return rc;
    if (tol > 0 && (it % 8 == 0 || it == max_iter)) {
      GT_HIP(hipMemcpyAsync(hstats.data(), stats, hstats.size() * sizeof(double), hipMemcpyDeviceToHost, s));
      GT_HIP(hipStreamSynchronize(s));
      bool all = true;
      for (int r = 0; r < R; ++r) {
        double dd = 0, nn = 0;
        for (int gi = 0; gi < ngroups; ++gi) {
          dd += hstats[((size_t)r * ngroups + gi) * 2];
          nn += hstats[((size_t)r * ngroups + gi) * 2 + 1];
        }
        rel[r] = nn > 0 ? std::sqrt(dd / nn) : std::sqrt(dd);
        if (rel[r] > tol) all = false;
      }
      if (all) {
        converged = true;
        break;
      }
    }
  }
  hipLaunchKernelGGL((k_copy<T>), dim3(nblk(n * R)), dim3(kVecBS), 0, s, n * R, fa, (C *)fhat);
  if ((rc = check("fista output"))) return rc;
  GT_HIP(hipMemcpyAsync(hstats.data(), stats, hstats.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  GT_HIP(hipStreamSynchronize(s));
  for (int r = 0; r < R; ++r) {
    double dd = 0, nn = 0;
    for (int gi = 0; gi < ngroups; ++gi) {
      dd += hstats[((size_t)r * ngroups + gi) * 2];
      nn += hstats[((size_t)r * ngroups + gi) * 2 + 1];
    }
    rel[r] = nn > 0 ? std::sqrt(dd / nn) : std::sqrt(dd);
    info[r].iters = std::min(it, max_iter);
    info[r].resid = rel[r];
    info[r].t_k = t;
    info[r].L = hL[r];
    int32_t fl = 0;
    if (tol > 0 && rel[r] <= tol) fl |= GT_SOLVE_CONVERGED;
    if (!converged) fl |= GT_SOLVE_MAX_ITER;
    if (capped[r]) fl |= GT_SOLVE_BACKTRACK_CAP;
    info[r].flags = fl;
  }
  (void)nchunk;
  return GT_OK;
}

// ---------------------------------------------------------------- sensitivity indices
// Global sensitivity indices (eq. gsi) by Parseval's identity: the squared L2 norm of ANOVA
// term u of the approximation is the sum of |fhat_{u,k}|^2 over the term's coefficients,
// and the variance is that sum over every term but the empty set.
// k_term_energy: one workgroup per (term, right-hand side), FP64 sum over the term's
// coefficients in a fixed order (strided per thread, then the block sum), into rho.
template <typename T>
__global__ __launch_bounds__(kVecBS) void k_term_energy(const cx_t<T> *__restrict__ fhat, int64_t ncoef,
                                                       const int64_t *__restrict__ goff, int nterms,
                                                       double *__restrict__ rho) {
  __shared__ double sh[kVecBS / 64 + 1];
  const int u = blockIdx.x, r = blockIdx.y;
  const cx_t<T> *f = fhat + (int64_t)r * ncoef;
  double e = 0;
  for (int64_t i = goff[u] + threadIdx.x; i < goff[u + 1]; i += blockDim.x) {
    const cx_t<T> c = f[i];
    e += (double)c.x * (double)c.x + (double)c.y * (double)c.y;
  }
  e = block_sum_all(e, sh);
  if (threadIdx.x == 0) rho[(int64_t)r * nterms + u] = e;
}

// k_term_gsi: one workgroup per right-hand side: the variance (terms 1 .. nterms-1, fixed
// order), then rho[u] = energy[u] / variance in place (0 for the empty set and for a zero
// variance).  Every energy is read before the block sum's barriers and overwritten after.
__global__ __launch_bounds__(kVecBS) void k_term_gsi(int nterms, double *__restrict__ rho) {
  __shared__ double sh[kVecBS / 64 + 1];
  double *q = rho + (int64_t)blockIdx.x * nterms;
  double v = 0;
  for (int u = 1 + threadIdx.x; u < nterms; u += blockDim.x) v += q[u];
  v = block_sum_all(v, sh);
  for (int u = threadIdx.x; u < nterms; u += blockDim.x) q[u] = (u > 0 && v > 0) ? q[u] / v : 0.0;
}

template <typename T>
int run_sensitivity(const int64_t *goff, int nterms, int64_t ncoef, int R, const void *fhat, double *rho,
                    hipStream_t s) {
  if (nterms <= 0) return GT_OK;
  hipLaunchKernelGGL((k_term_energy<T>), dim3(nterms, R), dim3(kVecBS), 0, s, (const cx_t<T> *)fhat, ncoef, goff,
                     nterms, rho);
  hipLaunchKernelGGL(k_term_gsi, dim3(R), dim3(kVecBS), 0, s, nterms, rho);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? GT_OK : hip_fail(e, "sensitivity kernels");
}

template int run_sensitivity<float>(const int64_t *, int, int64_t, int, const void *, double *, hipStream_t);
template int run_sensitivity<double>(const int64_t *, int, int64_t, int, const void *, double *, hipStream_t);
template int run_lsqr<float>(gt_plan *, const void *, const double *, const void *, int, double, void *, gt_solve_info *,
                             hipStream_t);
template int run_lsqr<double>(gt_plan *, const void *, const double *, const void *, int, double, void *,
                              gt_solve_info *, hipStream_t);
template int run_fista<float>(gt_plan *, const void *, const double *, const void *, int, double, double, double,
                              void *, gt_solve_info *, hipStream_t);
template int run_fista<double>(gt_plan *, const void *, const double *, const void *, int, double, double, double,
                               void *, gt_solve_info *, hipStream_t);
template int run_norm_estimate<float>(gt_plan *, int, double *, hipStream_t);
template int run_norm_estimate<double>(gt_plan *, int, double *, hipStream_t);

}  // namespace gt
