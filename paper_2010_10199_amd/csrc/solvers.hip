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
#include <mutex>
#include <string>
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

// State s = j R + r: damping value j (one per right-hand side when each r has its own
// lambda: J = 1, lambda index r) on right-hand side r, whose bidiagonalisation (alpha_r,
// beta_r) every j shares: the Golub-Kahan recurrences of A do not involve the damping,
// which enters only through the extra plane rotation of each step.
__device__ __forceinline__ double lsqr_lambda(const double *lambda, int s, int R, int path) {
  return path ? lambda[s / R] : lambda[s];
}

__global__ void k_lsqr_init(int S, int R, const double *__restrict__ alpha, const double *__restrict__ beta,
                            LsqrState *__restrict__ st) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S) return;
  const int r = i % R;
  LsqrState s{};
  s.alpha = alpha[r];
  s.beta = beta[r];
  s.rhobar = s.alpha;
  s.phibar = s.beta;
  s.normal = fabs(s.alpha * s.beta);
  s.normal0 = s.normal;
  s.done = (s.alpha == 0.0 || s.beta == 0.0) ? 1 : 0;
  s.iters = 0;
  st[i] = s;
}

__global__ void k_lsqr_step(int S, int R, int path, const double *__restrict__ lambda,
                            const double *__restrict__ alpha, const double *__restrict__ beta,
                            LsqrState *__restrict__ st) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S) return;
  const int r = i % R;
  LsqrState s = st[i];
  if (s.done) {
    s.cx = 0;
    s.cw = 0;
    st[i] = s;
    return;
  }
  const double a = alpha[r], b = beta[r];
  const double damp = sqrt(2.0 * lsqr_lambda(lambda, i, R, path));
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
  st[i] = s;
}

// x_s += cx_s w_s; w_s = v_r + cw_s w_s.  Grid (chunks, S).
template <typename T>
__global__ __launch_bounds__(kVecBS) void k_lsqr_xw(int64_t n, int R, const LsqrState *__restrict__ st,
                                                    const cx_t<T> *__restrict__ v, cx_t<T> *__restrict__ w,
                                                    cx_t<T> *__restrict__ x) {
  const int si = blockIdx.y, r = si % R;
  const double cx = st[si].cx, cw = st[si].cw;
  if (cx == 0.0 && cw == 0.0) return;
  const int64_t lo = (int64_t)blockIdx.x * kCoefChunk, hi = min(n, lo + kCoefChunk);
  for (int64_t i = lo + threadIdx.x; i < hi; i += kVecBS) {
    const int64_t k = (int64_t)si * n + i;
    const cx_t<T> wv = w[k], xv = x[k], vv = v[(int64_t)r * n + i];
    x[k] = mk<T>((T)(xv.x + cx * wv.x), (T)(xv.y + cx * wv.y));
    w[k] = mk<T>((T)(vv.x + cw * wv.x), (T)(vv.y + cw * wv.y));
  }
}

// w_s = v_r for every state (start of the recurrences).
template <typename T>
__global__ __launch_bounds__(kVecBS) void k_lsqr_wstart(int64_t n, int R, const cx_t<T> *__restrict__ v,
                                                        cx_t<T> *__restrict__ w) {
  const int si = blockIdx.y, r = si % R;
  const int64_t lo = (int64_t)blockIdx.x * kCoefChunk, hi = min(n, lo + kCoefChunk);
  for (int64_t i = lo + threadIdx.x; i < hi; i += kVecBS) w[(int64_t)si * n + i] = v[(int64_t)r * n + i];
}

template <typename T>
__global__ __launch_bounds__(kVecBS) void k_colscale(int64_t ncoef, const double *__restrict__ omega, T *__restrict__ cs,
                                                     int32_t *__restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * kVecBS + threadIdx.x;
  if (i >= ncoef) return;
  const double w = omega[i];
  if (!(w > 0.0) || !isfinite(w)) {
    atomicOr(bad, 1);
    if (cs) cs[i] = (T)1;
  } else if (cs) {
    cs[i] = (T)(1.0 / sqrt(w));
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
// Per right-hand side state of the device-resident FISTA iteration (all FP64).  A host
// step enqueues one trial of Algorithm algo:fista for every right-hand side; k_fista_decide
// then accepts the trial (the iteration advances) or, when the backtracking test fails,
// multiplies L by eta so that the next step retries the same h.
struct FistaState {
  double L;          // step constant of the current trial
  double t;          // t_k
  double beta;       // (t_{k-1} - 1) / t_k: h = f_k + beta (f_k - f_{k-1}), so F h from F f_k, F f_{k-1}
  double rel;        // relative step ||f_k - f_{k-1}|| / ||f_k|| of the last accepted iteration
  int32_t k;         // accepted iterations
  int32_t ninc;      // increases of L within the current iteration
  int32_t frozen;    // finished: max_iter reached or converged; no further updates
  int32_t accept;    // the current step's trial was accepted
  int32_t capped;    // an iteration reached the backtracking cap
  int32_t converged;
};

__global__ void k_fista_init(int R, const double *__restrict__ L0, FistaState *__restrict__ st) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  FistaState s{};
  s.L = L0[r];
  s.t = 1.0;
  st[r] = s;
}

// res = F h - y with F h = (1 + beta_r) F f_k - beta_r F f_{k-1} (F f_{k-1} unread when beta_r = 0).
template <typename T>
__global__ __launch_bounds__(kVecBS) void k_fista_resid(const WorkItem *__restrict__ items,
                                                        const FistaState *__restrict__ st,
                                                        const cx_t<T> *__restrict__ Fcur, const cx_t<T> *__restrict__ Fold,
                                                        const cx_t<T> *__restrict__ y, cx_t<T> *__restrict__ res) {
  const WorkItem it = items[blockIdx.x];
  const double beta = st[it.r].beta;
  for (int i = threadIdx.x; i < it.count; i += kVecBS) {
    const int64_t v = it.v0 + i;
    const cx_t<T> a = Fcur[v], c = y[v];
    double re = (1.0 + beta) * (double)a.x - (double)c.x, im = (1.0 + beta) * (double)a.y - (double)c.y;
    if (beta != 0.0) {
      const cx_t<T> b = Fold[v];
      re -= beta * (double)b.x;
      im -= beta * (double)b.y;
    }
    res[v] = mk<T>((T)re, (T)im);
  }
}

// t(xi) = sum_k w_k a_k xi^2 / (1 + xi w_k)^2 and its derivative (a_k = |z_k|^2).
struct GroupView {
  int64_t off, size;
};

// Proximal step on one (group, right-hand side): z = h - g / L_r, f_new = prox(z, lambda_r / L_r).
// stats[(r * ngroups + group) * 2 + {0,1}] = ||f_new - f_cur||^2, ||f_new||^2 over the group.
template <typename T>
__global__ __launch_bounds__(kVecBS) void k_fista_prox(int64_t ncoef, const int64_t *__restrict__ goff, int ngroups,
                                                       const double *__restrict__ lambda,
                                                       const FistaState *__restrict__ st,
                                                       const double *__restrict__ omega, const cx_t<T> *__restrict__ h,
                                                       const cx_t<T> *__restrict__ g, const cx_t<T> *__restrict__ fcur,
                                                       cx_t<T> *__restrict__ fnew, double *__restrict__ stats) {
  __shared__ double sh[kVecBS / 64 + 1];
  const int grp = blockIdx.x, r = blockIdx.y;
  if (st[r].frozen) return;   // uniform per workgroup
  const int64_t lo = goff[grp], hi = goff[grp + 1];
  const int64_t base = (int64_t)r * ncoef;
  const double L = st[r].L;
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
    const double w = omega ? omega[k] : 1.0;
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
        const double w = omega[k], a = zr * zr + zi * zi;
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
        const double w = omega[k], a = zr * zr + zi * zi;
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
        const double w = omega[k], a = zr * zr + zi * zi;
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
      const double sc = omega ? 1.0 / (1.0 + xi * omega[k]) : scale;
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

// One workgroup per right-hand side: the relative step from the prox statistics (sums over
// the groups in a fixed order), then the trial's verdict.  With backtracking the trial is
// accepted when ||F(f - h)||^2 <= L ||f - h||^2 (the algorithm's test in an equivalent
// form); otherwise L grows by eta and the next step retries, except after `cap` increases
// within one iteration, when the trial is taken as it is and the cap is flagged.
__global__ __launch_bounds__(kVecBS) void k_fista_decide(int ngroups, const double *__restrict__ stats,
                                                         const double *__restrict__ nd, const double *__restrict__ nFd,
                                                         int backtrack, double eta, int cap, int max_iter, double tol,
                                                         FistaState *__restrict__ st) {
  __shared__ double sh[kVecBS / 64 + 1];
  const int r = blockIdx.x;
  if (st[r].frozen) {   // uniform per workgroup
    if (threadIdx.x == 0) st[r].accept = 0;
    return;
  }
  double dd = 0, nn = 0;
  for (int gi = threadIdx.x; gi < ngroups; gi += kVecBS) {
    dd += stats[((int64_t)r * ngroups + gi) * 2];
    nn += stats[((int64_t)r * ngroups + gi) * 2 + 1];
  }
  dd = block_sum_all(dd, sh);
  nn = block_sum_all(nn, sh);
  if (threadIdx.x != 0) return;
  FistaState s = st[r];
  const bool pass = !backtrack || !(nFd[r] > s.L * nd[r]);
  if (!pass && s.ninc < cap) {
    s.L *= eta;
    s.ninc += 1;
    s.accept = 0;
    st[r] = s;
    return;
  }
  if (!pass) s.capped = 1;
  s.accept = 1;
  s.ninc = 0;
  s.k += 1;
  const double t_next = 0.5 * (1.0 + sqrt(1.0 + 4.0 * s.t * s.t));
  s.beta = (s.t - 1.0) / t_next;
  s.t = t_next;
  s.rel = nn > 0 ? sqrt(dd / nn) : sqrt(dd);
  if (tol > 0 && s.rel <= tol) {
    s.converged = 1;
    s.frozen = 1;
  }
  if (s.k >= max_iter) s.frozen = 1;
  st[r] = s;
}

// Accepted trial, coefficient space: h = f_new + beta (f_new - f_cur), f_cur = f_new.
template <typename T>
__global__ __launch_bounds__(kVecBS) void k_fista_apply_c(int64_t n, const FistaState *__restrict__ st,
                                                          const cx_t<T> *__restrict__ fnew, cx_t<T> *__restrict__ fcur,
                                                          cx_t<T> *__restrict__ h) {
  const int r = blockIdx.y;
  if (!st[r].accept) return;
  const double beta = st[r].beta;
  const int64_t lo = (int64_t)blockIdx.x * kCoefChunk, hi = min(n, lo + kCoefChunk);
  for (int64_t i = lo + threadIdx.x; i < hi; i += kVecBS) {
    const int64_t k = (int64_t)r * n + i;
    const cx_t<T> a = fnew[k], b = fcur[k];
    h[k] = mk<T>((T)((double)a.x + beta * ((double)a.x - b.x)), (T)((double)a.y + beta * ((double)a.y - b.y)));
    fcur[k] = a;
  }
}

// Accepted trial, sample space: F f_{k-1} = F f_k, F f_k = F f_new.
template <typename T>
__global__ __launch_bounds__(kVecBS) void k_fista_apply_v(const WorkItem *__restrict__ items,
                                                          const FistaState *__restrict__ st,
                                                          const cx_t<T> *__restrict__ Fnew, cx_t<T> *__restrict__ Fcur,
                                                          cx_t<T> *__restrict__ Fold) {
  const WorkItem it = items[blockIdx.x];
  if (!st[it.r].accept) return;
  for (int i = threadIdx.x; i < it.count; i += kVecBS) {
    const int64_t v = it.v0 + i;
    Fold[v] = Fcur[v];
    Fcur[v] = Fnew[v];
  }
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

__global__ void k_zero_flag(int32_t *f) { *f = 0; }

__global__ void k_neg(int R, const double *__restrict__ a, double *__restrict__ na) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < R) na[r] = -a[r];
}

unsigned nblk(int64_t total) { return (unsigned)((total + kVecBS - 1) / kVecBS); }

int check(const char *what) {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? GT_OK : hip_fail(e, what);
}

// Device scratch of one solver call.  By default every buffer is its own allocation, freed
// when the call ends.  In carve mode the buffers are consecutive 256-byte aligned pieces of
// one caller-provided region (nothing is allocated; a request past its end fails), and in
// measure mode nothing is handed out and `used` totals the bytes the buffers would take.
struct Scratch {
  enum Mode { Alloc, Carve, Measure };
  Mode mode = Alloc;
  unsigned char *base = nullptr;
  size_t cap = 0, used = 0;
  std::vector<void *> ptrs;
  Scratch() = default;
  Scratch(Mode m, void *b, size_t c) : mode(m), base((unsigned char *)b), cap(c) {}
  Scratch(const Scratch &) = delete;
  Scratch &operator=(const Scratch &) = delete;
  ~Scratch() {
    for (void *p : ptrs) dev_free(p, nullptr);
  }
  template <typename P>
  int get(P **p, size_t bytes) {
    bytes = std::max<size_t>(bytes, 16);
    const size_t need = (bytes + 255) & ~size_t(255);
    if (mode == Measure) {
      used += need;
      *p = nullptr;
      return GT_OK;
    }
    if (mode == Carve) {
      if (used + need > cap) return fail(GT_EINVAL, "work buffers exceed the fixed scratch region");
      *p = (P *)(base + used);
      used += need;
      return GT_OK;
    }
    void *q = nullptr;
    int rc = dev_alloc(&q, bytes, nullptr);
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
// Column scaling 1 / sqrt(omega) (device, T) from the FP64 weights, with the weights checked.
template <typename T>
static int weight_scale(const double *omega, int64_t n, Scratch &sc, T **cs, hipStream_t s) {
  int32_t *bad = nullptr;
  int rc;
  if ((rc = sc.get(&bad, sizeof(int32_t)))) return rc;
  if (cs && (rc = sc.get(cs, n * sizeof(T)))) return rc;
  hipLaunchKernelGGL(k_zero_flag, dim3(1), dim3(1), 0, s, bad);
  hipLaunchKernelGGL((k_colscale<T>), dim3(nblk(n)), dim3(kVecBS), 0, s, n, omega, cs ? *cs : (T *)nullptr, bad);
  int32_t hbad = 0;
  GT_HIP(hipMemcpyAsync(&hbad, bad, sizeof(hbad), hipMemcpyDeviceToHost, s));
  GT_HIP(hipStreamSynchronize(s));
  if (hbad) return fail(GT_EINVAL, "weights must be finite and > 0");
  return GT_OK;
}

// J damping values per right-hand side (path: lambda[j] for every r, J = nlam; otherwise
// J = 1 and lambda[r]); x, w and the rotations per state s = j R + r, everything else per r.
template <typename T>
static int lsqr_core(gt_plan *pl, const void *y, int nlam, bool path, const double *lambda, const double *omega,
                     int max_iter, double tol, void *fhat, gt_solve_info *info, hipStream_t s) {
  using C = cx_t<T>;
  const int R = pl->R, J = path ? nlam : 1, S = J * R;
  const int64_t V = pl->Vtot, n = pl->ncoef;
  Scratch sc;
  C *u, *v, *w, *x, *tV, *tI;
  double *alpha, *beta, *ialpha, *ibeta, *dlam;
  LsqrState *st;
  T *cs = nullptr;
  int rc;
  if ((rc = sc.get(&u, V * sizeof(C))) || (rc = sc.get(&tV, V * sizeof(C))) || (rc = sc.get(&v, n * R * sizeof(C))) ||
      (rc = sc.get(&w, n * S * sizeof(C))) || (rc = sc.get(&x, n * S * sizeof(C))) ||
      (rc = sc.get(&tI, n * R * sizeof(C))) || (rc = sc.get(&alpha, R * sizeof(double))) ||
      (rc = sc.get(&beta, R * sizeof(double))) || (rc = sc.get(&ialpha, R * sizeof(double))) ||
      (rc = sc.get(&ibeta, R * sizeof(double))) || (rc = sc.get(&dlam, (path ? J : R) * sizeof(double))) ||
      (rc = sc.get(&st, S * sizeof(LsqrState))))
    return rc;
  Norms<T> nm{pl};
  if ((rc = nm.init(sc))) return rc;
  GT_HIP(hipMemcpyAsync(dlam, lambda, (path ? J : R) * sizeof(double), hipMemcpyHostToDevice, s));
  if (omega && (rc = weight_scale<T>(omega, n, sc, &cs, s))) return rc;
  const unsigned nchunk = (unsigned)nm.nchunk;
  // beta_1 u_1 = y
  if ((rc = nm.v_axpby((const C *)y, nullptr, nullptr, nullptr, u, beta, ibeta, s))) return rc;
  hipLaunchKernelGGL((k_v_scale<T>), dim3((unsigned)pl->gitems.size()), dim3(kVecBS), 0, s, pl->d_gitems, ibeta, u);
  // alpha_1 v_1 = A^H u_1
  if ((rc = launch_adjoint<T>(pl, u, cs, v, s))) return rc;
  if ((rc = nm.c_axpby(v, nullptr, nullptr, nullptr, v, alpha, ialpha, s))) return rc;
  hipLaunchKernelGGL((k_c_scale<T>), dim3(nchunk, R), dim3(kVecBS), 0, s, n, ialpha, v);
  hipLaunchKernelGGL((k_lsqr_wstart<T>), dim3(nchunk, S), dim3(kVecBS), 0, s, n, R, (const C *)v, w);
  hipLaunchKernelGGL((k_c_fill<T>), dim3(nblk(n * S)), dim3(kVecBS), 0, s, n * S, x);
  hipLaunchKernelGGL(k_lsqr_init, dim3((S + 63) / 64), dim3(64), 0, s, S, R, alpha, beta, st);
  if ((rc = check("lsqr init"))) return rc;
  // -alpha and -beta for the axpby kernels
  double *nalpha, *nbeta;
  if ((rc = sc.get(&nalpha, R * sizeof(double))) || (rc = sc.get(&nbeta, R * sizeof(double)))) return rc;
  std::vector<LsqrState> hst(S);
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
    // rotations, x and w per state
    hipLaunchKernelGGL(k_lsqr_step, dim3((S + 63) / 64), dim3(64), 0, s, S, R, path ? 1 : 0, (const double *)dlam,
                       (const double *)alpha, (const double *)beta, st);
    hipLaunchKernelGGL((k_lsqr_xw<T>), dim3(nchunk, S), dim3(kVecBS), 0, s, n, R, (const LsqrState *)st,
                       (const C *)v, w, x);
    if ((rc = check("lsqr iteration"))) return rc;
    if (tol > 0 && (it % 8 == 0 || it == max_iter)) {
      GT_HIP(hipMemcpyAsync(hst.data(), st, S * sizeof(LsqrState), hipMemcpyDeviceToHost, s));
      GT_HIP(hipStreamSynchronize(s));
      bool all = true;
      for (int q = 0; q < S; ++q)
        if (!(hst[q].done || hst[q].normal <= tol * hst[q].normal0)) all = false;
      if (all) {
        converged = true;
        break;
      }
    }
  }
  // fhat = W^{-1/2} x
  hipLaunchKernelGGL((k_c_mul_colscale<T>), dim3(nchunk, S), dim3(kVecBS), 0, s, n, (const T *)cs, x, (C *)fhat);
  if ((rc = check("lsqr output"))) return rc;
  GT_HIP(hipMemcpyAsync(hst.data(), st, S * sizeof(LsqrState), hipMemcpyDeviceToHost, s));
  GT_HIP(hipStreamSynchronize(s));
  for (int q = 0; q < S; ++q) {
    info[q].iters = hst[q].iters;
    info[q].resid = hst[q].normal;
    info[q].t_k = hst[q].phibar;
    info[q].L = 0;
    int32_t fl = 0;
    if (hst[q].done) fl |= GT_SOLVE_BREAKDOWN;
    if (tol > 0 && (hst[q].done || hst[q].normal <= tol * hst[q].normal0)) fl |= GT_SOLVE_CONVERGED;
    if (!converged && it > max_iter) fl |= GT_SOLVE_MAX_ITER;
    info[q].flags = fl;
  }
  return GT_OK;
}

template <typename T>
int run_lsqr(gt_plan *pl, const void *y, const double *lambda, const double *omega, int max_iter, double tol, void *fhat,
             gt_solve_info *info, hipStream_t s) {
  return lsqr_core<T>(pl, y, 1, false, lambda, omega, max_iter, tol, fhat, info, s);
}

template <typename T>
int run_lsqr_path(gt_plan *pl, const void *y, int nlam, const double *lambda, const double *omega, int max_iter,
                  double tol, void *path, gt_solve_info *info, hipStream_t s) {
  return lsqr_core<T>(pl, y, nlam, true, lambda, omega, max_iter, tol, path, info, s);
}

// ================================================================== power iteration
// Rayleigh-quotient estimate of ||F||_2^2 per right-hand side from the all-ones start.
template <typename T>
struct PowerBuf {
  cx_t<T> *v = nullptr, *wv = nullptr, *tV = nullptr;
  double *nrm = nullptr, *inv = nullptr, *dot = nullptr, *partV = nullptr, *partC = nullptr;
  int get(const gt_plan *pl, Scratch &sc) {
    const int R = pl->R;
    const int64_t V = pl->Vtot, n = pl->ncoef;
    const int64_t nchunk = (n + kCoefChunk - 1) / kCoefChunk;
    using C = cx_t<T>;
    int rc;
    if ((rc = sc.get(&v, n * R * sizeof(C))) || (rc = sc.get(&wv, n * R * sizeof(C))) ||
        (rc = sc.get(&tV, V * sizeof(C))) || (rc = sc.get(&nrm, R * sizeof(double))) ||
        (rc = sc.get(&inv, R * sizeof(double))) || (rc = sc.get(&dot, R * sizeof(double))) ||
        (rc = sc.get(&partV, sizeof(double) * std::max<size_t>(1, pl->gitems.size()))) ||
        (rc = sc.get(&partC, sizeof(double) * (size_t)nchunk * R)))
      return rc;
    return GT_OK;
  }
};

// est_host receives the first ncopy right-hand sides' estimates (ncopy <= R).
template <typename T>
static int power_run(gt_plan *pl, int iters, PowerBuf<T> &b, double *est_host, int ncopy, hipStream_t s) {
  const int R = pl->R;
  const int64_t n = pl->ncoef;
  Norms<T> nm{pl};
  nm.partV = b.partV;
  nm.partC = b.partC;
  nm.nchunk = (int)((n + kCoefChunk - 1) / kCoefChunk);
  const unsigned nchunk = (unsigned)nm.nchunk;
  cx_t<T> *v = b.v, *wv = b.wv;
  int rc;
  // v = ones / sqrt(n)
  hipLaunchKernelGGL((k_c_fill_value<T>), dim3(nblk(n * R)), dim3(kVecBS), 0, s, n * R, (T)(1.0 / std::sqrt((double)n)),
                     v);
  for (int k = 0; k < iters; ++k) {
    if ((rc = launch_forward<T>(pl, v, nullptr, b.tV, s))) return rc;
    if ((rc = launch_adjoint<T>(pl, b.tV, nullptr, wv, s))) return rc;
    hipLaunchKernelGGL((k_c_dot<T>), dim3(nchunk, R), dim3(kVecBS), 0, s, n, v, wv, b.partC);
    hipLaunchKernelGGL(k_finalize, dim3(R), dim3(kVecBS), 0, s, b.partC, nullptr, (int)nchunk, R, b.dot, nullptr,
                       nullptr);
    if ((rc = nm.c_axpby(wv, nullptr, nullptr, nullptr, wv, b.nrm, b.inv, s))) return rc;
    hipLaunchKernelGGL((k_c_scale<T>), dim3(nchunk, R), dim3(kVecBS), 0, s, n, b.inv, wv);
    std::swap(v, wv);
    if ((rc = check("power iteration"))) return rc;
  }
  GT_HIP(hipMemcpyAsync(est_host, b.dot, std::min(ncopy, R) * sizeof(double), hipMemcpyDeviceToHost, s));
  GT_HIP(hipStreamSynchronize(s));
  return GT_OK;
}

template <typename T>
static int power_iter(gt_plan *pl, int iters, double *est_host, hipStream_t s) {
  Scratch sc;
  PowerBuf<T> b;
  if (int rc = b.get(pl, sc)) return rc;
  return power_run<T>(pl, iters, b, est_host, pl->R, s);
}

template <typename T>
int run_norm_estimate(gt_plan *pl, int iters, double *out, hipStream_t s) {
  std::vector<double> est(pl->R);
  int rc = power_iter<T>(pl, iters, est.data(), s);
  if (rc) return rc;
  *out = est[0];
  return GT_OK;
}

// The same estimate with every work buffer carved from a fixed device region; region NULL
// only measures (*need = bytes the buffers take).  Allocates nothing, device or host.
template <typename T>
int run_norm_estimate_region(gt_plan *pl, int iters, void *region, size_t cap, size_t *need, double *out,
                             hipStream_t s) {
  {
    Scratch m(Scratch::Measure, nullptr, 0);
    PowerBuf<T> b;
    (void)b.get(pl, m);
    *need = m.used;
  }
  if (!region) return GT_OK;
  if (*need > cap)
    return fail(GT_EINVAL, "the work buffers of this plan (" + std::to_string(*need) +
                               " bytes) exceed the fixed scratch region (" + std::to_string(cap) + " bytes)");
  Scratch sc(Scratch::Carve, region, cap);
  PowerBuf<T> b;
  if (int rc = b.get(pl, sc)) return rc;
  return power_run<T>(pl, iters, b, out, 1, s);
}

// ================================================================== FISTA
// Algorithm algo:fista for R right-hand sides, state on the device (FistaState).  Each host
// step enqueues one trial for every right-hand side:
//   res = F h - y  (F h by linearity from F f_k and F f_{k-1});  g = F^H res;
//   f_new = p_L(h - g / L) (k_fista_prox);  with backtracking: d = f_new - h, ||d||^2 and
//   ||F d||^2;  F f_new;  verdict (k_fista_decide);  accepted: h, f_k, F f_k, F f_{k-1} advance.
// A rejected trial only raises L, so the next step redoes the same h.  The host reads the
// state once per enqueued batch: exactly max_iter steps for the constant step without a
// tolerance; otherwise batches of (max_iter - the fewest accepted iterations) steps, or of at
// most 8 steps when a tolerance is set, until every right-hand side is frozen.  With backtracking
// a step costs one adjoint and two forward transforms, without it one of each.
template <typename T>
struct FistaWork {
  cx_t<T> *fa = nullptr, *fb = nullptr, *h = nullptr, *g = nullptr, *delta = nullptr;
  cx_t<T> *Fcur = nullptr, *Fold = nullptr, *Fnew = nullptr, *res = nullptr, *Fd = nullptr;
  double *dlam = nullptr, *dL = nullptr, *stats = nullptr, *nd = nullptr, *nFd = nullptr;
  int64_t *goff = nullptr;
  FistaState *st = nullptr;
  Norms<T> nm{nullptr};
  int get(gt_plan *pl, Scratch &sc, bool backtrack) {
    using C = cx_t<T>;
    const int R = pl->R, ngroups = pl->nterms;
    const int64_t V = pl->Vtot, n = pl->ncoef;
    int rc;
    if ((rc = sc.get(&fa, n * R * sizeof(C))) || (rc = sc.get(&fb, n * R * sizeof(C))) ||
        (rc = sc.get(&h, n * R * sizeof(C))) || (rc = sc.get(&g, n * R * sizeof(C))) ||
        (rc = sc.get(&Fcur, V * sizeof(C))) || (rc = sc.get(&Fold, V * sizeof(C))) ||
        (rc = sc.get(&Fnew, V * sizeof(C))) || (rc = sc.get(&res, V * sizeof(C))) ||
        (rc = sc.get(&dlam, R * sizeof(double))) || (rc = sc.get(&dL, R * sizeof(double))) ||
        (rc = sc.get(&stats, (size_t)R * ngroups * 2 * sizeof(double))) ||
        (rc = sc.get(&goff, (size_t)(ngroups + 1) * sizeof(int64_t))) ||
        (rc = sc.get(&st, R * sizeof(FistaState))))
      return rc;
    if (backtrack && ((rc = sc.get(&delta, n * R * sizeof(C))) || (rc = sc.get(&Fd, V * sizeof(C))) ||
                      (rc = sc.get(&nd, R * sizeof(double))) || (rc = sc.get(&nFd, R * sizeof(double)))))
      return rc;
    nm.pl = pl;
    return nm.init(sc);
  }
};

static constexpr int kBacktrackCap = 30;

// One FISTA solve from f0 (device, R x |I|) into out (may equal f0): lambda and L0 host, R each.
template <typename T>
static int fista_solve(gt_plan *pl, FistaWork<T> &w, const void *y, const double *lambda, const double *omega,
                       int max_iter, const double *L0, double eta, double tol, const void *f0, void *out,
                       gt_solve_info *info, hipStream_t s) {
  using C = cx_t<T>;
  const int R = pl->R, ngroups = pl->nterms;
  const int64_t n = pl->ncoef;
  const bool backtrack = eta > 1.0;
  const unsigned ngi = (unsigned)pl->gitems.size();
  const unsigned nchunk = (unsigned)w.nm.nchunk;
  GT_HIP(hipMemcpyAsync(w.dlam, lambda, R * sizeof(double), hipMemcpyHostToDevice, s));
  GT_HIP(hipMemcpyAsync(w.dL, L0, R * sizeof(double), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_fista_init, dim3((R + 63) / 64), dim3(64), 0, s, R, (const double *)w.dL, w.st);
  // f_0, h_1 = f_0, F f_0
  hipLaunchKernelGGL((k_copy<T>), dim3(nblk(n * R)), dim3(kVecBS), 0, s, n * R, (const C *)f0, w.fa);
  hipLaunchKernelGGL((k_copy<T>), dim3(nblk(n * R)), dim3(kVecBS), 0, s, n * R, (const C *)f0, w.h);
  int rc;
  if ((rc = launch_forward<T>(pl, w.fa, nullptr, w.Fcur, s))) return rc;
  auto step = [&]() -> int {
    int e;
    hipLaunchKernelGGL((k_fista_resid<T>), dim3(ngi), dim3(kVecBS), 0, s, pl->d_gitems, (const FistaState *)w.st,
                       (const C *)w.Fcur, (const C *)w.Fold, (const C *)y, w.res);
    if ((e = launch_adjoint<T>(pl, w.res, nullptr, w.g, s))) return e;
    hipLaunchKernelGGL((k_fista_prox<T>), dim3(ngroups, R), dim3(kVecBS), 0, s, n, (const int64_t *)w.goff, ngroups,
                       (const double *)w.dlam, (const FistaState *)w.st, omega, (const C *)w.h, (const C *)w.g,
                       (const C *)w.fa, w.fb, w.stats);
    if (backtrack) {
      hipLaunchKernelGGL((k_sub<T>), dim3(nblk(n * R)), dim3(kVecBS), 0, s, n * R, (const C *)w.fb, (const C *)w.h,
                         w.delta);
      if ((e = w.nm.c_axpby(w.delta, nullptr, nullptr, nullptr, w.delta, nullptr, nullptr, s, w.nd))) return e;
      if ((e = launch_forward<T>(pl, w.delta, nullptr, w.Fd, s))) return e;
      hipLaunchKernelGGL((k_v_axpby_norm<T>), dim3(ngi), dim3(kVecBS), 0, s, pl->d_gitems, (const C *)w.Fd,
                         (const double *)nullptr, (const C *)nullptr, (const double *)nullptr, w.Fd, w.nm.partV);
      hipLaunchKernelGGL(k_finalize, dim3(R), dim3(kVecBS), 0, s, (const double *)w.nm.partV, pl->d_gitem_begin, 0, R,
                         w.nFd, (double *)nullptr, (double *)nullptr);
    }
    if ((e = launch_forward<T>(pl, w.fb, nullptr, w.Fnew, s))) return e;
    hipLaunchKernelGGL(k_fista_decide, dim3(R), dim3(kVecBS), 0, s, ngroups, (const double *)w.stats,
                       (const double *)w.nd, (const double *)w.nFd, backtrack ? 1 : 0, eta, kBacktrackCap, max_iter,
                       tol, w.st);
    hipLaunchKernelGGL((k_fista_apply_c<T>), dim3(nchunk, R), dim3(kVecBS), 0, s, n, (const FistaState *)w.st,
                       (const C *)w.fb, w.fa, w.h);
    hipLaunchKernelGGL((k_fista_apply_v<T>), dim3(ngi), dim3(kVecBS), 0, s, pl->d_gitems, (const FistaState *)w.st,
                       (const C *)w.Fnew, w.Fcur, w.Fold);
    return check("fista step");
  };
  std::vector<FistaState> hs(R);
  auto read_state = [&]() -> int {
    GT_HIP(hipMemcpyAsync(hs.data(), w.st, R * sizeof(FistaState), hipMemcpyDeviceToHost, s));
    GT_HIP(hipStreamSynchronize(s));
    return GT_OK;
  };
  int64_t steps = 0;
  const int64_t step_cap = (int64_t)max_iter * (kBacktrackCap + 1);   // every step advances some state
  int min_k = 0;
  while (true) {
    int batch = max_iter - min_k;
    if (tol > 0) batch = std::min(batch, 8);
    batch = (int)std::min<int64_t>(std::max(batch, 1), step_cap - steps);
    for (int b = 0; b < batch; ++b)
      if ((rc = step())) return rc;
    steps += batch;
    if ((rc = read_state())) return rc;
    bool all = true;
    min_k = max_iter;
    for (int r = 0; r < R; ++r)
      if (!hs[r].frozen) {
        all = false;
        min_k = std::min(min_k, hs[r].k);
      }
    if (all || steps >= step_cap) break;
  }
  hipLaunchKernelGGL((k_copy<T>), dim3(nblk(n * R)), dim3(kVecBS), 0, s, n * R, (const C *)w.fa, (C *)out);
  if ((rc = check("fista output"))) return rc;
  GT_HIP(hipStreamSynchronize(s));
  for (int r = 0; r < R; ++r) {
    info[r].iters = hs[r].k;
    info[r].resid = hs[r].rel;
    info[r].t_k = hs[r].t;
    info[r].L = hs[r].L;
    int32_t fl = 0;
    if (hs[r].converged) fl |= GT_SOLVE_CONVERGED;
    if (hs[r].k >= max_iter && !hs[r].converged) fl |= GT_SOLVE_MAX_ITER;
    if (hs[r].capped) fl |= GT_SOLVE_BACKTRACK_CAP;
    info[r].flags = fl;
  }
  return GT_OK;
}

// Shared set-up of the FISTA entry points: weights checked, group offsets uploaded, the step
// constants L0 (per right-hand side) chosen.
template <typename T>
static int fista_setup(gt_plan *pl, FistaWork<T> &w, Scratch &sc, const double *omega, double L, double eta,
                       std::vector<double> &L0, hipStream_t s) {
  const int ngroups = pl->nterms;
  int rc;
  if ((rc = w.get(pl, sc, eta > 1.0))) return rc;
  if (omega && (rc = weight_scale<T>(omega, pl->ncoef, sc, (T **)nullptr, s))) return rc;
  std::vector<int64_t> hoff(ngroups + 1);
  for (int i = 0; i < ngroups; ++i) hoff[i] = pl->ext_off[i];
  hoff[ngroups] = pl->ncoef;
  GT_HIP(hipMemcpyAsync(w.goff, hoff.data(), hoff.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
  GT_HIP(hipStreamSynchronize(s));   // hoff is a host temporary
  L0.assign(pl->R, L);
  if (!(L > 0)) {
    std::vector<double> est(pl->R);
    if ((rc = power_iter<T>(pl, 50, est.data(), s))) return rc;
    for (int r = 0; r < pl->R; ++r) L0[r] = 1.05 * est[r];
  }
  for (int r = 0; r < pl->R; ++r)
    if (!(L0[r] > 0) || !std::isfinite(L0[r])) return fail(GT_EINVAL, "step constant L must be > 0");
  return GT_OK;
}

template <typename T>
int run_fista(gt_plan *pl, const void *y, const double *lambda, const double *omega, int max_iter, double L, double eta,
              double tol, void *fhat, gt_solve_info *info, hipStream_t s) {
  Scratch sc;
  FistaWork<T> w;
  std::vector<double> L0;
  if (int rc = fista_setup<T>(pl, w, sc, omega, L, eta, L0, s)) return rc;
  return fista_solve<T>(pl, w, y, lambda, omega, max_iter, L0.data(), eta, tol, fhat, fhat, info, s);
}

// The warm-started path over lambda[0..nlam-1] (every right-hand side takes lambda[j] at
// stage j): stage 0 starts from f0 (NULL: zero), each later stage from the previous
// solution; every stage restarts t_1 = 1 and the step constant at L0.
template <typename T>
int run_fista_path(gt_plan *pl, const void *y, int nlam, const double *lambda, const double *omega, int max_iter,
                   double L, double eta, double tol, const void *f0, void *path, gt_solve_info *info, hipStream_t s) {
  using C = cx_t<T>;
  const int R = pl->R;
  const int64_t nR = pl->ncoef * R;
  Scratch sc;
  FistaWork<T> w;
  std::vector<double> L0;
  int rc;
  if ((rc = fista_setup<T>(pl, w, sc, omega, L, eta, L0, s))) return rc;
  C *zero = nullptr;
  if (!f0) {
    if ((rc = sc.get(&zero, nR * sizeof(C)))) return rc;
    hipLaunchKernelGGL((k_c_fill<T>), dim3(nblk(nR)), dim3(kVecBS), 0, s, nR, zero);
  }
  std::vector<double> lam(R);
  for (int j = 0; j < nlam; ++j) {
    std::fill(lam.begin(), lam.end(), lambda[j]);
    const void *start = j == 0 ? (f0 ? f0 : (const void *)zero) : (const void *)((const C *)path + (j - 1) * nR);
    if ((rc = fista_solve<T>(pl, w, y, lam.data(), omega, max_iter, L0.data(), eta, tol, start,
                             (C *)path + j * nR, info + (size_t)j * R, s)))
      return rc;
  }
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

// ---------------------------------------------------------------- allocation-free work region
// A fixed device array for callers that cannot allocate (gt_plan_norm_estimate_noalloc): every
// device holds its own copy for the life of the process.  Host code never uses the array's
// name as an address; the device address comes from hipGetSymbolAddress, once per device,
// with that device current.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

int run_norm_estimate_noalloc(gt_plan *pl, int iters, double *out, hipStream_t s) {
  int dev = 0;
  GT_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(GT_EUNSUPPORTED, "device index beyond the scratch table");
  void *region = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      void *p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
      if (!p) return fail(GT_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
      g_scratch_ptr[dev] = p;
    }
    region = g_scratch_ptr[dev];
  }
  size_t need = 0;
  return pl->dtype == GT_C64 ? run_norm_estimate_region<float>(pl, iters, region, kNoAllocScratchBytes, &need, out, s)
                             : run_norm_estimate_region<double>(pl, iters, region, kNoAllocScratchBytes, &need, out, s);
}

template int run_sensitivity<float>(const int64_t *, int, int64_t, int, const void *, double *, hipStream_t);
template int run_sensitivity<double>(const int64_t *, int, int64_t, int, const void *, double *, hipStream_t);
template int run_lsqr<float>(gt_plan *, const void *, const double *, const double *, int, double, void *,
                             gt_solve_info *, hipStream_t);
template int run_lsqr<double>(gt_plan *, const void *, const double *, const double *, int, double, void *,
                              gt_solve_info *, hipStream_t);
template int run_lsqr_path<float>(gt_plan *, const void *, int, const double *, const double *, int, double, void *,
                                  gt_solve_info *, hipStream_t);
template int run_lsqr_path<double>(gt_plan *, const void *, int, const double *, const double *, int, double, void *,
                                   gt_solve_info *, hipStream_t);
template int run_fista<float>(gt_plan *, const void *, const double *, const double *, int, double, double, double,
                              void *, gt_solve_info *, hipStream_t);
template int run_fista<double>(gt_plan *, const void *, const double *, const double *, int, double, double, double,
                               void *, gt_solve_info *, hipStream_t);
template int run_fista_path<float>(gt_plan *, const void *, int, const double *, const double *, int, double, double,
                                   double, const void *, void *, gt_solve_info *, hipStream_t);
template int run_fista_path<double>(gt_plan *, const void *, int, const double *, const double *, int, double, double,
                                    double, const void *, void *, gt_solve_info *, hipStream_t);
template int run_norm_estimate<float>(gt_plan *, int, double *, hipStream_t);
template int run_norm_estimate<double>(gt_plan *, int, double *, hipStream_t);
template int run_norm_estimate_region<float>(gt_plan *, int, void *, size_t, size_t *, double *, hipStream_t);
template int run_norm_estimate_region<double>(gt_plan *, int, void *, size_t, size_t *, double *, hipStream_t);

}  // namespace gt
