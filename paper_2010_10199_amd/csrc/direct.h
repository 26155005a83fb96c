// Direct sums of the terms of one order, without window or FFT grid: the product of
// Definition def:skatoons written out,
//   forward  f_r(x_v) += sum_{k in I_u} fhat_{r,k} e^{2 pi i k . x_{v,u}}
//   adjoint  fhat_{r,k} = sum_v y_{r,v} e^{-2 pi i k . x_{v,u}}
// as dense contractions on 16x16x4 MFMA.  For a small group (|I_u| = (N - 1)^{|u|} against
// the window's (2m)^{|u|} points per node, e.g. N = 6 in three dimensions: 125 against 512 at
// m = 4, 4096 at m = 8) with several right-hand sides these take fewer operations than the
// window path, and they are exact up to rounding.  Shared nodes only (one node set, R <= 16
// right-hand sides as the columns of the contraction).
//
// Phases: per node, frequency and axis of the term from sincospi of 2 k x (the last axis of
// order 3 by repeated multiplication along its band k = -N/2..-1, 1..N/2-1), kept in LDS as
// described above k_direct_fwd; the phase of a frequency of the group is the product over
// its axes (frequencies row-major over the axes, last axis fastest, as the coefficient vector
// orders them).
//
// MFMA operands (lane l supplies A[l%16][l/16] and B[l/16][l%16]; see Mfma in spread.h),
// real form of the complex products:
//   forward:  rows = 16 nodes, K = (frequency kf, part p of the phase), columns = (r, part c of f);
//             f_re += ph_re F_re - ph_im F_im,  f_im += ph_re F_im + ph_im F_re,
//             so B[(kf,p)][(r,c)] = F_re if p == c, F_im if (p,c) = (0,1), -F_im if (1,0).
//             K slot q of step s holds kf = 2s + q/2, p = q%2.
//   adjoint:  rows = (kf, part c of fhat), K = (node v, part p of y), columns = r;
//             fhat_re += ph_re y_re + ph_im y_im,  fhat_im += ph_re y_im - ph_im y_re,
//             so A[(kf,c)][(v,p)] = ph_re if p == c, ph_im if (c,p) = (0,1), -ph_im if (1,0).
//             K slot q of step s holds v = 2s + q/2, p = q%2.
#pragma once

#include "spread.h"

namespace gt {

struct DirectArgs {
  int32_t K;       // frequencies per axis, N - 1
  int32_t G;       // frequencies of a group, K^order
  int32_t half;    // N / 2
  int32_t R;       // right-hand sides (<= 16)
  int64_t M;       // nodes
  int64_t ncoef;   // coefficient stride of one right-hand side
};

__device__ __forceinline__ void sincos_2pi(float x, float *s, float *c) { sincospif(2.0f * x, s, c); }
__device__ __forceinline__ void sincos_2pi(double x, double *s, double *c) { sincospi(2.0 * x, s, c); }

// Phase tables in LDS (per term and node block).  For the first axis of the term the band's
// phases are kept in "lane versions", so that the part of a product a lane needs is one FMA
// without a select: with ph = E0 * P (E0 the first axis's phase, P the product of the other
// axes' phases), fma(v.x, P.x, v.y * P.y) gives
//   v = (E0.x, -E0.y): Re ph,   v = (E0.y, E0.x): Im ph,   v = (-E0.y, -E0.x): -Im ph.
// P for all frequencies of the other axes is tabulated per node (order 2: the second axis's
// band; order 3: the K x K products).  Node rows are padded (kDirPad complex) so that the
// rows the lanes of one LDS read touch fall into different banks.
constexpr int kDirPad = 16;     // forward: rows of NB + 16 complex
constexpr int kDirRowA = 68;    // adjoint: rows of 64 + 4 complex

// The band's phase at index idx (k = idx - N/2 for idx < N/2, else idx - N/2 + 1) times
// 2 pi x, as sin and cos.
template <typename T>
__device__ __forceinline__ void band_sincos(T x, int idx, int half, T *s, T *c) {
  const int k = idx < half ? idx - half : idx - half + 1;
  sincos_2pi((T)k * x, s, c);
}

// The other axes' phase tables of a node block: order 2: P[k][n] = E1[k](x_n); order 3:
// P[i1 K + i2][n] = E1[i1](x_n) E2[i2](x_n), from per-axis tables T (2 x K rows, one sincos per
// entry) built first.  NBK nodes (a power of two) whose coordinates along the term's axes are
// staged in sX ([axis][NBK]), rows of `stride`; the caller synchronises between the two
// stages (stage 0: tables, stage 1: products).
template <typename T, int ORDER, int NBK>
__device__ __forceinline__ void other_axes(const T *sX, int K, int half, cx_t<T> *sP, cx_t<T> *sT, int stride,
                                           int stage) {
  if (ORDER == 2 && stage == 0) {
    for (int i = threadIdx.x; i < K * NBK; i += 256) {
      const int k = i / NBK, n = i % NBK;
      T sn, cs;
      band_sincos<T>(sX[NBK + n], k, half, &sn, &cs);
      sP[k * stride + n] = cmake<T>(cs, sn);
    }
  } else if (ORDER == 3 && stage == 0) {
    for (int i = threadIdx.x; i < 2 * K * NBK; i += 256) {
      const int ak = i / NBK, n = i % NBK, a = ak >= K ? 1 : 0, k = ak - a * K;
      T sn, cs;
      band_sincos<T>(sX[(1 + a) * NBK + n], k, half, &sn, &cs);
      sT[ak * stride + n] = cmake<T>(cs, sn);
    }
  } else if (ORDER == 3 && stage == 1) {
    for (int i = threadIdx.x; i < K * K * NBK; i += 256) {
      const int kk = i / NBK, n = i % NBK, i1 = kk / K, i2 = kk - i1 * K;
      const cx_t<T> e1 = sT[i1 * stride + n], e2 = sT[(K + i2) * stride + n];
      sP[kk * stride + n] = cmake<T>(e1.x * e2.x - e1.y * e2.y, fma(e1.x, e2.y, e1.y * e2.x));
    }
  }
}

// Coordinate of axis a (0..order-1) of a term (arithmetic selection: an indexed pick of the
// struct's fields would go through a private stack copy).
__device__ __forceinline__ int term_axis(const DevTerm &dt, int a) {
  return dt.c0 + (a >= 1 ? dt.c1 - dt.c0 : 0) + (a >= 2 ? dt.c2 - dt.c1 : 0);
}

// Forward, all terms [tb, te) of one order: each workgroup takes NB = 4 x RTW x 16
// consecutive nodes (RTW row tiles of 16 nodes per wavefront) and adds sum_u F_u fhat_u for
// its nodes into f (R x M), accumulating over the terms in registers.  Columns: CT blocks of
// 8 right-hand sides.  LDS:
//   sB   the coefficients as B rows of part p = 0: G + 1 rows kf x 16 CT columns (r, c) holding
//        F.x (c = 0) and F.y (c = 1), the last row zero, rows of 16 CT + 1 (an odd stride keeps
//        the staging stores of consecutive kf in different banks); a lane of part p = 1 reads
//        column (r, 1 - c) and negates it for c = 0 (-F.y, F.x);
//   sE0  the first axis's phases in two lane versions, 2 x (K + 1) x (NB + kDirPad) complex
//        (row K of each version zero);
//   sP   order >= 2: the other axes' products, KR2 x (NB + kDirPad) complex, KR2 = K^(order-1)
//        rounded up to even (the extra row zero);
//   sT   order 3: the two other axes' phase tables, 2 K x (NB + kDirPad) complex.
// Order >= 2 runs the K steps as (i0, pair of ir): frequency kf = i0 KR + ir with ir = 2 s + h
// for K slot q = 2 h + p, so the first axis's phase of a lane stays fixed over the inner loop
// and the products' row advances by two (no carries; a padded ir reads the zero row).
template <typename T, int ORDER, int CT, int RTW>
__global__ __launch_bounds__(256) void k_direct_fwd(const T *__restrict__ xT, const DevTerm *__restrict__ terms,
                                                    int tb, int te, DirectArgs da,
                                                    const cx_t<T> *__restrict__ fhat,
                                                    const T *__restrict__ colscale, cx_t<T> *__restrict__ f) {
  using MF = Mfma<T>;
  using acc_t = typename MF::acc;
  using C = cx_t<T>;
  constexpr int RP = 8 * CT;             // right-hand sides per column block, padded
  constexpr int WB = 16 * CT;            // B columns
  constexpr int SB = WB + 1;             // B row stride
  constexpr int NW = 16 * RTW;           // nodes per wavefront (RTW row tiles of 16)
  constexpr int NB = 4 * NW;             // nodes per workgroup
  constexpr int NBP = NB + kDirPad;      // padded node row
  extern __shared__ __align__(16) unsigned char smem_direct[];
  const int K = da.K, G = da.G, KR = G / K, KR2 = KR + (KR & 1);
  T *sB = reinterpret_cast<T *>(smem_direct);                            // (G + 1) x SB
  C *sE0 = reinterpret_cast<C *>(sB + (((size_t)(G + 1) * SB + 3) & ~(size_t)3));   // 2 x (K + 1) x NBP
  C *sP = sE0 + 2 * (K + 1) * NBP;                                      // KR2 x NBP
  C *sT = sP + (ORDER >= 2 ? KR2 * NBP : 0);                            // order 3: 2K x NBP
  T *sX = reinterpret_cast<T *>(sT + (ORDER == 3 ? 2 * K * NBP : 0));   // ORDER x NB coordinates
  constexpr int XPT = (ORDER * NB + 255) / 256;   // coordinates per thread
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, i16 = lane & 15, h = q >> 1, pim = q & 1;
  const int64_t v0 = (int64_t)blockIdx.x * NB;
  acc_t acc[RTW][CT];
#pragma unroll
  for (int j = 0; j < RTW; ++j)
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[j][c] = acc_t{0, 0, 0, 0};
  // rows that stay zero: sB's last row, sE0's row K of each version, sP's padding row
  for (int i = threadIdx.x; i < SB; i += 256) sB[(size_t)G * SB + i] = (T)0;
  for (int i = threadIdx.x; i < 2 * NBP; i += 256) sE0[((i / NBP) * (K + 1) + K) * NBP + i % NBP] = cmake<T>(0, 0);
  if (ORDER >= 2 && KR2 > KR)
    for (int i = threadIdx.x; i < NBP; i += 256) sP[KR * NBP + i] = cmake<T>(0, 0);
  const C *E0l = sE0 + pim * (K + 1) * NBP;   // this lane's version of the first axis
  const bool cim = (i16 & 1) != 0;
  const int bcol = i16 ^ pim;                    // B column read (the partner for part 1)
  const T bsgn = (pim && !cim) ? (T)-1 : (T)1;
  // The next term's coefficients (frequency threadIdx.x) and the block's coordinates along its
  // axes are loaded into registers while the current term's MFMA steps run.
  C pfF[RP];
  T pfS = 1, pfX[XPT];
  auto prefetch = [&](int u) {
    const DevTerm d2 = terms[u];
    const int kf = threadIdx.x;
#pragma unroll
    for (int r = 0; r < RP; ++r)
      pfF[r] = (kf < G && r < da.R) ? fhat[(int64_t)r * da.ncoef + d2.coef_off + kf] : cmake<T>(0, 0);
    pfS = (colscale && kf < G) ? colscale[d2.coef_off + kf] : (T)1;
#pragma unroll
    for (int x = 0; x < XPT; ++x) {
      const int i = threadIdx.x + 256 * x, a = i / NB, n = i % NB;
      const int64_t v = v0 + n;
      pfX[x] = (a < ORDER && v < da.M) ? xT[(int64_t)term_axis(d2, a) * da.M + v] : (T)0;
    }
  };
  if (tb < te) prefetch(tb);
  for (int u = tb; u < te; ++u) {
    const DevTerm dt = terms[u];
    __syncthreads();                     // the previous term's LDS reads are done
    // B rows of part 0: column (r, 0) F.x, (r, 1) F.y (frequencies past 256 loaded here)
    if ((int)threadIdx.x < G) {
      T *row = sB + (size_t)threadIdx.x * SB;
#pragma unroll
      for (int r = 0; r < RP; ++r) {
        row[2 * r] = pfF[r].x * pfS;
        row[2 * r + 1] = pfF[r].y * pfS;
      }
    }
    for (int kf = 256 + threadIdx.x; kf < G; kf += 256) {
      const T cs = colscale ? colscale[dt.coef_off + kf] : (T)1;
      T *row = sB + (size_t)kf * SB;
      for (int r = 0; r < RP; ++r) {
        const C val = r < da.R ? fhat[(int64_t)r * da.ncoef + dt.coef_off + kf] : cmake<T>(0, 0);
        row[2 * r] = val.x * cs;
        row[2 * r + 1] = val.y * cs;
      }
    }
#pragma unroll
    for (int x = 0; x < XPT; ++x) {
      const int i = threadIdx.x + 256 * x;
      if (i < ORDER * NB) sX[i] = pfX[x];
    }
    __syncthreads();
    // first axis: both lane versions, one thread per (node, frequency)
    for (int i = threadIdx.x; i < K * NB; i += 256) {
      const int k = i / NB, n = i % NB;
      T sn, cs;
      band_sincos<T>(sX[n], k, da.half, &sn, &cs);
      sE0[k * NBP + n] = cmake<T>(cs, -sn);
      sE0[(K + 1 + k) * NBP + n] = cmake<T>(sn, cs);
    }
    other_axes<T, ORDER, NB>(sX, K, da.half, sP, sT, NBP, 0);
    if (ORDER == 3) {
      __syncthreads();
      other_axes<T, ORDER, NB>(sX, K, da.half, sP, sT, NBP, 1);
    }
    if (u + 1 < te) prefetch(u + 1);
    __syncthreads();
    if (ORDER == 1) {
      // kf = 2 s + h: the phase is the lane's version of the first axis (row K: zero)
      const int nsteps = (2 * G + 3) >> 2;
      for (int s = 0; s < nsteps; ++s) {
        const int kf = 2 * s + h;
        const int row = kf < G ? kf : K;
        T av[RTW], bv[CT];
#pragma unroll
        for (int j = 0; j < RTW; ++j) av[j] = E0l[row * NBP + wave * NW + j * 16 + i16].x;
#pragma unroll
        for (int c = 0; c < CT; ++c) bv[c] = bsgn * sB[(size_t)(kf < G ? kf : G) * SB + 16 * c + bcol];
#pragma unroll
        for (int j = 0; j < RTW; ++j)
#pragma unroll
          for (int c = 0; c < CT; ++c) acc[j][c] = MF::run(av[j], bv[c], acc[j][c]);
      }
    } else {
      for (int i0 = 0; i0 < K; ++i0) {
        C e[RTW];
#pragma unroll
        for (int j = 0; j < RTW; ++j) e[j] = E0l[i0 * NBP + wave * NW + j * 16 + i16];
        const C *prow = sP + h * NBP + wave * NW + i16;
        const T *brow = sB + (size_t)(i0 * KR + h) * SB + bcol;
#pragma unroll 2
        for (int s2 = 0; s2 < KR2 / 2; ++s2) {
          T av[RTW], bv[CT];
#pragma unroll
          for (int j = 0; j < RTW; ++j) {
            const C pp = prow[j * 16];
            av[j] = fma(e[j].x, pp.x, e[j].y * pp.y);
          }
#pragma unroll
          for (int c = 0; c < CT; ++c) bv[c] = bsgn * brow[16 * c];
#pragma unroll
          for (int j = 0; j < RTW; ++j)
#pragma unroll
            for (int c = 0; c < CT; ++c) acc[j][c] = MF::run(av[j], bv[c], acc[j][c]);
          prow += 2 * NBP;
          brow += 2 * SB;
        }
      }
    }
  }
  // D[row][col] with col = i16 + 16c: right-hand side col / 2, real part in even columns
#pragma unroll
  for (int j = 0; j < RTW; ++j)
#pragma unroll
    for (int c = 0; c < CT; ++c)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const T mine = acc[j][c][e];
        const T other = __shfl_xor(mine, 1);
        const int64_t v = v0 + wave * NW + j * 16 + MF::row(lane, e);
        const int r = (i16 + 16 * c) >> 1;
        if (!cim && v < da.M && r < da.R) {
          C o = f[(int64_t)r * da.M + v];
          o.x += mine;
          o.y += other;
          f[(int64_t)r * da.M + v] = o;
        }
      }
}

// Adjoint, one term per blockIdx.y (term tb + blockIdx.y), the nodes split into nslice equal
// ranges (blockIdx.x): per 64-node chunk the samples (real and imaginary planes, 64 x 16
// right-hand sides) and the phase tables are staged in LDS, then each wavefront accumulates
// its RTW row tiles (rows 16 (wave + 4 j) + 0..15) over the chunk's nodes, two nodes per MFMA
// step.  The first axis's phases are kept in three lane versions (the row part c of fhat and
// the K part p of y select Re, Im or -Im of the phase), followed by a zero row that the rows
// past the group read.  The partial sums go to
// part[((term * nslice + slice) * 64 RTW + row) * 16 + r].
template <typename T, int ORDER, int RTW>
__global__ __launch_bounds__(256) void k_direct_adj(const T *__restrict__ xT, const DevTerm *__restrict__ terms, int tb,
                                                    DirectArgs da, int nslice, const cx_t<T> *__restrict__ y,
                                                    T *__restrict__ part) {
  using MF = Mfma<T>;
  using acc_t = typename MF::acc;
  using C = cx_t<T>;
  constexpr int ROWS = 64 * RTW;
  constexpr int NP = kDirRowA;
  __shared__ T sY[2 * 16 * 65];          // [part][r][node pair half][node / 2], rows of 65
  extern __shared__ __align__(16) unsigned char smem_direct[];
  const int K = da.K, G = da.G, KR = G / K;
  C *sE0 = reinterpret_cast<C *>(smem_direct);   // 3 versions x K x NP, then one zero row
  C *sP = sE0 + (3 * K + 1) * NP;                 // KR x NP (order >= 2)
  C *sT = sP + KR * NP;                           // order 3: 2K x NP
  const DevTerm dt = terms[tb + blockIdx.y];
  const int slice = blockIdx.x;
  const int64_t n0 = da.M * slice / nslice, n1 = da.M * (slice + 1) / nslice;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, i16 = lane & 15;
  const int cim = i16 & 1;               // row part: imaginary part of fhat
  const int pim = q & 1;                 // K part: imaginary part of y
  const int ver = cim == pim ? 0 : (cim ? 2 : 1);
  // the phase-table offsets of this lane's rows (rows past the group read the zero row)
  int e0off[RTW], poff[RTW];
#pragma unroll
  for (int j = 0; j < RTW; ++j) {
    const int kf = (16 * (wave + 4 * j) + i16) >> 1;
    e0off[j] = kf < G ? (ver * K + kf / KR) * NP : 3 * K * NP;
    poff[j] = kf < G ? (kf % KR) * NP : 0;
  }
  for (int i = threadIdx.x; i < NP; i += 256) sE0[3 * K * NP + i] = cmake<T>(0, 0);
  acc_t acc[RTW];
#pragma unroll
  for (int j = 0; j < RTW; ++j) acc[j] = acc_t{0, 0, 0, 0};
  const T *yl = sY + (pim * 16 + i16) * 65 + (q >> 1) * 32;   // this lane's samples: r = i16, part pim
  // The next chunk's samples and coordinates are loaded into registers while the current
  // chunk's MFMA steps run.
  __shared__ T sX[3 * 64];               // the chunk's coordinates along the term's axes
  C pfY[4];
  T pfX = 0;
  auto prefetch = [&](int64_t nb) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = threadIdx.x + 256 * k, r = i >> 6, n = i & 63;
      const int64_t v = nb + n;
      pfY[k] = (r < da.R && v < n1) ? y[(int64_t)r * da.M + v] : cmake<T>(0, 0);
    }
    const int a = threadIdx.x >> 6, n = threadIdx.x & 63;
    const int64_t v = nb + n;
    pfX = (a < ORDER && v < n1) ? xT[(int64_t)term_axis(dt, a) * da.M + v] : (T)0;
  };
  if (n0 < n1) prefetch(n0);
  for (int64_t nb = n0; nb < n1; nb += 64) {
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = threadIdx.x + 256 * k, r = i >> 6, n = i & 63;
      const int o = r * 65 + (n & 1) * 32 + (n >> 1);
      sY[o] = pfY[k].x;
      sY[16 * 65 + o] = pfY[k].y;
    }
    if ((int)(threadIdx.x >> 6) < ORDER) sX[threadIdx.x] = pfX;
    __syncthreads();
    for (int i = threadIdx.x; i < K * 64; i += 256) {
      const int k = i >> 6, n = i & 63;
      T sn, cs;
      band_sincos<T>(sX[n], k, da.half, &sn, &cs);
      sE0[k * NP + n] = cmake<T>(cs, -sn);
      sE0[(K + k) * NP + n] = cmake<T>(sn, cs);
      sE0[(2 * K + k) * NP + n] = cmake<T>(-sn, -cs);
    }
    other_axes<T, ORDER, 64>(sX, K, da.half, sP, sT, NP, 0);
    if (ORDER == 3) {
      __syncthreads();
      other_axes<T, ORDER, 64>(sX, K, da.half, sP, sT, NP, 1);
    }
    if (nb + 64 < n1) prefetch(nb + 64);
    __syncthreads();
    // (unrolled: the step's node offsets become immediate LDS offsets)
    const int hq = q >> 1;                 // the step's node 2 s + hq
    const C *ebase[RTW], *pbase[RTW];
#pragma unroll
    for (int j = 0; j < RTW; ++j) {
      ebase[j] = sE0 + e0off[j] + hq;
      pbase[j] = sP + poff[j] + hq;
    }
#pragma unroll
    for (int s = 0; s < 32; ++s) {
      const T bv = yl[s];
#pragma unroll
      for (int j = 0; j < RTW; ++j) {
        const C e = ebase[j][2 * s];
        T av;
        if (ORDER == 1) {
          av = e.x;
        } else {
          const C pp = pbase[j][2 * s];
          av = fma(e.x, pp.x, e.y * pp.y);
        }
        acc[j] = MF::run(av, bv, acc[j]);
      }
    }
  }
  T *out = part + ((int64_t)blockIdx.y * nslice + slice) * ROWS * 16;
#pragma unroll
  for (int j = 0; j < RTW; ++j)
#pragma unroll
    for (int e = 0; e < 4; ++e) out[(16 * (wave + 4 * j) + MF::row(lane, e)) * 16 + i16] = acc[j][e];
}

// Sums the adjoint partials over the node slices in slice order and writes the group's
// coefficients (times the column scale, if any): fhat[r][coef_off + kf].
template <typename T>
__global__ __launch_bounds__(256) void k_direct_adj_sum(const T *__restrict__ part, const DevTerm *__restrict__ terms,
                                                        int tb, DirectArgs da, int nslice, int rows,
                                                        const T *__restrict__ colscale, cx_t<T> *__restrict__ fhat) {
  const int tl = blockIdx.y;
  const DevTerm dt = terms[tb + tl];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= da.G * da.R) return;
  const int r = i / da.G, kf = i - r * da.G;
  const T *p = part + (int64_t)tl * nslice * rows * 16;
  T re = 0, im = 0;
  for (int sl = 0; sl < nslice; ++sl) {
    re += p[((int64_t)sl * rows + 2 * kf) * 16 + r];
    im += p[((int64_t)sl * rows + 2 * kf + 1) * 16 + r];
  }
  const T cs = colscale ? colscale[dt.coef_off + kf] : (T)1;
  fhat[(int64_t)r * da.ncoef + dt.coef_off + kf] = cmake<T>(re * cs, im * cs);
}

}  // namespace gt
