// Kernels of the absorbing-layer form of the step (Sec. 4.1, Sec. 4.2):
// the dense stages of the eigen-route Sylvester solve, the stretched explicit
// operator (for the Arnoldi step with its inner products, and for true
// residuals), copies and the residue-weighted sum.  FP64 throughout.
#include "pml.hpp"

namespace {

__device__ __forceinline__ double pml_wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Sum over a 256-thread workgroup in a fixed order; valid in thread 0.
__device__ __forceinline__ double pml_block_sum(double v, double* red) {
  v = pml_wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return threadIdx.x == 0 ? (red[0] + red[1]) + (red[2] + red[3]) : 0.0;
}

__device__ __forceinline__ const c128* pml_field(const PmlRef& r, int k, int m) {
  return r.tbl ? r.tbl[(size_t)k * (HP_MAXM + 1) + m] : r.base + (size_t)k * r.sp + (size_t)m * r.si;
}

// ------------------------------------------------------------------ dense stages

// Complex FP64 products on the vector ALU: on this chip the FP64 rate of the
// vector units equals that of the matrix cores, and the complex product needs
// no operand splitting there.  64 x 64 output tile per 256-thread workgroup,
// 4 x 4 outputs per thread (rows ty + 16 i, columns tx + 16 j), K in steps of
// 16 staged through LDS with the next step's global loads in flight during
// the current step's products.
constexpr int GT = 64, GK = 16, GWG = 256;

template <bool LEFT, int EPI>
__global__ __launch_bounds__(GWG) void k_pml_gemm(const c128* __restrict__ mat, PmlRef in, PmlRef out,
                                                  const PoleState* __restrict__ st, PoleList list,
                                                  int* __restrict__ active_out, const c128* __restrict__ lam, int N,
                                                  int ncomp) {
  // blockIdx.z: pole list entry a, field component comp (components are N x N planes)
  const int a_ = blockIdx.z / ncomp, comp = blockIdx.z % ncomp;
  const int k = list.k[a_];
  if (active_out && comp == 0 && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) active_out[a_] = k;
  if (st[k].flag) return;
  const int m = st[k].m;
  const size_t co = (size_t)comp * N * N;
  const c128* __restrict__ X = pml_field(in, k, m) + co;
  c128* __restrict__ Y = const_cast<c128*>(pml_field(out, k, m)) + co;
  const int r0 = blockIdx.y * GT, c0 = blockIdx.x * GT;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  // A[r][j] = Mat[r][j] (left) or X[r][j] (right); B[j][c] = X[j][c] (left) or Mat[c][j] (right)
  const c128* __restrict__ Ag = LEFT ? mat : X;
  const c128* __restrict__ Bg = LEFT ? X : mat;
  __shared__ c128 As[GK][GT + 1];
  __shared__ c128 Bs[GK][GT + 1];
  c128 ra[4], rb[4];
  auto fetch = [&](int j0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + GWG * q;
      ra[q] = Ag[(size_t)(r0 + (e >> 4)) * N + j0 + (e & 15)];
      if (LEFT)
        rb[q] = Bg[(size_t)(j0 + (e >> 6)) * N + c0 + (e & 63)];
      else
        rb[q] = Bg[(size_t)(c0 + (e >> 4)) * N + j0 + (e & 15)];
    }
  };
  c128 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = mk(0.0, 0.0);
  fetch(0);
  for (int j0 = 0; j0 < N; j0 += GK) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + GWG * q;
      As[e & 15][e >> 4] = ra[q];
      if (LEFT)
        Bs[e >> 6][e & 63] = rb[q];
      else
        Bs[e & 15][e >> 4] = rb[q];
    }
    __syncthreads();
    if (j0 + GK < N) fetch(j0 + GK);
#pragma unroll 4
    for (int kk = 0; kk < GK; ++kk) {
      c128 a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          acc[i][j].re = fma(a[i].re, b[j].re, fma(-a[i].im, b[j].im, acc[i][j].re));
          acc[i][j].im = fma(a[i].re, b[j].im, fma(a[i].im, b[j].re, acc[i][j].im));
        }
    }
    __syncthreads();
  }
  const c128 bk = st[k].bk;
  const double sg = st[k].sigma[m];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = r0 + ty + 16 * i;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = c0 + tx + 16 * j;
      c128 v = acc[i][j];
      if (EPI == 1) v = (r == 0 || c == 0) ? mk(0.0, 0.0) : cdiv(v, lam[r] + lam[c] - bk);
      if (EPI == 2) v = sg * v;
      Y[(size_t)r * N + c] = v;
    }
  }
}

// The same products on the matrix cores: v_mfma_f64_16x16x4f64 multiplies a
// 16 x 4 by a 4 x 16 FP64 block per wave (operand element (i, k) of A and
// (k, j) of B in lane i + 16 k and j + 16 k; result (i, j) in element i / 4 of
// lane j + 16 (i % 4), i.e. element r of lane l holds (4 r + l / 16, l % 16)).  A complex block takes four real products into two
// accumulators (re += Ar Br - Ai Bi, im += Ar Bi + Ai Br); each lane reads its
// complex operand from LDS with one 16-byte load, so LDS carries a quarter of
// the bytes per multiply-add that the vector-ALU form needs.  BT x BT block
// tile, four waves of BT/2 x BT/2, K staged through LDS in steps of 16 as there;
// at most 128 registers per lane (accumulators included), four waves per SIMD.
typedef double pml_d4 __attribute__((ext_vector_type(4)));

template <bool LEFT, int EPI, int BT, bool DIVB = false>
__global__ __launch_bounds__(GWG, 4) void k_pml_gemm_mfma(const c128* __restrict__ mat, PmlRef in, PmlRef out,
                                                       const PoleState* __restrict__ st, PoleList list,
                                                       int* __restrict__ active_out, const c128* __restrict__ lam,
                                                       int N, int ncomp) {
  constexpr int WT = BT / 2, MB = WT / 16, LPT = BT * GK / GWG;
  const int a_ = blockIdx.z / ncomp, comp = blockIdx.z % ncomp;
  const int k = list.k[a_];
  if (active_out && comp == 0 && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) active_out[a_] = k;
  if (st[k].flag) return;
  const int m = st[k].m;
  const size_t co = (size_t)comp * N * N;
  const c128* __restrict__ X = pml_field(in, k, m) + co;
  c128* __restrict__ Y = const_cast<c128*>(pml_field(out, k, m)) + co;
  // right products: consecutive workgroups (spread over the XCDs) take consecutive row
  // tiles, so each XCD keeps its row slabs of the field operand
  const int r0 = (LEFT ? blockIdx.y : blockIdx.x) * BT, c0 = (LEFT ? blockIdx.x : blockIdx.y) * BT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * WT, wc = (wave & 1) * WT;
  const c128* __restrict__ Ag = LEFT ? mat : X;
  const c128* __restrict__ Bg = LEFT ? X : mat;
  __shared__ c128 As[GK][BT + 1];
  __shared__ c128 Bs[GK][BT + 1];
  c128 ra[LPT], rb[LPT];
  const c128 bk0 = st[k].bk;
  auto fetch = [&](int j0) {
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
      const int e = tid + GWG * q;
      ra[q] = Ag[(size_t)(r0 + e / GK) * N + j0 + e % GK];
      if (LEFT) {
        const int jr = j0 + e / BT, jc = c0 + e % BT;
        rb[q] = Bg[(size_t)jr * N + jc];
        // the divide of the pole's middle stage, applied to a product shared by all poles
        if (DIVB) rb[q] = (jr == 0 || jc == 0) ? mk(0.0, 0.0) : cdiv(rb[q], lam[jr] + lam[jc] - bk0);
      } else {
        rb[q] = Bg[(size_t)(c0 + e / GK) * N + j0 + e % GK];
      }
    }
  };
  pml_d4 cr[MB][MB], ci[MB][MB];
#pragma unroll
  for (int a = 0; a < MB; ++a)
#pragma unroll
    for (int b = 0; b < MB; ++b) {
      cr[a][b] = pml_d4{0.0, 0.0, 0.0, 0.0};
      ci[a][b] = pml_d4{0.0, 0.0, 0.0, 0.0};
    }
  const int li = lane & 15, lk = lane >> 4;
  fetch(0);
  for (int j0 = 0; j0 < N; j0 += GK) {
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
      const int e = tid + GWG * q;
      As[e % GK][e / GK] = ra[q];
      if (LEFT)
        Bs[e / BT][e % BT] = rb[q];
      else
        Bs[e % GK][e / GK] = rb[q];
    }
    __syncthreads();
    if (j0 + GK < N) fetch(j0 + GK);
#pragma unroll
    for (int ks = 0; ks < GK; ks += 4) {
      double ar[MB], ai[MB], nai[MB], br[MB], bi[MB];
#pragma unroll
      for (int a = 0; a < MB; ++a) {
        const c128 v = As[ks + lk][wr + a * 16 + li];
        ar[a] = v.re;
        ai[a] = v.im;
        nai[a] = -v.im;
      }
#pragma unroll
      for (int b = 0; b < MB; ++b) {
        const c128 v = Bs[ks + lk][wc + b * 16 + li];
        br[b] = v.re;
        bi[b] = v.im;
      }
#pragma unroll
      for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int b = 0; b < MB; ++b) {
          cr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a], br[b], cr[a][b], 0, 0, 0);
          ci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a], bi[b], ci[a][b], 0, 0, 0);
        }
#pragma unroll
      for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int b = 0; b < MB; ++b) {
          cr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(nai[a], bi[b], cr[a][b], 0, 0, 0);
          ci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[a], br[b], ci[a][b], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  const c128 bk = st[k].bk;
  const double sg = st[k].sigma[m];
#pragma unroll
  for (int a = 0; a < MB; ++a)
#pragma unroll
    for (int b = 0; b < MB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + wr + a * 16 + 4 * r + lk, col = c0 + wc + b * 16 + li;
        c128 v = mk(cr[a][b][r], ci[a][b][r]);
        if (EPI == 1) v = (row == 0 || col == 0) ? mk(0.0, 0.0) : cdiv(v, lam[row] + lam[col] - bk);
        if (EPI == 2) v = sg * v;
        Y[(size_t)row * N + col] = v;
      }
}

// ------------------------------------------------------------------ stretched explicit operator

// x at node (i, j) with odd reflection about the Dirichlet nodes 0 and N
__device__ __forceinline__ c128 pml_ld(const c128* __restrict__ x, int i, int j, int N) {
  double sg = 1.0;
  if (i < 0) {
    i = -i;
    sg = -sg;
  } else if (i > N) {
    i = 2 * N - i;
    sg = -sg;
  }
  if (j < 0) {
    j = -j;
    sg = -sg;
  } else if (j > N) {
    j = 2 * N - j;
    sg = -sg;
  }
  if (i == 0 || j == 0 || i == N || j == N) return mk(0.0, 0.0);
  return sg * x[(size_t)i * N + j];
}

// Stencil sums of one component at interior node (i, j): the stretched
// Laplacian s (D2x~ + D2y~) x, the plain first derivatives D1x x and D1y x
// (the psi coupling's; it is zero where the stretching acts) and x itself.
struct PmlPoint {
  c128 lap, dx, dy, ctr;
};
// (Zbar~ - b I) x at interior node (i, j) for the NC components of x (planes fsz
// apart): the stretched Laplacian plus (V - b) x, and for vector fields the psi
// coupling of eq. Z_bar_eq (coefficient planes 1..5: s psi_x, s psi_y, s psi_xx,
// s psi_yy, s psi_xy, zero in the layers).
template <int NC>
__device__ __forceinline__ void pml_combine(const PmlPoint* pt, const double* __restrict__ coef, size_t idx,
                                            size_t fsz, c128 b, c128* out) {
  const double V = coef[idx];
#pragma unroll
  for (int c = 0; c < NC; ++c) out[c] = pt[c].lap + (V * pt[c].ctr - b * pt[c].ctr);
  if constexpr (NC == 2) {
    const double px = coef[fsz + idx], py = coef[2 * fsz + idx], pxx = coef[3 * fsz + idx],
                 pyy = coef[4 * fsz + idx], pxy = coef[5 * fsz + idx];
    out[0] = out[0] + pxx * pt[0].ctr + px * pt[0].dx + pxy * pt[1].ctr + py * pt[1].dx;
    out[1] = out[1] + pxy * pt[0].ctr + px * pt[0].dy + pyy * pt[1].ctr + py * pt[1].dy;
  }
}

// The tile layout of the operator pass below (64 x 16 points, 6-node halo).
constexpr int AP_X = 64, AP_Y = 16, AP_H = 6;
constexpr int AP_LX = AP_X + 2 * AP_H, AP_LY = AP_Y + 2 * AP_H;

// Stencil sums of one component at tile point lc (the LDS tile holds the
// component with its halo; node (i, j) of the field).
__device__ __forceinline__ PmlPoint pml_point_tile(const c128* t, int lc, int i, int j, const c128* __restrict__ a2,
                                                   const c128* __restrict__ a1, const StencilCoef& sc) {
  PmlPoint r;
  r.ctr = t[lc];
  c128 sxx = sc.c2x[0] * r.ctr, syy = sc.c2x[0] * r.ctr, sx1 = mk(0.0, 0.0), sy1 = mk(0.0, 0.0);
#pragma unroll
  for (int mm = 1; mm <= 6; ++mm) {
    const c128 xp = t[lc + mm], xm = t[lc - mm], yp = t[lc + mm * AP_LX], ym = t[lc - mm * AP_LX];
    sxx = sxx + sc.c2x[mm] * (xp + xm);
    sx1 = sx1 + sc.d1x[mm - 1] * (xp - xm);
    syy = syy + sc.c2x[mm] * (yp + ym);
    sy1 = sy1 + sc.d1x[mm - 1] * (yp - ym);
  }
  r.lap = (a2[j] * sxx - a1[j] * sx1) + (a2[i] * syy - a1[i] * sy1);
  r.dx = sx1;
  r.dy = sy1;
  return r;
}

// Field z (blockIdx.z) of a batch: y = rhs - (Zbar~ - b_z I) x (y = (Zbar~ - b I) x without rhs)
// on one 64 x 16 tile per workgroup (blockIdx.x), partial |y|^2 per workgroup.
template <int NC>
__global__ __launch_bounds__(256) void k_pml_residual(const c128* __restrict__ x, size_t xbs,
                                                      const c128* __restrict__ rhs, c128* __restrict__ y, size_t ybs,
                                                      const double* __restrict__ coef, const c128* __restrict__ a2,
                                                      const c128* __restrict__ a1, StencilCoef sc, ShiftList sh,
                                                      double* __restrict__ part, size_t pbs, int N) {
  __shared__ c128 tile[NC][AP_LY * AP_LX];
  __shared__ double red[4];
  const int z = blockIdx.z;
  x += (size_t)z * xbs;
  y += (size_t)z * ybs;
  const c128 b = sh.b[z];
  const size_t fsz = (size_t)N * N;
  const int ntx = N / AP_X;
  const int x0 = (blockIdx.x % ntx) * AP_X, y0 = (blockIdx.x / ntx) * AP_Y;
  const int tid = threadIdx.x, tx = tid & 63, tq = tid >> 6;
#pragma unroll
  for (int c = 0; c < NC; ++c)
    for (int e = tid; e < AP_LY * AP_LX; e += 256)
      tile[c][e] = pml_ld(x + c * fsz, y0 + e / AP_LX - AP_H, x0 + e % AP_LX - AP_H, N);
  __syncthreads();
  double nrm = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int ty = tq + 4 * q, i = y0 + ty, j = x0 + tx;
    const size_t idx = (size_t)i * N + j;
    c128 ax[NC];
    if (i > 0 && j > 0) {
      const int lc = (ty + AP_H) * AP_LX + tx + AP_H;
      PmlPoint pt[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) pt[c] = pml_point_tile(tile[c], lc, i, j, a2, a1, sc);
      pml_combine<NC>(pt, coef, idx, fsz, b, ax);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      c128 v = mk(0.0, 0.0);
      if (i > 0 && j > 0) v = rhs ? rhs[c * fsz + idx] - ax[c] : ax[c];
      y[c * fsz + idx] = v;
      nrm += abs2(v);
    }
  }
  const double s = pml_block_sum(nrm, red);
  if (threadIdx.x == 0 && part) part[(size_t)z * pbs + blockIdx.x] = s;
}

// ------------------------------------------------------------------ operator pass and inner products

// p = A_k z_m - sigma_m u_m with A_k applied by the explicit stretched stencil:
// then A_k z_m = ~v_m + p holds for the z_m actually stored, whatever the
// rounding of the dense stages (the eigenvector matrices of the stretched
// operator are far from unitary), so the Arnoldi relation of the stored Z is
// exact up to the rounding of p itself.

// The pass stages a 64 x 16 tile of every component of z with a 6-node halo
// (odd reflection applied while staging) in LDS, so each z value is read from
// memory about 1.6 times instead of once per stencil point; each thread then
// takes four points of a tile column.  The inner products are summed per wave.
template <int NC>
__global__ __launch_bounds__(256) void k_pml_apply(const c128* __restrict__ zbase, size_t zsp, size_t zsi,
                                                   c128* __restrict__ pbase, size_t psp, c128* const* __restrict__ uptr,
                                                   const double* __restrict__ coef, const c128* __restrict__ a2,
                                                   const c128* __restrict__ a1, StencilCoef sc,
                                                   const PoleState* __restrict__ st, const int* __restrict__ active,
                                                   double2* __restrict__ part, int nparts, int N) {
  __shared__ c128 tile[NC][AP_LY * AP_LX];
  const int k = active[blockIdx.y];
  if (st[k].flag) return;
  const int m = st[k].m;
  const size_t fsz = (size_t)N * N;
  const c128 bk = st[k].bk;
  const double sg = st[k].sigma[m];
  const c128* z = zbase + (size_t)k * zsp + (size_t)m * zsi;
  c128* p = pbase + (size_t)k * psp;
  const c128* const* up = uptr + (size_t)k * (HP_MAXM + 1);
  const int ntx = N / AP_X;
  const int x0 = (blockIdx.x % ntx) * AP_X, y0 = (blockIdx.x / ntx) * AP_Y;
  const int tid = threadIdx.x, tx = tid & 63, tq = tid >> 6;
#pragma unroll
  for (int c = 0; c < NC; ++c)
    for (int e = tid; e < AP_LY * AP_LX; e += 256)
      tile[c][e] = pml_ld(z + c * fsz, y0 + e / AP_LX - AP_H, x0 + e % AP_LX - AP_H, N);
  __syncthreads();
  c128 pv[4][NC], um[4][NC];
  {
    const c128* u = up[m];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ty = tq + 4 * q, i = y0 + ty, j = x0 + tx;
      const size_t idx = (size_t)i * N + j;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        um[q][c] = u[c * fsz + idx];
        pv[q][c] = mk(0.0, 0.0);
      }
      if (i > 0 && j > 0) {
        const int lc = (ty + AP_H) * AP_LX + tx + AP_H;
        PmlPoint pt[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) pt[c] = pml_point_tile(tile[c], lc, i, j, a2, a1, sc);
        c128 az[NC];
        pml_combine<NC>(pt, coef, idx, fsz, bk, az);
#pragma unroll
        for (int c = 0; c < NC; ++c) pv[q][c] = az[c] - sg * um[q][c];
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) p[c * fsz + idx] = pv[q][c];
    }
  }
  const int wave = tid >> 6, lane = tid & 63;
  const int slot = blockIdx.x * 4 + wave;
  for (int i = 0; i <= m; ++i) {
    const c128* u = up[i];
    double pr = 0.0, pi = 0.0, qr = 0.0, qi = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const size_t idx = (size_t)(y0 + tq + 4 * q) * N + x0 + tx;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const c128 a = (i == m) ? um[q][c] : u[c * fsz + idx];
        pr += a.re * pv[q][c].re + a.im * pv[q][c].im;
        pi += a.re * pv[q][c].im - a.im * pv[q][c].re;
        qr += a.re * um[q][c].re + a.im * um[q][c].im;
        qi += a.re * um[q][c].im - a.im * um[q][c].re;
      }
    }
    pr = pml_wave_sum(pr);
    pi = pml_wave_sum(pi);
    qr = pml_wave_sum(qr);
    qi = pml_wave_sum(qi);
    if (lane == 0) {
      const size_t b = (((size_t)k * (HP_MAXM + 1) + i) * 2) * nparts + slot;
      part[b] = make_double2(pr, pi);
      part[b + nparts] = make_double2(qr, qi);
    }
  }
}

// ------------------------------------------------------------------ copies and the sum

__global__ __launch_bounds__(256) void k_pml_copy(const c128* __restrict__ src, size_t sbs, PoleList isel,
                                                  c128* __restrict__ dst, size_t dbs, PoleList osel,
                                                  double* __restrict__ part, size_t part_bs, int N, int ncomp) {
  __shared__ double red[4];
  const int z = blockIdx.z;
  src += (size_t)isel.k[z] * sbs;
  dst += (size_t)osel.k[z] * dbs;
  const size_t fsz = (size_t)N * N, total = fsz * ncomp;
  double nrm = 0.0;
  for (size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (size_t)gridDim.x * 256) {
    const size_t e = idx % fsz;
    const int i = (int)(e / N), j = (int)(e % N);
    const c128 v = (i > 0 && j > 0) ? src[idx] : mk(0.0, 0.0);
    dst[idx] = v;
    nrm += abs2(v);
  }
  const double s = pml_block_sum(nrm, red);
  if (threadIdx.x == 0) part[(size_t)z * part_bs + blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_pml_final(const c128* __restrict__ w, c128* __restrict__ out,
                                                   const c128* __restrict__ zbase, size_t zsp, size_t zsi,
                                                   const c128* __restrict__ xacc, size_t xsp,
                                                   const PoleState* __restrict__ st, int npoles, c128 phase,
                                                   c128 rinf_phase, int N, int ncomp) {
  const size_t fsz = (size_t)N * N, total = fsz * ncomp;
  for (size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (size_t)gridDim.x * 256) {
    const size_t e = idx % fsz;
    const int i = (int)(e / N), j = (int)(e % N);
    c128 v = mk(0.0, 0.0);
    if (i > 0 && j > 0) {
      c128 acc = mk(0.0, 0.0);
      for (int k = 0; k < npoles; ++k) {
        const c128 ak = st[k].ak;
        if (st[k].has_x) acc = acc + ak * xacc[(size_t)k * xsp + idx];
        const int mk_ = st[k].m;
        const c128* zk = zbase + (size_t)k * zsp + idx;
        for (int q = 0; q < mk_; ++q) acc = acc + (ak * st[k].y[q]) * zk[(size_t)q * zsi];
      }
      v = phase * acc + rinf_phase * w[idx];
    }
    out[idx] = v;
  }
}

PoleList make_list(const int* sel, int n) {
  PoleList l;
  l.n = n;
  for (int a = 0; a < HP_MAXPOLES; ++a) l.k[a] = a < n ? sel[a] : 0;
  return l;
}

int flat_blocks(size_t n) {
  size_t b = (n + 1023) / 1024;
  return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

}  // namespace

__global__ void k_pml_shared_setup(PoleState* st, c128** tbl, const c128* u0) {
  if (threadIdx.x != 0) return;
  st->flag = 0;
  st->m = 0;
  st->bk = mk(0.0, 0.0);
  st->sigma[0] = 1.0;
  tbl[0] = const_cast<c128*>(u0);
}

void launch_pml_shared_setup(PoleState* st, c128** tbl, const c128* u0, hipStream_t s) {
  hipLaunchKernelGGL(k_pml_shared_setup, dim3(1), dim3(64), 0, s, st, tbl, u0);
}

void launch_pml_gemm_divided(const c128* mat, PmlRef in, PmlRef out, const PoleState* st, const int* list, int n,
                             int* active_out, const c128* lam, int N, int ncomp, hipStream_t s) {
  const PoleList l = make_list(list, n);
  const int big = n * ncomp * (N / 64) * (N / 64) >= 512;
  const int bt = big ? 64 : 32;
  const dim3 grid(N / bt, N / bt, n * ncomp);
  if (bt == 64)
    hipLaunchKernelGGL((k_pml_gemm_mfma<true, 0, 64, true>), grid, dim3(GWG), 0, s, mat, in, out, st, l, active_out,
                       lam, N, ncomp);
  else
    hipLaunchKernelGGL((k_pml_gemm_mfma<true, 0, 32, true>), grid, dim3(GWG), 0, s, mat, in, out, st, l, active_out,
                       lam, N, ncomp);
}

void launch_pml_gemm(int variant, bool left, int epilogue, const c128* mat, PmlRef in, PmlRef out,
                     const PoleState* st, const int* list, int n, int* active_out, const c128* lam, int N, int ncomp,
                     hipStream_t s) {
  const PoleList l = make_list(list, n);
  // variant 1 takes 64 x 64 tiles while they give every CU two workgroups, else 32 x 32
  const int big = n * ncomp * (N / 64) * (N / 64) >= 512;
  const int bt = (variant == 2 || (variant == 1 && !big)) ? 32 : 64;
  const dim3 grid(N / bt, N / bt, n * ncomp);
#define G_(L, E)                                                                                                   \
  do {                                                                                                             \
    if (variant == 0)                                                                                              \
      hipLaunchKernelGGL((k_pml_gemm<L, E>), grid, dim3(GWG), 0, s, mat, in, out, st, l, active_out, lam, N, ncomp); \
    else if (bt == 32)                                                                                             \
      hipLaunchKernelGGL((k_pml_gemm_mfma<L, E, 32>), grid, dim3(GWG), 0, s, mat, in, out, st, l, active_out, lam, \
                         N, ncomp);                                                                                \
    else                                                                                                           \
      hipLaunchKernelGGL((k_pml_gemm_mfma<L, E, 64>), grid, dim3(GWG), 0, s, mat, in, out, st, l, active_out, lam, \
                         N, ncomp);                                                                                \
  } while (0)
  if (left) {
    if (epilogue == 1)
      G_(true, 1);
    else if (epilogue == 2)
      G_(true, 2);
    else
      G_(true, 0);
  } else {
    if (epilogue == 1)
      G_(false, 1);
    else if (epilogue == 2)
      G_(false, 2);
    else
      G_(false, 0);
  }
#undef G_
}

int pml_tiles(int N) { return (N / AP_X) * (N / AP_Y); }

int pml_apply_parts(int N) { return pml_tiles(N) * 4; }

void launch_pml_apply(const c128* zbase, size_t zsp, size_t zsi, c128* pbase, size_t psp, c128* const* uptr,
                      const double* coef, const c128* a2, const c128* a1, const StencilCoef& sc, const PoleState* st,
                      const int* active, int nactive, double2* part, int N, int ncomp, hipStream_t s) {
  const int nparts = pml_apply_parts(N);
  if (ncomp == 2)
    hipLaunchKernelGGL(k_pml_apply<2>, dim3(nparts / 4, nactive), dim3(256), 0, s, zbase, zsp, zsi, pbase, psp,
                       uptr, coef, a2, a1, sc, st, active, part, nparts, N);
  else
    hipLaunchKernelGGL(k_pml_apply<1>, dim3(nparts / 4, nactive), dim3(256), 0, s, zbase, zsp, zsi, pbase, psp,
                       uptr, coef, a2, a1, sc, st, active, part, nparts, N);
}

bool launch_pml_residual(const c128* x, size_t xbs, const c128* rhs, c128* y, size_t ybs, const double* coef,
                         const c128* a2, const c128* a1, const StencilCoef& sc, const c128* shifts, int n,
                         double* part, size_t pbs, int nblk, int N, int ncomp, hipStream_t s) {
  ShiftList sh;
  for (int a = 0; a < HP_MAXPOLES; ++a) sh.b[a] = a < n ? shifts[a] : mk(0.0, 0.0);
  if (nblk != pml_tiles(N) || N % AP_X) return false;  // the caller's partial sums must match the tiles
  if (ncomp == 2)
    hipLaunchKernelGGL(k_pml_residual<2>, dim3(nblk, 1, n), dim3(256), 0, s, x, xbs, rhs, y, ybs, coef, a2, a1, sc,
                       sh, part, pbs, N);
  else
    hipLaunchKernelGGL(k_pml_residual<1>, dim3(nblk, 1, n), dim3(256), 0, s, x, xbs, rhs, y, ybs, coef, a2, a1, sc,
                       sh, part, pbs, N);
  return true;
}

void launch_pml_copy(const c128* src, size_t sbs, const int* isel, c128* dst, size_t dbs, const int* osel, int n,
                     double* part, size_t part_bs, int nblk, int N, int ncomp, hipStream_t s) {
  hipLaunchKernelGGL(k_pml_copy, dim3(nblk, 1, n), dim3(256), 0, s, src, sbs, make_list(isel, n), dst, dbs,
                     make_list(osel, n), part, part_bs, N, ncomp);
}

void launch_pml_final(const c128* w, c128* out, const c128* zbase, size_t zsp, size_t zsi, const c128* xacc,
                      size_t xsp, const PoleState* st, int npoles, c128 phase, c128 rinf_phase, int N, int ncomp,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_pml_final, dim3(flat_blocks((size_t)N * N * ncomp)), dim3(256), 0, s, w, out, zbase, zsp,
                     zsi, xacc, xsp, st, npoles, phase, rinf_phase, N, ncomp);
}
