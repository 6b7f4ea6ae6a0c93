// HIP kernels of one propagation step (gfx950).
//
// The step solves (Zbar - b_k I) x_k = w for every pole b_k by GMRES with the
// right preconditioner M_k = Zbar_fs - b_k I (Sec. 4.2).  Zbar = Zbar_fs + P
// where P holds the medium terms (V and, for the vector operator, the psi
// terms of eq. Z_bar_eq), so A_k M_k^{-1} v = v + P M_k^{-1} v exactly: the
// Laplacian stencil never runs inside the Arnoldi loop, only the medium part.
//
// Krylov vectors live in the row-transformed domain (DST-I along x applied,
// "R-domain"): the transform is orthonormal, so inner products and GMRES
// iterates are unchanged, and one Arnoldi step needs two passes over HBM:
//   column pass  z = S_y [(S_y u) / (mu_y + mu_x - b)]   (R-domain in, out)
//   row pass     p = S_x P S_x z  (+ the inner products with the basis)
// plus the Gram-Schmidt update.  All dot products, Givens rotations and the
// residue-weighted sum accumulate in FP64.
#include <math.h>

#include "fft.hpp"
#include "kernels.hpp"

namespace {

template <int L>
struct RowCfg {
  static constexpr int NT = L / 8;                       // threads per transform
  static constexpr int RPW = (256 / NT) > 0 ? 256 / NT : 1;  // transforms per workgroup
  static constexpr int WG = RPW * NT;
};

template <typename T, int L>
struct ColCfg {
  static constexpr int NT = L / 8;
  static constexpr int BYTES = L * (int)sizeof(cx<T>);
  static constexpr int C0 = 65536 / BYTES;
  static constexpr int C = C0 < 1 ? 1 : (C0 > 16 ? 16 : C0);  // columns per workgroup
  static constexpr int WG = C * NT;
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Sum over the workgroup in a fixed order; result valid in thread 0.
template <int WG>
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < (WG + 63) / 64; ++i) r += red[i];
  }
  return r;
}

// Workgroups are dealt to the 8 XCDs round-robin; map consecutive tiles onto
// one XCD so neighbouring column tiles share that XCD's L2.
__device__ __forceinline__ int xcd_tile(int bid, int nb) {
  if (nb % 8) return bid;
  return (bid % 8) * (nb / 8) + bid / 8;
}

template <typename T>
__device__ __forceinline__ cx<T> czero() {
  return mk<T>((T)0, (T)0);
}

__device__ __forceinline__ double edge_loss(int i, int j, int nx, int ny, int W, double eta, double coef) {
  int d = min(min(i, ny - i), min(j, nx - j));
  if (d < 1 || d > W) return 1.0;
  double f = (double)(W + 1 - d) / (double)W;
  return exp(-coef * eta * f * f);
}

// ------------------------------------------------------------------ row forward

template <typename T, int L>
__global__ __launch_bounds__(RowCfg<L>::WG) void k_row_fwd(const c128* __restrict__ in, cx<T>* __restrict__ out,
                                                           double* __restrict__ part, const cx<T>* __restrict__ tw,
                                                           int ny, size_t fsz, int nblk) {
  constexpr int N = L / 2, NT = RowCfg<L>::NT, RPW = RowCfg<L>::RPW, WG = RowCfg<L>::WG;
  __shared__ cx<T> lds[RPW * L];
  __shared__ double red[(WG + 63) / 64];
  const int g = threadIdx.x / NT, t = threadIdx.x % NT;
  const int row = 1 + blockIdx.x * RPW + g;
  const int comp = blockIdx.y;
  const bool valid = row < ny;
  cx<T>* buf = lds + g * L;
  const c128* src = in + comp * fsz + (size_t)row * N;
  double nrm = 0.0;
  for (int m = t; m < N; m += NT) {
    cx<T> v = czero<T>();
    if (valid && m > 0) {
      c128 a = src[m];
      nrm += abs2(a);
      v = cvt<T>(a);
    }
    odd_store(buf, N, m, v);
  }
  __syncthreads();
  fft<T, L>(buf, tw, t);
  const T scale = (T)(1.0 / sqrt(2.0 * N));
  if (valid) {
    cx<T>* dst = out + comp * fsz + (size_t)row * N;
    for (int p = t; p < N; p += NT) dst[p] = (p == 0) ? czero<T>() : dst_out(buf, p, scale);
  }
  double s = block_sum<WG>(nrm, red);
  if (threadIdx.x == 0) part[comp * nblk + blockIdx.x] = s;
}

// ------------------------------------------------------------------ row inverse (to complex128)

template <typename T, int L>
__global__ __launch_bounds__(RowCfg<L>::WG) void k_row_inv(const cx<T>* __restrict__ in, c128* __restrict__ out,
                                                           const cx<T>* __restrict__ tw, int ny, size_t fsz) {
  constexpr int N = L / 2, NT = RowCfg<L>::NT, RPW = RowCfg<L>::RPW;
  __shared__ cx<T> lds[RPW * L];
  const int g = threadIdx.x / NT, t = threadIdx.x % NT;
  const int row = blockIdx.x * RPW + g;  // all rows, row 0 -> zeros
  const int comp = blockIdx.y;
  const bool valid = row < ny && row > 0;
  cx<T>* buf = lds + g * L;
  const cx<T>* src = in + comp * fsz + (size_t)row * N;
  for (int m = t; m < N; m += NT) odd_store(buf, N, m, (valid && m > 0) ? src[m] : czero<T>());
  __syncthreads();
  fft<T, L>(buf, tw, t);
  const T scale = (T)(1.0 / sqrt(2.0 * N));
  if (row < ny) {
    c128* dst = out + comp * fsz + (size_t)row * N;
    for (int p = t; p < N; p += NT)
      dst[p] = (!valid || p == 0) ? mk(0.0, 0.0) : cvt<double>(dst_out(buf, p, scale));
  }
}

// ------------------------------------------------------------------ column pass (preconditioner)

template <typename T, int L, int NC, bool SHARED>
__global__ __launch_bounds__((ColCfg<T, L>::WG)) void k_col(const cx<T>* const* __restrict__ uptr,
                                                          cx<T>* __restrict__ zbase, size_t zsp, size_t zsi,
                                                          cx<T>* __restrict__ dzbase, size_t dzsp,
                                                          const PoleState* __restrict__ st,
                                                          const int* __restrict__ active, int nactive,
                                                          const double* __restrict__ mu_x,
                                                          const double* __restrict__ mu_y,
                                                          const cx<T>* __restrict__ tw, int nx, size_t fsz,
                                                          StencilCoef sc) {
  constexpr int N = L / 2, NT = ColCfg<T, L>::NT, C = ColCfg<T, L>::C, WG = ColCfg<T, L>::WG;
  constexpr int EPT = ((N - 1) * C + WG - 1) / WG;
  __shared__ cx<T> lds[C * L];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int col0 = 1 + tile * C;
  const int comp = blockIdx.y % NC;
  const int g = threadIdx.x / NT, t = threadIdx.x % NT;
  const T scale = (T)(1.0 / sqrt(2.0 * N));
  const int first = SHARED ? 0 : blockIdx.y / NC;
  const int last = SHARED ? nactive : first + 1;

  // load the column tile of u (row r = 1 + e / C, column col0 + e % C)
  {
    const int k0 = active[first];
    const int m0 = st[k0].m;
    const cx<T>* u = uptr[k0 * (HP_MAXM + 1) + m0] + comp * fsz;
    for (int e = threadIdx.x; e < (N - 1) * C; e += WG) {
      const int r = 1 + e / C, c = e % C, col = col0 + c;
      cx<T> v = (col < nx) ? u[(size_t)r * nx + col] : czero<T>();
      cx<T>* bc = lds + c * L;
      bc[r] = v;
      bc[L - r] = -v;
    }
    if (threadIdx.x < C) {
      lds[threadIdx.x * L] = czero<T>();
      lds[threadIdx.x * L + N] = czero<T>();
    }
  }
  __syncthreads();
  fft<T, L>(lds + g * L, tw, t);
  // spectral coefficients of this tile, kept in registers (row p, column c)
  cx<T> X[EPT];
#pragma unroll
  for (int s = 0; s < EPT; ++s) {
    const int e = threadIdx.x + s * WG;
    if (e < (N - 1) * C) {
      const int p = 1 + e / C, c = e % C;
      X[s] = dst_out(lds + c * L, p, scale);
    }
  }
  for (int a = first; a < last; ++a) {
    const int k = active[a];
    const int m = st[k].m;
    const c128 b = st[k].bk;
    const T sig = (T)st[k].sigma[m];
    __syncthreads();  // everyone is done reading lds
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
      const int e = threadIdx.x + s * WG;
      if (e < (N - 1) * C) {
        const int p = 1 + e / C, c = e % C, q = col0 + c;
        const double lr = mu_y[p] + (q < nx ? mu_x[q] : 0.0) - b.re, li = -b.im;
        const double den = lr * lr + li * li;
        const cx<T> inv = mk<T>((T)(lr / den), (T)(-li / den));
        const cx<T> zt = X[s] * inv;
        cx<T>* bc = lds + c * L;
        bc[p] = zt;
        bc[L - p] = -zt;
      }
    }
    if (threadIdx.x < C) {
      lds[threadIdx.x * L] = czero<T>();
      lds[threadIdx.x * L + N] = czero<T>();
    }
    __syncthreads();
    fft<T, L>(lds + g * L, tw, t);
    cx<T>* z = zbase + k * zsp + m * zsi + comp * fsz;
    const T sc2 = sig * scale;
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
      const int e = threadIdx.x + s * WG;
      if (e < (N - 1) * C) {
        const int p = 1 + e / C, c = e % C, col = col0 + c;
        if (col < nx) z[(size_t)p * nx + col] = sc2 * mul_i(lds[c * L + p]);
      }
    }
    if constexpr (NC == 2) {
      // D1y of the physical-in-y column (odd reflection about rows 0 and N)
      cx<T>* dz = dzbase + k * dzsp + comp * fsz;
#pragma unroll
      for (int s = 0; s < EPT; ++s) {
        const int e = threadIdx.x + s * WG;
        if (e < (N - 1) * C) {
          const int p = 1 + e / C, c = e % C, col = col0 + c;
          const cx<T>* bc = lds + c * L;
          cx<double> acc = mk(0.0, 0.0);
#pragma unroll
          for (int mm = 1; mm <= 6; ++mm) {
            int ip = p + mm, im = p - mm;
            cx<T> zp = czero<T>(), zm = czero<T>();
            if (ip < N) zp = bc[ip];
            else if (ip > N) zp = -bc[2 * N - ip];
            if (im > 0) zm = bc[im];
            else if (im < 0) zm = -bc[-im];
            cx<T> dif = zp - zm;
            acc = acc + sc.d1y[mm - 1] * cvt<double>(dif);
          }
          if (col < nx) dz[(size_t)p * nx + col] = sc2 * mul_i(cvt<T>(acc));
        }
      }
    }
  }
}

// ------------------------------------------------------------------ row pass (medium part + inner products)

template <int L, int NC>
struct ApplyCfg {
  static constexpr int NT = L / 8;
  static constexpr int G0 = 256 / NT;
  static constexpr int GROUPS = G0 < NC ? NC : G0;  // transforms per workgroup (NC per row)
  static constexpr int ROWS = GROUPS / NC;
  static constexpr int WG = GROUPS * NT;
};

template <typename T, int L, int NC>
__global__ __launch_bounds__((ApplyCfg<L, NC>::WG)) void k_row_apply(
    const cx<T>* __restrict__ zbase, size_t zsp, size_t zsi, const cx<T>* __restrict__ dzbase, size_t dzsp,
    cx<T>* __restrict__ pbase, size_t psp, const cx<T>* const* __restrict__ uptr, const double* __restrict__ coef,
    const PoleState* __restrict__ st, const int* __restrict__ active, double2* __restrict__ part, int nblk,
    const cx<T>* __restrict__ tw, int ny, size_t fsz, StencilCoef sc) {
  constexpr int N = L / 2, NT = ApplyCfg<L, NC>::NT, GROUPS = ApplyCfg<L, NC>::GROUPS;
  constexpr int ROWS = ApplyCfg<L, NC>::ROWS, WG = ApplyCfg<L, NC>::WG;
  constexpr int PT = N / NT;  // values per thread per row
  __shared__ cx<T> lds[GROUPS * L];
  __shared__ double red[(WG + 63) / 64];
  const int g = threadIdx.x / NT, t = threadIdx.x % NT;
  const int comp = g % NC;
  const int row = 1 + blockIdx.x * ROWS + g / NC;
  const bool valid = row < ny;
  const int k = active[blockIdx.y];
  const int m = st[k].m;
  cx<T>* buf = lds + g * L;
  const T scale = (T)(1.0 / sqrt(2.0 * N));
  const size_t roff = comp * fsz + (size_t)row * N;
  const size_t ci0 = (size_t)row * N;

  const cx<T>* z = zbase + k * zsp + m * zsi;
  for (int j = t; j < N; j += NT) odd_store(buf, N, j, (valid && j > 0) ? z[roff + j] : czero<T>());
  __syncthreads();
  fft<T, L>(buf, tw, t);
  cx<T> pz[PT];  // P z at the thread's points j = t + s * NT
  if constexpr (NC == 1) {
#pragma unroll
    for (int s = 0; s < PT; ++s) {
      const int j = t + s * NT;
      const cx<T> zj = (j == 0) ? czero<T>() : dst_out(buf, j, scale);
      const T v = valid ? (T)coef[ci0 + j] : (T)0;
      pz[s] = v * zj;
    }
  } else {
    // eq. Z_bar_eq, medium part (coefficient planes carry s = 1/(k0 n0)^2):
    //   (P w)_1 = psi_xx w1 + psi_x D1x w1 + psi_xy w2 + psi_y D1x w2 + V w1
    //   (P w)_2 = psi_xy w1 + psi_x D1y w1 + psi_yy w2 + psi_y D1y w2 + V w2
    cx<T> zc[PT], dxz[PT], dyz[PT];
#pragma unroll
    for (int s = 0; s < PT; ++s) {
      const int j = t + s * NT;
      zc[s] = (j == 0) ? czero<T>() : dst_out(buf, j, scale);
      cx<double> acc = mk(0.0, 0.0);
#pragma unroll
      for (int mm = 1; mm <= 6; ++mm) {
        const int jp = j + mm, jm = j - mm;
        cx<T> a = czero<T>(), b = czero<T>();
        if (jp < N) a = buf[jp];
        else if (jp > N) a = -buf[2 * N - jp];
        if (jm > 0) b = buf[jm];
        else if (jm < 0) b = -buf[-jm];
        acc = acc + sc.d1x[mm - 1] * cvt<double>(a - b);
      }
      dxz[s] = (j == 0) ? czero<T>() : scale * mul_i(cvt<T>(acc));
    }
    __syncthreads();
    const cx<T>* dz = dzbase + k * dzsp;
    for (int j = t; j < N; j += NT) odd_store(buf, N, j, (valid && j > 0) ? dz[roff + j] : czero<T>());
    __syncthreads();
    fft<T, L>(buf, tw, t);
#pragma unroll
    for (int s = 0; s < PT; ++s) {
      const int j = t + s * NT;
      dyz[s] = (j == 0) ? czero<T>() : dst_out(buf, j, scale);
    }
    __syncthreads();
    // exchange: component 0 needs w2 and D1x w2, component 1 needs w1 and D1y w1
#pragma unroll
    for (int s = 0; s < PT; ++s) {
      const int j = t + s * NT;
      buf[j] = zc[s];
      buf[N + j] = (comp == 0) ? dyz[s] : dxz[s];
    }
    __syncthreads();
    const cx<T>* other = lds + (g ^ 1) * L;
#pragma unroll
    for (int s = 0; s < PT; ++s) {
      const int j = t + s * NT;
      if (!valid) {
        pz[s] = czero<T>();
        continue;
      }
      const size_t ci = ci0 + j;
      const T v = (T)coef[ci], px = (T)coef[fsz + ci], py = (T)coef[2 * fsz + ci];
      const T pxx = (T)coef[3 * fsz + ci], pyy = (T)coef[4 * fsz + ci], pxy = (T)coef[5 * fsz + ci];
      const cx<T> zo = other[j], dzo = other[N + j];
      if (comp == 0)
        pz[s] = pxx * zc[s] + px * dxz[s] + pxy * zo + py * dzo + v * zc[s];
      else
        pz[s] = pxy * zo + px * dzo + pyy * zc[s] + py * dyz[s] + v * zc[s];
    }
    __syncthreads();
  }
  // forward transform of P z
#pragma unroll
  for (int s = 0; s < PT; ++s) odd_store(buf, N, t + s * NT, pz[s]);
  __syncthreads();
  fft<T, L>(buf, tw, t);
  cx<T> pv[PT];
  cx<T>* p = pbase + k * psp;
#pragma unroll
  for (int s = 0; s < PT; ++s) {
    const int j = t + s * NT;
    pv[s] = (j == 0 || !valid) ? czero<T>() : dst_out(buf, j, scale);
    if (valid) p[roff + j] = pv[s];
  }
  // <u_i, p> and <u_i, u_m>, i = 0..m, summed over the workgroup (rows and
  // components): the new direction's projections and the reorthogonalisation
  // of the provisional u_m, from the same reads of the basis.
  cx<T> um[PT];
  {
    const cx<T>* u = uptr[k * (HP_MAXM + 1) + m];
#pragma unroll
    for (int s = 0; s < PT; ++s) um[s] = valid ? u[roff + t + s * NT] : czero<T>();
  }
  for (int i = 0; i <= m; ++i) {
    const cx<T>* u = uptr[k * (HP_MAXM + 1) + i];
    double pr = 0.0, pi = 0.0, qr = 0.0, qi = 0.0;
    if (valid) {
#pragma unroll
      for (int s = 0; s < PT; ++s) {
        const int j = t + s * NT;
        const cx<double> a = cvt<double>(i == m ? um[s] : u[roff + j]);
        const cx<double> b = cvt<double>(pv[s]);
        const cx<double> c = cvt<double>(um[s]);
        pr += a.re * b.re + a.im * b.im;
        pi += a.re * b.im - a.im * b.re;
        qr += a.re * c.re + a.im * c.im;
        qi += a.re * c.im - a.im * c.re;
      }
    }
    pr = block_sum<WG>(pr, red);
    pi = block_sum<WG>(pi, red);
    qr = block_sum<WG>(qr, red);
    qi = block_sum<WG>(qi, red);
    if (threadIdx.x == 0) {
      const size_t base = (((size_t)k * (HP_MAXM + 1) + i) * 2) * nblk + blockIdx.x;
      part[base] = make_double2(pr, pi);
      part[base + nblk] = make_double2(qr, qi);
    }
  }
}

// ------------------------------------------------------------------ Gram-Schmidt update

constexpr int UPD_WG = 256;

// u_{m+1} = cu_{m+1} p + sum_{i<=m} cu_i u_i, and (delayed reorthogonalisation)
// u_m <- sum_{i<=m} cv_i u_i in place; partial |u_{m+1}|^2.
template <typename T>
__global__ __launch_bounds__(UPD_WG) void k_update(const cx<T>* __restrict__ pbase, size_t psp,
                                                   cx<T>* const* __restrict__ uptr, const PoleState* __restrict__ st,
                                                   const int* __restrict__ active, double* __restrict__ part, int nblk,
                                                   size_t total) {
  __shared__ c128 cf[HP_MAXM + 2];
  __shared__ c128 cv[HP_MAXM + 1];
  __shared__ cx<T>* up[HP_MAXM + 2];
  __shared__ double red[UPD_WG / 64];
  const int k = active[blockIdx.y];
  const int m = st[k].m;
  const int corr = st[k].correct;
  for (int i = threadIdx.x; i <= m + 1; i += UPD_WG) {
    cf[i] = st[k].cu[i];
    up[i] = uptr[k * (HP_MAXM + 1) + i];
    if (i <= m) cv[i] = st[k].cv[i];
  }
  __syncthreads();
  const cx<T>* p = pbase + k * psp;
  cx<T>* out = up[m + 1];
  cx<T>* um = up[m];
  double nrm = 0.0;
  for (size_t idx = (size_t)blockIdx.x * UPD_WG + threadIdx.x; idx < total; idx += (size_t)gridDim.x * UPD_WG) {
    cx<double> v = cf[m + 1] * cvt<double>(p[idx]);
    cx<double> c = mk(0.0, 0.0);
    for (int i = 0; i <= m; ++i) {
      const cx<double> ui = cvt<double>(up[i][idx]);
      v = v + cf[i] * ui;
      c = c + cv[i] * ui;
    }
    const cx<T> r = cvt<T>(v);
    out[idx] = r;
    if (corr) um[idx] = cvt<T>(c);
    nrm += abs2(cvt<double>(r));
  }
  double s = block_sum<UPD_WG>(nrm, red);
  if (threadIdx.x == 0) part[(size_t)k * nblk + blockIdx.x] = s;
}

// ------------------------------------------------------------------ reductions / small FP64 kernels

// Sum the partial inner products, then (one thread) the delayed
// reorthogonalisation algebra of step m in FP64:
//   s_i = <v_i, ~v_m>, t = <~v_m, ~v_m>, rho^2 = t - sum |s_i|^2,
//   v_m = (~v_m - sum s_i v_i) / rho,
//   column m-1:  H[i][m-1] += h~ s_i,  H[m][m-1] = h~ rho  (h~ = old H[m][m-1]),
//   c_i = <v_i, p>, c_m = (<~v_m, p> - sum conj(s_i) c_i) / rho,
//   A M^-1 v_m = (~v_m + p - sum_i s_i A M^-1 v_i) / rho   (A M^-1 ~v_m = ~v_m + p),
//   H[l][m] = <v_l, A M^-1 v_m>, u_{m+1} = A M^-1 v_m - sum_l H[l][m] v_l,
// expressed as coefficients of the stored vectors for the update kernel.
__global__ __launch_bounds__(256) void k_reduce_prep(const double2* __restrict__ part, int nblk,
                                                     PoleState* __restrict__ st, const int* __restrict__ active) {
  __shared__ double red[4];
  __shared__ c128 P[HP_MAXM + 1], Q[HP_MAXM + 1];
  const int k = active[blockIdx.x];
  const int m = st[k].m;
  for (int i = 0; i <= m; ++i) {
    for (int slot = 0; slot < 2; ++slot) {
      const double2* src = part + (((size_t)k * (HP_MAXM + 1) + i) * 2 + slot) * nblk;
      double re = 0.0, im = 0.0;
      for (int b = threadIdx.x; b < nblk; b += 256) {
        re += src[b].x;
        im += src[b].y;
      }
      re = block_sum<256>(re, red);
      im = block_sum<256>(im, red);
      if (threadIdx.x == 0) (slot ? Q : P)[i] = mk(re, im);
    }
  }
  if (threadIdx.x != 0) return;
  PoleState& S = st[k];
  constexpr int LD = HP_MAXM + 1;
  c128* Hr = S.Hraw;
  const double sm = S.sigma[m];
  c128 sv[HP_MAXM], cc[HP_MAXM + 1];
  double ssum = 0.0;
  for (int i = 0; i < m; ++i) {
    sv[i] = (S.sigma[i] * sm) * Q[i];
    ssum += abs2(sv[i]);
    cc[i] = S.sigma[i] * P[i];
  }
  const double t = sm * sm * Q[m].re;
  double rho2 = t - ssum;
  if (!(rho2 > 1e-300)) rho2 = 1e-300;
  const double rho = sqrt(rho2);
  for (int i = 0; i < m; ++i) S.Rc[i + m * LD] = sv[i];
  S.Rc[m + m * LD] = mk(rho, 0.0);
  if (m == 0) {
    S.g[0] = rho * S.g[0];
  } else {
    const double ht = Hr[m + (m - 1) * LD].re;
    for (int i = 0; i < m; ++i) Hr[i + (m - 1) * LD] = Hr[i + (m - 1) * LD] + ht * sv[i];
    Hr[m + (m - 1) * LD] = mk(ht * rho, 0.0);
  }
  c128 cm = sm * P[m];
  for (int i = 0; i < m; ++i) cm = cm - cmulc(sv[i], cc[i]);
  cc[m] = (1.0 / rho) * cm;
  // A_l = sum_{i<m, i>=l-1} s_i H[l][i]
  c128 h[HP_MAXM + 1];
  double gam_re = 0.0, gam_im = 0.0;
  for (int l = 0; l <= m; ++l) {
    c128 A = mk(0.0, 0.0);
    for (int i = (l > 0 ? l - 1 : 0); i < m; ++i) A = A + sv[i] * Hr[l + i * LD];
    c128 base = (l < m) ? sv[l] + cc[l] : mk(rho, 0.0) + cc[m];
    h[l] = (1.0 / rho) * (base - A);
    Hr[l + m * LD] = h[l];
    if (l == m) {
      const c128 gam = (1.0 / rho) * A + h[m];
      gam_re = gam.re;
      gam_im = gam.im;
    }
    // coefficient of v_l (l < m) without the gamma term: -(A_l / rho + h_l)
    if (l < m) S.cu[l] = -1.0 * ((1.0 / rho) * A + h[l]);
  }
  const c128 gam = mk(gam_re, gam_im);
  for (int l = 0; l < m; ++l) S.cu[l] = S.sigma[l] * (S.cu[l] + (1.0 / rho) * (gam * sv[l]));
  S.cu[m] = (sm / rho) * (mk(1.0, 0.0) - gam);
  S.cu[m + 1] = mk(1.0 / rho, 0.0);
  if (m == 0) {
    // v_0 = ~v_0 / rho is a rescale of the (possibly shared) stored vector
    S.sigma[0] = sm / rho;
    S.correct = 0;
  } else {
    for (int i = 0; i < m; ++i) S.cv[i] = (-S.sigma[i] / rho) * sv[i];
    S.cv[m] = mk(sm / rho, 0.0);
    S.sigma[m] = 1.0;
    S.correct = 1;
  }
}

__device__ __forceinline__ void givens(c128 a, double b, double& c, c128& sn, c128& r) {
  const double aa = sqrt(abs2(a));
  const double rho = sqrt(aa * aa + b * b);
  if (rho == 0.0) {
    c = 1.0;
    sn = mk(0.0, 0.0);
  } else if (aa == 0.0) {
    c = 0.0;
    sn = mk(1.0, 0.0);
  } else {
    c = aa / rho;
    sn = (b / (rho * aa)) * a;  // (a/|a|) conj(b)/rho with b real
  }
  r = c * a + b * sn;
}

__global__ __launch_bounds__(64) void k_arnoldi(PoleState* __restrict__ st, const int* __restrict__ active,
                                                const double* __restrict__ part, int nblk, int restart,
                                                int* __restrict__ flags, double* __restrict__ ests) {
  const int k = active[blockIdx.x];
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64) s += part[(size_t)k * nblk + b];
  s = wave_sum(s);
  if (threadIdx.x != 0) return;
  PoleState& S = st[k];
  constexpr int LD = HP_MAXM + 1;
  const int m = S.m;
  const double h = sqrt(s);
  S.Hraw[m + 1 + m * LD] = mk(h, 0.0);
  if (m >= 1) {
    // column m-1 was corrected by the reorthogonalisation: redo its rotation
    c128* col = S.H + (m - 1) * LD;
    for (int i = 0; i <= m; ++i) col[i] = S.Hraw[i + (m - 1) * LD];
    for (int i = 0; i < m - 1; ++i) {
      const c128 a = col[i], b = col[i + 1];
      col[i] = S.cs[i] * a + S.sn[i] * b;
      col[i + 1] = -1.0 * cmulc(S.sn[i], a) + S.cs[i] * b;
    }
    double c;
    c128 sn, r;
    givens(col[m - 1], col[m].re, c, sn, r);
    S.cs[m - 1] = c;
    S.sn[m - 1] = sn;
    col[m - 1] = r;
    col[m] = mk(0.0, 0.0);
    S.g[m - 1] = c * S.gpre[m - 1];
    S.g[m] = -1.0 * cmulc(sn, S.gpre[m - 1]);
  }
  c128* col = S.H + m * LD;
  for (int i = 0; i <= m + 1; ++i) col[i] = S.Hraw[i + m * LD];
  for (int i = 0; i < m; ++i) {
    const c128 a = col[i], b = col[i + 1];
    col[i] = S.cs[i] * a + S.sn[i] * b;
    col[i + 1] = -1.0 * cmulc(S.sn[i], a) + S.cs[i] * b;
  }
  double c;
  c128 sn, r;
  givens(col[m], h, c, sn, r);
  S.cs[m] = c;
  S.sn[m] = sn;
  col[m] = r;
  col[m + 1] = mk(0.0, 0.0);
  S.gpre[m] = S.g[m];
  S.g[m + 1] = -1.0 * cmulc(sn, S.g[m]);
  S.g[m] = c * S.g[m];
  S.sigma[m + 1] = (h > 0.0) ? 1.0 / h : 0.0;
  S.est = sqrt(abs2(S.g[m + 1]));
  S.m = m + 1;
  S.total += 1;
  int flag = 0;
  if (S.fixed > 0) {
    if (S.m >= S.fixed) flag = 1;
  } else if (S.est <= S.tol || h == 0.0) {
    flag = 1;
  } else if (S.m >= restart) {
    flag = 2;
  }
  S.flag = flag;
  if (flag) {
    // least squares R y = g, then y~ = Rc^{-1} y (the coefficients of the stored Z~)
    const int n = S.m;
    c128 y[HP_MAXM];
    for (int i = n - 1; i >= 0; --i) {
      c128 acc = S.g[i];
      for (int l = i + 1; l < n; ++l) acc = acc - S.H[i + l * LD] * y[l];
      const c128 d = S.H[i + i * LD];
      y[i] = (abs2(d) > 0.0) ? cdiv(acc, d) : mk(0.0, 0.0);
    }
    for (int i = n - 1; i >= 0; --i) {
      c128 acc = y[i];
      for (int l = i + 1; l < n; ++l) acc = acc - S.Rc[i + l * LD] * S.y[l];
      S.y[i] = cdiv(acc, S.Rc[i + i * LD]);
    }
    // The estimate measures the split operator I + P M~^-1; it differs from
    // A M~^-1 by about eps kappa(M_k) ||y|| (||y|| = ||M x||).  When that is not
    // well below tol, the true residual decides.
    if (flag == 1 && S.fixed == 0) {
      double yn = 0.0;
      for (int i = 0; i < n; ++i) yn += abs2(y[i]);
      if (S.incons * sqrt(yn) > 0.1 * S.tol) flag = 3;
      S.flag = flag;
    }
  }
  flags[k] = flag;
  ests[k] = S.est;
}

__global__ __launch_bounds__(64) void k_cycle_init(PoleState* __restrict__ st, const int* __restrict__ poles,
                                                   const double* __restrict__ part, int nblk, int first, double tol,
                                                   double rtol_cycle) {
  const int k = poles[blockIdx.x];
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64) s += part[b];
  s = wave_sum(s);
  if (threadIdx.x != 0) return;
  PoleState& S = st[k];
  const double beta = sqrt(s);
  if (first) {
    S.beta0 = beta;
    S.total = 0;
    S.cycle = 0;
    S.has_x = 0;
  } else {
    S.cycle += 1;
  }
  S.beta = beta;
  S.tol = fmax(tol * S.beta0, rtol_cycle * beta);
  S.m = 0;
  S.flag = 0;
  S.est = beta;
  S.g[0] = mk(beta, 0.0);
  S.sigma[0] = (beta > 0.0) ? 1.0 / beta : 0.0;
  S.correct = 0;
}

// ------------------------------------------------------------------ residue-weighted sum and output

template <typename T, int L>
__global__ __launch_bounds__(RowCfg<L>::WG) void k_final(const c128* __restrict__ w, c128* __restrict__ out,
                                                         const cx<T>* __restrict__ zbase, size_t zsp, size_t zsi,
                                                         const c128* __restrict__ xacc, size_t xsp,
                                                         const PoleState* __restrict__ st, int npoles, c128 phase,
                                                         c128 rinf_phase, double loss_coef, double eta, int W,
                                                         const c128* __restrict__ tw, int nx, int ny, size_t fsz) {
  constexpr int N = L / 2, NT = RowCfg<L>::NT, RPW = RowCfg<L>::RPW;
  constexpr int PT = N / NT;
  __shared__ c128 lds[RPW * L];
  const int g = threadIdx.x / NT, t = threadIdx.x % NT;
  const int row = blockIdx.x * RPW + g;  // rows 0..ny-1
  const int comp = blockIdx.y;
  const bool valid = row > 0 && row < ny;
  c128* buf = lds + g * L;
  const size_t roff = comp * fsz + (size_t)row * N;
  c128 acc[PT];
#pragma unroll
  for (int s = 0; s < PT; ++s) acc[s] = mk(0.0, 0.0);
  if (valid) {
    for (int k = 0; k < npoles; ++k) {
      const c128 ak = st[k].ak;
      if (st[k].has_x) {
        const c128* xk = xacc + k * xsp + roff;
#pragma unroll
        for (int s = 0; s < PT; ++s) acc[s] = acc[s] + ak * xk[t + s * NT];
      }
      const int mk_ = st[k].m;
      const cx<T>* zk = zbase + k * zsp + roff;
      for (int i = 0; i < mk_; ++i) {
        const c128 cf = ak * st[k].y[i];
        const cx<T>* zi = zk + i * zsi;
#pragma unroll
        for (int s = 0; s < PT; ++s) acc[s] = acc[s] + cf * cvt<double>(zi[t + s * NT]);
      }
    }
  }
#pragma unroll
  for (int s = 0; s < PT; ++s) odd_store(buf, N, t + s * NT, acc[s]);
  __syncthreads();
  fft<double, L>(buf, tw, t);
  const double scale = 1.0 / sqrt(2.0 * N);
  if (row < ny) {
#pragma unroll
    for (int s = 0; s < PT; ++s) {
      const int j = t + s * NT;
      c128 v = mk(0.0, 0.0);
      if (valid && j > 0) {
        const c128 sv = dst_out(buf, j, scale);
        v = edge_loss(row, j, nx, ny, W, eta, loss_coef) * (phase * sv + rinf_phase * w[roff + j]);
      }
      out[roff + j] = v;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_accum(c128* __restrict__ xacc, const cx<T>* __restrict__ z, size_t zsi,
                                               const PoleState* __restrict__ st, int pole, size_t total) {
  const int m = st[pole].m;
  const int hx = st[pole].has_x;
  for (size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (size_t)gridDim.x * 256) {
    c128 acc = hx ? xacc[idx] : mk(0.0, 0.0);
    for (int i = 0; i < m; ++i) acc = acc + st[pole].y[i] * cvt<double>(z[i * zsi + idx]);
    xacc[idx] = acc;
  }
}

// ------------------------------------------------------------------ explicit operator (FP64)

__device__ __forceinline__ c128 ld_odd(const c128* __restrict__ x, int i, int j, int nx, int ny) {
  double sg = 1.0;
  if (i < 0) {
    i = -i;
    sg = -sg;
  } else if (i > ny) {
    i = 2 * ny - i;
    sg = -sg;
  }
  if (j < 0) {
    j = -j;
    sg = -sg;
  } else if (j > nx) {
    j = 2 * nx - j;
    sg = -sg;
  }
  if (i == 0 || j == 0 || i == ny || j == nx) return mk(0.0, 0.0);
  return sg * x[(size_t)i * nx + j];
}

constexpr int OP_WG = 256;

__global__ __launch_bounds__(OP_WG) void k_apply_op(const c128* __restrict__ x, const c128* __restrict__ rhs,
                                                    c128* __restrict__ y, const double* __restrict__ coef, c128 b,
                                                    StencilCoef sc, int nx, int ny, int ncomp, size_t fsz,
                                                    double* __restrict__ part) {
  __shared__ double red[OP_WG / 64];
  double nrm = 0.0;
  const size_t idx = (size_t)blockIdx.x * OP_WG + threadIdx.x;
  if (idx < fsz) {
    const int i = (int)(idx / nx), j = (int)(idx % nx);
    const bool inner = i > 0 && j > 0;
    c128 lap[2], d1x[2], d1y[2], xc[2];
    for (int c = 0; c < ncomp; ++c) {
      const c128* xc_ = x + c * fsz;
      c128 l = mk(0.0, 0.0), ax = mk(0.0, 0.0), ay = mk(0.0, 0.0);
      const c128 x0 = inner ? xc_[idx] : mk(0.0, 0.0);
      if (inner) {
        l = (sc.c2x[0] + sc.c2y[0]) * x0;
        for (int mm = 1; mm <= 6; ++mm) {
          const c128 xp = ld_odd(xc_, i, j + mm, nx, ny), xm = ld_odd(xc_, i, j - mm, nx, ny);
          const c128 yp = ld_odd(xc_, i + mm, j, nx, ny), ym = ld_odd(xc_, i - mm, j, nx, ny);
          l = l + sc.c2x[mm] * (xp + xm) + sc.c2y[mm] * (yp + ym);
          ax = ax + sc.d1x[mm - 1] * (xp - xm);
          ay = ay + sc.d1y[mm - 1] * (yp - ym);
        }
      }
      lap[c] = l;
      d1x[c] = ax;
      d1y[c] = ay;
      xc[c] = x0;
    }
    const double V = coef[idx];
    for (int c = 0; c < ncomp; ++c) {
      c128 v = lap[c] + V * xc[c] - b * xc[c];
      if (ncomp == 2) {
        const double px = coef[fsz + idx], py = coef[2 * fsz + idx], pxx = coef[3 * fsz + idx],
                     pyy = coef[4 * fsz + idx], pxy = coef[5 * fsz + idx];
        if (c == 0)
          v = v + pxx * xc[0] + px * d1x[0] + pxy * xc[1] + py * d1x[1];
        else
          v = v + pxy * xc[0] + px * d1y[0] + pyy * xc[1] + py * d1y[1];
      }
      if (!inner) v = mk(0.0, 0.0);
      if (rhs) v = (inner ? rhs[c * fsz + idx] : mk(0.0, 0.0)) - v;
      y[c * fsz + idx] = v;
      nrm += abs2(v);
    }
  }
  double s = block_sum<OP_WG>(nrm, red);
  if (threadIdx.x == 0 && part) part[blockIdx.x] = s;
}

// ------------------------------------------------------------------ coefficient preparation

__global__ __launch_bounds__(256) void k_coef_a(const double* __restrict__ n2, double* __restrict__ coef,
                                                double* __restrict__ psi, double n0, int W, int nx, int ny,
                                                size_t fsz, int vector) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= fsz) return;
  const int i = (int)(idx / nx), j = (int)(idx % nx);
  const int d = min(min(i, ny - i), min(j, nx - j));
  const double v = n2[idx];
  coef[idx] = (d > W) ? (v - n0 * n0) / (n0 * n0) : 0.0;
  if (vector) psi[idx] = log(v);
}

// first derivative of psi along x (valid where the stencil stays inside)
__global__ __launch_bounds__(256) void k_coef_b(const double* __restrict__ psi, double* __restrict__ dpx,
                                                StencilCoef sc, int nx, int ny, size_t fsz) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= fsz) return;
  const int j = (int)(idx % nx);
  double a = 0.0;
  if (j >= 6 && j + 6 < nx)
    for (int mm = 1; mm <= 6; ++mm) a += sc.d1x[mm - 1] * (psi[idx + mm] - psi[idx - mm]);
  dpx[idx] = a;
}

__global__ __launch_bounds__(256) void k_coef_c(const double* __restrict__ psi, const double* __restrict__ dpx,
                                                double* __restrict__ coef, double s, StencilCoef sc, int W, int nx,
                                                int ny, size_t fsz) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= fsz) return;
  const int i = (int)(idx / nx), j = (int)(idx % nx);
  const int d = min(min(i, ny - i), min(j, nx - j));
  double px = 0, py = 0, pxx = 0, pyy = 0, pxy = 0;
  if (d > W) {
    // c2x, c2y already carry s; the psi terms of Zbar are multiplied by s too
    pxx = sc.c2x[0] * psi[idx];
    pyy = sc.c2y[0] * psi[idx];
    for (int mm = 1; mm <= 6; ++mm) {
      pxx += sc.c2x[mm] * (psi[idx + mm] + psi[idx - mm]);
      pyy += sc.c2y[mm] * (psi[idx + (size_t)mm * nx] + psi[idx - (size_t)mm * nx]);
      px += sc.d1x[mm - 1] * (psi[idx + mm] - psi[idx - mm]);
      py += sc.d1y[mm - 1] * (psi[idx + (size_t)mm * nx] - psi[idx - (size_t)mm * nx]);
      pxy += sc.d1y[mm - 1] * (dpx[idx + (size_t)mm * nx] - dpx[idx - (size_t)mm * nx]);
    }
    px *= s;
    py *= s;
    pxy *= s;
  }
  coef[fsz + idx] = px;
  coef[2 * fsz + idx] = py;
  coef[3 * fsz + idx] = pxx;
  coef[4 * fsz + idx] = pyy;
  coef[5 * fsz + idx] = pxy;
}

__global__ void k_fill_zero(c128* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = mk(0.0, 0.0);
}

}  // namespace

// ====================================================================== launchers

#define HP_DISPATCH_L(n, MACRO) \
  switch (n) {                  \
    case 64: MACRO(128); break; \
    case 128: MACRO(256); break;  \
    case 256: MACRO(512); break;  \
    case 512: MACRO(1024); break; \
    case 1024: MACRO(2048); break; \
    case 2048: MACRO(4096); break; \
    default: break;             \
  }

template <typename T>
int row_blocks(int nx) {
  int L = 2 * nx;
  int NT = L / 8;
  int RPW = (256 / NT) > 0 ? 256 / NT : 1;
  (void)sizeof(T);
  return RPW;  // rows per workgroup
}

template <typename T>
void launch_row_fwd(const c128* in, cx<T>* out, double* part, const cx<T>* tw, const Geo& g, hipStream_t s) {
  const int rpw = row_blocks<T>(g.nx);
  const int nblk = (g.ny - 1 + rpw - 1) / rpw;
  dim3 grid(nblk, g.ncomp);
#define L_(LL) \
  hipLaunchKernelGGL((k_row_fwd<T, LL>), grid, dim3(RowCfg<LL>::WG), 0, s, in, out, part, tw, g.ny, g.fsz, nblk)
  HP_DISPATCH_L(g.nx, L_)
#undef L_
}

template <typename T>
void launch_row_inv(const cx<T>* in, c128* out, const cx<T>* tw, const Geo& g, hipStream_t s) {
  const int rpw = row_blocks<T>(g.nx);
  const int nblk = (g.ny + rpw - 1) / rpw;
  dim3 grid(nblk, g.ncomp);
#define L_(LL) hipLaunchKernelGGL((k_row_inv<T, LL>), grid, dim3(RowCfg<LL>::WG), 0, s, in, out, tw, g.ny, g.fsz)
  HP_DISPATCH_L(g.nx, L_)
#undef L_
}

template <typename T>
void launch_col(const cx<T>* const* uptr, cx<T>* zbase, size_t zsp, size_t zsi, cx<T>* dzbase, size_t dzsp,
                const PoleState* st, const int* active, int nactive, bool shared, const double* mu_x,
                const double* mu_y, const cx<T>* tw, const Geo& g, const StencilCoef& sc, hipStream_t s) {
#define L_(LL)                                                                                               \
  {                                                                                                          \
    constexpr int C = ColCfg<T, LL>::C;                                                                      \
    dim3 grid((g.nx - 1 + C - 1) / C, g.ncomp * (shared ? 1 : nactive));                                    \
    if (g.ncomp == 1) {                                                                                      \
      if (shared)                                                                                            \
        hipLaunchKernelGGL((k_col<T, LL, 1, true>), grid, dim3(ColCfg<T, LL>::WG), 0, s, uptr, zbase, zsp,   \
                           zsi, dzbase, dzsp, st, active, nactive, mu_x, mu_y, tw, g.nx, g.fsz, sc);         \
      else                                                                                                   \
        hipLaunchKernelGGL((k_col<T, LL, 1, false>), grid, dim3(ColCfg<T, LL>::WG), 0, s, uptr, zbase, zsp,  \
                           zsi, dzbase, dzsp, st, active, nactive, mu_x, mu_y, tw, g.nx, g.fsz, sc);         \
    } else {                                                                                                 \
      if (shared)                                                                                            \
        hipLaunchKernelGGL((k_col<T, LL, 2, true>), grid, dim3(ColCfg<T, LL>::WG), 0, s, uptr, zbase, zsp,   \
                           zsi, dzbase, dzsp, st, active, nactive, mu_x, mu_y, tw, g.nx, g.fsz, sc);         \
      else                                                                                                   \
        hipLaunchKernelGGL((k_col<T, LL, 2, false>), grid, dim3(ColCfg<T, LL>::WG), 0, s, uptr, zbase, zsp,  \
                           zsi, dzbase, dzsp, st, active, nactive, mu_x, mu_y, tw, g.nx, g.fsz, sc);         \
    }                                                                                                        \
  }
  HP_DISPATCH_L(g.ny, L_)
#undef L_
}

template <typename T>
int row_apply_blocks(const Geo& g) {
  const int nt = (2 * g.nx) / 8;
  int groups = 256 / nt;
  if (groups < g.ncomp) groups = g.ncomp;
  const int rows = groups / g.ncomp;
  return (g.ny - 1 + rows - 1) / rows;
}

template <typename T>
void launch_row_apply(const cx<T>* zbase, size_t zsp, size_t zsi, const cx<T>* dzbase, size_t dzsp, cx<T>* pbase,
                      size_t psp, const cx<T>* const* uptr, const double* coef, const PoleState* st,
                      const int* active, int nactive, double2* part, const cx<T>* tw, const Geo& g,
                      const StencilCoef& sc, hipStream_t s) {
  const int nblk = row_apply_blocks<T>(g);
  dim3 grid(nblk, nactive);
#define L_(LL)                                                                                                  \
  if (g.ncomp == 1)                                                                                             \
    hipLaunchKernelGGL((k_row_apply<T, LL, 1>), grid, dim3(ApplyCfg<LL, 1>::WG), 0, s, zbase, zsp, zsi, dzbase,  \
                       dzsp, pbase, psp, uptr, coef, st, active, part, nblk, tw, g.ny, g.fsz, sc);              \
  else                                                                                                          \
    hipLaunchKernelGGL((k_row_apply<T, LL, 2>), grid, dim3(ApplyCfg<LL, 2>::WG), 0, s, zbase, zsp, zsi, dzbase,  \
                       dzsp, pbase, psp, uptr, coef, st, active, part, nblk, tw, g.ny, g.fsz, sc);
  HP_DISPATCH_L(g.nx, L_)
#undef L_
}

void launch_reduce_dots(const double2* part, int nblk, PoleState* st, const int* active, int nactive, int maxm,
                        hipStream_t s) {
  (void)maxm;
  hipLaunchKernelGGL(k_reduce_prep, dim3(nactive), dim3(256), 0, s, part, nblk, st, active);
}

int update_blocks(size_t total) {
  size_t b = (total + UPD_WG * 4 - 1) / (UPD_WG * 4);
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  return (int)b;
}

template <typename T>
void launch_update(const cx<T>* pbase, size_t psp, cx<T>* const* uptr, const PoleState* st, const int* active,
                   int nactive, double* part, int nblk, const Geo& g, hipStream_t s) {
  hipLaunchKernelGGL((k_update<T>), dim3(nblk, nactive), dim3(UPD_WG), 0, s, pbase, psp, uptr, st, active, part,
                     nblk, (size_t)g.ncomp * g.fsz);
}

void launch_arnoldi(PoleState* st, const int* active, int nactive, const double* part, int nblk, int restart,
                    int* flags, double* est, hipStream_t s) {
  hipLaunchKernelGGL(k_arnoldi, dim3(nactive), dim3(64), 0, s, st, active, part, nblk, restart, flags, est);
}

void launch_cycle_init(PoleState* st, const int* poles, int npoles_in, const double* part, int nblk, int first,
                       double tol, double rtol_cycle, hipStream_t s) {
  hipLaunchKernelGGL(k_cycle_init, dim3(npoles_in), dim3(64), 0, s, st, poles, part, nblk, first, tol, rtol_cycle);
}

template <typename T>
void launch_final(const c128* w, c128* out, const cx<T>* zbase, size_t zsp, size_t zsi, const c128* xacc, size_t xsp,
                  const PoleState* st, int npoles, c128 phase, c128 rinf_phase, double loss_coef, double eta, int W,
                  const c128* tw64, const Geo& g, hipStream_t s) {
  const int rpw = row_blocks<double>(g.nx);
  dim3 grid((g.ny + rpw - 1) / rpw, g.ncomp);
#define L_(LL)                                                                                                     \
  hipLaunchKernelGGL((k_final<T, LL>), grid, dim3(RowCfg<LL>::WG), 0, s, w, out, zbase, zsp, zsi, xacc, xsp, st, \
                     npoles, phase, rinf_phase, loss_coef, eta, W, tw64, g.nx, g.ny, g.fsz)
  HP_DISPATCH_L(g.nx, L_)
#undef L_
}

template <typename T>
void launch_accum(c128* xacc, const cx<T>* z, size_t zsi, const PoleState* st, int pole, const Geo& g,
                  hipStream_t s) {
  const size_t total = (size_t)g.ncomp * g.fsz;
  hipLaunchKernelGGL((k_accum<T>), dim3(update_blocks(total)), dim3(256), 0, s, xacc, z, zsi, st, pole, total);
}

int op_blocks(const Geo& g) { return (int)((g.fsz + OP_WG - 1) / OP_WG); }

void launch_apply_op(const c128* x, const c128* rhs, c128* y, const double* coef, c128 b, const StencilCoef& sc,
                     const Geo& g, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_apply_op, dim3(op_blocks(g)), dim3(OP_WG), 0, s, x, rhs, y, coef, b, sc, g.nx, g.ny, g.ncomp,
                     g.fsz, part);
}

void launch_coef(const double* n2, double* coef, double* scratch, double n0, double s_scale, int W,
                 const StencilCoef& sc, const Geo& g, hipStream_t s) {
  const int nb = (int)((g.fsz + 255) / 256);
  const int vector = g.ncomp == 2;
  hipLaunchKernelGGL(k_coef_a, dim3(nb), dim3(256), 0, s, n2, coef, scratch, n0, W, g.nx, g.ny, g.fsz, vector);
  if (vector) {
    hipLaunchKernelGGL(k_coef_b, dim3(nb), dim3(256), 0, s, scratch, scratch + g.fsz, sc, g.nx, g.ny, g.fsz);
    hipLaunchKernelGGL(k_coef_c, dim3(nb), dim3(256), 0, s, scratch, scratch + g.fsz, coef, s_scale, sc, W, g.nx,
                       g.ny, g.fsz);
  }
}

void launch_fill_zero_c128(c128* p, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_zero, dim3(1024), dim3(256), 0, s, p, n);
}

// explicit instantiations
#define HP_INST(T)                                                                                                   \
  template int row_blocks<T>(int);                                                                                   \
  template int row_apply_blocks<T>(const Geo&);                                                                      \
  template void launch_row_fwd<T>(const c128*, cx<T>*, double*, const cx<T>*, const Geo&, hipStream_t);              \
  template void launch_row_inv<T>(const cx<T>*, c128*, const cx<T>*, const Geo&, hipStream_t);                       \
  template void launch_col<T>(const cx<T>* const*, cx<T>*, size_t, size_t, cx<T>*, size_t, const PoleState*,         \
                              const int*, int, bool, const double*, const double*, const cx<T>*, const Geo&,         \
                              const StencilCoef&, hipStream_t);                                                      \
  template void launch_row_apply<T>(const cx<T>*, size_t, size_t, const cx<T>*, size_t, cx<T>*, size_t,              \
                                    const cx<T>* const*, const double*, const PoleState*, const int*, int, double2*, \
                                    const cx<T>*, const Geo&, const StencilCoef&, hipStream_t);                      \
  template void launch_update<T>(const cx<T>*, size_t, cx<T>* const*, const PoleState*, const int*, int, double*,    \
                                 int, const Geo&, hipStream_t);                                                      \
  template void launch_final<T>(const c128*, c128*, const cx<T>*, size_t, size_t, const c128*, size_t,               \
                                const PoleState*, int, c128, c128, double, double, int, const c128*, const Geo&,     \
                                hipStream_t);                                                                        \
  template void launch_accum<T>(c128*, const cx<T>*, size_t, const PoleState*, int, const Geo&, hipStream_t);

HP_INST(double)
HP_INST(float)
