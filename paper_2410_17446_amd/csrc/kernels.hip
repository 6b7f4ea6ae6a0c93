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
//
// R-domain fields are stored column-tiled, [nx/TW][ny][TW] with TW elements =
// 128 bytes, so the row pass reads whole 128-byte lines of each tile and the
// column pass reads each tile as one contiguous block.  Physical fields (the
// caller's E, n^2 and the coefficient planes) are row-major [ny][nx].
#include <math.h>

#include "fft.hpp"
#include "kernels.hpp"

namespace {

template <typename T>
struct Tile {
  static constexpr int W = 128 / (int)sizeof(cx<T>);  // elements per 128-byte tile row
};

// offset of element (row i, column q) of a tiled field with ny rows
template <int TW>
__device__ __forceinline__ size_t tix(int i, int q, int ny) {
  return ((size_t)(q / TW) * ny + i) * TW + (q % TW);
}

// Tiled offsets of the points q = t + s * NT (s = 0, 1, ...) of row i: when NT
// is a multiple of TW they step by a uniform stride (kept in a scalar
// register instead of one address per point).
template <int TW, int NT>
struct RowWalk {
  size_t o0, step;
  int i, t, ny;
  __device__ __forceinline__ RowWalk(size_t base, int i_, int t_, int ny_) : i(i_), t(t_), ny(ny_) {
    o0 = base + tix<TW>(i_, t_, ny_);
    step = (size_t)(NT / TW) * ny_ * TW;
  }
  __device__ __forceinline__ size_t at(int s) const {
    if constexpr (NT % TW == 0)
      return o0 + (size_t)s * step;
    else
      return o0 - tix<TW>(i, t, ny) + tix<TW>(i, t + s * NT, ny);
  }
};

template <int N>
struct RowCfg {
  static constexpr int NT = N / 8;                           // threads per transform
  static constexpr int RPW = (256 / NT) > 0 ? 256 / NT : 1;  // transforms per workgroup
  static constexpr int WG = RPW * NT;
  static constexpr int PT = N / NT;                          // values per thread per row (8)
  static constexpr int SCR = ScanScratch<NT>::SIZE;          // scan scratch per transform
};

// LDS budget of a column workgroup's transform buffers, which sets how many
// columns it transforms at once.  Three budgets are built; the plan uses the
// middle one (two complex128 columns of 1024 per workgroup, four workgroups per
// CU) unless hp_autotune measured another to be faster for its shape.
constexpr int kColLds[3] = {20480, 40960, 81920};

template <typename T, typename C, int N, int LB = 40960>
struct ColCfg {
  static constexpr int TW = Tile<T>::W;
  static constexpr int NT = N / 8;
  static constexpr int PB = plen<C>(N) * (int)sizeof(cx<C>);
  static constexpr int G0 = LB / PB;
  static constexpr int G1 = G0 < 1 ? 1 : (G0 > TW ? TW : G0);
  static constexpr int G2 = (G1 * NT > 1024) ? 1024 / NT : G1;
  // columns transformed at once: a power of two, so that it divides the tile width
  static constexpr int GC = G2 >= 16 ? 16 : G2 >= 8 ? 8 : G2 >= 4 ? 4 : G2 >= 2 ? 2 : 1;
  static_assert(TW % GC == 0, "column groups tile the 128-byte row");
  static constexpr int WG = GC * NT;
  static constexpr int SCR = ScanScratch<NT>::SIZE;
  // LDS stride between the GC column buffers: plen<C>(N) (a multiple of 256
  // bytes) plus 256/GC bytes, so that neighbouring threads, which alternate
  // columns in the load, divide and store loops, hit different banks
  static constexpr int SHIFT = (256 / GC) / (int)sizeof(cx<C>) > 0 ? (256 / GC) / (int)sizeof(cx<C>) : 1;
  static constexpr int PLC = plen<C>(N) + SHIFT;
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

// ------------------------------------------------------------------ row forward (physical -> R-domain)

template <typename T, typename C, int N, int TW>
__global__ __launch_bounds__(RowCfg<N>::WG) void k_row_fwd(const c128* __restrict__ in, cx<T>* __restrict__ out,
                                                           double* __restrict__ part, const cx<C>* __restrict__ tw,
                                                           int ny, size_t fsz, int nblk, const PoleList isel,
                                                           const PoleList osel, size_t in_bs, size_t out_bs,
                                                           size_t part_bs) {
  // batch entry z = blockIdx.z: input isel.k[z], output osel.k[z], partial sums z
  in += (size_t)isel.k[blockIdx.z] * in_bs;
  out += (size_t)osel.k[blockIdx.z] * out_bs;
  part += (size_t)blockIdx.z * part_bs;
  using RC = RowCfg<N>;
  constexpr int NT = RC::NT, RPW = RC::RPW, WG = RC::WG, PT = RC::PT;
  __shared__ cx<C> lds[RPW * plen<C>(N)];
  __shared__ cx<C> scr[RPW * RC::SCR];
  __shared__ double red[(WG + 63) / 64];
  const int g = threadIdx.x / NT, t = threadIdx.x % NT;
  const int row = 1 + blockIdx.x * RPW + g;
  const int comp = blockIdx.y;
  const bool valid = row < ny;
  cx<C>* buf = lds + g * plen<C>(N);
  const c128* src = in + comp * fsz + (size_t)row * N;
  const PStep<C, NT> at(t);  // LDS index of element t + s NT
  double nrm = 0.0;
#pragma unroll
  for (int s = 0; s < PT; ++s) {
    const int m = t + s * NT;
    cx<C> v = czero<C>();
    if (valid && m > 0) {
      const c128 a = src[m];
      nrm += abs2(a);
      v = cvt<C>(a);
    }
    buf[at(s)] = v;
  }
  __syncthreads();
  dst1<C, N>(buf, tw, scr + g * RC::SCR, t);
  const C scale = (C)sqrt(2.0 / N);
  if (valid) {
    cx<T>* dst = out + comp * fsz;
#pragma unroll
    for (int s = 0; s < PT; ++s) {
      const int p = t + s * NT;
      dst[tix<TW>(row, p, ny)] = (p == 0) ? czero<T>() : cvt<T>(scale * buf[at(s)]);
    }
  }
  double sum = block_sum<WG>(nrm, red);
  if (threadIdx.x == 0) part[comp * nblk + blockIdx.x] = sum;
}

// ------------------------------------------------------------------ row inverse (R-domain -> physical complex128)

template <typename T, typename C, int N, int TW>
__global__ __launch_bounds__(RowCfg<N>::WG) void k_row_inv(const cx<T>* __restrict__ in, c128* __restrict__ out,
                                                           const cx<C>* __restrict__ tw, int ny, size_t fsz,
                                                           const PoleList sel, size_t in_bs, size_t out_bs) {
  // batch entry z = blockIdx.z: input entry sel.k[z], output z
  in += (size_t)sel.k[blockIdx.z] * in_bs;
  out += (size_t)blockIdx.z * out_bs;
  using RC = RowCfg<N>;
  constexpr int NT = RC::NT, RPW = RC::RPW, PT = RC::PT;
  __shared__ cx<C> lds[RPW * plen<C>(N)];
  __shared__ cx<C> scr[RPW * RC::SCR];
  const int g = threadIdx.x / NT, t = threadIdx.x % NT;
  const int row = blockIdx.x * RPW + g;  // all rows, row 0 -> zeros
  const int comp = blockIdx.y;
  const bool valid = row < ny && row > 0;
  cx<C>* buf = lds + g * plen<C>(N);
  const cx<T>* src = in + comp * fsz;
  const PStep<C, NT> at(t);  // LDS index of element t + s NT
#pragma unroll
  for (int s = 0; s < PT; ++s) {
    const int m = t + s * NT;
    buf[at(s)] = (valid && m > 0) ? cvt<C>(src[tix<TW>(row, m, ny)]) : czero<C>();
  }
  __syncthreads();
  dst1<C, N>(buf, tw, scr + g * RC::SCR, t);
  const C scale = (C)sqrt(2.0 / N);
  if (row < ny) {
    c128* dst = out + comp * fsz + (size_t)row * N;
#pragma unroll
    for (int s = 0; s < PT; ++s) {
      const int p = t + s * NT;
      dst[p] = (!valid || p == 0) ? mk(0.0, 0.0) : cvt<double>(scale * buf[at(s)]);
    }
  }
}

// ------------------------------------------------------------------ column pass (preconditioner)
//
// One workgroup per group of GC columns of a tile (a tile row is one 128-byte
// line, TW columns).  Workgroups are dealt to the 8 XCDs round-robin; the
// TW/GC sibling groups of a tile get block indices with the same value mod 8,
// consecutive in dispatch order: they run at the
// same time on one XCD, so each line comes from HBM once and from that XCD's
// L2 for the siblings (one workgroup walking the groups in turn lost the
// lines from L2 between groups and read the tile about three times).
__device__ __forceinline__ void col_block(int bid, int ntiles, int S, int& tile, int& sub) {
  if (ntiles % 8 == 0) {
    tile = (bid / (8 * S)) * 8 + bid % 8;
    sub = (bid / 8) % S;
  } else {
    tile = bid / S;
    sub = bid % S;
  }
}

// Waves per SIMD for the column pass (as for the row pass: the most that
// compile without spilling, but for 12 bytes at n = 128).
template <typename C, int N>
struct ColWaves {
  static constexpr bool POW2 = (N & (N - 1)) == 0;
  static constexpr int V = (N <= 1024 && POW2) ? 4 : 2;
};

template <typename T, typename C, int N, int NC, int LB>
__global__ __launch_bounds__((ColCfg<T, C, N, LB>::WG), (ColWaves<C, N>::V)) void k_col(
    const cx<T>* const* __restrict__ uptr, cx<T>* __restrict__ zbase, size_t zsp, size_t zsi,
    cx<T>* __restrict__ dzbase, size_t dzsp, const PoleState* __restrict__ st, const PoleList list,
    int* __restrict__ active_out, const double* __restrict__ mu_x, const double* __restrict__ mu_y,
    const cx<C>* __restrict__ tw, size_t fsz, StencilCoef sc) {
  using CC = ColCfg<T, C, N, LB>;
  constexpr int NT = CC::NT, TW = CC::TW, GC = CC::GC, WG = CC::WG, S = TW / GC;
  constexpr int PL = CC::PLC;  // padded per-column stride
  __shared__ cx<C> lds[GC * PL];
  __shared__ cx<C> scr[GC * CC::SCR];
  int tile, sub;
  col_block(blockIdx.x, gridDim.x / S, S, tile, sub);
  const int col0 = tile * TW;
  const int c0 = sub * GC;
  const int comp = blockIdx.y % NC;
  const int tid = threadIdx.x;
  const int g = tid / NT, t = tid % NT;
  const C scale = (C)sqrt(2.0 / N);
  // workgroup (0, 0) stores the pole list for the round's later kernels
  const bool writer = active_out && blockIdx.x == 0 && blockIdx.y == 0;
  const int k = list.k[blockIdx.y / NC];
  if (st[k].flag) {
    if (writer && tid < list.n) active_out[tid] = list.k[tid];
    return;
  }
  const int m = st[k].m;
  const c128 b = st[k].bk;
  const C sc2 = (C)st[k].sigma[m] * scale;
  const size_t tbase = comp * fsz + (size_t)tile * N * TW;  // this tile, component comp (ny == N)
  const cx<T>* u = uptr[k * (HP_MAXM + 1) + m] + tbase;
  cx<T>* z = zbase + k * zsp + m * zsi + tbase;
  cx<T>* dz = (NC == 2) ? dzbase + k * dzsp + tbase : nullptr;
  // The loops below give consecutive threads the columns of a row in turn,
  // from row 0, so that every 16 threads touch one aligned run of rows:
  // thread tid takes column c = tid % GC, rows r0 + i NT (i = 0..7).
  const int c = tid % GC, r0 = tid / GC, q = col0 + c0 + c;
  const double mq = mu_x[q] - b.re, li = -b.im;
  cx<C>* bc = lds + c * PL;
  const PStep<C, NT> at(r0);
  const cx<C>* sintab = tw + N;
  // divide by mu_y[p] + mu_x[q] - b (one FP64 division)
  auto divide = [&](cx<C> X, int p) {
    const double lr = mu_y[p] + mq, inv = 1.0 / (lr * lr + li * li);
    return (scale * X) * mk<C>((C)(lr * inv), (C)(-li * inv));
  };
  {
    // load fused with the first transform's pre-processing: thread (c, r0) takes the
    // row pairs (j, N - j), j = r0 + i NT < N/2, of its column, and row N/2 when r0 = 0
#pragma unroll 2
    for (int i = 0; i < N / (2 * NT); ++i) {
      const int j = r0 + i * NT;
      if (j == 0) {
        bc[pidx<C>(0)] = czero<C>();
        bc[pidx<C>(N / 2)] = (C)2 * cvt<C>(u[(size_t)(N / 2) * TW + c0 + c]);
        continue;
      }
      cx<C> ya, yb;
      dst1_pair(cvt<C>(u[(size_t)j * TW + c0 + c]), cvt<C>(u[(size_t)(N - j) * TW + c0 + c]), sintab[j].re, ya,
                yb);
      bc[at(i)] = ya;
      bc[pidx<C>(N - j)] = yb;
    }
    __syncthreads();
    dst1_core<C, N>(lds + g * PL, tw, scr + g * CC::SCR, t);
    // the divide fused with the inverse transform's pre-processing, same pairs
#pragma unroll 1
    for (int i = 0; i < N / (2 * NT); ++i) {
      const int j = r0 + i * NT;
      if (j == 0) {
        bc[pidx<C>(0)] = czero<C>();
        bc[pidx<C>(N / 2)] = (C)2 * divide(bc[pidx<C>(N / 2)], N / 2);
        continue;
      }
      cx<C> ya, yb;
      dst1_pair(divide(bc[at(i)], j), divide(bc[pidx<C>(N - j)], N - j), sintab[j].re, ya, yb);
      bc[at(i)] = ya;
      bc[pidx<C>(N - j)] = yb;
    }
    __syncthreads();
    dst1_core<C, N>(lds + g * PL, tw, scr + g * CC::SCR, t);
#pragma unroll 2
    for (int i = 0; i < N / NT; ++i) {
      const int p = r0 + i * NT;
      if (p == 0) continue;
      z[(size_t)p * TW + c0 + c] = cvt<T>(sc2 * bc[at(i)]);
      if constexpr (NC == 2) {
        // D1y of the column, physical in y (odd reflection about rows 0 and N)
        cx<double> acc = mk(0.0, 0.0);
#pragma unroll
        for (int mm = 1; mm <= 6; ++mm)
          acc = acc + sc.d1y[mm - 1] * cvt<double>(odd_at(bc, N, p + mm) - odd_at(bc, N, p - mm));
        dz[(size_t)p * TW + c0 + c] = cvt<T>(sc2 * cvt<C>(acc));
      }
    }
  }
  if (writer && tid < list.n) active_out[tid] = list.k[tid];
}

// ------------------------------------------------------------------ row pass (medium part + inner products)

// Load of one row of an R-domain field fused with the DST-I pre-processing:
// thread t takes the point pairs (j, N - j), j = t + s NT < N/2, and point N/2
// when t = 0; an invalid row loads zeros.
template <typename T, typename C, int N, int NT, int TW>
__device__ __forceinline__ void load_pre_row(cx<C>* buf, const cx<T>* __restrict__ src, const RowWalk<TW, NT>& toff,
                                             size_t rbase, int ny, bool valid, int t, const PStep<C, NT>& at,
                                             const cx<C>* __restrict__ sintab) {
#pragma unroll 2
  for (int s = 0; s < N / (2 * NT); ++s) {
    const int j = t + s * NT;
    if (j == 0) {
      buf[pidx<C>(0)] = czero<C>();
      buf[pidx<C>(N / 2)] = valid ? (C)2 * cvt<C>(src[rbase + tix<TW>(0, N / 2, ny)]) : czero<C>();
      continue;
    }
    cx<C> ya = czero<C>(), yb = czero<C>();
    if (valid) dst1_pair(cvt<C>(src[toff.at(s)]), cvt<C>(src[rbase + tix<TW>(0, N - j, ny)]), sintab[j].re, ya, yb);
    buf[at(s)] = ya;
    buf[pidx<C>(N - j)] = yb;
  }
}

// The same value, which the compiler must take as new: the LDS addresses of a
// transform derive from the thread index alone, and without this the
// compiler keeps those of every transform in a kernel live from the first to
// the last (registers the vector row pass cannot spare).
__device__ __forceinline__ int fresh(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

// D1x at point j of a row held (unscaled) in the transform buffer b: the
// 13-point first-difference stencil, with the odd reflection about points 0
// and N taken only where the caller says the stencil may reach them.
template <typename C, int N, bool INTERIOR>
__device__ __forceinline__ cx<C> row_d1x(const cx<C>* b, int j, const StencilCoef& sc) {
  cx<C> acc = czero<C>();
#pragma unroll
  for (int mm = 1; mm <= 6; ++mm) {
    if constexpr (INTERIOR)
      acc = acc + (C)sc.d1x[mm - 1] * (b[pidx<C>(j + mm)] - b[pidx<C>(j - mm)]);
    else
      acc = acc + (C)sc.d1x[mm - 1] * (odd_at(b, N, j + mm) - odd_at(b, N, j - mm));
  }
  return acc;
}

template <int N, int NC>
struct ApplyCfg {
  static constexpr int NT = N / 8;
  static constexpr int G0 = (256 / NT) / NC * NC;
  static constexpr int GROUPS = G0 < NC ? NC : G0;  // transforms per workgroup (NC per row)
  static constexpr int ROWS = GROUPS / NC;
  static constexpr int WG = GROUPS * NT;
  static constexpr int WAVES = (WG + 63) / 64;
  static constexpr int SCR = ScanScratch<NT>::SIZE;
  static_assert(NT >= 8, "the stencil's interior points assume at least 8 threads per row");
};

// Waves per SIMD the register allocation must allow: scalar fields four (128
// VGPRs; 12 bytes spill at n = 128) for 2^k up to 1024, else three (complex128
// at 2048: two); vector fields four, which lets two 512-thread workgroups share
// a CU at 2048 (their LDS, one buffer per component, fits twice).
template <typename C, int N, int NC>
struct ApplyWaves {
  static constexpr bool POW2 = (N & (N - 1)) == 0;
  static constexpr int V = NC == 2 ? 4
                                   : ((N <= 1024 && POW2) ? 4 : (sizeof(C) == 4 || N < 2048 ? 3 : 2));
};

template <typename T, typename C, int N, int NC>
__global__ __launch_bounds__((ApplyCfg<N, NC>::WG), (ApplyWaves<C, N, NC>::V)) void k_row_apply(
    const cx<T>* __restrict__ zbase, size_t zsp, size_t zsi, const cx<T>* __restrict__ dzbase, size_t dzsp,
    cx<T>* __restrict__ pbase, size_t psp, const cx<T>* const* __restrict__ uptr, const C* __restrict__ coef,
    const PoleState* __restrict__ st, const int* __restrict__ active, int nactive, int nrb, double2* __restrict__ part,
    int nparts, const cx<C>* __restrict__ tw, int ny, size_t fsz, StencilCoef sc) {
  using AC = ApplyCfg<N, NC>;
  constexpr int NT = AC::NT, GROUPS = AC::GROUPS, ROWS = AC::ROWS, TW = Tile<T>::W;
  constexpr int PT = N / NT;  // values per thread per row
  constexpr int PL = plen<C>(N);
  __shared__ cx<C> lds[GROUPS * PL];
  __shared__ cx<C> scr[GROUPS * AC::SCR];
  const int g = threadIdx.x / NT, t = threadIdx.x % NT;
  const int comp = g % NC;
  // XCD-aware order (workgroups go round-robin to the eight XCDs): the
  // workgroups of one XCD take its row blocks in turn with every pole's
  // workgroup for a block next to the others, so the block's medium
  // coefficients (and, in a first cycle, the shared basis vector) come from
  // that XCD's L2 for all but the first pole
  const int xcd = blockIdx.x % 8, q = blockIdx.x / 8;
  const int rb = (q / nactive) * 8 + xcd;
  if (rb >= nrb) return;
  const int row = 1 + rb * ROWS + g / NC;
  const bool valid = row < ny;
  const int k = active[q % nactive];
  if (st[k].flag) return;
  const int m = st[k].m;
  cx<C>* buf = lds + g * PL;
  cx<C>* sg = scr + g * AC::SCR;
  const C scale = (C)sqrt(2.0 / N);
  const size_t cbase = comp * fsz;
  const size_t ci0 = (size_t)row * N;  // physical row offset
  const RowWalk<TW, NT> toff(cbase, valid ? row : 0, t, ny);  // tiled offsets of the thread's points
  const PStep<C, NT> at(t);                                    // LDS index of point t + s NT

  const cx<T>* z = zbase + k * zsp + m * zsi;
  cx<C> pz[PT];  // P z at the thread's points j = t + s * NT (vector fields)
  if constexpr (NC == 1) {
    // load fused with the inverse transform's pre-processing: thread t takes the point
    // pairs (j, N - j), j = t + s NT < N/2, of its row, and point N/2 when t = 0
    const cx<C>* sintab = tw + N;
    const size_t rbase = cbase + tix<TW>(valid ? row : 0, 0, ny);
#pragma unroll 2
    for (int s = 0; s < PT / 2; ++s) {
      const int j = t + s * NT;
      if (j == 0) {
        buf[pidx<C>(0)] = czero<C>();
        buf[pidx<C>(N / 2)] = valid ? (C)2 * cvt<C>(z[rbase + tix<TW>(0, N / 2, ny)]) : czero<C>();
        continue;
      }
      cx<C> ya = czero<C>(), yb = czero<C>();
      if (valid) dst1_pair(cvt<C>(z[toff.at(s)]), cvt<C>(z[rbase + tix<TW>(0, N - j, ny)]), sintab[j].re, ya, yb);
      buf[at(s)] = ya;
      buf[pidx<C>(N - j)] = yb;
    }
    __syncthreads();
    // the inverse transform's outputs leave multiplied by the medium: P z = V z
    dst1_core_op<C, N>(buf, tw, sg, t, [&](int p, cx<C> X) {
      return (valid ? coef[ci0 + p] : (C)0) * (scale * X);
    });
  } else {
    // eq. Z_bar_eq, medium part (coefficient planes carry s = 1/(k0 n0)^2):
    //   (P w)_1 = psi_xx w1 + psi_x D1x w1 + psi_xy w2 + psi_y D1x w2 + V w1
    //   (P w)_2 = psi_xy w1 + psi_x D1y w1 + psi_yy w2 + psi_y D1y w2 + V w2
    // A workgroup holds one transform buffer per component (two workgroups fit
    // a CU) and no partial product stays in registers across a transform: the
    // D1y rows (the column pass's second output) are transformed first, and
    // the D1y part of (P w)_2 waits in the component's own output row of p (in
    // the storage precision), which the final store overwrites.  Each group
    // reads its partner's buffer directly, and each takes one x-derivative
    // stencil.  Both loads are fused with their transforms' pre-processing, as
    // for scalar fields.
    const size_t rbase = cbase + tix<TW>(valid ? row : 0, 0, ny);
    const cx<C>* ob = lds + (g ^ 1) * PL;
    cx<T>* pk = pbase + k * psp;
    load_pre_row<T, C, N, NT, TW>(buf, dzbase + k * dzsp, toff, rbase, ny, valid, t, at, tw + N);
    __syncthreads();
    dst1_core<C, N>(buf, tw, sg, fresh(t));
    if (comp == 1 && valid) {
#pragma unroll
      for (int s = 0; s < PT; ++s) {
        const int j = t + s * NT;
        if (j == 0) continue;
        const size_t ci = ci0 + j;
        pk[toff.at(s)] = cvt<T>(coef[2 * fsz + ci] * (scale * buf[at(s)]) + coef[fsz + ci] * (scale * ob[at(s)]));
      }
    }
    __syncthreads();
    load_pre_row<T, C, N, NT, TW>(buf, z, toff, rbase, ny, valid, t, at, tw + N);
    __syncthreads();
    dst1_core<C, N>(buf, tw, sg, fresh(t));
    // component 1 takes psi_y D1x w2 of component 0's product from its own
    // buffer and leaves it (storage precision) in component 0's output row of
    // p, where component 0 picks it up after the barrier
    cx<T>* pk0 = pk - cbase;  // component 0's rows of p
    if (comp == 1 && valid) {
#pragma unroll
      for (int s = 0; s < PT; ++s) {
        const int j = t + s * NT;
        if (j == 0) continue;
        // the thread's middle points never reach the reflections at 0 and N
        const bool inner = s > 0 && s < PT - 1;
        const cx<C> dx = inner ? row_d1x<C, N, true>(buf, j, sc) : row_d1x<C, N, false>(buf, j, sc);
        pk0[toff.at(s)] = cvt<T>(coef[2 * fsz + ci0 + j] * (scale * dx));
        // one point at a time: hoisting every point's loads would spill
        __builtin_amdgcn_sched_barrier(0);
      }
    }
#pragma unroll
    for (int s = 0; s < PT; ++s) {
      const int j = t + s * NT;
      pz[s] = czero<C>();
      if (!valid || j == 0) continue;
      const size_t ci = ci0 + j;
      const cx<C> zc = scale * buf[at(s)], zo = scale * ob[at(s)];
      const C v = coef[ci], pxy = coef[5 * fsz + ci];
      if (comp == 0) {
        const bool inner = s > 0 && s < PT - 1;
        const cx<C> dx = inner ? row_d1x<C, N, true>(buf, j, sc) : row_d1x<C, N, false>(buf, j, sc);
        pz[s] = (coef[3 * fsz + ci] + v) * zc + coef[fsz + ci] * (scale * dx) + pxy * zo;
      } else {
        pz[s] = (coef[4 * fsz + ci] + v) * zc + pxy * zo + cvt<C>(pk[toff.at(s)]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
    if (comp == 0 && valid) {
#pragma unroll
      for (int s = 0; s < PT; ++s)
        if (t + s * NT > 0) pz[s] = pz[s] + cvt<C>(pk0[toff.at(s)]);
    }
  }
  // forward transform of P z (already in buf for scalar fields)
  if constexpr (NC == 2) {
#pragma unroll
    for (int s = 0; s < PT; ++s) {
      const int j = t + s * NT;
      buf[at(s)] = (j == 0) ? czero<C>() : pz[s];
    }
    __syncthreads();
  }
  dst1<C, N>(buf, tw, sg, NC == 1 ? t : fresh(t));
  // p as stored: the inner products use exactly what the update reads (vector
  // fields re-read it from LDS in each product, to keep fewer values live)
  auto pval = [&](int s) {
    const int j = t + s * NT;
    return (j == 0 || !valid) ? czero<T>() : cvt<T>(scale * buf[at(s)]);
  };
  cx<T> pv[NC == 1 ? PT : 1];
  cx<T>* p = pbase + k * psp;
#pragma unroll
  for (int s = 0; s < PT; ++s) {
    const cx<T> ps = pval(s);
    if constexpr (NC == 1) pv[s] = ps;
    if (valid) p[toff.at(s)] = ps;
  }
  // <u_i, p> and <u_i, u_m>, i = 0..m: the new direction's projections and
  // the reorthogonalisation of the provisional u_m, from the same reads of the
  // basis.  Partial sums per wave (no workgroup barrier).
  cx<T> um[PT];
  {
    const cx<T>* u = uptr[k * (HP_MAXM + 1) + m];
#pragma unroll
    for (int s = 0; s < PT; ++s) um[s] = valid ? u[toff.at(s)] : czero<T>();
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int slot = rb * AC::WAVES + wave;
  for (int i = 0; i <= m; ++i) {
    const cx<T>* u = uptr[k * (HP_MAXM + 1) + i];
    double pr = 0.0, pi = 0.0, qr = 0.0, qi = 0.0;
    if (valid) {
#pragma unroll
      for (int s = 0; s < PT; ++s) {
        const cx<double> a = cvt<double>(i == m ? um[s] : u[toff.at(s)]);
        const cx<double> bp = cvt<double>(NC == 1 ? pv[s] : pval(s));
        const cx<double> bq = cvt<double>(um[s]);
        pr += a.re * bp.re + a.im * bp.im;
        pi += a.re * bp.im - a.im * bp.re;
        qr += a.re * bq.re + a.im * bq.im;
        qi += a.re * bq.im - a.im * bq.re;
      }
    }
    pr = wave_sum(pr);
    pi = wave_sum(pi);
    qr = wave_sum(qr);
    qi = wave_sum(qi);
    if (lane == 0) {
      const size_t base = (((size_t)k * (HP_MAXM + 1) + i) * 2) * nparts + slot;
      part[base] = make_double2(pr, pi);
      part[base + nparts] = make_double2(qr, qi);
    }
  }
}

// ------------------------------------------------------------------ Gram-Schmidt update

constexpr int UPD_WG = 256;
constexpr int UPD_E = 4;

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
  if (st[k].flag) return;
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
  // UPD_E elements per thread, UPD_WG apart, so that each basis vector's
  // loads are in flight together
  const size_t chunk = (size_t)UPD_WG * UPD_E;
  for (size_t base = (size_t)blockIdx.x * chunk + threadIdx.x; base < total; base += (size_t)gridDim.x * chunk) {
    cx<double> v[UPD_E], c[UPD_E];
#pragma unroll
    for (int e = 0; e < UPD_E; ++e) {
      const size_t idx = base + (size_t)e * UPD_WG;
      v[e] = (idx < total) ? cf[m + 1] * cvt<double>(p[idx]) : mk(0.0, 0.0);
      c[e] = mk(0.0, 0.0);
    }
    for (int i = 0; i <= m; ++i) {
      const cx<T>* ui = up[i];
      cx<double> a[UPD_E];
#pragma unroll
      for (int e = 0; e < UPD_E; ++e) {
        const size_t idx = base + (size_t)e * UPD_WG;
        a[e] = (idx < total) ? cvt<double>(ui[idx]) : mk(0.0, 0.0);
      }
      const c128 fi = cf[i], gi = cv[i];
#pragma unroll
      for (int e = 0; e < UPD_E; ++e) {
        v[e] = v[e] + fi * a[e];
        c[e] = c[e] + gi * a[e];
      }
    }
#pragma unroll
    for (int e = 0; e < UPD_E; ++e) {
      const size_t idx = base + (size_t)e * UPD_WG;
      if (idx >= total) continue;
      const cx<T> r = cvt<T>(v[e]);
      out[idx] = r;
      if (corr) um[idx] = cvt<T>(c[e]);
      nrm += abs2(cvt<double>(r));
    }
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
// <u_i, p> and <u_i, u_m>: one block per (i, slot) pair sums the row pass's
// partials in a fixed order.
// The correction algebra of pole k's step from its reduced inner products
// (run by the last reduction workgroup of the pole, 256 threads).
__device__ __forceinline__ void prep_pole(PoleState* __restrict__ st, int k) {
  __shared__ c128 P[HP_MAXM + 1], Q[HP_MAXM + 1];
  __shared__ c128 sv[HP_MAXM], cc[HP_MAXM + 1], h[HP_MAXM + 1];
  const int m = st[k].m;
  for (int i = threadIdx.x; i <= m; i += 256) {
    P[i] = st[k].Pd[i];
    Q[i] = st[k].Qd[i];
  }
  __syncthreads();
  PoleState& S = st[k];
  constexpr int LD = HP_MAXM + 1;
  c128* Hr = S.Hraw;
  __shared__ double sh[4];  // rho, gamma (re, im), h~
  __shared__ double sig[HP_MAXM + 1];
  const int tid = threadIdx.x;
  const double sm = S.sigma[m];
  for (int i = tid; i <= m; i += 256) sig[i] = S.sigma[i];
  __syncthreads();
  for (int i = tid; i < m; i += 256) {
    sv[i] = (sig[i] * sm) * Q[i];
    cc[i] = sig[i] * P[i];
  }
  __syncthreads();
  if (tid == 0) {
    double ssum = 0.0;
    for (int i = 0; i < m; ++i) ssum += abs2(sv[i]);
    double rho2 = sm * sm * Q[m].re - ssum;
    if (!(rho2 > 1e-300)) rho2 = 1e-300;
    const double rho = sqrt(rho2);
    c128 cm = sm * P[m];
    for (int i = 0; i < m; ++i) cm = cm - cmulc(sv[i], cc[i]);
    cc[m] = (1.0 / rho) * cm;
    sh[0] = rho;
    sh[3] = (m > 0) ? Hr[m + (m - 1) * LD].re : 0.0;
    S.Rc[m + m * LD] = mk(rho, 0.0);
    if (m == 0) S.g[0] = rho * S.g[0];
  }
  __syncthreads();
  const double rho = sh[0], irho = 1.0 / rho;
  // Rc column m; correction of Hessenberg column m-1
  for (int i = tid; i < m; i += 256) {
    S.Rc[i + m * LD] = sv[i];
    Hr[i + (m - 1) * LD] = Hr[i + (m - 1) * LD] + sh[3] * sv[i];
  }
  __syncthreads();
  if (tid == 0 && m > 0) Hr[m + (m - 1) * LD] = mk(sh[3] * rho, 0.0);
  __syncthreads();
  // column m: h_l = (<v_l, ~v_m> + <v_l, p> - A_l) / rho, A_l = sum_{i<m, i>=l-1} s_i H[l][i]
  for (int l = tid; l <= m; l += 256) {
    c128 A = mk(0.0, 0.0);
    for (int i = (l > 0 ? l - 1 : 0); i < m; ++i) A = A + sv[i] * Hr[l + i * LD];
    const c128 base = (l < m) ? sv[l] + cc[l] : mk(rho, 0.0) + cc[m];
    h[l] = irho * (base - A);
    Hr[l + m * LD] = h[l];
    P[l] = irho * A + h[l];  // A_l / rho + h_l (P no longer needed)
  }
  __syncthreads();
  const c128 gam = P[m];
  // u_{m+1} = (1/rho) p + (1 - gam)/rho ~v_m + sum_{l<m} (gam s_l / rho - A_l / rho - h_l) v_l
  for (int l = tid; l < m; l += 256) {
    S.cu[l] = sig[l] * (irho * (gam * sv[l]) - P[l]);
    S.cv[l] = (-sig[l] * irho) * sv[l];
  }
  if (tid == 0) {
    S.cu[m] = (sm * irho) * (mk(1.0, 0.0) - gam);
    S.cu[m + 1] = mk(irho, 0.0);
    if (m == 0) {
      // v_0 = ~v_0 / rho rescales the (possibly shared) stored vector
      S.sigma[0] = sm * irho;
      S.correct = 0;
    } else {
      S.cv[m] = mk(sm * irho, 0.0);
      S.sigma[m] = 1.0;
      S.correct = 1;
    }
  }
}

__global__ __launch_bounds__(256) void k_reduce_pairs(const double2* __restrict__ part, int nparts,
                                                      PoleState* __restrict__ st, const int* __restrict__ active,
                                                      int* __restrict__ done) {
  __shared__ double red[4];
  __shared__ int last;
  const int k = active[blockIdx.y];
  if (st[k].flag) return;
  const int m = st[k].m;
  const int i = blockIdx.x >> 1, slot = blockIdx.x & 1;
  if (i > m) return;
  const double2* src = part + (((size_t)k * (HP_MAXM + 1) + i) * 2 + slot) * nparts;
  double re = 0.0, im = 0.0;
  {
    double ar[4] = {0, 0, 0, 0}, ai[4] = {0, 0, 0, 0};
    int b = threadIdx.x;
    for (; b + 3 * 256 < nparts; b += 4 * 256) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double2 v = src[b + u * 256];
        ar[u] += v.x;
        ai[u] += v.y;
      }
    }
    for (; b < nparts; b += 256) {
      ar[0] += src[b].x;
      ai[0] += src[b].y;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      re += ar[u];
      im += ai[u];
    }
  }
  re = block_sum<256>(re, red);
  im = block_sum<256>(im, red);
  // the last of the pole's 2 (m + 1) workgroups (counted in done[k], which it
  // clears again) continues with the correction algebra
  if (threadIdx.x == 0) {
    (slot ? st[k].Qd : st[k].Pd)[i] = mk(re, im);
    __threadfence();
    last = atomicAdd(&done[k], 1) == 2 * (m + 1) - 1;
  }
  __syncthreads();
  if (!last) return;
  if (threadIdx.x == 0) done[k] = 0;
  __threadfence();
  prep_pole(st, k);
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

// Upper triangle of an n x n matrix packed by columns: (r, c), r <= c.
__device__ __forceinline__ int pk(int r, int c) { return c * (c + 1) / 2 + r; }

// Back substitution R x = rhs (R packed upper triangular, n <= 64) by the one
// wave of the block: lane l keeps rhs[l] in a register, x[i] is broadcast by a
// shuffle; x is written to LDS.  rhs is not modified.
__device__ void upper_solve(const c128* __restrict__ R, const c128* rhs, c128* x, int n) {
  const int l = threadIdx.x;
  c128 r = (l < n) ? rhs[l] : mk(0.0, 0.0);
  for (int i = n - 1; i >= 0; --i) {
    c128 xi = mk(0.0, 0.0);
    if (l == i) {
      const c128 d = R[pk(i, i)];
      xi = (abs2(d) > 0.0) ? cdiv(r, d) : mk(0.0, 0.0);
      x[i] = xi;
    }
    xi.re = __shfl(xi.re, i, 64);
    xi.im = __shfl(xi.im, i, 64);
    if (l < i) r = r - R[pk(l, i)] * xi;
  }
  __syncthreads();
}

__global__ __launch_bounds__(64) void k_arnoldi(PoleState* __restrict__ st, const int* __restrict__ active,
                                                const double* __restrict__ part, int nblk, int restart,
                                                unsigned long long* __restrict__ ftag, unsigned long long seq,
                                                double* __restrict__ ests) {
  __shared__ c128 c1[HP_MAXM + 2], c2[HP_MAXM + 2], sn[HP_MAXM], rhs[HP_MAXM + 1], y[HP_MAXM];
  __shared__ double cs[HP_MAXM];
  __shared__ int flag_s;
  const int k = active[blockIdx.x];
  if (st[k].flag) return;
  const int tid = threadIdx.x;
  PoleState& S = st[k];
  constexpr int LD = HP_MAXM + 1;
  const int m = S.m;
  // scalars thread 0 needs, loaded up front so their latency overlaps the reduction
  const c128 gpre_m1 = (tid == 0 && m >= 1) ? S.gpre[m - 1] : mk(0.0, 0.0);
  const c128 g_m = (tid == 0) ? S.g[m] : mk(0.0, 0.0);
  const int fixed = S.fixed, total = S.total;
  const double tol = S.tol;
  double s = 0.0;
  {
    // eight independent accumulators keep eight loads in flight per thread
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const double* src = part + (size_t)k * nblk;
    int b = tid;
    for (; b + 7 * 64 < nblk; b += 8 * 64) {
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] += src[b + u * 64];
    }
    for (; b < nblk; b += 64) acc[0] += src[b];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += acc[u];
  }
  s = wave_sum(s);
  for (int i = tid; i <= m; i += 64) {
    c2[i] = S.Hraw[i + m * LD];
    if (m >= 1) c1[i] = S.Hraw[i + (m - 1) * LD];
  }
  for (int i = tid; i < m; i += 64) {
    cs[i] = S.cs[i];
    sn[i] = S.sn[i];
  }
  __syncthreads();
  if (tid == 0) {
    c128 gm_rot = mk(0.0, 0.0);
    const double h = sqrt(s);
    S.Hraw[m + 1 + m * LD] = mk(h, 0.0);
    c2[m + 1] = mk(h, 0.0);
    if (m >= 1) {
      // column m-1 was corrected by the reorthogonalisation: redo its rotation
      for (int i = 0; i < m - 1; ++i) {
        const c128 a = c1[i], b = c1[i + 1];
        c1[i] = cs[i] * a + sn[i] * b;
        c1[i + 1] = -1.0 * cmulc(sn[i], a) + cs[i] * b;
      }
      double c;
      c128 snn, r;
      givens(c1[m - 1], c1[m].re, c, snn, r);
      cs[m - 1] = c;
      sn[m - 1] = snn;
      c1[m - 1] = r;
      c1[m] = mk(0.0, 0.0);
      S.g[m - 1] = c * gpre_m1;
      gm_rot = -1.0 * cmulc(snn, gpre_m1);
      S.g[m] = gm_rot;
    }
    for (int i = 0; i < m; ++i) {
      const c128 a = c2[i], b = c2[i + 1];
      c2[i] = cs[i] * a + sn[i] * b;
      c2[i + 1] = -1.0 * cmulc(sn[i], a) + cs[i] * b;
    }
    double c;
    c128 snn, r;
    givens(c2[m], h, c, snn, r);
    cs[m] = c;
    sn[m] = snn;
    c2[m] = r;
    c2[m + 1] = mk(0.0, 0.0);
    const c128 gm = (m >= 1) ? gm_rot : g_m;  // g[m] as it stands after column m-1
    const c128 gnext = -1.0 * cmulc(snn, gm);
    const double est = sqrt(abs2(gnext));
    S.gpre[m] = gm;
    S.g[m + 1] = gnext;
    S.g[m] = c * gm;
    S.sigma[m + 1] = (h > 0.0) ? 1.0 / h : 0.0;
    S.est = est;
    S.m = m + 1;
    S.total = total + 1;
    int flag = 0;
    if (!isfinite(h) || !isfinite(est)) {
      flag = 4;  // a NaN or Inf reached the Krylov space (n^2 or the right-hand side): stop the pole
    } else if (fixed > 0) {
      if (m + 1 >= fixed) flag = 1;
    } else if (est <= tol || h == 0.0) {
      flag = 1;
    } else if (m + 1 >= restart) {
      flag = 2;
    }
    flag_s = flag;
  }
  __syncthreads();
  for (int i = tid; i <= m + 1; i += 64) {
    S.H[i + m * LD] = c2[i];
    if (m >= 1 && i <= m) S.H[i + (m - 1) * LD] = c1[i];
  }
  if (tid == 0 && m >= 1) {
    S.cs[m - 1] = cs[m - 1];
    S.sn[m - 1] = sn[m - 1];
  }
  if (tid == 0) {
    S.cs[m] = cs[m];
    S.sn[m] = sn[m];
  }
  int flag = flag_s;
  if (flag && flag != 4) {
    // least squares R y = g, then y~ = Rc^{-1} y (the coefficients of the stored Z~);
    // both triangles go through LDS, packed (one parallel load each)
    __shared__ c128 tri[HP_MAXM * (HP_MAXM + 1) / 2];
    const int n = m + 1, npk = n * (n + 1) / 2;
    // packed index e = c (c + 1)/2 + r: every thread loads entries of its own, all at once
    auto unpack = [](int e, int& r, int& c) {
      c = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
      if ((c + 1) * (c + 2) / 2 <= e) ++c;
      if (c * (c + 1) / 2 > e) --c;
      r = e - c * (c + 1) / 2;
    };
    for (int e = tid; e < npk; e += 64) {
      int r, c;
      unpack(e, r, c);
      tri[e] = (c == m) ? c2[r] : (c == m - 1 ? c1[r] : S.H[r + c * LD]);
    }
    for (int i = tid; i < n; i += 64) rhs[i] = S.g[i];
    __syncthreads();
    upper_solve(tri, rhs, y, n);
    for (int e = tid; e < npk; e += 64) {
      int r, c;
      unpack(e, r, c);
      tri[e] = S.Rc[r + c * LD];
    }
    for (int i = tid; i < n; i += 64) rhs[i] = y[i];  // the least-squares solution
    __syncthreads();
    upper_solve(tri, rhs, y, n);
    for (int i = tid; i < n; i += 64) S.y[i] = y[i];
    // The estimate measures the split operator I + P M~^-1; it differs from
    // A M~^-1 by about eps kappa(M_k) ||y|| (y the least-squares solution, so
    // ||y|| = ||M x||).  When that is not well below tol, the true residual decides.
    if (tid == 0 && flag == 1 && fixed == 0) {
      double yn = 0.0;
      for (int i = 0; i < n; ++i) yn += abs2(rhs[i]);
      if (S.incons * sqrt(yn) > 0.1 * S.tol) flag = 3;
    }
  }
  if (tid == 0) {
    S.flag = flag;
    ests[k] = S.est;
    // the round's tag and the flag in one 8-byte system-scope store to host
    // memory, which the host polls (no event per round); the host reads
    // nothing else of this round before a synchronisation, so no release
    __hip_atomic_store(&ftag[k], (seq << 8) | (unsigned long long)flag, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

__global__ __launch_bounds__(64) void k_cycle_init(PoleState* __restrict__ st, const int* __restrict__ poles,
                                                   const double* __restrict__ part, int nblk, int first, double tol,
                                                   double rtol_cycle, size_t part_bs, int set_has_x) {
  const int k = poles[blockIdx.x];
  part += (size_t)blockIdx.x * part_bs;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64) s += part[b];
  s = wave_sum(s);
  if (threadIdx.x != 0) return;
  PoleState& S = st[k];
  const double beta = sqrt(s);
  if (first) {  // 1: a step's first solve; 2: a later solve of the same step (the count runs on)
    S.beta0 = beta;
    if (first == 1) S.total = 0;
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
  if (set_has_x) S.has_x = 1;
}

// ------------------------------------------------------------------ residue-weighted sum and output

template <typename T, int N>
__global__ __launch_bounds__(RowCfg<N>::WG) void k_final(const c128* __restrict__ w, c128* __restrict__ out,
                                                         const cx<T>* __restrict__ zbase, size_t zsp, size_t zsi,
                                                         const c128* __restrict__ xacc, size_t xsp,
                                                         const PoleState* __restrict__ st, int npoles, c128 phase,
                                                         c128 rinf_phase, double loss_coef, double eta, int W,
                                                         const c128* __restrict__ tw, int nx, int ny, size_t fsz) {
  using RC = RowCfg<N>;
  constexpr int NT = RC::NT, RPW = RC::RPW, PT = RC::PT, TW = Tile<T>::W;
  __shared__ c128 lds[RPW * plen<double>(N)];
  __shared__ c128 scr[RPW * RC::SCR];
  const int g = threadIdx.x / NT, t = threadIdx.x % NT;
  const int row = blockIdx.x * RPW + g;  // rows 0..ny-1
  const int comp = blockIdx.y;
  const bool valid = row > 0 && row < ny;
  c128* buf = lds + g * plen<double>(N);
  const size_t roff = comp * fsz + (size_t)row * N;
  const RowWalk<TW, NT> toff(comp * fsz, valid ? row : 0, t, ny);
  c128 acc[PT];
#pragma unroll
  for (int s = 0; s < PT; ++s) acc[s] = mk(0.0, 0.0);
  if (valid) {
    for (int k = 0; k < npoles; ++k) {
      const c128 ak = st[k].ak;
      if (st[k].has_x) {
        const c128* xk = xacc + k * xsp;
#pragma unroll
        for (int s = 0; s < PT; ++s) acc[s] = acc[s] + ak * xk[toff.at(s)];
      }
      const int mk_ = st[k].m;
      const cx<T>* zk = zbase + k * zsp;
      for (int i = 0; i < mk_; ++i) {
        const c128 cf = ak * st[k].y[i];
        const cx<T>* zi = zk + i * zsi;
#pragma unroll
        for (int s = 0; s < PT; ++s) acc[s] = acc[s] + cf * cvt<double>(zi[toff.at(s)]);
      }
    }
  }
  const PStep<double, NT> at(t);  // LDS index of element t + s NT
#pragma unroll
  for (int s = 0; s < PT; ++s) buf[at(s)] = acc[s];
  __syncthreads();
  dst1<double, N>(buf, tw, scr + g * RC::SCR, t);
  const double scale = sqrt(2.0 / N);
  if (row < ny) {
#pragma unroll
    for (int s = 0; s < PT; ++s) {
      const int j = t + s * NT;
      c128 v = mk(0.0, 0.0);
      if (valid && j > 0) {
        const c128 sv = scale * buf[at(s)];
        v = edge_loss(row, j, nx, ny, W, eta, loss_coef) * (phase * sv + rinf_phase * w[roff + j]);
      }
      out[roff + j] = v;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_accum(c128* __restrict__ xacc, const cx<T>* __restrict__ z, size_t zsi,
                                               const PoleState* __restrict__ st, const PoleList sel, size_t xsp,
                                               size_t zsp, size_t total) {
  // one pole per blockIdx.y: X_k += its cycle's terms
  const int pole = sel.k[blockIdx.y];
  xacc += (size_t)pole * xsp;
  z += (size_t)pole * zsp;
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
constexpr int OP_TX = 64, OP_TY = 16, OP_H = 6;  // output tile, stencil half-width
constexpr int OP_LX = OP_TX + 2 * OP_H, OP_LY = OP_TY + 2 * OP_H;

// The explicit FP64 operator on LDS tiles: each workgroup stages a 64 x 16
// tile of every component with a 6-node halo (odd reflection about the
// Dirichlet nodes applied while staging), then each thread evaluates four
// pixels of a column of the tile.
template <int NC>
__global__ __launch_bounds__(OP_WG) void k_apply_op(const c128* __restrict__ x, const c128* __restrict__ rhs,
                                                    c128* __restrict__ y, const double* __restrict__ coef,
                                                    const ShiftList sh, StencilCoef sc, int nx, int ny, size_t fsz,
                                                    double* __restrict__ part, int medium_only, size_t xbs,
                                                    size_t ybs, size_t pbs) {
  // batch entry z = blockIdx.z: field z, shift sh.b[z]
  const c128 b = sh.b[blockIdx.z];
  x += (size_t)blockIdx.z * xbs;
  y += (size_t)blockIdx.z * ybs;
  if (part) part += (size_t)blockIdx.z * pbs;
  __shared__ c128 tile[NC][OP_LY * OP_LX];
  __shared__ double red[OP_WG / 64];
  const int ntx = (nx + OP_TX - 1) / OP_TX;
  const int x0 = (blockIdx.x % ntx) * OP_TX, y0 = (blockIdx.x / ntx) * OP_TY;
  for (int c = 0; c < NC; ++c)
    for (int e = threadIdx.x; e < OP_LY * OP_LX; e += OP_WG)
      tile[c][e] = ld_odd(x + c * fsz, y0 + e / OP_LX - OP_H, x0 + e % OP_LX - OP_H, nx, ny);
  __syncthreads();
  double nrm = 0.0;
  const int tx = threadIdx.x % OP_TX, tq = threadIdx.x / OP_TX;
#pragma unroll
  for (int q = 0; q < OP_TY / (OP_WG / OP_TX); ++q) {
    const int ty = tq + q * (OP_WG / OP_TX);
    const int i = y0 + ty, j = x0 + tx;
    if (i >= ny || j >= nx) continue;
    const size_t idx = (size_t)i * nx + j;
    const bool inner = i > 0 && j > 0;
    const int lc = (ty + OP_H) * OP_LX + tx + OP_H;
    c128 lap[NC], d1x[NC], d1y[NC], xc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const c128* t = tile[c];
      const c128 x0c = t[lc];
      c128 l = (sc.c2x[0] + sc.c2y[0]) * x0c, ax = mk(0.0, 0.0), ay = mk(0.0, 0.0);
#pragma unroll
      for (int mm = 1; mm <= 6; ++mm) {
        const c128 xp = t[lc + mm], xm = t[lc - mm], yp = t[lc + mm * OP_LX], ym = t[lc - mm * OP_LX];
        l = l + sc.c2x[mm] * (xp + xm) + sc.c2y[mm] * (yp + ym);
        ax = ax + sc.d1x[mm - 1] * (xp - xm);
        ay = ay + sc.d1y[mm - 1] * (yp - ym);
      }
      lap[c] = l;
      d1x[c] = ax;
      d1y[c] = ay;
      xc[c] = x0c;
    }
    const double V = coef[idx];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      c128 v = medium_only ? V * xc[c] : lap[c] + V * xc[c] - b * xc[c];
      if constexpr (NC == 2) {
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

// After X_k has absorbed the cycle's Z terms: X_k is the whole solution.
__global__ void k_mark_folded(PoleState* __restrict__ st, int first, int count) {
  const int k = first + (int)threadIdx.x;
  if ((int)threadIdx.x < count) {
    st[k].has_x = 1;
    st[k].m = 0;
  }
}

__global__ void k_mark_list(PoleState* __restrict__ st, const PoleList sel) {
  if ((int)threadIdx.x < sel.n) {
    st[sel.k[threadIdx.x]].has_x = 1;
    st[sel.k[threadIdx.x]].m = 0;
  }
}


// One stage of the classical fourth-order Runge-Kutta combination, over the
// fields in physical layout [ncomp][ny][nx]: acc_out = acc_in + ca L and, when
// v_out is given, v_out = u + cv L.  With loss_coef > 0, acc_out is multiplied
// by the edge layer's loss factor.  Row 0 and column 0 are written as zero.
// acc_in may alias acc_out (each element is read before it is written).
__global__ __launch_bounds__(256) void k_rk4_stage(const c128* __restrict__ L, const c128* acc_in, c128* acc_out,
                                                   const c128* __restrict__ u, c128* __restrict__ v_out, double ca,
                                                   double cv, double loss_coef, double eta, int W, int nx, int ny,
                                                   unsigned fsz, unsigned total) {
  for (unsigned idx = blockIdx.x * 256u + threadIdx.x; idx < total; idx += gridDim.x * 256u) {
    const unsigned e = idx % fsz;
    const int i = (int)(e / (unsigned)nx), j = (int)(e % (unsigned)nx);
    const bool inside = i > 0 && j > 0;
    c128 a = mk(0.0, 0.0), v = mk(0.0, 0.0);
    if (inside) {
      const c128 l = L[idx];
      a = acc_in[idx] + ca * l;
      if (loss_coef > 0.0) a = edge_loss(i, j, nx, ny, W, eta, loss_coef) * a;
      if (v_out) v = u[idx] + cv * l;
    }
    acc_out[idx] = a;
    if (v_out) v_out[idx] = v;
  }
}

}  // namespace

// ====================================================================== launchers

#define HP_DISPATCH_N(n, MACRO) \
  switch (n) {                  \
    case 64: MACRO(64); break;  \
    case 128: MACRO(128); break;  \
    case 192: MACRO(192); break;  \
    case 256: MACRO(256); break;  \
    case 384: MACRO(384); break;  \
    case 512: MACRO(512); break;  \
    case 768: MACRO(768); break;  \
    case 1024: MACRO(1024); break; \
    case 1536: MACRO(1536); break; \
    case 2048: MACRO(2048); break; \
    default: break;             \
  }

template <typename T>
int row_blocks(int nx) {
  const int NT = nx / 8;
  (void)sizeof(T);
  return (256 / NT) > 0 ? 256 / NT : 1;  // rows per workgroup
}

template <typename T, typename C>
void launch_row_fwd_batch(const c128* in, size_t in_bs, const int* isel_h, cx<T>* out, size_t out_bs,
                          const int* osel_h, int n, double* part, size_t part_bs, const cx<C>* tw, const Geo& g,
                          hipStream_t s, int tile_w) {
  const int rpw = row_blocks<T>(g.nx);
  const int nblk = (g.ny - 1 + rpw - 1) / rpw;
  dim3 grid(nblk, g.ncomp, n);
  if (tile_w <= 0) tile_w = tile_width<T>();
  PoleList isel, osel;
  isel.n = osel.n = n;
  for (int a = 0; a < HP_MAXPOLES; ++a) {
    isel.k[a] = a < n ? isel_h[a] : 0;
    osel.k[a] = a < n ? osel_h[a] : 0;
  }
#define L_(NN)                                                                                                    \
  if (tile_w == 8)                                                                                                \
    hipLaunchKernelGGL((k_row_fwd<T, C, NN, 8>), grid, dim3(RowCfg<NN>::WG), 0, s, in, out, part, tw, g.ny, g.fsz,   \
                       nblk, isel, osel, in_bs, out_bs, part_bs);                                                        \
  else                                                                                                            \
    hipLaunchKernelGGL((k_row_fwd<T, C, NN, 16>), grid, dim3(RowCfg<NN>::WG), 0, s, in, out, part, tw, g.ny, g.fsz,  \
                       nblk, isel, osel, in_bs, out_bs, part_bs);
  HP_DISPATCH_N(g.nx, L_)
#undef L_
}

template <typename T, typename C>
void launch_row_fwd(const c128* in, cx<T>* out, double* part, const cx<C>* tw, const Geo& g, hipStream_t s,
                    int tile_w) {
  const int zero = 0;
  launch_row_fwd_batch<T, C>(in, 0, &zero, out, 0, &zero, 1, part, 0, tw, g, s, tile_w);
}

template <typename T, typename C>
void launch_row_inv_batch(const cx<T>* in, size_t in_bs, const int* sel_h, int n, c128* out, size_t out_bs,
                          const cx<C>* tw, const Geo& g, int tile_w, hipStream_t s) {
  const int rpw = row_blocks<T>(g.nx);
  const int nblk = (g.ny + rpw - 1) / rpw;
  dim3 grid(nblk, g.ncomp, n);
  PoleList sel;
  sel.n = n;
  for (int a = 0; a < HP_MAXPOLES; ++a) sel.k[a] = a < n ? sel_h[a] : 0;
#define L_(NN)                                                                                                  \
  if (tile_w == 8)                                                                                              \
    hipLaunchKernelGGL((k_row_inv<T, C, NN, 8>), grid, dim3(RowCfg<NN>::WG), 0, s, in, out, tw, g.ny, g.fsz, sel,  \
                       in_bs, out_bs);                                                                          \
  else                                                                                                          \
    hipLaunchKernelGGL((k_row_inv<T, C, NN, 16>), grid, dim3(RowCfg<NN>::WG), 0, s, in, out, tw, g.ny, g.fsz, sel, \
                       in_bs, out_bs);
  HP_DISPATCH_N(g.nx, L_)
#undef L_
}

template <typename T, typename C>
void launch_row_inv(const cx<T>* in, c128* out, const cx<C>* tw, const Geo& g, int tile_w, hipStream_t s) {
  const int zero = 0;
  launch_row_inv_batch<T, C>(in, 0, &zero, 1, out, 0, tw, g, tile_w, s);
}

template <typename T, typename C>
void launch_col(const cx<T>* const* uptr, cx<T>* zbase, size_t zsp, size_t zsi, cx<T>* dzbase, size_t dzsp,
                const PoleState* st, const int* poles, int nactive, int* active_out, const double* mu_x,
                const double* mu_y, const cx<C>* tw, const Geo& g, const StencilCoef& sc, hipStream_t s) {
  PoleList list;
  list.n = nactive;
  for (int a = 0; a < HP_MAXPOLES; ++a) list.k[a] = a < nactive ? poles[a] : 0;
#define COLV_(NN, LB)                                                                                          \
  {                                                                                                            \
    dim3 grid(g.nx / ColCfg<T, C, NN, LB>::GC, g.ncomp * nactive);                                             \
    if (g.ncomp == 1)                                                                                          \
      hipLaunchKernelGGL((k_col<T, C, NN, 1, LB>), grid, dim3(ColCfg<T, C, NN, LB>::WG), 0, s, uptr, zbase,    \
                         zsp, zsi, dzbase, dzsp, st, list, active_out, mu_x, mu_y, tw, g.fsz, sc);             \
    else                                                                                                       \
      hipLaunchKernelGGL((k_col<T, C, NN, 2, LB>), grid, dim3(ColCfg<T, C, NN, LB>::WG), 0, s, uptr, zbase,    \
                         zsp, zsi, dzbase, dzsp, st, list, active_out, mu_x, mu_y, tw, g.fsz, sc);             \
  }
#define L_(NN)                                                                                                 \
  {                                                                                                            \
    if (g.col_variant == 0)                                                                                    \
      COLV_(NN, kColLds[0])                                                                                    \
    else if (g.col_variant == 2)                                                                               \
      COLV_(NN, kColLds[2])                                                                                    \
    else                                                                                                       \
      COLV_(NN, kColLds[1])                                                                                    \
  }
  HP_DISPATCH_N(g.ny, L_)
#undef L_
#undef COLV_
}

static int apply_groups(const Geo& g) {
  const int nt = g.nx / 8;
  int groups = (256 / nt) / g.ncomp * g.ncomp;
  if (groups < g.ncomp) groups = g.ncomp;
  return groups;
}

template <typename T>
int row_apply_blocks(const Geo& g) {
  const int rows = apply_groups(g) / g.ncomp;
  return (g.ny - 1 + rows - 1) / rows;
}

template <typename T>
int row_apply_parts(const Geo& g) {
  return row_apply_blocks<T>(g) * ((apply_groups(g) * (g.nx / 8) + 63) / 64);
}

template <typename T, typename C>
void launch_row_apply(const cx<T>* zbase, size_t zsp, size_t zsi, const cx<T>* dzbase, size_t dzsp, cx<T>* pbase,
                      size_t psp, const cx<T>* const* uptr, const C* coef, const PoleState* st,
                      const int* active, int nactive, double2* part, const cx<C>* tw, const Geo& g,
                      const StencilCoef& sc, hipStream_t s) {
  const int nblk = row_apply_blocks<T>(g);
  const int nparts = row_apply_parts<T>(g);
  // one workgroup per (row block, pole), row blocks padded to a multiple of 8
  dim3 grid((unsigned)((nblk + 7) / 8 * 8) * (unsigned)nactive);
#define L_(NN)                                                                                                  \
  if (g.ncomp == 1)                                                                                             \
    hipLaunchKernelGGL((k_row_apply<T, C, NN, 1>), grid, dim3(ApplyCfg<NN, 1>::WG), 0, s, zbase, zsp, zsi, dzbase,  \
                       dzsp, pbase, psp, uptr, coef, st, active, nactive, nblk, part, nparts, tw, g.ny, g.fsz, sc);  \
  else                                                                                                          \
    hipLaunchKernelGGL((k_row_apply<T, C, NN, 2>), grid, dim3(ApplyCfg<NN, 2>::WG), 0, s, zbase, zsp, zsi, dzbase,  \
                       dzsp, pbase, psp, uptr, coef, st, active, nactive, nblk, part, nparts, tw, g.ny, g.fsz, sc);
  HP_DISPATCH_N(g.nx, L_)
#undef L_
}

void launch_reduce_dots(const double2* part, int nblk, PoleState* st, const int* active, int nactive, int maxm,
                        int* done, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_pairs, dim3(2 * (maxm + 1), nactive), dim3(256), 0, s, part, nblk, st, active, done);
}

int update_blocks(size_t total) {
  size_t b = (total + UPD_WG * UPD_E - 1) / (UPD_WG * UPD_E);
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
                    unsigned long long* ftag, unsigned long long seq, double* est, hipStream_t s) {
  hipLaunchKernelGGL(k_arnoldi, dim3(nactive), dim3(64), 0, s, st, active, part, nblk, restart, ftag, seq, est);
}

void launch_cycle_init(PoleState* st, const int* poles, int npoles_in, const double* part, int nblk, int first,
                       double tol, double rtol_cycle, hipStream_t s, size_t part_bs, int set_has_x) {
  hipLaunchKernelGGL(k_cycle_init, dim3(npoles_in), dim3(64), 0, s, st, poles, part, nblk, first, tol, rtol_cycle,
                     part_bs, set_has_x);
}

template <typename T>
void launch_final(const c128* w, c128* out, const cx<T>* zbase, size_t zsp, size_t zsi, const c128* xacc, size_t xsp,
                  const PoleState* st, int npoles, c128 phase, c128 rinf_phase, double loss_coef, double eta, int W,
                  const c128* tw64, const Geo& g, hipStream_t s) {
  const int rpw = row_blocks<double>(g.nx);
  dim3 grid((g.ny + rpw - 1) / rpw, g.ncomp);
#define L_(NN)                                                                                                     \
  hipLaunchKernelGGL((k_final<T, NN>), grid, dim3(RowCfg<NN>::WG), 0, s, w, out, zbase, zsp, zsi, xacc, xsp, st, \
                     npoles, phase, rinf_phase, loss_coef, eta, W, tw64, g.nx, g.ny, g.fsz)
  HP_DISPATCH_N(g.nx, L_)
#undef L_
}

template <typename T>
void launch_accum_batch(c128* xacc, size_t xsp, const cx<T>* z, size_t zsp, size_t zsi, const PoleState* st,
                        const int* sel_h, int n, const Geo& g, hipStream_t s) {
  const size_t total = (size_t)g.ncomp * g.fsz;
  PoleList sel;
  sel.n = n;
  for (int a = 0; a < HP_MAXPOLES; ++a) sel.k[a] = a < n ? sel_h[a] : 0;
  const int nb = std::max(1, update_blocks(total) / n);
  hipLaunchKernelGGL((k_accum<T>), dim3(nb, n), dim3(256), 0, s, xacc, z, zsi, st, sel, xsp, zsp, total);
}

template <typename T>
void launch_accum(c128* xacc, const cx<T>* z, size_t zsi, const PoleState* st, int pole, const Geo& g,
                  hipStream_t s) {
  // xacc and z are pole k's already: a one-entry list with zero strides
  launch_accum_batch<T>(xacc, 0, z, 0, zsi, st, &pole, 1, g, s);
}

int op_blocks(const Geo& g) { return ((g.nx + OP_TX - 1) / OP_TX) * ((g.ny + OP_TY - 1) / OP_TY); }

void launch_apply_op_batch(const c128* x, size_t xbs, const c128* rhs, c128* y, size_t ybs, const double* coef,
                           const c128* shifts_h, int n, const StencilCoef& sc, const Geo& g, double* part, size_t pbs,
                           hipStream_t s, int medium_only) {
  ShiftList sh;
  for (int a = 0; a < HP_MAXPOLES; ++a) sh.b[a] = a < n ? shifts_h[a] : mk(0.0, 0.0);
  const dim3 grid(op_blocks(g), 1, n);
  if (g.ncomp == 2)
    hipLaunchKernelGGL((k_apply_op<2>), grid, dim3(OP_WG), 0, s, x, rhs, y, coef, sh, sc, g.nx, g.ny, g.fsz, part,
                       medium_only, xbs, ybs, pbs);
  else
    hipLaunchKernelGGL((k_apply_op<1>), grid, dim3(OP_WG), 0, s, x, rhs, y, coef, sh, sc, g.nx, g.ny, g.fsz, part,
                       medium_only, xbs, ybs, pbs);
}

void launch_apply_op(const c128* x, const c128* rhs, c128* y, const double* coef, c128 b, const StencilCoef& sc,
                     const Geo& g, double* part, hipStream_t s, int medium_only) {
  launch_apply_op_batch(x, 0, rhs, y, 0, coef, &b, 1, sc, g, part, 0, s, medium_only);
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

void launch_mark_list(PoleState* st, const int* poles, int n, hipStream_t s) {
  PoleList sel;
  sel.n = n;
  for (int a = 0; a < HP_MAXPOLES; ++a) sel.k[a] = a < n ? poles[a] : 0;
  hipLaunchKernelGGL(k_mark_list, dim3(1), dim3(HP_MAXPOLES), 0, s, st, sel);
}

void launch_mark_folded(PoleState* st, int first, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_mark_folded, dim3(1), dim3(HP_MAXPOLES), 0, s, st, first, count);
}

__global__ void k_to_float(const double* __restrict__ a, float* __restrict__ b, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] = (float)a[i];
}

void launch_to_float(const double* a, float* b, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_to_float, dim3(2048), dim3(256), 0, s, a, b, n);
}


void launch_rk4_stage(const c128* L, const c128* acc_in, c128* acc_out, const c128* u, c128* v_out, double ca,
                      double cv, double loss_coef, double eta, int W, const Geo& g, hipStream_t s) {
  const unsigned total = (unsigned)(g.ncomp * g.fsz);
  const unsigned nb = std::min(2048u, (total + 1023u) / 1024u);
  hipLaunchKernelGGL(k_rk4_stage, dim3(nb), dim3(256), 0, s, L, acc_in, acc_out, u, v_out, ca, cv, loss_coef, eta, W,
                     g.nx, g.ny, (unsigned)g.fsz, total);
}

// explicit instantiations
#define HP_INST(T)                                                                                                   \
  template int row_blocks<T>(int);                                                                                   \
  template int row_apply_blocks<T>(const Geo&);                                                                      \
  template int row_apply_parts<T>(const Geo&);                                                                       \
  template void launch_update<T>(const cx<T>*, size_t, cx<T>* const*, const PoleState*, const int*, int, double*,    \
                                 int, const Geo&, hipStream_t);                                                      \
  template void launch_final<T>(const c128*, c128*, const cx<T>*, size_t, size_t, const c128*, size_t,               \
                                const PoleState*, int, c128, c128, double, double, int, const c128*, const Geo&,     \
                                hipStream_t);                                                                        \
  template void launch_accum<T>(c128*, const cx<T>*, size_t, const PoleState*, int, const Geo&, hipStream_t);      \
  template void launch_accum_batch<T>(c128*, size_t, const cx<T>*, size_t, size_t, const PoleState*, const int*,     \
                                      int, const Geo&, hipStream_t);

// storage type T, compute type C of the transforms
#define HP_INST2(T, C)                                                                                               \
  template void launch_row_fwd<T, C>(const c128*, cx<T>*, double*, const cx<C>*, const Geo&, hipStream_t, int);      \
  template void launch_row_inv<T, C>(const cx<T>*, c128*, const cx<C>*, const Geo&, int, hipStream_t);               \
  template void launch_row_fwd_batch<T, C>(const c128*, size_t, const int*, cx<T>*, size_t, const int*, int,       \
                                           double*, size_t, const cx<C>*, const Geo&, hipStream_t, int);             \
  template void launch_row_inv_batch<T, C>(const cx<T>*, size_t, const int*, int, c128*, size_t, const cx<C>*,       \
                                           const Geo&, int, hipStream_t);                                            \
  template void launch_col<T, C>(const cx<T>* const*, cx<T>*, size_t, size_t, cx<T>*, size_t, const PoleState*,      \
                                 const int*, int, int*, const double*, const double*, const cx<C>*, const Geo&,      \
                                 const StencilCoef&, hipStream_t);                                                   \
  template void launch_row_apply<T, C>(const cx<T>*, size_t, size_t, const cx<T>*, size_t, cx<T>*, size_t,           \
                                       const cx<T>* const*, const C*, const PoleState*, const int*, int, double2*,   \
                                       const cx<C>*, const Geo&, const StencilCoef&, hipStream_t);

HP_INST(double)
HP_INST(float)
HP_INST2(double, double)
HP_INST2(float, float)
HP_INST2(float, double)
