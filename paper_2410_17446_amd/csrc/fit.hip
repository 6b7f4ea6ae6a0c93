// The rational approximation of Sec. 3.1 computed on the device: AAA with
// Lawson reweighting for exp(iK sqrt(1+z)) on uniform samples of [lo, hi],
// then its partial fractions.  One workgroup of 512 threads runs the whole
// fit in one launch (the work is a few dozen small least-squares problems in
// sequence, each too small to fill more than one CU); the smallest singular
// vector of each tall sample matrix comes from a QR factorisation by
// Gram-Schmidt with one reorthogonalisation, then one-sided (Hestenes) Jacobi
// on the small triangular factor, all FP64.  Poles are the roots of the
// barycentric denominator, found by the Aberth-Ehrlich simultaneous iteration.
#include <math.h>

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "cplx.hpp"

namespace {

constexpr int FWG = 512;           // threads of the one workgroup (223 registers each, no spills)
constexpr int FWAVES = FWG / 64;
constexpr int FMAXC = 64;          // columns of a sample matrix (2 x support points)
constexpr int FMAXS = 4096;        // samples
constexpr int FRQ = FMAXS / FWG;   // sample rows per thread
constexpr int FCH = 8;             // inner products reduced together

struct FitArgs {
  double K, lo, hi;
  int S, degree, lawson;
  double* Z;     // [S] samples
  c128* M;       // [FMAXC][S] sample matrix, column-major; becomes Q
  c128* F;       // [S] target values
  c128* approx;  // [S] AAA's current approximation
  double* wts;   // [S] Lawson weights
  double* err;   // [S]
  int* chosen;   // [S]
  c128* out;     // poles [degree], residues [degree], r_inf, then (max error, status) as reals
};

__device__ __forceinline__ double f_wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

__device__ __forceinline__ double f_wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
  return v;
}

// Sum over the workgroup; every thread gets the result.
__device__ double f_block_sum(double v, double* red) {
  v = f_wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < FWAVES; ++w) s += red[w];
  __syncthreads();
  return s;
}

__device__ double f_block_max(double v, double* red) {
  v = f_wave_max(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = red[0];
#pragma unroll
  for (int w = 1; w < FWAVES; ++w) s = fmax(s, red[w]);
  __syncthreads();
  return s;
}

// Index of the largest v over the workgroup (smallest index among equals); every thread gets it.
__device__ int f_block_argmax(double v, int idx, double* redv, int* redi) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_down(v, off, 64);
    const int oi = __shfl_down(idx, off, 64);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    redv[threadIdx.x >> 6] = v;
    redi[threadIdx.x >> 6] = idx;
  }
  __syncthreads();
  double bv = redv[0];
  int bi = redi[0];
  for (int w = 1; w < FWAVES; ++w)
    if (redv[w] > bv || (redv[w] == bv && redi[w] < bi)) {
      bv = redv[w];
      bi = redi[w];
    }
  __syncthreads();
  return bi;
}

// acc[0..FCH) summed over the workgroup into out[0..n) (shared memory); red holds FWAVES * 2 FCH.
__device__ void f_block_sum_vec(const c128* acc, int n, c128* out, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < FCH; ++k) {
    const double re = f_wave_sum(acc[k].re), im = f_wave_sum(acc[k].im);
    if (lane == 0) {
      red[wave * 2 * FCH + 2 * k] = re;
      red[wave * 2 * FCH + 2 * k + 1] = im;
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * n) {
    double s = 0.0;
    for (int w = 0; w < FWAVES; ++w) s += red[w * 2 * FCH + threadIdx.x];
    double* o = reinterpret_cast<double*>(out);
    o[threadIdx.x] = s;
  }
  __syncthreads();
}

__device__ __forceinline__ c128 f_conj(c128 a) { return mk(a.re, -a.im); }

// exp(iK sqrt(1+z)) on the principal branch (decay below z = -1)
__device__ __forceinline__ c128 f_target(double z, double K) {
  const double s = 1.0 + z;
  if (s >= 0.0) {
    const double ph = K * sqrt(s);
    return mk(cos(ph), sin(ph));
  }
  return mk(exp(-K * sqrt(-s)), 0.0);
}

// lo + i h with the product and the sum rounded separately (no fused multiply-add:
// next to the branch point z = -1 one rounding more or less moves the sample
// across it, and exp(iK sqrt(1+z)) changes by K sqrt(eps) there)
__device__ __attribute__((noinline)) double f_sample(double lo, double h, int i) {
#pragma clang fp contract(off)
  const double p = (double)i * h;
  return lo + p;
}

struct FitShared {
  double red[FWAVES * 2 * FCH];
  int redi[FWAVES];
  c128 dots[FMAXC];
  c128 vec[FMAXC];        // the smallest right singular vector
  double t[FMAXC / 2];    // support points
  double ts[FMAXC / 2];   // the same, sorted
  c128 ft[FMAXC / 2];
  c128 a[FMAXC / 2], b[FMAXC / 2];
  c128 besta[FMAXC / 2], bestb[FMAXC / 2];
  c128 z[FMAXC / 2], zn[FMAXC / 2];   // root estimates
  c128 pole[FMAXC / 2], res[FMAXC / 2];
  c128 rinf;
  int sidx[FMAXC / 2];
  int flag;
};

// v = right singular vector of the smallest singular value of M[:, 0..c), S rows.
// M is overwritten by Q; R and V ([FMAXC][FMAXC], column-major, in LDS) are scratch.
__device__ void f_min_right_sv(const FitArgs& A, int c, FitShared& sh, c128* R, c128* V) {
  const int S = A.S, tid = threadIdx.x;
  c128* M = A.M;
  // classical Gram-Schmidt with one reorthogonalisation, column by column
  for (int j = 0; j < c; ++j) {
    c128* mj = M + (size_t)j * S;
    for (int pass = 0; pass < 2; ++pass) {
      for (int k0 = 0; k0 < j; k0 += FCH) {
        const int kc = min(FCH, j - k0);
        c128 acc[FCH];
#pragma unroll
        for (int k = 0; k < FCH; ++k) acc[k] = mk(0.0, 0.0);
        for (int q = 0; q < FRQ; ++q) {
          const int i = tid + FWG * q;
          if (i >= S) break;
          const c128 m = mj[i];
#pragma unroll
          for (int k = 0; k < FCH; ++k)
            if (k < kc) acc[k] = acc[k] + cmulc(M[(size_t)(k0 + k) * S + i], m);
        }
        f_block_sum_vec(acc, kc, sh.dots + k0, sh.red);
      }
      for (int q = 0; q < FRQ; ++q) {
        const int i = tid + FWG * q;
        if (i >= S) break;
        c128 m = mj[i];
        for (int k = 0; k < j; ++k) m = m - M[(size_t)k * S + i] * sh.dots[k];
        mj[i] = m;
      }
      if (tid < j) {
        c128& r = R[tid + (size_t)j * FMAXC];
        r = pass == 0 ? sh.dots[tid] : r + sh.dots[tid];
      }
      __syncthreads();
    }
    double nn = 0.0;
    for (int q = 0; q < FRQ; ++q) {
      const int i = tid + FWG * q;
      if (i < S) nn += abs2(mj[i]);
    }
    const double nrm = sqrt(f_block_sum(nn, sh.red));
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    for (int q = 0; q < FRQ; ++q) {
      const int i = tid + FWG * q;
      if (i < S) mj[i] = inv * mj[i];
    }
    if (tid < c) {
      if (tid > j) R[tid + (size_t)j * FMAXC] = mk(0.0, 0.0);
      if (tid == j) R[tid + (size_t)j * FMAXC] = mk(nrm, 0.0);
    }
    __syncthreads();
  }
  // one-sided Jacobi on the columns of R (c x c), rotations accumulated in V
  for (int e = tid; e < c * c; e += FWG) {
    const int r = e % c, col = e / c;
    V[r + (size_t)col * FMAXC] = mk(r == col ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  const int cp = c + (c & 1);  // players of the round-robin; player c is a bye when c is odd
  // a wave per column pair (lane i holds row i), pairs of a round spread over the waves;
  // a pair is rotated while its columns' inner product exceeds 1e-14 of their norms
  const int wave = tid >> 6, lane = tid & 63;
  auto wsum = [](double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return __shfl(v, 0, 64);  // every lane takes lane 0's sum
  };
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) sh.flag = 0;
    __syncthreads();
    for (int round = 0; round < cp - 1; ++round) {
      for (int slot = wave; slot < cp / 2; slot += FWAVES) {
        int p, q;
        if (slot == 0) {
          p = round;
          q = cp - 1;
        } else {
          p = (round + slot) % (cp - 1);
          q = (round - slot + (cp - 1)) % (cp - 1);
        }
        if (p >= c || q >= c) continue;
        c128* rp = R + (size_t)p * FMAXC;
        c128* rq = R + (size_t)q * FMAXC;
        const c128 x = lane < c ? rp[lane] : mk(0.0, 0.0), y = lane < c ? rq[lane] : mk(0.0, 0.0);
        const double al = wsum(abs2(x)), be = wsum(abs2(y));
        const c128 xy = cmulc(x, y);
        const c128 ga = mk(wsum(xy.re), wsum(xy.im));
        const double g = sqrt(abs2(ga));
        if (!(g > 1e-14 * sqrt(al * be) && g > 0.0)) continue;
        const double zeta = (be - al) / (2.0 * g);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / sqrt(1.0 + t * t), sn = t * cs;
        const c128 ph = mk(ga.re / g, ga.im / g);  // e^{i phi}
        const c128 phc = f_conj(ph);
        if (lane < c) {
          rp[lane] = cs * x - sn * (phc * y);
          rq[lane] = sn * (ph * x) + cs * y;
          c128* vp = V + (size_t)p * FMAXC;
          c128* vq = V + (size_t)q * FMAXC;
          const c128 u = vp[lane], w = vq[lane];
          vp[lane] = cs * u - sn * (phc * w);
          vq[lane] = sn * (ph * u) + cs * w;
        }
        if (lane == 0) sh.flag = 1;
      }
      __syncthreads();
    }
    const int any = sh.flag;
    __syncthreads();
    if (!any) break;
  }
  // the column of smallest norm
  if (tid == 0) {
    int jm = 0;
    double best = 1e300;
    for (int j = 0; j < c; ++j) {
      double s = 0.0;
      for (int i = 0; i < c; ++i) s += abs2(R[i + (size_t)j * FMAXC]);
      if (s < best) {
        best = s;
        jm = j;
      }
    }
    sh.redi[0] = jm;
  }
  __syncthreads();
  const int jm = sh.redi[0];
  if (tid < c) sh.vec[tid] = V[tid + (size_t)jm * FMAXC];
  __syncthreads();
}

// Partial fractions of the barycentric form with weights a (numerator), b
// (denominator) at the n support points: poles (roots of sum_k b_k/(z - t_k))
// by Aberth-Ehrlich, residues n(p)/d'(p), r_inf = sum a / sum b.  Returns the
// number of finite poles found (n - 1 when the form is regular).
__device__ int f_partial_fractions(int n, const c128* a, const c128* b, FitShared& sh) {
  const int tid = threadIdx.x, np = n - 1;
  // start from the midpoints of the sorted support points, slightly below the axis
  if (tid == 0) {
    double* ts = sh.ts;
    for (int k = 0; k < n; ++k) ts[k] = sh.t[k];
    for (int k = 1; k < n; ++k) {
      const double v = ts[k];
      int j = k - 1;
      while (j >= 0 && ts[j] > v) {
        ts[j + 1] = ts[j];
        --j;
      }
      ts[j + 1] = v;
    }
    for (int k = 0; k < np; ++k) {
      const double gap = ts[k + 1] - ts[k];
      sh.z[k] = mk(0.5 * (ts[k] + ts[k + 1]) + 0.1 * gap, -0.3 * gap - 1e-3);
    }
    sh.flag = 0;
  }
  __syncthreads();
  for (int it = 0; it < 200; ++it) {
    double step = 0.0;
    if (tid < np) {
      const c128 zi = sh.z[tid];
      c128 d = mk(0.0, 0.0), dd = mk(0.0, 0.0), s1 = mk(0.0, 0.0);
      for (int k = 0; k < n; ++k) {
        const c128 u = cdiv(mk(1.0, 0.0), zi - mk(sh.t[k], 0.0));
        d = d + b[k] * u;
        dd = dd - b[k] * (u * u);
        s1 = s1 + u;
      }
      // N/N' for N = d prod(z - t_k): d / (d' + d sum 1/(z - t_k)), 0 at an exact root
      const c128 den = dd + d * s1;
      const c128 ratio = abs2(den) > 0.0 ? cdiv(d, den) : mk(0.0, 0.0);
      c128 ab = mk(0.0, 0.0);
      for (int j = 0; j < np; ++j)
        if (j != tid) ab = ab + cdiv(mk(1.0, 0.0), zi - sh.z[j]);
      const c128 w = cdiv(ratio, mk(1.0, 0.0) - ratio * ab);
      sh.zn[tid] = zi - w;
      const double az = sqrt(abs2(zi));
      step = sqrt(abs2(w)) / (az > 1e-300 ? az : 1.0);
      if (!(step == step)) step = 1e300;
    }
    const double mx = f_block_max(tid < np ? step : 0.0, sh.red);
    if (tid < np) sh.z[tid] = sh.zn[tid];
    __syncthreads();
    if (mx < 1e-14) break;
  }
  // residues and the value at infinity
  if (tid == 0) {
    int count = 0;
    c128 sa = mk(0.0, 0.0), sb = mk(0.0, 0.0);
    for (int k = 0; k < n; ++k) {
      sa = sa + a[k];
      sb = sb + b[k];
    }
    sh.rinf = cdiv(sa, sb);
    for (int i = 0; i < np; ++i) {
      const c128 p = sh.z[i];
      const bool ok = isfinite(p.re) && isfinite(p.im) && sqrt(abs2(p)) < 1e12;
      if (!ok) continue;
      c128 num = mk(0.0, 0.0), den = mk(0.0, 0.0);
      for (int k = 0; k < n; ++k) {
        const c128 u = cdiv(mk(1.0, 0.0), p - mk(sh.t[k], 0.0));
        num = num + a[k] * u;
        den = den - b[k] * (u * u);
      }
      sh.pole[count] = p;
      sh.res[count] = cdiv(num, den);
      ++count;
    }
    sh.flag = count;
  }
  __syncthreads();
  const int count = sh.flag;
  __syncthreads();
  return count;
}

// Largest |r - F| over the samples for the partial fractions in sh (inf if not finite).
__device__ double f_pf_error(const FitArgs& A, int np, FitShared& sh) {
  double mx = 0.0;
  for (int q = 0; q < FRQ; ++q) {
    const int i = threadIdx.x + FWG * q;
    if (i >= A.S) break;
    const double z = A.Z[i];
    c128 r = sh.rinf;
    for (int k = 0; k < np; ++k) r = r + cdiv(sh.res[k], mk(z, 0.0) - sh.pole[k]);
    double e = sqrt(abs2(r - A.F[i]));
    if (!(e <= 1e300)) e = 1e300;
    mx = fmax(mx, e);
  }
  return f_block_max(mx, sh.red);
}

__global__ __launch_bounds__(FWG) void k_fit(FitArgs A) {
  __shared__ FitShared sh;
  __shared__ c128 R[FMAXC * FMAXC];  // the small factor and the rotations of the Jacobi sweeps
  __shared__ c128 V[FMAXC * FMAXC];
  const int tid = threadIdx.x, S = A.S, n = A.degree + 1;
  const double h = (A.hi - A.lo) / (S - 1);
  // samples lo + i h (the product and the sum each rounded once, the last sample hi itself)
  // and the target; AAA starts from the mean
  c128 fs = mk(0.0, 0.0);
  for (int q = 0; q < FRQ; ++q) {
    const int i = tid + FWG * q;
    if (i >= S) break;
    const double zi = i == S - 1 ? A.hi : f_sample(A.lo, h, i);
    A.Z[i] = zi;
    const c128 f = f_target(zi, A.K);
    A.F[i] = f;
    A.chosen[i] = 0;
    fs = fs + f;
  }
  const c128 mean = mk(f_block_sum(fs.re, sh.red) / S, f_block_sum(fs.im, sh.red) / S);
  for (int q = 0; q < FRQ; ++q) {
    const int i = tid + FWG * q;
    if (i < S) A.approx[i] = mean;
  }
  __syncthreads();
  // ---- AAA: greedy support points, weights from the Loewner matrix
  for (int m = 0; m < n; ++m) {
    double bv = -1.0;
    int bi = 0x7fffffff;
    for (int q = 0; q < FRQ; ++q) {
      const int i = tid + FWG * q;
      if (i >= S || A.chosen[i]) continue;
      const double e = sqrt(abs2(A.F[i] - A.approx[i]));
      if (e > bv) {
        bv = e;
        bi = i;
      }
    }
    const int pick = f_block_argmax(bv, bi, sh.red, sh.redi);
    if (tid == 0) {
      A.chosen[pick] = 1;
      sh.sidx[m] = pick;
      sh.t[m] = A.Z[pick];
      sh.ft[m] = A.F[pick];
    }
    __syncthreads();
    const int c = m + 1;
    for (int q = 0; q < FRQ; ++q) {
      const int i = tid + FWG * q;
      if (i >= S) break;
      const bool ch = A.chosen[i];
      const double z = A.Z[i];
      for (int k = 0; k < c; ++k)
        A.M[(size_t)k * S + i] = ch ? mk(0.0, 0.0) : (1.0 / (z - sh.t[k])) * (A.F[i] - sh.ft[k]);
    }
    __syncthreads();
    f_min_right_sv(A, c, sh, R, V);
    for (int q = 0; q < FRQ; ++q) {
      const int i = tid + FWG * q;
      if (i >= S) break;
      if (A.chosen[i]) {
        A.approx[i] = A.F[i];
        continue;
      }
      const double z = A.Z[i];
      c128 num = mk(0.0, 0.0), den = mk(0.0, 0.0);
      for (int k = 0; k < c; ++k) {
        const double u = 1.0 / (z - sh.t[k]);
        num = num + u * (sh.vec[k] * sh.ft[k]);
        den = den + u * sh.vec[k];
      }
      A.approx[i] = cdiv(num, den);
    }
    __syncthreads();
  }
  if (tid < n) {
    sh.b[tid] = sh.vec[tid];
    sh.a[tid] = sh.vec[tid] * sh.ft[tid];
  }
  __syncthreads();
  // ---- Lawson: reweighted linearised least squares; keep the iterate whose partial
  // fractions have the smallest largest error on the samples (AAA's own included)
  double best = 1e300;
  {
    const int np = f_partial_fractions(n, sh.a, sh.b, sh);
    best = np == A.degree ? f_pf_error(A, np, sh) : 1e300;
    if (tid < n) {
      sh.besta[tid] = sh.a[tid];
      sh.bestb[tid] = sh.b[tid];
    }
  }
  for (int q = 0; q < FRQ; ++q) {
    const int i = tid + FWG * q;
    if (i < S) A.wts[i] = 1.0 / S;
  }
  __syncthreads();
  // row of sample i: the Cauchy row 1/(z_i - t_k), or e_j / h for support point j
  for (int step = 0; step < A.lawson; ++step) {
    for (int q = 0; q < FRQ; ++q) {
      const int i = tid + FWG * q;
      if (i >= S) break;
      const double sw = sqrt(A.wts[i]);
      const c128 f = A.F[i];
      const double z = A.Z[i];
      int sup = -1;
      if (A.chosen[i])
        for (int k = 0; k < n; ++k)
          if (sh.sidx[k] == i) sup = k;
      for (int k = 0; k < n; ++k) {
        const double ck = sup >= 0 ? (k == sup ? 1.0 / h : 0.0) : 1.0 / (z - sh.t[k]);
        A.M[(size_t)k * S + i] = (sw * ck) * f;              // unknowns b
        A.M[(size_t)(n + k) * S + i] = mk(-sw * ck, 0.0);    // unknowns a
      }
    }
    __syncthreads();
    f_min_right_sv(A, 2 * n, sh, R, V);
    if (tid < n) {
      sh.b[tid] = sh.vec[tid];
      sh.a[tid] = sh.vec[n + tid];
    }
    __syncthreads();
    // errors of the linearised form on every row
    double emax = 0.0;
    int finite = 0;
    for (int q = 0; q < FRQ; ++q) {
      const int i = tid + FWG * q;
      if (i >= S) break;
      const double z = A.Z[i];
      int sup = -1;
      if (A.chosen[i])
        for (int k = 0; k < n; ++k)
          if (sh.sidx[k] == i) sup = k;
      c128 num = mk(0.0, 0.0), den = mk(0.0, 0.0);
      if (sup >= 0) {
        num = (1.0 / h) * sh.a[sup];
        den = (1.0 / h) * sh.b[sup];
      } else {
        for (int k = 0; k < n; ++k) {
          const double u = 1.0 / (z - sh.t[k]);
          num = num + u * sh.a[k];
          den = den + u * sh.b[k];
        }
      }
      double e = (abs2(den) > 0.0) ? sqrt(abs2(A.F[i] - cdiv(num, den))) : INFINITY;
      if (!(e == e)) e = INFINITY;
      A.err[i] = e;
      if (e < INFINITY) {
        emax = fmax(emax, e);
        finite = 1;
      }
    }
    const double emx = f_block_max(emax, sh.red);
    const double anyf = f_block_max((double)finite, sh.red);
    const int np = f_partial_fractions(n, sh.a, sh.b, sh);
    const double score = np == A.degree ? f_pf_error(A, np, sh) : 1e300;
    if (score < best) {
      best = score;
      if (tid < n) {
        sh.besta[tid] = sh.a[tid];
        sh.bestb[tid] = sh.b[tid];
      }
    }
    __syncthreads();
    if (anyf == 0.0) break;
    double ws = 0.0;
    for (int q = 0; q < FRQ; ++q) {
      const int i = tid + FWG * q;
      if (i >= S) break;
      const double e = fmin(A.err[i], emx);
      const double wv = A.wts[i] * fmax(e, 1e-300);
      A.wts[i] = wv;
      ws += wv;
    }
    const double tot = f_block_sum(ws, sh.red);
    for (int q = 0; q < FRQ; ++q) {
      const int i = tid + FWG * q;
      if (i < S) A.wts[i] = A.wts[i] / tot;
    }
    __syncthreads();
  }
  // ---- the kept iterate's partial fractions
  const int np = f_partial_fractions(n, sh.besta, sh.bestb, sh);
  const double emax = np == A.degree ? f_pf_error(A, np, sh) : 1e300;
  if (tid == 0) {
    for (int k = 0; k < np && k < A.degree; ++k) {
      A.out[k] = sh.pole[k];
      A.out[A.degree + k] = sh.res[k];
    }
    A.out[2 * A.degree] = sh.rinf;
    A.out[2 * A.degree + 1] = mk(emax, (double)np);
  }
}

}  // namespace

// The fit on stream s: h receives poles [degree], residues [degree], r_inf and
// (largest sample error, number of finite poles); 0 on success, else a HIP
// error (why says which call failed).
int fit_exp_sqrt_device(double K, int degree, int lawson_steps, hipStream_t s, std::vector<c128>& h,
                        std::string* why) {
  const int S = 4001;
  const size_t bytes = ((size_t)FMAXC * S + 2 * (size_t)FMAXC * FMAXC + 2 * (size_t)S + 2 * (size_t)degree + 2) *
                           sizeof(c128) +
                       3 * (size_t)S * sizeof(double) + (size_t)S * sizeof(int) + 4096;
  char* mem = nullptr;
  if (hipMalloc(&mem, bytes) != hipSuccess) {
    *why = "hipMalloc of the fit's scratch failed";
    return 1;
  }
  char* next = mem;
  auto take = [&](size_t n) {
    char* p = next;
    next += (n + 255) & ~(size_t)255;
    return p;
  };
  FitArgs A;
  A.K = K;
  A.lo = -4.0;
  A.hi = 2.0;
  A.S = S;
  A.degree = degree;
  A.lawson = lawson_steps;
  A.Z = reinterpret_cast<double*>(take((size_t)S * sizeof(double)));
  A.M = reinterpret_cast<c128*>(take((size_t)FMAXC * S * sizeof(c128)));
  A.F = reinterpret_cast<c128*>(take((size_t)S * sizeof(c128)));
  A.approx = reinterpret_cast<c128*>(take((size_t)S * sizeof(c128)));
  A.wts = reinterpret_cast<double*>(take((size_t)S * sizeof(double)));
  A.err = reinterpret_cast<double*>(take((size_t)S * sizeof(double)));
  A.chosen = reinterpret_cast<int*>(take((size_t)S * sizeof(int)));
  A.out = reinterpret_cast<c128*>(take((2 * (size_t)degree + 2) * sizeof(c128)));
  int rc = 0;
  hipLaunchKernelGGL(k_fit, dim3(1), dim3(FWG), 0, s, A);
  h.assign(2 * (size_t)degree + 2, mk(0.0, 0.0));
  if (hipGetLastError() != hipSuccess) {
    *why = "k_fit launch failed";
    rc = 1;
  } else if (hipMemcpyAsync(h.data(), A.out, h.size() * sizeof(c128), hipMemcpyDeviceToHost, s) != hipSuccess ||
             hipStreamSynchronize(s) != hipSuccess) {
    *why = "copying the fit back failed";
    rc = 1;
  }
  (void)hipFree(mem);
  return rc;
}
