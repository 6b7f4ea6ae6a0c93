// In-LDS Stockham FFT and the DST-I built on it.
//
// The free-space preconditioner (Sec. 4.2.2, eq. fs_sylvester) is
// diagonalised by the orthonormal DST-I of length n-1 on each axis:
//   X_p = sqrt(2/n) sum_{j=1}^{n-1} x_j sin(pi p j / n).
// S is symmetric and S S = I, so the same routine is its own inverse.
//
// dst1() computes it with one complex FFT of length n (not the 2n of the odd
// extension).  With x_0 = x_n = 0 and
//   y_j = sin(pi j/n) (x_j + x_{n-j}) + (x_j - x_{n-j}) / 2,   F = FFT_n(y),
// the sums sum_j y_j sin(2 pi j k/n) and sum_j y_j cos(2 pi j k/n) reduce (the
// terms pair up under j -> n - j) to
//   X_{2k}   = (i/2) (F_k - F_{n-k}),
//   X_{2k+1} = X_{2k-1} + (F_k + F_{n-k}) / 2,   X_1 = F_0 / 2,
// so the odd outputs are a prefix sum (a shuffle scan here).  This holds for
// complex x because every step is linear with real coefficients.
//
// FFT: self-sorting Stockham radix-16/8/4/2 (and 3) with the data in LDS, one group of
// NT = L/8 threads per transform, each thread holding R values of a stage in
// registers.  Twiddles come from a table tw[m] = exp(-2 pi i m / L).
//
// LDS layout of a transform buffer: element e sits at pidx<T>(e) =
// e XOR ((e / 8) mod S), S = 256 / sizeof(cx<T>) elements per 256 bytes (16
// for complex128, 32 for complex64).  The XOR only permutes each aligned run
// of S elements, so the buffer needs no padding; measured with the LDS
// bank-conflict counter, a wave reading an aligned run (every stage's reads),
// writing with a stride of 8 elements (the first stage) or in runs of 8 at a
// stride of 64 (the second) then meets no conflicts, where a one-in-eight pad
// left every aligned read with one.
#pragma once
#include "cplx.hpp"

template <typename T>
__host__ __device__ constexpr int lds_run() {
  return 256 / (int)sizeof(cx<T>);
}
template <typename T>
__host__ __device__ constexpr int pidx(int e) {
  return e ^ ((e >> 3) & (lds_run<T>() - 1));
}
// Indices e0 + k STRIDE of one thread: when STRIDE is a multiple of
// 8 lds_run<T>() the XOR term of every one of them equals that of e0, so they
// are pidx(e0) + k STRIDE (constant offsets, no per-element address VGPRs).
template <typename T, int STRIDE>
struct PStep {
  static constexpr bool LINEAR = STRIDE % (8 * lds_run<T>()) == 0;
  int e0, p0;
  __device__ __forceinline__ explicit PStep(int e) : e0(e), p0(pidx<T>(e)) {}
  __device__ __forceinline__ int operator()(int k) const {
    if constexpr (LINEAR)
      return p0 + k * STRIDE;
    else
      return pidx<T>(e0 + k * STRIDE);
  }
};

// LDS elements of one transform buffer of length L (whole runs)
template <typename T>
__host__ __device__ constexpr int plen(int L) {
  return (L + lds_run<T>() - 1) / lds_run<T>() * lds_run<T>();
}

template <typename T>
__device__ __forceinline__ void dft4(cx<T>& a0, cx<T>& a1, cx<T>& a2, cx<T>& a3) {
  cx<T> t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3, t3 = mul_mi(a1 - a3);
  a0 = t0 + t2;
  a1 = t1 + t3;
  a2 = t0 - t2;
  a3 = t1 - t3;
}

template <typename T, int R>
__device__ __forceinline__ void dft(cx<T>* v) {
  if constexpr (R == 3) {
    // X1 = a + w b + w^2 c, w = exp(-2 pi i / 3)
    const T h3 = (T)0.866025403784438646763723170752936183;
    const cx<T> t1 = v[1] + v[2];
    const cx<T> t2 = v[0] - (T)0.5 * t1;
    const cx<T> t3 = h3 * mul_mi(v[1] - v[2]);
    v[0] = v[0] + t1;
    v[1] = t2 + t3;
    v[2] = t2 - t3;
  } else if constexpr (R == 2) {
    cx<T> t = v[0];
    v[0] = t + v[1];
    v[1] = t - v[1];
  } else if constexpr (R == 4) {
    dft4(v[0], v[1], v[2], v[3]);
  } else if constexpr (R == 16) {
    // 16 = 4 x 4: length-4 DFTs over n1 (n = 4 n1 + n2), twiddles W16^(n2 k1),
    // length-4 DFTs over n2; output k = k1 + 4 k2
    const T c1 = (T)0.923879532511286756128183189396788933;  // cos(pi/8)
    const T s1 = (T)0.382683432365089771728459984030398866;  // sin(pi/8)
    const T h = (T)0.707106781186547524400844362104849039;
    cx<T> a[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      a[n2][0] = v[n2];
      a[n2][1] = v[4 + n2];
      a[n2][2] = v[8 + n2];
      a[n2][3] = v[12 + n2];
      dft4(a[n2][0], a[n2][1], a[n2][2], a[n2][3]);
    }
    // W16^m = cos(m pi/8) - i sin(m pi/8), m = n2 k1 in {1, 2, 3, 4, 6, 9}
    a[1][1] = a[1][1] * mk<T>(c1, -s1);
    a[1][2] = a[1][2] * mk<T>(h, -h);
    a[1][3] = a[1][3] * mk<T>(s1, -c1);
    a[2][1] = a[2][1] * mk<T>(h, -h);
    a[2][2] = mul_mi(a[2][2]);
    a[2][3] = a[2][3] * mk<T>(-h, -h);
    a[3][1] = a[3][1] * mk<T>(s1, -c1);
    a[3][2] = a[3][2] * mk<T>(-h, -h);
    a[3][3] = a[3][3] * mk<T>(-c1, s1);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      cx<T> b0 = a[0][k1], b1 = a[1][k1], b2 = a[2][k1], b3 = a[3][k1];
      dft4(b0, b1, b2, b3);
      v[k1] = b0;
      v[k1 + 4] = b1;
      v[k1 + 8] = b2;
      v[k1 + 12] = b3;
    }
  } else {
    static_assert(R == 8, "radix");
    cx<T> a0 = v[0], a1 = v[2], a2 = v[4], a3 = v[6];
    cx<T> b0 = v[1], b1 = v[3], b2 = v[5], b3 = v[7];
    dft4(a0, a1, a2, a3);
    dft4(b0, b1, b2, b3);
    const T h = (T)0.707106781186547524400844362104849039;
    cx<T> t1 = mk<T>(h * (b1.re + b1.im), h * (b1.im - b1.re));   // b1 * e^{-i pi/4}
    cx<T> t2 = mul_mi(b2);                                        // b2 * e^{-i pi/2}
    cx<T> t3 = mk<T>(h * (b3.im - b3.re), -h * (b3.re + b3.im));  // b3 * e^{-3i pi/4}
    v[0] = a0 + b0;
    v[4] = a0 - b0;
    v[1] = a1 + t1;
    v[5] = a1 - t1;
    v[2] = a2 + t2;
    v[6] = a2 - t2;
    v[3] = a3 + t3;
    v[7] = a3 - t3;
  }
}

// One Stockham stage: butterflies j = t, t+NT, ... (< L/R); input stride L/R,
// output (j / NS) * NS * R + (j % NS) + r * NS.
template <typename T, int L, int R, int NS, int NT>
__device__ __forceinline__ void fft_stage(cx<T>* buf, const cx<T>* __restrict__ tw, int t) {
  constexpr int NB = L / R;
  constexpr int PER = (NB + NT - 1) / NT;
  constexpr bool EXACT = PER * NT == NB;
  cx<T> v[PER][R];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int j = t + q * NT;
    if (!EXACT && j >= NB) continue;
    const PStep<T, NB> at(j);
#pragma unroll
    for (int r = 0; r < R; ++r) v[q][r] = buf[at(r)];
    if constexpr (NS > 1) {
      const int k = j % NS;
      constexpr int STEP = L / (NS * R);
      if constexpr (sizeof(T) == 8 && R > 2) {
        // complex128: powers of one table twiddle (fewer live registers; the
        // products add a few ulps, far below the FP64 step tolerance)
        const cx<T> w1 = tw[k * STEP];
        cx<T> wr = w1;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          v[q][r] = v[q][r] * wr;
          if (r + 1 < R) wr = wr * w1;
        }
      } else {
#pragma unroll
        for (int r = 1; r < R; ++r) v[q][r] = v[q][r] * tw[r * k * STEP];
      }
    }
    dft<T, R>(v[q]);
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int j = t + q * NT;
    if (!EXACT && j >= NB) continue;
    const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
    for (int r = 0; r < R; ++r) buf[pidx<T>(base + r * NS)] = v[q][r];
  }
  __syncthreads();
}

template <typename T, int L, int NS, int NT>
__device__ __forceinline__ void fft_stages(cx<T>* buf, const cx<T>* __restrict__ tw, int t) {
  if constexpr (NS < L) {
    constexpr int REM = L / NS;
    // radix 8 where it leaves no radix-2 stage; 16 for remainders 16 and 256
    // (so 1024 = 8 8 16 and 2048 = 8 16 16: three passes through LDS, not four)
    constexpr int R = (REM == 16 || REM == 256) ? 16
                                                : ((REM % 8 == 0) ? 8 : ((REM % 4 == 0) ? 4 : ((REM % 2 == 0) ? 2 : 3)));
    static_assert(REM % R == 0, "lengths are 2^k or 3 * 2^k");
    fft_stage<T, L, R, NS, NT>(buf, tw, t);
    fft_stages<T, L, NS * R, NT>(buf, tw, t);
  }
}

// Forward DFT of length L of buf (in place, natural order).  Every thread of
// the workgroup must call it (it contains __syncthreads); t in [0, L/8).
template <typename T, int L>
__device__ __forceinline__ void fft(cx<T>* buf, const cx<T>* __restrict__ tw, int t) {
  fft_stages<T, L, 1, L / 8>(buf, tw, t);
}

// Value at index i (any integer in (-n, 2n)) of the odd-periodic sequence whose
// entries 1..n-1 sit (FFT output, unscaled) in buf: reflection about 0 and n.
template <typename T>
__device__ __forceinline__ cx<T> odd_at(const cx<T>* buf, int n, int i) {
  if (i > 0 && i < n) return buf[pidx<T>(i)];
  if (i < 0 && i > -n) return -buf[pidx<T>(-i)];
  if (i > n && i < 2 * n) return -buf[pidx<T>(2 * n - i)];
  return mk<T>(0, 0);
}

// Inclusive prefix sum of v over the NT threads t = 0..NT-1 of one transform
// (groups of NT consecutive threads are independent).  Power-of-two NT: wave
// shuffles, plus LDS across waves; scr holds NT/64 elements per group.  Other
// NT (3 * 2^k lengths): Hillis-Steele in LDS; scr holds 2 NT elements per
// group.  Contains __syncthreads: every thread of the workgroup must call it.
template <int NT>
struct ScanScratch {
  static constexpr bool POW2 = (NT & (NT - 1)) == 0;
  static constexpr int SIZE = POW2 ? (NT > 64 ? NT / 64 : 1) : 2 * NT;
};

template <typename T, int NT>
__device__ __forceinline__ cx<T> group_scan(cx<T> v, cx<T>* scr, int t) {
  if constexpr (!ScanScratch<NT>::POW2) {
    cx<T>* a = scr;
    cx<T>* b = scr + NT;
    a[t] = v;
    __syncthreads();
#pragma unroll
    for (int d = 1; d < NT; d <<= 1) {
      const cx<T> x = (t >= d) ? a[t] + a[t - d] : a[t];
      b[t] = x;
      __syncthreads();
      cx<T>* tmp = a;
      a = b;
      b = tmp;
    }
    const cx<T> r = a[t];
    __syncthreads();
    return r;
  }
  constexpr int W = NT < 64 ? NT : 64;
#pragma unroll
  for (int d = 1; d < W; d <<= 1) {
    const T re = __shfl_up(v.re, d, W), im = __shfl_up(v.im, d, W);
    if ((t & (W - 1)) >= d) {
      v.re += re;
      v.im += im;
    }
  }
  if constexpr (NT > 64) {
    const int w = t >> 6;
    if ((t & 63) == 63) scr[w] = v;
    __syncthreads();
    cx<T> off = mk<T>(0, 0);
    for (int i = 0; i < w; ++i) off = off + scr[i];
    v = v + off;
    __syncthreads();
  }
  return v;
}

// In-place DST-I (unnormalised: X_p = sum_j x_j sin(pi p j/n)) of the LDS
// buffer buf holding x_0..x_{n-1} in natural order (x_0 ignored); on return
// buf holds X_0 = 0, X_1..X_{n-1}.  tw: n FFT twiddles followed by
// sin(pi j/n), j = 0..n/2, in the real parts.  NT = n/8 threads per transform,
// t in [0, NT).  The caller synchronises before (buf written) and reads after.
// Pre-processing of one pair (j, n - j), 0 < j < n/2, of the DST-I below: with
// s = sin(pi j/n), y_j = s (x_j + x_{n-j}) + (x_j - x_{n-j})/2 and
// y_{n-j} = s (x_j + x_{n-j}) - (x_j - x_{n-j})/2 (y_{n/2} = 2 x_{n/2}, y_0 = 0).
template <typename T>
__device__ __forceinline__ void dst1_pair(cx<T> a, cx<T> b, T sj, cx<T>& ya, cx<T>& yb) {
  const cx<T> sum = sj * (a + b), dif = (T)0.5 * (a - b);
  ya = sum + dif;
  yb = sum - dif;
}

// The DST-I below from its pre-processed input y (in buf): the length-n FFT
// and the post-processing, which stores op(p, X_p) for p = 1..n-1 (X_0 = 0
// stays).  Same calling rules as dst1.
template <typename T, int N, typename Op>
__device__ __forceinline__ void dst1_core_op(cx<T>* buf, const cx<T>* __restrict__ tw, cx<T>* scr, int t, Op op);

template <typename T, int N>
__device__ __forceinline__ void dst1_core(cx<T>* buf, const cx<T>* __restrict__ tw, cx<T>* scr, int t) {
  dst1_core_op<T, N>(buf, tw, scr, t, [](int, cx<T> v) { return v; });
}

template <typename T, int N>
__device__ __forceinline__ void dst1(cx<T>* buf, const cx<T>* __restrict__ tw, cx<T>* scr, int t) {
  constexpr int NT = N / 8;
  static_assert(N % 8 == 0, "n must be a multiple of 8");
  const cx<T>* sintab = tw + N;
  // pre-processing, one thread per pair (j, n - j), j = 1..n/2
  for (int j = 1 + t; j <= N / 2; j += NT) {
    const cx<T> a = buf[pidx<T>(j)];
    const T sj = sintab[j].re;
    if (j == N / 2) {
      buf[pidx<T>(j)] = (T)2 * sj * a;
    } else {
      cx<T> ya, yb;
      dst1_pair(a, buf[pidx<T>(N - j)], sj, ya, yb);
      buf[pidx<T>(j)] = ya;
      buf[pidx<T>(N - j)] = yb;
    }
  }
  if (t == 0) buf[pidx<T>(0)] = mk<T>(0, 0);
  __syncthreads();
  dst1_core<T, N>(buf, tw, scr, t);
}

template <typename T, int N, typename Op>
__device__ __forceinline__ void dst1_core_op(cx<T>* buf, const cx<T>* __restrict__ tw, cx<T>* scr, int t, Op op) {
  constexpr int NT = N / 8;
  fft<T, N>(buf, tw, t);
  // post-processing: thread t owns k = 4t+1 .. 4t+4 (k <= n/2 - 1)
  const cx<T> f0 = buf[pidx<T>(0)];
  cx<T> ev[4], od[4];
  cx<T> run = mk<T>(0, 0);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int k = 4 * t + 1 + i;
    if (k < N / 2) {
      const cx<T> fk = buf[pidx<T>(k)], fn = buf[pidx<T>(N - k)];
      ev[i] = (T)0.5 * mul_i(fk - fn);
      run = run + (T)0.5 * (fk + fn);
    }
    od[i] = run;
  }
  cx<T> incl = group_scan<T, NT>(run, scr, t);
  const cx<T> base = (T)0.5 * f0 + (incl - run);  // X_1 plus the sums of earlier threads
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int k = 4 * t + 1 + i;
    if (k < N / 2) {
      buf[pidx<T>(2 * k)] = op(2 * k, ev[i]);
      buf[pidx<T>(2 * k + 1)] = op(2 * k + 1, base + od[i]);
    }
  }
  if (t == 0) {
    buf[pidx<T>(0)] = mk<T>(0, 0);
    buf[pidx<T>(1)] = op(1, (T)0.5 * f0);
  }
  __syncthreads();
}

// Orthonormal DST-I value p from dst1 output.
template <typename T>
__device__ __forceinline__ cx<T> dst_val(const cx<T>* buf, int p, T scale) {
  return scale * buf[pidx<T>(p)];
}
