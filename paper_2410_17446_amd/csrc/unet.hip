// U-Net for GMRES initial guesses: forward, backward, Adam, and the feature
// packing that connects it to a propagation step (declared in hp_unet.h).
//
// Architecture: L levels, C * 2^l channels at level l; two 3x3 convolutions
// with ReLU per level on the way down and on the way up; 2x2 average pooling
// down; nearest-neighbour upsampling and channel concatenation [upsampled,
// skip] up; a 1x1 output convolution.  Activations float32 NCHW [B][C][H][W],
// weights float32, float32 accumulation.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "../../include/hp_unet.h"
#include "cplx.hpp"

namespace {

constexpr int TILE = 16;  // 16 x 16 output pixels per workgroup
constexpr int COB = 8;    // output channels per workgroup

__device__ __forceinline__ double wsum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}
__device__ __forceinline__ float wsumf(float v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// y[b][co](p) = sum_ci sum_k w(co, ci, k) x[b][ci](p + d_k) + bias[co], zero padding,
// d_k = (k / 3 - 1, k % 3 - 1).  The weight of (co, ci, k) is read at
// co * wso + ci * wsi + (flip ? 8 - k : k): the forward pass uses wso = Cin*9,
// wsi = 9; the data gradient runs the same loop with the channel roles swapped
// and the taps flipped.
__global__ __launch_bounds__(256) void k_conv3(const float* __restrict__ x, const float* __restrict__ w,
                                               const float* __restrict__ bias, float* __restrict__ y, int cin,
                                               int cout, int H, int W, int wso, int wsi, int flip, int relu) {
  __shared__ float tile[(TILE + 2) * (TILE + 2)];
  __shared__ float ws[COB * 9];
  const int tx = threadIdx.x % TILE, ty = threadIdx.x / TILE;
  const int ntx = (W + TILE - 1) / TILE;
  const int x0 = (blockIdx.x % ntx) * TILE, y0 = (blockIdx.x / ntx) * TILE;
  const int co0 = blockIdx.y * COB;
  const int b = blockIdx.z;
  const size_t plane = (size_t)H * W;
  float acc[COB];
#pragma unroll
  for (int c = 0; c < COB; ++c) acc[c] = 0.f;
  for (int ci = 0; ci < cin; ++ci) {
    const float* xp = x + ((size_t)b * cin + ci) * plane;
    __syncthreads();
    for (int e = threadIdx.x; e < (TILE + 2) * (TILE + 2); e += 256) {
      const int yy = y0 + e / (TILE + 2) - 1, xx = x0 + e % (TILE + 2) - 1;
      tile[e] = (yy >= 0 && yy < H && xx >= 0 && xx < W) ? xp[(size_t)yy * W + xx] : 0.f;
    }
    if (threadIdx.x < COB * 9) {
      const int c = threadIdx.x / 9, k = threadIdx.x % 9;
      const int co = co0 + c;
      ws[threadIdx.x] = (co < cout) ? w[(size_t)co * wso + (size_t)ci * wsi + (flip ? 8 - k : k)] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const float v = tile[(ty + k / 3) * (TILE + 2) + tx + k % 3];
#pragma unroll
      for (int c = 0; c < COB; ++c) acc[c] += ws[c * 9 + k] * v;
    }
  }
  const int oy = y0 + ty, ox = x0 + tx;
  if (oy >= H || ox >= W) return;
#pragma unroll
  for (int c = 0; c < COB; ++c) {
    const int co = co0 + c;
    if (co >= cout) break;
    float v = acc[c] + (bias ? bias[co] : 0.f);
    if (relu) v = fmaxf(v, 0.f);
    y[((size_t)b * cout + co) * plane + (size_t)oy * W + ox] = v;
  }
}

// ---------------------------------------------------------------- BF16 MFMA 3x3 convolution
//
// The same convolution as an implicit GEMM on the matrix cores:
// D[co][pixel] = sum over (tap, ci) of W(co, ci, tap) X[ci](pixel + d_tap), the
// reduction taken 32 input channels at a time per tap by
// v_mfma_f32_16x16x32_bf16 (bf16 operands, float32 accumulation).  Lane l of a
// wave holds, for A (16 x 32), row l % 16 and reduction indices 8 (l / 16) ..
// + 7; for B (32 x 16), column l % 16 and the same reduction indices; the 16 x
// 16 float result has column l % 16 and rows 4 (l / 16) .. + 3.
//
// Operands are prepared once per convolution: the input as bf16 in channel
// chunks of 32, channel-innermost ([b][chunk][y][x][32], 64 bytes a pixel), and
// the weights as bf16 A fragments in lane order ([co tile][chunk][tap][block]
// [lane][8]), so a wave reads each fragment as one contiguous 1 KB block.
//
// A workgroup (4 waves) computes 64 output channels x an 8 x 16 pixel tile:
// wave w takes the channel blocks 2 (w % 2), + 1 and the pixel rows 4 (w / 2)
// .. + 3 (one 16-pixel row per MFMA column block): 8 accumulators, 2 A and 4 B
// fragments per tap.  The halo patch (10 x 18 pixels) of each chunk goes
// through LDS with 40-element pixel rows (80 bytes: the 16 lanes of one
// reduction group read disjoint banks).
namespace mf {
constexpr int TH = 8, TWD = 16;           // pixel tile
constexpr int CO = 64, CK = 32, CS = 40;  // channels per tile, per chunk, LDS pixel stride
constexpr int CB = CO / 16;               // 16-channel blocks per tile
constexpr int HX = TH + 2, HY = TWD + 2;  // halo rows, columns
}  // namespace mf

typedef float mf_f4 __attribute__((ext_vector_type(4)));
typedef __bf16 mf_b8 __attribute__((ext_vector_type(8)));

// x [B][C][H][W] float -> xb [B][ceil(C/32)][H][W][32] bf16 (channels past C are 0)
__global__ void k_to_bf16c(const float* __restrict__ x, __bf16* __restrict__ xb, int B, int C, int H, int W) {
  const int nch = (C + mf::CK - 1) / mf::CK;
  const size_t plane = (size_t)H * W;
  const size_t n = (size_t)B * nch * plane;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const size_t p = e % plane;
    const int ch = (int)((e / plane) % nch), b = (int)(e / (plane * nch));
    mf_b8 v[4];
#pragma unroll
    for (int c = 0; c < mf::CK; ++c) {
      const int ci = ch * mf::CK + c;
      v[c / 8][c % 8] = (__bf16)(ci < C ? x[((size_t)b * C + ci) * plane + p] : 0.f);
    }
    mf_b8* o = reinterpret_cast<mf_b8*>(xb + e * mf::CK);
#pragma unroll
    for (int q = 0; q < 4; ++q) o[q] = v[q];
  }
}

// A fragments of the weights: wp[(((ct * nch + ch) * 9 + tap) * CB + blk) * 64 + lane][j] =
// w(co, ci, tap) with co = 64 ct + 16 blk + lane % 16, ci = 32 ch + 8 (lane / 16) + j, the
// weight of (co, ci, tap) read at co * wso + ci * wsi + (flip ? 8 - tap : tap); 0 outside.
__global__ void k_pack_w(const float* __restrict__ w, __bf16* __restrict__ wp, int cin, int cout, int wso, int wsi,
                         int flip) {
  const int nch = (cin + mf::CK - 1) / mf::CK, nct = (cout + mf::CO - 1) / mf::CO;
  const size_t n = (size_t)nct * nch * 9 * mf::CB * 64 * 8;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(e % 8), lane = (int)((e / 8) % 64), blk = (int)((e / 512) % mf::CB);
    const size_t r = e / (512 * mf::CB);
    const int tap = (int)(r % 9), ch = (int)((r / 9) % nch), ct = (int)(r / (9 * (size_t)nch));
    const int co = ct * mf::CO + blk * 16 + lane % 16, ci = ch * mf::CK + (lane / 16) * 8 + j;
    float v = 0.f;
    if (co < cout && ci < cin) v = w[(size_t)co * wso + (size_t)ci * wsi + (flip ? 8 - tap : tap)];
    wp[e] = (__bf16)v;
  }
}

__global__ __launch_bounds__(256) void k_conv3_mfma(const __bf16* __restrict__ xb, const __bf16* __restrict__ wp,
                                                    const float* __restrict__ bias, float* __restrict__ y, int cin,
                                                    int cout, int H, int W, int relu) {
  using namespace mf;
  __shared__ __attribute__((aligned(16))) __bf16 xs[HX * HY * CS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ntx = (W + TWD - 1) / TWD;
  const int x0 = (blockIdx.x % ntx) * TWD, y0 = (blockIdx.x / ntx) * TH;
  const int ct = blockIdx.y, b = blockIdx.z;
  const int nch = (cin + CK - 1) / CK;
  const size_t plane = (size_t)H * W;
  const int cb0 = (wave & 1) * 2;  // first channel block of this wave
  const int r0 = (wave >> 1) * 4;  // first pixel row of this wave
  const int col = lane & 15, kg = lane >> 4;
  mf_f4 acc[2][4];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[c][r] = mf_f4{0.f, 0.f, 0.f, 0.f};
  const mf_b8* wf = reinterpret_cast<const mf_b8*>(wp) + (size_t)ct * nch * 9 * CB * 64;
  for (int ch = 0; ch < nch; ++ch) {
    __syncthreads();
    // halo patch of this chunk: 4 x 16 bytes per pixel
    const mf_b8* src = reinterpret_cast<const mf_b8*>(xb) + ((size_t)b * nch + ch) * plane * 4;
    for (int e = tid; e < HX * HY * 4; e += 256) {
      const int q = e & 3, r = e >> 2;
      const int gy = y0 + r / HY - 1, gx = x0 + r % HY - 1;
      mf_b8 v;
      if (gy >= 0 && gy < H && gx >= 0 && gx < W)
        v = src[((size_t)gy * W + gx) * 4 + q];
      else
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = (__bf16)0.f;
      *reinterpret_cast<mf_b8*>(&xs[r * CS + q * 8]) = v;
    }
    __syncthreads();
    const mf_b8* wc = wf + (size_t)ch * 9 * CB * 64;
#pragma unroll 3
    for (int tap = 0; tap < 9; ++tap) {
      const int dy = tap / 3, dx = tap % 3;
      const mf_b8 a0 = wc[(tap * CB + cb0) * 64 + lane];
      const mf_b8 a1 = wc[(tap * CB + cb0 + 1) * 64 + lane];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const mf_b8 bv = *reinterpret_cast<const mf_b8*>(&xs[((r0 + r + dy) * HY + col + dx) * CS + kg * 8]);
        acc[0][r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bv, acc[0][r], 0, 0, 0);
        acc[1][r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bv, acc[1][r], 0, 0, 0);
      }
    }
  }
  // D: column = pixel x0 + col of row y0 + r0 + r; rows = channels 16 (cb0 + c) + 4 kg + i
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int oy = y0 + r0 + r, ox = x0 + col;
    if (oy >= H || ox >= W) continue;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int co = ct * CO + (cb0 + c) * 16 + kg * 4 + i;
        if (co >= cout) continue;
        float v = acc[c][r][i] + (bias ? bias[co] : 0.f);
        if (relu) v = fmaxf(v, 0.f);
        y[((size_t)b * cout + co) * plane + (size_t)oy * W + ox] = v;
      }
  }
}

// dW[co][ci][k] = sum_b sum_p dy[b][co](p) x[b][ci](p + d_k): one workgroup per (co, ci).
__global__ __launch_bounds__(256) void k_conv3_wgrad(const float* __restrict__ x, const float* __restrict__ dy,
                                                     float* __restrict__ dw, int B, int cin, int cout, int H, int W) {
  __shared__ float red[9][4];
  const int co = blockIdx.x / cin, ci = blockIdx.x % cin;
  const size_t plane = (size_t)H * W;
  float acc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = 0.f;
  for (int b = 0; b < B; ++b) {
    const float* d = dy + ((size_t)b * cout + co) * plane;
    const float* xp = x + ((size_t)b * cin + ci) * plane;
    for (size_t p = threadIdx.x; p < plane; p += 256) {
      const int yy = (int)(p / W), xx = (int)(p % W);
      const float g = d[p];
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const int sy = yy + k / 3 - 1, sx = xx + k % 3 - 1;
        if (sy >= 0 && sy < H && sx >= 0 && sx < W) acc[k] += g * xp[(size_t)sy * W + sx];
      }
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const float v = wsumf(acc[k]);
    if (lane == 0) red[k][wv] = v;
  }
  __syncthreads();
  if (threadIdx.x < 9) {
    const int k = threadIdx.x;
    dw[((size_t)co * cin + ci) * 9 + k] = red[k][0] + red[k][1] + red[k][2] + red[k][3];
  }
}

// Weight gradient on the matrix cores.  The contraction runs over pixels: one
// v_mfma_f32_16x16x32_bf16 takes 32 pixels of one image row (lane group kg
// holds the 8 consecutive pixels 8 kg .. 8 kg + 7 of the segment) for 16 output
// channels (A = dy, row = lane % 16) against 16 input channels (B = x moved by
// the tap, column = lane % 16).  A workgroup owns 32 output x 16 input
// channels and a contiguous share of the row segments; its four waves take
// every fourth segment (the next one's operands loaded while the current one
// is multiplied), sum through LDS in wave order, and the workgroup writes
// part[split][co][ci][tap]; workgroups of the first input-channel block also
// sum dy for the bias gradient into part[split][cout * cin * 9 + co].
// k_wgrad_sum adds the splits in a fixed order, so the result does not depend
// on scheduling.
namespace wgm {
constexpr int CO = 32, CI = 16, SEG = 32;
constexpr int SUM_WAVES = 16;  // waves per output chunk in k_wgrad_sum
}

// v[j] = p[j] for j < valid, else 0; vec: p is 16-byte aligned (two float4 loads when valid >= 8)
__device__ __forceinline__ void ld8(const float* __restrict__ p, int vec, int valid, float* v) {
  if (vec && valid >= 8) {
    const float4 a = *reinterpret_cast<const float4*>(p), b = *reinterpret_cast<const float4*>(p + 4);
    v[0] = a.x, v[1] = a.y, v[2] = a.z, v[3] = a.w, v[4] = b.x, v[5] = b.y, v[6] = b.z, v[7] = b.w;
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = j < valid ? p[j] : 0.f;
  }
}

// Operands of one row segment as loaded: dy of the lane's two output channels
// (8 pixels each) and x of its input channel on the three rows around, pixels
// px - 1 .. px + 8.
struct WgSeg {
  float a[2][8];
  float b[3][10];
};

__device__ __forceinline__ void wg_load(WgSeg& g, const float* __restrict__ x, const float* __restrict__ dy, long q,
                                        int ws, int B, int cin, int cout, int H, int W, int co0, int ci, int l16, int kg,
                                        int vec) {
  const size_t plane = (size_t)H * W;
  const int xs = (int)(q % ws);
  const long r = q / ws;
  const int yy = (int)(r % H), b = (int)(r / H);
  const int px = xs * wgm::SEG + kg * 8;
  const int nv = W - px;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int co = co0 + 16 * c + l16;
    const bool cv = co < cout;
    ld8(dy + ((size_t)b * cout + (cv ? co : 0)) * plane + (size_t)yy * W + px, vec, cv ? nv : 0, g.a[c]);
  }
#pragma unroll
  for (int ky = 0; ky < 3; ++ky) {
    const int sy = yy + ky - 1;
    const bool rv = ci < cin && sy >= 0 && sy < H;
    const float* s = x + ((size_t)b * cin + (rv ? ci : 0)) * plane + (size_t)(rv ? sy : 0) * W;
    ld8(s + px, vec, rv ? nv : 0, g.b[ky] + 1);
    g.b[ky][0] = (rv && px >= 1 && px - 1 < W) ? s[px - 1] : 0.f;
    g.b[ky][9] = (rv && px + 8 < W) ? s[px + 8] : 0.f;
  }
}

__global__ __launch_bounds__(256) void k_conv3_wgrad_mfma(const float* __restrict__ x, const float* __restrict__ dy,
                                                          float* __restrict__ part, int B, int cin, int cout, int H,
                                                          int W, int nsplit, int vec) {
  __shared__ float red[2 * 9 * 256];
  __shared__ float bred[4][2][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, kg = lane >> 4;
  const int co0 = blockIdx.x * wgm::CO, ci0 = blockIdx.y * wgm::CI, split = blockIdx.z;
  const int ws = (W + wgm::SEG - 1) / wgm::SEG;
  const long nseg = (long)B * H * ws;
  const long q0 = nseg * split / nsplit, q1 = nseg * (split + 1) / nsplit;
  const int ci = ci0 + l16;
  const size_t stride = (size_t)cout * cin * 9 + cout;  // floats per split
  mf_f4 acc[2][9];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[c][t] = mf_f4{0.f, 0.f, 0.f, 0.f};
  float bs[2] = {0.f, 0.f};
  WgSeg cur;
  long q = q0 + wave;
  if (q < q1) wg_load(cur, x, dy, q, ws, B, cin, cout, H, W, co0, ci, l16, kg, vec);
  for (; q < q1; q += 4) {
    WgSeg nxt;
    if (q + 4 < q1) wg_load(nxt, x, dy, q + 4, ws, B, cin, cout, H, W, co0, ci, l16, kg, vec);
    mf_b8 a[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        a[c][j] = (__bf16)cur.a[c][j];
        bs[c] += cur.a[c][j];
      }
    }
#pragma unroll
    for (int ky = 0; ky < 3; ++ky)
#pragma unroll
      for (int kx = 0; kx < 3; ++kx) {
        mf_b8 bv;
#pragma unroll
        for (int j = 0; j < 8; ++j) bv[j] = (__bf16)cur.b[ky][j + kx];
        acc[0][ky * 3 + kx] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], bv, acc[0][ky * 3 + kx], 0, 0, 0);
        acc[1][ky * 3 + kx] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], bv, acc[1][ky * 3 + kx], 0, 0, 0);
      }
    cur = nxt;
  }
  // D lane layout: column (input channel) lane % 16, rows (output channels) 4 kg + i
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int t = 0; t < 9; ++t)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            float& d = red[((c * 9 + t) * 16 + kg * 4 + i) * 16 + l16];
            d = (w == 0 ? 0.f : d) + acc[c][t][i];
          }
    }
    __syncthreads();
  }
  float* out = part + (size_t)split * stride;
  for (int e = threadIdx.x; e < 2 * 9 * 256; e += 256) {
    const int cil = e & 15, col = (e >> 4) & 15, t = (e >> 8) % 9, c = e / (9 * 256);
    const int co = co0 + 16 * c + col, cc = ci0 + cil;
    if (co < cout && cc < cin) out[((size_t)co * cin + cc) * 9 + t] = red[e];
  }
  if (blockIdx.y == 0) {
    bred[wave][0][lane] = bs[0];
    bred[wave][1][lane] = bs[1];
    __syncthreads();
    if (threadIdx.x < 32) {
      const int c = threadIdx.x >> 4, col = threadIdx.x & 15, co = co0 + threadIdx.x;
      float a = 0.f;
      for (int w = 0; w < 4; ++w)
        for (int g = 0; g < 4; ++g) a += bred[w][c][g * 16 + col];
      if (co < cout) out[(size_t)cout * cin * 9 + co] = a;
    }
  }
}

// dw[e] = sum over splits of part[s][e], e < n: a workgroup per 64 outputs,
// wave w sums the splits w, w + SUM_WAVES, ... in order, then the waves' sums
// are added in wave order.
__global__ __launch_bounds__(64 * wgm::SUM_WAVES) void k_wgrad_sum(const float* __restrict__ part,
                                                                  float* __restrict__ dw, size_t n, int nsplit) {
  __shared__ float red[wgm::SUM_WAVES][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const size_t e = (size_t)blockIdx.x * 64 + lane;
  float a = 0.f;
  if (e < n)
    for (int s = wave; s < nsplit; s += wgm::SUM_WAVES) a += part[(size_t)s * n + e];
  red[wave][lane] = a;
  __syncthreads();
  if (wave == 0 && e < n) {
    float t = 0.f;
    for (int w = 0; w < wgm::SUM_WAVES; ++w) t += red[w][lane];
    dw[e] = t;
  }
}

// db[c] = sum_b sum_p dy[b][c](p)
__global__ __launch_bounds__(256) void k_bias_grad(const float* __restrict__ dy, float* __restrict__ db, int B, int C,
                                                   size_t plane) {
  __shared__ float red[4];
  const int c = blockIdx.x;
  float acc = 0.f;
  for (int b = 0; b < B; ++b) {
    const float* d = dy + ((size_t)b * C + c) * plane;
    for (size_t p = threadIdx.x; p < plane; p += 256) acc += d[p];
  }
  acc = wsumf(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) db[c] = red[0] + red[1] + red[2] + red[3];
}

// 1x1 convolution y[b][co](p) = sum_ci w[co][ci] x[b][ci](p) (+ bias); transpose:
// y[b][ci](p) = sum_co w[co][ci] x[b][co](p) (the data gradient).
__global__ __launch_bounds__(256) void k_conv1(const float* __restrict__ x, const float* __restrict__ w,
                                               const float* __restrict__ bias, float* __restrict__ y, int B, int cin,
                                               int cout, size_t plane, int transpose) {
  const size_t n = (size_t)B * plane;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const int b = (int)(i / plane);
    const size_t p = i % plane;
    for (int co = 0; co < cout; ++co) {
      float acc = bias ? bias[co] : 0.f;
      for (int ci = 0; ci < cin; ++ci)
        acc += (transpose ? w[(size_t)ci * cout + co] : w[(size_t)co * cin + ci]) *
               x[((size_t)b * cin + ci) * plane + p];
      y[((size_t)b * cout + co) * plane + p] = acc;
    }
  }
}

// Split form of the 1x1 weight and bias gradients: output e < cout * cin is
// dW1[e / cin][e % cin], e = cout * cin + co is db[co]; split s sums the pixels
// i = (b, p) of its contiguous share of B * plane into part[s][e] (summed over
// the splits by k_wgrad_sum).
__global__ __launch_bounds__(256) void k_conv1_wgrad_split(const float* __restrict__ x, const float* __restrict__ dy,
                                                           float* __restrict__ part, int B, int cin, int cout,
                                                           unsigned plane, int nsplit) {
  __shared__ float red[4];
  const int e = blockIdx.x, s = blockIdx.y;
  const int n = cout * (cin + 1);
  const bool bias = e >= cout * cin;
  const int co = bias ? e - cout * cin : e / cin, ci = bias ? 0 : e % cin;
  const unsigned total = (unsigned)B * plane;
  const unsigned i0 = (unsigned)((unsigned long long)total * s / nsplit);
  const unsigned i1 = (unsigned)((unsigned long long)total * (s + 1) / nsplit);
  float acc = 0.f;
  for (unsigned i = i0 + threadIdx.x; i < i1; i += 256) {
    const unsigned b = i / plane, p = i - b * plane;
    const float d = dy[((size_t)b * cout + co) * plane + p];
    acc += bias ? d : d * x[((size_t)b * cin + ci) * plane + p];
  }
  acc = wsumf(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[(size_t)s * n + e] = red[0] + red[1] + red[2] + red[3];
}

// dy = 0 where the ReLU output y is 0 (the derivative at 0 is taken as 0)
__global__ void k_relu_bwd(const float* __restrict__ y, float* __restrict__ dy, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    if (y[i] <= 0.f) dy[i] = 0.f;
}

// 2x2 average pooling of [planes][H][W] -> [planes][H/2][W/2], and its adjoint
__global__ void k_pool(const float* __restrict__ x, float* __restrict__ y, size_t planes, int H, int W) {
  const int h = H / 2, w = W / 2;
  const size_t n = planes * h * w;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const size_t pl = i / ((size_t)h * w);
    const int r = (int)(i % ((size_t)h * w));
    const int yy = r / w, xx = r % w;
    const float* s = x + pl * H * W + (size_t)(2 * yy) * W + 2 * xx;
    y[i] = 0.25f * (s[0] + s[1] + s[W] + s[W + 1]);
  }
}
__global__ void k_pool_bwd(const float* __restrict__ dy, float* __restrict__ dx, size_t planes, int H, int W) {
  const size_t n = planes * H * W;
  const int w = W / 2;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const size_t pl = i / ((size_t)H * W);
    const int r = (int)(i % ((size_t)H * W));
    const int yy = r / W, xx = r % W;
    dx[i] = 0.25f * dy[pl * (H / 2) * w + (size_t)(yy / 2) * w + xx / 2];
  }
}
// nearest-neighbour 2x upsampling of [B][C][h][w] into channels [c0, c0+C) of
// [B][Ctot][2h][2w], and its adjoint (sum over each 2x2 block)
__global__ void k_up(const float* __restrict__ x, float* __restrict__ y, int B, int C, int Ctot, int c0, int h,
                     int w) {
  const int H = 2 * h, W = 2 * w;
  const size_t n = (size_t)B * C * H * W;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const int xx = (int)(i % W), yy = (int)((i / W) % H);
    const size_t bc = i / ((size_t)H * W);
    const int c = (int)(bc % C), b = (int)(bc / C);
    y[(((size_t)b * Ctot + c0 + c) * H + yy) * W + xx] = x[(((size_t)b * C + c) * h + yy / 2) * w + xx / 2];
  }
}
__global__ void k_up_bwd(const float* __restrict__ dy, float* __restrict__ dx, int B, int C, int Ctot, int c0, int h,
                         int w) {
  const int H = 2 * h, W = 2 * w;
  const size_t n = (size_t)B * C * h * w;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const int xx = (int)(i % w), yy = (int)((i / w) % h);
    const size_t bc = i / ((size_t)h * w);
    const int c = (int)(bc % C), b = (int)(bc / C);
    const float* s = dy + (((size_t)b * Ctot + c0 + c) * H + 2 * yy) * W + 2 * xx;
    dx[i] = s[0] + s[1] + s[W] + s[W + 1];
  }
}
// small [B][C][P] <-> channels [c0, c0+C) of big [B][Ctot][P]; dir 0: small -> big
__global__ void k_chcopy(float* __restrict__ big, float* __restrict__ small, int B, int C, int Ctot, int c0, size_t P,
                         int dir) {
  const size_t n = (size_t)B * C * P;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const size_t p = i % P;
    const size_t bc = i / P;
    const int c = (int)(bc % C), b = (int)(bc / C);
    const size_t j = ((size_t)b * Ctot + c0 + c) * P + p;
    if (dir == 0)
      big[j] = small[i];
    else
      small[i] = big[j];
  }
}
__global__ void k_add(float* __restrict__ a, const float* __restrict__ b, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    a[i] += b[i];
}
// loss = mean (y - t)^2: d = 2 (y - t) / n and per-block partial sums of (y - t)^2
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ y, const float* __restrict__ t,
                                             float* __restrict__ d, double* __restrict__ part, size_t n) {
  __shared__ double red[4];
  double acc = 0.0;
  const float sc = (float)(2.0 / (double)n);
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const float e = y[i] - t[i];
    acc += (double)e * e;
    d[i] = sc * e;
  }
  acc = wsum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}
// Adam (Kingma & Ba 2015, Algorithm 1) with bias corrections c1 = 1 - b1^t, c2 = 1 - b2^t
// (omb1 = 1 - b1 and omb2 = 1 - b2 are rounded from double, not formed in float)
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       size_t n, float lr, float b1, float b2, float omb1, float omb2, float c1, float c2, float eps) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + omb1 * gi;
    const float vi = b2 * v[i] + omb2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// ---------------------------------------------------------------- guess features

__device__ __forceinline__ double medium_v(const double* n2, size_t idx, int i, int j, int nx, int ny, double n0,
                                           int W) {
  const int d = min(min(i, ny - i), min(j, nx - j));
  return d > W ? (n2[idx] - n0 * n0) / (n0 * n0) : 0.0;
}

// scal[0] = rms w, scal[1] = rms V (interior nodes), scal[2 + b] = rms y_b; each
// floored at 1e-300.  Block 0: w and V; block 1 + b: y_b.
__global__ __launch_bounds__(256) void k_guess_stats(const c128* __restrict__ w, const c128* __restrict__ y,
                                                     const double* __restrict__ n2, double n0, int Wl, int nx,
                                                     int ny, int ncomp, double* __restrict__ scal) {
  __shared__ double red[2][4];
  const size_t fsz = (size_t)nx * ny, fn = fsz * ncomp;
  const double cnt = (double)(nx - 1) * (ny - 1);
  double a = 0.0, v = 0.0;
  if (blockIdx.x == 0) {
    for (size_t idx = threadIdx.x; idx < fsz; idx += 256) {
      const int i = (int)(idx / nx), j = (int)(idx % nx);
      if (i == 0 || j == 0) continue;
      for (int c = 0; c < ncomp; ++c) a += abs2(w[c * fsz + idx]);
      const double vv = medium_v(n2, idx, i, j, nx, ny, n0, Wl);
      v += vv * vv;
    }
  } else {
    const c128* yb = y + (size_t)(blockIdx.x - 1) * fn;
    for (size_t idx = threadIdx.x; idx < fn; idx += 256) {
      const size_t q = idx % fsz;
      if (q / nx == 0 || q % nx == 0) continue;
      a += abs2(yb[idx]);
    }
  }
  a = wsum(a);
  v = wsum(v);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = a;
    red[1][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double sa = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    const double sv = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    if (blockIdx.x == 0) {
      scal[0] = fmax(sqrt(sa / (cnt * ncomp)), 1e-300);
      scal[1] = fmax(sqrt(sv / cnt), 1e-300);
    } else {
      scal[1 + blockIdx.x] = fmax(sqrt(sa / (cnt * ncomp)), 1e-300);
    }
  }
}

// Input planes of sample b, [B][4 ncomp + 3][ny][nx] float: Re, Im of each
// component of w / rms w; Re, Im of each component of y_b / rms y_b; V / rms V;
// the two pole features of sample b (constant planes).  Row 0 and column 0 are 0.
__global__ void k_guess_pack(const c128* __restrict__ w, const c128* __restrict__ y, const double* __restrict__ n2,
                             const double* __restrict__ scal, const double* __restrict__ feat, double n0, int Wl,
                             int nx, int ny, int ncomp, int B, float* __restrict__ out) {
  const size_t fsz = (size_t)nx * ny, fn = fsz * ncomp;
  const int cin = 4 * ncomp + 3;
  const size_t n = (size_t)B * fsz;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const int b = (int)(e / fsz);
    const size_t idx = e % fsz;
    const int i = (int)(idx / nx), j = (int)(idx % nx);
    const bool in = i > 0 && j > 0;
    float* o = out + (size_t)b * cin * fsz + idx;
    const double iw = 1.0 / scal[0], iy = 1.0 / scal[2 + b], iv = 1.0 / scal[1];
    int ch = 0;
    for (int c = 0; c < ncomp; ++c) {
      const c128 v = in ? w[c * fsz + idx] : mk(0.0, 0.0);
      o[(ch++) * fsz] = (float)(v.re * iw);
      o[(ch++) * fsz] = (float)(v.im * iw);
    }
    for (int c = 0; c < ncomp; ++c) {
      const c128 v = in ? y[(size_t)b * fn + c * fsz + idx] : mk(0.0, 0.0);
      o[(ch++) * fsz] = (float)(v.re * iy);
      o[(ch++) * fsz] = (float)(v.im * iy);
    }
    o[(ch++) * fsz] = in ? (float)(medium_v(n2, idx, i, j, nx, ny, n0, Wl) * iv) : 0.f;
    o[(ch++) * fsz] = in ? (float)feat[2 * b] : 0.f;
    o[(ch++) * fsz] = in ? (float)feat[2 * b + 1] : 0.f;
  }
}

// t_b = w + sigma_b net_b, sigma_b = rms y_b * rms V; zero on row 0 and column 0.
__global__ void k_guess_unpack(const c128* __restrict__ w, const float* __restrict__ net,
                               const double* __restrict__ scal, int nx, int ny, int ncomp, int B,
                               c128* __restrict__ t) {
  const size_t fsz = (size_t)nx * ny, fn = fsz * ncomp;
  const size_t n = (size_t)B * fn;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const int b = (int)(e / fn);
    const size_t r = e % fn;
    const int c = (int)(r / fsz);
    const size_t idx = r % fsz;
    const int i = (int)(idx / nx), j = (int)(idx % nx);
    c128 v = mk(0.0, 0.0);
    if (i > 0 && j > 0) {
      const double sg = scal[2 + b] * scal[1];
      const float* o = net + ((size_t)b * 2 * ncomp + 2 * c) * fsz + idx;
      v = w[c * fsz + idx] + mk(sg * (double)o[0], sg * (double)o[fsz]);
    }
    t[e] = v;
  }
}

// Training target of sample b: -(P x_b) / sigma_b as [B][2 ncomp][ny][nx] float.
__global__ void k_guess_target(const c128* __restrict__ px, const double* __restrict__ scal, int nx, int ny,
                               int ncomp, int B, float* __restrict__ out) {
  const size_t fsz = (size_t)nx * ny, fn = fsz * ncomp;
  const size_t n = (size_t)B * fn;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const int b = (int)(e / fn);
    const size_t r = e % fn;
    const int c = (int)(r / fsz);
    const size_t idx = r % fsz;
    const double is = -1.0 / (scal[2 + b] * scal[1]);
    const c128 v = px[e];
    float* o = out + ((size_t)b * 2 * ncomp + 2 * c) * fsz + idx;
    o[0] = (float)(v.re * is);
    o[fsz] = (float)(v.im * is);
  }
}

int eblocks(size_t n) { return (int)std::min<size_t>((n + 255) / 256, 8192); }

}  // namespace

// ---------------------------------------------------------------------- network object

struct hp_unet_s {
  int levels = 4, base = 32, cin = 7, cout = 2;
  bool bf16 = false;  // 3x3 convolutions (forward, data gradient) on bf16 matrix cores
  struct Conv {
    int ci, co, k;  // k = 3 or 1
    size_t w, b;    // offsets (floats) of weights [co][ci][k][k] and bias [co]
  };
  std::vector<Conv> enc_a, enc_b, dec_a, dec_b;
  Conv out{};
  size_t nparam = 0;
  float *P = nullptr, *G = nullptr, *M = nullptr, *V = nullptr;  // params, grads, Adam moments
  long step = 0;
  // activations of the last forward (B, H, W)
  int B = 0, H = 0, W = 0;
  std::vector<float*> enc1, enc2, pool, up, dec1, dec2, dskip;
  float *y = nullptr, *dy = nullptr, *ga = nullptr, *gb = nullptr;
  __bf16* xb = nullptr;   // bf16 channel-chunked copy of a convolution's input
  __bf16* wpk = nullptr;  // bf16 weight fragments of one convolution
  float* wgpart = nullptr;  // per-split partial weight gradients (matrix-core path)
  std::vector<float*> owned;
  double* part = nullptr;    // device partial sums (loss)
  double* part_h = nullptr;  // pinned
  double* feat = nullptr;    // device pole features [2 * 64]
  double* feat_h = nullptr;  // pinned
  hipStream_t stream = nullptr;
  std::string err;
};

namespace {

thread_local std::string g_err;

int ufail(hp_unet n, int code, const std::string& msg) {
  (n ? n->err : g_err) = msg;
  return code;
}

int ch(const hp_unet_s* n, int l) { return n->base << l; }

// Splits of the pixel contraction in the matrix-core weight gradient: about
// 1024 workgroups in all, each with at least 16 row segments (four per wave).
int wgrad_splits(int B, int H, int W, int cin, int cout) {
  const long nseg = (long)B * H * ((W + wgm::SEG - 1) / wgm::SEG);
  const long blocks = (long)((cout + wgm::CO - 1) / wgm::CO) * ((cin + wgm::CI - 1) / wgm::CI);
  return (int)std::max(1L, std::min(nseg / 16, 1024 / blocks));
}

// Splits of the 1x1 weight and bias gradients: about 1024 workgroups, each
// with at least 4096 pixels.
int conv1_splits(int B, int H, int W, int cin, int cout) {
  const long pix = (long)B * H * W;
  return (int)std::max(1L, std::min(pix / 4096, 1024L / ((long)cout * (cin + 1))));
}

void unet_layout(hp_unet n) {
  size_t off = 0;
  auto conv = [&](int ci, int co, int k) {
    hp_unet_s::Conv c{ci, co, k, off, 0};
    off += (size_t)ci * co * k * k;
    c.b = off;
    off += co;
    return c;
  };
  const int L = n->levels;
  for (int l = 0; l < L; ++l) {
    n->enc_a.push_back(conv(l == 0 ? n->cin : ch(n, l - 1), ch(n, l), 3));
    n->enc_b.push_back(conv(ch(n, l), ch(n, l), 3));
  }
  for (int l = 0; l < L - 1; ++l) {
    n->dec_a.push_back(conv(ch(n, l + 1) + ch(n, l), ch(n, l), 3));
    n->dec_b.push_back(conv(ch(n, l), ch(n, l), 3));
  }
  n->out = conv(ch(n, 0), n->cout, 1);
  n->nparam = off;
}

void free_acts(hp_unet n) {
  for (float* p : n->owned) (void)hipFree(p);
  n->owned.clear();
  for (auto* v : {&n->enc1, &n->enc2, &n->pool, &n->up, &n->dec1, &n->dec2, &n->dskip}) v->clear();
  n->y = n->dy = n->ga = n->gb = nullptr;
  n->xb = n->wpk = nullptr;
  n->wgpart = nullptr;
  n->B = n->H = n->W = 0;
}

float* dalloc(hp_unet n, size_t count, bool* ok) {
  float* p = nullptr;
  if (hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(float)) != hipSuccess) {
    *ok = false;
    return nullptr;
  }
  n->owned.push_back(p);
  return p;
}

// Activation buffers for (B, H, W); reallocated only when the shape changes.
int ensure_acts(hp_unet n, int B, int H, int W) {
  if (n->B == B && n->H == H && n->W == W) return HP_OK;
  (void)hipStreamSynchronize(n->stream);
  free_acts(n);
  const int L = n->levels;
  bool ok = true;
  for (int l = 0; l < L; ++l) {
    const size_t pl = (size_t)(H >> l) * (W >> l);
    const size_t c = (size_t)B * ch(n, l) * pl;
    const bool last = l + 1 == L;
    n->enc1.push_back(dalloc(n, c, &ok));
    n->enc2.push_back(dalloc(n, c, &ok));
    n->pool.push_back(last ? nullptr : dalloc(n, c / 4, &ok));
    n->up.push_back(last ? nullptr : dalloc(n, (size_t)B * (ch(n, l + 1) + ch(n, l)) * pl, &ok));
    n->dec1.push_back(last ? nullptr : dalloc(n, c, &ok));
    n->dec2.push_back(last ? nullptr : dalloc(n, c, &ok));
    n->dskip.push_back(last ? nullptr : dalloc(n, c, &ok));
  }
  const size_t pl0 = (size_t)H * W;
  const size_t g = (size_t)B * pl0 * std::max({3 * n->base, n->cin, n->cout});
  n->y = dalloc(n, (size_t)B * n->cout * pl0, &ok);
  n->dy = dalloc(n, (size_t)B * n->cout * pl0, &ok);
  n->ga = dalloc(n, g, &ok);
  n->gb = dalloc(n, g, &ok);
  // bf16 operand buffers: every convolution input (forward or data gradient)
  // has at most 3 base channels at full resolution (or cin / cout)
  {
    const int cmax = std::max({3 * n->base, n->cin, n->base << (L - 1)});
    const size_t ch32 = (size_t)((cmax + mf::CK - 1) / mf::CK) * mf::CK;
    n->xb = reinterpret_cast<__bf16*>(dalloc(n, (size_t)B * pl0 * ch32 / 2 + 8, &ok));
    size_t wmax = 0;
    auto wsz = [&](int ci, int co) {
      return (size_t)((co + mf::CO - 1) / mf::CO) * ((ci + mf::CK - 1) / mf::CK) * 9 * mf::CB * 64 * 8;
    };
    for (auto* v : {&n->enc_a, &n->enc_b, &n->dec_a, &n->dec_b})
      for (auto& c : *v) wmax = std::max({wmax, wsz(c.ci, c.co), wsz(c.co, c.ci)});
    n->wpk = reinterpret_cast<__bf16*>(dalloc(n, wmax / 2 + 8, &ok));
    size_t pmax = 0;
    for (int l = 0; l < L; ++l) {
      auto part = [&](const hp_unet_s::Conv& c) {
        pmax = std::max(pmax, (size_t)wgrad_splits(B, H >> l, W >> l, c.ci, c.co) * (c.ci * 9 + 1) * c.co);
      };
      part(n->enc_a[l]);
      part(n->enc_b[l]);
      if (l + 1 < L) {
        part(n->dec_a[l]);
        part(n->dec_b[l]);
      }
    }
    pmax = std::max(pmax, (size_t)conv1_splits(B, H, W, n->out.ci, n->out.co) * n->out.co * (n->out.ci + 1));
    n->wgpart = dalloc(n, pmax, &ok);
  }
  if (!ok) {
    free_acts(n);
    return ufail(n, HP_ENOMEM, "activation allocation failed");
  }
  n->B = B;
  n->H = H;
  n->W = W;
  return HP_OK;
}

// y = conv(x) with weights addressed as in k_conv3; float32 or bf16 matrix cores
void conv3_any(hp_unet n, const float* x, const float* w, const float* bias, float* y, int cin, int cout, int B,
               int H, int W, int wso, int wsi, int flip, int relu) {
  if (n->bf16) {
    const int nch = (cin + mf::CK - 1) / mf::CK, nct = (cout + mf::CO - 1) / mf::CO;
    const size_t xn = (size_t)B * nch * H * W, wn = (size_t)nct * nch * 9 * mf::CB * 64 * 8;
    hipLaunchKernelGGL(k_to_bf16c, dim3(eblocks(xn)), dim3(256), 0, n->stream, x, n->xb, B, cin, H, W);
    hipLaunchKernelGGL(k_pack_w, dim3(eblocks(wn)), dim3(256), 0, n->stream, w, n->wpk, cin, cout, wso, wsi, flip);
    dim3 grid(((W + mf::TWD - 1) / mf::TWD) * ((H + mf::TH - 1) / mf::TH), nct, B);
    hipLaunchKernelGGL(k_conv3_mfma, grid, dim3(256), 0, n->stream, n->xb, n->wpk, bias, y, cin, cout, H, W, relu);
  } else {
    dim3 grid(((W + TILE - 1) / TILE) * ((H + TILE - 1) / TILE), (cout + COB - 1) / COB, B);
    hipLaunchKernelGGL(k_conv3, grid, dim3(256), 0, n->stream, x, w, bias, y, cin, cout, H, W, wso, wsi, flip,
                       relu);
  }
}

void conv3(hp_unet n, const float* x, const hp_unet_s::Conv& c, float* y, int B, int H, int W, int relu) {
  conv3_any(n, x, n->P + c.w, n->P + c.b, y, c.ci, c.co, B, H, W, c.ci * 9, 9, 0, relu);
}

// Gradients of one 3x3 convolution: dW, db into G; dx (when wanted) from dy.
void conv3_bwd(hp_unet n, const float* x, const float* dy, const hp_unet_s::Conv& c, float* dx, int B, int H,
               int W) {
  if (dx) conv3_any(n, dy, n->P + c.w, nullptr, dx, c.co, c.ci, B, H, W, 9, c.ci * 9, 1, 0);
  if (n->bf16) {
    const int ns = wgrad_splits(B, H, W, c.ci, c.co);
    const int vec = (W % 8 == 0) && ((uintptr_t)x % 16 == 0) && ((uintptr_t)dy % 16 == 0);
    const dim3 grid((c.co + wgm::CO - 1) / wgm::CO, (c.ci + wgm::CI - 1) / wgm::CI, ns);
    hipLaunchKernelGGL(k_conv3_wgrad_mfma, grid, dim3(256), 0, n->stream, x, dy, n->wgpart, B, c.ci, c.co, H, W, ns,
                       vec);
    // weights then bias: contiguous in the parameter layout
    const size_t nw = (size_t)c.co * c.ci * 9 + c.co;
    hipLaunchKernelGGL(k_wgrad_sum, dim3((unsigned)((nw + 63) / 64)), dim3(64 * wgm::SUM_WAVES), 0, n->stream,
                       n->wgpart, n->G + c.w, nw, ns);
  } else {
    hipLaunchKernelGGL(k_conv3_wgrad, dim3(c.co * c.ci), dim3(256), 0, n->stream, x, dy, n->G + c.w, B, c.ci, c.co,
                       H, W);
    hipLaunchKernelGGL(k_bias_grad, dim3(c.co), dim3(256), 0, n->stream, dy, n->G + c.b, B, c.co, (size_t)H * W);
  }
}

void relu_bwd(hp_unet n, const float* y, float* dy, size_t count) {
  hipLaunchKernelGGL(k_relu_bwd, dim3(eblocks(count)), dim3(256), 0, n->stream, y, dy, count);
}

int forward(hp_unet n, const float* x, int B, int H, int W) {
  int rc = ensure_acts(n, B, H, W);
  if (rc) return rc;
  const int L = n->levels;
  const float* in = x;
  for (int l = 0; l < L; ++l) {
    const int h = H >> l, w = W >> l;
    conv3(n, in, n->enc_a[l], n->enc1[l], B, h, w, 1);
    conv3(n, n->enc1[l], n->enc_b[l], n->enc2[l], B, h, w, 1);
    if (l + 1 < L) {
      const size_t planes = (size_t)B * ch(n, l);
      hipLaunchKernelGGL(k_pool, dim3(eblocks(planes * h * w / 4)), dim3(256), 0, n->stream, n->enc2[l], n->pool[l],
                         planes, h, w);
      in = n->pool[l];
    }
  }
  const float* cur = n->enc2[L - 1];
  for (int l = L - 2; l >= 0; --l) {
    const int h = H >> l, w = W >> l;
    const int cu = ch(n, l + 1), cs = ch(n, l), ct = cu + cs;
    hipLaunchKernelGGL(k_up, dim3(eblocks((size_t)B * cu * h * w)), dim3(256), 0, n->stream, cur, n->up[l], B, cu,
                       ct, 0, h / 2, w / 2);
    hipLaunchKernelGGL(k_chcopy, dim3(eblocks((size_t)B * cs * h * w)), dim3(256), 0, n->stream, n->up[l],
                       n->enc2[l], B, cs, ct, cu, (size_t)h * w, 0);
    conv3(n, n->up[l], n->dec_a[l], n->dec1[l], B, h, w, 1);
    conv3(n, n->dec1[l], n->dec_b[l], n->dec2[l], B, h, w, 1);
    cur = n->dec2[l];
  }
  const size_t pl0 = (size_t)H * W;
  hipLaunchKernelGGL(k_conv1, dim3(eblocks((size_t)B * pl0)), dim3(256), 0, n->stream, cur, n->P + n->out.w,
                     n->P + n->out.b, n->y, B, n->out.ci, n->out.co, pl0, 0);
  return HP_OK;
}

// Reverse pass from dy = dLoss/dy (n->dy) of the last forward on input x.
void backward(hp_unet n, const float* x) {
  const int B = n->B, H = n->H, W = n->W, L = n->levels;
  const size_t pl0 = (size_t)H * W;
  const float* top = (L > 1) ? n->dec2[0] : n->enc2[0];
  float* ga = n->ga;
  float* gb = n->gb;
  {
    // output layer: weights then bias, contiguous in the parameter layout
    const int ns = conv1_splits(B, H, W, n->out.ci, n->out.co);
    const int ne = n->out.co * (n->out.ci + 1);
    hipLaunchKernelGGL(k_conv1_wgrad_split, dim3(ne, ns), dim3(256), 0, n->stream, top, n->dy, n->wgpart, B,
                       n->out.ci, n->out.co, (unsigned)pl0, ns);
    hipLaunchKernelGGL(k_wgrad_sum, dim3((unsigned)((ne + 63) / 64)), dim3(64 * wgm::SUM_WAVES), 0, n->stream,
                       n->wgpart, n->G + n->out.w, (size_t)ne, ns);
  }
  hipLaunchKernelGGL(k_conv1, dim3(eblocks((size_t)B * pl0)), dim3(256), 0, n->stream, n->dy, n->P + n->out.w,
                     nullptr, ga, B, n->out.co, n->out.ci, pl0, 1);
  // decoder, top level first: ga = gradient w.r.t. dec2[l]
  for (int l = 0; l < L - 1; ++l) {
    const int h = H >> l, w = W >> l;
    const size_t pl = (size_t)h * w;
    const int cu = ch(n, l + 1), cs = ch(n, l), ct = cu + cs;
    relu_bwd(n, n->dec2[l], ga, (size_t)B * cs * pl);
    conv3_bwd(n, n->dec1[l], ga, n->dec_b[l], gb, B, h, w);
    relu_bwd(n, n->dec1[l], gb, (size_t)B * cs * pl);
    conv3_bwd(n, n->up[l], gb, n->dec_a[l], ga, B, h, w);  // ga = gradient w.r.t. up[l]
    hipLaunchKernelGGL(k_chcopy, dim3(eblocks((size_t)B * cs * pl)), dim3(256), 0, n->stream, ga, n->dskip[l], B, cs,
                       ct, cu, pl, 1);
    hipLaunchKernelGGL(k_up_bwd, dim3(eblocks((size_t)B * cu * pl / 4)), dim3(256), 0, n->stream, ga, gb, B, cu, ct,
                       0, h / 2, w / 2);
    std::swap(ga, gb);  // ga = gradient w.r.t. the level below's output
  }
  // encoder, bottom level first: ga = gradient w.r.t. enc2[L-1], then w.r.t. pool[l]
  for (int l = L - 1; l >= 0; --l) {
    const int h = H >> l, w = W >> l;
    const size_t pl = (size_t)h * w;
    const int c = ch(n, l);
    if (l < L - 1) {
      hipLaunchKernelGGL(k_pool_bwd, dim3(eblocks((size_t)B * c * pl)), dim3(256), 0, n->stream, ga, gb,
                         (size_t)B * c, h, w);
      hipLaunchKernelGGL(k_add, dim3(eblocks((size_t)B * c * pl)), dim3(256), 0, n->stream, gb, n->dskip[l],
                         (size_t)B * c * pl);
      std::swap(ga, gb);
    }
    relu_bwd(n, n->enc2[l], ga, (size_t)B * c * pl);
    conv3_bwd(n, n->enc1[l], ga, n->enc_b[l], gb, B, h, w);
    relu_bwd(n, n->enc1[l], gb, (size_t)B * c * pl);
    conv3_bwd(n, l == 0 ? x : n->pool[l - 1], gb, n->enc_a[l], l == 0 ? nullptr : ga, B, h, w);
  }
}

int check_shape(hp_unet n, int B, int H, int W) {
  const int m = 1 << (n->levels - 1);
  if (B < 1 || H < m || W < m || (H % m) || (W % m))
    return ufail(n, HP_EINVAL, "B >= 1 and H, W multiples of 2^(levels-1) required");
  return HP_OK;
}

int hipchk(hp_unet n, hipError_t e, const char* where) {
  if (e == hipSuccess) return HP_OK;
  return ufail(n, HP_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

int check_fields(hp_unet n, int ncomp, int nx, int ny, int B) {
  if ((ncomp != 1 && ncomp != 2) || nx < 2 || ny < 2 || B < 1 || B > 64)
    return ufail(n, HP_EINVAL, "ncomp 1 or 2, nx, ny >= 2, 1 <= B <= 64 required");
  return HP_OK;
}

}  // namespace

// For the plan's learned-guess mode (hp_api.hip): the net's stream and shape.
hipStream_t unet_stream(hp_unet n) { return n ? n->stream : nullptr; }
void unet_shape(hp_unet n, int* levels, int* cin, int* cout) {
  *levels = n ? n->levels : 0;
  *cin = n ? n->cin : 0;
  *cout = n ? n->cout : 0;
}

extern "C" {

int hp_unet_create(int levels, int base, int cin, int cout, unsigned long long seed, void* stream, hp_unet* out) {
  if (!out) return ufail(nullptr, HP_EINVAL, "out is NULL");
  *out = nullptr;
  if (levels < 1 || levels > 6 || base < 1 || base > 256 || cin < 1 || cin > 64 || cout < 1 || cout > 64)
    return ufail(nullptr, HP_EINVAL, "levels 1..6, base 1..256, cin and cout 1..64");
  hp_unet n = new (std::nothrow) hp_unet_s();
  if (!n) return ufail(nullptr, HP_ENOMEM, "host allocation failed");
  n->levels = levels;
  n->base = base;
  n->cin = cin;
  n->cout = cout;
  n->stream = reinterpret_cast<hipStream_t>(stream);
  unet_layout(n);
  // He-normal weights (std sqrt(2 / fan_in)), zero biases; the output layer scaled by 0.1
  std::vector<float> h(n->nparam, 0.f);
  std::mt19937_64 rng(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  auto init = [&](const hp_unet_s::Conv& c, double gain) {
    const double sd = gain * std::sqrt(2.0 / (double)(c.ci * c.k * c.k));
    for (size_t i = 0; i < (size_t)c.ci * c.co * c.k * c.k; ++i) h[c.w + i] = (float)(sd * nd(rng));
  };
  for (int l = 0; l < levels; ++l) {
    init(n->enc_a[l], 1.0);
    init(n->enc_b[l], 1.0);
  }
  for (int l = 0; l + 1 < levels; ++l) {
    init(n->dec_a[l], 1.0);
    init(n->dec_b[l], 1.0);
  }
  init(n->out, 0.1);
  const size_t bytes = n->nparam * sizeof(float);
  if (hipMalloc(&n->P, bytes) != hipSuccess || hipMalloc(&n->G, bytes) != hipSuccess ||
      hipMalloc(&n->M, bytes) != hipSuccess || hipMalloc(&n->V, bytes) != hipSuccess ||
      hipMalloc(&n->part, 8192 * sizeof(double)) != hipSuccess ||
      hipMalloc(&n->feat, 2 * 64 * sizeof(double)) != hipSuccess ||
      hipHostMalloc(&n->part_h, 8192 * sizeof(double)) != hipSuccess ||
      hipHostMalloc(&n->feat_h, 2 * 64 * sizeof(double)) != hipSuccess) {
    hp_unet_destroy(n);
    return ufail(nullptr, HP_ENOMEM, "device allocation failed");
  }
  if (hipMemcpy(n->P, h.data(), bytes, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(n->M, 0, bytes) != hipSuccess || hipMemset(n->V, 0, bytes) != hipSuccess ||
      hipMemset(n->G, 0, bytes) != hipSuccess) {
    hp_unet_destroy(n);
    return ufail(nullptr, HP_EHIP, "parameter upload failed");
  }
  *out = n;
  return HP_OK;
}

long hp_unet_num_params(hp_unet n) { return n ? (long)n->nparam : 0; }

int hp_unet_set_precision(hp_unet n, int precision) {
  if (!n) return ufail(nullptr, HP_EINVAL, "net is NULL");
  if (precision != HP_UNET_F32 && precision != HP_UNET_BF16) return ufail(n, HP_EINVAL, "unknown precision");
  n->bf16 = precision == HP_UNET_BF16;
  return HP_OK;
}

int hp_unet_get_params(hp_unet n, float* params, float* grads, float* adam_m, float* adam_v, long* adam_step) {
  if (!n) return ufail(nullptr, HP_EINVAL, "net is NULL");
  int rc = hipchk(n, hipStreamSynchronize(n->stream), "sync");
  const size_t bytes = n->nparam * sizeof(float);
  if (!rc && params) rc = hipchk(n, hipMemcpy(params, n->P, bytes, hipMemcpyDeviceToHost), "params");
  if (!rc && grads) rc = hipchk(n, hipMemcpy(grads, n->G, bytes, hipMemcpyDeviceToHost), "grads");
  if (!rc && adam_m) rc = hipchk(n, hipMemcpy(adam_m, n->M, bytes, hipMemcpyDeviceToHost), "adam m");
  if (!rc && adam_v) rc = hipchk(n, hipMemcpy(adam_v, n->V, bytes, hipMemcpyDeviceToHost), "adam v");
  if (!rc && adam_step) *adam_step = n->step;
  return rc;
}

int hp_unet_set_params(hp_unet n, const float* params, const float* adam_m, const float* adam_v, long adam_step) {
  if (!n) return ufail(nullptr, HP_EINVAL, "net is NULL");
  if (!params || adam_step < 0) return ufail(n, HP_EINVAL, "params NULL or adam_step < 0");
  const size_t bytes = n->nparam * sizeof(float);
  int rc = hipchk(n, hipStreamSynchronize(n->stream), "sync");
  if (!rc) rc = hipchk(n, hipMemcpy(n->P, params, bytes, hipMemcpyHostToDevice), "params");
  if (!rc)
    rc = adam_m ? hipchk(n, hipMemcpy(n->M, adam_m, bytes, hipMemcpyHostToDevice), "adam m")
                : hipchk(n, hipMemset(n->M, 0, bytes), "adam m");
  if (!rc)
    rc = adam_v ? hipchk(n, hipMemcpy(n->V, adam_v, bytes, hipMemcpyHostToDevice), "adam v")
                : hipchk(n, hipMemset(n->V, 0, bytes), "adam v");
  if (!rc) n->step = adam_step;
  return rc;
}

int hp_unet_forward(hp_unet n, const float* x, int B, int H, int W, float* y) {
  if (!n) return ufail(nullptr, HP_EINVAL, "net is NULL");
  if (!x || !y) return ufail(n, HP_EINVAL, "NULL argument");
  int rc = check_shape(n, B, H, W);
  if (!rc) rc = forward(n, x, B, H, W);
  if (rc) return rc;
  rc = hipchk(n,
              hipMemcpyAsync(y, n->y, (size_t)B * n->cout * H * W * sizeof(float), hipMemcpyDeviceToDevice,
                             n->stream),
              "copy out");
  return rc ? rc : hipchk(n, hipGetLastError(), "forward");
}

int hp_unet_grad(hp_unet n, const float* x, const float* target, int B, int H, int W, double* loss) {
  if (!n) return ufail(nullptr, HP_EINVAL, "net is NULL");
  if (!x || !target) return ufail(n, HP_EINVAL, "NULL argument");
  int rc = check_shape(n, B, H, W);
  if (!rc) rc = forward(n, x, B, H, W);
  if (rc) return rc;
  const size_t nout = (size_t)B * n->cout * H * W;
  const int nb = eblocks(nout);
  hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, n->stream, n->y, target, n->dy, n->part, nout);
  backward(n, x);
  rc = hipchk(n, hipGetLastError(), "backward");
  if (rc) return rc;
  if (loss) {
    rc = hipchk(n, hipMemcpyAsync(n->part_h, n->part, nb * sizeof(double), hipMemcpyDeviceToHost, n->stream),
                "loss");
    if (!rc) rc = hipchk(n, hipStreamSynchronize(n->stream), "sync");
    if (rc) return rc;
    double s = 0.0;
    for (int i = 0; i < nb; ++i) s += n->part_h[i];
    *loss = s / (double)nout;
  }
  return HP_OK;
}

int hp_unet_adam(hp_unet n, double lr, double beta1, double beta2, double eps) {
  if (!n) return ufail(nullptr, HP_EINVAL, "net is NULL");
  if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return ufail(n, HP_EINVAL, "lr > 0, 0 <= beta < 1, eps > 0 required");
  n->step += 1;
  const float c1 = (float)(1.0 - std::pow(beta1, (double)n->step));
  const float c2 = (float)(1.0 - std::pow(beta2, (double)n->step));
  hipLaunchKernelGGL(k_adam, dim3(eblocks(n->nparam)), dim3(256), 0, n->stream, n->P, n->G, n->M, n->V, n->nparam,
                     (float)lr, (float)beta1, (float)beta2, (float)(1.0 - beta1), (float)(1.0 - beta2), c1, c2,
                     (float)eps);
  return hipchk(n, hipGetLastError(), "adam");
}

int hp_guess_stats(hp_unet n, int ncomp, int nx, int ny, double n0, int edge_width, const void* w, const void* y,
                   const double* n2, int B, double* scal) {
  if (!n) return ufail(nullptr, HP_EINVAL, "net is NULL");
  if (!w || !y || !n2 || !scal) return ufail(n, HP_EINVAL, "NULL argument");
  int rc = check_fields(n, ncomp, nx, ny, B);
  if (rc) return rc;
  hipLaunchKernelGGL(k_guess_stats, dim3(B + 1), dim3(256), 0, n->stream, reinterpret_cast<const c128*>(w),
                     reinterpret_cast<const c128*>(y), n2, n0, edge_width, nx, ny, ncomp, scal);
  return hipchk(n, hipGetLastError(), "guess stats");
}

int hp_guess_pack(hp_unet n, int ncomp, int nx, int ny, double n0, int edge_width, const void* w, const void* y,
                  const double* n2, const double* scal, const double* pole_feat, int B, float* x_in) {
  if (!n) return ufail(nullptr, HP_EINVAL, "net is NULL");
  if (!w || !y || !n2 || !scal || !pole_feat || !x_in) return ufail(n, HP_EINVAL, "NULL argument");
  int rc = check_fields(n, ncomp, nx, ny, B);
  if (rc) return rc;
  if (n->cin != 4 * ncomp + 3) return ufail(n, HP_EINVAL, "the net needs cin = 4 ncomp + 3");
  rc = hipchk(n, hipStreamSynchronize(n->stream), "sync");  // the pinned feature buffer is reused
  if (rc) return rc;
  memcpy(n->feat_h, pole_feat, 2 * B * sizeof(double));
  rc = hipchk(n, hipMemcpyAsync(n->feat, n->feat_h, 2 * B * sizeof(double), hipMemcpyHostToDevice, n->stream),
              "features");
  if (rc) return rc;
  hipLaunchKernelGGL(k_guess_pack, dim3(eblocks((size_t)B * nx * ny)), dim3(256), 0, n->stream,
                     reinterpret_cast<const c128*>(w), reinterpret_cast<const c128*>(y), n2, scal, n->feat, n0,
                     edge_width, nx, ny, ncomp, B, x_in);
  return hipchk(n, hipGetLastError(), "guess pack");
}

int hp_guess_unpack(hp_unet n, int ncomp, int nx, int ny, const void* w, const float* net_out, const double* scal,
                    int B, void* t) {
  if (!n) return ufail(nullptr, HP_EINVAL, "net is NULL");
  if (!w || !net_out || !scal || !t) return ufail(n, HP_EINVAL, "NULL argument");
  int rc = check_fields(n, ncomp, nx, ny, B);
  if (rc) return rc;
  if (n->cout != 2 * ncomp) return ufail(n, HP_EINVAL, "the net needs cout = 2 ncomp");
  hipLaunchKernelGGL(k_guess_unpack, dim3(eblocks((size_t)B * ncomp * nx * ny)), dim3(256), 0, n->stream,
                     reinterpret_cast<const c128*>(w), net_out, scal, nx, ny, ncomp, B, reinterpret_cast<c128*>(t));
  return hipchk(n, hipGetLastError(), "guess unpack");
}

int hp_guess_target(hp_unet n, int ncomp, int nx, int ny, const void* px, const double* scal, int B, float* target) {
  if (!n) return ufail(nullptr, HP_EINVAL, "net is NULL");
  if (!px || !scal || !target) return ufail(n, HP_EINVAL, "NULL argument");
  int rc = check_fields(n, ncomp, nx, ny, B);
  if (rc) return rc;
  hipLaunchKernelGGL(k_guess_target, dim3(eblocks((size_t)B * ncomp * nx * ny)), dim3(256), 0, n->stream,
                     reinterpret_cast<const c128*>(px), scal, nx, ny, ncomp, B, target);
  return hipchk(n, hipGetLastError(), "guess target");
}

const char* hp_unet_last_error(hp_unet n) { return n ? n->err.c_str() : g_err.c_str(); }

void hp_unet_destroy(hp_unet n) {
  if (!n) return;
  if (n->stream)
    (void)hipStreamSynchronize(n->stream);
  else
    (void)hipDeviceSynchronize();
  free_acts(n);
  for (void* p : {(void*)n->P, (void*)n->G, (void*)n->M, (void*)n->V, (void*)n->part, (void*)n->feat})
    if (p) (void)hipFree(p);
  if (n->part_h) (void)hipHostFree(n->part_h);
  if (n->feat_h) (void)hipHostFree(n->feat_h);
  delete n;
}

}  // extern "C"
