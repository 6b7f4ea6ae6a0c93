// Launch wrappers of the HIP kernels (host side).  Every wrapper only enqueues
// work on `s`; sizes are validated by the caller (the plan).  T is the storage
// type of R-domain fields; C (default T) the arithmetic type of the transforms
// (complex64 storage with FP64 transforms: T = float, C = double).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "state.hpp"

struct StencilCoef {
  double c2x[7], c2y[7];  // s * c_m / h^2 (second derivative, scaled by s = 1/(k0 n0)^2)
  double d1x[6], d1y[6];  // d_m / h (first derivative)
};

struct Geo {
  int nx, ny, ncomp;
  size_t fsz;           // nx * ny
  int col_variant = 1;  // column-pass LDS budget: 0, 1, 2 = 20, 40, 80 KB per workgroup
};

// Row DST-I of the unknowns of a complex128 field (physical, row-major): out
// (R-domain, T, column-tiled with tile_w elements per tile row; 0 = the width
// of T's own layout) and per-block partial sums of |in|^2.
template <typename T, typename C = T>
void launch_row_fwd(const c128* in, cx<T>* out, double* part, const cx<C>* tw, const Geo& g, hipStream_t s,
                    int tile_w = 0);
template <typename T>
int row_blocks(int nx);

// Row DST-I back to complex128 (out = S_x in); in is column-tiled with tile_w
// elements per tile row.
template <typename T, typename C = T>
void launch_row_inv(const cx<T>* in, c128* out, const cx<C>* tw, const Geo& g, int tile_w, hipStream_t s);
// Batched forms (index lists are host arrays of n entries): row_fwd entry z
// reads in + isel[z] in_bs, writes out + osel[z] out_bs and its partial norms
// to part + z part_bs; row_inv entry z reads in + sel[z] in_bs and writes
// out + z out_bs.
template <typename T, typename C = T>
void launch_row_fwd_batch(const c128* in, size_t in_bs, const int* isel, cx<T>* out, size_t out_bs, const int* osel,
                          int n, double* part, size_t part_bs, const cx<C>* tw, const Geo& g, hipStream_t s,
                          int tile_w = 0);
template <typename T, typename C = T>
void launch_row_inv_batch(const cx<T>* in, size_t in_bs, const int* sel, int n, c128* out, size_t out_bs,
                          const cx<C>* tw, const Geo& g, int tile_w, hipStream_t s);

// Column pass: z = sigma_m * S_y diag(1/(mu_y + mu_x - b_k)) S_y u_m for the
// poles poles[0..nactive) (a host array, passed by value in the kernel
// arguments; the kernel also stores it to active_out, when not null, for the
// kernels after it on the stream).  Vector fields also get dz = D1y z (the y
// derivative the row pass needs).
template <typename T, typename C = T>
void launch_col(const cx<T>* const* uptr, cx<T>* zbase, size_t zsp, size_t zsi, cx<T>* dzbase, size_t dzsp,
                const PoleState* st, const int* poles, int nactive, int* active_out, const double* mu_x,
                const double* mu_y, const cx<C>* tw, const Geo& g, const StencilCoef& sc, hipStream_t s);

// Row pass: p = S_x (P (S_x z_m)) with P the medium part of Zbar, plus the
// partial inner products <u_i, p>, i = 0..m.  coef: the coefficient planes in
// the working precision.
template <typename T, typename C = T>
void launch_row_apply(const cx<T>* zbase, size_t zsp, size_t zsi, const cx<T>* dzbase, size_t dzsp, cx<T>* pbase,
                      size_t psp, const cx<T>* const* uptr, const C* coef, const PoleState* st,
                      const int* active, int nactive, double2* part, const cx<C>* tw, const Geo& g,
                      const StencilCoef& sc, hipStream_t s);
template <typename T>
int row_apply_blocks(const Geo& g);
// partial sums per inner product written by the row pass (one per wave)
template <typename T>
int row_apply_parts(const Geo& g);
// elements per 128-byte tile row of a column-tiled R-domain field
template <typename T>
constexpr int tile_width() {
  return 128 / (int)sizeof(cx<T>);
}

// hc_i = sigma_i * sum of the partial inner products, then (in the same
// launch, by each pole's last workgroup) the correction algebra that gives the
// update coefficients.  done: HP_MAXPOLES device counters, zero between calls.
void launch_reduce_dots(const double2* part, int nblk, PoleState* st, const int* active, int nactive, int maxm,
                        int* done, hipStream_t s);

// u_{m+1} = p - sum_i hc_i v_i and partial |u_{m+1}|^2.
template <typename T>
void launch_update(const cx<T>* pbase, size_t psp, cx<T>* const* uptr, const PoleState* st, const int* active,
                   int nactive, double* part, int nblk, const Geo& g, hipStream_t s);
int update_blocks(size_t total);

// Hessenberg column, Givens rotation, residual estimate, convergence flag and
// the least-squares solution at the end of a cycle.
// ftag[k] = (seq << 8) | flag for every pole that takes the step (flag 0: going
// on, 1: converged, 2: restart length reached, 3: the true residual decides,
// 4: a non-finite value reached the Krylov space), stored with system scope to
// host-coherent memory.
void launch_arnoldi(PoleState* st, const int* active, int nactive, const double* part, int nblk, int restart,
                    unsigned long long* ftag, unsigned long long seq, double* est, hipStream_t s);

// Start a cycle: beta = sqrt(sum part), g = beta e1, sigma_0 = 1/beta.
// first: 0 a restart; 1 the first cycle of a step's solve (the iteration count
// starts at 0); 2 the first cycle of a further solve in the same step (the
// count runs on).
// Cycle tolerance on the estimate: max(tol * beta0, rtol_cycle * beta).
// part_bs: stride between the poles' partial sums (0: all read the same);
// set_has_x: the poles' X accumulators hold a solution so far.
void launch_cycle_init(PoleState* st, const int* poles, int npoles_in, const double* part, int nblk, int first,
                       double tol, double rtol_cycle, hipStream_t s, size_t part_bs = 0, int set_has_x = 0);

// out = mask * (e^{-iK} r_inf w + e^{-iK} S_x (sum_k a_k [X_k + sum_i y_ki Z_ki])).
template <typename T>
void launch_final(const c128* w, c128* out, const cx<T>* zbase, size_t zsp, size_t zsi, const c128* xacc, size_t xsp,
                  const PoleState* st, int npoles, c128 phase, c128 rinf_phase, double loss_coef, double eta,
                  int W, const c128* tw64, const Geo& g, hipStream_t s);

// X_k += sum_i y_ki Z_ki (R-domain, complex128 accumulator).
template <typename T>
void launch_accum(c128* xacc, const cx<T>* z, size_t zsi, const PoleState* st, int pole, const Geo& g,
                  hipStream_t s);
// The same for the poles sel[0..n) (host array): X at xacc + k xsp, Z at z + k zsp.
template <typename T>
void launch_accum_batch(c128* xacc, size_t xsp, const cx<T>* z, size_t zsp, size_t zsi, const PoleState* st,
                        const int* sel, int n, const Geo& g, hipStream_t s);

// y = rhs - (Zbar - b I) x  (rhs may be NULL: y = (Zbar - b I) x), explicit
// 13-point stencils, complex128; partial |y|^2 per block.  medium_only: the
// medium part P of Zbar alone (V x, plus the psi terms of the vector operator).
void launch_apply_op(const c128* x, const c128* rhs, c128* y, const double* coef, c128 b, const StencilCoef& sc,
                     const Geo& g, double* part, hipStream_t s, int medium_only = 0);
// n fields at once: field z at x + z xbs, y + z ybs, partial sums part + z pbs,
// shift shifts[z] (host array of n <= HP_MAXPOLES).
void launch_apply_op_batch(const c128* x, size_t xbs, const c128* rhs, c128* y, size_t ybs, const double* coef,
                           const c128* shifts, int n, const StencilCoef& sc, const Geo& g, double* part, size_t pbs,
                           hipStream_t s, int medium_only = 0);
int op_blocks(const Geo& g);

// Coefficient planes from n^2: V (plane 0) and, for the vector operator,
// s psi_x, s psi_y, s psi_xx, s psi_yy, s psi_xy (planes 1..5).
void launch_coef(const double* n2, double* coef, double* scratch, double n0, double s_scale, int W,
                 const StencilCoef& sc, const Geo& g, hipStream_t s);

// Poles first..first+count-1 (count <= HP_MAXPOLES): has_x = 1, m = 0 (their
// X accumulators now hold the whole solution).
void launch_mark_folded(PoleState* st, int first, int count, hipStream_t s);
// The same for the poles poles[0..n) (host array, n <= HP_MAXPOLES).
void launch_mark_list(PoleState* st, const int* poles, int n, hipStream_t s);


// Classical RK4 combination of one stage (physical fields, complex128):
// acc_out = acc_in + ca L; v_out = u + cv L unless v_out is NULL; with
// loss_coef > 0 acc_out is multiplied by the edge layer's loss factor.
void launch_rk4_stage(const c128* L, const c128* acc_in, c128* acc_out, const c128* u, c128* v_out, double ca,
                      double cv, double loss_coef, double eta, int W, const Geo& g, hipStream_t s);
void launch_to_float(const double* a, float* b, size_t n, hipStream_t s);
