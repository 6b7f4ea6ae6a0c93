// The absorbing-layer form of the step (Sec. 4.1: complex-coordinate
// stretching of the derivative matrices at the periphery; Sec. 4.2: the
// free-space problem as the Sylvester equation of eq. fs_sylvester with those
// matrices).  FP64, square grids with N nodes per axis: fields are ncomp
// (1, or 2 for (E_x, E_y)) N x N complex128 planes, row-major, physical (no
// row transform); node 0 and the virtual node N of each axis are Dirichlet
// nodes and row 0 and column 0 of every plane the kernels write are zero.
//
// Along either axis the stretched second derivative at node j is
//   s d^2/dx~^2 x = a2[j] (sum_m c2_m x_{j+m}) - a1[j] (sum_m d1_m (x_{j+m} - x_{j-m}))
// with g = 1 + i sigma the stretch, a2 = 1/g^2, a1 = s g'/g^3, c2_m = s c_m/h^2,
// d1_m = d_m/h, s = 1/(k0 n0)^2 and odd reflection about the Dirichlet nodes.
// The free-space operator of one axis, s D~ = Q diag(lam) Q^-1, is given by its
// eigen-decomposition: the dense matrices are stored padded to N x N (row and
// column 0 zero) and lam to N entries (lam[0] unused), so that every product
// runs on whole 64 x 64 tiles.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "kernels.hpp"

// Where a dense stage reads or writes pole k's field (m = the pole's current
// Arnoldi index): the basis table entry tbl[k (HP_MAXM + 1) + m] when tbl is
// set, else base + k sp + m si.
struct PmlRef {
  c128* const* tbl;
  c128* base;
  size_t sp, si;
};

// One of the four dense stages of
//   M_k^-1 y = Q [(Q^-1 y Q^-T) / (lam_p + lam_q - b_k)] Q^T,
// over the poles list[0..n) (host array, by value; poles with a nonzero flag
// skip themselves): left Out = Mat In, or right Out = In Mat^T; epilogue 0
// none, 1 divide entry (p, q) by lam_p + lam_q - b_k, 2 scale by the pole's
// sigma_m.  active_out (may be NULL) receives the list for later kernels.
// variant: 0 vector-ALU products on 64 x 64 tiles; matrix-core products on
// 1 64 x 64 tiles while n (N/64)^2 >= 512 (two workgroups per CU), else
// 32 x 32, 2 always 32 x 32 (four times the workgroups), 3 always 64 x 64.
// Each component plane of a field is transformed on its own (the free-space
// operator does not couple components).
void launch_pml_gemm(int variant, bool left, int epilogue, const c128* mat, PmlRef in, PmlRef out,
                     const PoleState* st, const int* list, int n, int* active_out, const c128* lam, int N, int ncomp,
                     hipStream_t s);

// A round whose poles all start from the step's shared first basis vector u_0
// shares the first two products: T = Q^-1 u_0 Q^-T once (one-entry pole list
// with the state k_pml_shared_setup writes: m = 0, b = 0, sigma_0 = 1, tbl[0] =
// u0), then per pole Q [T / (lam_p + lam_q - b_k)] with the divide applied as
// the operand is loaded (launch_pml_gemm_divided, matrix cores; tiles as
// variant 1), then the last stage as usual.
void launch_pml_shared_setup(PoleState* st, c128** tbl, const c128* u0, hipStream_t s);
void launch_pml_gemm_divided(const c128* mat, PmlRef in, PmlRef out, const PoleState* st, const int* list, int n,
                             int* active_out, const c128* lam, int N, int ncomp, hipStream_t s);

// p = (Zbar~ - b_k I) z_m - sigma_m u_m into P[k] (so that A_k z_m = ~v_m + p
// for the z_m as stored) and the partial inner products <u_i, p>, <u_i, u_m>,
// i = 0..m, in the layout the dot reduction reads (pml_apply_parts per product).
// coef: the plan's coefficient planes (V; for ncomp = 2 also the psi planes).
int pml_apply_parts(int N);
void launch_pml_apply(const c128* zbase, size_t zsp, size_t zsi, c128* pbase, size_t psp, c128* const* uptr,
                      const double* coef, const c128* a2, const c128* a1, const StencilCoef& sc, const PoleState* st,
                      const int* active, int nactive, double2* part, int N, int ncomp, hipStream_t s);

// y = rhs - (Zbar~ - b I) x (rhs NULL: y = (Zbar~ - b I) x) with the stretched
// stencils, for n fields (field z at x + z xbs, y + z ybs, shift shifts[z], host
// array); partial |y|^2 of each of the nblk = pml_tiles(N) 64 x 16 tiles per
// field at part + z pbs; false (nothing launched) for another nblk.
int pml_tiles(int N);
bool launch_pml_residual(const c128* x, size_t xbs, const c128* rhs, c128* y, size_t ybs, const double* coef,
                         const c128* a2, const c128* a1, const StencilCoef& sc, const c128* shifts, int n,
                         double* part, size_t pbs, int nblk, int N, int ncomp, hipStream_t s);

// dst + osel[z] dbs = src + isel[z] sbs with row and column 0 zeroed (host
// index arrays of n entries); partial |dst|^2 of nblk blocks per entry at
// part + z part_bs.
void launch_pml_copy(const c128* src, size_t sbs, const int* isel, c128* dst, size_t dbs, const int* osel, int n,
                     double* part, size_t part_bs, int nblk, int N, int ncomp, hipStream_t s);

// out = phase sum_k a_k (X_k + sum_{i<m_k} y_ki Z_ki) + rinf_phase w (X_k only
// where the pole's has_x is set); row and column 0 zero.
void launch_pml_final(const c128* w, c128* out, const c128* zbase, size_t zsp, size_t zsi, const c128* xacc,
                      size_t xsp, const PoleState* st, int npoles, c128 phase, c128 rinf_phase, int N, int ncomp,
                      hipStream_t s);
