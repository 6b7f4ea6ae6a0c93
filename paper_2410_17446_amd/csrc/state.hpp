// Device-side state shared by the kernels and the host driver.
#pragma once
#include "cplx.hpp"

#define HP_MAXM 64      // largest GMRES restart length
#define HP_MAXPOLES 64  // largest number of partial-fraction terms

// GMRES state of one shifted solve (one pole), FP64 throughout (Arnoldi
// coefficients, Givens rotations, least-squares right-hand side).
//
// Orthogonalisation is classical Gram-Schmidt with delayed reorthogonalisation:
// the basis vector made in step m-1 (provisional, ~v_m) is reorthogonalised in
// step m from inner products taken in the same pass as those of the new
// direction; the Hessenberg column m-1 and the solution coefficients are
// corrected to match (Hraw holds the unrotated Hessenberg, Rc the triangular
// map ~v = V Rc, so Z~ = Z Rc and x = Z~ Rc^{-1} y).
struct PoleState {
  int m;          // Arnoldi columns completed in the current cycle
  int flag;       // 0 running, 1 converged / fixed count reached, 2 cycle ended unconverged,
                  // 3 converged on the estimate but the true residual must decide,
                  // 4 stopped: a non-finite value (NaN/Inf in n^2 or the right-hand side)
  int total;      // Arnoldi steps over all cycles
  int fixed;      // > 0: force exactly this many steps in one cycle
  int has_x;      // 1 once an earlier cycle's solution sits in the X accumulator
  int cycle;
  int pad0, pad1;
  double beta0;   // ||w|| of the step's right-hand side
  double beta;    // ||r|| at the start of the current cycle
  double est;     // current least-squares residual estimate |g_{m}|
  double tol;
  double incons;  // eps kappa(M_k): bound on the split operator's rounding per unit ||y||
  double pad3;
  c128 bk;        // pole
  c128 ak;        // residue
  double sigma[HP_MAXM + 1];          // scale of the stored vector: v_i = sigma_i u_i
  c128 cu[HP_MAXM + 2];               // update coefficients: u_i (i < m), ~v_m at m, p at m+1
  c128 cv[HP_MAXM + 1];               // correction of ~v_m: v_m = sum_i cv_i u_i (i <= m)
  int correct;                        // 1 when the update also rewrites u_m
  int pad2;
  c128 H[(HP_MAXM + 1) * HP_MAXM];    // rotated Hessenberg (R factor), column-major (i + col * (MAXM+1))
  c128 Hraw[(HP_MAXM + 1) * HP_MAXM]; // unrotated Hessenberg
  c128 Rc[(HP_MAXM + 1) * HP_MAXM];   // ~v_l = Rc[l][l] v_l + sum_{i<l} Rc[i][l] v_i
  double cs[HP_MAXM];                 // Givens cosines
  c128 sn[HP_MAXM];                   // Givens sines
  c128 g[HP_MAXM + 1];                // rotated beta e1
  c128 gpre[HP_MAXM + 1];             // g[i] before rotation i
  c128 y[HP_MAXM];                    // coefficients of Z~ in the cycle's solution
  c128 Pd[HP_MAXM + 1];               // reduced <u_i, p> of the current step
  c128 Qd[HP_MAXM + 1];               // reduced <u_i, u_m> of the current step
};

// The poles of one launch, passed by value in the kernel arguments (no copy to
// the device before the launch).
struct PoleList {
  int n;
  int k[HP_MAXPOLES];
};

// Shifts b_k of the fields of one batched launch of the explicit operator.
struct ShiftList {
  c128 b[HP_MAXPOLES];
};
