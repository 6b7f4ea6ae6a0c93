/*
 * hp.h -- C ABI of the MI355X library for one step of the one-way
 * (vector) Helmholtz propagator in its exponential-operator form.
 *
 * Method (Keefe, McDaniel, Cubillos, Zilberter, Madden, "A vector Helmholtz
 * electromagnetic wave propagator for inhomogeneous media"):
 *   Sec. 2, eq. expop_prop:   w(z+dz) = exp(iK(-I + sqrt(I + Zbar))) w(z),
 *                             K = k0 n0 dz, Zbar the operator of eq. Z_bar_eq;
 *   Sec. 2, eqs. rational approximation / pf_expan_eq:
 *                             exp(iK sqrt(1+z)) ~ r_inf + sum_k a_k/(z - b_k);
 *   Sec. 2, eqs. Wk_define / approx_prop / W_k_def:
 *                             w(z+dz) = e^{-iK} (r_inf w + sum_k a_k x_k),
 *                             (Zbar - b_k I) x_k = w, one sparse solve per pole;
 *   Sec. 4.2:                 each solve by right-preconditioned GMRES whose
 *                             preconditioner is the free-space operator
 *                             Zbar_fs - b_k I (eq. Z_bar_fs_def), solved as the
 *                             Sylvester equation of eq. fs_sylvester;
 *   Sec. 4.1:                 13-point fourth-order differences.
 *
 * Grid: an nx-by-ny array per field component, row-major [ny][nx] (x fastest).
 * Node 0 and the virtual node n of each axis are homogeneous-Dirichlet nodes
 * (odd reflection closes the stencils there, so the free-space preconditioner
 * is diagonalised exactly by DST-I); unknowns are nodes 1..n-1.  Row 0 and
 * column 0 of every input field are ignored; they are written as 0 on output.
 * Fields are complex128, interleaved (re, im), component-major
 * [ncomp][ny][nx]; ncomp = 1 (scalar) or 2 (E_x, E_y coupled by the
 * cross-polarisation terms of eq. Z_bar_eq).
 *
 * Edge layer: for distance d = min(i, n-i, j, n-j) <= edge_width the medium
 * terms of Zbar are zero (Sec. 4.1 zeroes them in its boundary layers).  In
 * place of the paper's PML the layer is a lossy medium n^2 = n0^2 + i eta(d),
 * eta(d) = edge_eta ((W+1-d)/W)^2, whose loss over a step multiplies the
 * stepped field by exp(-k0 dz eta(d) / (2 n0)).
 *
 * Memory: every field pointer is a DEVICE pointer (hipMalloc'd or a torch
 * tensor's storage).  The caller owns inputs, outputs and (when given) the
 * workspace; the plan copies the pole/residue table and stencils at create.
 * All calls are asynchronous on the plan's stream except where stated; the
 * GMRES driver keeps one Arnoldi step in flight ahead of the one whose
 * convergence flags it reads (the flags are written by the device into
 * host-coherent pinned memory and polled, no event per step), and
 * synchronises the stream when cycles end to read FP64 true residuals.  A plan
 * is not re-entrant; different plans may run on different streams.  No call
 * falls back to the CPU.
 *
 * Errors: a negative return means nothing valid was written; a positive
 * return is a warning with the output written.  hp_last_error() gives a
 * message for the last failing call on the plan (or the thread, for NULL).
 */
#ifndef HP_H
#define HP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hp_plan_s* hp_plan;
typedef struct { double re, im; } hp_c128;

enum {
  HP_OK = 0,
  HP_WARN_NOCONV = 1,      /* some solve missed tol after max_cycles restarts */
  HP_WARN_UNSTABLE = 2,    /* max |e^{-iK} r(mu_p + mu_q)| > 1 + 1e-6 on the free-space spectrum */
  HP_EINVAL = -1,
  HP_ENOMEM = -2,
  HP_EHIP = -3,
  HP_ESTATE = -4
};

/* Precision of the GMRES inner loop (Sec. 4.2).  In every mode the Arnoldi
 * coefficients, Givens rotations, least squares, the solution accumulator,
 * the true residual and the residue-weighted sum are FP64.
 *   HP_FP64:    complex128 Krylov vectors and transforms.
 *   HP_MIXED:   complex64 Krylov vectors and complex64 transforms; each
 *               complex64 cycle stops at 1e-5 of its starting residual and the
 *               FP64 true residual restarts it (iterative refinement).
 *   HP_MIXED64: complex64 Krylov vectors (half the HBM traffic), transforms in
 *               FP64 arithmetic; a cycle runs to tol and the FP64 true
 *               residual decides, restarting the solve if the rounding of the
 *               stored vectors kept it above tol. */
enum { HP_FP64 = 0, HP_MIXED = 1, HP_MIXED64 = 2 };

typedef struct {
  int nx, ny;                 /* cells per axis = array dims: 64, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048 */
  double dx, dy;              /* grid spacing */
  double k0, n0, dz;          /* vacuum wavenumber, reference index, step; K = k0 n0 dz */
  int ncomp;                  /* 1 scalar, 2 vector */
  int npoles;                 /* N of the (N,N) rational approximation, 1..60 */
  const hp_c128* poles;       /* host [npoles]: b_k */
  const hp_c128* residues;    /* host [npoles]: a_k */
  hp_c128 r_inf;              /* alpha_NN / beta_NN */
  const double* d2;           /* host [7]: c0..c6 of the 13-point second derivative */
  const double* d1;           /* host [6]: d1..d6 of the 13-point first derivative */
  int edge_width;             /* W >= 6 cells; n >= 2W + 14 */
  double edge_eta;            /* peak Im(n^2) of the edge layer (>= 0) */
  double tol;                 /* relative residual ||w - A x|| / ||w|| per solve */
  int restart;                /* GMRES(m) restart length, 1..64 */
  int max_cycles;             /* restarts before HP_WARN_NOCONV, >= 1 */
  int precision;              /* HP_FP64, HP_MIXED or HP_MIXED64 */
} hp_plan_desc;

/* Device bytes a plan needs; 0 if desc is invalid.  Dominated by the Krylov
 * storage, npoles * (2 restart + 3) fields of ncomp nx ny elements (16 bytes
 * in HP_FP64, 8 otherwise): about 16 GB for 1024^2 scalar, 16 poles, restart
 * 30 in FP64, and 206 GB for 2048^2 vector, 24 poles, in FP64. */
size_t hp_workspace_bytes(const hp_plan_desc* desc);

/* Create a plan.  stream: a hipStream_t (NULL = default stream).  workspace:
 * NULL (the plan allocates hp_workspace_bytes with hipMalloc and frees it at
 * destroy) or a caller-owned device buffer of at least that size, 256-byte
 * aligned.  Validates the descriptor (HP_EINVAL: sizes, W, a pole within
 * 1e-14 of a free-space eigenvalue mu_p + mu_q), uploads tables, and returns
 * HP_WARN_UNSTABLE (plan still valid) when the rational function exceeds 1 in
 * modulus on the free-space spectrum. */
int hp_plan_create(const hp_plan_desc* desc, void* stream, void* workspace, hp_plan* out);

/* Coefficient preparation (Sec. 2 eq. Z_bar_eq, Sec. 4.1): from the real
 * refractive-index field n2 (device, [ny][nx] doubles) compute the medium
 * terms of Zbar: V = (n^2 - n0^2)/n0^2 and, for ncomp = 2, the derivatives of
 * psi = ln n^2.  Kept in the plan until the next call. */
int hp_set_medium(hp_plan plan, const double* n2);

/* One step (Sec. 2 eq. approx_prop).  E_in, E_out: device [ncomp][ny][nx]
 * complex128; E_out may equal E_in.  n2: device [ny][nx] or NULL to keep the
 * medium of the last call.  Returns HP_WARN_NOCONV (output written, each solve
 * at its best iterate) when some solve missed tol within max_cycles cycles, and
 * HP_EINVAL (output undefined) when a NaN or Inf reached a solve: a non-finite
 * E_in or n2, or n2 <= 0 where the vector operator takes ln n2. */
int hp_step(hp_plan plan, const void* E_in, const double* n2, void* E_out);

/* The propagation loop of Sec. 2 (after eq. expop_prop: the field is advanced
 * step by step in z, n and psi refreshed for every new step): nsteps calls of
 * hp_step, E_in -> E_out, each step's output the next step's input.  n2 may be
 * NULL (keep the plan's medium), or n2 + s * n2_step_stride is the medium of
 * step s (stride 0: one z-independent medium); n2 is device memory of
 * nsteps planes when the stride is not 0.  E_out may equal E_in; nsteps = 0
 * copies E_in to E_out.  Returns the most severe step status (a negative one
 * stops the loop, E_out then undefined). */
int hp_propagate(hp_plan plan, const void* E_in, const double* n2, long n2_step_stride,
                 int nsteps, void* E_out);

/* One shifted solve of the step (Sec. 2 eq. W_k_def, Sec. 4.2): x = (Zbar -
 * b_k I)^{-1} rhs by the same preconditioned GMRES as hp_step, to the plan's
 * tolerance, on the medium of the last hp_set_medium.  rhs, x: device
 * [ncomp][ny][nx] complex128 (distinct).  Synchronous.  Used to check single
 * poles at full size and to generate solve pairs. */
int hp_solve(hp_plan plan, int pole, const void* rhs, void* x);

/* Initial guesses.  The method is unchanged by them: every solve still ends
 * on the same test ||w - A_k x_k|| <= tol ||w|| (A_k = Zbar - b_k I); a guess
 * only moves the point GMRES starts from, x_k = x0 + M_k^{-1} V y (Sec. 4.2).
 *
 * hp_step_guess: one step like hp_step, with x0[k] (device [ncomp][ny][nx]
 * complex128, or NULL for a zero start) the guess of pole k; x0 itself may be
 * NULL (no guesses).  Each guess is judged by its FP64 residual
 * r0 = w - A_k x0 (explicit stencils): it is used when ||r0|| < ||w||, else
 * that pole starts from zero (the fallback).  accepted: host [npoles] or
 * NULL; 1 where the guess was used.  All guesses are judged together with one
 * stream synchronisation; the first guess step on a plan allocates one
 * complex128 field per pole (hipMalloc) for their residuals, freed with the
 * plan. */
int hp_step_guess(hp_plan plan, const void* E_in, const double* n2, const void* const* x0, int* accepted,
                  void* E_out);

/* Start of every pole's GMRES in hp_step / hp_propagate (and in
 * hp_step_guess when its x0 is NULL): HP_GUESS_ZERO (default); HP_GUESS_PREV,
 * the same pole's solution of the previous step on this plan (the first step
 * after the call starts from zero), which keeps each pole's solution in the
 * workspace after the step (one extra pass over each pole's Krylov basis); or
 * HP_GUESS_LEARNED, starting points from the U-Net attached by
 * hp_set_guess_net (hp_unet.h), computed by the library at the start of every
 * step: y_k = M_k^{-1} w, the net's correction from (w, y_k, the medium, the
 * pole), x0_k = M_k^{-1}(w + sigma_k net_k).  Every guess is judged as in
 * hp_step_guess (used only when its FP64 residual is below ||w||), so the
 * solves end on the same test with any mode.  HP_ESTATE for HP_GUESS_LEARNED
 * without a net.  Guesses apply to the exponential form only. */
enum { HP_GUESS_ZERO = 0, HP_GUESS_PREV = 1, HP_GUESS_LEARNED = 2 };
int hp_set_guess(hp_plan plan, int mode);

/* Autotuner of the launch shape (not an operation of the method: it changes
 * no arithmetic, only how the shifted solves are launched).  The column
 * pass of the preconditioner is built for three LDS budgets per workgroup (20,
 * 40 and 80 KB: one to four complex128 columns of 1024 at once, more for
 * complex64 or shorter columns); which is fastest depends on the grid, the
 * precision and the number of poles.  hp_autotune takes one step E_in -> E_out
 * with each variant untimed, then `reps` (1..100) timed steps each from the
 * same E_in, keeps the fastest variant in the plan for every later call, and
 * ends with one step by it, so E_out and hp_get_stats are that variant's.
 * E_in, E_out: device [ncomp][ny][nx] complex128, E_out must not alias E_in;
 * n2 as for hp_step (NULL keeps the medium).  variant (may be NULL) receives
 * 0, 1 or 2.  Synchronises the plan's stream; returns the last step's code
 * (HP_EINVAL on bad arguments, the plan unchanged).  A new plan uses variant 1. */
int hp_autotune(hp_plan plan, const void* E_in, const double* n2, int reps, void* E_out, int* variant);

/* Set the column-pass variant (0, 1 or 2, as hp_autotune reports it) directly,
 * e.g. to reuse a choice measured once for plans of the same shape.  HP_EINVAL
 * for another value.  With absorbing layers (hp_set_pml) the variant picks the
 * form of the preconditioner's dense complex products instead (0..3), and
 * hp_autotune chooses among those: 0 vector-ALU products on 64 x 64 tiles;
 * matrix-core (FP64 MFMA) products on 1 64 x 64 tiles while the round's poles
 * give every CU two workgroups, else 32 x 32 tiles, 2 always 32 x 32, 3 always
 * 64 x 64.  Removing the layers turns variant 3 back into 1. */
int hp_set_launch(hp_plan plan, int col_variant);

/* What a step does with the pole table.
 *
 * HP_FORM_EXP (default): the table is the partial-fraction form of a rational
 * approximation of exp(iK sqrt(1+z)), K = k0 n0 dz, and a step is the
 * exponential-operator step of Sec. 2 eq. approx_prop.
 *
 * HP_FORM_SQRT: the table approximates sqrt(1+z) (for example the
 * Cauchy-integral / Gauss-Jacobi partial fractions of Sec. 3.2 and Appendix A,
 * r_inf = c_alpha + sum wt_j, b_j = -(1 + i alpha sigma_j),
 * a_j = -i alpha wt_j (1 + sigma_j)), and a step integrates the
 * pseudo-differential form of the propagator, Sec. 2 eq. eq_barZfactor2,
 *     dw/dz = i k0 n0 (r(Zbar) - 1) w,
 * over dz with `substeps` (1..1024) classical fourth-order Runge-Kutta steps of
 * h = dz / substeps.  Each RK stage is one solve of every pole (eq.
 * Auxiliary_W) with the same GMRES, tolerance and restarts as the exponential
 * form, so a step costs 4 * substeps lockstep solves.  The edge layer's loss is
 * applied after every substep (factor exp(-k0 h eta / (2 n0))).  hp_get_stats
 * then sums each pole's iterations over the step's stages.  The paper does not
 * fix the z-integrator: RK4 is this library's choice.  The first call
 * allocates three complex128 fields (hipMalloc), freed with the plan; the
 * previous-step guesses of HP_GUESS_PREV are dropped, and hp_step_guess
 * returns HP_ESTATE while the form is HP_FORM_SQRT.
 *
 * Returns HP_WARN_UNSTABLE (form still set) when one substep amplifies some
 * free-space mode: the maximum of |P(h i k0 n0 (r(mu) - 1))| over the interval
 * the free-space eigenvalues mu span exceeds 1 + 1e-6, P(z) = 1 + z + z^2/2 +
 * z^3/6 + z^4/24.  Too long a substep fails it by orders of magnitude (the
 * evanescent modes below mu = -1); the error of r next to mu = -1 alone can
 * fail it slightly (about 1e-4 per lambda/8 substep for 25 Cauchy terms, a
 * slow growth of the modes at grazing angles).  hp_plan_create's own
 * check measures |r| against 1, which a table of sqrt(1+z) exceeds by design,
 * so for such a table its HP_WARN_UNSTABLE is expected and this check is the
 * one that applies.  HP_EINVAL for an unknown form or substeps out of range. */
enum { HP_FORM_EXP = 0, HP_FORM_SQRT = 1 };
int hp_set_form(hp_plan plan, int form, int substeps);

/* The rational approximation of Sec. 3.1 computed on the device, for a
 * step size without a table entry: AAA (greedy support points, weights from
 * the smallest singular vector of the Loewner matrix) followed by
 * lawson_steps (0..1000; 40 is what the host fit uses) Lawson reweightings of
 * the linearised least-squares problem, on 4001 uniform samples of
 * z in [-4, 2] of exp(iK sqrt(1+z)) (principal branch), keeping the iterate
 * whose partial fractions have the smallest largest sample error (AAA's own
 * included).  K = k0 n0 dz > 0, degree = number of poles (1..31).  One
 * workgroup runs the whole fit in one launch on `stream` (NULL: the null
 * stream; hipMalloc of about 5 MB of scratch, freed before returning);
 * synchronous.  Outputs (host arrays): poles [degree], residues [degree],
 * *r_inf, and *max_err (may be NULL) the largest |r - f| on the samples.
 * HP_EINVAL for bad arguments or when the kept denominator does not have
 * degree finite roots; the message is in hp_last_error(NULL). */
int hp_fit_exp_sqrt(double K, int degree, int lawson_steps, void* stream, hp_c128* poles, hp_c128* residues,
                    hp_c128* r_inf, double* max_err);

/* Absorbing layers (Sec. 4.1): the periphery of W = edge_width cells along
 * each axis becomes a perfectly matched layer by complex-coordinate
 * stretching of the transverse derivatives, d/dx -> (1/g) d/dx with
 *   g(x) = 1 + i sigma,  sigma = sigma_max ((W + 1 - d)/W)^2 for 1 <= d <= W,
 *   0 beyond (d: distance in cells to the axis's nearer Dirichlet node),
 * so that along each axis
 *   d^2/dx~^2 = (1/g^2) d^2/dx^2 - (g'/g^3) d/dx,
 * discretised node by node with the plan's 13-point D2 and D1 (odd
 * reflection about the Dirichlet nodes) and the exact derivative g'.  Zbar
 * keeps its medium term V = (n^2 - n0^2)/n0^2 and, for vector fields, its psi
 * coupling, both zero inside the layers (so only the Laplacian rows of the
 * layers change, in each component); the
 * free-space problem of pole b_k is the Sylvester equation of Sec. 4.2 eq.
 * fs_sylvester with the stretched matrices, solved by eigen-decomposition of
 * the one-axis operator s D~ = Q diag(lam) Q^-1 (s = 1/(k0 n0)^2; both axes
 * share it):  W = Q [(Q^-1 Y Q^-T) / (lam_p + lam_q - b_k)] Q^T.  The step of
 * eq. approx_prop then has no separate edge loss (edge_eta is ignored): the
 * layers absorb.  GMRES ends every solve on its FP64 true residual.
 *
 * Q, Qinv: host complex128 [N-1][N-1] row-major, lam: host complex128 [N-1],
 * N = nx = ny, for the unknowns 1..N-1 of one axis (computed by the caller,
 * e.g. by a dense eigensolver); the library copies them (2 N^2 complex128 on
 * the device) and checks on the host that Q diag(lam) Qinv reproduces its own
 * s D~ on two pseudo-random vectors to 1e-3 (HP_EINVAL otherwise; the dense
 * stages only precondition, since every Arnoldi step applies the explicit
 * stretched operator to the stored z, but wide layers with a weak sigma_max
 * make Q so ill-conditioned, cond(Q) above 1e13, that its rounding breaks that
 * bound) and that no pole meets lam_p + lam_q.  The first call allocates the tables, one field
 * per pole and the inner-product partials (hipMalloc), freed with the plan.
 * Requires nx = ny, dx = dy, HP_FP64 (HP_EINVAL otherwise; ncomp 1 or 2), the
 * exponential form and HP_GUESS_ZERO (HP_ESTATE otherwise); while the layers
 * are set hp_set_form, hp_set_guess and hp_step_guess with guesses return
 * HP_ESTATE, hp_apply_operator and hp_apply_preconditioner apply the stretched
 * operators, and hp_apply_preconditioner_noalloc returns HP_ESTATE.
 * sigma_max = 0 with Q, Qinv, lam all NULL removes the layers.  In the
 * kernel timing the class HP_K_PML holds the four dense stages of every
 * round, and its byte figure counts floating-point operations instead
 * (8 (N-1)^3 ncomp per complex product: four per pole and round, except in a
 * round where every pole starts from the step's shared first basis vector,
 * whose first two products are pole-independent and run once). */
int hp_set_pml(hp_plan plan, double sigma_max, const void* Q, const void* Qinv, const void* lam);

/* x_k of the last step, guess step or solve for pole k (Sec. 2 eq. W_k_def):
 * device [ncomp][ny][nx] complex128.  Synchronous. */
int hp_get_solution(hp_plan plan, int pole, void* x);

/* y = P x, the medium part of Zbar (eq. Z_bar_eq without the transverse
 * Laplacian: V x, and for ncomp = 2 the psi terms), FP64, zero in the edge
 * layer; x, y distinct device [ncomp][ny][nx] complex128. */
int hp_apply_medium(hp_plan plan, const void* x, void* y);

/* Statistics of the last step (synchronous): GMRES iterations and final
 * relative residual estimate per pole (either pointer may be NULL). */
int hp_get_stats(hp_plan plan, int* iters_per_pole, double* final_relres);

/* Fixed-iteration mode (reproducibility / replay): iters[k] > 0 forces a
 * single GMRES cycle of exactly iters[k] Arnoldi steps for pole k in every
 * later step; NULL restores tolerance-driven iterations. */
int hp_set_fixed_iters(hp_plan plan, const int* iters);

/* Operator-level entry points on device fields [ncomp][ny][nx] complex128,
 * FP64 (used for checking; they share the step's kernels):
 *   y = (Zbar - b_k I) x         (Sec. 2 eq. W_k_def; the explicit stencils)
 *   y = (Zbar_fs - b_k I)^{-1} x (Sec. 4.2.2 eq. fs_sylvester by DST-I)
 * pole < 0 means the shift b = 0. */
int hp_apply_operator(hp_plan plan, int pole, const void* x, void* y);
int hp_apply_preconditioner(hp_plan plan, int pole, const void* x, void* y);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the solve of
 * hp_apply_preconditioner, y = (Zbar_fs - b_k I)^{-1} x (pole < 0: b = 0), with
 * every intermediate buffer (the row-transformed input, the column pass's
 * output and its y derivative, the pole state and partial norms) in a static
 * device array of the library, 49 MiB per GPU (48 MiB of fields, 1 MiB of
 * state) held from load until the process ends.  It calls no hipMalloc,
 * hipFree, memset or host-to-device copy, does not synchronise (asynchronous on
 * the plan's stream) and uses only set-up done by hp_plan_create.  x, y: device
 * [ncomp][ny][nx] complex128, distinct.  HP_EINVAL for a field beyond the
 * array (ncomp nx ny above 1048576 in HP_FP64; twice that in the mixed modes,
 * whose intermediate fields are complex64), HP_EHIP if the array's device
 * address could not be looked up.  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (plans on different streams, or
 * threads) race and must be serialised by the caller; the array keeps the
 * last call's contents. */
int hp_apply_preconditioner_noalloc(hp_plan plan, int pole, const void* x, void* y);

/* Kernel timing (diagnostics).  enable: 0 off, -1 every kernel class, else a
 * bitmask of classes (1 << HP_K_*).  Each launch of a timed class is
 * bracketed by HIP events on the plan's stream (an event pair costs a few
 * microseconds of stream time, so time one class to keep the rest of the step
 * undisturbed) and its algorithmic HBM bytes (the bytes the operation must
 * move: fields read and written once) are counted.  hp_profile_read
 * synchronises and returns, per kernel class (HP_K_*), launches, summed event
 * milliseconds and summed algorithmic bytes since the last hp_profile call;
 * arrays have HP_K_COUNT entries (NULL to skip). */
enum { HP_K_ROW_FWD = 0, HP_K_COL = 1, HP_K_ROW_APPLY = 2, HP_K_UPDATE = 3, HP_K_SMALL = 4,
       HP_K_FINAL = 5, HP_K_RESIDUAL = 6, HP_K_GUESS = 7, HP_K_PML = 8, HP_K_COUNT = 9 };
int hp_profile(hp_plan plan, int enable);
int hp_profile_read(hp_plan plan, long* launches, double* ms, double* bytes);
/* Time only every period-th launch of each timed class (period >= 1, counted
 * per class from the last hp_profile call; 1 = every launch, the default).
 * A period above 1 takes the event pairs out of most launches, so the step
 * keeps its untimed rate while the timed launches sample the class. */
int hp_profile_sample(hp_plan plan, int period);
/* Per kernel class: launches and algorithmic bytes of EVERY launch of every
 * class since the last hp_profile call that enabled profiling, timed or not
 * (untimed classes and, with a sampling period above 1, untimed launches
 * included), so that the bytes of a run can be paired with a profiler's
 * per-dispatch counters over the same launches.  Host-side counts, no
 * synchronisation. */
int hp_profile_totals(hp_plan plan, long* launches, double* bytes);

const char* hp_last_error(hp_plan plan);
void hp_plan_destroy(hp_plan plan);

/* Batches of independent propagations (serving workload; the paper's pole
 * parallelism, Sec. 3.1, extended across problems).  nworkers host threads,
 * each with its own HIP stream on the current device, take problems
 * longest-first (cost nx ny ncomp npoles nsteps), create the problem's plan
 * in the worker's workspace (allocated on first use, sized for the largest
 * problem, freed by hp_batch_destroy), propagate and destroy it; problems of
 * different sizes run concurrently.  descs is copied (tables included).
 * hp_batch_propagate blocks until every problem is done; per problem: E_in,
 * E_out device [ncomp][ny][nx] complex128 (may alias), n2 device [ny][nx]
 * (z-independent medium), nsteps >= 0.  Returns the most severe status. */
typedef struct hp_batch_s* hp_batch;
int hp_batch_create(const hp_plan_desc* descs, int nprob, int nworkers, hp_batch* out);
int hp_batch_propagate(hp_batch batch, const void* const* E_in, const double* const* n2, const int* nsteps,
                       void* const* E_out);
/* Per problem: GMRES iterations summed over poles and steps, wall seconds. */
int hp_batch_stats(hp_batch batch, long* iters, double* seconds);
/* Column-pass launch variant per problem (nprob values, each 0, 1 or 2, as
 * hp_autotune reports them for a plan of that problem's shape; 1 until set).
 * HP_EINVAL for a NULL argument or a value out of range (nothing changed). */
int hp_batch_set_launch(hp_batch batch, const int* variants);
void hp_batch_destroy(hp_batch batch);

#ifdef __cplusplus
}
#endif

#endif /* HP_H */
