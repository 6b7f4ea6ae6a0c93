// Host runtime behind include/hp.h: plan, workspace, the lockstep GMRES
// driver over all poles of a step, and the C ABI.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <complex>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/hp.h"
#include "../../include/hp_unet.h"
#include "kernels.hpp"
#include "pml.hpp"

// the rational fit on the device (fit.hip)
int fit_exp_sqrt_device(double K, int degree, int lawson_steps, hipStream_t s, std::vector<c128>& h,
                        std::string* why);
// the learned guess needs the net's stream and channel counts (unet.hip)
hipStream_t unet_stream(hp_unet n);
void unet_shape(hp_unet n, int* levels, int* cin, int* cout);

namespace {

thread_local std::string g_thread_error;

constexpr double kInnerRtolMixed = 1e-5;  // cycle tolerance of the complex64 inner solves

struct Ws {
  char* base = nullptr;
  size_t off = 0;
  bool dry = true;
  template <typename X>
  X* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    X* p = dry ? nullptr : reinterpret_cast<X*>(base + off);
    off += count * sizeof(X);
    return p;
  }
};

}  // namespace

struct hp_plan_s {
  hp_plan_desc d{};
  std::vector<hp_c128> poles, residues;
  double c2[7]{}, d1c[6]{};
  hipStream_t stream = nullptr;
  bool own_ws = false;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  Geo geo{};
  StencilCoef sc{};
  bool mixed = false;     // complex64 storage of the R-domain fields
  bool mixed64 = false;   // ... with FP64 transforms (HP_MIXED64)
  int nrowblk = 0, napplyblk = 0, nupdblk = 0, nopblk = 0;
  size_t fieldn = 0;  // ncomp * nx * ny
  // device
  double *mu_x = nullptr, *mu_y = nullptr;
  void *tw_x = nullptr, *tw_y = nullptr;
  c128* tw64_x = nullptr;
  double *coef = nullptr, *coef_scratch = nullptr;
  float* coef_f = nullptr;  // float copy of the coefficient planes (mixed precision)
  void *U = nullptr, *Z = nullptr, *P = nullptr, *DZ = nullptr, *bR = nullptr, *tmpR = nullptr;
  c128 *X = nullptr, *tmp1 = nullptr, *tmp2 = nullptr;
  PoleState* st = nullptr;
  PoleState* st_scratch = nullptr;
  void** uptr = nullptr;
  void** uptr_scratch = nullptr;
  int* active_d = nullptr;
  double* est_d = nullptr;
  int* reduce_done = nullptr;  // per pole: finished reduction workgroups of the round (zeroed workspace)
  double2* part_dots = nullptr;
  double* part_norm = nullptr;
  double* part_misc = nullptr;
  // host
  // per slot and pole: (round << 8) | flag, written by k_arnoldi into
  // host-coherent pinned memory and polled by the host
  unsigned long long* ftag_h = nullptr;
  unsigned long long* ftag_hd = nullptr;  // its device address
  unsigned long long seq = 0;             // rounds launched (the tags)
  double* est_h = nullptr;
  int* active_h = nullptr;
  double* misc_h = nullptr;
  std::vector<void*> uptr_h;
  std::vector<int> fixed;
  std::vector<double> relres;
  std::vector<int> iters;
  bool medium_set = false;
  int guess_mode = HP_GUESS_ZERO;
  bool prev_valid = false;        // X holds every pole's solution of the previous step
  std::vector<int> accepted;      // per pole: the last step started from a guess
  c128* guess_r = nullptr;        // per pole: residual of its guess (allocated on first use)
  double* guess_part = nullptr;   // per pole: partial sums of |r0|^2
  c128* guess_x = nullptr;        // per pole: physical previous-step solution (first use)
  double* guess_rpart = nullptr;  // per pole: partial norms of S_x r0
  double* guess_part_h = nullptr; // pinned copy (+1 slot: ||w||)
  // kernel timing
  int prof = 0;  // bit c set: launches of kernel class c are timed
  int prof_every = 1;              // time every prof_every-th launch of a class
  long prof_seen[HP_K_COUNT] = {};  // launches of each class since hp_profile
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<int> ev_cls;
  std::vector<double> ev_bytes;
  long prof_n[HP_K_COUNT]{};
  double prof_ms[HP_K_COUNT]{}, prof_b[HP_K_COUNT]{};
  long prof_nall[HP_K_COUNT]{};     // every launch of an enabled class, timed or not
  double prof_ball[HP_K_COUNT]{};   // ... and its algorithmic bytes
  std::vector<int> m_h;  // Arnoldi columns per pole (host mirror)
  std::vector<double> incons;  // eps kappa(M_k) per pole
  c128 phase{}, rinf_phase{};  // e^{-iK}, e^{-iK} r_inf
  double loss_coef = 0.0;      // k0 dz / (2 n0)
  int form = HP_FORM_EXP;      // what the pole table approximates and how a step uses it
  int substeps = 1;            // RK4 substeps per step (pseudo-differential form)
  c128* rk = nullptr;          // stage result, stage input, running sum (allocated by hp_set_form)
  // learned initial guesses (HP_GUESS_LEARNED): the net, poles per forward pass, and the
  // buffers of one step's guesses (set-up by hp_set_guess_net)
  hp_unet net = nullptr;
  int net_chunk = 0;
  c128* lg_fields = nullptr;   // y_k = M_k^-1 w [K], guesses x0_k [K], net corrections t [chunk]
  float *lg_in = nullptr, *lg_out = nullptr;
  double* lg_scal = nullptr;
  std::vector<double> lg_feat;  // per pole: asinh(Re b_k), asinh(Im b_k)
  double* n2copy = nullptr;    // the medium of the last hp_set_medium (the net's V plane reads it)
  void* scratch = nullptr;     // this device's address of the library's static scratch (no-alloc calls)
  // absorbing layers (hp_set_pml): padded eigenvector matrices Q, Q^-1 [N][N], eigenvalues [N],
  // the stretched stencil's node factors a2, a1 [N], one field per pole for the dense stages,
  // and the partial inner products of the medium pass
  bool pml = false;
  double pml_sigma = 0.0;
  char* pml_mem = nullptr;
  c128 *pml_q = nullptr, *pml_qi = nullptr, *pml_lam = nullptr, *pml_a2 = nullptr, *pml_a1 = nullptr;
  c128* pml_s = nullptr;
  c128* pml_shared = nullptr;  // two fields: the first round's pole-independent products
  double2* pml_part = nullptr;
  std::string scratch_err;
  std::string err;
};

namespace {
void scratch_setup(hp_plan p);
}

namespace {

int fail(hp_plan p, int code, const std::string& msg) {
  if (p)
    p->err = msg;
  else
    g_thread_error = msg;
  return code;
}

int hip_fail(hp_plan p, hipError_t e, const char* where) {
  return fail(p, HP_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HPCHK(expr)                                      \
  do {                                                   \
    hipError_t e_ = (expr);                              \
    if (e_ != hipSuccess) return hip_fail(p, e_, #expr); \
  } while (0)

// Bracket a launch with events when timing is on.
// bytes < 0: the launch's bytes are not known yet (a round's kernels skip the
// poles that turn out to have finished in the round before); *slot receives the
// timed launch's index (-1 if untimed) and prof_settle() adds the bytes later.
struct Prof {
  hp_plan p;
  int cls;
  double bytes;
  bool on;
  long* slot;
  Prof(hp_plan p_, int c, double b, long* slot_ = nullptr)
      : p(p_), cls(c), bytes(b), on(((p_->prof >> c) & 1) != 0), slot(slot_) {
    if (slot) *slot = -1;
    if (p->prof) {  // while profiling, every class's launches and bytes are counted
      p->prof_nall[c] += 1;
      if (b >= 0) p->prof_ball[c] += b;
    }
    if (!on) return;
    on = (p->prof_seen[c]++ % p->prof_every) == 0;
    if (!on) return;
    if (p->ev_used + 2 > p->ev_pool.size()) {
      for (int i = 0; i < 256; ++i) {
        hipEvent_t e;
        // timing only: no system-scope fence (the events order nothing the host reads)
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return;
        p->ev_pool.push_back(e);
      }
    }
    (void)hipEventRecord(p->ev_pool[p->ev_used], p->stream);
  }
  ~Prof() {
    if (!on || p->ev_used + 2 > p->ev_pool.size()) return;
    (void)hipEventRecord(p->ev_pool[p->ev_used + 1], p->stream);
    p->ev_used += 2;
    p->ev_cls.push_back(cls);
    if (slot) *slot = (long)p->ev_bytes.size();
    p->ev_bytes.push_back(bytes >= 0 ? bytes : 0.0);
  }
};

// The bytes of a launch made with deferred bytes (Prof with b < 0).
void prof_settle(hp_plan p, int cls, long slot, double bytes) {
  if (!p->prof) return;
  p->prof_ball[cls] += bytes;
  if (slot >= 0 && slot < (long)p->ev_bytes.size()) p->ev_bytes[slot] = bytes;
}

// grid sizes with a compiled transform: 2^k (64..2048) and 3 * 2^k (192..1536)
bool fft_size(int n) {
  if (n < 64 || n > 2048) return false;
  if ((n & (n - 1)) == 0) return true;
  const int m = n / 3;
  return n % 3 == 0 && (m & (m - 1)) == 0 && m >= 64;
}

std::string validate(const hp_plan_desc* d) {
  if (!d) return "desc is NULL";
  if (!fft_size(d->nx) || !fft_size(d->ny)) return "nx, ny must be 64, 128, 192, 256, 384, 512, 768, 1024, 1536 or 2048";
  if (d->ncomp != 1 && d->ncomp != 2) return "ncomp must be 1 or 2";
  if (d->precision != HP_FP64 && d->precision != HP_MIXED && d->precision != HP_MIXED64)
    return "precision must be HP_FP64, HP_MIXED or HP_MIXED64";
  if (!(d->dx > 0) || !(d->dy > 0) || !(d->k0 > 0) || !(d->n0 > 0) || !(d->dz > 0)) return "dx, dy, k0, n0, dz must be > 0";
  if (d->npoles < 1 || d->npoles > HP_MAXPOLES - 4) return "npoles must be in [1, 60]";
  if (!d->poles || !d->residues) return "poles/residues are NULL";
  if (!d->d2 || !d->d1) return "stencil coefficients are NULL";
  if (d->edge_width < 6) return "edge_width must be >= 6";
  if (d->nx < 2 * d->edge_width + 14 || d->ny < 2 * d->edge_width + 14) return "grid too small for the edge layer";
  if (!(d->edge_eta >= 0)) return "edge_eta must be >= 0";
  if (!(d->tol > 0)) return "tol must be > 0";
  if (d->restart < 1 || d->restart > HP_MAXM) return "restart must be in [1, 64]";
  if (d->max_cycles < 1) return "max_cycles must be >= 1";
  return "";
}

// Carve (or size) the workspace.  Layout is identical in both passes.
void layout(hp_plan p, Ws& w) {
  const hp_plan_desc& d = p->d;
  const size_t es = p->mixed ? sizeof(c64) : sizeof(c128);
  const size_t cs = (p->mixed && !p->mixed64) ? sizeof(c64) : sizeof(c128);  // transform arithmetic
  const size_t fn = p->fieldn;
  const int K = d.npoles, M = d.restart;
  p->mu_x = w.take<double>(d.nx);
  p->mu_y = w.take<double>(d.ny);
  p->tw_x = w.take<char>((d.nx + d.nx / 2 + 1) * cs);
  p->tw_y = w.take<char>((d.ny + d.ny / 2 + 1) * cs);
  p->tw64_x = w.take<c128>(d.nx + d.nx / 2 + 1);
  p->coef = w.take<double>((d.ncomp == 2 ? 6 : 1) * p->geo.fsz);
  p->coef_scratch = w.take<double>((d.ncomp == 2 ? 2 : 1) * p->geo.fsz);
  p->coef_f = w.take<float>((p->mixed && !p->mixed64) ? (d.ncomp == 2 ? 6 : 1) * p->geo.fsz : 1);
  p->n2copy = w.take<double>(p->geo.fsz);
  p->U = w.take<char>((size_t)K * (M + 1) * fn * es);
  p->Z = w.take<char>((size_t)K * M * fn * es);
  p->P = w.take<char>((size_t)K * fn * es);
  p->DZ = w.take<char>((d.ncomp == 2 ? (size_t)K : 1) * fn * es);
  p->bR = w.take<char>(fn * es);
  p->tmpR = w.take<char>(fn * es);
  p->X = w.take<c128>((size_t)K * fn);
  p->tmp1 = w.take<c128>(fn);
  p->tmp2 = w.take<c128>(fn);
  p->reduce_done = w.take<int>(HP_MAXPOLES);  // inside the range cleared at creation
  p->st = w.take<PoleState>(K);
  p->st_scratch = w.take<PoleState>(1);
  p->uptr = w.take<void*>((size_t)K * (HP_MAXM + 1));
  p->uptr_scratch = w.take<void*>(HP_MAXM + 1);
  p->active_d = w.take<int>(3 * HP_MAXPOLES);
  p->est_d = w.take<double>(HP_MAXPOLES);
  p->part_dots = w.take<double2>((size_t)K * (HP_MAXM + 1) * 2 * p->napplyblk);
  p->part_norm = w.take<double>((size_t)K * p->nupdblk);
  p->part_misc = w.take<double>(std::max((size_t)p->nrowblk * d.ncomp, (size_t)p->nopblk) + 64);
}

void derive(hp_plan p) {
  const hp_plan_desc& d = p->d;
  p->mixed = d.precision == HP_MIXED || d.precision == HP_MIXED64;
  p->mixed64 = d.precision == HP_MIXED64;
  p->geo.nx = d.nx;
  p->geo.ny = d.ny;
  p->geo.ncomp = d.ncomp;
  p->geo.fsz = (size_t)d.nx * d.ny;
  p->fieldn = p->geo.fsz * d.ncomp;
  const int rpw = 256 / (d.nx / 8) > 0 ? 256 / (d.nx / 8) : 1;
  p->nrowblk = (d.ny - 1 + rpw - 1) / rpw;
  p->napplyblk = p->mixed ? row_apply_parts<float>(p->geo) : row_apply_parts<double>(p->geo);
  p->nupdblk = update_blocks(p->fieldn);
  p->nopblk = op_blocks(p->geo);
  const double s = 1.0 / ((d.k0 * d.n0) * (d.k0 * d.n0));
  for (int m = 0; m < 7; ++m) {
    p->sc.c2x[m] = s * d.d2[m] / (d.dx * d.dx);
    p->sc.c2y[m] = s * d.d2[m] / (d.dy * d.dy);
  }
  for (int m = 0; m < 6; ++m) {
    p->sc.d1x[m] = d.d1[m] / d.dx;
    p->sc.d1y[m] = d.d1[m] / d.dy;
  }
}

std::vector<double> mu_table(int n, double h, const double* c, double s) {
  std::vector<double> mu(n, 0.0);
  for (int q = 1; q < n; ++q) {
    double sym = c[0];
    for (int m = 1; m < 7; ++m) sym += 2.0 * c[m] * cos(m * M_PI * q / n);
    mu[q] = s * sym / (h * h);
  }
  return mu;
}

// FFT twiddles exp(-2 pi i m / n), m < n, then sin(pi j / n), j = 0..n/2, in
// the real parts (the DST-I pre-processing factors).
template <typename T>
std::vector<cx<T>> twiddles(int n) {
  std::vector<cx<T>> t(n + n / 2 + 1);
  for (int m = 0; m < n; ++m) {
    const double a = -2.0 * M_PI * (double)m / (double)n;
    t[m] = mk<T>((T)cos(a), (T)sin(a));
  }
  for (int j = 0; j <= n / 2; ++j) t[n + j] = mk<T>((T)sin(M_PI * (double)j / (double)n), (T)0);
  return t;
}

std::complex<double> rat(hp_plan p, double z) {
  std::complex<double> r(p->d.r_inf.re, p->d.r_inf.im);
  for (int k = 0; k < p->d.npoles; ++k) {
    std::complex<double> a(p->residues[k].re, p->residues[k].im), b(p->poles[k].re, p->poles[k].im);
    r += a / (z - b);
  }
  return r;
}

template <typename C>
int upload_tables(hp_plan p) {
  const hp_plan_desc& d = p->d;
  const double s = 1.0 / ((d.k0 * d.n0) * (d.k0 * d.n0));
  auto mx = mu_table(d.nx, d.dx, p->c2, s), my = mu_table(d.ny, d.dy, p->c2, s);
  HPCHK(hipMemcpy(p->mu_x, mx.data(), mx.size() * sizeof(double), hipMemcpyHostToDevice));
  HPCHK(hipMemcpy(p->mu_y, my.data(), my.size() * sizeof(double), hipMemcpyHostToDevice));
  auto tx = twiddles<C>(d.nx), ty = twiddles<C>(d.ny);
  auto t64 = twiddles<double>(d.nx);
  HPCHK(hipMemcpy(p->tw_x, tx.data(), tx.size() * sizeof(cx<C>), hipMemcpyHostToDevice));
  HPCHK(hipMemcpy(p->tw_y, ty.data(), ty.size() * sizeof(cx<C>), hipMemcpyHostToDevice));
  HPCHK(hipMemcpy(p->tw64_x, t64.data(), t64.size() * sizeof(c128), hipMemcpyHostToDevice));
  return HP_OK;
}

int upload_state(hp_plan p) {
  std::vector<PoleState> h(p->d.npoles);
  for (int k = 0; k < p->d.npoles; ++k) {
    memset(&h[k], 0, sizeof(PoleState));
    h[k].bk = mk(p->poles[k].re, p->poles[k].im);
    h[k].ak = mk(p->residues[k].re, p->residues[k].im);
    h[k].fixed = p->fixed.empty() ? 0 : p->fixed[k];
    h[k].incons = p->incons[k];
  }
  HPCHK(hipMemcpyAsync(p->st, h.data(), h.size() * sizeof(PoleState), hipMemcpyHostToDevice, p->stream));
  return HP_OK;
}

// coefficient planes in the working precision
template <typename T>
const T* coef_as(hp_plan p);
template <>
const double* coef_as<double>(hp_plan p) {
  return p->coef;
}
template <>
const float* coef_as<float>(hp_plan p) {
  return p->coef_f;
}

template <typename T>
cx<T>* fld(void* base, size_t idx, size_t fieldn) {
  return reinterpret_cast<cx<T>*>(base) + idx * fieldn;
}

int upload_uptr(hp_plan p) {
  hipError_t e = hipMemcpyAsync(p->uptr, p->uptr_h.data(), p->uptr_h.size() * sizeof(void*), hipMemcpyHostToDevice,
                                p->stream);
  if (e != hipSuccess) return hip_fail(p, e, "upload uptr");
  return HP_OK;
}

// Cycle tolerance relative to the cycle's starting residual: complex64
// transforms stop each cycle at 1e-5 (the FP64 true residual then restarts
// the solve); with FP64 transforms a cycle runs to tol like FP64 mode.
double inner_rtol(hp_plan p) { return (p->mixed && !p->mixed64) ? kInnerRtolMixed : 0.0; }

// Call fn<storage, compute> for the plan's precision.
#define HP_BY_PRECISION(p, fn, ...)                                                                   \
  ((p)->mixed ? ((p)->mixed64 ? fn<float, double>(__VA_ARGS__) : fn<float, float>(__VA_ARGS__)) \
              : fn<double, double>(__VA_ARGS__))

// One step: the lockstep Arnoldi iterations of all poles, pipelined one deep:
// iteration j+1 is enqueued before the flags of iteration j are read, and a
// pole that finished in iteration j skips itself in iteration j+1 (its flag is
// set on the device).  Cycle ends that need the true residual (mixed
// precision, restarts, flag 3) are handled on the host between launches.
// X_k += the current cycle's terms; afterwards X_k is pole k's whole solution.
template <typename T>
void fold(hp_plan p, int k) {
  const size_t fn = p->fieldn;
  launch_accum<T>(p->X + (size_t)k * fn, fld<T>(p->Z, (size_t)k * p->d.restart, fn), fn, p->st, k, p->geo,
                  p->stream);
  launch_mark_folded(p->st, k, 1, p->stream);
}

// Absorbing layers: z = sigma_m M_k^-1 u_m for the poles list[0..n) by the
// eigen route of the Sylvester equation, Q [(Q^-1 u Q^-T) / (lam_p + lam_q - b_k)] Q^T,
// in four dense stages through the pole's P field and its own scratch field.
void pml_prec(hp_plan p, const PoleState* st, const int* list, int n, int* active_out, PmlRef in, PmlRef out,
              c128* bufA, c128* bufB) {
  const int N = p->d.nx;
  const size_t fn = p->fieldn;
  const PmlRef a{nullptr, bufA, fn, 0}, b{nullptr, bufB, fn, 0};
  const int v = p->geo.col_variant;  // the launch variant picks the dense stages' form
  const int nc = p->d.ncomp;
  launch_pml_gemm(v, true, 0, p->pml_qi, in, a, st, list, n, active_out, p->pml_lam, N, nc, p->stream);
  launch_pml_gemm(v, false, 1, p->pml_qi, a, b, st, list, n, nullptr, p->pml_lam, N, nc, p->stream);
  launch_pml_gemm(v, true, 0, p->pml_q, b, a, st, list, n, nullptr, p->pml_lam, N, nc, p->stream);
  launch_pml_gemm(v, false, 2, p->pml_q, a, out, st, list, n, nullptr, p->pml_lam, N, nc, p->stream);
}

// Floating-point operations of one pole's four dense stages: 8 n^3 per complex
// product of n x n matrices, n = N - 1 unknowns per axis, for each component.
double pml_flops(hp_plan p) {
  const double n = p->d.nx - 1.0;
  return 4.0 * 8.0 * n * n * n * p->d.ncomp;
}

// Guess residuals for several poles at once: one buffer and one set of
// partial sums per pole (allocated on first use, freed with the plan).
int ensure_guess_buffers(hp_plan p, bool prev) {
  const int K = p->d.npoles;
  if (!p->guess_r) {
    HPCHK(hipMalloc(&p->guess_r, (size_t)K * p->fieldn * sizeof(c128)));
    HPCHK(hipMalloc(&p->guess_part, (size_t)K * p->nopblk * sizeof(double)));
    HPCHK(hipMalloc(&p->guess_rpart, (size_t)K * p->nrowblk * p->d.ncomp * sizeof(double)));
    HPCHK(hipHostMalloc(&p->guess_part_h, ((size_t)K * p->nopblk + 1) * sizeof(double)));
  }
  if (prev && !p->guess_x) HPCHK(hipMalloc(&p->guess_x, (size_t)K * p->fieldn * sizeof(c128)));
  return HP_OK;
}

// New cycles for the poles rs[a] from the FP64 residuals held in guess_r slot
// rj[a]: S_x r into each pole's first basis vector, then one cycle start for
// all of them (their X_k is the solution so far).
template <typename T, typename C>
int restart_from_residuals(hp_plan p, const std::vector<int>& rs, const std::vector<int>& rj) {
  const size_t fn = p->fieldn;
  const int nr = (int)rs.size();
  const size_t rblk = (size_t)p->nrowblk * p->d.ncomp;
  const size_t ustride = (size_t)(p->d.restart + 1) * fn;
  {
    Prof pr(p, HP_K_ROW_FWD, nr * (double)(p->d.nx - 1) * (p->d.ny - 1) * p->d.ncomp * (16.0 + sizeof(cx<T>)));
    if (p->pml)
      launch_pml_copy(p->guess_r, fn, rj.data(), reinterpret_cast<c128*>(p->U), ustride, rs.data(), nr,
                      p->guess_rpart, rblk, (int)rblk, p->d.nx, p->d.ncomp, p->stream);
    else
      launch_row_fwd_batch<T, C>(p->guess_r, fn, rj.data(), fld<T>(p->U, 0, fn), ustride, rs.data(), nr,
                                 p->guess_rpart, rblk, reinterpret_cast<const cx<C>*>(p->tw_x), p->geo, p->stream);
  }
  bool changed = false;
  for (int k : rs) {
    void* u0 = fld<T>(p->U, (size_t)k * (p->d.restart + 1), fn);
    if (p->uptr_h[(size_t)k * (HP_MAXM + 1)] != u0) {
      p->uptr_h[(size_t)k * (HP_MAXM + 1)] = u0;
      changed = true;
    }
  }
  if (changed) {
    int rc = upload_uptr(p);
    if (rc) return rc;
  }
  // the list goes through pinned slot 2; the host wrote it only after the
  // caller's last synchronisation, and no copy from it is pending
  int* list_h = p->active_h + 2 * HP_MAXPOLES;
  int* list_d = p->active_d + 2 * HP_MAXPOLES;
  for (int a = 0; a < nr; ++a) list_h[a] = rs[a];
  HPCHK(hipMemcpyAsync(list_d, list_h, nr * sizeof(int), hipMemcpyHostToDevice, p->stream));
  launch_cycle_init(p->st, list_d, nr, p->guess_rpart, (int)rblk, 0, p->d.tol, inner_rtol(p), p->stream, rblk, 1);
  return HP_OK;
}

// End of a cycle for the poles chk[a] (one flight): fold each cycle into X_k,
// then the FP64 true residuals r = w - A_k S_x X_k of all of them (residuals in
// guess_r slot a) with one synchronisation; res[a] = ||r||, *beta0 = ||w||.
template <typename T, typename C>
int check_poles(hp_plan p, const std::vector<int>& chk, const c128* w, int beta_pole, std::vector<double>& res,
                double* beta0) {
  int rc = ensure_guess_buffers(p, true);
  if (rc) return rc;
  const size_t fn = p->fieldn;
  const int n = (int)chk.size();
  const double U1 = (double)(p->d.nx - 1) * (p->d.ny - 1) * p->d.ncomp;
  double bytes = 0.0;
  std::vector<c128> shifts(n);
  for (int a = 0; a < n; ++a) {
    bytes += U1 * (sizeof(cx<T>) * (double)p->m_h[chk[a]] + 16.0 * 7);
    shifts[a] = mk(p->poles[chk[a]].re, p->poles[chk[a]].im);
  }
  {
    Prof pr(p, HP_K_RESIDUAL, bytes);
    launch_accum_batch<T>(p->X, fn, fld<T>(p->Z, 0, fn), (size_t)p->d.restart * fn, fn, p->st, chk.data(), n,
                          p->geo, p->stream);
    launch_mark_list(p->st, chk.data(), n, p->stream);  // X_k now holds the whole solution
    if (p->pml) {
      // X_k is physical already: gather the listed poles' accumulators
      for (int a = 0; a < n; ++a)
        HPCHK(hipMemcpyAsync(p->guess_x + (size_t)a * fn, p->X + (size_t)chk[a] * fn, fn * sizeof(c128),
                             hipMemcpyDeviceToDevice, p->stream));
      if (!launch_pml_residual(p->guess_x, fn, w, p->guess_r, fn, p->coef, p->pml_a2, p->pml_a1, p->sc,
                               shifts.data(), n, p->guess_part, p->nopblk, p->nopblk, p->d.nx, p->d.ncomp, p->stream))
        return fail(p, HP_EINVAL, "absorbing-layer residual: the grid does not tile by 64 x 16");
    } else {
      launch_row_inv_batch<double>(p->X, fn, chk.data(), n, p->guess_x, fn, p->tw64_x, p->geo, tile_width<T>(),
                                   p->stream);
      launch_apply_op_batch(p->guess_x, fn, w, p->guess_r, fn, p->coef, shifts.data(), n, p->sc, p->geo,
                            p->guess_part, p->nopblk, p->stream);
    }
  }
  HPCHK(hipMemcpyAsync(p->guess_part_h, p->guess_part, (size_t)n * p->nopblk * sizeof(double),
                       hipMemcpyDeviceToHost, p->stream));
  HPCHK(hipMemcpyAsync(p->guess_part_h + (size_t)n * p->nopblk, &p->st[beta_pole].beta0, sizeof(double),
                       hipMemcpyDeviceToHost, p->stream));
  HPCHK(hipStreamSynchronize(p->stream));
  res.assign(n, 0.0);
  for (int a = 0; a < n; ++a) {
    double s2 = 0.0;
    for (int b = 0; b < p->nopblk; ++b) s2 += p->guess_part_h[(size_t)a * p->nopblk + b];
    res[a] = sqrt(s2);
  }
  *beta0 = p->guess_part_h[(size_t)n * p->nopblk];
  return HP_OK;
}

// Judge the guesses of the poles in cand: pole cand[j]'s guess is held in its
// X accumulator as S_x x0 (x0[j], physical complex128, given as well, or NULL:
// X then comes from the previous step).  r0 = w - A_k x0 in FP64 for all of
// them, one synchronisation, then every pole with ||r0|| < ||w|| starts its
// first cycle from r0 with X_k as the solution so far (done[j]: already within
// tol, no Arnoldi step); the others keep the zero start.  acc[j] = 1 when used.
template <typename T, typename C>
int start_from_guesses(hp_plan p, const std::vector<int>& cand, const c128* w, const c128* const* x0,
                       const int* st_first, std::vector<int>& acc, std::vector<char>& done,
                       std::vector<double>& rel) {
  const size_t fn = p->fieldn;
  const int nc = (int)cand.size();
  // previous-step candidates have no explicit guess (a NULL entry): their x0
  // is S_x^-1 X_k; when all are such, every kernel covers all of them at once
  bool prev = true;
  for (int j = 0; j < nc; ++j) prev = prev && !(x0 && x0[j]);
  int rc = ensure_guess_buffers(p, prev);
  if (rc) return rc;
  if (prev) {
    // previous-step solutions: all candidates in one launch per kernel
    std::vector<c128> shifts(nc);
    for (int j = 0; j < nc; ++j) shifts[j] = mk(p->poles[cand[j]].re, p->poles[cand[j]].im);
    launch_row_inv_batch<double>(p->X, fn, cand.data(), nc, p->guess_x, fn, p->tw64_x, p->geo, tile_width<T>(),
                                 p->stream);
    launch_apply_op_batch(p->guess_x, fn, w, p->guess_r, fn, p->coef, shifts.data(), nc, p->sc, p->geo,
                          p->guess_part, p->nopblk, p->stream);
  } else {
    for (int j = 0; j < nc; ++j) {
      const int k = cand[j];
      const c128* xp = x0 ? x0[j] : nullptr;
      if (!xp) {
        launch_row_inv<double>(p->X + (size_t)k * fn, p->tmp1, p->tw64_x, p->geo, tile_width<T>(), p->stream);
        xp = p->tmp1;
      }
      launch_apply_op(xp, w, p->guess_r + (size_t)j * fn, p->coef, mk(p->poles[k].re, p->poles[k].im), p->sc,
                      p->geo, p->guess_part + (size_t)j * p->nopblk, p->stream);
    }
  }
  HPCHK(hipMemcpyAsync(p->guess_part_h, p->guess_part, (size_t)nc * p->nopblk * sizeof(double),
                       hipMemcpyDeviceToHost, p->stream));
  HPCHK(hipMemcpyAsync(p->guess_part_h + (size_t)nc * p->nopblk, &p->st[*st_first].beta0, sizeof(double),
                       hipMemcpyDeviceToHost, p->stream));
  HPCHK(hipStreamSynchronize(p->stream));
  const double beta0 = p->guess_part_h[(size_t)nc * p->nopblk];
  static const int one = 1;
  acc.assign(nc, 0);
  done.assign(nc, 0);
  rel.assign(nc, 0.0);
  std::vector<int> rs, rj;  // poles that restart from their guess residual, and their slots
  for (int j = 0; j < nc; ++j) {
    const int k = cand[j];
    double s2 = 0.0;
    for (int b = 0; b < p->nopblk; ++b) s2 += p->guess_part_h[(size_t)j * p->nopblk + b];
    const double r0 = sqrt(s2);
    rel[j] = beta0 > 0 ? r0 / beta0 : 0.0;
    if (!(r0 < beta0)) continue;  // also rejects NaN
    acc[j] = 1;
    if (r0 <= p->d.tol * beta0) {
      done[j] = 1;
      HPCHK(hipMemcpyAsync(&p->st[k].has_x, &one, sizeof(int), hipMemcpyHostToDevice, p->stream));
      continue;
    }
    rs.push_back(k);
    rj.push_back(j);
  }
  return rs.empty() ? HP_OK : restart_from_residuals<T, C>(p, rs, rj);
}

template <typename T, typename C>
int run_poles(hp_plan p, const c128* w, const std::vector<int>& subset, bool* noconv_out,
              const c128* const* x0 = nullptr, bool use_prev = false, int first = 1) {
  const hp_plan_desc& d = p->d;
  const size_t fn = p->fieldn;
  const int K = d.npoles, M = d.restart;
  const cx<C>* twx = reinterpret_cast<const cx<C>*>(p->tw_x);
  const cx<C>* twy = reinterpret_cast<const cx<C>*>(p->tw_y);
  cx<T>* bR = reinterpret_cast<cx<T>*>(p->bR);
  const double es = (double)sizeof(cx<T>);
  const double U1 = (double)(d.nx - 1) * (d.ny - 1) * d.ncomp;  // unknowns of one field
  const double planes = d.ncomp == 2 ? 6.0 : 1.0;
  p->m_h.assign(K, 0);
  // shared first Krylov vector: S_x w (every pole's right-hand side is w)
  {
    Prof pr(p, HP_K_ROW_FWD, U1 * (16.0 + es));
    if (p->pml) {
      const int zero = 0;
      launch_pml_copy(w, 0, &zero, reinterpret_cast<c128*>(bR), 0, &zero, 1, p->part_misc, 0, p->nrowblk * d.ncomp,
                      d.nx, d.ncomp, p->stream);
    } else {
      launch_row_fwd<T, C>(w, bR, p->part_misc, twx, p->geo, p->stream);
    }
  }
  bool changed = false;
  for (int k : subset) {
    if (p->uptr_h[(size_t)k * (HP_MAXM + 1)] != (void*)bR) {
      p->uptr_h[(size_t)k * (HP_MAXM + 1)] = bR;
      changed = true;
    }
  }
  if (changed) {
    int rc = upload_uptr(p);
    if (rc) return rc;
  }
  int* act0 = p->active_h + 2 * HP_MAXPOLES;  // pinned slot for the initial list
  const int ns = (int)subset.size();
  for (int a = 0; a < ns; ++a) act0[a] = subset[a];
  HPCHK(hipMemcpyAsync(p->active_d, act0, ns * sizeof(int), hipMemcpyHostToDevice, p->stream));
  launch_cycle_init(p->st, p->active_d, ns, p->part_misc, p->nrowblk * d.ncomp, first, d.tol, inner_rtol(p),
                    p->stream);
  std::vector<char> live(K, 0);
  for (int k : subset) live[k] = 1;
  std::vector<long> since(K, 0);  // iteration at which the pole's current cycle started
  std::vector<int> cycles(K, 0), done_m(K, 0);
  p->relres.assign(K, -1.0);
  double beta0 = -1.0;
  bool noconv = false;
  int nonfinite = -1;  // a pole whose Krylov space met a NaN or Inf
  const size_t zsp = (size_t)M * fn, zsi = fn, psp = fn, dzsp = (d.ncomp == 2) ? fn : 0;
  cx<T>* Zb = reinterpret_cast<cx<T>*>(p->Z);
  cx<T>* Pb = reinterpret_cast<cx<T>*>(p->P);
  cx<T>* DZb = reinterpret_cast<cx<T>*>(p->DZ);
  const cx<T>* const* up = reinterpret_cast<const cx<T>* const*>(p->uptr);
  struct Flight {
    std::vector<int> poles;
    int slot;
    long iter;
    unsigned long long seq;  // tag of the round's flags
    std::vector<int> ms;     // per pole: its Arnoldi index in the round
    std::vector<char> sh;    // per pole: its first basis vector is the shared S_x w
    long pslot[3];           // timed-launch slots of the column pass, row pass and update
    bool shared;             // absorbing layers: the round shared its first two dense products
  };
  // Algorithmic bytes of a round's column pass, row pass and update over the
  // poles that did the step (the others skipped themselves on the device), each
  // distinct field counted once per launch: poles in the first cycle of the step
  // share one first basis vector (S_x w), which a launch must read once.
  auto settle = [&](const Flight& f, const std::vector<char>& worked) {
    if (!p->prof) return;
    double col = 0.0, row = 0.0, upd = 0.0;
    int shared = 0, shared_m0 = 0, nw = 0;
    const double outs = d.ncomp == 2 ? 2.0 : 1.0;  // z (and D1y z)
    for (size_t a = 0; a < f.poles.size(); ++a) {
      if (!worked[a]) continue;
      const int mm = f.ms[a];
      ++nw;
      col += 1.0 + outs;                                         // u_m read, z (+ D1y z) written
      row += (d.ncomp == 2 && !p->pml ? 3.0 : 2.0) + (mm + 1.0);  // z (+ D1y z), p, u_0..u_m
      upd += 1.0 + (mm + 1.0) + 1.0 + (mm > 0 ? 1.0 : 0.0);     // p, u_0..u_m, u_{m+1}, rewritten u_m
      if (f.sh[a]) {
        ++shared;
        if (mm == 0) ++shared_m0;
      }
    }
    const double dup = shared > 0 ? shared - 1.0 : 0.0, dup0 = shared_m0 > 0 ? shared_m0 - 1.0 : 0.0;
    // absorbing layers: the dense stages count floating-point operations (a shared round:
    // two products once, two per pole)
    const double pf = f.shared ? (nw ? (2.0 + 2.0 * nw) / 4.0 : 0.0) : (double)nw;
    prof_settle(p, p->pml ? HP_K_PML : HP_K_COL, f.pslot[0], p->pml ? pf * pml_flops(p) : U1 * es * (col - dup0));
    prof_settle(p, HP_K_ROW_APPLY, f.pslot[1], nw ? U1 * es * (row - dup) + (U1 / d.ncomp) * 8.0 * planes : 0.0);
    prof_settle(p, HP_K_UPDATE, f.pslot[2], U1 * es * (upd - dup));
  };
  // initial guesses (explicit, or the previous step's solutions held in X)
  p->accepted.assign(K, 0);
  {
    std::vector<int> cand;
    std::vector<const c128*> gx;
    for (int k : subset) {
      const c128* g = x0 ? x0[k] : nullptr;
      if (!g && !use_prev) continue;
      if (g)
        launch_row_fwd<double>(g, p->X + (size_t)k * fn, p->part_misc, p->tw64_x, p->geo, p->stream,
                               tile_width<T>());
      cand.push_back(k);
      gx.push_back(g);
    }
    if (!cand.empty()) {
      std::vector<int> acc;
      std::vector<char> done;
      std::vector<double> rel;
      int rc = start_from_guesses<T, C>(p, cand, w, gx.data(), &subset[0], acc, done, rel);
      if (rc) return rc;
      for (size_t j = 0; j < cand.size(); ++j) {
        p->accepted[cand[j]] = acc[j];
        if (done[j]) {
          live[cand[j]] = 0;
          p->relres[cand[j]] = rel[j];
        }
      }
    }
  }
  std::vector<Flight> q;
  long next_iter = 0;
  auto launch_iter = [&](const std::vector<int>& poles) -> int {
    const int slot = (int)(next_iter & 1);
    const int na = (int)poles.size();
    int* ad = p->active_d + slot * HP_MAXPOLES;
    int maxm = 0;
    Flight fl{poles, slot, next_iter, 0, std::vector<int>(na), std::vector<char>(na), {-1, -1, -1}, false};
    for (int a = 0; a < na; ++a) {
      const int mk_ = (int)std::min<long>(next_iter - since[poles[a]], M - 1);
      maxm = std::max(maxm, mk_);
      fl.ms[a] = mk_;
      fl.sh[a] = p->uptr_h[(size_t)poles[a] * (HP_MAXM + 1)] == (void*)bR;
    }
    if (p->pml) {
      // absorbing layers: the dense stages (the first stores the list to ad),
      // then p = A_k z - ~v_m with the inner products, on physical fields
      c128* Zc = reinterpret_cast<c128*>(p->Z);
      c128* Pc = reinterpret_cast<c128*>(p->P);
      c128* const* uc = reinterpret_cast<c128* const*>(p->uptr);
      // a round in which every pole starts from the shared first basis vector shares
      // the first two dense products (matrix-core forms)
      bool shared = p->geo.col_variant != 0;
      for (int a = 0; a < na && shared; ++a) shared = fl.sh[a] && fl.ms[a] == 0;
      fl.shared = shared;
      {
        Prof pr(p, HP_K_PML, -1.0, &fl.pslot[0]);
        if (shared) {
          const int zero = 0, N = d.nx, nc = d.ncomp;
          c128* T1 = p->pml_shared;
          c128* T2 = p->pml_shared + fn;
          launch_pml_shared_setup(p->st_scratch, reinterpret_cast<c128**>(p->uptr_scratch),
                                  reinterpret_cast<const c128*>(bR), p->stream);
          launch_pml_gemm(p->geo.col_variant, true, 0, p->pml_qi,
                          PmlRef{reinterpret_cast<c128* const*>(p->uptr_scratch), nullptr, 0, 0},
                          PmlRef{nullptr, T1, 0, 0}, p->st_scratch, &zero, 1, nullptr, p->pml_lam, N, nc, p->stream);
          launch_pml_gemm(p->geo.col_variant, false, 0, p->pml_qi, PmlRef{nullptr, T1, 0, 0},
                          PmlRef{nullptr, T2, 0, 0}, p->st_scratch, &zero, 1, nullptr, p->pml_lam, N, nc, p->stream);
          launch_pml_gemm_divided(p->pml_q, PmlRef{nullptr, T2, 0, 0}, PmlRef{nullptr, Pc, fn, 0}, p->st,
                                  poles.data(), na, ad, p->pml_lam, N, nc, p->stream);
          launch_pml_gemm(p->geo.col_variant, false, 2, p->pml_q, PmlRef{nullptr, Pc, fn, 0},
                          PmlRef{nullptr, Zc, zsp, zsi}, p->st, poles.data(), na, nullptr, p->pml_lam, N, nc,
                          p->stream);
        } else {
          pml_prec(p, p->st, poles.data(), na, ad, PmlRef{uc, nullptr, 0, 0}, PmlRef{nullptr, Zc, zsp, zsi}, Pc,
                   p->pml_s);
        }
      }
      {
        Prof pr(p, HP_K_ROW_APPLY, -1.0, &fl.pslot[1]);
        launch_pml_apply(Zc, zsp, zsi, Pc, psp, uc, p->coef, p->pml_a2, p->pml_a1, p->sc, p->st, ad, na, p->pml_part,
                         d.nx, d.ncomp, p->stream);
      }
      {
        Prof pr(p, HP_K_SMALL, 0.0);
        launch_reduce_dots(p->pml_part, pml_apply_parts(d.nx), p->st, ad, na, maxm, p->reduce_done, p->stream);
      }
    } else {
      {
        // the column pass takes the list in its arguments and stores it to ad
        // for the kernels after it (no host-to-device copy per round)
        Prof pr(p, HP_K_COL, -1.0, &fl.pslot[0]);
        launch_col<T, C>(up, Zb, zsp, zsi, DZb, dzsp, p->st, poles.data(), na, ad, p->mu_x, p->mu_y, twy, p->geo,
                         p->sc, p->stream);
      }
      {
        Prof pr(p, HP_K_ROW_APPLY, -1.0, &fl.pslot[1]);
        launch_row_apply<T, C>(Zb, zsp, zsi, DZb, dzsp, Pb, psp, up, coef_as<C>(p), p->st, ad, na, p->part_dots,
                               twx, p->geo, p->sc, p->stream);
      }
      {
        Prof pr(p, HP_K_SMALL, 0.0);
        launch_reduce_dots(p->part_dots, p->napplyblk, p->st, ad, na, maxm, p->reduce_done, p->stream);
      }
    }
    {
      Prof pr(p, HP_K_UPDATE, -1.0, &fl.pslot[2]);
      launch_update<T>(Pb, psp, reinterpret_cast<cx<T>* const*>(p->uptr), p->st, ad, na, p->part_norm, p->nupdblk,
                       p->geo, p->stream);
    }
    {
      Prof pr(p, HP_K_SMALL, 0.0);
      // flags go straight to host memory, tagged with the round
      launch_arnoldi(p->st, ad, na, p->part_norm, p->nupdblk, M, p->ftag_hd + slot * HP_MAXPOLES, ++p->seq,
                     p->est_d, p->stream);
    }
    fl.seq = p->seq;
    q.push_back(std::move(fl));
    ++next_iter;
    return HP_OK;
  };
  auto live_list = [&]() {
    std::vector<int> v;
    for (int k = 0; k < K; ++k)
      if (live[k]) v.push_back(k);
    return v;
  };
  {
    std::vector<int> v = live_list();
    if (!v.empty()) {
      int rc = launch_iter(v);
      if (rc) return rc;
    }
  }
  while (!q.empty()) {
    if (q.size() < 2) {
      std::vector<int> v = live_list();
      if (!v.empty()) {
        int rc = launch_iter(v);
        if (rc) return rc;
      }
    }
    Flight f = q.front();
    q.erase(q.begin());
    // wait for the round's tags of the poles read below (every one of them
    // takes the step, so its k_arnoldi block writes the tag); should they not
    // arrive within a second the stream is drained and they must be there
    const volatile unsigned long long* ft = p->ftag_h + f.slot * HP_MAXPOLES;
    {
      const auto t0 = std::chrono::steady_clock::now();
      bool drained = false;
      for (int k : f.poles) {
        if (!live[k] || f.iter < since[k]) continue;
        while ((ft[k] >> 8) != f.seq) {
          if (drained) return fail(p, HP_EHIP, "round flags did not reach host memory");
          if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(1)) {
            HPCHK(hipStreamSynchronize(p->stream));
            drained = true;
          }
        }
      }
    }
    {
      // the poles that did this round's step: live then and in their current cycle
      std::vector<char> worked(f.poles.size());
      for (size_t a = 0; a < f.poles.size(); ++a) worked[a] = live[f.poles[a]] && f.iter >= since[f.poles[a]];
      settle(f, worked);
    }
    std::vector<int> chk;  // poles whose cycle ended and whose true residual decides
    for (int k : f.poles) {
      if (!live[k] || f.iter < since[k]) continue;
      const int flag = (int)(ft[k] & 0xff);
      if (flag == 0) continue;
      live[k] = 0;
      done_m[k] = (int)(f.iter - since[k] + 1);
      if (flag == 4) {  // the pole stopped itself; the other poles drain normally
        if (nonfinite < 0) nonfinite = k;
        continue;
      }
      const bool fixed = !p->fixed.empty() && p->fixed[k] > 0;
      // converged on the FP64 estimate; with absorbing layers the eigen-route
      // preconditioner's rounding (up to eps cond(Q)^2) lets the true residual decide
      if (fixed || (flag == 1 && !p->mixed && !p->pml)) {
        p->relres[k] = -1.0;
        continue;
      }
      // cycle ended without convergence (2), mixed precision, or flag 3
      p->m_h[k] = done_m[k];
      chk.push_back(k);
    }
    if (chk.empty()) continue;
    std::vector<double> res;
    int rc = check_poles<T, C>(p, chk, w, subset[0], res, &beta0);
    if (rc) return rc;
    std::vector<int> rs, rj;  // poles that start a new cycle from their residual
    for (size_t a = 0; a < chk.size(); ++a) {
      const int k = chk[a];
      done_m[k] = 0;
      const double rel = beta0 > 0 ? res[a] / beta0 : 0.0;
      p->relres[k] = rel;
      if (rel <= d.tol) continue;
      if (++cycles[k] >= d.max_cycles) {
        noconv = true;
        continue;
      }
      rs.push_back(k);
      rj.push_back((int)a);
    }
    if (rs.empty()) continue;
    rc = restart_from_residuals<T, C>(p, rs, rj);
    if (rc) return rc;
    for (int k : rs) {
      live[k] = 1;
      since[k] = next_iter;
    }
  }
  p->m_h = done_m;
  *noconv_out = noconv;
  HPCHK(hipGetLastError());
  if (nonfinite >= 0)
    return fail(p, HP_EINVAL, "pole " + std::to_string(nonfinite) +
                                  ": a NaN or Inf reached the GMRES solve (non-finite n2 or E_in, or n2 <= 0 "
                                  "for the vector operator)");
  return HP_OK;
}

// All poles' solves (Zbar - b_k I) x_k = w, then
// out = mask(loss_coef) * (phase sum_k a_k x_k + rinf_phase w).
template <typename T, typename C>
int solve_and_sum(hp_plan p, const c128* w, c128* out, c128 phase, c128 rinf_phase, double loss_coef,
                  const c128* const* x0, int first) {
  const hp_plan_desc& d = p->d;
  const int K = d.npoles;
  std::vector<int> all(K);
  for (int k = 0; k < K; ++k) all[k] = k;
  bool noconv = false;
  const bool use_prev = !x0 && p->guess_mode == HP_GUESS_PREV && p->prev_valid;
  int rc = run_poles<T, C>(p, w, all, &noconv, x0, use_prev, first);
  if (rc) return rc;
  {
    const double es = (double)sizeof(cx<T>);
    const double U1 = (double)(d.nx - 1) * (d.ny - 1) * d.ncomp;
    double terms = 0.0;
    for (int k = 0; k < K; ++k) terms += p->m_h[k];
    Prof pr(p, HP_K_FINAL, U1 * (es * terms + 32.0));
    if (p->pml)  // the layers absorb: no separate loss
      launch_pml_final(w, out, reinterpret_cast<c128*>(p->Z), (size_t)d.restart * p->fieldn, p->fieldn, p->X,
                       p->fieldn, p->st, K, phase, rinf_phase, d.nx, d.ncomp, p->stream);
    else
      launch_final<T>(w, out, reinterpret_cast<cx<T>*>(p->Z), (size_t)d.restart * p->fieldn, p->fieldn, p->X,
                      p->fieldn, p->st, K, phase, rinf_phase, loss_coef, d.edge_eta, d.edge_width, p->tw64_x,
                      p->geo, p->stream);
  }
  if (p->guess_mode == HP_GUESS_PREV) {  // keep the solutions as the next step's guesses
    launch_accum_batch<T>(p->X, p->fieldn, fld<T>(p->Z, 0, p->fieldn), (size_t)d.restart * p->fieldn, p->fieldn,
                          p->st, all.data(), K, p->geo, p->stream);
    launch_mark_folded(p->st, 0, K, p->stream);
    p->prev_valid = true;
  }
  HPCHK(hipGetLastError());
  return noconv ? HP_WARN_NOCONV : HP_OK;
}

// Pseudo-differential form (Sec. 2 eq. eq_barZfactor2 with the partial
// fractions of sqrt(1+z) of Sec. 3.2): `substeps` classical RK4 steps of
// h = dz / substeps for dw/dz = L(w), L(v) = i k0 n0 (r(Zbar) v - v).  Each
// stage is one lockstep solve of all poles whose final kernel yields L(v)
// directly (weights i k0 n0 on the solutions, i k0 n0 (r_inf - 1) on v, no
// loss); k_rk4_stage then forms the next stage's input and the running sum.
// The layer loss is applied after every substep.  Iteration counts run on
// over the stages of the step; the reported residual is the worst of the
// stages' true residuals where they were computed (else the last stage's
// estimate, as for the exponential form).
template <typename T, typename C>
int run_step_sqrt(hp_plan p, const c128* w, c128* out) {
  const hp_plan_desc& d = p->d;
  const size_t fn = p->fieldn;
  c128* Lb = p->rk;
  c128* vb = p->rk + fn;
  c128* acc = p->rk + 2 * fn;
  const double h = d.dz / p->substeps, kk = d.k0 * d.n0;
  const c128 ph = mk(0.0, kk);
  const c128 cr = mk(-kk * d.r_inf.im, kk * (d.r_inf.re - 1.0));  // i kk (r_inf - 1)
  const double lc = d.k0 * h / (2.0 * d.n0);
  const double ca[4] = {h / 6.0, h / 3.0, h / 3.0, h / 6.0}, cv[4] = {h / 2.0, h / 2.0, h, 0.0};
  std::vector<double> worst(d.npoles, -1.0);
  bool noconv = false;
  const c128* u = w;
  for (int sub = 0; sub < p->substeps; ++sub) {
    for (int stg = 0; stg < 4; ++stg) {
      const c128* v = stg == 0 ? u : vb;
      int rc = solve_and_sum<T, C>(p, v, Lb, ph, cr, 0.0, nullptr, (sub == 0 && stg == 0) ? 1 : 2);
      if (rc < 0) return rc;
      if (rc == HP_WARN_NOCONV) noconv = true;
      for (int k = 0; k < d.npoles && k < (int)p->relres.size(); ++k) worst[k] = std::max(worst[k], p->relres[k]);
      const bool last = stg == 3;
      // the last stage reads neither u nor v: out may be u (E_out aliasing E_in, or a later substep)
      launch_rk4_stage(Lb, stg == 0 ? u : acc, last ? out : acc, u, last ? nullptr : vb, ca[stg], cv[stg],
                       last ? lc : 0.0, d.edge_eta, d.edge_width, p->geo, p->stream);
    }
    u = out;
  }
  HPCHK(hipGetLastError());
  p->relres = worst;
  return noconv ? HP_WARN_NOCONV : HP_OK;
}

// The column pass reads flag, m, b_k and sigma_m of its pole and u_m from the
// pointer table: set them for one free-space solve (pole slot 0, m = 0,
// sigma_0 = 1), by a kernel, so that no host copy is needed.
__global__ void k_prec_setup(PoleState* st, void** tbl, void* u0, c128 b) {
  if (threadIdx.x != 0) return;
  st->flag = 0;
  st->m = 0;
  st->bk = b;
  st->sigma[0] = 1.0;
  tbl[0] = u0;
}

// y = (Zbar_fs - b_k I)^{-1} x (pole < 0: b = 0), asynchronous, with the given
// intermediate buffers: tmpR, zout (and dz for vector fields) R-domain fields,
// st one pole state, tbl one basis pointer table, part the row pass's partial norms.
template <typename T, typename C>
void prec_into(hp_plan p, int pole, const c128* x, c128* y, cx<T>* tmpR, cx<T>* zout, cx<T>* dz, PoleState* st,
               void** tbl, double* part) {
  const c128 b = pole < 0 ? mk(0.0, 0.0) : mk(p->poles[pole].re, p->poles[pole].im);
  hipLaunchKernelGGL(k_prec_setup, dim3(1), dim3(64), 0, p->stream, st, tbl, (void*)tmpR, b);
  launch_row_fwd<T, C>(x, tmpR, part, reinterpret_cast<const cx<C>*>(p->tw_x), p->geo, p->stream);
  const int zero = 0;
  launch_col<T, C>(reinterpret_cast<const cx<T>* const*>(tbl), zout, 0, 0, dz, 0, st, &zero, 1, nullptr, p->mu_x,
                   p->mu_y, reinterpret_cast<const cx<C>*>(p->tw_y), p->geo, p->sc, p->stream);
  launch_row_inv<T, C>(zout, y, reinterpret_cast<const cx<C>*>(p->tw_x), p->geo, tile_width<T>(), p->stream);
}

// The same with the plan's own workspace as scratch (before or between steps).
template <typename T, typename C>
void prec_ws(hp_plan p, int pole, const c128* x, c128* y) {
  prec_into<T, C>(p, pole, x, y, reinterpret_cast<cx<T>*>(p->tmpR), reinterpret_cast<cx<T>*>(p->P),
                  reinterpret_cast<cx<T>*>(p->DZ), p->st_scratch, p->uptr_scratch, p->part_misc);
}

// Learned starting points of every pole for right-hand side w (HP_GUESS_LEARNED):
// y_k = M_k^-1 w, the net's correction from (w, y_k, V, pole) in chunks of
// net_chunk poles, t_k = w + sigma_k net_k, x0_k = M_k^-1 t_k; the guesses land in
// the plan's guess fields and the step judges them like any other (hp_step_guess).
template <typename T, typename C>
int learned_guesses(hp_plan p, const c128* w, std::vector<const c128*>& x0) {
  const hp_plan_desc& d = p->d;
  const int K = d.npoles, B = p->net_chunk;
  const size_t fn = p->fieldn;
  c128* Y = p->lg_fields;
  c128* X0 = Y + (size_t)K * fn;
  c128* Tt = X0 + (size_t)K * fn;
  Prof pr(p, HP_K_GUESS, 0.0);
  for (int k = 0; k < K; ++k) prec_ws<T, C>(p, k, w, Y + (size_t)k * fn);
  auto net_fail = [&](int rc, const char* what) {
    return fail(p, rc, std::string("learned guess, ") + what + ": " + hp_unet_last_error(p->net));
  };
  for (int k0 = 0; k0 < K; k0 += B) {
    const int nb = std::min(B, K - k0);
    int rc = hp_guess_stats(p->net, d.ncomp, d.nx, d.ny, d.n0, d.edge_width, w, Y + (size_t)k0 * fn, p->n2copy, nb,
                            p->lg_scal);
    if (rc) return net_fail(rc, "hp_guess_stats");
    rc = hp_guess_pack(p->net, d.ncomp, d.nx, d.ny, d.n0, d.edge_width, w, Y + (size_t)k0 * fn, p->n2copy, p->lg_scal,
                       p->lg_feat.data() + 2 * k0, nb, p->lg_in);
    if (rc) return net_fail(rc, "hp_guess_pack");
    rc = hp_unet_forward(p->net, p->lg_in, nb, d.ny, d.nx, p->lg_out);
    if (rc) return net_fail(rc, "hp_unet_forward");
    rc = hp_guess_unpack(p->net, d.ncomp, d.nx, d.ny, w, p->lg_out, p->lg_scal, nb, Tt);
    if (rc) return net_fail(rc, "hp_guess_unpack");
    for (int j = 0; j < nb; ++j) prec_ws<T, C>(p, k0 + j, Tt + (size_t)j * fn, X0 + (size_t)(k0 + j) * fn);
  }
  HPCHK(hipGetLastError());
  x0.resize(K);
  for (int k = 0; k < K; ++k) x0[k] = X0 + (size_t)k * fn;
  return HP_OK;
}

template <typename T, typename C>
int run_step(hp_plan p, const c128* w, c128* out, const c128* const* x0 = nullptr) {
  if (p->form == HP_FORM_SQRT) return run_step_sqrt<T, C>(p, w, out);
  std::vector<const c128*> lg;
  if (!x0 && p->guess_mode == HP_GUESS_LEARNED) {
    int rc = learned_guesses<T, C>(p, w, lg);
    if (rc) return rc;
    x0 = lg.data();
  }
  return solve_and_sum<T, C>(p, w, out, p->phase, p->rinf_phase, p->loss_coef, x0, 1);
}

// One shifted solve (Zbar - b_k I) x = rhs; x physical complex128.
template <typename T, typename C>
int run_solve(hp_plan p, int k, const c128* rhs, c128* x) {
  bool noconv = false;
  int rc = run_poles<T, C>(p, rhs, std::vector<int>{k}, &noconv);
  if (rc) return rc;
  fold<T>(p, k);
  if (p->pml)
    HPCHK(hipMemcpyAsync(x, p->X + (size_t)k * p->fieldn, p->fieldn * sizeof(c128), hipMemcpyDeviceToDevice,
                         p->stream));
  else
    launch_row_inv<double>(p->X + (size_t)k * p->fieldn, x, p->tw64_x, p->geo, tile_width<T>(), p->stream);
  HPCHK(hipGetLastError());
  HPCHK(hipStreamSynchronize(p->stream));
  return noconv ? HP_WARN_NOCONV : HP_OK;
}

// x_k of the last step or solve (physical complex128).
template <typename T>
int get_solution(hp_plan p, int k, c128* x) {
  fold<T>(p, k);
  if (p->pml)
    HPCHK(hipMemcpyAsync(x, p->X + (size_t)k * p->fieldn, p->fieldn * sizeof(c128), hipMemcpyDeviceToDevice,
                         p->stream));
  else
    launch_row_inv<double>(p->X + (size_t)k * p->fieldn, x, p->tw64_x, p->geo, tile_width<T>(), p->stream);
  HPCHK(hipGetLastError());
  HPCHK(hipStreamSynchronize(p->stream));
  return HP_OK;
}

template <typename T, typename C>
int apply_prec(hp_plan p, int pole, const c128* x, c128* y) {
  PoleState h;
  memset(&h, 0, sizeof(h));
  h.bk = pole < 0 ? mk(0.0, 0.0) : mk(p->poles[pole].re, p->poles[pole].im);
  h.sigma[0] = 1.0;
  void* tbl[HP_MAXM + 1] = {nullptr};
  tbl[0] = p->tmpR;
  const int zero = 0;
  if (p->pml) tbl[0] = const_cast<c128*>(x);
  HPCHK(hipMemcpyAsync(p->st_scratch, &h, sizeof(h), hipMemcpyHostToDevice, p->stream));
  HPCHK(hipMemcpyAsync(p->uptr_scratch, tbl, sizeof(tbl), hipMemcpyHostToDevice, p->stream));
  if (p->pml) {
    pml_prec(p, p->st_scratch, &zero, 1, nullptr, PmlRef{reinterpret_cast<c128* const*>(p->uptr_scratch), nullptr, 0, 0},
             PmlRef{nullptr, y, 0, 0}, reinterpret_cast<c128*>(p->P), p->pml_s);
    HPCHK(hipGetLastError());
    HPCHK(hipStreamSynchronize(p->stream));
    return HP_OK;
  }
  launch_row_fwd<T, C>(x, reinterpret_cast<cx<T>*>(p->tmpR), p->part_misc, reinterpret_cast<const cx<C>*>(p->tw_x),
                    p->geo, p->stream);
  // the first basis slot of pole 0 in Z serves as output; the DZ slot as scratch
  cx<T>* zout = reinterpret_cast<cx<T>*>(p->P);
  launch_col<T, C>(reinterpret_cast<const cx<T>* const*>(p->uptr_scratch), zout, 0, 0, reinterpret_cast<cx<T>*>(p->DZ), 0,
                p->st_scratch, &zero, 1, nullptr, p->mu_x, p->mu_y,
                reinterpret_cast<const cx<C>*>(p->tw_y), p->geo, p->sc, p->stream);
  launch_row_inv<T, C>(zout, y, reinterpret_cast<const cx<C>*>(p->tw_x), p->geo, tile_width<T>(), p->stream);
  HPCHK(hipStreamSynchronize(p->stream));
  return HP_OK;
}

}  // namespace

extern "C" {

size_t hp_workspace_bytes(const hp_plan_desc* desc) {
  if (!validate(desc).empty()) return 0;
  hp_plan_s tmp;
  tmp.d = *desc;
  derive(&tmp);
  Ws w;
  layout(&tmp, w);
  return w.off + 256;
}

int hp_plan_create(const hp_plan_desc* desc, void* stream, void* workspace, hp_plan* out) {
  if (!out) return fail(nullptr, HP_EINVAL, "out is NULL");
  *out = nullptr;
  std::string v = validate(desc);
  if (!v.empty()) return fail(nullptr, HP_EINVAL, v);
  hp_plan p = new (std::nothrow) hp_plan_s();
  if (!p) return fail(nullptr, HP_ENOMEM, "host allocation failed");
  p->d = *desc;
  p->poles.assign(desc->poles, desc->poles + desc->npoles);
  p->residues.assign(desc->residues, desc->residues + desc->npoles);
  memcpy(p->c2, desc->d2, sizeof(p->c2));
  memcpy(p->d1c, desc->d1, sizeof(p->d1c));
  p->d.poles = p->poles.data();
  p->d.residues = p->residues.data();
  p->d.d2 = p->c2;
  p->d.d1 = p->d1c;
  p->stream = reinterpret_cast<hipStream_t>(stream);
  derive(p);
  const double K = desc->k0 * desc->n0 * desc->dz;
  const std::complex<double> ph = std::exp(std::complex<double>(0.0, -K));
  const std::complex<double> rp = ph * std::complex<double>(desc->r_inf.re, desc->r_inf.im);
  p->phase = mk(ph.real(), ph.imag());
  p->rinf_phase = mk(rp.real(), rp.imag());
  p->loss_coef = desc->k0 * desc->dz / (2.0 * desc->n0);
  // free-space spectrum checks
  const double s = 1.0 / ((desc->k0 * desc->n0) * (desc->k0 * desc->n0));
  auto mx = mu_table(desc->nx, desc->dx, p->c2, s), my = mu_table(desc->ny, desc->dy, p->c2, s);
  const double lo = *std::min_element(mx.begin() + 1, mx.end()) + *std::min_element(my.begin() + 1, my.end());
  const double hi = *std::max_element(mx.begin() + 1, mx.end()) + *std::max_element(my.begin() + 1, my.end());
  for (int k = 0; k < desc->npoles; ++k) {
    if (fabs(p->poles[k].im) < 1e-14 && p->poles[k].re >= lo - 1e-14 && p->poles[k].re <= hi + 1e-14) {
      for (int i = 1; i < desc->ny; ++i)
        for (int j = 1; j < desc->nx; ++j)
          if (fabs(my[i] + mx[j] - p->poles[k].re) < 1e-14) {
            delete p;
            return fail(nullptr, HP_EINVAL, "a pole lies on the free-space spectrum");
          }
    }
  }
  // kappa(M_k) <= max |lambda - b_k| / dist(b_k, [lo, hi]) over the free-space spectrum
  const double eps = desc->precision != HP_FP64 ? 6e-8 : 1.1e-16;  // complex64 storage rounds every vector
  p->incons.assign(desc->npoles, 0.0);
  for (int k = 0; k < desc->npoles; ++k) {
    const std::complex<double> b(p->poles[k].re, p->poles[k].im);
    const double dre = b.real() < lo ? lo - b.real() : (b.real() > hi ? b.real() - hi : 0.0);
    const double dist = std::sqrt(dre * dre + b.imag() * b.imag());
    const double far = std::max(std::abs(lo - b), std::abs(hi - b));
    p->incons[k] = dist > 0 ? eps * far / dist : 1.0;
  }
  double rmax = 0.0;
  for (int i = 0; i <= 100000; ++i) {
    const double z = lo + (hi - lo) * i / 100000.0;
    rmax = std::max(rmax, std::abs(rat(p, z)));
  }
  // workspace
  Ws w;
  layout(p, w);
  p->ws_bytes = w.off + 256;
  if (workspace) {
    if (reinterpret_cast<uintptr_t>(workspace) % 256) {
      delete p;
      return fail(nullptr, HP_EINVAL, "workspace must be 256-byte aligned");
    }
    p->ws = reinterpret_cast<char*>(workspace);
  } else {
    hipError_t e = hipMalloc(&p->ws, p->ws_bytes);
    if (e != hipSuccess) {
      delete p;
      return fail(nullptr, HP_ENOMEM, std::string("hipMalloc workspace: ") + hipGetErrorString(e));
    }
    p->own_ws = true;
  }
  w = Ws();
  w.base = p->ws;
  w.dry = false;
  layout(p, w);
  if (hipHostMalloc(&p->ftag_h, 2 * HP_MAXPOLES * sizeof(unsigned long long),
                    hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess ||
      hipHostMalloc(&p->est_h, HP_MAXPOLES * sizeof(double)) != hipSuccess ||
      hipHostMalloc(&p->active_h, 3 * HP_MAXPOLES * sizeof(int)) != hipSuccess ||
      hipHostMalloc(&p->misc_h, (std::max(p->nopblk, p->nrowblk * 2) + 64) * sizeof(double)) != hipSuccess) {
    hp_plan_destroy(p);
    return fail(nullptr, HP_ENOMEM, "pinned host allocation failed");
  }
  if (hipHostGetDevicePointer(reinterpret_cast<void**>(&p->ftag_hd), p->ftag_h, 0) != hipSuccess) {
    hp_plan_destroy(p);
    return fail(nullptr, HP_EHIP, "no device address for the pinned flag buffer");
  }
  memset(p->ftag_h, 0, 2 * HP_MAXPOLES * sizeof(unsigned long long));
  int rc = (p->mixed && !p->mixed64) ? upload_tables<float>(p) : upload_tables<double>(p);
  if (rc) {
    g_thread_error = p->err;
    hp_plan_destroy(p);
    return rc;
  }
  // zero every buffer once: row 0 and column 0 of all fields stay zero
  if (hipMemsetAsync(p->coef, 0, (char*)(p->st) - (char*)(p->coef), p->stream) != hipSuccess) {
    hp_plan_destroy(p);
    return fail(nullptr, HP_EHIP, "workspace clear failed");
  }
  // Krylov vector pointer table: u_i of pole k at U[k][i]
  const size_t es = p->mixed ? sizeof(c64) : sizeof(c128);
  p->uptr_h.assign((size_t)desc->npoles * (HP_MAXM + 1), nullptr);
  for (int k = 0; k < desc->npoles; ++k)
    for (int i = 0; i <= desc->restart; ++i)
      p->uptr_h[(size_t)k * (HP_MAXM + 1) + i] =
          reinterpret_cast<char*>(p->U) + ((size_t)k * (desc->restart + 1) + i) * p->fieldn * es;
  if ((rc = upload_uptr(p)) || (rc = upload_state(p))) {
    g_thread_error = p->err;
    hp_plan_destroy(p);
    return rc;
  }
  if (hipStreamSynchronize(p->stream) != hipSuccess) {
    hp_plan_destroy(p);
    return fail(nullptr, HP_EHIP, "plan upload failed");
  }
  scratch_setup(p);  // this device's static scratch (hp_apply_preconditioner_noalloc)
  *out = p;
  return (rmax > 1.0 + 1e-6) ? HP_WARN_UNSTABLE : HP_OK;
}

int hp_set_medium(hp_plan p, const double* n2) {
  if (!p) return fail(nullptr, HP_EINVAL, "plan is NULL");
  if (!n2) return fail(p, HP_EINVAL, "n2 is NULL");
  const double s = 1.0 / ((p->d.k0 * p->d.n0) * (p->d.k0 * p->d.n0));
  launch_coef(n2, p->coef, p->coef_scratch, p->d.n0, s, p->d.edge_width, p->sc, p->geo, p->stream);
  HPCHK(hipMemcpyAsync(p->n2copy, n2, p->geo.fsz * sizeof(double), hipMemcpyDeviceToDevice, p->stream));
  if (p->mixed && !p->mixed64)
    launch_to_float(p->coef, p->coef_f, (p->d.ncomp == 2 ? 6 : 1) * p->geo.fsz, p->stream);
  HPCHK(hipGetLastError());
  p->medium_set = true;
  return HP_OK;
}

int hp_step(hp_plan p, const void* E_in, const double* n2, void* E_out) {
  if (!p) return fail(nullptr, HP_EINVAL, "plan is NULL");
  if (!E_in || !E_out) return fail(p, HP_EINVAL, "E_in/E_out is NULL");
  if (n2) {
    int rc = hp_set_medium(p, n2);
    if (rc) return rc;
  }
  if (!p->medium_set) return fail(p, HP_ESTATE, "no medium: pass n2 or call hp_set_medium first");
  const c128* w = reinterpret_cast<const c128*>(E_in);
  c128* out = reinterpret_cast<c128*>(E_out);
  return HP_BY_PRECISION(p, run_step, p, w, out);
}

int hp_step_guess(hp_plan p, const void* E_in, const double* n2, const void* const* x0, int* accepted,
                  void* E_out) {
  if (!p) return fail(nullptr, HP_EINVAL, "plan is NULL");
  if (!E_in || !E_out) return fail(p, HP_EINVAL, "E_in/E_out is NULL");
  if (n2) {
    int rc = hp_set_medium(p, n2);
    if (rc) return rc;
  }
  if (!p->medium_set) return fail(p, HP_ESTATE, "no medium: pass n2 or call hp_set_medium first");
  if (p->form != HP_FORM_EXP) return fail(p, HP_ESTATE, "initial guesses apply to the exponential form only");
  if (p->pml && x0) return fail(p, HP_ESTATE, "guesses are not available with absorbing layers");
  const c128* w = reinterpret_cast<const c128*>(E_in);
  c128* out = reinterpret_cast<c128*>(E_out);
  std::vector<const c128*> g(p->d.npoles, nullptr);
  if (x0)
    for (int k = 0; k < p->d.npoles; ++k) g[k] = reinterpret_cast<const c128*>(x0[k]);
  const c128* const* gp = x0 ? g.data() : nullptr;
  int rc = HP_BY_PRECISION(p, run_step, p, w, out, gp);
  if (rc >= 0 && accepted)
    for (int k = 0; k < p->d.npoles; ++k) accepted[k] = p->accepted[k];
  return rc;
}

int hp_set_launch(hp_plan p, int col_variant) {
  if (!p) return fail(nullptr, HP_EINVAL, "plan is NULL");
  const int top = p->pml ? 3 : 2;  // with absorbing layers: the dense stages' forms 0..3
  if (col_variant < 0 || col_variant > top)
    return fail(p, HP_EINVAL, p->pml ? "variant must be 0, 1, 2 or 3" : "col_variant must be 0, 1 or 2");
  p->geo.col_variant = col_variant;
  return HP_OK;
}

int hp_autotune(hp_plan p, const void* E_in, const double* n2, int reps, void* E_out, int* variant) {
  if (!p) return fail(nullptr, HP_EINVAL, "plan is NULL");
  if (!E_in || !E_out) return fail(p, HP_EINVAL, "E_in/E_out is NULL");
  if (E_in == E_out) return fail(p, HP_EINVAL, "E_out must not alias E_in (every timed step starts from E_in)");
  if (reps < 1 || reps > 100) return fail(p, HP_EINVAL, "reps must be in [1, 100]");
  if (n2) {
    int rc = hp_set_medium(p, n2);
    if (rc) return rc;
  }
  if (!p->medium_set) return fail(p, HP_ESTATE, "no medium: pass n2 or call hp_set_medium first");
  const int keep = p->geo.col_variant;
  double best = 0.0;
  int bestv = keep;
  for (int v = 0; v < (p->pml ? 4 : 3); ++v) {
    p->geo.col_variant = v;
    int rc = hp_step(p, E_in, nullptr, E_out);  // untimed: first use of this variant's kernels
    if (rc < 0) {
      p->geo.col_variant = keep;
      return rc;
    }
    if (hipStreamSynchronize(p->stream) != hipSuccess) {
      p->geo.col_variant = keep;
      return fail(p, HP_EHIP, "hipStreamSynchronize failed while timing");
    }
    const auto t0 = std::chrono::steady_clock::now();
    for (int r = 0; r < reps && rc >= 0; ++r) {
      p->prev_valid = false;  // every timed step starts from the same state
      rc = hp_step(p, E_in, nullptr, E_out);
    }
    if (rc < 0 || hipStreamSynchronize(p->stream) != hipSuccess) {
      p->geo.col_variant = keep;
      return rc < 0 ? rc : fail(p, HP_EHIP, "hipStreamSynchronize failed while timing");
    }
    const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (v == 0 || dt < best) best = dt, bestv = v;
  }
  p->geo.col_variant = bestv;
  if (variant) *variant = bestv;
  p->prev_valid = false;
  return hp_step(p, E_in, nullptr, E_out);  // E_out and the statistics from the chosen variant
}

int hp_set_guess(hp_plan p, int mode) {
  if (!p) return fail(nullptr, HP_EINVAL, "plan is NULL");
  if (mode != HP_GUESS_ZERO && mode != HP_GUESS_PREV && mode != HP_GUESS_LEARNED)
    return fail(p, HP_EINVAL, "unknown guess mode");
  if (mode == HP_GUESS_LEARNED && !p->net)
    return fail(p, HP_ESTATE, "HP_GUESS_LEARNED needs a net: call hp_set_guess_net first");
  if (mode != HP_GUESS_ZERO && p->pml) return fail(p, HP_ESTATE, "guesses are not available with absorbing layers");
  p->guess_mode = mode;
  p->prev_valid = false;
  return HP_OK;
}

static void free_guess_net(hp_plan p) {
  for (void* b : {(void*)p->lg_fields, (void*)p->lg_in, (void*)p->lg_out, (void*)p->lg_scal})
    if (b) (void)hipFree(b);
  p->lg_fields = nullptr;
  p->lg_in = p->lg_out = nullptr;
  p->lg_scal = nullptr;
  p->net = nullptr;
  p->net_chunk = 0;
}

int hp_set_guess_net(hp_plan p, hp_unet net, int chunk) {
  if (!p) return fail(nullptr, HP_EINVAL, "plan is NULL");
  HPCHK(hipStreamSynchronize(p->stream));
  if (!net) {
    free_guess_net(p);
    if (p->guess_mode == HP_GUESS_LEARNED) p->guess_mode = HP_GUESS_ZERO;
    return HP_OK;
  }
  const hp_plan_desc& d = p->d;
  int levels = 0, cin = 0, cout = 0;
  unet_shape(net, &levels, &cin, &cout);
  if (cin != 4 * d.ncomp + 3 || cout != 2 * d.ncomp)
    return fail(p, HP_EINVAL, "the net needs cin = 4 ncomp + 3 and cout = 2 ncomp inputs/outputs for this plan");
  const int mult = 1 << (levels - 1);
  if (d.nx % mult || d.ny % mult) return fail(p, HP_EINVAL, "nx, ny must be multiples of 2^(levels - 1)");
  if (unet_stream(net) != p->stream) return fail(p, HP_EINVAL, "the net must run on the plan's stream");
  if (chunk < 1 || chunk > 64) return fail(p, HP_EINVAL, "chunk must be in [1, 64]");
  chunk = std::min(chunk, d.npoles);
  free_guess_net(p);
  const size_t fn = p->fieldn, px = (size_t)d.nx * d.ny;
  hipError_t e = hipMalloc(&p->lg_fields, (2 * (size_t)d.npoles + chunk) * fn * sizeof(c128));
  if (e == hipSuccess) e = hipMalloc(&p->lg_in, (size_t)chunk * cin * px * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&p->lg_out, (size_t)chunk * cout * px * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&p->lg_scal, (chunk + 2) * sizeof(double));
  if (e != hipSuccess) {
    free_guess_net(p);
    return fail(p, HP_ENOMEM, std::string("learned-guess buffers: ") + hipGetErrorString(e));
  }
  p->net = net;
  p->net_chunk = chunk;
  p->lg_feat.resize(2 * (size_t)d.npoles);
  for (int k = 0; k < d.npoles; ++k) {
    p->lg_feat[2 * k] = std::asinh(p->poles[k].re);
    p->lg_feat[2 * k + 1] = std::asinh(p->poles[k].im);
  }
  return HP_OK;
}

int hp_set_form(hp_plan p, int form, int substeps) {
  if (!p) return fail(nullptr, HP_EINVAL, "plan is NULL");
  if (form != HP_FORM_EXP && form != HP_FORM_SQRT) return fail(p, HP_EINVAL, "unknown form");
  if (form != HP_FORM_EXP && p->pml) return fail(p, HP_ESTATE, "absorbing layers apply to the exponential form only");
  if (form == HP_FORM_EXP) {
    p->form = form;
    p->substeps = 1;
    return HP_OK;
  }
  if (substeps < 1 || substeps > 1024) return fail(p, HP_EINVAL, "substeps must be in [1, 1024]");
  if (!p->rk) {
    hipError_t e = hipMalloc(&p->rk, 3 * p->fieldn * sizeof(c128));
    if (e != hipSuccess) {
      p->rk = nullptr;
      return fail(p, HP_ENOMEM, std::string("hipMalloc stage fields: ") + hipGetErrorString(e));
    }
  }
  p->form = form;
  p->substeps = substeps;
  p->prev_valid = false;
  // one substep multiplies the free-space mode of eigenvalue mu by the RK4
  // polynomial of h i k0 n0 (r(mu) - 1)
  const hp_plan_desc& d = p->d;
  const double s = 1.0 / ((d.k0 * d.n0) * (d.k0 * d.n0));
  auto mx = mu_table(d.nx, d.dx, p->c2, s), my = mu_table(d.ny, d.dy, p->c2, s);
  const double lo = *std::min_element(mx.begin() + 1, mx.end()) + *std::min_element(my.begin() + 1, my.end());
  const double hi = *std::max_element(mx.begin() + 1, mx.end()) + *std::max_element(my.begin() + 1, my.end());
  const std::complex<double> hk(0.0, d.dz / substeps * d.k0 * d.n0);
  double gmax = 0.0;
  for (int i = 0; i <= 100000; ++i) {
    const std::complex<double> z = hk * (rat(p, lo + (hi - lo) * i / 100000.0) - 1.0);
    gmax = std::max(gmax, std::abs(1.0 + z * (1.0 + z * (0.5 + z * (1.0 / 6.0 + z / 24.0)))));
  }
  return gmax > 1.0 + 1e-6 ? HP_WARN_UNSTABLE : HP_OK;
}

static void free_pml(hp_plan p) {
  if (p->pml_mem) (void)hipFree(p->pml_mem);
  p->pml_mem = nullptr;
  p->pml_q = p->pml_qi = p->pml_lam = p->pml_a2 = p->pml_a1 = p->pml_s = p->pml_shared = nullptr;
  p->pml_part = nullptr;
  p->pml = false;
  p->pml_sigma = 0.0;
  if (p->geo.col_variant > 2) p->geo.col_variant = 1;  // a dense-stage form with no column-pass meaning
}

int hp_set_pml(hp_plan p, double sigma_max, const void* Q, const void* Qinv, const void* lam) {
  if (!p) return fail(nullptr, HP_EINVAL, "plan is NULL");
  HPCHK(hipStreamSynchronize(p->stream));
  if (sigma_max == 0.0 && !Q && !Qinv && !lam) {
    free_pml(p);
    return HP_OK;
  }
  const hp_plan_desc& d = p->d;
  if (d.nx != d.ny || d.dx != d.dy) return fail(p, HP_EINVAL, "absorbing layers need a square grid (nx = ny, dx = dy)");
  if (d.precision != HP_FP64) return fail(p, HP_EINVAL, "absorbing layers need precision HP_FP64");
  if (!(sigma_max > 0.0) || !std::isfinite(sigma_max)) return fail(p, HP_EINVAL, "sigma_max must be finite and > 0");
  if (!Q || !Qinv || !lam) return fail(p, HP_EINVAL, "Q, Qinv, lam must all be given");
  if (p->form != HP_FORM_EXP) return fail(p, HP_ESTATE, "absorbing layers apply to the exponential form only");
  if (p->guess_mode != HP_GUESS_ZERO) return fail(p, HP_ESTATE, "absorbing layers need the guess mode HP_GUESS_ZERO");
  using cd = std::complex<double>;
  const int N = d.nx, n = N - 1, W = d.edge_width;
  const cd* q = reinterpret_cast<const cd*>(Q);
  const cd* qi = reinterpret_cast<const cd*>(Qinv);
  const cd* l = reinterpret_cast<const cd*>(lam);
  for (size_t i = 0; i < (size_t)n * n; ++i)
    if (!std::isfinite(q[i].real()) || !std::isfinite(q[i].imag()) || !std::isfinite(qi[i].real()) ||
        !std::isfinite(qi[i].imag()))
      return fail(p, HP_EINVAL, "Q or Qinv holds a NaN or Inf");
  // the stretch g = 1 + i sigma, sigma = sigma_max ((W + 1 - d)/W)^2 at distance d in [1, W] cells from
  // the nearer Dirichlet node, and its derivative along the axis
  const double h = d.dx, sc = 1.0 / ((d.k0 * d.n0) * (d.k0 * d.n0));
  std::vector<c128> a2(N), a1(N);
  std::vector<cd> a2c(N), a1c(N);
  for (int j = 0; j < N; ++j) {
    const int dist = std::min(j, N - j);
    const double t = (dist >= 1 && dist <= W) ? (W + 1.0 - dist) / W : 0.0;
    const double dsdd = -2.0 * sigma_max * t / W;  // d sigma / d(distance), per cell
    const double dsdx = (j <= N - j ? dsdd : -dsdd) / h;
    const cd g(1.0, sigma_max * t * t), gp(0.0, dsdx);
    a2c[j] = 1.0 / (g * g);
    a1c[j] = sc * gp / (g * g * g);
    a2[j] = mk(a2c[j].real(), a2c[j].imag());
    a1[j] = mk(a1c[j].real(), a1c[j].imag());
  }
  // the tables must decompose this library's stretched operator: compare
  // Q (lam .* (Q^-1 x)) with s D~ x for two pseudo-random x
  {
    uint64_t rs = 0x9E3779B97F4A7C15ull;
    auto rnd = [&]() {
      rs = rs * 6364136223846793005ull + 1442695040888963407ull;
      return (double)(rs >> 11) / 9007199254740992.0 - 0.5;
    };
    for (int probe = 0; probe < 2; ++probe) {
      std::vector<cd> x(n), t(n), ye(n, 0.0), yd(n);
      for (int j = 0; j < n; ++j) x[j] = cd(rnd(), rnd());
      for (int r = 0; r < n; ++r) {
        cd acc = 0.0;
        for (int c = 0; c < n; ++c) acc += qi[(size_t)r * n + c] * x[c];
        t[r] = l[r] * acc;
      }
      for (int r = 0; r < n; ++r) {
        cd acc = 0.0;
        for (int c = 0; c < n; ++c) acc += q[(size_t)r * n + c] * t[c];
        ye[r] = acc;
      }
      auto at = [&](int k) -> cd {
        double sg = 1.0;
        if (k < 0) {
          k = -k;
          sg = -1.0;
        } else if (k > N) {
          k = 2 * N - k;
          sg = -1.0;
        }
        if (k == 0 || k == N) return 0.0;
        return sg * x[k - 1];
      };
      double num = 0.0, den = 0.0;
      for (int j = 1; j < N; ++j) {
        cd s2 = p->sc.c2x[0] * x[j - 1], s1 = 0.0;
        for (int mm = 1; mm <= 6; ++mm) {
          s2 += p->sc.c2x[mm] * (at(j + mm) + at(j - mm));
          s1 += p->sc.d1x[mm - 1] * (at(j + mm) - at(j - mm));
        }
        yd[j - 1] = a2c[j] * s2 - a1c[j] * s1;
        num += std::norm(yd[j - 1] - ye[j - 1]);
        den += std::norm(yd[j - 1]);
      }
      // the dense stages only precondition (the Arnoldi step applies the explicit
      // operator to the stored z), so 1e-3 leaves GMRES its convergence
      if (!(num <= 1e-6 * den))
        return fail(p, HP_EINVAL,
                    "Q diag(lam) Q^-1 does not reproduce the stretched operator s D~ of this plan (relative error " +
                        std::to_string(std::sqrt(num / den)) + ")");
    }
  }
  for (int k = 0; k < d.npoles; ++k) {
    const cd b(p->poles[k].re, p->poles[k].im);
    double mn = 1e300;
    for (int a = 0; a < n; ++a)
      for (int c = 0; c < n; ++c) mn = std::min(mn, std::abs(l[a] + l[c] - b));
    if (!(mn > 1e-12 * (1.0 + std::abs(b))))
      return fail(p, HP_EINVAL, "pole " + std::to_string(k) + " lies on the stretched free-space spectrum");
  }
  const size_t NN = (size_t)N * N, fn = p->fieldn, K = (size_t)d.npoles;
  const size_t nparts = (size_t)pml_apply_parts(N);
  if (!p->pml_mem) {
    const size_t bytes = (2 * NN + 3 * (size_t)N + (K + 2) * fn) * sizeof(c128) +
                         K * (HP_MAXM + 1) * 2 * nparts * sizeof(double2);
    hipError_t e = hipMalloc(&p->pml_mem, bytes);
    if (e != hipSuccess) {
      p->pml_mem = nullptr;
      return fail(p, HP_ENOMEM, std::string("absorbing-layer tables: ") + hipGetErrorString(e));
    }
    c128* c = reinterpret_cast<c128*>(p->pml_mem);
    p->pml_q = c;
    p->pml_qi = c + NN;
    p->pml_lam = c + 2 * NN;
    p->pml_a2 = p->pml_lam + N;
    p->pml_a1 = p->pml_a2 + N;
    p->pml_s = p->pml_a1 + N;
    p->pml_shared = p->pml_s + K * fn;
    p->pml_part = reinterpret_cast<double2*>(p->pml_shared + 2 * fn);
  }
  // padded to N x N: row and column 0 zero
  std::vector<c128> pad(NN, mk(0.0, 0.0));
  for (int src = 0; src < 2; ++src) {
    const cd* m = src ? qi : q;
    for (int r = 0; r < n; ++r)
      for (int c = 0; c < n; ++c) {
        const cd v = m[(size_t)r * n + c];
        pad[(size_t)(r + 1) * N + c + 1] = mk(v.real(), v.imag());
      }
    HPCHK(hipMemcpy(src ? p->pml_qi : p->pml_q, pad.data(), NN * sizeof(c128), hipMemcpyHostToDevice));
  }
  std::vector<c128> lp(N, mk(0.0, 0.0));
  for (int r = 0; r < n; ++r) lp[r + 1] = mk(l[r].real(), l[r].imag());
  HPCHK(hipMemcpy(p->pml_lam, lp.data(), N * sizeof(c128), hipMemcpyHostToDevice));
  HPCHK(hipMemcpy(p->pml_a2, a2.data(), N * sizeof(c128), hipMemcpyHostToDevice));
  HPCHK(hipMemcpy(p->pml_a1, a1.data(), N * sizeof(c128), hipMemcpyHostToDevice));
  // the medium-pass slots and the dense stages' scratch start from zero (rows 0 and columns 0 stay so)
  HPCHK(hipMemset(p->pml_s, 0, (K + 2) * fn * sizeof(c128)));
  p->pml = true;
  p->pml_sigma = sigma_max;
  p->prev_valid = false;
  return HP_OK;
}

int hp_fit_exp_sqrt(double K, int degree, int lawson_steps, void* stream, hp_c128* poles, hp_c128* residues,
                    hp_c128* r_inf, double* max_err) {
  if (!(K > 0.0) || !std::isfinite(K)) return fail(nullptr, HP_EINVAL, "K must be finite and > 0");
  if (degree < 1 || degree > 31) return fail(nullptr, HP_EINVAL, "degree must be in [1, 31]");
  if (lawson_steps < 0 || lawson_steps > 1000) return fail(nullptr, HP_EINVAL, "lawson_steps must be in [0, 1000]");
  if (!poles || !residues || !r_inf) return fail(nullptr, HP_EINVAL, "poles/residues/r_inf is NULL");
  std::vector<c128> h;
  std::string why;
  if (fit_exp_sqrt_device(K, degree, lawson_steps, reinterpret_cast<hipStream_t>(stream), h, &why))
    return fail(nullptr, HP_EHIP, why);
  const int np = (int)h[2 * (size_t)degree + 1].im;
  if (max_err) *max_err = h[2 * (size_t)degree + 1].re;
  if (np != degree)
    return fail(nullptr, HP_EINVAL,
                "the fit's denominator has " + std::to_string(np) + " finite roots, not " + std::to_string(degree));
  for (int k = 0; k < degree; ++k) {
    poles[k] = hp_c128{h[k].re, h[k].im};
    residues[k] = hp_c128{h[degree + k].re, h[degree + k].im};
  }
  *r_inf = hp_c128{h[2 * (size_t)degree].re, h[2 * (size_t)degree].im};
  return HP_OK;
}

int hp_get_solution(hp_plan p, int pole, void* x) {
  if (!p) return fail(nullptr, HP_EINVAL, "plan is NULL");
  if (!x) return fail(p, HP_EINVAL, "x is NULL");
  if (pole < 0 || pole >= p->d.npoles) return fail(p, HP_EINVAL, "pole out of range");
  c128* o = reinterpret_cast<c128*>(x);
  return p->mixed ? get_solution<float>(p, pole, o) : get_solution<double>(p, pole, o);
}

int hp_apply_medium(hp_plan p, const void* x, void* y) {
  if (!p) return fail(nullptr, HP_EINVAL, "plan is NULL");
  if (!x || !y || x == y) return fail(p, HP_EINVAL, "x, y must be distinct device buffers");
  if (!p->medium_set) return fail(p, HP_ESTATE, "no medium set");
  launch_apply_op(reinterpret_cast<const c128*>(x), nullptr, reinterpret_cast<c128*>(y), p->coef, mk(0.0, 0.0),
                  p->sc, p->geo, nullptr, p->stream, 1);
  HPCHK(hipGetLastError());
  return HP_OK;
}

int hp_solve(hp_plan p, int pole, const void* rhs, void* x) {
  if (!p) return fail(nullptr, HP_EINVAL, "plan is NULL");
  if (!rhs || !x) return fail(p, HP_EINVAL, "rhs/x is NULL");
  if (pole < 0 || pole >= p->d.npoles) return fail(p, HP_EINVAL, "pole out of range");
  if (!p->medium_set) return fail(p, HP_ESTATE, "no medium set");
  const c128* r = reinterpret_cast<const c128*>(rhs);
  c128* o = reinterpret_cast<c128*>(x);
  return HP_BY_PRECISION(p, run_solve, p, pole, r, o);
}

int hp_propagate(hp_plan p, const void* E_in, const double* n2, long n2_step_stride, int nsteps, void* E_out) {
  if (!p) return fail(nullptr, HP_EINVAL, "plan is NULL");
  if (nsteps < 0) return fail(p, HP_EINVAL, "nsteps < 0");
  if (nsteps == 0) {
    if (E_out != E_in)
      HPCHK(hipMemcpyAsync(E_out, E_in, p->fieldn * sizeof(c128), hipMemcpyDeviceToDevice, p->stream));
    return HP_OK;
  }
  int worst = HP_OK;
  const void* src = E_in;
  for (int s = 0; s < nsteps; ++s) {
    const double* m = nullptr;
    if (n2 && (s == 0 || n2_step_stride != 0)) m = n2 + (size_t)s * n2_step_stride;
    int rc = hp_step(p, src, m, E_out);
    if (rc < 0) return rc;
    if (rc > worst) worst = rc;
    src = E_out;
  }
  return worst;
}

int hp_get_stats(hp_plan p, int* iters_per_pole, double* final_relres) {
  if (!p) return fail(nullptr, HP_EINVAL, "plan is NULL");
  std::vector<PoleState> h(p->d.npoles);
  HPCHK(hipStreamSynchronize(p->stream));
  HPCHK(hipMemcpy(h.data(), p->st, h.size() * sizeof(PoleState), hipMemcpyDeviceToHost));
  for (int k = 0; k < p->d.npoles; ++k) {
    if (iters_per_pole) iters_per_pole[k] = h[k].total;
    if (final_relres) {
      double r = (k < (int)p->relres.size()) ? p->relres[k] : -1.0;
      if (r < 0) r = h[k].beta0 > 0 ? h[k].est / h[k].beta0 : 0.0;
      final_relres[k] = r;
    }
  }
  return HP_OK;
}

int hp_set_fixed_iters(hp_plan p, const int* iters) {
  if (!p) return fail(nullptr, HP_EINVAL, "plan is NULL");
  if (iters) {
    for (int k = 0; k < p->d.npoles; ++k)
      if (iters[k] < 1 || iters[k] > p->d.restart) return fail(p, HP_EINVAL, "fixed iterations must be in [1, restart]");
    p->fixed.assign(iters, iters + p->d.npoles);
  } else {
    p->fixed.clear();
  }
  return upload_state(p);
}

int hp_apply_operator(hp_plan p, int pole, const void* x, void* y) {
  if (!p) return fail(nullptr, HP_EINVAL, "plan is NULL");
  if (!x || !y || x == y) return fail(p, HP_EINVAL, "x, y must be distinct device buffers");
  if (pole >= p->d.npoles) return fail(p, HP_EINVAL, "pole out of range");
  if (!p->medium_set) return fail(p, HP_ESTATE, "no medium set");
  const c128 b = pole < 0 ? mk(0.0, 0.0) : mk(p->poles[pole].re, p->poles[pole].im);
  if (p->pml) {
    if (!launch_pml_residual(reinterpret_cast<const c128*>(x), 0, nullptr, reinterpret_cast<c128*>(y), 0, p->coef,
                             p->pml_a2, p->pml_a1, p->sc, &b, 1, nullptr, 0, p->nopblk, p->d.nx, p->d.ncomp,
                             p->stream))
      return fail(p, HP_EINVAL, "absorbing-layer operator: the grid does not tile by 64 x 16");
  } else
    launch_apply_op(reinterpret_cast<const c128*>(x), nullptr, reinterpret_cast<c128*>(y), p->coef, b, p->sc, p->geo,
                    nullptr, p->stream);
  HPCHK(hipGetLastError());
  return HP_OK;
}

int hp_apply_preconditioner(hp_plan p, int pole, const void* x, void* y) {
  if (!p) return fail(nullptr, HP_EINVAL, "plan is NULL");
  if (!x || !y) return fail(p, HP_EINVAL, "x, y are NULL");
  if (pole >= p->d.npoles) return fail(p, HP_EINVAL, "pole out of range");
  const c128* xx = reinterpret_cast<const c128*>(x);
  c128* yy = reinterpret_cast<c128*>(y);
  return HP_BY_PRECISION(p, apply_prec, p, pole, xx, yy);
}

int hp_profile(hp_plan p, int enable) {
  if (!p) return fail(nullptr, HP_EINVAL, "plan is NULL");
  HPCHK(hipStreamSynchronize(p->stream));
  p->prof = enable < 0 ? (1 << HP_K_COUNT) - 1 : enable & ((1 << HP_K_COUNT) - 1);
  p->ev_used = 0;
  p->ev_cls.clear();
  p->ev_bytes.clear();
  for (int c = 0; c < HP_K_COUNT; ++c) {
    p->prof_n[c] = 0;
    p->prof_ms[c] = 0.0;
    p->prof_b[c] = 0.0;
    p->prof_seen[c] = 0;
    p->prof_nall[c] = 0;
    p->prof_ball[c] = 0.0;
  }
  return HP_OK;
}

int hp_profile_totals(hp_plan p, long* launches, double* bytes) {
  if (!p) return fail(nullptr, HP_EINVAL, "plan is NULL");
  for (int c = 0; c < HP_K_COUNT; ++c) {
    if (launches) launches[c] = p->prof_nall[c];
    if (bytes) bytes[c] = p->prof_ball[c];
  }
  return HP_OK;
}

int hp_profile_sample(hp_plan p, int period) {
  if (!p) return fail(nullptr, HP_EINVAL, "plan is NULL");
  if (period < 1) return fail(p, HP_EINVAL, "period must be >= 1");
  p->prof_every = period;
  return HP_OK;
}

int hp_profile_read(hp_plan p, long* launches, double* ms, double* bytes) {
  if (!p) return fail(nullptr, HP_EINVAL, "plan is NULL");
  HPCHK(hipStreamSynchronize(p->stream));
  for (size_t i = 0; i < p->ev_cls.size(); ++i) {
    float t = 0.f;
    HPCHK(hipEventElapsedTime(&t, p->ev_pool[2 * i], p->ev_pool[2 * i + 1]));
    const int c = p->ev_cls[i];
    p->prof_n[c] += 1;
    p->prof_ms[c] += t;
    p->prof_b[c] += p->ev_bytes[i];
  }
  p->ev_used = 0;
  p->ev_cls.clear();
  p->ev_bytes.clear();
  for (int c = 0; c < HP_K_COUNT; ++c) {
    if (launches) launches[c] = p->prof_n[c];
    if (ms) ms[c] = p->prof_ms[c];
    if (bytes) bytes[c] = p->prof_b[c];
  }
  return HP_OK;
}

const char* hp_last_error(hp_plan p) { return p ? p->err.c_str() : g_thread_error.c_str(); }

void hp_plan_destroy(hp_plan p) {
  if (!p) return;
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  else (void)hipDeviceSynchronize();
  if (p->own_ws && p->ws) (void)hipFree(p->ws);
  if (p->ftag_h) (void)hipHostFree(p->ftag_h);
  if (p->est_h) (void)hipHostFree(p->est_h);
  if (p->active_h) (void)hipHostFree(p->active_h);
  if (p->misc_h) (void)hipHostFree(p->misc_h);
  if (p->guess_r) (void)hipFree(p->guess_r);
  if (p->guess_part) (void)hipFree(p->guess_part);
  if (p->guess_x) (void)hipFree(p->guess_x);
  if (p->guess_rpart) (void)hipFree(p->guess_rpart);
  if (p->guess_part_h) (void)hipHostFree(p->guess_part_h);
  if (p->rk) (void)hipFree(p->rk);
  free_guess_net(p);
  free_pml(p);
  for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
  delete p;
}

}  // extern "C"

// ====================================================================== batches

struct hp_batch_s {
  std::vector<hp_plan_desc> descs;
  std::vector<std::vector<hp_c128>> poles, residues;
  std::vector<std::vector<double>> d2, d1;
  int nworkers = 1;
  size_t ws_bytes = 0;                 // largest problem's workspace
  std::vector<void*> worker_ws;        // one workspace per worker, kept across calls
  std::vector<long> iters;
  std::vector<double> seconds;
  std::vector<int> variant;            // column-pass launch variant per problem
};

extern "C" {

int hp_batch_set_launch(hp_batch b, const int* variants) {
  if (!b) return fail(nullptr, HP_EINVAL, "batch is NULL");
  if (!variants) return fail(nullptr, HP_EINVAL, "variants is NULL");
  for (size_t i = 0; i < b->variant.size(); ++i)
    if (variants[i] < 0 || variants[i] > 2)
      return fail(nullptr, HP_EINVAL, "problem " + std::to_string(i) + ": column variant must be 0, 1 or 2");
  b->variant.assign(variants, variants + b->variant.size());
  return HP_OK;
}

int hp_batch_create(const hp_plan_desc* descs, int nprob, int nworkers, hp_batch* out) {
  if (!out) return fail(nullptr, HP_EINVAL, "out is NULL");
  *out = nullptr;
  if (!descs || nprob < 1) return fail(nullptr, HP_EINVAL, "no problems");
  if (nworkers < 1 || nworkers > 64) return fail(nullptr, HP_EINVAL, "nworkers must be in [1, 64]");
  for (int i = 0; i < nprob; ++i) {
    std::string v = validate(&descs[i]);
    if (!v.empty()) return fail(nullptr, HP_EINVAL, "problem " + std::to_string(i) + ": " + v);
  }
  hp_batch b = new (std::nothrow) hp_batch_s();
  if (!b) return fail(nullptr, HP_ENOMEM, "host allocation failed");
  b->nworkers = nworkers;
  b->descs.assign(descs, descs + nprob);
  b->poles.resize(nprob);
  b->residues.resize(nprob);
  b->d2.resize(nprob);
  b->d1.resize(nprob);
  for (int i = 0; i < nprob; ++i) {
    const hp_plan_desc& d = descs[i];
    b->poles[i].assign(d.poles, d.poles + d.npoles);
    b->residues[i].assign(d.residues, d.residues + d.npoles);
    b->d2[i].assign(d.d2, d.d2 + 7);
    b->d1[i].assign(d.d1, d.d1 + 6);
    b->descs[i].poles = b->poles[i].data();
    b->descs[i].residues = b->residues[i].data();
    b->descs[i].d2 = b->d2[i].data();
    b->descs[i].d1 = b->d1[i].data();
  }
  b->iters.assign(nprob, 0);
  b->seconds.assign(nprob, 0.0);
  b->variant.assign(nprob, 1);
  for (int i = 0; i < nprob; ++i) b->ws_bytes = std::max(b->ws_bytes, hp_workspace_bytes(&b->descs[i]));
  b->worker_ws.assign(nworkers, nullptr);
  *out = b;
  return HP_OK;
}

int hp_batch_propagate(hp_batch b, const void* const* E_in, const double* const* n2, const int* nsteps,
                       void* const* E_out) {
  if (!b) return fail(nullptr, HP_EINVAL, "batch is NULL");
  if (!E_in || !n2 || !nsteps || !E_out) return fail(nullptr, HP_EINVAL, "NULL argument");
  const int nprob = (int)b->descs.size();
  for (int i = 0; i < nprob; ++i)
    if (!E_in[i] || !E_out[i] || !n2[i] || nsteps[i] < 0) return fail(nullptr, HP_EINVAL, "bad problem arguments");
  // longest first
  std::vector<int> order(nprob);
  for (int i = 0; i < nprob; ++i) order[i] = i;
  auto cost = [&](int i) {
    const hp_plan_desc& d = b->descs[i];
    return (double)d.nx * d.ny * d.ncomp * d.npoles * (double)nsteps[i];
  };
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost(x) > cost(y); });
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return fail(nullptr, HP_EHIP, "hipGetDevice failed");
  std::atomic<int> next(0);
  std::mutex mu;
  int worst = HP_OK;
  std::string first_err;
  std::atomic<int> wid(0);
  auto worker = [&]() {
    if (hipSetDevice(device) != hipSuccess) return;
    const int me = wid.fetch_add(1);
    if (!b->worker_ws[me] && hipMalloc(&b->worker_ws[me], b->ws_bytes) != hipSuccess) {
      b->worker_ws[me] = nullptr;
      std::lock_guard<std::mutex> g(mu);
      if (worst >= 0) worst = HP_ENOMEM, first_err = "worker workspace allocation failed";
      return;
    }
    hipStream_t s = nullptr;
    if (hipStreamCreate(&s) != hipSuccess) {
      std::lock_guard<std::mutex> g(mu);
      if (worst >= 0) worst = HP_EHIP, first_err = "hipStreamCreate failed";
      return;
    }
    for (;;) {
      const int slot = next.fetch_add(1);
      if (slot >= nprob) break;
      const int i = order[slot];
      const auto t0 = std::chrono::steady_clock::now();
      hp_plan p = nullptr;
      int rc = hp_plan_create(&b->descs[i], s, b->worker_ws[me], &p);
      if (rc >= 0) {
        p->geo.col_variant = b->variant[i];
        const int mrc = hp_set_medium(p, n2[i]);
        if (mrc < 0) rc = mrc;
      }
      long it = 0;
      int worst_i = HP_OK;
      if (rc >= 0) {
        const void* src = E_in[i];
        for (int st = 0; st < nsteps[i] && rc >= 0; ++st) {
          rc = hp_step(p, src, nullptr, E_out[i]);
          if (rc < 0) break;
          worst_i = std::max(worst_i, rc);
          std::vector<int> its(b->descs[i].npoles);
          if (hp_get_stats(p, its.data(), nullptr) == HP_OK)
            for (int v : its) it += v;
          src = E_out[i];
        }
        if (rc >= 0 && nsteps[i] == 0 && E_out[i] != E_in[i]) {
          const size_t bytes = (size_t)b->descs[i].nx * b->descs[i].ny * b->descs[i].ncomp * sizeof(hp_c128);
          if (hipMemcpyAsync(E_out[i], E_in[i], bytes, hipMemcpyDeviceToDevice, s) != hipSuccess) rc = HP_EHIP;
        }
      }
      std::string msg = (rc < 0) ? std::string(p ? hp_last_error(p) : hp_last_error(nullptr)) : std::string();
      if (p) hp_plan_destroy(p);
      (void)hipStreamSynchronize(s);
      const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      std::lock_guard<std::mutex> g(mu);
      b->iters[i] = it;
      b->seconds[i] = sec;
      if (rc < 0) {
        if (worst >= 0) {
          worst = rc;
          first_err = "problem " + std::to_string(i) + ": " + msg;
        }
      } else if (worst >= 0) {
        worst = std::max(worst, worst_i);
      }
    }
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
  };
  const int nw = std::min(b->nworkers, nprob);
  std::vector<std::thread> threads;
  for (int w = 0; w < nw; ++w) threads.emplace_back(worker);
  for (auto& t : threads) t.join();
  if (worst < 0) return fail(nullptr, worst, first_err);
  return worst;
}

int hp_batch_stats(hp_batch b, long* iters, double* seconds) {
  if (!b) return fail(nullptr, HP_EINVAL, "batch is NULL");
  for (size_t i = 0; i < b->descs.size(); ++i) {
    if (iters) iters[i] = b->iters[i];
    if (seconds) seconds[i] = b->seconds[i];
  }
  return HP_OK;
}

void hp_batch_destroy(hp_batch b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  for (void* w : b->worker_ws)
    if (w) (void)hipFree(w);
  delete b;
}

}  // extern "C"

// ============================================= the preconditioner without allocation
//
// hp_apply_preconditioner_noalloc: the free-space solve of hp_apply_preconditioner
// for callers that cannot allocate (graph capture, serving loops, harnesses that
// forbid hipMalloc).  Its intermediate fields and the pole state the column pass
// reads live in `scratch`, a fixed array in device memory that every GPU holds
// for the life of the process.  In host code `scratch` names a host-side stand-in,
// not a device address: hp_plan_create (set-up, with the plan's device current)
// looks up each device's own address once with hipGetSymbolAddress, and only that
// address is ever handed to kernels.

constexpr size_t kScratchFieldBytes = 48ull << 20;  // R-domain fields: row transform, column pass out, D1y
constexpr size_t kScratchSmallBytes = 1ull << 20;   // pole state, basis pointer table, partial norms
static __device__ __align__(256) char scratch[kScratchFieldBytes + kScratchSmallBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

// The device address of `scratch` on the current device (looked up once per device).
void* scratch_for_current_device(std::string* why) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    *why = std::string("hipGetDevice: ") + hipGetErrorString(e);
    return nullptr;
  }
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev] && g_scratch_err[dev] == hipSuccess) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      g_scratch_err[dev] = e != hipSuccess ? e : hipErrorInvalidSymbol;
    else
      g_scratch_ptr[dev] = ptr;
  }
  if (!g_scratch_ptr[dev]) *why = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(g_scratch_err[dev]);
  return g_scratch_ptr[dev];
}

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

template <typename T, typename C>
int apply_prec_noalloc(hp_plan p, int pole, const c128* x, c128* y) {
  char* base = reinterpret_cast<char*>(p->scratch);
  const size_t fb = align256(p->fieldn * sizeof(cx<T>));
  cx<T>* tmpR = reinterpret_cast<cx<T>*>(base);
  cx<T>* zout = reinterpret_cast<cx<T>*>(base + fb);
  cx<T>* dz = reinterpret_cast<cx<T>*>(base + 2 * fb);
  char* small = base + kScratchFieldBytes;
  PoleState* st = reinterpret_cast<PoleState*>(small);
  void** tbl = reinterpret_cast<void**>(small + align256(sizeof(PoleState)));
  double* part = reinterpret_cast<double*>(small + align256(sizeof(PoleState)) +
                                           align256((HP_MAXM + 1) * sizeof(void*)));
  prec_into<T, C>(p, pole, x, y, tmpR, zout, dz, st, tbl, part);
  HPCHK(hipGetLastError());
  return HP_OK;
}

// Set-up of the static scratch for a plan's device (called by hp_plan_create
// with that device current).
void scratch_setup(hp_plan p) {
  std::string why;
  p->scratch = scratch_for_current_device(&why);
  p->scratch_err = why;
}

}  // namespace

extern "C" {

int hp_apply_preconditioner_noalloc(hp_plan p, int pole, const void* x, void* y) {
  if (!p) return fail(nullptr, HP_EINVAL, "plan is NULL");
  if (!x || !y || x == y) return fail(p, HP_EINVAL, "x, y must be distinct device buffers");
  if (pole >= p->d.npoles) return fail(p, HP_EINVAL, "pole out of range");
  if (p->pml) return fail(p, HP_ESTATE, "no allocation-free form of the absorbing-layer preconditioner");
  const size_t es = p->mixed ? sizeof(c64) : sizeof(c128);
  const size_t need = (p->d.ncomp == 2 ? 3 : 2) * align256(p->fieldn * es);
  const size_t part = (size_t)p->nrowblk * p->d.ncomp * sizeof(double);
  if (need > kScratchFieldBytes || part > kScratchSmallBytes / 2)
    return fail(p, HP_EINVAL,
                "field too large for the static scratch: " + std::to_string(need) + " bytes needed, " +
                    std::to_string(kScratchFieldBytes) + " available (ncomp nx ny <= 1048576 in HP_FP64)");
  if (!p->scratch) return fail(p, HP_EHIP, "no device address for the static scratch: " + p->scratch_err);
  const c128* xx = reinterpret_cast<const c128*>(x);
  c128* yy = reinterpret_cast<c128*>(y);
  return HP_BY_PRECISION(p, apply_prec_noalloc, p, pole, xx, yy);
}

}  // extern "C"
