// Internal declarations shared by the HIP kernels and the host engine.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "fisherbt.h"

namespace fbt {

constexpr int NB = 256;        // block size of the tiled factorisation and solves
constexpr int NLEV = 5;        // quadrature step levels of the Bessel integrals
constexpr int TAB_L0 = 256;    // nodes of level 0 (step 0.2)
constexpr int TAB_LN = 64;     // nodes of levels 1..NLEV-1
constexpr int TAB_MAX = TAB_L0 + (NLEV - 1) * TAB_LN;

// Quadrature node of the scaled integrals (see fbt_kernels.hip):
//   cm1 = cosh(t) - 1,  wk = w cosh(nu t),  wk1 = w cosh((nu-1) t),  wd = w t sinh(nu t),
//   wkp, wkm = w cosh((nu +- PAPER_LAG) t) (paper mode only; zero otherwise)
struct Node {
    double cm1, wk, wk1, wd, wkp, wkm;
};

// Paper mode: dC/dnu by the case scheme of Supplementary A (see fbt_kernels.hip).
constexpr double PAPER_LAG = 1e-9;  // case 5: central difference in nu
constexpr int PC_SER = 20;          // case 2: terms of the power series
constexpr int PC_DEB = 34;          // case 3: coefficients per polynomial in p (12 terms)
constexpr int PC_HAN = 5;           // case 4: terms of the Hankel expansion
// coefficient table layout (doubles)
constexpr int PC_A1 = 0;                          // A'_k
constexpr int PC_B0 = PC_A1 + PC_SER;             // B_k
constexpr int PC_B1 = PC_B0 + PC_SER;             // B'_k
constexpr int PC_D12 = PC_B1 + PC_SER;            // S0, S1, S2 for 12 terms (3 x PC_DEB)
constexpr int PC_D8 = PC_D12 + 3 * PC_DEB;        // S0, S1, S2 for 8 terms
constexpr int PC_HA = PC_D8 + 3 * PC_DEB;         // a_k
constexpr int PC_HB = PC_HA + PC_HAN;             // a_k b_k
constexpr int PC_LOGNU = PC_HB + PC_HAN;          // log nu
constexpr int PC_SQPI = PC_LOGNU + 1;             // sqrt(pi / (2 nu))
constexpr int PC_SIZE = PC_SQPI + 1;

struct GenParams {
    double sigma2, alpha, nu, abs_nu;
    double cnu;        // 2^(1-nu) / Gamma(nu)
    double log2_psi;   // log 2 + psi(nu)
    double h[NLEV];    // trapezoid step of each level
    double xtop[NLEV]; // level L serves x <= xtop[L]
    int off[NLEV];     // first node of each level in the table
    int len[NLEV];     // nodes of each level
    int paper;         // 1: Sigma_nu by the case scheme (paper mode)
    int fd_small;      // paper mode: nu within 1e-6 of an integer (case 5 for x < 8.5)
    int fd_large;      // paper mode: nu + 1/2 within 1e-6 of an integer (case 5 for x >= 30)
    const double *pc;  // paper mode coefficient table (device, PC_SIZE doubles)
    const Node *tab;   // quadrature node table (device, TAB_MAX nodes)
    int64_t n;         // observations
    int64_t npad;      // padded order (multiple of NB, > n)
    int64_t ld;        // leading dimension of the matrices
};

enum GenMode { GEN_SIGMA = 1, GEN_DERIV = 2, GEN_ALL = 3 };

// node table followed by the paper-mode coefficient table (one upload per theta)
constexpr size_t TAB_BYTES = TAB_MAX * sizeof(Node) + PC_SIZE * sizeof(double);

// Generation parameters for theta = (sigma2, alpha, nu): prefactors, and the
// quadrature node table (plus, with paper_mode, the coefficient table of the
// paper's scheme) written to host_tab (TAB_BYTES) for upload to dev_tab.
GenParams theta_params(const double *th, int paper_mode, int64_t n, int64_t npad, int64_t ld,
                       void *host_tab, const void *dev_tab);

// Field batching.  One launch can cover `count` independent fields of the same
// padded order whose buffers are laid out one after another with uniform
// strides (in elements): field f (blockIdx.z, or the dimension a kernel
// documents) uses each pointer offset by f times the stride of its buffer.
// A single field is count = 1 with all offsets zero.
struct Fields {
    int count;
    int64_t sA;    // factor / covariance matrix (npad x npad)
    int64_t sS2;   // derivative pair (npad x 2 npad)
    int64_t sLinv; // diagonal-block inverses (T NB^2)
    int64_t sVec;  // npad-vectors (locations, observations, w)
    int64_t sPart; // partial sums
    int64_t sLog;  // log-det partials (T)
    const int64_t *n; // per-field n (device; nullptr: the launch's n for every field)
    int64_t sXf;   // FP32 copies of a pair of solved block rows (2 x 2 NB x 2 npad floats)
};

// kernel launchers (fbt_kernels.hip); all asynchronous on `s`.  Launchers
// with a `Fields` argument process F.count fields (see above); gpa then holds
// one GenParams per field (device memory for count > 1).
void launch_gen(hipStream_t s, const GenParams &gp, const GenParams *gpa, const Fields &F,
                const double *xs, const double *ys, const double *z, double *S, double *Sa,
                double *Sn, int mode);
void launch_init_info(hipStream_t s, int *info, int count);
void launch_potrf_diag(hipStream_t s, const Fields &F, double *A, int64_t lda, int k, int64_t n,
                       double *Linv, double *logdet_part, int *info);
void launch_panel(hipStream_t s, const Fields &F, double *P, int64_t ld, int64_t rows,
                  const double *Linv);
// sC: stride of C0/C1/A0/A1 (F.sA or F.sS2), sB: stride of B (F.sA)
void launch_update_lower(hipStream_t s, const Fields &F, int64_t sC, int64_t sB, int nmat,
                         double *C0, double *C1, int64_t ldc, const double *A0,
                         const double *A1, int64_t lda, const double *B, int64_t ldb, int nblk,
                         int K, int mixed);
void launch_update_rect(hipStream_t s, const Fields &F, int64_t sC, int64_t sB, int nmat,
                        double *C0, double *C1, int64_t ldc, const double *A0, const double *A1,
                        int64_t lda, const double *B, int64_t ldb, int64_t rows, int64_t ncol,
                        int K, int mixed);
// sS: stride of S (F.sS2, or F.sA for the adjoint's inverse)
// With Xf (FP32 form of the left solve), the solved rows are also stored as
// floats at Xf[(kofs + row) + col * 2 NB] (per field offset F.sXf).
void launch_diag_apply(hipStream_t s, const Fields &F, int64_t sS, int nmat, double *S,
                       int64_t ld, int64_t krow, const double *Linv, int64_t ncols,
                       int64_t col_shift, float *Xf = nullptr, int kofs = 0);
// FP32 (or, with bf16, BF16) form of the left-solve update from FP32 operand
// copies: S[r0.., cols] -= Lf[r0.., krow:krow+NB] * Xf[kofs:kofs+NB, cols] (one
// NB-deep slice; Lf per field offset F.sA, Xf as written by launch_diag_apply)
void launch_update_nn_f32(hipStream_t s, const Fields &F, int64_t sS, int nmat, double *S,
                          int64_t ld, const float *Lf, int64_t r0, int64_t krow, const float *Xf,
                          int kofs, int64_t rows, int64_t ncols, int64_t col_shift, bool bf16);
// Lf = (float) A on the block-lower part (NB blocks at or below the diagonal)
void launch_to_f32_lower(hipStream_t s, const Fields &F, const double *A, int64_t ld, int64_t npad,
                         float *Lf);
void launch_update_nn(hipStream_t s, const Fields &F, int64_t sS, int nmat, double *S, int64_t ld,
                      const double *L, int64_t lda, int64_t r0, int64_t krow, int64_t rows,
                      int64_t ncols, int64_t col_shift, int K, int mixed);
void launch_panel_reduce(hipStream_t s, const Fields &F, double *Xa, double *Xn, int64_t ld,
                         int64_t r0, int64_t kcol, int64_t rows, const double *Linv, int64_t n,
                         double *partials);
void launch_reduce_loglik(hipStream_t s, const Fields &F, const double *A, int64_t lda,
                          int64_t n, int T, const double *logdet_part, double *out);
void launch_reduce_terms(hipStream_t s, const Fields &F, const double *partials, int64_t count,
                         double *out);
// two-sided reduction of the W phase (see fbt_kernels.hip).  Both derivative
// matrices: matrix 1 at +mofs (S2), +vofs (Vd), +ymofs (Y); per-field strides
// sPd, sVd, sY (Pd, Vd, Y), F.sS2 (S2), F.sA (A), F.sLinv, F.sPart.
void launch_sygst_diag(hipStream_t s, const Fields &F, const double *S2, int64_t ld, int64_t mofs,
                       int64_t krow, const double *Linv, double *Pd, int64_t sPd, double *Vd,
                       int64_t vofs, int64_t sVd);
void launch_sygst_panel(hipStream_t s, const Fields &F, double *S2, int64_t ld, int64_t mofs,
                        const double *A, int64_t r0, int64_t rows, int64_t krow,
                        const double *Linv, const double *Vd, int64_t vofs, int64_t sVd,
                        double *Y, int64_t ldy, int64_t ymofs, int64_t sY);
// Rank-2k lower update of the trailing part (the blocks among the first `skip`
// block rows are left out).  mixed: 0 FP64, 1 FP32 MFMA with FP32 sums per
// NB-deep slice, 2 BF16 operands
void launch_syr2k_lower(hipStream_t s, const Fields &F, double *S2, int64_t ld, int64_t mofs,
                        const double *A, int64_t t0, int nblk, int64_t kcol, int KS,
                        const double *Y, int64_t ldy, int64_t ymofs, int64_t sY, int skip,
                        int mixed);
void launch_syr2k_rect(hipStream_t s, const Fields &F, double *S2, int64_t ld, int64_t mofs,
                       const double *A, int64_t r0, int64_t rows, int64_t c0, int64_t ncol,
                       int64_t kcol, int KS, const double *Y, int64_t ldy, int64_t ymofs,
                       int64_t sY, int mixed);
void launch_zero_diag_blocks(hipStream_t s, const Fields &F, double *S2, int64_t ld, int64_t mofs,
                             int k0, int count);
void launch_sygst_reduce(hipStream_t s, const Fields &F, const double *S2, int64_t ld,
                         int64_t mofs, const double *Vd, int64_t vofs, int64_t sVd, int T,
                         int64_t n, double *partials);
// allocation-free entry point: SoA observations (npad, zero padded) from the
// caller's device arrays; flag[0] = 1 if an input is not finite
void launch_pack_data(hipStream_t s, const double *locs, const double *zin, int64_t n, int64_t npad,
                      double *x, double *y, double *z, double *flag);
// iterative refinement of w = Sigma^{-1} Z (FBT_MIXED_FP32_ALL): x <- L^{-1} x
// (trans 0) or L^{-T} x (trans 1) on the block-lower factor with its diagonal
// inverses
void launch_trsv(hipStream_t s, double *x, const double *L, int64_t ld, int64_t npad,
                 const double *Linv, int trans);
// x <- Sigma^{-1} x: L^{-1} with the bordered factor, the border and padding
// entries cleared, then L^{-T}
void launch_solve_sigma(hipStream_t s, double *x, const double *L, int64_t ld, int64_t n,
                        int64_t npad, const double *Linv);
// Sc (n x n, both triangles, leading dimension ld) = Sigma from A's lower triangle
void launch_copy_sym(hipStream_t s, const double *A, int64_t ld, int64_t n, double *Sc);
// r = z - Sc w (part: npad x nq doubles of partial products)
void launch_residual(hipStream_t s, const double *Sc, int64_t ld, int64_t n, int64_t npad,
                     const double *z, const double *w, int nq, double *part, double *r);
// out[0] = w^T M w (M n x n, both triangles)
void launch_quad_form(hipStream_t s, const double *M, int64_t ld, int64_t n, int64_t npad,
                      const double *w, int nq, double *part, double *out);
// w = row n of the bordered factor (y = L^{-1} Z), zero from n on
void launch_border_row(hipStream_t s, const double *A, int64_t ld, int64_t n, int64_t npad,
                       double *w);
// x += d and out[0] = z^T x (d or out may be null)
void launch_axpy_dot(hipStream_t s, double *x, const double *d, const double *z, int64_t n,
                     int64_t npad, double *out);
// adjoint gradient
void launch_fill_identity(hipStream_t s, double *X, int64_t ld, int64_t rows, int64_t ncols);
void launch_lauum(hipStream_t s, double *P, const double *X, int64_t ld, int64_t npad,
                  int64_t ncols);
void launch_extract_w(hipStream_t s, const double *X, int64_t ld, int64_t n, double *w);
void launch_adjoint(hipStream_t s, const GenParams &gp, const double *xs, const double *ys,
                    const Node *tab, const double *P, const double *w, double *part);
void launch_reduce_pairs(hipStream_t s, const double *part, int64_t count, double *out);

// Batched group of fields of one padded order (fbt_engine.hip), used by the
// batch executor; see the definitions for the contract.  group_run is
// prepare + stage + enqueue + wait + results; a graph captures group_enqueue.
fbt_status group_run(fbt_ctx *c, int G, const int64_t *n, const double *const *locs,
                     const double *const *z, const double *thetas, int mode, double *loglik,
                     double *score, double *fisher, int32_t *status);
fbt_status group_prepare(fbt_ctx *c, int G, const int64_t *n, const double *const *locs,
                         const double *const *z);
void group_stage(fbt_ctx *c, const double *thetas, int *bad);
fbt_status group_enqueue(fbt_ctx *c, int mode);
fbt_status group_results(fbt_ctx *c, int mode, const double *thetas, const int *bad,
                         double *loglik, double *score, double *fisher, int32_t *status);
hipStream_t ctx_stream(fbt_ctx *c);
// Restrict the context to streams a HIP graph capture accepts (no CU-masked stream).
void ctx_set_capturable(fbt_ctx *c, bool on);

// Persistent round execution of batched fields (fbt_round.hip): one launch
// evaluates every field of a call (mode 1: Algorithm 2, 2: Algorithm 3; other
// modes are left out) with BT x BT tiles (bt = 64 or 128).  The device arena
// and the task order are rebuilt when the field set (version), the modes or
// bt change.  Per-field status as fbt_batch_eval; returns FBT_EDEVICE /
// FBT_ENOMEM / FBT_EINVAL with *err on failure of the whole call.
struct RoundExec;
RoundExec *round_create(int device);
void round_destroy(RoundExec *r);
fbt_status round_eval(RoundExec *r, int bt, int nf, const int64_t *n, const double *const *locs,
                      const double *const *z, uint64_t version, const double *thetas,
                      const int32_t *mode, double *loglik, double *score, double *fisher,
                      int32_t *status, std::string *err);
float round_last_ms(const RoundExec *r);          // kernel time of the last call
double round_plan_estimate_us(const RoundExec *r); // planner's makespan estimate
int round_task_count(const RoundExec *r);
// per-task trace of later calls (wall-clock ticks at ticket, waits done, end);
// round_trace copies the last call's: 5 int64 per task (ft, ij, times), up
// to cap tasks; returns the task count (0: no trace)
void round_set_trace(RoundExec *r, bool on);
// later calls (without trace) replay a HIP graph of the round, captured once
// per arena
void round_set_graph(RoundExec *r, bool on);
// task queues (1..8; a new plan at the next call when it changes)
void round_set_queues(RoundExec *r, int queues);
int round_queues(const RoundExec *r);
int64_t round_trace(const RoundExec *r, int64_t *out, int64_t cap);

// Eq. (1) from log det and the quadratic form; Eqs. (1)-(3) from the nine
// terms (log det, q, tr W_a, tr W_n, y'W_a y, y'W_n y, <W_a,W_a>, <W_a,W_n>,
// <W_n,W_n>).
double loglik_terms(int64_t n, double logdet, double quad);
void assemble_terms(int64_t nobs, const double *theta, const double *t, double *loglik,
                    double *score, double *fisher);

// Derivative evaluation of the Fisher-BT driver with the switch from a mixed
// precision to FP64 near the optimum (fbt_fit_options.mixed_switch);
// *state becomes 1 at the switch.  Defined in fbt_engine.hip.
fbt_status fit_eval(fbt_ctx *c, const double *th, double mixed_switch, int *state,
                    double *loglik, double *score, double *fisher);
// the context's fbt_precision
int ctx_precision(const fbt_ctx *c);

}  // namespace fbt
