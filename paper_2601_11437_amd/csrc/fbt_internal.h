// Internal declarations shared by the HIP kernels and the host engine.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fbt {

constexpr int NB = 256;        // block size of the tiled factorisation and solves
constexpr int NLEV = 5;        // quadrature step levels of the Bessel integrals
constexpr int TAB_L0 = 256;    // nodes of level 0 (step 0.2)
constexpr int TAB_LN = 64;     // nodes of levels 1..NLEV-1
constexpr int TAB_MAX = TAB_L0 + (NLEV - 1) * TAB_LN;

// Quadrature node of the scaled integrals (see fbt_kernels.hip):
//   cm1 = cosh(t) - 1,  wk = w cosh(nu t),  wk1 = w cosh((nu-1) t),  wd = w t sinh(nu t)
struct Node {
    double cm1, wk, wk1, wd;
};

struct GenParams {
    double sigma2, alpha, nu, abs_nu;
    double cnu;        // 2^(1-nu) / Gamma(nu)
    double log2_psi;   // log 2 + psi(nu)
    double h[NLEV];    // trapezoid step of each level
    double xtop[NLEV]; // level L serves x <= xtop[L]
    int off[NLEV];     // first node of each level in the table
    int len[NLEV];     // nodes of each level
    int64_t n;         // observations
    int64_t npad;      // padded order (multiple of NB, > n)
    int64_t ld;        // leading dimension of the matrices
};

enum GenMode { GEN_SIGMA = 1, GEN_DERIV = 2, GEN_ALL = 3 };

// kernel launchers (fbt_kernels.hip); all asynchronous on `s`
void launch_gen(hipStream_t s, const GenParams &gp, const double *xs, const double *ys,
                const double *z, const Node *tab, double *S, double *Sa, double *Sn, int mode);
void launch_init_info(hipStream_t s, int *info);
void launch_potrf_diag(hipStream_t s, double *A, int64_t lda, int k, int64_t n, double *Linv,
                       double *logdet_part, int *info);
void launch_panel(hipStream_t s, double *P, int64_t ld, int64_t rows, const double *Linv);
void launch_update_lower(hipStream_t s, int nmat, double *C0, double *C1, int64_t ldc,
                         const double *A0, const double *A1, int64_t lda, const double *B,
                         int64_t ldb, int nblk, int mixed);
void launch_update_rect(hipStream_t s, int nmat, double *C0, double *C1, int64_t ldc,
                        const double *A0, const double *A1, int64_t lda, const double *B,
                        int64_t ldb, int64_t rows, int mixed);
void launch_diag_apply(hipStream_t s, double *S, int64_t ld, int64_t krow, const double *Linv,
                       int64_t ncols, int64_t col_shift);
void launch_update_nn(hipStream_t s, double *S, int64_t ld, const double *L, int64_t lda,
                      int64_t r0, int64_t krow, int64_t rows, int64_t ncols, int64_t col_shift,
                      int mixed);
void launch_panel_reduce(hipStream_t s, double *Xa, double *Xn, int64_t ld, int64_t r0,
                         int64_t kcol, int64_t rows, const double *Linv, int64_t n,
                         double *partials);
void launch_reduce_loglik(hipStream_t s, const double *A, int64_t lda, int64_t n, int T,
                          const double *logdet_part, double *out);
void launch_reduce_terms(hipStream_t s, const double *partials, int64_t count, double *out);

}  // namespace fbt
