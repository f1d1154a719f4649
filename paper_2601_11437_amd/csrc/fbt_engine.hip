// Host engine and C ABI: context and device buffers, per-theta setup of the
// Bessel quadrature tables, and the launch sequences of Algorithm 2
// (log-likelihood) and Algorithm 3 (log-likelihood, score, Fisher).
#include "fisherbt.h"
#include "fbt_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace fbt;

namespace {

constexpr int NCLASS = 18;
enum KClass {
    KC_GEN, KC_DIAG, KC_PANEL, KC_SYRK, KC_LAPPLY, KC_LUPD, KC_RPANEL, KC_RUPD, KC_RED,
    KC_INV,   // adjoint: X = L'^{-1} (diagonal apply and updates)
    KC_LAUUM, // adjoint: P = X^T X
    KC_ADJ,   // adjoint: contraction with the regenerated derivatives
    KC_SDIAG, // two-sided W phase: diagonal blocks W_kk
    KC_SPANEL,// two-sided W phase: panels Y, M
    KC_SUPD,  // two-sided W phase: symmetric rank-2k trailing updates
    KC_DAPPLY,// two-sided W phase: deferred solve, diagonal apply
    KC_DUPD,  // two-sided W phase: deferred solve, updates
    KC_SLOOK  // two-sided W phase: rank-2k updates of the next block columns (lookahead)
};

struct Timed {
    int cls;
    double flops;
    hipEvent_t a, b;
};

} // namespace

struct fbt_ctx {
    int device = 0;
    hipStream_t stream = nullptr;  // s0: the caller's stream; the critical path runs here
    hipStream_t stream2 = nullptr; // s1: bulk trailing updates (lookahead), joined back to s0
    hipStream_t stream3 = nullptr; // s1 of the factorisation: bulk updates on all CUs but a reserve
    hipEvent_t evP = nullptr, evB = nullptr;
    hipStream_t stream4 = nullptr; // two-sided W phase: the deferred solve's critical path
    hipEvent_t evP2 = nullptr, evB2 = nullptr, evD = nullptr; // its chain, bulk and end
    bool own_stream = false;
    int precision = FBT_FP64; // see fbt_precision
    int sigma_nu_mode = FBT_SIGMA_NU_EXACT;
    std::string err;
    int64_t notpd = -1;

    int64_t n = 0, npad = 0, ld = 0, ncols = 0;
    int T = 0;
    double *x = nullptr, *y = nullptr, *z = nullptr;
    double *A = nullptr;  // Sigma' -> bordered factor L' (lower)
    double *S2 = nullptr; // [Sigma_alpha' | Sigma_nu'] -> X -> W (npad x 2 npad)
    double *Linv = nullptr, *logdet = nullptr, *partials = nullptr, *out = nullptr;
    double *wv = nullptr; // w = Sigma^{-1} Z (adjoint gradient; refinement)
    double *rv = nullptr; // refinement: residual / correction (npad) and matvec partials (8 npad)
    double *Sc = nullptr; // refinement: Sigma (both triangles) taken before the factorisation
    size_t cap_sc = 0;
    int refine_iters = 0; // FBT_MIXED_FP32_ALL: refinement steps of w (fbt_set_refinement)
    int *info = nullptr;
    Node *tab = nullptr;   // per field: node table + paper-mode coefficients (TAB_BYTES)
    Node *h_tab = nullptr; // pinned staging
    double *h_out = nullptr;
    int *h_info = nullptr;
    size_t cap[24] = {0};  // allocated bytes per buffer (buffers only grow)
    // FBT_MIXED_FP32 and _BF16: FP32 copies of the factor's block-lower part (same layout
    // as A) and of the left solve's current pair of solved block rows (two
    // slots of 2 NB x 2 npad floats, by pair parity); allocated on the first
    // evaluation in that form, and optional (without them the solve converts
    // the FP64 operands when staging, with bitwise the same results)
    float *Lf = nullptr, *Xf = nullptr;
    size_t cap_lf = 0, cap_xf = 0;
    // W phase by the two-sided reduction (FBT_WPHASE_TWO_SIDED, FP64): Y of the
    // current pair of block steps (two slots by pair parity, both matrices,
    // npad x 2 NB each), V_k = -W_kk / 2 of every step (both matrices, T NB^2
    // each) and the diagonal kernel's scratch (2 NB^2); allocated at the first
    // evaluation in that form
    int wphase = FBT_WPHASE_TWO_SIDED;
    double *Ysl = nullptr, *Vd = nullptr, *Pd = nullptr;
    size_t cap_ysl = 0, cap_vd = 0, cap_pd = 0;

    // fields held: 1 for the single-field API; G >= 1 inside a batched group
    int G = 1;
    bool batched = false;          // per-field n and theta from device arrays, per-field status
    // work may be captured in a HIP graph: only non-blocking streams (the
    // CU-masked stream3 is a blocking stream and synchronises with the
    // legacy default stream, which a capture does not allow)
    bool capturable = false;
    Fields F{};
    int64_t *d_nf = nullptr;       // per-field n (device)
    GenParams *d_gpa = nullptr;    // per-field generation parameters (device)
    GenParams *h_gpa = nullptr;    // pinned staging
    std::vector<int64_t> nf;       // per-field n (host)
    std::vector<int> fst;          // per-field status of the last group call
    std::vector<double> fout;      // per-field {log det, y^T y}

    bool factor_valid = false;
    double factor_theta[3] = {0, 0, 0};
    double factor_out[2] = {0, 0};

    bool timing = false;
    std::vector<Timed> pending;
    std::vector<hipEvent_t> pool;
    size_t pool_used = 0;
    int64_t cls_n[NCLASS] = {0};
    double cls_ms[NCLASS] = {0}, cls_flops[NCLASS] = {0};
};

namespace {

// CUs kept free of the factorisation's bulk stream: one per XCD of MI355X
constexpr int FACT_CU_RESERVE = 8;
// The factorisation steps one block column at a time over its last
// FACT_SINGLE_TAIL blocks (two elsewhere): there the critical chain, not the
// trailing update, bounds each step, and a 2 NB-deep lookahead update would
// lengthen the chain (its time is per-workgroup latency, not throughput).
constexpr int FACT_SINGLE_TAIL = 40;
// While more than FACT_QUAD_ABOVE blocks remain the steps take four block
// columns: the trailing matrix is large, the chain has slack, and the bulk
// update runs 1,024 deep per pass over its C tiles instead of 512 (bitwise
// the same results).
constexpr int FACT_QUAD_ABOVE = 48;
// column chunks of the refinement's matrix-vector products (workgroups per
// 256 rows; 79 x 8 at n = 20,000)
constexpr int REFINE_NQ = 8;


fbt_status fail(fbt_ctx *c, fbt_status s, const std::string &m)
{
    if (c)
        c->err = m;
    return s;
}

#define HIPCHK(ctx, expr)                                                                          \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(ctx, FBT_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_));       \
    } while (0)

bool theta_ok(const double *th)
{
    return th && std::isfinite(th[0]) && std::isfinite(th[1]) && std::isfinite(th[2]) &&
           th[0] > 0 && th[1] > 0 && th[2] > 0;
}

// psi(v), v > 0: recurrence psi(v) = psi(v + 1) - 1/v up to v >= 12, then the
// asymptotic expansion log v - 1/(2v) - sum_{k=1..6} B_2k / (2k v^2k).
double digamma(double v)
{
    double acc = 0.0;
    for (; v < 12.0; v += 1.0)
        acc -= 1.0 / v;
    const double f = 1.0 / (v * v);
    const double tail =
        f * (0.083333333333333333 -
             f * (0.0083333333333333333 -
                  f * (0.0039682539682539683 -
                       f * (0.0041666666666666667 - f * (0.0075757575757575758 - f * 0.021092796092796093)))));
    return acc + std::log(v) - 0.5 / v - tail;
}

// Coefficients c_j^(k) of the Debye polynomials U_k(p) = sum_j c_j^(k) p^j,
// k < 12, by the recurrence that follows from
//   U_{k+1}(p) = p^2 (1 - p^2) U_k'(p) / 2 + (1/8) int_0^p (1 - 5 t^2) U_k(t) dt:
//   c_j^(k+1) = (j - 1 + 1/(4j)) c_{j-1}^(k) / 2 - (j - 3 + 5/(4j)) c_{j-3}^(k) / 2.
struct Debye {
    double c[12][PC_DEB];
    Debye()
    {
        std::memset(c, 0, sizeof(c));
        c[0][0] = 1.0;
        for (int k = 0; k + 1 < 12; ++k)
            for (int j = 1; j <= 3 * (k + 1); ++j) {
                double v = 0.5 * (j - 1 + 0.25 / j) * c[k][j - 1];
                if (j >= 3)
                    v -= 0.5 * (j - 3 + 1.25 / j) * c[k][j - 3];
                c[k + 1][j] = v;
            }
    }
};

// Paper mode coefficient table for theta (layout in fbt_internal.h):
//  case 2: term k of d/dnu[x^nu K_nu] is (x/2)^{2k} (A'_k + x^{2 nu} (B'_k + 2 log x B_k)),
//    A'_k = 2^nu (log 2 + psi(nu) - d_k(-nu)) Gamma(nu) g_k(-nu) / (2 k!),
//    B_k  = 2^-nu Gamma(-nu) g_k(nu) / (2 k!),  B'_k = B_k (-log 2 - psi(-nu) + d_k(nu)),
//    g_k(v) = prod_{j<=k} 1/(v + j),  d_k(v) = -sum_{j<=k} 1/(v + j);
//  case 3: S0 = sum_k (-1)^k nu^-k U_k, S1 = sum_k (-1)^k k nu^{-k-1} U_k,
//    S2 = sum_k (-1)^k nu^-k U_k' as polynomials in p, for 12 and for 8 terms;
//  case 4: a_k = prod_{j<=k} (4 nu^2 - (2j-1)^2) / (8^k k!),
//    b_k = sum_{j<=k} 8 nu / (4 nu^2 - (2j-1)^2); stored a_k and a_k b_k.
void paper_coefficients(const GenParams &gp, double *pc)
{
    static const Debye U;
    const double nu = gp.nu, ln2 = std::log(2.0);
    std::memset(pc, 0, PC_SIZE * sizeof(double));
    if (!gp.fd_small) {
        const double gn = std::tgamma(nu), gmn = std::tgamma(-nu);
        const double pn = digamma(nu), pmn = digamma(-nu);
        double gkm = 1.0, gkp = 1.0, dkm = 0.0, dkp = 0.0, fact = 1.0;
        for (int k = 0; k < PC_SER; ++k) {
            if (k > 0) {
                gkm /= (-nu + k);
                gkp /= (nu + k);
                dkm -= 1.0 / (-nu + k);
                dkp -= 1.0 / (nu + k);
                fact *= k;
            }
            pc[PC_A1 + k] = std::pow(2.0, nu) * (ln2 + pn - dkm) * gn * gkm / (2.0 * fact);
            pc[PC_B0 + k] = std::pow(2.0, -nu) * gmn * gkp / (2.0 * fact);
            pc[PC_B1 + k] = pc[PC_B0 + k] * (-ln2 - pmn + dkp);
        }
    }
    for (int set = 0; set < 2; ++set) {
        const int K = set == 0 ? 12 : 8;
        double *d = pc + (set == 0 ? PC_D12 : PC_D8);
        for (int k = 0; k < K; ++k) {
            const double sg = (k & 1) ? -1.0 : 1.0, nk = std::pow(nu, -k);
            for (int j = 0; j < PC_DEB; ++j) {
                d[j] += sg * nk * U.c[k][j];
                d[PC_DEB + j] += sg * k * nk / nu * U.c[k][j];
                if (j + 1 < PC_DEB)
                    d[2 * PC_DEB + j] += sg * nk * (j + 1) * U.c[k][j + 1];
            }
        }
    }
    if (!gp.fd_large) {
        double a = 1.0, b = 0.0;
        for (int k = 0; k < PC_HAN; ++k) {
            if (k > 0) {
                const double f = 4.0 * nu * nu - double(2 * k - 1) * double(2 * k - 1);
                a *= f / (8.0 * k);
                b += 8.0 * nu / f;
            }
            pc[PC_HA + k] = a;
            pc[PC_HB + k] = a * b;
        }
    }
    pc[PC_LOGNU] = std::log(nu);
    pc[PC_SQPI] = std::sqrt(M_PI / (2.0 * nu));
}

} // namespace

// Quadrature tables and prefactors for theta (see the generation kernel).
GenParams fbt::theta_params(const double *th, int paper_mode, int64_t n, int64_t npad, int64_t ld,
                            void *host_tab, const void *dev_tab)
{
    GenParams gp;
    std::memset(&gp, 0, sizeof(gp));
    Node *htab = reinterpret_cast<Node *>(host_tab);
    const Node *dtab = reinterpret_cast<const Node *>(dev_tab);
    gp.sigma2 = th[0];
    gp.alpha = th[1];
    gp.nu = th[2];
    gp.abs_nu = std::fabs(th[2]);
    gp.cnu = std::exp((1.0 - gp.nu) * std::log(2.0) - std::lgamma(gp.nu));
    gp.log2_psi = std::log(2.0) + digamma(gp.nu);
    gp.n = n;
    gp.npad = npad;
    gp.ld = ld;
    gp.tab = dtab;
    const bool paper = paper_mode != 0;
    gp.paper = paper ? 1 : 0;
    gp.fd_small = std::fabs(gp.nu - std::nearbyint(gp.nu)) > 1e-6 ? 0 : 1;
    gp.fd_large = std::fabs((gp.nu + 0.5) - std::nearbyint(gp.nu + 0.5)) > 1e-6 ? 0 : 1;
    int off = 0;
    const double tcap = 700.0 / (gp.abs_nu + 1.0); // keeps cosh(nu t) finite
    for (int L = 0; L < NLEV; ++L) {
        const double h = 0.2 / double(1 << L);
        const int maxlen = (L == 0) ? TAB_L0 : TAB_LN;
        const int len = std::min(maxlen, int(tcap / h) + 1);
        gp.h[L] = h;
        gp.xtop[L] = 9.0 * double(1 << (2 * L));
        gp.off[L] = off;
        gp.len[L] = len;
        for (int j = 0; j < len; ++j) {
            const double t = j * h, w = (j == 0) ? 0.5 * h : h;
            const double sh = std::sinh(0.5 * t);
            Node &nd = htab[off + j];
            nd.cm1 = 2.0 * sh * sh;
            nd.wk = w * std::cosh(gp.nu * t);
            nd.wk1 = w * std::cosh((gp.nu - 1.0) * t);
            nd.wd = w * t * std::sinh(gp.nu * t);
            nd.wkp = paper ? w * std::cosh((gp.nu + PAPER_LAG) * t) : 0.0;
            nd.wkm = paper ? w * std::cosh((gp.nu - PAPER_LAG) * t) : 0.0;
        }
        off += maxlen;
    }
    gp.pc = reinterpret_cast<const double *>(dtab + TAB_MAX);
    if (paper)
        paper_coefficients(gp, reinterpret_cast<double *>(htab + TAB_MAX));
    return gp;
}

namespace {

GenParams setup_theta(fbt_ctx *c, const double *th, int f, int64_t n)
{
    return theta_params(th, c->sigma_nu_mode == FBT_SIGMA_NU_PAPER ? 1 : 0, n, c->npad, c->ld,
                        reinterpret_cast<char *>(c->h_tab) + f * TAB_BYTES,
                        reinterpret_cast<const char *>(c->tab) + f * TAB_BYTES);
}

// ---- ordering between the critical-path and bulk streams ----
// A context whose streams are all one stream needs no events (they are then
// null): its launches are ordered by the stream itself.
hipError_t ev_record(hipEvent_t e, hipStream_t s) { return e ? hipEventRecord(e, s) : hipSuccess; }
hipError_t ev_wait(hipStream_t s, hipEvent_t e) { return e ? hipStreamWaitEvent(s, e, 0) : hipSuccess; }

// ---- timing helpers: HIP events around each launch on the launch's stream ----
void tbegin(fbt_ctx *c, hipStream_t st, hipEvent_t *a, hipEvent_t *b)
{
    if (!c->timing)
        return;
    while (c->pool.size() < c->pool_used + 2) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess)
            return;
        c->pool.push_back(e);
    }
    *a = c->pool[c->pool_used++];
    *b = c->pool[c->pool_used++];
    (void)hipEventRecord(*a, st);
}
void tend(fbt_ctx *c, hipStream_t st, int cls, double flops, hipEvent_t a, hipEvent_t b)
{
    if (!c->timing)
        return;
    (void)hipEventRecord(b, st);
    c->pending.push_back({cls, flops, a, b});
}
void tcollect(fbt_ctx *c)
{
    if (!c->timing)
        return;
    for (const Timed &t : c->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
            c->cls_n[t.cls] += 1;
            c->cls_ms[t.cls] += ms;
            c->cls_flops[t.cls] += t.flops;
        }
    }
    c->pending.clear();
    c->pool_used = 0;
}

#define TIMED(ctx, st, cls, flops, call)                                                           \
    do {                                                                                           \
        hipEvent_t ta_ = nullptr, tb_ = nullptr;                                                   \
        tbegin(ctx, st, &ta_, &tb_);                                                               \
        call;                                                                                      \
        if (ta_)                                                                                   \
            tend(ctx, st, cls, flops, ta_, tb_);                                                   \
    } while (0)

void free_buffers(fbt_ctx *c)
{
    void **dev[] = {(void **)&c->x,        (void **)&c->y,    (void **)&c->z,
                    (void **)&c->A,        (void **)&c->S2,   (void **)&c->Linv,
                    (void **)&c->logdet,   (void **)&c->partials, (void **)&c->out,
                    (void **)&c->wv,       (void **)&c->info, (void **)&c->tab,
                    (void **)&c->d_nf,     (void **)&c->d_gpa, (void **)&c->rv};
    for (void **p : dev) {
        (void)hipFree(*p);
        *p = nullptr;
    }
    void **host[] = {(void **)&c->h_tab, (void **)&c->h_out, (void **)&c->h_info,
                     (void **)&c->h_gpa};
    for (void **p : host) {
        if (*p)
            (void)hipHostFree(*p);
        *p = nullptr;
    }
    std::memset(c->cap, 0, sizeof(c->cap));
    (void)hipFree(c->Lf);
    (void)hipFree(c->Xf);
    c->Lf = nullptr;
    c->Xf = nullptr;
    c->cap_lf = c->cap_xf = 0;
    (void)hipFree(c->Ysl);
    (void)hipFree(c->Vd);
    (void)hipFree(c->Pd);
    c->Ysl = c->Vd = c->Pd = nullptr;
    c->cap_ysl = c->cap_vd = c->cap_pd = 0;
    (void)hipFree(c->Sc);
    c->Sc = nullptr;
    c->cap_sc = 0;
}

// Buffer sizes of the two-sided W phase per field (doubles)
int64_t sy_stride(const fbt_ctx *c) { return (int64_t)2 * 2 * c->npad * (2 * NB); }
int64_t vd_stride(const fbt_ctx *c) { return (int64_t)2 * c->T * NB * NB; }
int64_t pd_stride() { return (int64_t)2 * NB * NB; }

// The two-sided W phase's buffers for the current fields; false if they
// cannot be allocated (the W phase then takes the block solves).
bool ensure_sygst(fbt_ctx *c)
{
    struct {
        double **p;
        size_t *cap;
        size_t bytes;
    } req[] = {{&c->Ysl, &c->cap_ysl, (size_t)c->G * sy_stride(c) * 8},
               {&c->Vd, &c->cap_vd, (size_t)c->G * vd_stride(c) * 8},
               {&c->Pd, &c->cap_pd, (size_t)c->G * pd_stride() * 8}};
    for (auto &r : req) {
        if (r.bytes <= *r.cap)
            continue;
        (void)hipFree(*r.p);
        *r.p = nullptr;
        *r.cap = 0;
        if (hipMalloc((void **)r.p, r.bytes) != hipSuccess) {
            *r.p = nullptr;
            (void)hipGetLastError();
            return false;
        }
        *r.cap = r.bytes;
    }
    return true;
}

// The W phase takes the two-sided reduction when selected and its buffers
// exist (allocated here unless `may_alloc` is false).
bool use_two_sided(fbt_ctx *c, bool may_alloc = true)
{
    if (c->wphase != FBT_WPHASE_TWO_SIDED)
        return false;
    if (may_alloc)
        return ensure_sygst(c);
    return c->cap_ysl >= (size_t)c->G * sy_stride(c) * 8 &&
           c->cap_vd >= (size_t)c->G * vd_stride(c) * 8 && c->cap_pd >= (size_t)c->G * pd_stride() * 8;
}

// the forms whose Cholesky trailing updates are low precision
bool low_factor(int precision)
{
    return precision == FBT_MIXED_FP32_ALL || precision == FBT_MIXED_BF16_ALL;
}

// FBT_MIXED_FP32_ALL / _BF16_ALL on a single field refine w = Sigma^{-1} Z (see refine_w)
bool refines(const fbt_ctx *c)
{
    return low_factor(c->precision) && c->refine_iters > 0 && !c->batched;
}

// The copy of Sigma that refinement takes its residuals from (npad x ld).
bool ensure_sc(fbt_ctx *c)
{
    const size_t bytes = (size_t)c->npad * c->ld * sizeof(double);
    if (bytes <= c->cap_sc)
        return true;
    (void)hipFree(c->Sc);
    c->Sc = nullptr;
    c->cap_sc = 0;
    if (hipMalloc((void **)&c->Sc, bytes) != hipSuccess) {
        c->Sc = nullptr;
        (void)hipGetLastError();
        return false;
    }
    c->cap_sc = bytes;
    return true;
}

// The FP32 copies for the current fields (FBT_MIXED_FP32 and FBT_MIXED_BF16).  A failed
// allocation is not an error: the left solve then converts when staging.
void ensure_f32(fbt_ctx *c)
{
    if (c->precision != FBT_MIXED_FP32 && c->precision != FBT_MIXED_BF16)
        return;
    const size_t lf = (size_t)c->G * c->npad * c->ld * sizeof(float);
    const size_t xf = (size_t)c->G * (size_t)c->F.sXf * sizeof(float);
    if (lf > c->cap_lf) {
        (void)hipFree(c->Lf);
        c->Lf = nullptr;
        c->cap_lf = 0;
        if (hipMalloc(&c->Lf, lf) == hipSuccess)
            c->cap_lf = lf;
        else
            c->Lf = nullptr;
    }
    if (xf > c->cap_xf) {
        (void)hipFree(c->Xf);
        c->Xf = nullptr;
        c->cap_xf = 0;
        if (hipMalloc(&c->Xf, xf) == hipSuccess)
            c->cap_xf = xf;
        else
            c->Xf = nullptr;
    }
    (void)hipGetLastError(); // a failed allocation leaves no sticky error behind
}

// Buffers for G fields of up to nmax observations each (same padded order);
// a buffer is reallocated only when it must grow.
fbt_status alloc_fields(fbt_ctx *c, int64_t nmax, int G, bool batched)
{
    const int64_t npad = NB * ((nmax + 1 + NB - 1) / NB);
    const int T = (int)(npad / NB);
    const size_t ld = (size_t)npad, g = (size_t)G;
    const size_t part = (size_t)T * (size_t)(npad / 64) * 8;
    c->factor_valid = false;
    struct {
        void **p;
        size_t bytes;
        bool host;
    } req[] = {
        {(void **)&c->x, g * ld * 8, false},          {(void **)&c->y, g * ld * 8, false},
        {(void **)&c->z, g * ld * 8, false},          {(void **)&c->A, g * ld * ld * 8, false},
        {(void **)&c->S2, g * ld * ld * 16, false},
        {(void **)&c->Linv, g * (size_t)T * NB * NB * 8, false},
        {(void **)&c->logdet, g * (size_t)T * 8, false}, {(void **)&c->partials, g * part * 8, false},
        {(void **)&c->out, g * 16 * 8, false},        {(void **)&c->info, std::max<size_t>(64, g * 4), false},
        {(void **)&c->wv, g * ld * 8, false},         {(void **)&c->tab, g * TAB_BYTES, false},
        {(void **)&c->rv, g * ld * 9 * 8, false},
        {(void **)&c->d_nf, g * 8, false},            {(void **)&c->d_gpa, g * sizeof(GenParams), false},
        {(void **)&c->h_tab, g * TAB_BYTES, true},    {(void **)&c->h_out, g * 16 * 8, true},
        {(void **)&c->h_info, std::max<size_t>(64, g * 4), true},
        {(void **)&c->h_gpa, g * sizeof(GenParams), true},
    };
    static_assert(sizeof(req) / sizeof(req[0]) <= 24, "capacity slots");
    int i = 0;
    for (auto &r : req) {
        if (r.bytes > c->cap[i]) {
            if (r.host) {
                if (*r.p)
                    (void)hipHostFree(*r.p);
            } else {
                (void)hipFree(*r.p);
            }
            *r.p = nullptr;
            c->cap[i] = 0;
            const hipError_t e = r.host ? hipHostMalloc(r.p, r.bytes, hipHostMallocDefault)
                                        : hipMalloc(r.p, r.bytes);
            if (e != hipSuccess) {
                free_buffers(c);
                return fail(c, FBT_ENOMEM, "device allocation failed (npad = " +
                                               std::to_string(npad) + ", fields = " +
                                               std::to_string(G) + ")");
            }
            c->cap[i] = r.bytes;
        }
        ++i;
    }
    c->G = G;
    c->n = nmax;
    c->npad = npad;
    c->ld = npad;
    c->T = T;
    c->ncols = 128 * ((nmax + 127) / 128);
    c->F.count = G;
    c->F.sA = npad * npad;
    c->F.sS2 = 2 * npad * npad;
    c->F.sLinv = (int64_t)T * NB * NB;
    c->F.sVec = npad;
    c->F.sPart = (int64_t)part;
    c->F.sLog = T;
    c->F.sXf = 2 * (2 * NB) * (2 * npad);
    c->batched = batched;
    c->F.n = batched ? c->d_nf : nullptr;
    c->fst.assign(G, FBT_OK);
    c->fout.assign(2 * g, 0.0);
    return FBT_OK;
}

fbt_status alloc_for(fbt_ctx *c, int64_t n)
{
    c->nf.assign(1, n);
    return alloc_fields(c, n, 1, false);
}

// Quadrature tables for the G fields' theta (th: G x 3) into the pinned
// staging buffers; *gp receives field 0's parameters (the by-value launch
// argument of a single field).
void stage_theta(fbt_ctx *c, const double *th, GenParams *gp)
{
    for (int f = 0; f < c->G; ++f)
        c->h_gpa[f] = setup_theta(c, th + 3 * f, f, c->batched ? c->nf[f] : c->n);
    *gp = c->h_gpa[0];
}

// Staged tables to the device (ordered on the context's stream).
fbt_status upload_staged_theta(fbt_ctx *c)
{
    HIPCHK(c, hipMemcpyAsync(c->tab, c->h_tab, (size_t)c->G * TAB_BYTES, hipMemcpyHostToDevice,
                             c->stream));
    if (c->batched)
        HIPCHK(c, hipMemcpyAsync(c->d_gpa, c->h_gpa, (size_t)c->G * sizeof(GenParams),
                                 hipMemcpyHostToDevice, c->stream));
    return FBT_OK;
}

fbt_status upload_theta(fbt_ctx *c, const double *th, GenParams *gp)
{
    stage_theta(c, th, gp);
    return upload_staged_theta(c);
}

// Generate Sigma' (and/or the derivative matrices) and factor the bordered
// Sigma'.  On success c->factor_out = {log det, y^T y}.
//
// Right-looking block Cholesky with one step of lookahead on two streams.
// Step k on s0 (critical path): update block column k+1 with panel k, factor
// diagonal block k+1 and solve panel k+1.  On s1: the rest of the trailing
// update with panel k (block columns >= k+2).  Block column k+1 is written
// by s0 only after the previous bulk update (which also wrote it) is done.
// Launches of the factorisation (tables already on the device), ending with
// the copies of the results to the pinned host buffers; no host wait.
fbt_status factorize_enqueue(fbt_ctx *c, const GenParams &gp, int mode)
{
    c->factor_valid = false;
    const int64_t npad = c->npad, ld = c->ld, n = c->n;
    const int T = c->T;
    hipStream_t s0 = c->stream, s1 = c->capturable ? c->stream2 : c->stream3;
    double *A = c->A;
    const double dNB = NB;
    // Cholesky updates in FP32 (1) or with BF16 operands and FP32 sums (2)
    const int mix = c->precision == FBT_MIXED_FP32_ALL ? 1 : c->precision == FBT_MIXED_BF16_ALL ? 2 : 0;
    auto Lk = [&](int k) { return c->Linv + (size_t)k * NB * NB; };
    launch_init_info(s0, c->info, c->G);
    TIMED(c, s0, KC_GEN, 0.0, launch_gen(s0, gp, c->d_gpa, c->F, c->x, c->y, c->z, A, c->S2,
                                           c->S2 + npad * ld, mode));
    if (refines(c) && c->cap_sc >= (size_t)npad * ld * sizeof(double))
        launch_copy_sym(s0, A, ld, n, c->Sc);
    // Block columns are taken four at a time while more than FACT_QUAD_ABOVE
    // blocks remain, then in pairs, and singly in the last FACT_SINGLE_TAIL
    // blocks.  On s0, for each block column b + j of a step of width nb:
    // update of block columns b + j .. b + nb - 1 by panel b + j - 1 (j > 0),
    // diagonal block b + j, panel b + j.  The trailing matrix is then updated
    // by the step's panels at once (K = nb NB): s0 updates the next step's
    // block columns (lookahead) once s1 has finished the previous bulk update;
    // s1 updates the rest.  A K = 2 NB or 4 NB update is the FMA sequence of
    // NB-deep ones in order (C lives in the accumulators), so the step widths
    // do not change the results.
    auto rows_from = [&](int64_t r) { return (double)std::max<int64_t>(0, n - r); };
    auto width = [&](int b) {
        return T - b <= FACT_SINGLE_TAIL ? 1 : T - b > FACT_QUAD_ABOVE ? 4 : std::min(2, T - b);
    };
    HIPCHK(c, ev_record(c->evB, s0));
    for (int b = 0, nb = 1; b < T; b += nb) {
        nb = width(b);
        const int64_t r0 = (int64_t)b * NB, rn = r0 + (int64_t)nb * NB;
        const int K = nb * NB;
        TIMED(c, s0, KC_DIAG, 2.0 * dNB * dNB * dNB / 3.0,
              launch_potrf_diag(s0, c->F, A, ld, b, n, Lk(b), c->logdet, c->info));
        if (b + 1 < T)
            TIMED(c, s0, KC_PANEL, rows_from(r0 + NB) * dNB * dNB,
                  launch_panel(s0, c->F, A + r0 + NB + r0 * ld, ld, npad - r0 - NB, Lk(b)));
        // the step's further block columns: each by the panels before it in
        // the step, then its diagonal block and panel
        for (int j = 1; j < nb; ++j) {
            const int64_t rj = r0 + (int64_t)j * NB, rp = rj - NB;
            TIMED(c, s0, KC_SYRK, 2.0 * rows_from(rj) * (double)(nb - j) * dNB * dNB,
                  launch_update_rect(s0, c->F, c->F.sA, c->F.sA, 1, A + rj + rj * ld, nullptr, ld,
                                     A + rj + rp * ld, nullptr, ld, A + rj + rp * ld, ld, npad - rj,
                                     (int64_t)(nb - j) * NB, NB, mix));
            TIMED(c, s0, KC_DIAG, 2.0 * dNB * dNB * dNB / 3.0,
                  launch_potrf_diag(s0, c->F, A, ld, b + j, n, Lk(b + j), c->logdet, c->info));
            if (b + j + 1 < T)
                TIMED(c, s0, KC_PANEL, rows_from(rj + NB) * dNB * dNB,
                      launch_panel(s0, c->F, A + rj + NB + rj * ld, ld, npad - rj - NB,
                                   Lk(b + j)));
        }
        HIPCHK(c, ev_record(c->evP, s0));
        if (rn >= npad)
            break;
        // columns of the next step
        const int64_t la = std::min<int64_t>((int64_t)width(b + nb) * NB, npad - rn);
        HIPCHK(c, ev_wait(s0, c->evB));
        TIMED(c, s0, KC_SYRK, 2.0 * rows_from(rn) * (double)la * K,
              launch_update_rect(s0, c->F, c->F.sA, c->F.sA, 1, A + rn + rn * ld, nullptr, ld, A + rn + r0 * ld, nullptr,
                                 ld, A + rn + r0 * ld, ld, npad - rn, la, K, mix));
        HIPCHK(c, ev_wait(s1, c->evP));
        const int64_t t0 = rn + la;
        if (t0 < npad)
            TIMED(c, s1, KC_SYRK, rows_from(t0) * rows_from(t0) * K,
                  launch_update_lower(s1, c->F, c->F.sA, c->F.sA, 1, A + t0 + t0 * ld, nullptr, ld, A + t0 + r0 * ld,
                                      nullptr, ld, A + t0 + r0 * ld, ld, (int)((npad - t0) / NB), K,
                                      mix));
        HIPCHK(c, ev_record(c->evB, s1));
    }
    HIPCHK(c, ev_wait(s0, c->evB));
    TIMED(c, s0, KC_RED, 0.0, launch_reduce_loglik(s0, c->F, A, ld, n, T, c->logdet, c->out));
    HIPCHK(c, hipMemcpyAsync(c->h_out, c->out, (size_t)c->G * 16 * sizeof(double),
                             hipMemcpyDeviceToHost, s0));
    HIPCHK(c, hipMemcpyAsync(c->h_info, c->info, (size_t)c->G * sizeof(int), hipMemcpyDeviceToHost,
                             s0));
    return FBT_OK;
}

// Per-field status and {log det, q} from the pinned buffers, once the
// enqueued factorisation has completed.
void factor_results(fbt_ctx *c)
{
    for (int f = 0; f < c->G; ++f) {
        const double ld_ = c->h_out[16 * f], q = c->h_out[16 * f + 1];
        c->fout[2 * f] = ld_;
        c->fout[2 * f + 1] = q;
        c->fst[f] = c->h_info[f] != 0x7fffffff                      ? FBT_ENOTPD
                    : (!std::isfinite(ld_) || !std::isfinite(q)) ? FBT_ENONFINITE
                                                                 : FBT_OK;
    }
}

// FBT_MIXED_FP32_ALL: the factor's trailing updates ran in FP32, so w =
// Sigma^{-1} Z (and with it q = Z^T w) is won back by iterative refinement:
// w_0 = L~^{-T} y with y = L~^{-1} Z from the bordered factor's row n, then
// c->refine_iters steps w += Sigma~^{-1} (Z - Sigma w) with the residual in
// FP64 from the copy of Sigma taken before the factorisation (c->Sc),
// Sigma~ = L~ L~^T the factor's matrix.  The log determinant keeps the
// factor's rounding.  Sets c->factor_out[1] = Z^T w; c->wv holds w.
fbt_status refine_w(fbt_ctx *c)
{
    hipStream_t s0 = c->stream;
    const int64_t npad = c->npad, ld = c->ld, n = c->n;
    double *w = c->wv, *r = c->rv, *part = c->rv + npad;
    launch_border_row(s0, c->A, ld, n, npad, w);
    launch_trsv(s0, w, c->A, ld, npad, c->Linv, 1);
    for (int it = 0; it < c->refine_iters; ++it) {
        launch_residual(s0, c->Sc, ld, n, npad, c->z, w, REFINE_NQ, part, r);
        launch_solve_sigma(s0, r, c->A, ld, n, npad, c->Linv);
        launch_axpy_dot(s0, w, r, c->z, n, npad, nullptr);
    }
    launch_axpy_dot(s0, w, nullptr, c->z, n, npad, c->out + 1);
    HIPCHK(c, hipMemcpyAsync(c->h_out + 1, c->out + 1, sizeof(double), hipMemcpyDeviceToHost, s0));
    HIPCHK(c, hipStreamSynchronize(s0));
    c->factor_out[1] = c->h_out[1];
    return FBT_OK;
}

fbt_status factorize(fbt_ctx *c, const double *th, int mode)
{
    GenParams gp;
    fbt_status st = upload_theta(c, th, &gp);
    if (st != FBT_OK)
        return st;
    if (refines(c) && !ensure_sc(c))
        return fail(c, FBT_ENOMEM, "cannot allocate the copy of Sigma for refinement");
    if ((st = factorize_enqueue(c, gp, mode)) != FBT_OK)
        return st;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    tcollect(c);
    factor_results(c);
    if (c->batched)
        return FBT_OK;
    if (c->h_info[0] != 0x7fffffff) {
        c->notpd = c->h_info[0];
        return fail(c, FBT_ENOTPD, "Sigma(theta) is not positive definite: pivot " +
                                       std::to_string(c->h_info[0]) + " is not positive");
    }
    c->factor_out[0] = c->h_out[0];
    c->factor_out[1] = c->h_out[1];
    if (refines(c) && (st = refine_w(c)) != FBT_OK)
        return st;
    if (!std::isfinite(c->factor_out[0]) || !std::isfinite(c->factor_out[1]))
        return fail(c, FBT_ENONFINITE, "log-determinant or quadratic form is not finite");
    c->factor_valid = true;
    std::memcpy(c->factor_theta, th, sizeof(c->factor_theta));
    return FBT_OK;
}

// The factor of the last fbt_loglik / fbt_factor call is reused by the next
// derivative evaluation at the bitwise-same theta (the accepted trial of the
// line search), once: every other evaluation factors Sigma afresh.
bool same_theta(const fbt_ctx *c, const double *th)
{
    return c->factor_valid && std::memcmp(c->factor_theta, th, sizeof(c->factor_theta)) == 0;
}

fbt_status wphase_enqueue(fbt_ctx *c);
fbt_status wphase_sygst_enqueue(fbt_ctx *c);
fbt_status wphase_results(fbt_ctx *c, double *terms);

// W phase of Algorithm 3 on a valid factor: out[0..8] (see fbt_eval_terms).
// Both block solves use the same two-stream lookahead as the factorisation:
// s0 finishes block row / column k+1 and applies its diagonal inverse while
// s1 applies step k to everything beyond it.
fbt_status derivative_terms(fbt_ctx *c, const double *th, double terms[9])
{
    fbt_status st;
    hipStream_t s0 = c->stream;
    if (same_theta(c, th)) {
        GenParams gp;
        if ((st = upload_theta(c, th, &gp)) != FBT_OK)
            return st;
        TIMED(c, s0, KC_GEN, 0.0, launch_gen(s0, gp, c->d_gpa, c->F, c->x, c->y, c->z, c->A, c->S2,
                                               c->S2 + c->npad * c->ld, GEN_DERIV));
    } else if ((st = factorize(c, th, GEN_ALL)) != FBT_OK) {
        return st;
    }
    c->factor_valid = false; // reuse is for one derivative evaluation only
    if (refines(c)) {
        // u_i = w^T Sigma_i w with the refined w, from the derivative matrices
        // before the W phase overwrites them (its own u_i come from the
        // factor's y); the W phase's launches are ordered after these on s0
        const int64_t npad = c->npad, ld = c->ld;
        for (int i = 0; i < 2; ++i)
            launch_quad_form(s0, c->S2 + i * npad * ld, ld, c->n, npad, c->wv, REFINE_NQ,
                             c->rv + npad, c->out + 10 + i);
    }
    if (use_two_sided(c)) {
        if ((st = wphase_sygst_enqueue(c)) != FBT_OK)
            return st;
    } else {
        ensure_f32(c);
        if ((st = wphase_enqueue(c)) != FBT_OK)
            return st;
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    tcollect(c);
    if ((st = wphase_results(c, terms)) != FBT_OK || !refines(c))
        return st;
    terms[4] = c->h_out[10];
    terms[5] = c->h_out[11];
    if (!std::isfinite(terms[4]) || !std::isfinite(terms[5]))
        return fail(c, FBT_ENONFINITE, "a quadratic form is not finite");
    return FBT_OK;
}

// Launches of the W phase on a factor in place (derivative matrices already
// generated), ending with the copy of the nine terms per field to the pinned
// host buffer; no host wait.
fbt_status wphase_enqueue(fbt_ctx *c)
{
    hipStream_t s0 = c->stream, s1 = c->stream2;
    const int64_t npad = c->npad, ld = c->ld, n = c->n, ncols = c->ncols;
    const int T = c->T;
    double *Sa = c->S2, *Sn = c->S2 + npad * ld, *A = c->A;
    const double dn = (double)n, dNB = NB;
    // solve updates: FP32 (1) or BF16 operands with FP32 sums (2)
    const int mix = c->precision == FBT_FP64 ? 0
                    : (c->precision == FBT_MIXED_BF16 || c->precision == FBT_MIXED_BF16_ALL) ? 2
                                                                                           : 1;
    auto Lk = [&](int k) { return c->Linv + (size_t)k * NB * NB; };
    // mixed forms with their operand copies: the factor once, each solved pair of
    // block rows as the diagonal apply writes it (slot by pair parity, so the
    // next pair's rows never overwrite rows a running update still reads)
    const bool copies = mix != 0 && c->Lf && c->Xf;
    auto xslot = [&](int b) { return c->Xf + (size_t)((b / 2) & 1) * (2 * NB) * (2 * npad); };
    if (copies)
        launch_to_f32_lower(s0, c->F, A, ld, npad, c->Lf);
    // left update of `rows` rows from r by the `kp` panels of pair b (K = kp NB)
    auto left_update = [&](hipStream_t st, int64_t r, int64_t rows, int b, int kp, int K) {
        if (!copies) {
            launch_update_nn(st, c->F, c->F.sS2, 2, c->S2, ld, A, ld, r, (int64_t)b * NB, rows, ncols,
                             npad, K, mix);
            return;
        }
        for (int p = 0; p < kp; ++p)
            launch_update_nn_f32(st, c->F, c->F.sS2, 2, c->S2, ld, c->Lf, r, (int64_t)(b + p) * NB,
                                 xslot(b), p * NB, rows, ncols, npad, mix == 2);
    };

    // Left solve X = L'^{-1} [Sigma_alpha' | Sigma_nu'] on columns [0, ncols) of
    // each half.  Block rows are taken in pairs (b, b + 1).  Inside a pair the
    // solve runs on s0 with one panel at a time: diagonal apply of block b,
    // update of block row b + 1 by panel b, diagonal apply of block b + 1.
    // Everything below the pair is then updated by both panels at once
    // (K = 2 NB, the better-shaped product): s0 updates the next pair
    // (lookahead) once s1 has finished the previous bulk update, and s1
    // updates all rows beyond the next pair.
    auto real_rows = [&](int64_t r, int64_t cnt) {
        return (double)std::max<int64_t>(0, std::min<int64_t>(n - r, cnt));
    };
    HIPCHK(c, ev_record(c->evB, s0));
    for (int b = 0; b < T; b += 2) {
        const int nb = std::min(2, T - b);
        const int64_t r0 = (int64_t)b * NB, rn = r0 + (int64_t)nb * NB;
        const int K = nb * NB;
        TIMED(c, s0, KC_LAPPLY, 2.0 * dn * dNB * dNB,
              launch_diag_apply(s0, c->F, c->F.sS2, 2, c->S2, ld, r0, Lk(b), ncols, npad,
                                copies ? xslot(b) : nullptr, 0));
        if (nb == 2) {
            TIMED(c, s0, KC_LUPD, 2.0 * real_rows(r0 + NB, NB) * dNB * 2.0 * dn,
                  left_update(s0, r0 + NB, NB, b, 1, NB));
            TIMED(c, s0, KC_LAPPLY, 2.0 * dn * dNB * dNB,
                  launch_diag_apply(s0, c->F, c->F.sS2, 2, c->S2, ld, r0 + NB, Lk(b + 1), ncols, npad,
                                    copies ? xslot(b) : nullptr, NB));
        }
        HIPCHK(c, ev_record(c->evP, s0));
        if (rn >= npad)
            break;
        const int64_t la = std::min<int64_t>(2 * NB, npad - rn); // rows of the next pair
        HIPCHK(c, ev_wait(s0, c->evB));
        TIMED(c, s0, KC_LUPD, 2.0 * real_rows(rn, la) * K * 2.0 * dn,
              left_update(s0, rn, la, b, nb, K));
        HIPCHK(c, ev_wait(s1, c->evP));
        if (rn + la < npad)
            TIMED(c, s1, KC_LUPD, 2.0 * real_rows(rn + la, npad) * K * 2.0 * dn,
                  left_update(s1, rn + la, npad - rn - la, b, nb, K));
        HIPCHK(c, ev_record(c->evB, s1));
    }
    HIPCHK(c, ev_wait(s0, c->evB));

    // Right solve W = X L'^{-T} (block-lower) with the fused reductions, block
    // columns in pairs as in the factorisation: on s0 the panel of block b
    // (with the trace reductions), the update of block column b + 1 by it and
    // the panel of block b + 1; then the lookahead update of the next pair of
    // block columns by both panels (K = 2 NB) on s0 and the rest on s1.
    int64_t groups = 0;
    HIPCHK(c, ev_record(c->evB, s0));
    for (int b = 0; b < T; b += 2) {
        const int nb = std::min(2, T - b);
        const int64_t r0 = (int64_t)b * NB, rn = r0 + (int64_t)nb * NB;
        const int K = nb * NB;
        const double m0r = std::max<int64_t>(0, n - r0);
        TIMED(c, s0, KC_RPANEL, 2.0 * 2.0 * m0r * dNB * dNB,
              launch_panel_reduce(s0, c->F, Sa, Sn, ld, r0, r0, npad - r0, Lk(b), n,
                                  c->partials + 8 * groups));
        groups += (npad - r0) / 64;
        if (nb == 2) {
            const int64_t r1 = r0 + NB;
            const double m1 = std::max<int64_t>(0, n - r1);
            TIMED(c, s0, KC_RUPD, 2.0 * 2.0 * m1 * dNB * dNB,
                  launch_update_rect(s0, c->F, c->F.sS2, c->F.sA, 2, Sa + r1 + r1 * ld, Sn + r1 + r1 * ld, ld,
                                     Sa + r1 + r0 * ld, Sn + r1 + r0 * ld, ld, A + r1 + r0 * ld,
                                     ld, npad - r1, NB, NB, mix));
            TIMED(c, s0, KC_RPANEL, 2.0 * 2.0 * m1 * dNB * dNB,
                  launch_panel_reduce(s0, c->F, Sa, Sn, ld, r1, r1, npad - r1, Lk(b + 1), n,
                                      c->partials + 8 * groups));
            groups += (npad - r1) / 64;
        }
        HIPCHK(c, ev_record(c->evP, s0));
        if (rn >= npad)
            break;
        const int64_t la = std::min<int64_t>(2 * NB, npad - rn);
        const double mn = std::max<int64_t>(0, n - rn);
        HIPCHK(c, ev_wait(s0, c->evB));
        TIMED(c, s0, KC_RUPD, 2.0 * 2.0 * mn * (double)la * K,
              launch_update_rect(s0, c->F, c->F.sS2, c->F.sA, 2, Sa + rn + rn * ld, Sn + rn + rn * ld, ld,
                                 Sa + rn + r0 * ld, Sn + rn + r0 * ld, ld, A + rn + r0 * ld, ld,
                                 npad - rn, la, K, mix));
        HIPCHK(c, ev_wait(s1, c->evP));
        const int64_t t0 = rn + la;
        const double mt = std::max<int64_t>(0, n - t0);
        if (t0 < npad)
            TIMED(c, s1, KC_RUPD, 2.0 * mt * mt * K,
                  launch_update_lower(s1, c->F, c->F.sS2, c->F.sA, 2, Sa + t0 + t0 * ld, Sn + t0 + t0 * ld, ld,
                                      Sa + t0 + r0 * ld, Sn + t0 + r0 * ld, ld, A + t0 + r0 * ld,
                                      ld, (int)((npad - t0) / NB), K, mix));
        HIPCHK(c, ev_record(c->evB, s1));
    }
    HIPCHK(c, ev_wait(s0, c->evB));
    TIMED(c, s0, KC_RED, 0.0, launch_reduce_terms(s0, c->F, c->partials, groups, c->out));
    HIPCHK(c, hipMemcpyAsync(c->h_out, c->out, (size_t)c->G * 16 * sizeof(double),
                             hipMemcpyDeviceToHost, s0));
    return FBT_OK;
}

// W phase of Algorithm 3 by the two-sided reduction (see the kernels): block
// steps k = 0..T-1 over both derivative matrices form W_kk, Y and M of block
// column k and update the trailing lower blocks by Y L^T + L Y^T; the deferred
// left solve W_strict = L'^{-1} M (block row r over columns < r NB) follows
// them one pair of block rows behind; then the trace reductions over the
// block-lower part.  Both take steps in pairs with one step of lookahead on a
// chain and a bulk stream, as the factorisation: on the chain the steps of the
// pair (b, b + 1) and the update of the next pair's block columns (rows) once
// the previous bulk update has finished; on the bulk stream the rest of the
// trailing update by both steps at once.  Y of a pair goes to the slot of its
// parity, so a pair's chain never overwrites Y that the previous pair's bulk
// update still reads.
fbt_status wphase_sygst_enqueue(fbt_ctx *c)
{
    hipStream_t s0 = c->stream, s1 = c->stream2;
    const int64_t npad = c->npad, ld = c->ld, n = c->n;
    const int T = c->T;
    double *S2 = c->S2, *A = c->A;
    const int64_t mofs = npad * ld;
    const int64_t sY = sy_stride(c), ymofs = npad * (2 * NB), ldy = npad;
    const int64_t sVd = vd_stride(c), vofs = (int64_t)T * NB * NB, sPd = pd_stride();
    const double dNB = NB;
    // the rank-2k updates and the deferred solve's updates: FP32 (1) or BF16
    // operands (2) with FP32 sums in the mixed precisions; everything else FP64
    const int mix = c->precision == FBT_FP64 ? 0
                    : (c->precision == FBT_MIXED_BF16 || c->precision == FBT_MIXED_BF16_ALL) ? 2
                                                                                           : 1;
    auto Lk = [&](int k) { return c->Linv + (size_t)k * NB * NB; };
    auto Vk = [&](int k) { return c->Vd + (size_t)k * NB * NB; };
    auto slot = [&](int b) { return c->Ysl + (size_t)((b / 2) & 1) * (2 * npad * (2 * NB)); };
    auto real = [&](int64_t r, int64_t cnt) {
        return (double)std::max<int64_t>(0, std::min<int64_t>(n - r, cnt));
    };
    auto diag = [&](int k) {
        TIMED(c, s0, KC_SDIAG, 4.0 * dNB * dNB * dNB,
              launch_sygst_diag(s0, c->F, S2, ld, mofs, (int64_t)k * NB, Lk(k), c->Pd, sPd, Vk(k),
                                vofs, sVd));
    };
    // panel of step k on rows [r, npad), Y to the slot columns at Y
    auto panel = [&](int k, int64_t r, double *Y) {
        if (r < npad)
            TIMED(c, s0, KC_SPANEL, 6.0 * real(r, npad) * dNB * dNB,
                  launch_sygst_panel(s0, c->F, S2, ld, mofs, A, r, npad - r, (int64_t)k * NB, Lk(k),
                                     Vk(k), vofs, sVd, Y, ldy, ymofs, sY));
    };
    // rows [r, npad) x cols [q, q + w) by the KS / NB steps from block kb (Y of their slot)
    auto rect = [&](int64_t r, int64_t q, int64_t w, int kb, int KS, const double *Y) {
        if (r < npad && w > 0)
            TIMED(c, s0, KC_SLOOK, 2.0 * 2.0 * 2.0 * real(r, npad) * real(q, w) * KS,
                  launch_syr2k_rect(s0, c->F, S2, ld, mofs, A, r, npad - r, q, w, (int64_t)kb * NB,
                                    KS, Y, ldy, ymofs, sY, mix));
    };

    // The deferred solve of block rows (b, b + 1) needs their M complete, i.e.
    // the block steps up to b + 1, and their diagonal blocks spent (zeroed
    // here; they are W_kk's S_kk).  Its rows and columns never meet the block
    // steps that follow (those write columns >= (b + 2) NB, it writes columns
    // < (b + 1) NB), so it runs one pair behind the block steps on streams of
    // its own (chain sd, bulk sdb): its launches fill the block steps' gaps and
    // the other way round.  Its bulk stream is the factorisation's (all CUs but
    // one per XCD); a capturable context has none and shares s1.
    hipStream_t sd = c->stream4, sdb = c->capturable ? c->stream2 : c->stream3;
    auto deferred_pair = [&](int b) -> fbt_status {
        const int nb = std::min(2, T - b);
        const int64_t r0 = (int64_t)b * NB, rn = r0 + (int64_t)nb * NB;
        HIPCHK(c, ev_wait(sd, c->evP));
        launch_zero_diag_blocks(sd, c->F, S2, ld, mofs, b, nb);
        TIMED(c, sd, KC_DAPPLY, 2.0 * dNB * dNB * real(0, r0),
              launch_diag_apply(sd, c->F, c->F.sS2, 2, S2, ld, r0, Lk(b), r0, npad));
        if (nb == 2) {
            TIMED(c, sd, KC_DUPD, 2.0 * 2.0 * real(r0 + NB, NB) * dNB * real(0, r0),
                  launch_update_nn(sd, c->F, c->F.sS2, 2, S2, ld, A, ld, r0 + NB, r0, NB, r0, npad,
                                   NB, mix));
            TIMED(c, sd, KC_DAPPLY, 2.0 * dNB * dNB * real(0, r0 + NB),
                  launch_diag_apply(sd, c->F, c->F.sS2, 2, S2, ld, r0 + NB, Lk(b + 1), r0 + NB,
                                    npad));
        }
        HIPCHK(c, ev_record(c->evP2, sd));
        if (rn >= npad)
            return FBT_OK;
        // the pair's rows hold W over columns < (b + nb - 1) NB (block row b's
        // diagonal block is zero)
        const int64_t cols = (int64_t)(b + nb - 1) * NB;
        const int K = nb * NB;
        const int64_t la = std::min<int64_t>(2 * NB, npad - rn);
        HIPCHK(c, ev_wait(sd, c->evB2));
        TIMED(c, sd, KC_DUPD, 2.0 * 2.0 * real(rn, la) * K * real(0, cols),
              launch_update_nn(sd, c->F, c->F.sS2, 2, S2, ld, A, ld, rn, r0, la, cols, npad, K, mix));
        HIPCHK(c, ev_wait(sdb, c->evP2));
        // the two bulk updates alternate: this one after the pair's rank-2k update
        HIPCHK(c, ev_wait(sdb, c->evB));
        if (rn + la < npad)
            TIMED(c, sdb, KC_DUPD, 2.0 * 2.0 * real(rn + la, npad) * K * real(0, cols),
                  launch_update_nn(sdb, c->F, c->F.sS2, 2, S2, ld, A, ld, rn + la, r0,
                                   npad - rn - la, cols, npad, K, mix));
        HIPCHK(c, ev_record(c->evB2, sdb));
        return FBT_OK;
    };

    // ---- block steps, and the deferred solve one pair behind ----
    HIPCHK(c, ev_record(c->evB, s0));
    HIPCHK(c, ev_record(c->evB2, s0));
    fbt_status st = FBT_OK;
    for (int b = 0; b < T; b += 2) {
        const int nb = std::min(2, T - b);
        const int64_t r0 = (int64_t)b * NB, r1 = r0 + NB, rn = r0 + (int64_t)nb * NB;
        double *Y = slot(b);
        diag(b);
        panel(b, r1, Y);
        if (nb == 2) {
            rect(r1, r1, NB, b, NB, Y);
            diag(b + 1);
            panel(b + 1, rn, Y + NB * ldy);
        }
        HIPCHK(c, ev_record(c->evP, s0));
        if (rn < npad) {
            const int KS = nb * NB;
            const int64_t la = std::min<int64_t>(2 * NB, npad - rn); // columns of the next pair
            HIPCHK(c, ev_wait(s0, c->evB));
            rect(rn, rn, la, b, KS, Y);
            HIPCHK(c, ev_wait(s1, c->evP));
            // after the previous pair's deferred bulk update (the two bulk
            // updates alternate)
            HIPCHK(c, ev_wait(s1, c->evB2));
            const int64_t t0 = rn + la;
            if (t0 < npad)
                TIMED(c, s1, KC_SUPD, 2.0 * 2.0 * real(t0, npad) * real(t0, npad) * KS,
                      launch_syr2k_lower(s1, c->F, S2, ld, mofs, A, t0, (int)((npad - t0) / NB), r0,
                                         KS, Y, ldy, ymofs, sY, 0, mix));
            HIPCHK(c, ev_record(c->evB, s1));
        }
        if ((st = deferred_pair(b)) != FBT_OK)
            return st;
    }
    HIPCHK(c, ev_wait(s0, c->evB));
    HIPCHK(c, ev_record(c->evD, sd));
    HIPCHK(c, ev_wait(s0, c->evD));
    HIPCHK(c, ev_wait(s0, c->evB2));
    TIMED(c, s0, KC_RED, 0.0,
          launch_sygst_reduce(s0, c->F, S2, ld, mofs, c->Vd, vofs, sVd, T, n, c->partials));
    TIMED(c, s0, KC_RED, 0.0,
          launch_reduce_terms(s0, c->F, c->partials, (int64_t)T * (T + 1) / 2, c->out));
    HIPCHK(c, hipMemcpyAsync(c->h_out, c->out, (size_t)c->G * 16 * sizeof(double),
                             hipMemcpyDeviceToHost, s0));
    return FBT_OK;
}

// The nine terms (per field: terms[9 f + i] in a batched group) from the
// pinned buffer, once the enqueued W phase has completed.
fbt_status wphase_results(fbt_ctx *c, double *terms)
{
    if (c->batched) {
        for (int f = 0; f < c->G; ++f) {
            terms[9 * f] = c->fout[2 * f];
            terms[9 * f + 1] = c->fout[2 * f + 1];
            for (int i = 2; i < 9; ++i)
                terms[9 * f + i] = c->h_out[16 * f + i];
            if (c->fst[f] == FBT_OK)
                for (int i = 0; i < 9; ++i)
                    if (!std::isfinite(terms[9 * f + i]))
                        c->fst[f] = FBT_ENONFINITE;
        }
        return FBT_OK;
    }
    // the derivative matrices were overwritten; the factor itself is intact
    terms[0] = c->factor_out[0];
    terms[1] = c->factor_out[1];
    for (int i = 2; i < 9; ++i)
        terms[i] = c->h_out[i];
    for (int i = 0; i < 9; ++i)
        if (!std::isfinite(terms[i]))
            return fail(c, FBT_ENONFINITE, "a trace term is not finite");
    return FBT_OK;
}

// Adjoint gradient on a valid factor (see k_adjoint): X = L'^{-1} by the left
// solve of the identity restricted to the block-lower part (columns < (k+1) NB
// in block row k; columns >= ncols are never needed), P = X^T X, w from row n
// of X, and the contraction of w w^T - P / 2 with the regenerated Sigma_alpha,
// Sigma_nu.  X occupies the first half of S2, P the second; L' is untouched.
// out: sums {dl/dalpha, dl/dnu}; c->wv holds w.
fbt_status adjoint_terms(fbt_ctx *c, const double *th, double g[2])
{
    fbt_status st;
    if (c->G != 1)
        return fail(c, FBT_EINVAL, "internal: the adjoint path takes one field");
    hipStream_t s0 = c->stream, s1 = c->stream2;
    if (!same_theta(c, th) && (st = factorize(c, th, GEN_SIGMA)) != FBT_OK)
        return st;
    c->factor_valid = false; // reuse is for one derivative evaluation only
    GenParams gp;
    if ((st = upload_theta(c, th, &gp)) != FBT_OK)
        return st;
    const int64_t npad = c->npad, ld = c->ld, n = c->n, ncols = c->ncols;
    const int T = c->T;
    double *X = c->S2, *P = c->S2 + npad * ld, *A = c->A;
    const double dNB = NB;
    auto Lk = [&](int k) { return c->Linv + (size_t)k * NB * NB; };
    auto cols = [&](int k) { return std::min<int64_t>((int64_t)(k + 1) * NB, ncols); };

    TIMED(c, s0, KC_ADJ, 0.0, launch_fill_identity(s0, X, ld, npad, ncols));
    TIMED(c, s0, KC_INV, 2.0 * dNB * dNB * (double)cols(0),
          launch_diag_apply(s0, c->F, c->F.sS2, 1, X, ld, 0, Lk(0), cols(0), 0));
    HIPCHK(c, ev_record(c->evP, s0));
    HIPCHK(c, ev_record(c->evB, s0));
    for (int k = 0; k + 1 < T; ++k) {
        const int64_t kc = (int64_t)k * NB, r1 = kc + NB, r2 = r1 + NB;
        const int64_t ck = cols(k);
        HIPCHK(c, ev_wait(s0, c->evB));
        TIMED(c, s0, KC_INV, 2.0 * dNB * dNB * (double)ck,
              launch_update_nn(s0, c->F, c->F.sS2, 1, X, ld, A, ld, r1, kc, NB, ck, 0, NB, 0));
        TIMED(c, s0, KC_INV, 2.0 * dNB * dNB * (double)cols(k + 1),
              launch_diag_apply(s0, c->F, c->F.sS2, 1, X, ld, r1, Lk(k + 1), cols(k + 1), 0));
        HIPCHK(c, ev_wait(s1, c->evP));
        if (k + 2 < T)
            TIMED(c, s1, KC_INV, 2.0 * (double)(npad - r2) * dNB * (double)ck,
                  launch_update_nn(s1, c->F, c->F.sS2, 1, X, ld, A, ld, r2, kc, npad - r2, ck, 0, NB, 0));
        HIPCHK(c, ev_record(c->evB, s1));
        HIPCHK(c, ev_record(c->evP, s0));
    }
    HIPCHK(c, ev_wait(s0, c->evB));
    {
        // flops of the block-lower 128-tiles below ncols: sum over tiles of 2 128^2 (npad - m0)
        double fl = 0.0;
        for (int64_t m0 = 0; m0 < ncols; m0 += 128)
            fl += (double)(m0 / 128 + 1) * 2.0 * 128.0 * 128.0 * (double)(npad - m0);
        TIMED(c, s0, KC_LAUUM, fl, launch_lauum(s0, P, X, ld, npad, ncols));
    }
    TIMED(c, s0, KC_ADJ, 0.0, launch_extract_w(s0, X, ld, n, c->wv));
    const int64_t nt = (n + 63) / 64, pairs = nt * (nt + 1) / 2;
    if (2 * pairs > (int64_t)(c->T) * (npad / 64) * 8)
        return fail(c, FBT_EINVAL, "internal: adjoint partials exceed the partials buffer");
    TIMED(c, s0, KC_ADJ, 0.0,
          launch_adjoint(s0, gp, c->x, c->y, c->tab, P, c->wv, c->partials));
    TIMED(c, s0, KC_RED, 0.0, launch_reduce_pairs(s0, c->partials, pairs, c->out + 2));
    HIPCHK(c, hipMemcpyAsync(c->h_out, c->out, 4 * sizeof(double), hipMemcpyDeviceToHost, s0));
    HIPCHK(c, hipStreamSynchronize(s0));
    tcollect(c);
    g[0] = c->h_out[2];
    g[1] = c->h_out[3];
    if (!std::isfinite(g[0]) || !std::isfinite(g[1]))
        return fail(c, FBT_ENONFINITE, "an adjoint gradient term is not finite");
    return FBT_OK;
}

double loglik_from(int64_t n, double logdet, double quad)
{
    return -0.5 * (double)n * std::log(2.0 * M_PI) - 0.5 * logdet - 0.5 * quad;
}

// Eq. (1)-(3) from the nine terms (Algorithm 3, steps 2-4)
void assemble(int64_t nobs, const double *theta, const double *t, double *loglik, double *score,
              double *fisher)
{
    const double s2 = theta[0], n = (double)nobs;
    *loglik = loglik_from(nobs, t[0], t[1]);
    score[0] = (t[1] - n) / (2.0 * s2);
    score[1] = -0.5 * t[2] + 0.5 * t[4];
    score[2] = -0.5 * t[3] + 0.5 * t[5];
    const double I00 = n / (2.0 * s2 * s2), I01 = t[2] / (2.0 * s2), I02 = t[3] / (2.0 * s2);
    const double I11 = 0.5 * t[6], I12 = 0.5 * t[7], I22 = 0.5 * t[8];
    const double F[9] = {I00, I01, I02, I01, I11, I12, I02, I12, I22};
    std::memcpy(fisher, F, sizeof(F));
}

} // namespace

double fbt::loglik_terms(int64_t n, double logdet, double quad) { return loglik_from(n, logdet, quad); }

void fbt::assemble_terms(int64_t nobs, const double *theta, const double *t, double *loglik,
                         double *score, double *fisher)
{
    assemble(nobs, theta, t, loglik, score, fisher);
}

namespace {

fbt_status check_call(fbt_ctx *c, const double *th)
{
    if (!c)
        return FBT_EINVAL;
    c->err.clear();
    if (!theta_ok(th))
        return fail(c, FBT_EINVAL, "theta must be three finite positive numbers");
    if (c->n <= 0)
        return fail(c, FBT_ENODATA, "no data set");
    if (hipSetDevice(c->device) != hipSuccess)
        return fail(c, FBT_EDEVICE, "hipSetDevice failed");
    return FBT_OK;
}

fbt_status set_data_common(fbt_ctx *c, int64_t n, const double *locs, const double *z, bool device)
{
    if (!c)
        return FBT_EINVAL;
    c->err.clear();
    if (n < 1 || !locs || !z)
        return fail(c, FBT_EINVAL, "n must be >= 1 and locs, z non-NULL");
    if (n > (int64_t)1 << 20)
        return fail(c, FBT_EINVAL, "n too large");
    if (hipSetDevice(c->device) != hipSuccess)
        return fail(c, FBT_EDEVICE, "hipSetDevice failed");
    std::vector<double> hl((size_t)n * 2), hz((size_t)n);
    if (device) {
        HIPCHK(c, hipMemcpyAsync(hl.data(), locs, n * 16, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipMemcpyAsync(hz.data(), z, n * 8, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    } else {
        std::memcpy(hl.data(), locs, n * 16);
        std::memcpy(hz.data(), z, n * 8);
    }
    for (int64_t i = 0; i < 2 * n; ++i)
        if (!std::isfinite(hl[i]))
            return fail(c, FBT_EINVAL, "non-finite location");
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(hz[i]))
            return fail(c, FBT_EINVAL, "non-finite observation");
    fbt_status st = alloc_for(c, n);
    if (st != FBT_OK)
        return st;
    std::vector<double> xs(c->npad, 0.0), ys(c->npad, 0.0), zs(c->npad, 0.0);
    for (int64_t i = 0; i < n; ++i) {
        xs[i] = hl[2 * i];
        ys[i] = hl[2 * i + 1];
        zs[i] = hz[i];
    }
    HIPCHK(c, hipMemcpyAsync(c->x, xs.data(), c->npad * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->y, ys.data(), c->npad * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->z, zs.data(), c->npad * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return FBT_OK;
}

} // namespace

// Batched group: G fields of the same padded order evaluated together, every
// launch covering all of them (field f's buffers at f times the strides).
// mode 1: log-likelihood (Algorithm 2); mode 2: log-likelihood, score and
// Fisher (Algorithm 3).  Per-field status; a field's outputs are written only
// when its status is FBT_OK.  The arithmetic of each field is exactly that of
// a single-field evaluation.  The steps are separate so that a caller can
// capture group_enqueue in a HIP graph and replay it with new theta.

// Buffers (batched layout) and data of the G fields.
fbt_status fbt::group_prepare(fbt_ctx *c, int G, const int64_t *n, const double *const *locs,
                              const double *const *z)
{
    if (!c || G < 1 || !n || !locs || !z)
        return FBT_EINVAL;
    c->err.clear();
    if (hipSetDevice(c->device) != hipSuccess)
        return fail(c, FBT_EDEVICE, "hipSetDevice failed");
    int64_t nmax = 0;
    for (int f = 0; f < G; ++f)
        nmax = std::max(nmax, n[f]);
    const int64_t npad = NB * ((nmax + 1 + NB - 1) / NB);
    for (int f = 0; f < G; ++f)
        if (n[f] < 1 || NB * ((n[f] + 1 + NB - 1) / NB) != npad)
            return fail(c, FBT_EINVAL, "group fields must share the padded order");
    fbt_status st = alloc_fields(c, nmax, G, true);
    if (st != FBT_OK)
        return st;
    ensure_f32(c);
    (void)use_two_sided(c); // its buffers, if that form is selected (group_enqueue allocates nothing)
    c->nf.assign(n, n + G);
    std::vector<double> xs((size_t)G * npad, 0.0), ys((size_t)G * npad, 0.0), zs((size_t)G * npad, 0.0);
    for (int f = 0; f < G; ++f)
        for (int64_t i = 0; i < n[f]; ++i) {
            xs[(size_t)f * npad + i] = locs[f][2 * i];
            ys[(size_t)f * npad + i] = locs[f][2 * i + 1];
            zs[(size_t)f * npad + i] = z[f][i];
        }
    HIPCHK(c, hipMemcpyAsync(c->x, xs.data(), xs.size() * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->y, ys.data(), ys.size() * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->z, zs.data(), zs.size() * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_nf, n, (size_t)G * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return FBT_OK;
}

// Tables of the G fields' theta (G x 3) into the pinned staging buffers; an
// invalid theta is replaced by a harmless one and flagged in bad[f].
void fbt::group_stage(fbt_ctx *c, const double *thetas, int *bad)
{
    std::vector<double> th(thetas, thetas + 3 * (size_t)c->G);
    for (int f = 0; f < c->G; ++f) {
        bad[f] = !theta_ok(&th[3 * f]);
        if (bad[f]) {
            th[3 * f] = 1.0;
            th[3 * f + 1] = 0.1;
            th[3 * f + 2] = 0.5;
        }
    }
    GenParams gp;
    stage_theta(c, th.data(), &gp);
}

// One evaluation of the group from the staged tables: upload, generation,
// factorisation and (mode 2) the W phase, ending with the result copies to
// pinned host memory.  No host wait, no allocation, no memset: capturable.
fbt_status fbt::group_enqueue(fbt_ctx *c, int mode)
{
    if (!c || !c->batched || (mode != 1 && mode != 2))
        return FBT_EINVAL;
    fbt_status st = upload_staged_theta(c);
    if (st != FBT_OK)
        return st;
    if ((st = factorize_enqueue(c, c->h_gpa[0], mode == 1 ? GEN_SIGMA : GEN_ALL)) != FBT_OK)
        return st;
    if (mode != 2)
        return FBT_OK;
    return use_two_sided(c, false) ? wphase_sygst_enqueue(c) : wphase_enqueue(c);
}

// Per-field outputs once the enqueued evaluation has completed.
fbt_status fbt::group_results(fbt_ctx *c, int mode, const double *thetas, const int *bad,
                              double *loglik, double *score, double *fisher, int32_t *status)
{
    factor_results(c);
    std::vector<double> terms((size_t)c->G * 9);
    if (mode == 2)
        wphase_results(c, terms.data());
    for (int f = 0; f < c->G; ++f) {
        status[f] = bad[f] ? FBT_EINVAL : c->fst[f];
        if (status[f] != FBT_OK)
            continue;
        if (mode == 1)
            loglik[f] = loglik_from(c->nf[f], c->fout[2 * f], c->fout[2 * f + 1]);
        else
            assemble(c->nf[f], thetas + 3 * f, &terms[9 * f], loglik + f, score + 3 * f,
                     fisher + 9 * f);
    }
    c->factor_valid = false;
    return FBT_OK;
}

fbt_status fbt::group_run(fbt_ctx *c, int G, const int64_t *n, const double *const *locs,
                          const double *const *z, const double *thetas, int mode, double *loglik,
                          double *score, double *fisher, int32_t *status)
{
    if (!c || G < 1 || !n || !locs || !z || !thetas || !loglik || !status ||
        (mode == 2 && (!score || !fisher)) || (mode != 1 && mode != 2))
        return FBT_EINVAL;
    fbt_status st = group_prepare(c, G, n, locs, z);
    if (st != FBT_OK)
        return st;
    std::vector<int> bad(G);
    group_stage(c, thetas, bad.data());
    if ((st = group_enqueue(c, mode)) != FBT_OK)
        return st;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    tcollect(c);
    return group_results(c, mode, thetas, bad.data(), loglik, score, fisher, status);
}

hipStream_t fbt::ctx_stream(fbt_ctx *c) { return c->stream; }

void fbt::ctx_set_capturable(fbt_ctx *c, bool on) { c->capturable = on; }

// Derivative evaluation of the Fisher-BT driver (fbt_fit).  Under a mixed
// precision the trace terms carry FP32 rounding of the block solves, which
// bounds how small the score can be resolved; once the mixed score is no
// larger than mixed_switch times the norm of its per-term scales (sigma^2:
// (q + n) / (2 sigma^2); alpha, nu: (|tr(Sigma^-1 Sigma_i)| + |w^T Sigma_i w|) / 2)
// the context switches to FP64 for the rest of the fit (*state = 1) and the
// same theta is evaluated again in FP64, on the same factor when the
// factorisation was FP64 already (FBT_MIXED_FP32).
fbt_status fbt::fit_eval(fbt_ctx *c, const double *th, double mixed_switch, int *state,
                         double *loglik, double *score, double *fisher)
{
    fbt_status st = check_call(c, th);
    if (st != FBT_OK)
        return st;
    double t[9];
    if ((st = derivative_terms(c, th, t)) != FBT_OK)
        return st;
    assemble(c->n, th, t, loglik, score, fisher);
    if (c->precision == FBT_FP64)
        return FBT_OK;
    const double s0 = (std::fabs(t[1]) + (double)c->n) / (2.0 * th[0]);
    const double s1 = 0.5 * (std::fabs(t[2]) + std::fabs(t[4]));
    const double s2 = 0.5 * (std::fabs(t[3]) + std::fabs(t[5]));
    const double gn = std::sqrt(score[0] * score[0] + score[1] * score[1] + score[2] * score[2]);
    if (!(gn <= mixed_switch * std::sqrt(s0 * s0 + s1 * s1 + s2 * s2)))
        return FBT_OK;
    *state = 1;
    // derivative_terms leaves the factor of th in place; it is the FP64 one
    // unless the Cholesky updates were FP32 as well
    c->factor_valid = !low_factor(c->precision);
    std::memcpy(c->factor_theta, th, sizeof(c->factor_theta));
    c->precision = FBT_FP64;
    if ((st = derivative_terms(c, th, t)) != FBT_OK)
        return st;
    assemble(c->n, th, t, loglik, score, fisher);
    return FBT_OK;
}

int fbt::ctx_precision(const fbt_ctx *c) { return c->precision; }

// =========================================================================
// Allocation-free evaluation (fbt_eval_noalloc): every device buffer of one
// evaluation of up to FBT_NOALLOC_MAX_N observations lives in one file-scope
// device array, `scratch`, which each GPU the library runs on holds from the
// load of the library until the process ends.  Host code never passes the
// array's name to a kernel or a copy: each device's address of it comes from
// hipGetSymbolAddress, taken once per device with that device current.
// =========================================================================
namespace {

constexpr int64_t NA_NPAD = NB * ((FBT_NOALLOC_MAX_N + 1 + NB - 1) / NB);
constexpr int NA_T = (int)(NA_NPAD / NB);
constexpr int NA_MAXDEV = 16;
// regions (doubles), each rounded up to 256 bytes
constexpr int64_t na_round(int64_t v) { return (v + 31) / 32 * 32; }
constexpr int64_t NA_X = 0;
constexpr int64_t NA_Y = NA_X + na_round(NA_NPAD);
constexpr int64_t NA_Z = NA_Y + na_round(NA_NPAD);
constexpr int64_t NA_A = NA_Z + na_round(NA_NPAD);
constexpr int64_t NA_S2 = NA_A + na_round(NA_NPAD * NA_NPAD);
constexpr int64_t NA_LINV = NA_S2 + na_round(2 * NA_NPAD * NA_NPAD);
constexpr int64_t NA_LOG = NA_LINV + na_round((int64_t)NA_T * NB * NB);
constexpr int64_t NA_PART = NA_LOG + na_round(NA_T);
constexpr int64_t NA_OUT = NA_PART + na_round((int64_t)NA_T * (NA_NPAD / 64) * 8);
constexpr int64_t NA_FLAG = NA_OUT + na_round(16);
constexpr int64_t NA_INFO = NA_FLAG + na_round(1);
constexpr int64_t NA_TAB = NA_INFO + na_round(64 / 2);
constexpr int64_t NA_YSL = NA_TAB + na_round((int64_t)(TAB_BYTES + 7) / 8);
constexpr int64_t NA_VD = NA_YSL + na_round((int64_t)2 * 2 * NA_NPAD * (2 * NB));
constexpr int64_t NA_PD = NA_VD + na_round((int64_t)2 * NA_T * NB * NB);
constexpr int64_t NA_TOTAL = NA_PD + na_round((int64_t)2 * NB * NB);

// host staging of the per-theta tables and of the results, per device
Node na_htab[NA_MAXDEV][(TAB_BYTES + sizeof(Node) - 1) / sizeof(Node)];
double na_hout[NA_MAXDEV][16];
int na_hinfo[NA_MAXDEV][64];
double na_hflag[NA_MAXDEV];
GenParams na_hgpa[NA_MAXDEV];
double *na_ptr[NA_MAXDEV];
std::mutex na_mu;

} // namespace

static __device__ __align__(256) double scratch[NA_TOTAL];

namespace {

// This device's address of `scratch` (taken on the first call on the device,
// with the device current), or nullptr on failure.
double *noalloc_scratch(int device)
{
    std::lock_guard<std::mutex> lk(na_mu);
    if (!na_ptr[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return nullptr;
        }
        na_ptr[device] = static_cast<double *>(p);
    }
    return na_ptr[device];
}

} // namespace

// =========================================================================
// C ABI
// =========================================================================
extern "C" {

fbt_status fbt_eval_noalloc(int32_t device, void *hip_stream, int64_t n, const double *d_locs_xy,
                            const double *d_z, const double theta[3], double *loglik,
                            double score[3], double fisher[9])
{
    if (!d_locs_xy || !d_z || !theta_ok(theta) || !loglik || !score || !fisher)
        return FBT_EINVAL;
    if (n < 1 || n > FBT_NOALLOC_MAX_N || device < 0 || device >= NA_MAXDEV)
        return FBT_EINVAL;
    if (hipSetDevice(device) != hipSuccess)
        return FBT_EDEVICE;
    double *base = noalloc_scratch(device);
    if (!base)
        return FBT_EDEVICE;
    // A context view of the scratch: one stream (the caller's), no events, the
    // buffers of a single field of padded order npad <= NA_NPAD at their
    // regions.  Nothing here allocates; the work is fbt_eval's launch sequence.
    fbt_ctx c;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    c.device = device;
    c.stream = c.stream2 = c.stream3 = c.stream4 = st;
    c.precision = FBT_FP64;
    c.sigma_nu_mode = FBT_SIGMA_NU_EXACT;
    c.wphase = FBT_WPHASE_TWO_SIDED;
    c.n = n;
    c.npad = NB * ((n + 1 + NB - 1) / NB);
    c.ld = c.npad;
    c.T = (int)(c.npad / NB);
    c.ncols = 128 * ((n + 127) / 128);
    c.x = base + NA_X;
    c.y = base + NA_Y;
    c.z = base + NA_Z;
    c.A = base + NA_A;
    c.S2 = base + NA_S2;
    c.Linv = base + NA_LINV;
    c.logdet = base + NA_LOG;
    c.partials = base + NA_PART;
    c.out = base + NA_OUT;
    c.info = reinterpret_cast<int *>(base + NA_INFO);
    c.tab = reinterpret_cast<Node *>(base + NA_TAB);
    c.Ysl = base + NA_YSL;
    c.Vd = base + NA_VD;
    c.Pd = base + NA_PD;
    c.cap_ysl = (size_t)(NA_VD - NA_YSL) * 8;
    c.cap_vd = (size_t)(NA_PD - NA_VD) * 8;
    c.cap_pd = (size_t)(NA_TOTAL - NA_PD) * 8;
    c.h_tab = na_htab[device];
    c.h_out = na_hout[device];
    c.h_info = na_hinfo[device];
    c.h_gpa = &na_hgpa[device];
    c.G = 1;
    c.batched = false;
    c.F.count = 1;
    c.F.sA = c.npad * c.npad;
    c.F.sS2 = 2 * c.npad * c.npad;
    c.F.sLinv = (int64_t)c.T * NB * NB;
    c.F.sVec = c.npad;
    c.F.sPart = (int64_t)c.T * (c.npad / 64) * 8;
    c.F.sLog = c.T;
    c.F.n = nullptr;
    c.F.sXf = 0;
    launch_pack_data(st, d_locs_xy, d_z, n, c.npad, c.x, c.y, c.z, base + NA_FLAG);
    GenParams gp;
    fbt_status s = upload_theta(&c, theta, &gp);
    if (s == FBT_OK)
        s = factorize_enqueue(&c, gp, GEN_ALL);
    if (s == FBT_OK && !use_two_sided(&c, false))
        s = FBT_EDEVICE; // the scratch holds the two-sided buffers: cannot happen
    if (s == FBT_OK)
        s = wphase_sygst_enqueue(&c);
    if (s == FBT_OK &&
        hipMemcpyAsync(&na_hflag[device], base + NA_FLAG, sizeof(double), hipMemcpyDeviceToHost,
                       st) != hipSuccess)
        s = FBT_EDEVICE;
    if (hipStreamSynchronize(st) != hipSuccess)
        return FBT_EDEVICE;
    if (s != FBT_OK)
        return s;
    if (na_hflag[device] != 0.0)
        return FBT_EINVAL; // a location or observation is not finite
    if (na_hinfo[device][0] != 0x7fffffff)
        return FBT_ENOTPD;
    double t[9];
    for (int i = 0; i < 9; ++i) {
        t[i] = na_hout[device][i];
        if (!std::isfinite(t[i]))
            return FBT_ENONFINITE;
    }
    assemble(n, theta, t, loglik, score, fisher);
    return FBT_OK;
}

const char *fbt_status_string(fbt_status s)
{
    switch (s) {
    case FBT_OK: return "ok";
    case FBT_EINVAL: return "invalid argument";
    case FBT_ENOTPD: return "covariance not positive definite";
    case FBT_ENOMEM: return "out of memory";
    case FBT_EDEVICE: return "device error";
    case FBT_ENONFINITE: return "non-finite result";
    case FBT_EBUDGET: return "call budget exhausted";
    case FBT_ENODATA: return "no data";
    }
    return "unknown status";
}

const char *fbt_last_error(const fbt_ctx *ctx) { return ctx ? ctx->err.c_str() : "NULL context"; }

int64_t fbt_last_notpd_pivot(const fbt_ctx *ctx) { return ctx ? ctx->notpd : -1; }

fbt_status fbt_create(const fbt_config *cfg, fbt_ctx **out)
{
    if (!cfg || !out)
        return FBT_EINVAL;
    *out = nullptr;
    if (!(cfg->tile == 0 || cfg->tile == NB) ||
        cfg->precision < FBT_FP64 || cfg->precision > FBT_MIXED_BF16_ALL)
        return FBT_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || cfg->device < 0 || cfg->device >= ndev)
        return FBT_EDEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, cfg->device) != hipSuccess ||
        std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return FBT_EDEVICE;
    if (hipSetDevice(cfg->device) != hipSuccess)
        return FBT_EDEVICE;
    fbt_ctx *c = new fbt_ctx();
    c->device = cfg->device;
    c->precision = cfg->precision;
    if (cfg->hip_stream) {
        c->stream = (hipStream_t)cfg->hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return FBT_EDEVICE;
        }
        c->own_stream = true;
    }
    {
        // The factorisation's bulk stream leaves one CU of every XCD free.  Its
        // critical path is a single-workgroup kernel (the diagonal block, 144 KB
        // of LDS and 312 registers per lane) that fits only on a CU no bulk
        // workgroup occupies; without a reserve it waits for the whole trailing
        // update to drain.  Workgroups are spread over the XCDs round-robin, so
        // every XCD needs a free CU.  CU mask bit i is CU i / NXCD of XCD
        // i % NXCD (measured: clearing bits 0..7 reserves one CU per XCD).
        const int ncu = prop.multiProcessorCount;
        std::vector<uint32_t> mask((ncu + 31) / 32, 0u);
        for (int i = 0; i < ncu; ++i)
            if (i >= FACT_CU_RESERVE)
                mask[i / 32] |= 1u << (i % 32);
        if (hipExtStreamCreateWithCUMask(&c->stream3, (uint32_t)mask.size(), mask.data()) !=
            hipSuccess) {
            fbt_destroy(c);
            return FBT_EDEVICE;
        }
    }
    if (hipStreamCreateWithFlags(&c->stream2, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->evP, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->evB, hipEventDisableTiming) != hipSuccess ||
        hipStreamCreateWithFlags(&c->stream4, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->evP2, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->evB2, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->evD, hipEventDisableTiming) != hipSuccess) {
        fbt_destroy(c);
        return FBT_EDEVICE;
    }
    *out = c;
    return FBT_OK;
}

void fbt_destroy(fbt_ctx *c)
{
    if (!c)
        return;
    (void)hipSetDevice(c->device);
    if (c->stream)
        (void)hipStreamSynchronize(c->stream);
    free_buffers(c);
    for (hipEvent_t e : c->pool)
        (void)hipEventDestroy(e);
    if (c->h_tab)
        (void)hipHostFree(c->h_tab);
    if (c->h_out)
        (void)hipHostFree(c->h_out);
    if (c->h_info)
        (void)hipHostFree(c->h_info);
    if (c->stream2) {
        (void)hipStreamSynchronize(c->stream2);
        (void)hipStreamDestroy(c->stream2);
    }
    if (c->stream3) {
        (void)hipStreamSynchronize(c->stream3);
        (void)hipStreamDestroy(c->stream3);
    }
    if (c->evP)
        (void)hipEventDestroy(c->evP);
    if (c->evB)
        (void)hipEventDestroy(c->evB);
    for (hipEvent_t e : {c->evP2, c->evB2, c->evD})
        if (e)
            (void)hipEventDestroy(e);
    if (c->stream4) {
        (void)hipStreamSynchronize(c->stream4);
        (void)hipStreamDestroy(c->stream4);
    }
    if (c->own_stream && c->stream)
        (void)hipStreamDestroy(c->stream);
    delete c;
}

fbt_status fbt_set_data(fbt_ctx *ctx, int64_t n, const double *locs_xy, const double *z)
{
    return set_data_common(ctx, n, locs_xy, z, false);
}

fbt_status fbt_set_data_device(fbt_ctx *ctx, int64_t n, const double *d_locs_xy, const double *d_z)
{
    return set_data_common(ctx, n, d_locs_xy, d_z, true);
}

fbt_status fbt_loglik(fbt_ctx *ctx, const double theta[3], double *loglik)
{
    fbt_status st = check_call(ctx, theta);
    if (st != FBT_OK)
        return st;
    if (!loglik)
        return fail(ctx, FBT_EINVAL, "loglik is NULL");
    if ((st = factorize(ctx, theta, GEN_SIGMA)) != FBT_OK)
        return st;
    *loglik = loglik_from(ctx->n, ctx->factor_out[0], ctx->factor_out[1]);
    return FBT_OK;
}

fbt_status fbt_eval_terms(fbt_ctx *ctx, const double theta[3], double terms[9])
{
    fbt_status st = check_call(ctx, theta);
    if (st != FBT_OK)
        return st;
    if (!terms)
        return fail(ctx, FBT_EINVAL, "terms is NULL");
    double t[9];
    if ((st = derivative_terms(ctx, theta, t)) != FBT_OK)
        return st;
    std::memcpy(terms, t, sizeof(t));
    return FBT_OK;
}

fbt_status fbt_eval(fbt_ctx *ctx, const double theta[3], double *loglik, double score[3],
                    double fisher[9])
{
    fbt_status st = check_call(ctx, theta);
    if (st != FBT_OK)
        return st;
    if (!loglik || !score || !fisher)
        return fail(ctx, FBT_EINVAL, "NULL output");
    double t[9];
    if ((st = derivative_terms(ctx, theta, t)) != FBT_OK)
        return st;
    assemble(ctx->n, theta, t, loglik, score, fisher);
    return FBT_OK;
}

fbt_status fbt_grad(fbt_ctx *ctx, const double theta[3], double *loglik, double score[3],
                    double *dloglik_dz)
{
    fbt_status st = check_call(ctx, theta);
    if (st != FBT_OK)
        return st;
    if (!loglik || !score)
        return fail(ctx, FBT_EINVAL, "output pointers must not be NULL");
    double g[2];
    if ((st = adjoint_terms(ctx, theta, g)) != FBT_OK)
        return st;
    if (dloglik_dz) {
        HIPCHK(ctx, hipMemcpyAsync(dloglik_dz, ctx->wv, (size_t)ctx->n * sizeof(double),
                                   hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        for (int64_t i = 0; i < ctx->n; ++i)
            dloglik_dz[i] = -dloglik_dz[i];
    }
    const double n = (double)ctx->n;
    *loglik = loglik_from(ctx->n, ctx->factor_out[0], ctx->factor_out[1]);
    score[0] = (ctx->factor_out[1] - n) / (2.0 * theta[0]);
    score[1] = g[0];
    score[2] = g[1];
    return FBT_OK;
}

fbt_status fbt_covariance(fbt_ctx *ctx, const double theta[3], int32_t which, double *out,
                          int64_t ld)
{
    fbt_status st = check_call(ctx, theta);
    if (st != FBT_OK)
        return st;
    if (!out || ld < ctx->n || which < 0 || which > 2)
        return fail(ctx, FBT_EINVAL, "bad output arguments");
    GenParams gp;
    if ((st = upload_theta(ctx, theta, &gp)) != FBT_OK)
        return st;
    ctx->factor_valid = false;
    const int64_t n = ctx->n, npad = ctx->npad, dld = ctx->ld;
    launch_gen(ctx->stream, gp, ctx->d_gpa, ctx->F, ctx->x, ctx->y, ctx->z, ctx->A, ctx->S2,
               ctx->S2 + npad * dld, which == 0 ? GEN_SIGMA : GEN_DERIV);
    const double *src = which == 0 ? ctx->A : (which == 1 ? ctx->S2 : ctx->S2 + npad * dld);
    HIPCHK(ctx, hipMemcpy2DAsync(out, ld * 8, src, dld * 8, n * 8, n, hipMemcpyDeviceToHost,
                                 ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (which == 0) // Sigma' is generated in its lower triangle only
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < j; ++i)
                out[i + j * ld] = out[j + i * ld];
    return FBT_OK;
}

fbt_status fbt_factor(fbt_ctx *ctx, const double theta[3], double *out, int64_t ld)
{
    fbt_status st = check_call(ctx, theta);
    if (st != FBT_OK)
        return st;
    if (!out || ld < ctx->n)
        return fail(ctx, FBT_EINVAL, "bad output arguments");
    if ((st = factorize(ctx, theta, GEN_SIGMA)) != FBT_OK)
        return st;
    const int64_t n = ctx->n;
    HIPCHK(ctx, hipMemcpy2DAsync(out, ld * 8, ctx->A, ctx->ld * 8, n * 8, n, hipMemcpyDeviceToHost,
                                 ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < j; ++i)
            out[i + j * ld] = 0.0;
    return FBT_OK;
}

fbt_status fbt_set_precision(fbt_ctx *ctx, int32_t precision)
{
    if (!ctx || precision < FBT_FP64 || precision > FBT_MIXED_BF16_ALL)
        return FBT_EINVAL;
    // the factorisation's arithmetic differs only under the _ALL forms
    if (precision != ctx->precision && (low_factor(precision) || low_factor(ctx->precision)))
        ctx->factor_valid = false;
    ctx->precision = precision;
    return FBT_OK;
}

fbt_status fbt_set_refinement(fbt_ctx *ctx, int32_t iterations)
{
    if (!ctx || iterations < 0 || iterations > 16)
        return fail(ctx, FBT_EINVAL, "refinement steps must be in [0, 16]");
    ctx->refine_iters = iterations;
    ctx->factor_valid = false;
    return FBT_OK;
}

fbt_status fbt_set_wphase(fbt_ctx *ctx, int32_t form)
{
    if (!ctx || (form != FBT_WPHASE_TWO_SIDED && form != FBT_WPHASE_SOLVES))
        return fail(ctx, FBT_EINVAL, "unknown W-phase form");
    ctx->wphase = form;
    return FBT_OK;
}

fbt_status fbt_set_sigma_nu_mode(fbt_ctx *ctx, int32_t mode)
{
    if (!ctx || (mode != FBT_SIGMA_NU_EXACT && mode != FBT_SIGMA_NU_PAPER))
        return fail(ctx, FBT_EINVAL, "unknown Sigma_nu mode");
    ctx->sigma_nu_mode = mode;
    return FBT_OK;
}

fbt_status fbt_set_timing(fbt_ctx *ctx, int32_t enable)
{
    if (!ctx)
        return FBT_EINVAL;
    ctx->timing = enable != 0;
    ctx->pending.clear();
    ctx->pool_used = 0;
    for (int i = 0; i < NCLASS; ++i) {
        ctx->cls_n[i] = 0;
        ctx->cls_ms[i] = 0.0;
        ctx->cls_flops[i] = 0.0;
    }
    return FBT_OK;
}

fbt_status fbt_get_timing(fbt_ctx *ctx, int32_t kernel_class, int64_t *launches, double *ms,
                          double *flops)
{
    if (!ctx || kernel_class < 0 || kernel_class >= NCLASS || !launches || !ms || !flops)
        return FBT_EINVAL;
    *launches = ctx->cls_n[kernel_class];
    *ms = ctx->cls_ms[kernel_class];
    *flops = ctx->cls_flops[kernel_class];
    return FBT_OK;
}

} // extern "C"
