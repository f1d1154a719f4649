// Persistent round kernel: the evaluations of all fields of one batched
// Fisher-BT round (Algorithm 2 or 3 per field) in one launch.  Workgroups take
// tile tasks (fbt_round.h) by ticket from one counter, in the order the host
// planner chose; a task first waits until the counters of the tiles it reads
// reach their values, and advances its own counters when its tiles are
// stored.  Tasks wait only on tasks with smaller tickets (checked on the host
// for every plan), and every ticket below a workgroup's own is held by a
// running workgroup, so the smallest unfinished ticket can always proceed:
// the launch drains for any number of resident workgroups.  Every wait is
// also bounded in wall-clock time; a wait that runs out raises an abort flag,
// after which all remaining waits return at once and the host reports the
// failure (no path can spin forever).
//
// Tiles are BT x BT (64 or 128) in the bordered, column-major storage of the
// single-field path (Sigma' with the observation row n, identity padding;
// Sigma_alpha' and Sigma_nu' side by side).  Products run on FP64 MFMA with a
// 2 x 2 arrangement of waves; the diagonal factorisation and its inverse on
// 64 x 64 blocks in LDS.
#include "fbt_internal.h"
#include "fbt_device.h"
#include "fbt_plan.h"
#include "fbt_round.h"

#include <math.h>

namespace fbt {

struct RField {
    GenParams gp;         // theta, node table; gp.n = n
    double *A;            // Sigma' then L' (npad x npad)
    double *S;            // Sigma_alpha' | Sigma_nu', then X, then W (npad x 2 npad)
    double *Linv;         // T inverses of the diagonal tiles (BT x BT each)
    double *part;         // rpart(T) slots
    double *out;          // 16: logdet, q, tr_a, tr_n, u_a, u_n, F_aa, F_an, F_nn
    int *cnt;             // rcount(T) counters
    const double *x, *y, *z;
    int64_t n, ld;        // ld = npad = T BT
    int T, mode, skip;    // skip: no arithmetic (invalid theta); counters still advance
};

namespace {

// Threads per workgroup: 4 waves, two workgroups per CU (two waves per SIMD,
// at most 256 registers per lane).  The tasks other than the tile products
// are separate functions (not inlined), so that the kernel's register
// allocation at the product is that of the product alone.
constexpr int rthreads(int) { return 256; }

// ---------------------------------------------------------------------------
// MFMA product of one BT x BT tile: acc -= A (BT x K) B^T with A M-contiguous
// (element (m, k) at A[m + k lda]) and B N-contiguous (element (n, k) at
// B[n + k ldb]) or, with bkc, K-contiguous (at B[k + n ldb]).  The four
// waves of the workgroup in 2 x 2, each a (BT/2)^2 block of 16 x 16
// accumulators; K in chunks of 16 through double-buffered LDS (A is negated
// when staged).  With the B
// fragment as the MFMA's first operand, lane l holds in accumulator (i, j),
// element r, the entry (16 i + l % 16, 16 j + l / 16 + 4 r) of the wave's
// block.  The kernel has one call site of run (every product of every task
// goes through it), which keeps its register allocation that of one product.
// ---------------------------------------------------------------------------
template <int BT> struct RTile {
    static constexpr int NT = rthreads(BT), WN = NT / 128; // waves: 2 x WN
    static constexpr int WTM = BT / 2, WTN = BT / WN;      // wave block
    static constexpr int MI = WTM / 16, NJ = WTN / 16;     // accumulators per wave
    static constexpr int KC = 16, LS = BT + 4;
    static constexpr int STAGE = 2 * KC * LS;
    static constexpr int NL = BT * KC / (2 * NT);

    __device__ static void load(double2 *ra, double2 *rb, const double *A, int64_t lda,
                                const double *B, int64_t ldb, int k0, bool bkc)
    {
        const int t = threadIdx.x;
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int q = t + NT * i;
            const int m2 = q % (BT / 2), k = q / (BT / 2);
            ra[i] = *(const double2 *)(A + 2 * m2 + (int64_t)(k0 + k) * lda);
        }
        if (!bkc) {
#pragma unroll
            for (int i = 0; i < NL; ++i) {
                const int q = t + NT * i;
                const int n2 = q % (BT / 2), k = q / (BT / 2);
                rb[i] = *(const double2 *)(B + 2 * n2 + (int64_t)(k0 + k) * ldb);
            }
        } else {
#pragma unroll
            for (int i = 0; i < NL; ++i) {
                const int q = t + NT * i;
                const int k2 = q % (KC / 2), nn = q / (KC / 2);
                rb[i] = *(const double2 *)(B + (k0 + 2 * k2) + (int64_t)nn * ldb);
            }
        }
    }
    __device__ static void store(const double2 *ra, const double2 *rb, double *st, bool bkc)
    {
        const int t = threadIdx.x;
        double *As = st, *Bs = st + KC * LS;
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int q = t + NT * i;
            const int m2 = q % (BT / 2), k = q / (BT / 2);
            double2 v = ra[i];
            v.x = -v.x;
            v.y = -v.y;
            *(double2 *)(As + k * LS + 2 * m2) = v;
        }
        if (!bkc) {
#pragma unroll
            for (int i = 0; i < NL; ++i) {
                const int q = t + NT * i;
                const int n2 = q % (BT / 2), k = q / (BT / 2);
                *(double2 *)(Bs + k * LS + 2 * n2) = rb[i];
            }
        } else {
#pragma unroll
            for (int i = 0; i < NL; ++i) {
                const int q = t + NT * i;
                const int k2 = q % (KC / 2), nn = q / (KC / 2);
                Bs[(2 * k2) * LS + nn] = rb[i].x;
                Bs[(2 * k2 + 1) * LS + nn] = rb[i].y;
            }
        }
    }
    __device__ static void compute(d4 (&acc)[MI][NJ], const double *st, int wm, int wn, int lane)
    {
        const double *As = st + wm * WTM + (lane & 15);
        const double *Bs = st + KC * LS + wn * WTN + (lane & 15);
#pragma unroll
        for (int s = 0; s < KC / 4; ++s) {
            const int kk = 4 * s + (lane >> 4);
            double a[MI], b[NJ];
#pragma unroll
            for (int i = 0; i < MI; ++i)
                a[i] = As[kk * LS + 16 * i];
#pragma unroll
            for (int j = 0; j < NJ; ++j)
                b[j] = Bs[kk * LS + 16 * j];
#pragma unroll
            for (int i = 0; i < MI; ++i)
#pragma unroll
                for (int j = 0; j < NJ; ++j)
                    acc[i][j] = mfma(b[j], a[i], acc[i][j]);
        }
    }
    // K % 16 == 0, K > 0; ends with a barrier after the last LDS use, and all
    // global reads of A and B are complete before it.
    __device__ static void run(d4 (&acc)[MI][NJ], const double *A, int64_t lda, const double *B,
                               int64_t ldb, int K, bool bkc, double *lds)
    {
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const int wm = wave & 1, wn = wave >> 1;
        double2 ra[NL], rb[NL];
        load(ra, rb, A, lda, B, ldb, 0, bkc);
        store(ra, rb, lds, bkc);
        __syncthreads();
        const int nch = K / KC;
        for (int c = 0; c < nch; ++c) {
            if (c + 1 < nch)
                load(ra, rb, A, lda, B, ldb, (c + 1) * KC, bkc);
            compute(acc, lds + (c & 1) * STAGE, wm, wn, lane);
            if (c + 1 < nch)
                store(ra, rb, lds + ((c + 1) & 1) * STAGE, bkc);
            __syncthreads();
        }
    }
};

template <int BT> struct RAcc {
    typedef RTile<BT> E;
    static constexpr int MI = E::MI, NJ = E::NJ;
    d4 v[MI][NJ];
    __device__ int row(int i, int lane, int wm) const { return wm * E::WTM + 16 * i + (lane & 15); }
    __device__ int col(int j, int r, int lane, int wn) const
    {
        return wn * E::WTN + 16 * j + (lane >> 4) + 4 * r;
    }
    __device__ void zero()
    {
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
            for (int j = 0; j < NJ; ++j)
                v[i][j] = (d4){0.0, 0.0, 0.0, 0.0};
    }
    // The tile's base and leading dimension pass through an empty asm so that
    // the 64-bit addresses of a load and the later store of the same tile are
    // not kept live across the product in between.
    __device__ void load(const double *C, int64_t ldc)
    {
        asm volatile("" : "+s"(C), "+s"(ldc));
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const int wm = wave & 1, wn = wave >> 1;
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
            for (int j = 0; j < NJ; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    v[i][j][r] = C[row(i, lane, wm) + (int64_t)col(j, r, lane, wn) * ldc];
    }
    __device__ void store(double *C, int64_t ldc, bool neg) const
    {
        asm volatile("" : "+s"(C), "+s"(ldc));
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const int wm = wave & 1, wn = wave >> 1;
        const double sg = neg ? -1.0 : 1.0;
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
            for (int j = 0; j < NJ; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    C[row(i, lane, wm) + (int64_t)col(j, r, lane, wn) * ldc] = sg * v[i][j][r];
    }
};

// ---- waits and releases ---------------------------------------------------
// ctl[1]: abort flag (a wait ran out of time); ctl[RQ_CTL + RQ_STRIDE q]:
// ticket counter of queue q (one 128-byte line each).
constexpr int RQ_CTL = 32, RQ_STRIDE = 32, RQ_MAX = 8;
constexpr int R_CTL_WORDS = RQ_CTL + RQ_STRIDE * RQ_MAX;

// thread 0: wait until *p >= v (acquire), at most `limit` ticks of the
// 100 MHz wall clock; false on timeout or abort.
__device__ bool wait_ge(const int *p, int v, int *ctl, int64_t limit)
{
    if (__hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >= v)
        return true;
    const int64_t t0 = wall_clock64();
    for (;;) {
        __builtin_amdgcn_s_sleep(8);
        if (__hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >= v)
            return true;
        if (__hip_atomic_load(ctl + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
            return false;
        if (wall_clock64() - t0 > limit) {
            __hip_atomic_store(ctl + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
    }
}

// whole workgroup: waits a of counters off[a0..a1) (>= need); uniform result
__device__ bool wait_all(const int *cnt, const int *off, const int *need, int a0, int a1, int *ctl,
                         int64_t limit, int *sflag)
{
    if (threadIdx.x == 0) {
        bool ok = true;
        for (int a = a0; a < a1 && ok; ++a)
            ok = wait_ge(cnt + off[a], need[a], ctl, limit);
        *sflag = ok ? 1 : 0;
    }
    __syncthreads();
    const bool ok = __builtin_amdgcn_readfirstlane(*sflag) != 0;
    __syncthreads();
    return ok;
}

// whole workgroup: make every thread's stores visible device-wide, then
// advance the counters (release)
__device__ void release(int *cnt, const int *off, int k)
{
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0)
        for (int a = 0; a < k; ++a)
            __hip_atomic_fetch_add(cnt + off[a], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double wsum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

// fixed-order workgroup sum of one value per thread (result in thread 0)
template <int NT> __device__ double bsum(double v, double *sh)
{
    v = wsum(v);
    if ((threadIdx.x & 63) == 0)
        sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < NT / 64; ++w)
            s += sh[w];
    __syncthreads();
    return s;
}

// ---- diagonal tiles: 64 x 64 blocks in LDS (element (r, c) at P[r RP + c]) --
constexpr int RP = 65;

// In-place Cholesky of the lower part of P.  Pivot rule of the single-field
// path: rows g >= n (observation border, padding) take pivot 1; a pivot <= 0
// or not finite at g < n records the first such row in *bad (thread 0) and
// takes pivot 1.  Thread 0 adds log(pivot) over rows g < n to *logsum.
template <int NT>
__device__ void chol64(double *P, int64_t g0, int64_t n, double *logsum, int64_t *bad)
{
    const int t = threadIdx.x;
    for (int k = 0; k < 64; ++k) {
        const double a = P[k * RP + k];
        const int64_t g = g0 + k;
        double d;
        if (g >= n) {
            d = 1.0;
        } else if (a > 0.0 && a <= 1.7976931348623157e308) {
            d = sqrt(a);
            if (t == 0)
                *logsum += log(d);
        } else {
            d = 1.0;
            if (t == 0 && *bad < 0)
                *bad = g;
        }
        __syncthreads(); // every thread has read the pivot
        if (t == 0)
            P[k * RP + k] = d;
        if (t < 63 - k)
            P[(k + 1 + t) * RP + k] /= d;
        __syncthreads();
        const int r = t & 63;
        if (r > k) {
            const double lrk = P[r * RP + k];
            for (int c = k + 1 + (t >> 6); c <= r; c += NT / 64)
                P[r * RP + c] -= lrk * P[c * RP + k];
        }
        __syncthreads();
    }
}

// Q = inverse of the lower-triangular P (lower; zeros above), by one wave:
// lane c forward-substitutes column c.
__device__ void trtri64(const double *P, double *Q)
{
    const int c = threadIdx.x;
    if (c < 64) {
        for (int r = 0; r < 64; ++r) {
            double s = 0.0;
            for (int m = 0; m < r; ++m)
                s = fma(P[r * RP + m], Q[m * RP + c], s);
            Q[r * RP + c] = (r < c) ? 0.0 : (((r == c) ? 1.0 : 0.0) - s) / P[r * RP + r];
        }
    }
    __syncthreads();
}

// 64 x 64 products with 4 x 4 blocks per thread of the first 256 threads:
// out = sum_k X(r, k) Y(k, c) for element accessors X, Y; the 16 results go
// to o[] (rows r0.., cols c0..).  Other threads return at once (false).
template <class FX, class FY>
__device__ bool mul64(FX X, FY Y, double (&o)[4][4], int &r0, int &c0)
{
    const int t = threadIdx.x;
    if (t >= 256)
        return false;
    r0 = (t & 15) * 4;
    c0 = (t >> 4) * 4;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
            o[a][b] = 0.0;
    for (int k = 0; k < 64; ++k) {
        double x[4], y[4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
            x[a] = X(r0 + a, k);
#pragma unroll
        for (int b = 0; b < 4; ++b)
            y[b] = Y(k, c0 + b);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
                o[a][b] = fma(x[a], y[b], o[a][b]);
    }
    return true;
}

// Factor of the diagonal tile D (global, ld) in place (lower part; the upper
// part is not used) and its inverse into Li (BT x BT, zeros above the
// diagonal).  BT = 64: one block.  BT = 128: blocks 0 and 1 of 64,
//   L00 = chol(A00), L10 = A10 L00^{-T}, L11 = chol(A11 - L10 L10^T),
//   Li = [[L00^{-1}, 0], [-L11^{-1} L10 L00^{-1}, L11^{-1}]].
template <int BT, int NT>
__device__ __attribute__((noinline)) void diag_factor(double *D, int64_t ld, double *Li, int64_t g0, int64_t n, double *lds,
                            double *logsum, int64_t *bad)
{
    const int t = threadIdx.x;
    double *P = lds, *Q = lds + 64 * RP;
    for (int e = t; e < 64 * 64; e += NT) {
        const int r = e & 63, c = e >> 6;
        P[r * RP + c] = D[r + (int64_t)c * ld];
    }
    __syncthreads();
    chol64<NT>(P, g0, n, logsum, bad);
    trtri64(P, Q);
    for (int e = t; e < 64 * 64; e += NT) {
        const int r = e & 63, c = e >> 6;
        if (r >= c)
            D[r + (int64_t)c * ld] = P[r * RP + c];
        Li[r + c * BT] = Q[r * RP + c];
    }
    if (BT == 128) {
        for (int e = t; e < 64 * 64; e += NT) {
            const int r = e & 63, c = e >> 6;
            Li[r + (c + 64) * BT] = 0.0; // upper-right block of the inverse
        }
        double o[4][4];
        int r0, c0;
        // L10 = A10 D0^T (A10 from D, D0 = L00^{-1} in Q)
        const double *A10 = D + 64;
        bool act = mul64([&](int r, int k) { return A10[r + (int64_t)k * ld]; },
                         [&](int k, int c) { return Q[c * RP + k]; }, o, r0, c0);
        __syncthreads(); // all reads of A10 done
        double *L10 = D + 64;
        if (act)
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    L10[(r0 + a) + (int64_t)(c0 + b) * ld] = o[a][b];
        __syncthreads();
        // P = A11 - L10 L10^T
        const double *A11 = D + 64 + (int64_t)64 * ld;
        act = mul64([&](int r, int k) { return L10[r + (int64_t)k * ld]; },
                    [&](int k, int c) { return L10[c + (int64_t)k * ld]; }, o, r0, c0);
        if (act)
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    P[(r0 + a) * RP + (c0 + b)] =
                        A11[(r0 + a) + (int64_t)(c0 + b) * ld] - o[a][b];
        __syncthreads();
        chol64<NT>(P, g0 + 64, n, logsum, bad);
        trtri64(P, Q); // D1 = L11^{-1} (D0 is kept in Li)
        double *L11 = D + 64 + (int64_t)64 * ld;
        for (int e = t; e < 64 * 64; e += NT) {
            const int r = e & 63, c = e >> 6;
            if (r >= c)
                L11[r + (int64_t)c * ld] = P[r * RP + c];
            Li[(r + 64) + (c + 64) * BT] = Q[r * RP + c];
        }
        __syncthreads();
        // M = L10 D0 into P, then Li10 = -D1 M
        act = mul64([&](int r, int k) { return L10[r + (int64_t)k * ld]; },
                    [&](int k, int c) { return Li[k + c * BT]; }, o, r0, c0);
        if (act)
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    P[(r0 + a) * RP + (c0 + b)] = o[a][b];
        __syncthreads();
        act = mul64([&](int r, int k) { return Q[r * RP + k]; },
                    [&](int k, int c) { return P[k * RP + c]; }, o, r0, c0);
        if (act)
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    Li[(r0 + a + 64) + (c0 + b) * BT] = -o[a][b];
    }
}

// ---- tasks ------------------------------------------------------------------

// GEN(i, j): entries of Sigma' (lower part of the tile) and, for Algorithm 3,
// of Sigma_alpha' and Sigma_nu' at (a, b) and (b, a).
template <int BT>
__device__ __attribute__((noinline)) void task_gen(const RField &F, int ti, int tj, double *lds)
{
    Node *tab = reinterpret_cast<Node *>(lds);
    // the stores go through restrict pointers, so the descriptor's loads
    // are not repeated for every entry
    const GenParams &gp = F.gp;
    const double *xs = F.x, *ys = F.y, *zs = F.z;
    double *__restrict__ A = F.A;
    const int fmode = F.mode;
    const int t = threadIdx.x;
    const int ntab = gp.off[NLEV - 1] + gp.len[NLEV - 1];
    constexpr int NT = rthreads(BT);
    for (int i = t; i < ntab; i += NT)
        tab[i] = gp.tab[i];
    __syncthreads();
    const int mode = fmode == 2 ? GEN_ALL : GEN_SIGMA;
    const int64_t n = F.n, ld = F.ld;
    const int r = t % BT;
    const int64_t a = (int64_t)ti * BT + r;
    const double xa = a < n ? xs[a] : 0.0, ya = a < n ? ys[a] : 0.0;
    const double inv_alpha = 1.0 / gp.alpha;
    double *__restrict__ Sa = F.S;
    double *__restrict__ Sn = F.S + ld * ld;
    for (int c = t / BT; c < BT; c += NT / BT) {
        if (ti == tj && c > r)
            continue;
        const int64_t b = (int64_t)tj * BT + c;
        double cv = 0.0, ca = 0.0, cn = 0.0;
        if (a < n) {
            const double dx = xa - xs[b], dy = ya - ys[b];
            matern3(gp, tab, sqrt(dx * dx + dy * dy) * inv_alpha, mode, cv, ca, cn);
        } else if (a == n) {
            cv = (b < n) ? zs[b] : 1.0;
        } else {
            cv = (a == b) ? 1.0 : 0.0;
        }
        A[a + b * ld] = cv;
        if (mode == GEN_ALL) {
            Sa[a + b * ld] = ca;
            Sn[a + b * ld] = cn;
            if (a != b) {
                Sa[b + a * ld] = ca;
                Sn[b + a * ld] = cn;
            }
        }
    }
}

// Tile products of the CHOL, LSOLVE and RSOLVE tasks as a list of steps
//   C = (loadc ? C : 0) - A B^T (or A B with bkc; K = 0: no product),
//   then C is stored, negated with negstore.
// Two-step tasks store -T after the first step so that the second step's
// "- A B^T" with A = -T is the product with the diagonal inverse:
//   CHOL(i > j):  T = A_ij - L_i,<j L_j,<j^T;  L_ij = T Li_j^T
//   LSOLVE(k, c): T = S_kc - L_k,<k X_<k,c;    X_kc = Li_k T
//   RSOLVE(i, j): T = X_ij - W_i,<j L_j,<j^T;  W_ij = T Li_j^T   (both matrices)
struct Step {
    double *C;
    const double *A, *B;
    int64_t ldc, lda, ldb;
    int K, bkc, loadc, negstore;
};

__device__ __forceinline__ int step_count(int ty, int i, int j)
{
    if (ty == R_CHOL)
        return i > j ? 2 : (j > 0 ? 1 : 0);
    return ty == R_LSOLVE ? 2 : 4;
}

// step s of a CHOL, LSOLVE or RSOLVE task (uniform values)
template <int BT>
__device__ __forceinline__ Step make_step(const RField &F, int ty, int i, int j, int s)
{
    const int64_t ld = F.ld;
    const double *Li_j = F.Linv + (int64_t)j * BT * BT;
    if (ty == R_CHOL) {
        double *C = F.A + (int64_t)i * BT + (int64_t)j * BT * ld;
        if (s == 0)
            return Step{C, F.A + (int64_t)i * BT, F.A + (int64_t)j * BT, ld, ld, ld, j * BT, 0, 1,
                        i > j ? 1 : 0};
        return Step{C, C, Li_j, ld, ld, BT, BT, 0, 0, 0};
    }
    if (ty == R_LSOLVE) {
        double *C = F.S + (int64_t)i * BT + (int64_t)j * BT * ld;
        if (s == 0)
            return Step{C, F.A + (int64_t)i * BT, F.S + (int64_t)j * BT * ld, ld, ld, ld, i * BT,
                        1, 1, 1};
        return Step{C, F.Linv + (int64_t)i * BT * BT, C, ld, BT, ld, BT, 1, 0, 0};
    }
    const int64_t c0 = (int64_t)(s >> 1) * F.T * BT;
    double *C = F.S + (int64_t)i * BT + (c0 + (int64_t)j * BT) * ld;
    if ((s & 1) == 0)
        return Step{C, F.S + (int64_t)i * BT + c0 * ld, F.A + (int64_t)j * BT, ld, ld, ld, j * BT,
                    0, 1, 1};
    return Step{C, C, Li_j, ld, ld, BT, BT, 0, 0, 0};
}

// RSOLVE: shares of tr W_h, y^T W_h y = W'[n][n], <W_h, W_h> and, for h = 1
// (nu), <W_alpha, W_nu>, read back from the stored tiles (i, j) of W_h and
// W_alpha (the workgroup's own stores, after a barrier).  Entries a, b < n;
// the strictly lower part of a diagonal tile counts twice, its upper part not
// at all.  The workgroup sums go to red[] (thread 0, fixed order).
template <int BT>
__device__ __attribute__((noinline)) void rsolve_shares(const RField &F, int i, int j, int h, double *sh, double *red)
{
    constexpr int NT = rthreads(BT);
    const int64_t n = F.n, ld = F.ld;
    const double *Wa = F.S + (int64_t)i * BT + (int64_t)j * BT * ld;
    const double *Wh = Wa + (int64_t)h * F.T * BT * ld;
    double tr = 0.0, u = 0.0, fhh = 0.0, fan = 0.0;
    for (int e = threadIdx.x; e < BT * BT; e += NT) {
        const int rr = e % BT, cc = e / BT;
        const int64_t a = (int64_t)i * BT + rr, b = (int64_t)j * BT + cc;
        const double w = Wh[rr + (int64_t)cc * ld];
        if (a < n && b < n) {
            const double wt = (i != j || rr > cc) ? 2.0 : (rr == cc ? 1.0 : 0.0);
            fhh = fma(wt * w, w, fhh);
            if (h == 1)
                fan = fma(wt * w, Wa[rr + (int64_t)cc * ld], fan);
            if (a == b)
                tr += w;
        } else if (a == n && b == n) {
            u = w;
        }
    }
    const double s0 = bsum<NT>(tr, sh), s1 = bsum<NT>(u, sh), s2 = bsum<NT>(fhh, sh);
    const double s3 = h == 1 ? bsum<NT>(fan, sh) : 0.0;
    if (threadIdx.x == 0) {
        red[h] = s0;         // tr_a, tr_n
        red[2 + h] = s1;     // u_a, u_n
        red[4 + 2 * h] = s2; // F_aa, F_nn
        if (h == 1)
            red[5] = s3;     // F_an
    }
}

template <int BT>
__device__ __attribute__((noinline)) void task_reduce(const RField &F, double *lds, bool work)
{
    const int64_t n = F.n, ld = F.ld;
    const int T = F.T;
    const RPart pp = rpart(T);
    double q = 0.0;
    if (work)
        for (int64_t c = threadIdx.x; c < n; c += rthreads(BT)) {
            const double v = F.A[n + c * ld];
            q = fma(v, v, q);
        }
    q = bsum<rthreads(BT)>(q, lds);
    if (threadIdx.x == 0) {
        double *out = F.out;
        double ldet = 0.0;
        for (int j = 0; j < T; ++j)
            ldet += F.part[pp.logdet + 16 * j];
        out[0] = 2.0 * ldet;
        out[1] = q;
        if (F.mode == 2) {
            double s[7] = {0, 0, 0, 0, 0, 0, 0};
            for (int p = 0; p < T * (T + 1) / 2; ++p)
                for (int k = 0; k < 7; ++k)
                    s[k] += F.part[pp.wpart + 16 * p + k];
            for (int k = 0; k < 7; ++k)
                out[2 + k] = s[k];
        }
    }
}

} // namespace

constexpr int R_LDS = 2 * 16 * (128 + 4) * 2; // doubles: the BT = 128 product stages

template <int BT>
__global__ __launch_bounds__(rthreads(BT)) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_round(const RField *__restrict__ fields,
                                               const RTask *__restrict__ tasks,
                                               const int64_t *__restrict__ qoff, int nq,
                                               int *ctl, int64_t limit, long long *trace)
{
    // queue of this workgroup: workgroups are dealt to the XCDs round-robin,
    // so with nq = 8 a queue's workgroups share one XCD (and its L2)
    const int q = blockIdx.x % nq;
    const int64_t q0 = qoff[q], qn = qoff[q + 1] - q0;
    int *qctl = ctl + RQ_CTL + RQ_STRIDE * q;
    __shared__ __attribute__((aligned(16))) double lds[R_LDS];
    __shared__ int s_ticket, s_flag;
    __shared__ double s_red[8];
    static_assert(2 * 64 * RP <= R_LDS, "diagonal blocks exceed the LDS");
    static_assert(TAB_MAX * sizeof(Node) <= R_LDS * sizeof(double), "node table exceeds the LDS");
    for (;;) {
        if (threadIdx.x == 0)
            s_ticket = atomicAdd(qctl, 1);
        __syncthreads();
        // the ticket, and all task data read with it, are uniform: keep them in
        // scalar registers
        const int64_t tk = q0 + __builtin_amdgcn_readfirstlane(s_ticket);
        __syncthreads();
        if (tk >= q0 + qn)
            break;
        long long t_take = 0;
        if (trace && threadIdx.x == 0)
            t_take = wall_clock64();
        const RTask task = tasks[tk];
        const RField &F = fields[rt_field(task)];
        const int ty = rt_type(task), i = rt_i(task), j = rt_j(task);
        int off[4], need[4];
        const int nd = rdeps(task, F.T, F.mode, off, need);
        // CHOL(i > j) takes its last wait inside the task
        const int nfirst = (ty == R_CHOL && i > j) ? nd - 1 : nd;
        const bool ok = wait_all(F.cnt, off, need, 0, nfirst, ctl, limit, &s_flag);
        long long t_ready = 0;
        if (trace && threadIdx.x == 0)
            t_ready = wall_clock64();
        int failed = 0;
        if (threadIdx.x == 0)
            failed = __hip_atomic_load(F.cnt + rcount(F.T).info, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
        if (threadIdx.x == 0)
            s_flag = failed;
        __syncthreads();
        failed = __builtin_amdgcn_readfirstlane(s_flag);
        __syncthreads();
        // no arithmetic after an abort, for a skipped field, or after a failed pivot
        const bool work = ok && !F.skip && failed == 0;
        if (ty == R_GEN) {
            if (work)
                task_gen<BT>(F, i, j, lds);
        } else if (ty == R_REDUCE) {
            task_reduce<BT>(F, lds, ok && !F.skip);
        } else if (work) {
            const int ns = step_count(ty, i, j);
            bool go = true;
#pragma unroll 1
            for (int s = 0; s < ns; ++s) {
                if (ty == R_CHOL && s == 1) {
                    // CHOL(i > j): the diagonal tile's factor and inverse
                    go = wait_all(F.cnt, off, need, nd - 1, nd, ctl, limit, &s_flag);
                    if (!go)
                        break;
                }
                const Step st = make_step<BT>(F, ty, i, j, s);
                RAcc<BT> acc;
                if (st.loadc)
                    acc.load(st.C, st.ldc);
                else
                    acc.zero();
                if (st.K > 0)
                    RTile<BT>::run(acc.v, st.A, st.lda, st.B, st.ldb, st.K, st.bkc != 0, lds);
                acc.store(st.C, st.ldc, st.negstore != 0);
                __syncthreads();
                if (ty == R_RSOLVE && (s & 1))
                    rsolve_shares<BT>(F, i, j, s >> 1, lds, s_red);
            }
            if (ty == R_CHOL && i == j) {
                double logsum = 0.0;
                int64_t bad = -1;
                double *C = F.A + (int64_t)j * BT * (F.ld + 1);
                diag_factor<BT, rthreads(BT)>(C, F.ld, F.Linv + (int64_t)j * BT * BT, (int64_t)j * BT, F.n, lds,
                                &logsum, &bad);
                if (threadIdx.x == 0) {
                    F.part[rpart(F.T).logdet + 16 * j] = logsum;
                    int none = 0; // first failing row (a field's diagonal tiles run in order)
                    if (bad >= 0)
                        __hip_atomic_compare_exchange_strong(
                            F.cnt + rcount(F.T).info, &none, (int)(bad + 1), __ATOMIC_RELAXED,
                            __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            if (ty == R_RSOLVE && go && threadIdx.x == 0) {
                double *dst = F.part + rpart(F.T).wpart + 16 * rpair(i, j);
                for (int q = 0; q < 7; ++q)
                    dst[q] = s_red[q];
            }
        }
        const int np = rpublish(task, F.T, off);
        release(F.cnt, off, np);
        if (trace && threadIdx.x == 0) {
            trace[3 * tk] = t_take;
            trace[3 * tk + 1] = t_ready;
            trace[3 * tk + 2] = wall_clock64();
        }
    }
}

// counters to zero before a round (a kernel, not a memset: it may be
// recorded into a HIP graph)
__global__ __launch_bounds__(256) void k_zero_ints(int *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        p[i] = 0;
}

} // namespace fbt

// ===========================================================================
// Host side: device arena for a set of fields, the plan, and one launch per
// call.
// ===========================================================================
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

namespace fbt {

struct RoundExec {
    int device = 0;
    hipStream_t stream = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int64_t tick_khz = 100000; // wall clock of the waits
    // current arena: field set, modes and tile size it was built for
    int bt = 0;
    uint64_t version = ~(uint64_t)0;
    std::vector<int32_t> modes;
    std::vector<int64_t> n;
    int nf = 0;
    char *arena = nullptr;
    RTask *d_tasks = nullptr;
    int ntasks = 0;
    int grid = 0;
    double est_us = 0.0;
    std::vector<RField> hfield; // device pointers per field (theta filled per call)
    std::vector<int64_t> cnt_off; // first counter of each field
    size_t cnt_ints = 0;          // counters of all fields, then 64 control words
    RField *d_fields = nullptr;
    int *d_cnt = nullptr;
    char *d_tab = nullptr;
    double *d_out = nullptr;
    // pinned staging
    char *h_tab = nullptr;
    RField *h_fields = nullptr;
    double *h_out = nullptr;
    int *h_cnt = nullptr;
    float last_ms = 0.0f;
    // optional per-task trace of the last call: ticket taken, waits done, end
    // (wall-clock ticks)
    bool trace_on = false;
    long long *d_trace = nullptr;
    std::vector<long long> h_trace;
    std::vector<RTask> order;
    // task queues (one per XCD by default)
    int queues = 8;
    int nq = 1;
    std::vector<int64_t> qoff;
    int64_t *d_qoff = nullptr;
    // HIP graph of the round (uploads, counter clearing, the kernel, result
    // copies), captured once per arena when graph_on
    bool graph_on = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
};

namespace {

size_t up256(size_t b) { return (b + 255) / 256 * 256; }

void drop_graph(RoundExec *r)
{
    if (r->gexec)
        (void)hipGraphExecDestroy(r->gexec);
    if (r->graph)
        (void)hipGraphDestroy(r->graph);
    r->gexec = nullptr;
    r->graph = nullptr;
}

void free_arena(RoundExec *r)
{
    drop_graph(r);
    if (r->arena)
        (void)hipFree(r->arena);
    if (r->d_tasks)
        (void)hipFree(r->d_tasks);
    if (r->d_trace)
        (void)hipFree(r->d_trace);
    r->d_trace = nullptr;
    r->d_qoff = nullptr; // inside the task allocation
    r->h_trace.clear();
    if (r->h_tab)
        (void)hipHostFree(r->h_tab);
    if (r->h_fields)
        (void)hipHostFree(r->h_fields);
    if (r->h_out)
        (void)hipHostFree(r->h_out);
    if (r->h_cnt)
        (void)hipHostFree(r->h_cnt);
    r->arena = nullptr;
    r->d_tasks = nullptr;
    r->h_tab = nullptr;
    r->h_fields = nullptr;
    r->h_out = nullptr;
    r->h_cnt = nullptr;
    r->version = ~(uint64_t)0;
    r->bt = 0;
    r->nf = 0;
    r->ntasks = 0;
}

#define RCHK(expr)                                                                                 \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) {                                                                    \
            if (err)                                                                               \
                *err = std::string("round: " #expr ": ") + hipGetErrorString(e_);                  \
            return FBT_EDEVICE;                                                                    \
        }                                                                                          \
    } while (0)

template <int BT> int round_occupancy()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_round<BT>, rthreads(BT), 0) !=
        hipSuccess)
        return 0;
    return nb;
}

fbt_status build(RoundExec *r, int bt, int nf, const int64_t *n, const double *const *locs,
                 const double *const *z, const int32_t *mode, uint64_t version, std::string *err)
{
    free_arena(r);
    std::vector<RPlanField> pf(nf);
    std::vector<size_t> off_field(nf, 0);
    size_t bytes = 0;
    const size_t tab_off = bytes;
    bytes = up256(bytes + (size_t)nf * TAB_BYTES);
    const size_t fields_off = bytes;
    bytes = up256(bytes + (size_t)nf * sizeof(RField));
    const size_t out_off = bytes;
    bytes = up256(bytes + (size_t)nf * 16 * sizeof(double));
    r->cnt_off.assign(nf, 0);
    size_t ci = 0;
    for (int f = 0; f < nf; ++f) {
        const int m = (mode[f] == 1 || mode[f] == 2) ? mode[f] : 0;
        const int T = (int)((n[f] + 1 + bt - 1) / bt);
        pf[f] = {n[f], T, m};
        r->cnt_off[f] = (int64_t)ci;
        if (m)
            ci += rcount(T).size;
    }
    r->cnt_ints = ci + R_CTL_WORDS;
    const size_t cnt_off = bytes;
    bytes = up256(bytes + r->cnt_ints * sizeof(int));
    for (int f = 0; f < nf; ++f) {
        if (!pf[f].mode)
            continue;
        const size_t T = pf[f].T, np = T * bt;
        off_field[f] = bytes;
        bytes = up256(bytes + np * np * 8);                               // A
        bytes = up256(bytes + (pf[f].mode == 2 ? 2 * np * np * 8 : 0));   // S
        bytes = up256(bytes + T * bt * bt * 8);                           // Linv
        bytes = up256(bytes + (size_t)rpart((int)T).size * 8);            // part
        bytes = up256(bytes + 3 * np * 8);                                // x, y, z
    }
    hipError_t e = hipMalloc((void **)&r->arena, bytes);
    if (e != hipSuccess) {
        r->arena = nullptr;
        if (err)
            *err = "round: device memory for the fields (" + std::to_string(bytes >> 20) +
                   " MiB): " + hipGetErrorString(e);
        return FBT_ENOMEM;
    }
    RCHK(hipHostMalloc((void **)&r->h_tab, (size_t)std::max(nf, 1) * TAB_BYTES, 0));
    RCHK(hipHostMalloc((void **)&r->h_fields, (size_t)std::max(nf, 1) * sizeof(RField), 0));
    RCHK(hipHostMalloc((void **)&r->h_out, (size_t)std::max(nf, 1) * 16 * sizeof(double), 0));
    RCHK(hipHostMalloc((void **)&r->h_cnt, r->cnt_ints * sizeof(int), 0));
    r->d_tab = r->arena + tab_off;
    r->d_fields = reinterpret_cast<RField *>(r->arena + fields_off);
    r->d_out = reinterpret_cast<double *>(r->arena + out_off);
    r->d_cnt = reinterpret_cast<int *>(r->arena + cnt_off);
    r->hfield.assign(nf, RField());
    std::vector<double> xyz;
    for (int f = 0; f < nf; ++f) {
        RField &F = r->hfield[f];
        std::memset(&F, 0, sizeof(F));
        if (!pf[f].mode)
            continue;
        const size_t T = pf[f].T, np = T * bt;
        char *p = r->arena + off_field[f];
        F.A = reinterpret_cast<double *>(p);
        p += up256(np * np * 8);
        F.S = pf[f].mode == 2 ? reinterpret_cast<double *>(p) : nullptr;
        p += up256(pf[f].mode == 2 ? 2 * np * np * 8 : 0);
        F.Linv = reinterpret_cast<double *>(p);
        p += up256(T * bt * bt * 8);
        F.part = reinterpret_cast<double *>(p);
        p += up256((size_t)rpart((int)T).size * 8);
        double *xd = reinterpret_cast<double *>(p);
        F.x = xd;
        F.y = xd + np;
        F.z = xd + 2 * np;
        F.out = r->d_out + 16 * f;
        F.cnt = r->d_cnt + r->cnt_off[f];
        F.n = n[f];
        F.ld = (int64_t)np;
        F.T = (int)T;
        F.mode = pf[f].mode;
        xyz.assign(3 * np, 0.0);
        for (int64_t i = 0; i < n[f]; ++i) {
            xyz[i] = locs[f][2 * i];
            xyz[np + i] = locs[f][2 * i + 1];
            xyz[2 * np + i] = z[f][i];
        }
        RCHK(hipMemcpy(xd, xyz.data(), 3 * np * 8, hipMemcpyHostToDevice));
    }
    // plan for the workgroups that fit at once
    hipDeviceProp_t prop;
    RCHK(hipGetDeviceProperties(&prop, r->device));
    const int per_cu = bt == 64 ? round_occupancy<64>() : round_occupancy<128>();
    if (per_cu < 1) {
        if (err)
            *err = "round: the kernel does not fit on a compute unit";
        return FBT_EDEVICE;
    }
    const int slots = per_cu * prop.multiProcessorCount;
    std::string perr;
    const int nq = (r->queues > 0 && slots % r->queues == 0) ? r->queues : 1;
    const RPlan plan = rplan_queues(pf, bt, slots, nq, &perr);
    if (!perr.empty()) {
        if (err)
            *err = perr;
        return FBT_EINVAL;
    }
    r->ntasks = (int)plan.order.size();
    r->order = plan.order;
    r->nq = nq;
    r->qoff = plan.qoff;
    r->est_us = plan.est_us;
    // every queue gets slots / nq workgroups (all resident at once)
    r->grid = slots;
    if (r->ntasks > 0) {
        RCHK(hipMalloc((void **)&r->d_tasks, plan.order.size() * sizeof(RTask) +
                                                 (nq + 1) * sizeof(int64_t)));
        RCHK(hipMemcpy(r->d_tasks, plan.order.data(), plan.order.size() * sizeof(RTask),
                       hipMemcpyHostToDevice));
        r->d_qoff = reinterpret_cast<int64_t *>(r->d_tasks + plan.order.size());
        RCHK(hipMemcpy(r->d_qoff, plan.qoff.data(), (nq + 1) * sizeof(int64_t),
                       hipMemcpyHostToDevice));
    }
    r->bt = bt;
    r->nf = nf;
    r->version = version;
    r->modes.assign(nf, 0);
    r->n.assign(n, n + nf);
    for (int f = 0; f < nf; ++f)
        r->modes[f] = pf[f].mode;
    return FBT_OK;
}

} // namespace

// The device work of one round on r->stream: theta tables and field
// descriptors up, counters cleared, the kernel (between r->e0 and r->e1 with
// timing), results and counters down.  No allocation and no host wait, so it
// can be captured.
static hipError_t round_enqueue(RoundExec *r, int bt, int nf, long long *trace, bool timing)
{
    hipError_t e;
    if ((e = hipMemcpyAsync(r->d_tab, r->h_tab, (size_t)nf * TAB_BYTES, hipMemcpyHostToDevice,
                            r->stream)) != hipSuccess)
        return e;
    if ((e = hipMemcpyAsync(r->d_fields, r->h_fields, (size_t)nf * sizeof(RField),
                            hipMemcpyHostToDevice, r->stream)) != hipSuccess)
        return e;
    const int64_t nz = (int64_t)r->cnt_ints;
    hipLaunchKernelGGL(k_zero_ints, dim3((unsigned)std::min<int64_t>(1024, (nz + 255) / 256)),
                       dim3(256), 0, r->stream, r->d_cnt, nz);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    int *ctl = r->d_cnt + (r->cnt_ints - R_CTL_WORDS);
    const int64_t limit = (int64_t)5000 * r->tick_khz; // 5 s of waiting for one counter
    if (timing && (e = hipEventRecord(r->e0, r->stream)) != hipSuccess)
        return e;
    if (bt == 64)
        hipLaunchKernelGGL(k_round<64>, dim3(r->grid), dim3(rthreads(64)), 0, r->stream,
                           r->d_fields, r->d_tasks, r->d_qoff, r->nq, ctl, limit, trace);
    else
        hipLaunchKernelGGL(k_round<128>, dim3(r->grid), dim3(rthreads(128)), 0, r->stream,
                           r->d_fields, r->d_tasks, r->d_qoff, r->nq, ctl, limit, trace);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    if (timing && (e = hipEventRecord(r->e1, r->stream)) != hipSuccess)
        return e;
    if ((e = hipMemcpyAsync(r->h_out, r->d_out, (size_t)nf * 16 * sizeof(double),
                            hipMemcpyDeviceToHost, r->stream)) != hipSuccess)
        return e;
    return hipMemcpyAsync(r->h_cnt, r->d_cnt, r->cnt_ints * sizeof(int), hipMemcpyDeviceToHost,
                          r->stream);
}

void round_set_graph(RoundExec *r, bool on)
{
    if (r)
        r->graph_on = on;
}

RoundExec *round_create(int device)
{
    RoundExec *r = new RoundExec();
    r->device = device;
    if (hipSetDevice(device) != hipSuccess || hipStreamCreate(&r->stream) != hipSuccess ||
        hipEventCreate(&r->e0) != hipSuccess || hipEventCreate(&r->e1) != hipSuccess) {
        round_destroy(r);
        return nullptr;
    }
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess &&
        khz > 0)
        r->tick_khz = khz;
    return r;
}

void round_destroy(RoundExec *r)
{
    if (!r)
        return;
    (void)hipSetDevice(r->device);
    if (r->stream)
        (void)hipStreamSynchronize(r->stream);
    free_arena(r);
    if (r->e0)
        (void)hipEventDestroy(r->e0);
    if (r->e1)
        (void)hipEventDestroy(r->e1);
    if (r->stream)
        (void)hipStreamDestroy(r->stream);
    delete r;
}

float round_last_ms(const RoundExec *r) { return r ? r->last_ms : 0.0f; }

void round_set_queues(RoundExec *r, int queues)
{
    if (r && queues != r->queues) {
        r->queues = queues;
        r->version = ~(uint64_t)0; // new plan at the next call
    }
}

int round_queues(const RoundExec *r) { return r ? r->queues : 0; }

void round_set_trace(RoundExec *r, bool on)
{
    if (r)
        r->trace_on = on;
}

int64_t round_trace(const RoundExec *r, int64_t *out, int64_t cap)
{
    if (!r || r->h_trace.empty())
        return 0;
    const int64_t n = (int64_t)r->order.size();
    for (int64_t q = 0; q < n && q < cap; ++q) {
        out[5 * q] = r->order[q].ft;
        out[5 * q + 1] = r->order[q].ij;
        for (int k = 0; k < 3; ++k)
            out[5 * q + 2 + k] = r->h_trace[3 * q + k];
    }
    return n;
}
double round_plan_estimate_us(const RoundExec *r) { return r ? r->est_us : 0.0; }
int round_task_count(const RoundExec *r) { return r ? r->ntasks : 0; }

fbt_status round_eval(RoundExec *r, int bt, int nf, const int64_t *n, const double *const *locs,
                      const double *const *z, uint64_t version, const double *thetas,
                      const int32_t *mode, double *loglik, double *score, double *fisher,
                      int32_t *status, std::string *err)
{
    if (!r || (bt != 64 && bt != 128) || nf < 0)
        return FBT_EINVAL;
    if (hipSetDevice(r->device) != hipSuccess) {
        if (err)
            *err = "round: hipSetDevice failed";
        return FBT_EDEVICE;
    }
    bool same = r->arena && r->bt == bt && r->version == version && r->nf == nf;
    for (int f = 0; same && f < nf; ++f)
        same = r->modes[f] == ((mode[f] == 1 || mode[f] == 2) ? mode[f] : 0);
    if (!same) {
        const fbt_status st = build(r, bt, nf, n, locs, z, mode, version, err);
        if (st != FBT_OK) {
            free_arena(r);
            return st;
        }
    }
    if (r->ntasks == 0)
        return FBT_OK;
    for (int f = 0; f < nf; ++f) {
        RField &F = r->h_fields[f];
        F = r->hfield[f];
        if (!F.mode)
            continue;
        const double *th = thetas + 3 * f;
        const bool ok = std::isfinite(th[0]) && std::isfinite(th[1]) && std::isfinite(th[2]) &&
                        th[0] > 0 && th[1] > 0 && th[2] > 0;
        if (!ok) {
            F.skip = 1;
            status[f] = FBT_EINVAL;
            continue;
        }
        F.gp = theta_params(th, 0, F.n, F.ld, F.ld, r->h_tab + (size_t)f * TAB_BYTES,
                            r->d_tab + (size_t)f * TAB_BYTES);
    }
    if (r->trace_on && !r->d_trace)
        RCHK(hipMalloc((void **)&r->d_trace, (size_t)r->ntasks * 3 * sizeof(long long)));
    long long *trace = r->trace_on ? r->d_trace : nullptr;
    if (r->graph_on && !trace) {
        if (!r->gexec) {
            // the round's work on the stream, captured once per arena: the
            // copies read the pinned staging buffers at every replay
            RCHK(hipStreamBeginCapture(r->stream, hipStreamCaptureModeThreadLocal));
            const hipError_t e = round_enqueue(r, bt, nf, nullptr, false);
            hipGraph_t g = nullptr;
            const hipError_t e2 = hipStreamEndCapture(r->stream, &g);
            r->graph = g;
            RCHK(e);
            RCHK(e2);
            RCHK(hipGraphInstantiate(&r->gexec, r->graph, nullptr, nullptr, 0));
        }
        RCHK(hipEventRecord(r->e0, r->stream));
        RCHK(hipGraphLaunch(r->gexec, r->stream));
        RCHK(hipEventRecord(r->e1, r->stream));
    } else {
        RCHK(round_enqueue(r, bt, nf, trace, true));
    }
    if (trace) {
        r->h_trace.resize((size_t)r->ntasks * 3);
        RCHK(hipMemcpyAsync(r->h_trace.data(), trace, r->h_trace.size() * sizeof(long long),
                            hipMemcpyDeviceToHost, r->stream));
    }
    RCHK(hipStreamSynchronize(r->stream));
    RCHK(hipEventElapsedTime(&r->last_ms, r->e0, r->e1));
    const int *hctl = r->h_cnt + (r->cnt_ints - R_CTL_WORDS);
    bool drained = hctl[1] == 0;
    for (int q = 0; q < r->nq; ++q)
        drained = drained && hctl[RQ_CTL + RQ_STRIDE * q] >= r->qoff[q + 1] - r->qoff[q];
    if (!drained) {
        if (err)
            *err = "round: a dependency wait of the persistent kernel ran out of time";
        return FBT_EDEVICE;
    }
    for (int f = 0; f < nf; ++f) {
        const RField &F = r->h_fields[f];
        if (!F.mode || F.skip)
            continue;
        const int info = r->h_cnt[r->cnt_off[f] + rcount(F.T).info];
        if (info != 0) {
            status[f] = FBT_ENOTPD;
            continue;
        }
        const double *t = r->h_out + 16 * f;
        bool finite = true;
        for (int k = 0; k < (F.mode == 2 ? 9 : 2); ++k)
            finite = finite && std::isfinite(t[k]);
        if (!finite) {
            status[f] = FBT_ENONFINITE;
            continue;
        }
        if (F.mode == 1)
            loglik[f] = loglik_terms(F.n, t[0], t[1]);
        else
            assemble_terms(F.n, thetas + 3 * f, t, loglik + f, score + 3 * f, fisher + 9 * f);
        status[f] = FBT_OK;
    }
    return FBT_OK;
}

} // namespace fbt
