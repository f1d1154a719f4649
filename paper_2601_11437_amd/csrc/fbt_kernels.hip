// HIP kernels for gfx950 (MI355X): Matern covariance generation, tiled FP64
// Cholesky, the two triangular solves that form W_i = L^{-1} Sigma_i L^{-T},
// and the trace reductions of the score and Fisher information.
//
// Storage: every matrix is column-major with leading dimension ld and padded
// order npad = NB * ceil((n + 1) / NB).  Row/column n of Sigma' carries the
// observations (Sigma'[n][j] = Z_j for j < n), so the factorisation of the
// bordered matrix returns y = L^{-1} Z in row n of the factor; all rows and
// columns beyond n are identity (Sigma') or zero (Sigma_alpha', Sigma_nu').
// The padded problem has exactly the same log-determinant, quadratic form,
// traces and Frobenius products as the n x n one, and needs no ragged tiles.
#include "fbt_internal.h"
#include "fbt_device.h"

#include <math.h>
#include <type_traits>

namespace fbt {

constexpr int GT = 64; // generation tile (rows x cols)

__global__ __launch_bounds__(256) void k_gen(GenParams gp1, const GenParams *__restrict__ gpa,
                                             Fields F, const double *__restrict__ xs,
                                             const double *__restrict__ ys,
                                             const double *__restrict__ z, double *__restrict__ S,
                                             double *__restrict__ Sa, double *__restrict__ Sn,
                                             int mode)
{
    __shared__ Node tab[TAB_MAX];
    const int f = blockIdx.y; // field
    const GenParams gp = gpa ? gpa[f] : gp1;
    const Node *__restrict__ gtab = gp.tab;
    xs += f * F.sVec;
    ys += f * F.sVec;
    z += f * F.sVec;
    S += f * F.sA;
    Sa += f * F.sS2;
    Sn += f * F.sS2;
    const int t = threadIdx.x;
    const int ntab = gp.off[NLEV - 1] + gp.len[NLEV - 1];
    for (int i = t; i < ntab; i += 256)
        tab[i] = gtab[i];
    // tile pair (ti >= tj) from the linear block index
    const int64_t p = blockIdx.x;
    int64_t ti = (int64_t)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= p)
        ++ti;
    while (ti * (ti + 1) / 2 > p)
        --ti;
    const int64_t tj = p - ti * (ti + 1) / 2;
    const bool diag = (ti == tj);
    const int al = t & 63;
    const int64_t a = ti * GT + al;
    const int64_t n = gp.n, ld = gp.ld;
    const double xa = a < n ? xs[a] : 0.0, ya = a < n ? ys[a] : 0.0;
    const double inv_alpha = 1.0 / gp.alpha;
    __syncthreads();

#pragma unroll 1
    for (int e = 0; e < 16; ++e) {
        const int bl = (t >> 6) * 16 + e;
        const int64_t b = tj * GT + bl;
        if (diag && al < bl)
            continue;
        double c = 0.0, ca = 0.0, cn = 0.0;
        if (a < n) {
            const double dx = xa - xs[b], dy = ya - ys[b];
            matern3(gp, tab, sqrt(dx * dx + dy * dy) * inv_alpha, mode, c, ca, cn);
        } else if (a == n) {
            c = (b < n) ? z[b] : 1.0;
        } else {
            c = (a == b) ? 1.0 : 0.0;
        }
        if (mode & GEN_SIGMA)
            S[a + b * ld] = c;
        if (mode & GEN_DERIV) {
            // full symmetric storage: the entry and its mirror.  The mirrored
            // stores are strided, but the kernel is bound by the quadrature
            // arithmetic (hundreds of instructions per entry), not by stores.
            Sa[a + b * ld] = ca;
            Sn[a + b * ld] = cn;
            if (a != b) {
                Sa[b + a * ld] = ca;
                Sn[b + a * ld] = cn;
            }
        }
    }
}

void launch_gen(hipStream_t s, const GenParams &gp, const GenParams *gpa, const Fields &F,
                const double *xs, const double *ys, const double *z, double *S, double *Sa,
                double *Sn, int mode)
{
    const int64_t nt = gp.npad / GT;
    const int64_t pairs = nt * (nt + 1) / 2;
    hipLaunchKernelGGL(k_gen, dim3((unsigned)pairs, F.count), dim3(256), 0, s, gp,
                       F.n ? gpa : nullptr, F, xs, ys, z, S, Sa, Sn, mode);
}

// ---------------------------------------------------------------------------
// Diagonal block: Cholesky factor L_kk (in place) and its inverse Linv_k, by
// one workgroup of 512 threads over 32-column panels p = 0..7 (jb = 32 p).
// Per panel:
//  A. the panel's 32 x 32 top block T = L_t L_t^T is factored by wave 0 and
//     D_p = L_t^{-1} formed by wave 1 a column or two behind it, both in
//     registers with one row per lane (columns of L_t go through LDS,
//     published to wave 1 in pairs by a counter).  At the same time waves 2..7 finish the previous
//     panel's updates: trailing tiles outside the next two tile columns, and
//     the inverse rows below it, B_i -= Lp[i] X_{p-1};
//  B. L_t and D_p are stored; the rows below the top block L_b = A_b D_p^T
//     and the inverse block row X_p = D_p [B_p | I] (B_p: block row p of
//     Linv as updated by the earlier panels) are formed on MFMA;
//  C. X_p goes to Linv, and the trailing tiles of the next two tile columns
//     (the next panel, whose top block also lands in LDS) are updated with
//     L_b on MFMA, so the next panel's top block is ready for step A.
// MFMA operands come from LDS (Lp, D_p, X_p) or, for L_b, from the block
// itself; C tiles stay in L2 and are loaded in batches of four 16 x 16 tiles
// per wave.  Linv starts at zero, so its strict upper part is exactly zero.
// Pivot rule: rows g >= n (the observation border and the identity padding)
// take pivot 1; a pivot <= 0 or NaN at g < n records min(g) in *info and
// continues with pivot 1 so that nothing downstream becomes non-finite.
// logdet_part[k] = sum of log(pivot) over rows g < n of the block.
// ---------------------------------------------------------------------------
constexpr int PW = 32;
constexpr int LPS = PW + 1; // LDS row stride of the panel, the top block and D_p
constexpr int XPS = NB + 1; // LDS row stride of X_p (PW x NB)
constexpr int DT = 512;     // threads of the diagonal kernel
constexpr int NWD = DT / 64;

// value of v in lane l (l wave-uniform) as a scalar
__device__ __forceinline__ double lane_value(double v, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// row and column of the u-th tile of a lower triangle of tiles (row-major order)
__device__ __forceinline__ void tri_tile(int u, int *ti, int *tj)
{
    int i = (int)((sqrt(8.0 * u + 1.0) - 1.0) * 0.5);
    while ((i + 1) * (i + 2) / 2 <= u)
        ++i;
    while (i * (i + 1) / 2 > u)
        --i;
    *ti = i;
    *tj = u - i * (i + 1) / 2;
}

// C -= L_b[ia..] X^T over 16 x 16 tiles, four per wave at a time.  map(u,
// ...) returns the C tile pointer of unit u and sets ia (its first row within
// the panel), jbk (its first column: a row of Lp, or a column of X_p when
// inv) and ldc; with tb, the tiles of the next panel's top block are also
// written to tb.
template <class Map>
__device__ __forceinline__ void tile_update(int nu, int wv, int nw, int lane, const double *Lp,
                                            const double *Xp, double *tb, Map map)
{
    for (int u0 = wv * 4; u0 < nu; u0 += nw * 4) {
        d4 acc[4];
        double *cp[4];
        int ia[4], jbk[4];
        int64_t ldc[4];
        bool inv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            cp[q] = (u0 + q < nu) ? map(u0 + q, &ia[q], &jbk[q], &ldc[q], &inv[q]) : nullptr;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (cp[q]) {
#pragma unroll
                for (int rr = 0; rr < 4; ++rr)
                    acc[q][rr] = cp[q][(lane & 15) + (int64_t)((lane >> 4) + 4 * rr) * ldc[q]];
            }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (cp[q]) {
#pragma unroll
                for (int s4 = 0; s4 < PW / 4; ++s4) {
                    const int k = 4 * s4 + (lane >> 4);
                    const double a = -Lp[(ia[q] + (lane & 15)) * LPS + k];
                    const double b = inv[q] ? Xp[k * XPS + jbk[q] + (lane & 15)]
                                            : Lp[(jbk[q] + (lane & 15)) * LPS + k];
                    acc[q] = mfma(b, a, acc[q]);
                }
            }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (cp[q]) {
#pragma unroll
                for (int rr = 0; rr < 4; ++rr)
                    cp[q][(lane & 15) + (int64_t)((lane >> 4) + 4 * rr) * ldc[q]] = acc[q][rr];
                // the next panel's top block: trailing rows / columns 0..31
                if (tb && !inv[q] && ia[q] < 2 * PW && jbk[q] < 2 * PW) {
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr)
                        tb[(ia[q] - PW + (lane & 15)) * LPS + jbk[q] - PW + (lane >> 4) + 4 * rr] =
                            acc[q][rr];
                }
            }
    }
}

__global__ __launch_bounds__(DT) void k_potrf_diag(Fields F, double *__restrict__ A, int64_t lda,
                                                   int kblk, int64_t n1, double *__restrict__ Linv,
                                                   double *__restrict__ logdet_part,
                                                   int *__restrict__ info)
{
    const int f = blockIdx.x; // field
    A += f * F.sA;
    Linv += f * F.sLinv;
    logdet_part += f * F.sLog;
    info += f;
    const int64_t n = F.n ? F.n[f] : n1;
    __shared__ double Lp[NB * LPS];   // the panel: L_t in rows 0..31, L_b below
    __shared__ double Xp[PW * XPS];   // X_p
    __shared__ double Tb[PW * LPS];   // top block of the panel -> L_t
    __shared__ double Db[PW * LPS];   // D_p (strict upper part stays zero)
    __shared__ double colb[PW * PW];  // column c of L_t at colb[c PW + i]
    __shared__ double piv[NB];
    __shared__ double sh[NWD];
    __shared__ double ipv[PW];        // 1 / pivot of each column of L_t
    __shared__ int colready;          // columns of L_t published by wave 0
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t o = (int64_t)kblk * NB;
    double *Ab = A + o + o * lda;

    for (int idx = t; idx < NB * NB; idx += DT)
        Linv[idx] = 0.0;
    for (int idx = t; idx < PW * PW; idx += DT) {
        const int row = idx % PW, col = idx / PW;
        Tb[row * LPS + col] = Ab[row + (int64_t)col * lda];
        Db[row * LPS + col] = 0.0;
    }
    if (t == 0)
        colready = 0;
    __syncthreads();

    for (int p = 0; p < NB / PW; ++p) {
        const int jb = p * PW, M = NB - jb;
        const int nt = (M - PW) / 16; // 16-row tiles below the panel's top block
        // ---- A. top block of panel p ‖ the rest of panel p - 1's updates ----
        if (wave == 0) {
            int i = lane & 31;
            // fresh per panel: keeps the lane masks below from being hoisted
            // out of the panel loop (they would not fit in scalar registers)
            asm volatile("" : "+v"(i));
            double r[PW];
            // whole rows: entries above the diagonal are never used (rows
            // above c are cleared at step c before anything reads them)
#pragma unroll
            for (int c = 0; c < PW; ++c)
                r[c] = Tb[i * LPS + c];
            int firstbad = 0x7fffffff; // wave-uniform
#pragma unroll
            for (int c = 0; c < PW; ++c) {
                const double d = lane_value(r[c], c);
                const int g = (int)(o + jb + c);
                const bool bad = (g < n) && !(d > 0.0); // the same in every lane
                const bool one = g >= n || bad;
                const double ip = one ? 1.0 : rsqrt(d);
                const double pv = one ? 1.0 : d * ip;
                firstbad = (bad && firstbad == 0x7fffffff) ? g : firstbad;
                r[c] = (i > c) ? r[c] * ip : (i == c ? pv : 0.0);
                // column c and 1 / pivot to wave 1
                if (lane < PW)
                    colb[c * PW + i] = r[c];
                if (lane == 0)
                    ipv[c] = ip;
#pragma unroll
                for (int j = c + 1; j < PW; ++j) {
                    r[j] -= r[c] * lane_value(r[c], j);
                    asm volatile("" : "+v"(r[j])); // update in place: no broadcast outlives its use
                }
                // columns are published in pairs, after the row updates: the
                // stores above complete behind the updates instead of stalling
                // the column chain at the fence
                if ((c & 1) || c == PW - 1) {
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                    if (lane == 0)
                        __hip_atomic_store(&colready, c + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            }
            if (lane == 0 && firstbad != 0x7fffffff)
                atomicMin(info, firstbad);
            if (lane < PW) {
#pragma unroll
                for (int c = 0; c < PW; ++c)
                    Tb[i * LPS + c] = r[c];
            }
        } else if (wave == 1) {
            // D_p = L_t^{-1} by forward elimination, one column of L_t behind
            // wave 0: row m is final once divided by its pivot, then it is
            // removed from the rows below it (broadcast by readlane)
            int i = lane & 31;
            asm volatile("" : "+v"(i));
            double x[PW], myip = 1.0;
#pragma unroll
            for (int k = 0; k < PW; ++k)
                x[k] = (k == i) ? 1.0 : 0.0;
#pragma unroll
            for (int m = 0; m < PW; ++m) {
                while (__hip_atomic_load(&colready, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) <= m)
                    __builtin_amdgcn_s_sleep(1);
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                const double ipm = ipv[m];
                const double lim = (i > m) ? colb[m * PW + i] : 0.0;
                myip = (i == m) ? ipm : myip;
#pragma unroll
                for (int k = 0; k <= m; ++k) {
                    x[k] -= lim * (lane_value(x[k], m) * ipm);
                    asm volatile("" : "+v"(x[k]));
                }
            }
            // row i of D_p: the eliminated row divided by its pivot
            asm volatile("" : "+v"(i));
            if (lane < PW) {
#pragma unroll
                for (int k = 0; k < PW; ++k)
                    if (k <= i)
                        Db[i * LPS + k] = x[k] * myip;
            }
        } else if (p > 0) {
            // panel p - 1: trailing tiles in tile columns >= 2 of its trailing
            // block, then the inverse rows below it
            const int jq = jb - PW, ntq = nt + 2;
            const int nr = (ntq - 2) * (ntq - 1) / 2, nc6 = jb / 16;
            tile_update(nr + ntq * nc6, wave - 2, NWD - 2, lane, Lp, Xp, nullptr,
                        [&](int u, int *ia, int *jbk, int64_t *ldc, bool *inv) -> double * {
                            if (u < nr) {
                                int i, j;
                                tri_tile(u, &i, &j);
                                *ia = PW + 16 * (i + 2);
                                *jbk = PW + 16 * (j + 2);
                                *ldc = lda;
                                *inv = false;
                                return Ab + (jq + *ia) + (int64_t)(jq + *jbk) * lda;
                            }
                            const int v = u - nr;
                            *ia = PW + 16 * (v % ntq);
                            *jbk = 16 * (v / ntq);
                            *ldc = NB;
                            *inv = true;
                            return Linv + (jq + *ia) + (int64_t)*jbk * NB;
                        });
        }
        __syncthreads();
        // ---- B. store L_t and D_p; L_b = A_b D_p^T; X_p[:, 0:jb] = D_p B_p ----
        if (t == 0)
            colready = 0;
        for (int idx = t; idx < PW * PW; idx += DT) {
            const int row = idx % PW, col = idx / PW;
            const double lv = Tb[row * LPS + col], dv = Db[row * LPS + col];
            Lp[row * LPS + col] = lv;
            Xp[row * XPS + jb + col] = dv;
            if (col <= row) {
                Ab[(jb + row) + (int64_t)(jb + col) * lda] = lv;
                Linv[(jb + row) + (int64_t)(jb + col) * NB] = dv;
            }
            if (row == col)
                piv[jb + row] = lv;
        }
        // one unit per 16-row tile of L_b (both column halves: the unit
        // overwrites the A_b rows it reads), then the tiles of X_p
        for (int u = wave; u < nt + 2 * (jb / 16); u += NWD) {
            d4 acc = {0, 0, 0, 0};
            if (u < nt) {
                d4 acc1 = {0, 0, 0, 0};
                const double *Arow = Ab + (jb + PW + 16 * u + (lane & 15)) + (int64_t)jb * lda;
#pragma unroll
                for (int s4 = 0; s4 < PW / 4; ++s4) {
                    const int k = 4 * s4 + (lane >> 4);
                    const double a = Arow[(int64_t)k * lda];
                    acc = mfma(Db[(lane & 15) * LPS + k], a, acc);
                    acc1 = mfma(Db[(16 + (lane & 15)) * LPS + k], a, acc1);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int R = PW + 16 * u + (lane & 15), C = (lane >> 4) + 4 * q;
                    Lp[R * LPS + C] = acc[q];
                    Lp[R * LPS + C + 16] = acc1[q];
                    Ab[(jb + R) + (int64_t)(jb + C) * lda] = acc[q];
                    Ab[(jb + R) + (int64_t)(jb + C + 16) * lda] = acc1[q];
                }
            } else {
                const int v = u - nt, ti = v & 1, tj = v >> 1;
#pragma unroll
                for (int s4 = 0; s4 < PW / 4; ++s4) {
                    const int k = 4 * s4 + (lane >> 4);
                    const double a = Db[(16 * ti + (lane & 15)) * LPS + k];
                    const double b = Linv[(jb + k) + (int64_t)(16 * tj + (lane & 15)) * NB];
                    acc = mfma(b, a, acc);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    Xp[(16 * ti + (lane & 15)) * XPS + 16 * tj + (lane >> 4) + 4 * q] = acc[q];
            }
        }
        __syncthreads();
        // ---- C. X_p to Linv; the next panel's two tile columns ----
        for (int idx = t; idx < PW * jb; idx += DT) {
            const int row = idx % PW, col = idx / PW;
            Linv[(jb + row) + (int64_t)col * NB] = Xp[row * XPS + col];
        }
        if (nt > 0)
            tile_update(2 * nt - 1, wave, NWD, lane, Lp, Xp, Tb,
                        [&](int u, int *ia, int *jbk, int64_t *ldc, bool *inv) -> double * {
                            const int j = u < nt ? 0 : 1, i = u < nt ? u : u - nt + 1;
                            *ia = PW + 16 * i;
                            *jbk = PW + 16 * j;
                            *ldc = lda;
                            *inv = false;
                            return Ab + (jb + *ia) + (int64_t)(jb + *jbk) * lda;
                        });
        __syncthreads();
    }
    // log-determinant of the block: fixed-order tree over the NB pivots
    double lg = (t < NB && o + t < n) ? log(piv[t]) : 0.0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        lg += __shfl_xor(lg, off, 64);
    if (lane == 0)
        sh[wave] = lg;
    __syncthreads();
    if (t == 0) {
        double s = 0.0;
        for (int w = 0; w < NWD; ++w)
            s += sh[w];
        logdet_part[kblk] = s;
    }
}

__global__ __launch_bounds__(256) void k_init_info(int *info, int count)
{
    const int f = blockIdx.x * 256 + threadIdx.x;
    if (f < count)
        info[f] = 0x7fffffff;
}

void launch_init_info(hipStream_t s, int *info, int count)
{
    hipLaunchKernelGGL(k_init_info, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, info,
                       count);
}

// one workgroup per field
void launch_potrf_diag(hipStream_t s, const Fields &F, double *A, int64_t lda, int k, int64_t n,
                       double *Linv, double *logdet_part, int *info)
{
    hipLaunchKernelGGL(k_potrf_diag, dim3((unsigned)F.count), dim3(DT), 0, s, F, A, lda, k, n,
                       Linv, logdet_part, info);
}

// Workgroups are dealt to MI355X's 8 XCDs round-robin by linear index, and
// each XCD has its own L2.  xcd_tile renumbers a launch's tiles so that each
// XCD takes a contiguous range of them: tiles that share operand panels
// (neighbours in the tile order) then meet in one L2.  A bijection on
// [0, total) for any total.
constexpr int NXCD = 8;
__device__ __forceinline__ int64_t xcd_tile(int64_t bid, int64_t total)
{
    const int64_t x = bid % NXCD, i = bid / NXCD, q = total / NXCD, r = total % NXCD;
    return x * q + (x < r ? x : r) + i;
}

// ---------------------------------------------------------------------------
// FP64 MFMA tile engine.  A workgroup of 4 waves computes a (64 WM) x (64 WN)
// tile of A * B^T, each wave a 64 x 64 block held as 4 x 4 MFMA accumulators.
// A is M-contiguous (element (m, k) at A[m + k lda]).  B is N-contiguous
// (element (n, k) at B[n + k ldb]) or, with BKC, K-contiguous (at B[k + n ldb]).
// With AKC, A is K-contiguous too (element (m, k) at A[k + m lda]).
// K is streamed in chunks of 16 through double-buffered LDS.  With the MFMA
// operands swapped (B fragment first), lane l holds in accumulator (i, j),
// element r, the tile entry (16 i + l % 16, 16 j + l / 16 + 4 r): 16
// consecutive rows per column, so stores are 128-byte segments.
// ---------------------------------------------------------------------------
template <int WM, int WN, bool BKC, bool NEG = false, bool AKC = false> struct Tile {
    static constexpr int BM = 64 * WM, BN = 64 * WN, KC = 16;
    static constexpr int LSA = BM + 4, LSB = BN + 4; // padded LDS rows (doubles)
    static constexpr int STAGE = KC * (LSA + LSB);
    static constexpr int LDS = 2 * STAGE;
    static constexpr int NA = BM * KC / 512; // double2 loads per thread
    static constexpr int NBL = BN * KC / 512;

    __device__ static void load(double2 *ra, double2 *rb, const double *A, int64_t lda,
                                const double *B, int64_t ldb, int k0)
    {
        const int t = threadIdx.x;
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int q = t + 256 * i;
            if (!AKC) {
                const int m2 = q % (BM / 2), k = q / (BM / 2);
                ra[i] = *(const double2 *)(A + 2 * m2 + (int64_t)(k0 + k) * lda);
            } else {
                const int k2 = q % (KC / 2), mm = q / (KC / 2);
                ra[i] = *(const double2 *)(A + (k0 + 2 * k2) + (int64_t)mm * lda);
            }
        }
#pragma unroll
        for (int i = 0; i < NBL; ++i) {
            const int q = t + 256 * i;
            if (!BKC) {
                const int n2 = q % (BN / 2), k = q / (BN / 2);
                rb[i] = *(const double2 *)(B + 2 * n2 + (int64_t)(k0 + k) * ldb);
            } else {
                const int k2 = q % (KC / 2), nn = q / (KC / 2);
                rb[i] = *(const double2 *)(B + (k0 + 2 * k2) + (int64_t)nn * ldb);
            }
        }
    }
    __device__ static void store(const double2 *ra, const double2 *rb, double *st)
    {
        const int t = threadIdx.x;
        double *As = st, *Bs = st + KC * LSA;
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int q = t + 256 * i;
            double2 v = ra[i];
            if (NEG) {
                v.x = -v.x;
                v.y = -v.y;
            }
            if (!AKC) {
                const int m2 = q % (BM / 2), k = q / (BM / 2);
                *(double2 *)(As + k * LSA + 2 * m2) = v;
            } else {
                const int k2 = q % (KC / 2), mm = q / (KC / 2);
                As[(2 * k2) * LSA + mm] = v.x;
                As[(2 * k2 + 1) * LSA + mm] = v.y;
            }
        }
#pragma unroll
        for (int i = 0; i < NBL; ++i) {
            const int q = t + 256 * i;
            if (!BKC) {
                const int n2 = q % (BN / 2), k = q / (BN / 2);
                *(double2 *)(Bs + k * LSB + 2 * n2) = rb[i];
            } else {
                const int k2 = q % (KC / 2), nn = q / (KC / 2);
                Bs[(2 * k2) * LSB + nn] = rb[i].x;
                Bs[(2 * k2 + 1) * LSB + nn] = rb[i].y;
            }
        }
    }
    __device__ static void compute(d4 (&acc)[4][4], const double *st, int wm, int wn, int lane)
    {
        const double *As = st + wm * 64 + (lane & 15);
        const double *Bs = st + KC * LSA + wn * 64 + (lane & 15);
#pragma unroll
        for (int s = 0; s < KC / 4; ++s) {
            const int kk = 4 * s + (lane >> 4);
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                a[i] = As[kk * LSA + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                b[j] = Bs[kk * LSB + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = mfma(b[j], a[i], acc[i][j]);
        }
    }
    // acc += (NEG ? -A : A)(BM x K) * B(BN x K)^T for the workgroup tile; K % 16 == 0.
    // A wave multiplies only the first `cmax` chunks of 16: callers whose operand is a
    // lower-triangular NB x NB block pass the chunks that can hold nonzeros for the wave's
    // rows (every chunk is still staged by the whole workgroup).
    __device__ static void run(d4 (&acc)[4][4], const double *A, int64_t lda, const double *B,
                               int64_t ldb, int K, double *lds, int cmax = 1 << 30)
    {
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const int wm = wave % WM, wn = wave / WM;
        double2 ra[NA], rb[NBL];
        load(ra, rb, A, lda, B, ldb, 0);
        store(ra, rb, lds);
        __syncthreads();
        const int nch = K / KC;
        for (int c = 0; c < nch; ++c) {
            if (c + 1 < nch)
                load(ra, rb, A, lda, B, ldb, (c + 1) * KC);
            if (c < cmax)
                compute(acc, lds + (c & 1) * STAGE, wm, wn, lane);
            if (c + 1 < nch)
                store(ra, rb, lds + ((c + 1) & 1) * STAGE);
            __syncthreads();
        }
    }
    __device__ static void zero(d4 (&acc)[4][4])
    {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = (d4){0, 0, 0, 0};
    }
    // acc = the C tile (column-major, ldc), for C -= A B^T run with NEG: the
    // accumulators start from C, so the epilogue only stores.
    __device__ static void load_c(d4 (&acc)[4][4], const double *C, int64_t ldc)
    {
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const int wm = wave % WM, wn = wave / WM;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    acc[i][j][r] = C[row(i, lane, wm) + (int64_t)col(j, r, lane, wn) * ldc];
    }
    __device__ static void store_c(const d4 (&acc)[4][4], double *C, int64_t ldc)
    {
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const int wm = wave % WM, wn = wave / WM;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    C[row(i, lane, wm) + (int64_t)col(j, r, lane, wn) * ldc] = acc[i][j][r];
    }
    // row / column of accumulator (i, j) element r inside the workgroup tile
    __device__ static int row(int i, int lane, int wm) { return wm * 64 + 16 * i + (lane & 15); }
    __device__ static int col(int j, int r, int lane, int wn) { return wn * 64 + 16 * j + (lane >> 4) + 4 * r; }
};

// FP32-compute variant for the mixed-precision form: FP64 operands are
// rounded to FP32 when staged into LDS, multiplied on v_mfma_f32_16x16x4_f32
// with FP32 accumulation, and the product is subtracted from the FP64 C tile.
// FP32 MFMA output layout: lane l holds D[4 (l/16) + r][l%16], so with the
// B fragment first lane l holds tile entry (16 i + l%16, 16 j + 4 (l/16) + r).
typedef float f4 __attribute__((ext_vector_type(4)));

template <int WM, int WN, bool BKC> struct TileF {
    static constexpr int BM = 64 * WM, BN = 64 * WN, KC = 16;
    static constexpr int LSA = BM + 8, LSB = BN + 8; // padded LDS rows (floats)
    static constexpr int STAGE = KC * (LSA + LSB);
    static constexpr int LDS = 2 * STAGE;            // floats
    static constexpr int NA = BM * KC / 512;          // double2 loads per thread
    static constexpr int NBL = BN * KC / 512;

    __device__ static void load(double2 *ra, double2 *rb, const double *A, int64_t lda,
                                const double *B, int64_t ldb, int k0)
    {
        const int t = threadIdx.x;
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int q = t + 256 * i, m2 = q % (BM / 2), k = q / (BM / 2);
            ra[i] = *(const double2 *)(A + 2 * m2 + (int64_t)(k0 + k) * lda);
        }
#pragma unroll
        for (int i = 0; i < NBL; ++i) {
            const int q = t + 256 * i;
            if (!BKC) {
                const int n2 = q % (BN / 2), k = q / (BN / 2);
                rb[i] = *(const double2 *)(B + 2 * n2 + (int64_t)(k0 + k) * ldb);
            } else {
                const int k2 = q % (KC / 2), nn = q / (KC / 2);
                rb[i] = *(const double2 *)(B + (k0 + 2 * k2) + (int64_t)nn * ldb);
            }
        }
    }
    __device__ static void store(const double2 *ra, const double2 *rb, float *st)
    {
        const int t = threadIdx.x;
        float *As = st, *Bs = st + KC * LSA;
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int q = t + 256 * i, m2 = q % (BM / 2), k = q / (BM / 2);
            *(float2 *)(As + k * LSA + 2 * m2) = make_float2((float)ra[i].x, (float)ra[i].y);
        }
#pragma unroll
        for (int i = 0; i < NBL; ++i) {
            const int q = t + 256 * i;
            if (!BKC) {
                const int n2 = q % (BN / 2), k = q / (BN / 2);
                *(float2 *)(Bs + k * LSB + 2 * n2) = make_float2((float)rb[i].x, (float)rb[i].y);
            } else {
                const int k2 = q % (KC / 2), nn = q / (KC / 2);
                Bs[(2 * k2) * LSB + nn] = (float)rb[i].x;
                Bs[(2 * k2 + 1) * LSB + nn] = (float)rb[i].y;
            }
        }
    }
    __device__ static void compute(f4 (&acc)[4][4], const float *st, int wm, int wn, int lane)
    {
        const float *As = st + wm * 64 + (lane & 15);
        const float *Bs = st + KC * LSA + wn * 64 + (lane & 15);
#pragma unroll
        for (int s = 0; s < KC / 4; ++s) {
            const int kk = 4 * s + (lane >> 4);
            float a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                a[i] = As[kk * LSA + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                b[j] = Bs[kk * LSB + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[j], a[i], acc[i][j], 0, 0, 0);
        }
    }
    // C(BM x BN, FP64) -= A(BM x K) * B(BN x K)^T computed in FP32; the FP32
    // sums cover NB-deep slices of K and each slice is added into C in FP64,
    // so the FP32 accumulation error does not grow with K beyond NB.
    __device__ __forceinline__ static void update(double *C, int64_t ldc, const double *A, int64_t lda,
                                  const double *B, int64_t ldb, int K, float *lds)
    {
#pragma unroll 1
        for (int k0 = 0; k0 < K; k0 += NB)
            update_slice(C, ldc, A + (int64_t)k0 * lda, lda, BKC ? B + k0 : B + (int64_t)k0 * ldb,
                         ldb, K - k0 < NB ? K - k0 : NB, lds);
    }
    __device__ __forceinline__ static void update_slice(double *C, int64_t ldc, const double *A,
                                                        int64_t lda, const double *B, int64_t ldb,
                                                        int K, float *lds)
    {
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const int wm = wave % WM, wn = wave / WM;
        f4 acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = (f4){0.f, 0.f, 0.f, 0.f};
        double2 ra[NA], rb[NBL];
        load(ra, rb, A, lda, B, ldb, 0);
        store(ra, rb, lds);
        __syncthreads();
        const int nch = K / KC;
        for (int c = 0; c < nch; ++c) {
            if (c + 1 < nch)
                load(ra, rb, A, lda, B, ldb, (c + 1) * KC);
            compute(acc, lds + (c & 1) * STAGE, wm, wn, lane);
            if (c + 1 < nch)
                store(ra, rb, lds + ((c + 1) & 1) * STAGE);
            __syncthreads();
        }
        // one per-lane base pointer; the (i, j, r) offsets are wave-uniform
        double *cb = C + (wm * 64 + (lane & 15)) + (int64_t)(wn * 64 + 4 * (lane >> 4)) * ldc;
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double *cc = cb + (int64_t)(16 * j + r) * ldc;
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    cc[16 * i] = cc[16 * i] - (double)acc[i][j][r];
            }
    }
};

// TileF with the operands already in FP32 in memory (the FP32 copies of the
// factor and of the solved block rows): A M-contiguous (element (m, k) at
// A[m + k lda]), B K-contiguous (element (n, k) at B[k + n ldb]); 16-byte
// loads, no conversion when staging.  Same LDS layout, MFMA sequence and C
// update as TileF, so the results are bitwise those of TileF on the FP64
// operands.
template <int WM, int WN> struct TileG {
    using T = TileF<WM, WN, true>;
    static constexpr int BM = T::BM, BN = T::BN, KC = T::KC, LSA = T::LSA, LSB = T::LSB;
    static constexpr int STAGE = T::STAGE, LDS = T::LDS;
    static constexpr int NA = BM * KC / 1024, NBL = BN * KC / 1024; // float4 loads per thread

    __device__ static void load(float4 *ra, float4 *rb, const float *A, int64_t lda,
                                const float *B, int64_t ldb, int k0)
    {
        const int t = threadIdx.x;
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int q = t + 256 * i, m4 = q % (BM / 4), k = q / (BM / 4);
            ra[i] = *(const float4 *)(A + 4 * m4 + (int64_t)(k0 + k) * lda);
        }
#pragma unroll
        for (int i = 0; i < NBL; ++i) {
            const int q = t + 256 * i, k4 = q % (KC / 4), nn = q / (KC / 4);
            rb[i] = *(const float4 *)(B + (k0 + 4 * k4) + (int64_t)nn * ldb);
        }
    }
    __device__ static void store(const float4 *ra, const float4 *rb, float *st)
    {
        const int t = threadIdx.x;
        float *As = st, *Bs = st + KC * LSA;
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int q = t + 256 * i, m4 = q % (BM / 4), k = q / (BM / 4);
            *(float4 *)(As + k * LSA + 4 * m4) = ra[i];
        }
#pragma unroll
        for (int i = 0; i < NBL; ++i) {
            const int q = t + 256 * i, k4 = q % (KC / 4), nn = q / (KC / 4);
            Bs[(4 * k4) * LSB + nn] = rb[i].x;
            Bs[(4 * k4 + 1) * LSB + nn] = rb[i].y;
            Bs[(4 * k4 + 2) * LSB + nn] = rb[i].z;
            Bs[(4 * k4 + 3) * LSB + nn] = rb[i].w;
        }
    }
    // C(BM x BN, FP64) -= A(BM x NB) * B(BN x NB)^T, one NB-deep FP32 slice
    __device__ static void update_slice(double *C, int64_t ldc, const float *A, int64_t lda,
                                        const float *B, int64_t ldb, float *lds)
    {
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const int wm = wave % WM, wn = wave / WM;
        f4 acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = (f4){0.f, 0.f, 0.f, 0.f};
        float4 ra[NA], rb[NBL];
        load(ra, rb, A, lda, B, ldb, 0);
        store(ra, rb, lds);
        __syncthreads();
        constexpr int nch = NB / KC;
        for (int c = 0; c < nch; ++c) {
            if (c + 1 < nch)
                load(ra, rb, A, lda, B, ldb, (c + 1) * KC);
            T::compute(acc, lds + (c & 1) * STAGE, wm, wn, lane);
            if (c + 1 < nch)
                store(ra, rb, lds + ((c + 1) & 1) * STAGE);
            __syncthreads();
        }
        double *cb = C + (wm * 64 + (lane & 15)) + (int64_t)(wn * 64 + 4 * (lane >> 4)) * ldc;
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double *cc = cb + (int64_t)(16 * j + r) * ldc;
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    cc[16 * i] = cc[16 * i] - (double)acc[i][j][r];
            }
    }
};

// BF16 variant of TileF: operands rounded to bfloat16 (round to nearest
// even, through FP32) when staged into LDS, products summed in FP32 on
// v_mfma_f32_16x16x16_bf16 over NB-deep slices, each slice subtracted from the
// FP64 C tile.  LDS rows hold one row of A or B with k contiguous, so a lane
// reads its four consecutive-k operands with one 8-byte load.
typedef short s4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short to_bf16(double v)
{
    const unsigned int u = __float_as_uint((float)v);
    return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

template <int WM, int WN, bool BKC> struct TileB {
    static constexpr int BM = 64 * WM, BN = 64 * WN, KC = 16;
    static constexpr int LK = KC + 4;                 // padded LDS row (bf16 elements)
    static constexpr int STAGE = (BM + BN) * LK;
    static constexpr int LDS = 2 * STAGE;             // bf16 elements
    static constexpr int NA = BM * KC / 512;          // double2 loads per thread
    static constexpr int NBL = BN * KC / 512;

    __device__ static void store(const double2 *ra, const double2 *rb, unsigned short *st)
    {
        const int t = threadIdx.x;
        unsigned short *As = st, *Bs = st + BM * LK;
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int q = t + 256 * i, m2 = q % (BM / 2), k = q / (BM / 2);
            As[(2 * m2) * LK + k] = to_bf16(ra[i].x);
            As[(2 * m2 + 1) * LK + k] = to_bf16(ra[i].y);
        }
#pragma unroll
        for (int i = 0; i < NBL; ++i) {
            const int q = t + 256 * i;
            if (!BKC) {
                const int n2 = q % (BN / 2), k = q / (BN / 2);
                Bs[(2 * n2) * LK + k] = to_bf16(rb[i].x);
                Bs[(2 * n2 + 1) * LK + k] = to_bf16(rb[i].y);
            } else {
                const int k2 = q % (KC / 2), nn = q / (KC / 2);
                Bs[nn * LK + 2 * k2] = to_bf16(rb[i].x);
                Bs[nn * LK + 2 * k2 + 1] = to_bf16(rb[i].y);
            }
        }
    }
    __device__ static void compute(f4 (&acc)[4][4], const unsigned short *st, int wm, int wn,
                                   int lane)
    {
        const unsigned short *As = st + (wm * 64 + (lane & 15)) * LK + 4 * (lane >> 4);
        const unsigned short *Bs = st + BM * LK + (wn * 64 + (lane & 15)) * LK + 4 * (lane >> 4);
        s4v a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            a[i] = *(const s4v *)(As + 16 * i * LK);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            b[j] = *(const s4v *)(Bs + 16 * j * LK);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(b[j], a[i], acc[i][j], 0, 0, 0);
    }
    __device__ __forceinline__ static void update(double *C, int64_t ldc, const double *A, int64_t lda,
                                                  const double *B, int64_t ldb, int K,
                                                  unsigned short *lds)
    {
#pragma unroll 1
        for (int k0 = 0; k0 < K; k0 += NB)
            update_slice(C, ldc, A + (int64_t)k0 * lda, lda, BKC ? B + k0 : B + (int64_t)k0 * ldb,
                         ldb, K - k0 < NB ? K - k0 : NB, lds);
    }
    __device__ __forceinline__ static void update_slice(double *C, int64_t ldc, const double *A,
                                                        int64_t lda, const double *B, int64_t ldb,
                                                        int K, unsigned short *lds)
    {
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const int wm = wave % WM, wn = wave / WM;
        f4 acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = (f4){0.f, 0.f, 0.f, 0.f};
        double2 ra[NA], rb[NBL];
        TileF<WM, WN, BKC>::load(ra, rb, A, lda, B, ldb, 0);
        store(ra, rb, lds);
        __syncthreads();
        const int nch = K / KC;
        for (int c = 0; c < nch; ++c) {
            if (c + 1 < nch)
                TileF<WM, WN, BKC>::load(ra, rb, A, lda, B, ldb, (c + 1) * KC);
            compute(acc, lds + (c & 1) * STAGE, wm, wn, lane);
            if (c + 1 < nch)
                store(ra, rb, lds + ((c + 1) & 1) * STAGE);
            __syncthreads();
        }
        double *cb = C + (wm * 64 + (lane & 15)) + (int64_t)(wn * 64 + 4 * (lane >> 4)) * ldc;
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double *cc = cb + (int64_t)(16 * j + r) * ldc;
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    cc[16 * i] = cc[16 * i] - (double)acc[i][j][r];
            }
    }
};

// TileB from the FP32 operand copies (A M-contiguous, B K-contiguous, as in
// TileG): the floats are rounded to bfloat16 when staged, which gives the same
// operands as TileB's rounding of the FP64 values through FP32, so the results
// are bitwise TileB's.
__device__ __forceinline__ unsigned short to_bf16f(float v)
{
    const unsigned int u = __float_as_uint(v);
    return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

template <int WM, int WN> struct TileBG {
    using T = TileB<WM, WN, true>;
    static constexpr int BM = T::BM, BN = T::BN, KC = T::KC, LK = T::LK, STAGE = T::STAGE;
    static constexpr int LDS = T::LDS;
    static constexpr int NA = BM * KC / 1024, NBL = BN * KC / 1024; // float4 loads per thread

    __device__ static void store(const float4 *ra, const float4 *rb, unsigned short *st)
    {
        const int t = threadIdx.x;
        unsigned short *As = st, *Bs = st + BM * LK;
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int q = t + 256 * i, m4 = q % (BM / 4), k = q / (BM / 4);
            As[(4 * m4) * LK + k] = to_bf16f(ra[i].x);
            As[(4 * m4 + 1) * LK + k] = to_bf16f(ra[i].y);
            As[(4 * m4 + 2) * LK + k] = to_bf16f(ra[i].z);
            As[(4 * m4 + 3) * LK + k] = to_bf16f(ra[i].w);
        }
#pragma unroll
        for (int i = 0; i < NBL; ++i) {
            const int q = t + 256 * i, k4 = q % (KC / 4), nn = q / (KC / 4);
            Bs[nn * LK + 4 * k4] = to_bf16f(rb[i].x);
            Bs[nn * LK + 4 * k4 + 1] = to_bf16f(rb[i].y);
            Bs[nn * LK + 4 * k4 + 2] = to_bf16f(rb[i].z);
            Bs[nn * LK + 4 * k4 + 3] = to_bf16f(rb[i].w);
        }
    }
    // C(BM x BN, FP64) -= A(BM x NB) * B(BN x NB)^T, one NB-deep slice
    __device__ static void update_slice(double *C, int64_t ldc, const float *A, int64_t lda,
                                        const float *B, int64_t ldb, unsigned short *lds)
    {
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const int wm = wave % WM, wn = wave / WM;
        f4 acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = (f4){0.f, 0.f, 0.f, 0.f};
        float4 ra[NA], rb[NBL];
        TileG<WM, WN>::load(ra, rb, A, lda, B, ldb, 0);
        store(ra, rb, lds);
        __syncthreads();
        constexpr int nch = NB / KC;
        for (int c = 0; c < nch; ++c) {
            if (c + 1 < nch)
                TileG<WM, WN>::load(ra, rb, A, lda, B, ldb, (c + 1) * KC);
            T::compute(acc, lds + (c & 1) * STAGE, wm, wn, lane);
            if (c + 1 < nch)
                store(ra, rb, lds + ((c + 1) & 1) * STAGE);
            __syncthreads();
        }
        double *cb = C + (wm * 64 + (lane & 15)) + (int64_t)(wn * 64 + 4 * (lane >> 4)) * ldc;
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double *cc = cb + (int64_t)(16 * j + r) * ldc;
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    cc[16 * i] = cc[16 * i] - (double)acc[i][j][r];
            }
    }
};

// C -= A * B^T over the block-lower tiles of a trailing matrix of nblk x nblk
// NB-blocks (128 x 128 tiles; both 128-tiles above the diagonal inside a
// diagonal NB-block are included), depth K (one, two or four panels).  blockIdx.y
// selects (C0, A0) or (C1, A1).
template <int MIX, int K = NB>
__global__ __launch_bounds__(256) void k_update_lower(int nmat, int64_t sC, int64_t sB,
                                                      double *C0, double *C1, int64_t ldc,
                                                      const double *A0, const double *A1,
                                                      int64_t lda, const double *B, int64_t ldb)
{
    using TL = Tile<2, 2, false, true>;
    using TF = TileF<2, 2, false>;
    using TBF = TileB<2, 2, false>;
    __shared__ double lds[MIX == 2 ? (TBF::LDS + 3) / 4 : MIX ? (TF::LDS + 1) / 2 : TL::LDS];
    const int64_t u = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t p = u >> 2;
    const int s = u & 3;
    int64_t I = (int64_t)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= p)
        ++I;
    while (I * (I + 1) / 2 > p)
        --I;
    const int64_t J = p - I * (I + 1) / 2;
    const int64_t m0 = I * NB + 128 * (s >> 1), n0 = J * NB + 128 * (s & 1);
    const int mat = blockIdx.y % nmat, f = blockIdx.y / nmat; // matrix, field
    double *C = (mat ? C1 : C0) + f * sC + m0 + n0 * ldc;
    const double *A = (mat ? A1 : A0) + f * sC + m0;
    B += f * sB;
    if constexpr (MIX == 2) {
        TBF::update(C, ldc, A, lda, B + n0, ldb, K, (unsigned short *)lds);
    } else if constexpr (MIX == 1) {
        TF::update(C, ldc, A, lda, B + n0, ldb, K, (float *)lds);
    } else {
        d4 acc[4][4];
        TL::load_c(acc, C, ldc);
        TL::run(acc, A, lda, B + n0, ldb, K, lds);
        TL::store_c(acc, C, ldc);
    }
}

// C -= A * B^T on a rectangle of rows x ncol (128 x 128 tiles, depth K): the
// next block column(s) of a trailing update (lookahead).  blockIdx.z selects
// the matrix.
template <int MIX, int K = NB>
__global__ __launch_bounds__(256) void k_update_rect(int nmat, int64_t sC, int64_t sB, double *C0,
                                                     double *C1, int64_t ldc, const double *A0,
                                                     const double *A1, int64_t lda,
                                                     const double *B, int64_t ldb)
{
    using TL = Tile<2, 2, false, true>;
    using TF = TileF<2, 2, false>;
    using TBF = TileB<2, 2, false>;
    __shared__ double lds[MIX == 2 ? (TBF::LDS + 3) / 4 : MIX ? (TF::LDS + 1) / 2 : TL::LDS];
    const int64_t m0 = 128 * (int64_t)blockIdx.x, n0 = 128 * (int64_t)blockIdx.y;
    const int mat = blockIdx.z % nmat, f = blockIdx.z / nmat; // matrix, field
    double *C = (mat ? C1 : C0) + f * sC + m0 + n0 * ldc;
    const double *A = (mat ? A1 : A0) + f * sC + m0;
    B += f * sB;
    if constexpr (MIX == 2) {
        TBF::update(C, ldc, A, lda, B + n0, ldb, K, (unsigned short *)lds);
    } else if constexpr (MIX == 1) {
        TF::update(C, ldc, A, lda, B + n0, ldb, K, (float *)lds);
    } else {
        d4 acc[4][4];
        TL::load_c(acc, C, ldc);
        TL::run(acc, A, lda, B + n0, ldb, K, lds);
        TL::store_c(acc, C, ldc);
    }
}

// Both launchers take K = NB or 2 NB.  The FP32 form applies two panels as
// two NB-deep launches (its NB-deep kernel keeps four workgroups per CU);
// A and B then advance by NB columns.
void launch_update_rect(hipStream_t s, const Fields &F, int64_t sC, int64_t sB, int nmat,
                        double *C0, double *C1, int64_t ldc, const double *A0, const double *A1,
                        int64_t lda, const double *B, int64_t ldb, int64_t rows, int64_t ncol,
                        int K, int mixed)
{
    if (rows <= 0 || ncol <= 0 || (K != NB && K != 2 * NB && K != 4 * NB))
        return;
    const dim3 g((unsigned)(rows / 128), (unsigned)(ncol / 128), (unsigned)(nmat * F.count));
    if (mixed) {
        auto kern = mixed == 2 ? k_update_rect<2> : k_update_rect<1>;
        for (int p = 0; p < K / NB; ++p) {
            const int64_t o = (int64_t)p * NB;
            hipLaunchKernelGGL(kern, g, dim3(256), 0, s, nmat, sC, sB, C0, C1, ldc,
                               A0 + o * lda, A1 ? A1 + o * lda : nullptr, lda, B + o * ldb, ldb);
        }
        return;
    }
    auto kern = K == 4 * NB   ? k_update_rect<0, 4 * NB>
                : K == 2 * NB ? k_update_rect<0, 2 * NB>
                              : k_update_rect<0, NB>;
    hipLaunchKernelGGL(kern, g, dim3(256), 0, s, nmat, sC, sB, C0, C1, ldc, A0, A1, lda, B, ldb);
}

void launch_update_lower(hipStream_t s, const Fields &F, int64_t sC, int64_t sB, int nmat,
                         double *C0, double *C1, int64_t ldc, const double *A0,
                         const double *A1, int64_t lda, const double *B, int64_t ldb, int nblk,
                         int K, int mixed)
{
    if (nblk <= 0 || (K != NB && K != 2 * NB && K != 4 * NB))
        return;
    const int64_t pairs = (int64_t)nblk * (nblk + 1) / 2;
    const dim3 g((unsigned)(4 * pairs), (unsigned)(nmat * F.count));
    if (mixed) {
        auto kern = mixed == 2 ? k_update_lower<2> : k_update_lower<1>;
        for (int p = 0; p < K / NB; ++p) {
            const int64_t o = (int64_t)p * NB;
            hipLaunchKernelGGL(kern, g, dim3(256), 0, s, nmat, sC, sB, C0, C1,
                               ldc, A0 + o * lda, A1 ? A1 + o * lda : nullptr, lda, B + o * ldb,
                               ldb);
        }
        return;
    }
    auto kern = K == 4 * NB   ? k_update_lower<0, 4 * NB>
                : K == 2 * NB ? k_update_lower<0, 2 * NB>
                              : k_update_lower<0, NB>;
    hipLaunchKernelGGL(kern, g, dim3(256), 0, s, nmat, sC, sB, C0, C1, ldc, A0, A1, lda, B, ldb);
}

// Panel solve of the factorisation: P (rows x NB, in place) = P Linv^T.
// A workgroup owns 64 full rows, so the in-place update is race free.
__global__ __launch_bounds__(256) void k_panel(Fields F, double *P, int64_t ld, const double *Linv)
{
    using TL = Tile<1, 4, false>;
    __shared__ double lds[TL::LDS];
    const int f = blockIdx.y; // field
    Linv += f * F.sLinv;
    double *Pb = P + f * F.sA + (int64_t)blockIdx.x * 64;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    d4 acc[4][4];
    TL::zero(acc);
    // output columns 64 wave.. of P Linv^T: Linv rows there vanish past column 64 wave + 63
    TL::run(acc, Pb, ld, Linv, NB, NB, lds, 4 * (wave + 1));
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                Pb[TL::row(i, lane, 0) + (int64_t)TL::col(j, r, lane, wave) * ld] = acc[i][j][r];
}

void launch_panel(hipStream_t s, const Fields &F, double *P, int64_t ld, int64_t rows,
                  const double *Linv)
{
    if (rows <= 0)
        return;
    hipLaunchKernelGGL(k_panel, dim3((unsigned)(rows / 64), F.count), dim3(256), 0, s, F, P, ld,
                       Linv);
}

// Left solve, diagonal block: S[krow:krow+NB, cols] = Linv * S[krow:krow+NB, cols]
// (in place; a workgroup owns all NB rows of 64 columns).  Column tile c maps
// to column 64 c, shifted by col_shift past the first half (two right-hand
// sides stored side by side; with one right-hand side only the first half is
// launched).  With Xf (the mixed forms), the solved rows are also stored as
// floats at Xf[(kofs + row) + col * 2 NB], the operand copy of the updates.
__global__ __launch_bounds__(256) void k_diag_apply(Fields F, int64_t sS, double *S, int64_t ld,
                                                    int64_t krow, const double *Linv,
                                                    int64_t half_tiles, int64_t col_shift,
                                                    float *Xf, int kofs)
{
    using TL = Tile<4, 1, true>;
    __shared__ double lds[TL::LDS];
    const int f = blockIdx.y; // field
    S += f * sS;
    Linv += f * F.sLinv;
    const int64_t ct = blockIdx.x;
    const int64_t c0 = (ct < half_tiles) ? 64 * ct : col_shift + 64 * (ct - half_tiles);
    double *Sb = S + krow + c0 * ld;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    d4 acc[4][4];
    TL::zero(acc);
    // rows 64 wave.. of Linv vanish past column 64 wave + 63
    TL::run(acc, Linv, NB, Sb, ld, NB, lds, 4 * (wave + 1));
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                Sb[TL::row(i, lane, wave) + (int64_t)TL::col(j, r, lane, 0) * ld] = acc[i][j][r];
    if (Xf) {
        float *xb = Xf + f * F.sXf + kofs + c0 * (2 * NB);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    xb[TL::row(i, lane, wave) + (int64_t)TL::col(j, r, lane, 0) * (2 * NB)] =
                        (float)acc[i][j][r];
    }
}

void launch_diag_apply(hipStream_t s, const Fields &F, int64_t sS, int nmat, double *S,
                       int64_t ld, int64_t krow, const double *Linv, int64_t ncols,
                       int64_t col_shift, float *Xf, int kofs)
{
    const int64_t half = ncols / 64;
    if (half <= 0)
        return;
    hipLaunchKernelGGL(k_diag_apply, dim3((unsigned)(nmat * half), F.count), dim3(256), 0, s, F,
                       sS, S, ld, krow, Linv, half, col_shift, Xf, kofs);
}

// Left solve, update below the diagonal block(s):
// S[r0 + 128 y, cols] -= L[r0 + 128 y, krow:krow+K] * S[krow:krow+K, cols]
// (K = NB for one panel, 2 NB for two consecutive panels at once).
template <int MIX, int K = NB>
__global__ __launch_bounds__(256) void k_update_nn(Fields F, int64_t sS, double *S, int64_t ld,
                                                   const double *L, int64_t lda, int64_t r0,
                                                   int64_t krow, int64_t half_tiles,
                                                   int64_t col_shift)
{
    using TL = Tile<2, 2, true, true>;
    using TF = TileF<2, 2, true>;
    using TBF = TileB<2, 2, true>;
    __shared__ double lds[MIX == 2 ? (TBF::LDS + 3) / 4 : MIX ? (TF::LDS + 1) / 2 : TL::LDS];
    const int f = blockIdx.z; // field
    S += f * sS;
    L += f * F.sA;
    // row-major tile order (tiles of a row share the L panel), renumbered per XCD
    const int64_t u = xcd_tile(blockIdx.x + (int64_t)blockIdx.y * gridDim.x,
                               (int64_t)gridDim.x * gridDim.y);
    const int64_t ct = u % gridDim.x;
    const int64_t c0 = (ct < half_tiles) ? 128 * ct : col_shift + 128 * (ct - half_tiles);
    const int64_t m0 = r0 + 128 * (u / gridDim.x);
    double *C = S + m0 + c0 * ld;
    if constexpr (MIX == 2) {
        TBF::update(C, ld, L + m0 + krow * lda, lda, S + krow + c0 * ld, ld, K,
                    (unsigned short *)lds);
    } else if constexpr (MIX == 1) {
        TF::update(C, ld, L + m0 + krow * lda, lda, S + krow + c0 * ld, ld, K, (float *)lds);
    } else {
        d4 acc[4][4];
        TL::load_c(acc, C, ld);
        TL::run(acc, L + m0 + krow * lda, lda, S + krow + c0 * ld, ld, K, lds);
        TL::store_c(acc, C, ld);
    }
}

void launch_update_nn(hipStream_t s, const Fields &F, int64_t sS, int nmat, double *S, int64_t ld,
                      const double *L, int64_t lda, int64_t r0, int64_t krow, int64_t rows,
                      int64_t ncols, int64_t col_shift, int K, int mixed)
{
    const int64_t half = ncols / 128;
    if (rows <= 0 || half <= 0 || (K != NB && K != 2 * NB))
        return;
    const dim3 g((unsigned)(nmat * half), (unsigned)(rows / 128), F.count);
    // The depth K is a template parameter (a known trip count keeps the main
    // loop as fast as the fixed-depth form).  The FP32 form applies two panels
    // as two NB-deep launches: its NB-deep kernel keeps four workgroups per CU.
    if (mixed) {
        auto kern = mixed == 2 ? k_update_nn<2> : k_update_nn<1>;
        for (int p = 0; p < K / NB; ++p)
            hipLaunchKernelGGL(kern, g, dim3(256), 0, s, F, sS, S, ld, L, lda, r0,
                               krow + p * NB, half, col_shift);
        return;
    }
    auto kern = K == 2 * NB ? k_update_nn<0, 2 * NB> : k_update_nn<0, NB>;
    hipLaunchKernelGGL(kern, g, dim3(256), 0, s, F, sS, S, ld, L, lda, r0, krow, half, col_shift);
}

// FP32 form of the left-solve update from the FP32 copies (one NB-deep slice):
// C = S[m0.., c0..] -= Lf[m0.., krow:krow+NB] * Xf[kofs.., c0..]^T, 128 x 128 tiles.
// Bitwise the same as k_update_nn<1, NB> on the FP64 operands.
template <bool BF>
__global__ __launch_bounds__(256) void k_update_nn_f32(Fields F, int64_t sS, double *S, int64_t ld,
                                                       const float *Lf, int64_t r0, int64_t krow,
                                                       const float *Xf, int kofs,
                                                       int64_t half_tiles, int64_t col_shift)
{
    // BF: bfloat16 operands (TileB's rounding) instead of FP32
    using TG = typename std::conditional<BF, TileBG<2, 2>, TileG<2, 2>>::type;
    using E = typename std::conditional<BF, unsigned short, float>::type;
    __shared__ E lds[TG::LDS];
    const int f = blockIdx.z; // field
    S += f * sS;
    Lf += f * F.sA;
    Xf += f * F.sXf;
    const int64_t ct = blockIdx.x;
    const int64_t c0 = (ct < half_tiles) ? 128 * ct : col_shift + 128 * (ct - half_tiles);
    const int64_t m0 = r0 + 128 * (int64_t)blockIdx.y;
    TG::update_slice(S + m0 + c0 * ld, ld, Lf + m0 + krow * ld, ld, Xf + kofs + c0 * (2 * NB),
                     2 * NB, lds);
}

void launch_update_nn_f32(hipStream_t s, const Fields &F, int64_t sS, int nmat, double *S,
                          int64_t ld, const float *Lf, int64_t r0, int64_t krow, const float *Xf,
                          int kofs, int64_t rows, int64_t ncols, int64_t col_shift, bool bf16)
{
    const int64_t half = ncols / 128;
    if (rows <= 0 || half <= 0)
        return;
    const dim3 g((unsigned)(nmat * half), (unsigned)(rows / 128), F.count);
    hipLaunchKernelGGL(bf16 ? k_update_nn_f32<true> : k_update_nn_f32<false>, g, dim3(256), 0, s, F,
                       sS, S, ld, Lf, r0, krow, Xf, kofs, half, col_shift);
}

// Lf = (float) A on the NB blocks at or below the diagonal; blockIdx.x walks
// the columns of a block column (y = block column, z = field), 64 threads per
// 64 rows.
__global__ __launch_bounds__(256) void k_to_f32_lower(Fields F, const double *A, int64_t ld,
                                                      int64_t npad, float *Lf)
{
    const int f = blockIdx.z;
    A += f * F.sA;
    Lf += f * F.sA;
    const int64_t col = (int64_t)blockIdx.y * NB + blockIdx.x;  // one column per workgroup
    const int64_t r0 = (int64_t)blockIdx.y * NB;                // rows from its block's diagonal
    for (int64_t r = r0 + 2 * (int64_t)threadIdx.x; r < npad; r += 512) {
        const double2 v = *(const double2 *)(A + r + col * ld);
        *(float2 *)(Lf + r + col * ld) = make_float2((float)v.x, (float)v.y);
    }
}

void launch_to_f32_lower(hipStream_t s, const Fields &F, const double *A, int64_t ld, int64_t npad,
                         float *Lf)
{
    hipLaunchKernelGGL(k_to_f32_lower, dim3(NB, (unsigned)(npad / NB), F.count), dim3(256), 0, s, F,
                       A, ld, npad, Lf);
}

// ---------------------------------------------------------------------------
// Right solve panel with the trace reductions.  For block column k, both
// right-hand sides: W_i[r0 + 64 x, kcol:kcol+NB] = X_i[...] Linv^T in place,
// after which those entries of W_i are final.  The epilogue accumulates, over
// entries (a, b) with a, b < n,
//   t_i = sum_a W_i[a][a],  F_ij = sum w_ab W_i[a][b] W_j[a][b]
// with weight w_ab = 1 inside a diagonal NB-block (stored in full) and 2 below
// it (the mirrored upper block is not stored), and picks u_i = W_i[n][n]
// = y^T W_i y from the observation border.  Seven partial sums per workgroup
// go to partials[8 blockIdx.x + 0..6] in a fixed order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

__global__ __launch_bounds__(256) void k_panel_reduce(Fields F, double *Xa, double *Xn,
                                                      int64_t ld, int64_t r0, int64_t kcol,
                                                      const double *Linv, int64_t n1,
                                                      double *partials)
{
    using TL = Tile<1, 4, false>;
    __shared__ double lds[TL::LDS];
    __shared__ double red[4][8];
    const int f = blockIdx.y; // field
    Xa += f * F.sS2;
    Xn += f * F.sS2;
    Linv += f * F.sLinv;
    partials += f * F.sPart;
    const int64_t n = F.n ? F.n[f] : n1;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t m0 = r0 + (int64_t)blockIdx.x * 64;
    d4 acc[4][4];
    double s[7] = {0, 0, 0, 0, 0, 0, 0}; // t_a, t_n, u_a, u_n, F_aa, F_an, F_nn
    TL::zero(acc);
    // output columns 64 wave.. of X Linv^T: Linv rows there vanish past column 64 wave + 63
    TL::run(acc, Xa + m0 + kcol * ld, ld, Linv, NB, NB, lds, 4 * (wave + 1));
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                Xa[m0 + TL::row(i, lane, 0) + (kcol + TL::col(j, r, lane, wave)) * ld] = acc[i][j][r];
    TL::zero(acc);
    TL::run(acc, Xn + m0 + kcol * ld, ld, Linv, NB, NB, lds, 4 * (wave + 1));
    // W_alpha is read back by the lane that stored it (program order makes its
    // own stores visible), which keeps the workgroup small enough to share a
    // CU with a trailing-update workgroup.
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t a = m0 + TL::row(i, lane, 0);
                const int64_t b = kcol + TL::col(j, r, lane, wave);
                const double vn = acc[i][j][r], va = Xa[a + b * ld];
                Xn[a + b * ld] = vn;
                if (a < n && b < n) {
                    const double w = (a / NB == b / NB) ? 1.0 : 2.0;
                    s[4] = fma(w * va, va, s[4]);
                    s[5] = fma(w * va, vn, s[5]);
                    s[6] = fma(w * vn, vn, s[6]);
                    if (a == b) {
                        s[0] += va;
                        s[1] += vn;
                    }
                } else if (a == n && b == n) {
                    s[2] = va;
                    s[3] = vn;
                }
            }
#pragma unroll
    for (int q = 0; q < 7; ++q) {
        const double v = wave_sum(s[q]);
        if (lane == 0)
            red[wave][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < 7) {
        const int q = threadIdx.x;
        partials[8 * (int64_t)blockIdx.x + q] = ((red[0][q] + red[1][q]) + red[2][q]) + red[3][q];
    }
}

void launch_panel_reduce(hipStream_t s, const Fields &F, double *Xa, double *Xn, int64_t ld,
                         int64_t r0, int64_t kcol, int64_t rows, const double *Linv, int64_t n,
                         double *partials)
{
    hipLaunchKernelGGL(k_panel_reduce, dim3((unsigned)(rows / 64), F.count), dim3(256), 0, s, F,
                       Xa, Xn, ld, r0, kcol, Linv, n, partials);
}

// ---------------------------------------------------------------------------
// Deterministic reductions (fixed summation order, one workgroup).
// out[0] = log det Sigma = 2 sum_k logdet_part[k];  out[1] = y^T y with
// y = row n of the bordered factor.
// ---------------------------------------------------------------------------
__device__ double block_sum(double v, double *sh)
{
    const int t = threadIdx.x;
    v = wave_sum(v);
    if ((t & 63) == 0)
        sh[t >> 6] = v;
    __syncthreads();
    double r = ((sh[0] + sh[1]) + sh[2]) + sh[3];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void k_reduce_loglik(Fields F, const double *A, int64_t lda,
                                                       int64_t n1, int T,
                                                       const double *logdet_part, double *out)
{
    __shared__ double sh[4];
    const int t = threadIdx.x;
    const int f = blockIdx.x; // field
    A += f * F.sA;
    logdet_part += f * F.sLog;
    out += 16 * f;
    const int64_t n = F.n ? F.n[f] : n1;
    double q = 0.0;
    for (int64_t c = t; c < n; c += 256) {
        const double y = A[n + c * lda];
        q = fma(y, y, q);
    }
    double ld = 0.0;
    for (int k = t; k < T; k += 256)
        ld += logdet_part[k];
    q = block_sum(q, sh);
    ld = block_sum(ld, sh);
    if (t == 0) {
        out[0] = 2.0 * ld;
        out[1] = q;
    }
}

void launch_reduce_loglik(hipStream_t s, const Fields &F, const double *A, int64_t lda,
                          int64_t n, int T, const double *logdet_part, double *out)
{
    hipLaunchKernelGGL(k_reduce_loglik, dim3((unsigned)F.count), dim3(256), 0, s, F, A, lda, n, T,
                       logdet_part, out);
}

// out[2..8] = sums over `count` groups of 8 partials (t_a, t_n, u_a, u_n, F_aa, F_an, F_nn)
__global__ __launch_bounds__(256) void k_reduce_terms(Fields F, const double *partials,
                                                      int64_t count, double *out)
{
    __shared__ double sh[4];
    const int t = threadIdx.x;
    const int f = blockIdx.x; // field
    partials += f * F.sPart;
    out += 16 * f;
    for (int q = 0; q < 7; ++q) {
        double v = 0.0;
        for (int64_t g = t; g < count; g += 256)
            v += partials[8 * g + q];
        v = block_sum(v, sh);
        if (t == 0)
            out[2 + q] = v;
    }
}

void launch_reduce_terms(hipStream_t s, const Fields &F, const double *partials, int64_t count,
                         double *out)
{
    hipLaunchKernelGGL(k_reduce_terms, dim3((unsigned)F.count), dim3(256), 0, s, F, partials,
                       count, out);
}

// ---------------------------------------------------------------------------
// Two-sided reduction W_i = L^{-1} Sigma_i L^{-T} (the W phase of Algorithm 3
// with n^3 flops per derivative matrix instead of the 4 n^3 / 3 of a left
// solve followed by a lower-half right solve).  With L = [[L11, 0], [L21, L22]]
// (L11 one NB-block) and S = Sigma_i partitioned alike, L W L^T = S gives
//   W11 = L11^{-1} S11 L11^{-T},
//   L22 W21 = M21 = S21 L11^{-T} - L21 W11,
//   L22 W22 L22^T = S22 - Y21 L21^T - L21 Y21^T,  Y21 = S21 L11^{-T} - L21 W11 / 2,
// so one block step forms W11, Y21 and M21 and applies a symmetric rank-2 NB
// update to the trailing S22 (only its lower blocks are kept); the solves
// L22^{-1} M21 of all steps are deferred.  Since M21 of step k is zero above
// block row k + 1, they are one left solve W_strict = L^{-1} M of the
// block-strictly-lower matrix M, whose block row r has nonzeros in columns
// < r NB only (n^3 / 3 flops per matrix; the steps cost 2 n^3 / 3).
// Storage: M replaces S's strictly lower blocks; V_k = -W_kk / 2 (full,
// exactly symmetric) goes to a separate NB x NB block per step; Y of the
// current pair of steps to a slot of npad x 2 NB per matrix.
// ---------------------------------------------------------------------------

// Diagonal block of step k for both matrices (blockIdx.y): with P = S_kk Linv_k^T
// (scratch Pd, NB x NB per matrix), W_kk = Linv_k P; stores V = -W_kk / 2,
// its lower triangle and the mirror of it, so V is exactly symmetric.  A
// workgroup forms 64 columns of P and then the same 64 columns of W.
__global__ __launch_bounds__(256) void k_sygst_diag(Fields F, const double *S2, int64_t ld,
                                                    int64_t mofs, int64_t krow,
                                                    const double *Linv, double *Pd,
                                                    int64_t sPd, double *Vd, int64_t vofs,
                                                    int64_t sVd)
{
    using TA = Tile<4, 1, false>;
    using TB = Tile<4, 1, true>;
    static_assert(TA::LDS == TB::LDS, "one LDS buffer for both products");
    __shared__ double lds[TA::LDS];
    const int m = blockIdx.y, f = blockIdx.z; // matrix, field
    const int c0 = 64 * blockIdx.x;
    const double *S = S2 + f * F.sS2 + m * mofs + krow + krow * ld;
    Linv += f * F.sLinv;
    double *P = Pd + f * sPd + m * (NB * NB);
    double *V = Vd + f * sVd + m * vofs;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    d4 acc[4][4];
    TA::zero(acc);
    // P[:, c0 + j] = S_kk Linv[c0 + j, :]^T: row c0 + j of Linv vanishes past column c0 + j
    TA::run(acc, S, ld, Linv + c0, NB, c0 + 64, lds);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                P[TA::row(i, lane, wave) + (int64_t)(c0 + TA::col(j, r, lane, 0)) * NB] = acc[i][j][r];
    // the other waves read these columns of P below
    __threadfence();
    __syncthreads();
    TB::zero(acc);
    // W[:, c0 + j] = Linv P[:, c0 + j]: rows 64 wave.. of Linv vanish past column 64 wave + 63
    TB::run(acc, Linv, NB, P + (int64_t)c0 * NB, NB, NB, lds, 4 * (wave + 1));
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int a = TB::row(i, lane, wave), b = c0 + TB::col(j, r, lane, 0);
                if (a >= b) {
                    const double v = -0.5 * acc[i][j][r];
                    V[a + b * NB] = v;
                    if (a != b)
                        V[b + a * NB] = v;
                }
            }
}

void launch_sygst_diag(hipStream_t s, const Fields &F, const double *S2, int64_t ld, int64_t mofs,
                       int64_t krow, const double *Linv, double *Pd, int64_t sPd, double *Vd,
                       int64_t vofs, int64_t sVd)
{
    hipLaunchKernelGGL(k_sygst_diag, dim3(NB / 64, 2, F.count), dim3(256), 0, s, F, S2, ld, mofs,
                       krow, Linv, Pd, sPd, Vd, vofs, sVd);
}

// Panel of step k, rows r0.., both matrices: with P = S[rows, k] Linv_k^T and
// Q = L[rows, k] W_kk,
//   Y = P - Q / 2 -> the slot (ld ldy),  M = P - Q -> in place of S[rows, k].
// A workgroup owns 128 full rows of the block column (blockIdx.x: row tile,
// y: matrix + 2 field) and forms them as two 128 x 128 tiles with the tile
// engine of the bulk updates.  The right tile (columns 128..255) goes first:
// its P reads S over all 256 columns, the left tile's only over columns
// 0..127, so each tile's M can be stored in place as soon as it is formed.
// -Q / 2 = L V is formed first and parked in the slot, where the lane that
// stored it reads it back (program order) after P has been added.
__global__ __launch_bounds__(256) void k_sygst_panel(Fields F, double *S2, int64_t ld,
                                                        int64_t mofs, const double *A, int64_t r0,
                                                        int64_t krow, const double *Linv,
                                                        const double *Vd, int64_t vofs,
                                                        int64_t sVd, double *Y, int64_t ldy,
                                                        int64_t ymofs, int64_t sY)
{
    using TL = Tile<2, 2, false>;
    __shared__ double lds[TL::LDS];
    const int m = blockIdx.y & 1, f = blockIdx.y >> 1; // matrix, field
    const int64_t mr = r0 + 128 * (int64_t)blockIdx.x;
    double *S = S2 + f * F.sS2 + m * mofs + mr + krow * ld;
    const double *Lp = A + f * F.sA + mr + krow * ld;
    Linv += f * F.sLinv;
    const double *V = Vd + f * sVd + m * vofs;
    double *Yp = Y + f * sY + m * ymofs + mr;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wm = wave % 2, wn = wave / 2;
#pragma unroll 1
    for (int ct = 1; ct >= 0; --ct) {
        const int c0 = 128 * ct;
        d4 acc[4][4];
        TL::zero(acc);
        TL::run(acc, Lp, ld, V + c0, NB, NB, lds); // -Q / 2 (V symmetric)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    Yp[TL::row(i, lane, wm) + (int64_t)(c0 + TL::col(j, r, lane, wn)) * ldy] =
                        acc[i][j][r];
        // += S Linv^T over columns c0..: row c0 + j of Linv vanishes past column
        // c0 + j, so the tile needs depth c0 + 128 and the wave's 64 columns
        // depth c0 + 64 (wn + 1)
        TL::run(acc, S, ld, Linv + c0, NB, c0 + 128, lds, (c0 + 64 * (wn + 1)) / 16);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int a = TL::row(i, lane, wm), b = c0 + TL::col(j, r, lane, wn);
                    const double y = acc[i][j][r], h = Yp[a + (int64_t)b * ldy];
                    S[a + (int64_t)b * ld] = y + h;
                    Yp[a + (int64_t)b * ldy] = y;
                }
    }
}

void launch_sygst_panel(hipStream_t s, const Fields &F, double *S2, int64_t ld, int64_t mofs,
                        const double *A, int64_t r0, int64_t rows, int64_t krow,
                        const double *Linv, const double *Vd, int64_t vofs, int64_t sVd,
                        double *Y, int64_t ldy, int64_t ymofs, int64_t sY)
{
    if (rows <= 0)
        return;
    hipLaunchKernelGGL(k_sygst_panel, dim3((unsigned)(rows / 128), 2 * F.count), dim3(256), 0, s,
                       F, S2, ld, mofs, A, r0, krow, Linv, Vd, vofs, sVd, Y, ldy, ymofs, sY);
}

// C -= Y L^T + L Y^T on one 128 x 128 tile at (m0, n0) of matrix m: the
// symmetric update by the KS / NB steps whose Y fill slot columns 0..KS and
// whose factor columns start at kcol.  FP64 (MIX = 0): the two products are
// accumulated one after the other onto C (held in the accumulators), so a
// tile is read and written once for a 2 KS-deep update.  MIX = 1 (FP32) and 2
// (BF16 operands): TileF / TileB, FP32 sums per NB-deep slice subtracted from
// the FP64 C tile.
template <int MIX, int KS>
__device__ __forceinline__ void syr2k_tile(double *C, int64_t ld, const double *Ym, int64_t ldy,
                                           const double *L, int64_t kcol, int64_t m0, int64_t n0,
                                           double *lds)
{
    if constexpr (MIX == 0) {
        using TL = Tile<2, 2, false, true>;
        d4 acc[4][4];
        TL::load_c(acc, C + m0 + n0 * ld, ld);
        // one copy of the main loop for both products (two inlined copies cost
        // registers and the second workgroup per CU)
#pragma unroll 1
        for (int q = 0; q < 2; ++q) {
            const double *Aq = q ? L + m0 + kcol * ld : Ym + m0;
            const double *Bq = q ? Ym + n0 : L + n0 + kcol * ld;
            TL::run(acc, Aq, q ? ld : ldy, Bq, q ? ldy : ld, KS, lds);
        }
        TL::store_c(acc, C + m0 + n0 * ld, ld);
    } else {
        using TF = typename std::conditional<MIX == 2, TileB<2, 2, false>, TileF<2, 2, false>>::type;
        using E = typename std::conditional<MIX == 2, unsigned short, float>::type;
#pragma unroll 1
        for (int q = 0; q < 2; ++q) {
            const double *Aq = q ? L + m0 + kcol * ld : Ym + m0;
            const double *Bq = q ? Ym + n0 : L + n0 + kcol * ld;
            TF::update(C + m0 + n0 * ld, ld, Aq, q ? ld : ldy, Bq, q ? ldy : ld, KS, (E *)lds);
        }
    }
}

template <int MIX>
struct Syr2kLds {
    static constexpr int N = MIX == 2   ? (TileB<2, 2, false>::LDS + 3) / 4
                             : MIX == 1 ? (TileF<2, 2, false>::LDS + 1) / 2
                                        : Tile<2, 2, false, true>::LDS;
};

// over the block-lower tiles of the trailing nblk x nblk blocks from t0
// (both 128-tiles above the diagonal inside a diagonal NB-block included),
// block pairs (I, J) in row-major order from the p0-th on (p0 = skip (skip + 1)
// / 2 leaves out the blocks among the first `skip` block rows)
template <int MIX, int KS>
__global__ __launch_bounds__(256) void k_syr2k_lower(Fields F, double *S2, int64_t ld,
                                                     int64_t mofs, const double *A, int64_t t0,
                                                     int64_t kcol, const double *Y, int64_t ldy,
                                                     int64_t ymofs, int64_t sY, int64_t p0)
{
    __shared__ double lds[Syr2kLds<MIX>::N];
    const int64_t u = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t p = p0 + (u >> 2);
    const int s = u & 3;
    int64_t I = (int64_t)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= p)
        ++I;
    while (I * (I + 1) / 2 > p)
        --I;
    const int64_t J = p - I * (I + 1) / 2;
    const int64_t m0 = t0 + I * NB + 128 * (s >> 1), n0 = t0 + J * NB + 128 * (s & 1);
    const int m = blockIdx.y & 1, f = blockIdx.y >> 1; // matrix, field
    syr2k_tile<MIX, KS>(S2 + f * F.sS2 + m * mofs, ld, Y + f * sY + m * ymofs, ldy, A + f * F.sA,
                        kcol, m0, n0, lds);
}

// on a rectangle of rows x ncol from (r0, c0) (lookahead of the next block columns)
template <int MIX, int KS>
__global__ __launch_bounds__(256) void k_syr2k_rect(Fields F, double *S2, int64_t ld, int64_t mofs,
                                                    const double *A, int64_t r0, int64_t c0,
                                                    int64_t kcol, const double *Y, int64_t ldy,
                                                    int64_t ymofs, int64_t sY)
{
    __shared__ double lds[Syr2kLds<MIX>::N];
    const int64_t m0 = r0 + 128 * (int64_t)blockIdx.x, n0 = c0 + 128 * (int64_t)blockIdx.y;
    const int m = blockIdx.z & 1, f = blockIdx.z >> 1; // matrix, field
    syr2k_tile<MIX, KS>(S2 + f * F.sS2 + m * mofs, ld, Y + f * sY + m * ymofs, ldy, A + f * F.sA,
                        kcol, m0, n0, lds);
}

template <int KS>
static decltype(&k_syr2k_lower<0, KS>) syr2k_lower_kernel(int mixed)
{
    return mixed == 2 ? k_syr2k_lower<2, KS> : mixed == 1 ? k_syr2k_lower<1, KS> : k_syr2k_lower<0, KS>;
}
template <int KS>
static decltype(&k_syr2k_rect<0, KS>) syr2k_rect_kernel(int mixed)
{
    return mixed == 2 ? k_syr2k_rect<2, KS> : mixed == 1 ? k_syr2k_rect<1, KS> : k_syr2k_rect<0, KS>;
}

void launch_syr2k_lower(hipStream_t s, const Fields &F, double *S2, int64_t ld, int64_t mofs,
                        const double *A, int64_t t0, int nblk, int64_t kcol, int KS,
                        const double *Y, int64_t ldy, int64_t ymofs, int64_t sY, int skip,
                        int mixed)
{
    if (nblk <= skip || (KS != NB && KS != 2 * NB))
        return;
    // block pairs with I < skip come first in the enumeration: start past them
    const int64_t first = (int64_t)skip * (skip + 1) / 2;
    const int64_t pairs = (int64_t)nblk * (nblk + 1) / 2;
    const dim3 g((unsigned)(4 * (pairs - first)), (unsigned)(2 * F.count));
    hipLaunchKernelGGL(KS == NB ? syr2k_lower_kernel<NB>(mixed) : syr2k_lower_kernel<2 * NB>(mixed),
                       g, dim3(256), 0, s, F, S2, ld, mofs, A, t0, kcol, Y, ldy, ymofs, sY, first);
}

void launch_syr2k_rect(hipStream_t s, const Fields &F, double *S2, int64_t ld, int64_t mofs,
                       const double *A, int64_t r0, int64_t rows, int64_t c0, int64_t ncol,
                       int64_t kcol, int KS, const double *Y, int64_t ldy, int64_t ymofs,
                       int64_t sY, int mixed)
{
    if (rows <= 0 || ncol <= 0 || (KS != NB && KS != 2 * NB))
        return;
    const dim3 g((unsigned)(rows / 128), (unsigned)(ncol / 128), (unsigned)(2 * F.count));
    hipLaunchKernelGGL(KS == NB ? syr2k_rect_kernel<NB>(mixed) : syr2k_rect_kernel<2 * NB>(mixed), g,
                       dim3(256), 0, s, F, S2, ld, mofs, A, r0, c0, kcol, Y, ldy, ymofs, sY);
}

// Zero the NB x NB diagonal blocks k0, k0 + 1, .. of both matrices (blockIdx.x
// = block, y = matrix, z = field): after their block steps they hold spent
// S_kk, and the deferred solve reads block row k over columns up to (k + 1) NB.
__global__ __launch_bounds__(256) void k_zero_diag_blocks(Fields F, double *S2, int64_t ld,
                                                          int64_t mofs, int kfirst)
{
    const int64_t k0 = (int64_t)(kfirst + blockIdx.x) * NB;
    double *B = S2 + blockIdx.z * F.sS2 + blockIdx.y * mofs + k0 + k0 * ld;
    for (int c = 0; c < NB; ++c)
        B[threadIdx.x + c * ld] = 0.0;
}

void launch_zero_diag_blocks(hipStream_t s, const Fields &F, double *S2, int64_t ld, int64_t mofs,
                             int k0, int count)
{
    if (count <= 0)
        return;
    hipLaunchKernelGGL(k_zero_diag_blocks, dim3((unsigned)count, 2, F.count), dim3(256), 0, s, F,
                       S2, ld, mofs, k0);
}

// Trace reductions of the two-sided form over the block-lower NB-blocks
// (I >= J, one workgroup each, thread t on row t of the block): W is V_k * -2
// on a diagonal block (stored in full) and the deferred solve's result below
// it.  Over entries (a, b) with a, b < n:
//   t_i = sum W_i[a][a],  F_ij = sum w_ab W_i[a][b] W_j[a][b]
// with w_ab = 1 in a diagonal block and 2 below it, and u_i = W_i[n][n]
// (= y^T W_i y, the observation border).  Seven partial sums per workgroup
// go to partials[8 blockIdx.x + 0..6] (t_a, t_n, u_a, u_n, F_aa, F_an, F_nn).
__global__ __launch_bounds__(256) void k_sygst_reduce(Fields F, const double *S2, int64_t ld,
                                                      int64_t mofs, const double *Vd,
                                                      int64_t vofs, int64_t sVd, int64_t n1,
                                                      double *partials)
{
    __shared__ double sh[4];
    const int f = blockIdx.y;
    const int64_t n = F.n ? F.n[f] : n1;
    const int64_t p = blockIdx.x;
    int64_t I = (int64_t)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= p)
        ++I;
    while (I * (I + 1) / 2 > p)
        --I;
    const int64_t J = p - I * (I + 1) / 2;
    const int t = threadIdx.x;
    const int64_t a = I * NB + t;
    double s[7] = {0, 0, 0, 0, 0, 0, 0};
    if (I == J) {
        const double *Va = Vd + f * sVd + I * (NB * NB), *Vn = Va + vofs;
        for (int c = 0; c < NB; ++c) {
            const int64_t b = J * NB + c;
            const double wa = -2.0 * Va[t + c * NB], wn = -2.0 * Vn[t + c * NB];
            if (a < n && b < n) {
                s[4] = fma(wa, wa, s[4]);
                s[5] = fma(wa, wn, s[5]);
                s[6] = fma(wn, wn, s[6]);
                if (a == b) {
                    s[0] += wa;
                    s[1] += wn;
                }
            } else if (a == n && b == n) {
                s[2] = wa;
                s[3] = wn;
            }
        }
    } else if (a < n) {
        const double *Wa = S2 + f * F.sS2 + a + J * NB * ld, *Wn = Wa + mofs;
        const int64_t cend = n - J * NB < NB ? n - J * NB : NB;
        for (int64_t c = 0; c < cend; ++c) {
            const double wa = Wa[c * ld], wn = Wn[c * ld];
            s[4] = fma(2.0 * wa, wa, s[4]);
            s[5] = fma(2.0 * wa, wn, s[5]);
            s[6] = fma(2.0 * wn, wn, s[6]);
        }
    }
    for (int q = 0; q < 7; ++q) {
        const double v = block_sum(s[q], sh);
        if (t == 0)
            partials[f * F.sPart + 8 * p + q] = v;
    }
}

void launch_sygst_reduce(hipStream_t s, const Fields &F, const double *S2, int64_t ld,
                         int64_t mofs, const double *Vd, int64_t vofs, int64_t sVd, int T,
                         int64_t n, double *partials)
{
    const int64_t blocks = (int64_t)T * (T + 1) / 2;
    hipLaunchKernelGGL(k_sygst_reduce, dim3((unsigned)blocks, F.count), dim3(256), 0, s, F, S2,
                       ld, mofs, Vd, vofs, sVd, n, partials);
}

// Observations of the allocation-free entry point: x, y, z (npad each, zero
// past n) from the caller's device arrays (locations n x 2 row-major, z);
// flag[0] = 1 if any input is not finite, else 0.  One workgroup.
__global__ __launch_bounds__(256) void k_pack_data(const double *__restrict__ locs,
                                                   const double *__restrict__ zin, int64_t n,
                                                   int64_t npad, double *__restrict__ x,
                                                   double *__restrict__ y, double *__restrict__ z,
                                                   double *__restrict__ flag)
{
    __shared__ int bad;
    if (threadIdx.x == 0)
        bad = 0;
    __syncthreads();
    int b = 0;
    for (int64_t i = threadIdx.x; i < npad; i += 256) {
        double xi = 0.0, yi = 0.0, zi = 0.0;
        if (i < n) {
            xi = locs[2 * i];
            yi = locs[2 * i + 1];
            zi = zin[i];
            b |= !(isfinite(xi) && isfinite(yi) && isfinite(zi));
        }
        x[i] = xi;
        y[i] = yi;
        z[i] = zi;
    }
    if (b)
        atomicOr(&bad, 1);
    __syncthreads();
    if (threadIdx.x == 0)
        flag[0] = bad ? 1.0 : 0.0;
}

void launch_pack_data(hipStream_t s, const double *locs, const double *zin, int64_t n, int64_t npad,
                      double *x, double *y, double *z, double *flag)
{
    hipLaunchKernelGGL(k_pack_data, dim3(1), dim3(256), 0, s, locs, zin, n, npad, x, y, z, flag);
}

// ---------------------------------------------------------------------------
// Iterative refinement of w = Sigma^{-1} Z on a factor whose trailing updates
// ran in FP32 (FBT_MIXED_FP32_ALL): residuals r = Z - Sigma w in FP64 from a
// copy of Sigma taken before the factorisation, corrections from the factor
// by blocked triangular solves; and the quadratic forms w^T Sigma_i w from
// the derivative matrices.  The matrix-vector products are HBM-bound (one
// read of the matrix), the triangular solves latency-bound (one diagonal
// step and one update per block).
// ---------------------------------------------------------------------------

// Diagonal block step of the triangular solves: x_k <- Linv_k x_k (trans 0)
// or Linv_k^T x_k (trans 1), one workgroup of 1024 threads with x_k staged in
// LDS.  Linv_k's strict upper triangle is zero, so every row takes all 256
// products.  trans 0: thread (t, q) sums the 64 products of row t with j in
// [64 q, 64 q + 64) (a column slice is read coalesced over t), the four
// partial sums are added in order.  trans 1: output t is column t of Linv_k
// (contiguous) dotted with x_k; a wave takes 16 outputs, eight at a time with
// all their loads issued first, and sums each over its lanes in a fixed
// butterfly order.
constexpr int TRSV_DT = 1024;
__global__ __launch_bounds__(TRSV_DT) void k_trsv_diag(double *x, int64_t krow,
                                                       const double *__restrict__ Linv, int trans)
{
    __shared__ double xs[NB];
    __shared__ double part[4][NB];
    const int tid = threadIdx.x;
    if (tid < NB)
        xs[tid] = x[krow + tid];
    __syncthreads();
    if (!trans) {
        const int t = tid & (NB - 1), q = tid >> 8;
        const double *col = Linv + t + (int64_t)(64 * q) * NB;
        double v0 = 0.0, v1 = 0.0;
#pragma unroll 16
        for (int j = 0; j < 64; j += 2) {
            v0 = fma(col[(int64_t)j * NB], xs[64 * q + j], v0);
            v1 = fma(col[(int64_t)(j + 1) * NB], xs[64 * q + j + 1], v1);
        }
        part[q][t] = v0 + v1;
        __syncthreads();
        if (tid < NB)
            x[krow + tid] = ((part[0][tid] + part[1][tid]) + part[2][tid]) + part[3][tid];
    } else {
        const int lane = tid & 63, wv = tid >> 6;
        const double x0 = xs[lane], x1 = xs[lane + 64], x2 = xs[lane + 128], x3 = xs[lane + 192];
        for (int h = 0; h < 2; ++h) {
            const int t0 = 16 * wv + 8 * h;
            double c[8][4];
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int m = 0; m < 4; ++m)
                    c[u][m] = Linv[lane + 64 * m + (int64_t)(t0 + u) * NB];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                double v = fma(c[u][0], x0, c[u][1] * x1);
                v = fma(c[u][2], x2, v);
                v = fma(c[u][3], x3, v);
#pragma unroll
                for (int off = 32; off > 0; off >>= 1)
                    v += __shfl_xor(v, off, 64);
                if (lane == 0)
                    part[0][t0 + u] = v;
            }
        }
        __syncthreads();
        if (tid < NB)
            x[krow + tid] = part[0][tid];
    }
}

// Forward update: x[r] -= sum_j L[r][krow + j] x[krow + j] for rows r0 <= r <
// npad.  A workgroup takes 64 rows; thread (r, q) sums the 64 products with j
// in [64 q, 64 q + 64) (coalesced over r), the four partial sums are added in
// order.
__global__ __launch_bounds__(256) void k_trsv_update(double *x, const double *__restrict__ L,
                                                     int64_t ld, int64_t krow, int64_t r0,
                                                     int64_t npad)
{
    __shared__ double xs[NB];
    __shared__ double part[4][64];
    const int t = threadIdx.x, rl = t & 63, q = t >> 6;
    xs[t] = x[krow + t];
    __syncthreads();
    const int64_t r = r0 + (int64_t)blockIdx.x * 64 + rl;
    double v0 = 0.0, v1 = 0.0;
    if (r < npad) {
        const double *row = L + r + (krow + 64 * q) * ld;
#pragma unroll 16
        for (int j = 0; j < 64; j += 2) {
            v0 = fma(row[(int64_t)j * ld], xs[64 * q + j], v0);
            v1 = fma(row[(int64_t)(j + 1) * ld], xs[64 * q + j + 1], v1);
        }
    }
    part[q][rl] = v0 + v1;
    __syncthreads();
    if (t < 64 && r < npad)
        x[r] -= ((part[0][t] + part[1][t]) + part[2][t]) + part[3][t];
}

// Backward update of x = L^{-T} x after block k is solved: x[c] -= sum_i
// L[krow + i][c] x[krow + i] for columns c < krow.  A wave takes TRSV_CPW
// columns: its lanes read each column's 256 entries of the block row (four
// coalesced loads, all columns' loads issued first), and each column's
// products are summed in a fixed order (the four loads, then a butterfly over
// the lanes).  Four waves per workgroup.
constexpr int TRSV_CPW = 8;
__global__ __launch_bounds__(256) void k_trsv_update_t(double *x, const double *__restrict__ L,
                                                       int64_t ld, int64_t krow)
{
    __shared__ double xs[NB];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    xs[t] = x[krow + t];
    __syncthreads();
    const double x0 = xs[lane], x1 = xs[lane + 64], x2 = xs[lane + 128], x3 = xs[lane + 192];
    const int64_t c0 = ((int64_t)blockIdx.x * 4 + wv) * TRSV_CPW;
    double e[TRSV_CPW][4];
#pragma unroll
    for (int j = 0; j < TRSV_CPW; ++j) {
        const int64_t c = c0 + j < krow ? c0 + j : krow - 1; // in bounds; not stored
        const double *col = L + krow + c * ld;
#pragma unroll
        for (int m = 0; m < 4; ++m)
            e[j][m] = col[lane + 64 * m];
    }
#pragma unroll
    for (int j = 0; j < TRSV_CPW; ++j) {
        double v = fma(e[j][0], x0, e[j][1] * x1);
        v = fma(e[j][2], x2, v);
        v = fma(e[j][3], x3, v);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
            v += __shfl_xor(v, off, 64);
        if (lane == 0 && c0 + j < krow)
            x[c0 + j] -= v;
    }
}

void launch_trsv(hipStream_t s, double *x, const double *L, int64_t ld, int64_t npad,
                 const double *Linv, int trans)
{
    const int T = (int)(npad / NB);
    if (!trans) {
        for (int k = 0; k < T; ++k) {
            const int64_t krow = (int64_t)k * NB;
            hipLaunchKernelGGL(k_trsv_diag, dim3(1), dim3(TRSV_DT), 0, s, x, krow,
                               Linv + (int64_t)k * NB * NB, 0);
            if (krow + NB < npad)
                hipLaunchKernelGGL(k_trsv_update, dim3((unsigned)((npad - krow - NB + 63) / 64)),
                                   dim3(256), 0, s, x, L, ld, krow, krow + NB, npad);
        }
    } else {
        for (int k = T - 1; k >= 0; --k) {
            const int64_t krow = (int64_t)k * NB;
            hipLaunchKernelGGL(k_trsv_diag, dim3(1), dim3(TRSV_DT), 0, s, x, krow,
                               Linv + (int64_t)k * NB * NB, 1);
            if (krow > 0)
                hipLaunchKernelGGL(k_trsv_update_t,
                                   dim3((unsigned)((krow + 4 * TRSV_CPW - 1) / (4 * TRSV_CPW))),
                                   dim3(256), 0, s, x, L, ld, krow);
        }
    }
}

// Sc = Sigma on rows and columns < n, both triangles, from the generated
// lower triangle of A (before the factorisation overwrites it).  One 64 x 64
// tile pair (ti >= tj) per workgroup, staged in LDS so that the mirrored
// tile is written with coalesced stores; a diagonal tile takes its upper
// part from its lower one.
__global__ __launch_bounds__(256) void k_copy_sym(const double *A, int64_t ld, int64_t n,
                                                  double *Sc)
{
    __shared__ double T[64][65];
    const int64_t p = blockIdx.x;
    int64_t ti = (int64_t)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= p)
        ++ti;
    while (ti * (ti + 1) / 2 > p)
        --ti;
    const int64_t tj = p - ti * (ti + 1) / 2;
    const int64_t a0 = ti * 64, b0 = tj * 64;
    const int t = threadIdx.x, r = t & 63;
    for (int cc = t >> 6; cc < 64; cc += 4) {
        const int64_t a = a0 + r, b = b0 + cc;
        double v = 0.0;
        if (a < n && b < n)
            v = (ti == tj && r < cc) ? A[b + a * ld] : A[a + b * ld];
        T[r][cc] = v;
    }
    __syncthreads();
    for (int cc = t >> 6; cc < 64; cc += 4) {
        const int64_t a = a0 + r, b = b0 + cc;
        if (a < n && b < n)
            Sc[a + b * ld] = T[r][cc];
        // mirrored tile: row b0 + r, column a0 + cc holds T[cc][r]
        const int64_t a2 = b0 + r, b2 = a0 + cc;
        if (ti != tj && a2 < n && b2 < n)
            Sc[a2 + b2 * ld] = T[cc][r];
    }
}

void launch_copy_sym(hipStream_t s, const double *A, int64_t ld, int64_t n, double *Sc)
{
    const int64_t nt = (n + 63) / 64, pairs = nt * (nt + 1) / 2;
    hipLaunchKernelGGL(k_copy_sym, dim3((unsigned)pairs), dim3(256), 0, s, A, ld, n, Sc);
}

// Partial products part[a + npad q] = sum over the q-th of nq column chunks
// of M[a][b] w[b] (a, b < n; M column-major, both triangles stored).  One
// thread per row; the rows of a workgroup read each column coalesced.
__global__ __launch_bounds__(256) void k_matvec_part(const double *__restrict__ M, int64_t ld,
                                                     int64_t n, int64_t npad,
                                                     const double *__restrict__ w, int nq,
                                                     double *__restrict__ part)
{
    const int64_t a = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t clen = (n + nq - 1) / nq, b0 = (int64_t)blockIdx.y * clen;
    const int64_t b1 = b0 + clen < n ? b0 + clen : n;
    if (a >= n)
        return;
    // four accumulators (columns b mod 4), added in a fixed order
    double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
    int64_t b = b0;
#pragma unroll 2
    for (; b + 3 < b1; b += 4) {
        v0 = fma(M[a + b * ld], w[b], v0);
        v1 = fma(M[a + (b + 1) * ld], w[b + 1], v1);
        v2 = fma(M[a + (b + 2) * ld], w[b + 2], v2);
        v3 = fma(M[a + (b + 3) * ld], w[b + 3], v3);
    }
    for (; b < b1; ++b)
        v0 = fma(M[a + b * ld], w[b], v0);
    part[a + npad * (int64_t)blockIdx.y] = (v0 + v1) + (v2 + v3);
}

// r[a] = z[a] - sum_q part[a + npad q] (a < n; 0 beyond), the chunks in order.
__global__ __launch_bounds__(256) void k_residual(const double *z, const double *part, int nq,
                                                  int64_t n, int64_t npad, double *r)
{
    const int64_t a = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (a >= npad)
        return;
    double v = 0.0;
    if (a < n)
        for (int q = 0; q < nq; ++q)
            v += part[a + npad * q];
    r[a] = a < n ? z[a] - v : 0.0;
}

void launch_residual(hipStream_t s, const double *Sc, int64_t ld, int64_t n, int64_t npad,
                     const double *z, const double *w, int nq, double *part, double *r)
{
    hipLaunchKernelGGL(k_matvec_part, dim3((unsigned)((n + 255) / 256), (unsigned)nq), dim3(256),
                       0, s, Sc, ld, n, npad, w, nq, part);
    hipLaunchKernelGGL(k_residual, dim3((unsigned)((npad + 255) / 256)), dim3(256), 0, s, z, part,
                       nq, n, npad, r);
}

// out[0] = sum_a w[a] (sum_q part[a + npad q]) over a < n: w^T M w from the
// partial products (one workgroup, fixed order)
__global__ __launch_bounds__(256) void k_quad_form(const double *w, const double *part, int nq,
                                                   int64_t n, int64_t npad, double *out)
{
    __shared__ double sh[4];
    double v = 0.0;
    for (int64_t a = threadIdx.x; a < n; a += 256) {
        double m = 0.0;
        for (int q = 0; q < nq; ++q)
            m += part[a + npad * q];
        v = fma(w[a], m, v);
    }
    v = block_sum(v, sh);
    if (threadIdx.x == 0)
        out[0] = v;
}

void launch_quad_form(hipStream_t s, const double *M, int64_t ld, int64_t n, int64_t npad,
                      const double *w, int nq, double *part, double *out)
{
    hipLaunchKernelGGL(k_matvec_part, dim3((unsigned)((n + 255) / 256), (unsigned)nq), dim3(256),
                       0, s, M, ld, n, npad, w, nq, part);
    hipLaunchKernelGGL(k_quad_form, dim3(1), dim3(256), 0, s, w, part, nq, n, npad, out);
}

// w[b] = A[n + b ld] (b < n), 0 for n <= b < npad: y = L^{-1} Z from the
// bordered factor's row n
__global__ __launch_bounds__(256) void k_border_row(const double *A, int64_t ld, int64_t n,
                                                    int64_t npad, double *w)
{
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (b < npad)
        w[b] = b < n ? A[n + b * ld] : 0.0;
}

void launch_border_row(hipStream_t s, const double *A, int64_t ld, int64_t n, int64_t npad,
                       double *w)
{
    hipLaunchKernelGGL(k_border_row, dim3((unsigned)((npad + 255) / 256)), dim3(256), 0, s, A, ld,
                       n, npad, w);
}

// x[a] = 0 for n <= a < npad: between the forward and the backward solve with
// the bordered factor, whose row n (y^T, 1) must not feed back into x[< n]
__global__ __launch_bounds__(256) void k_zero_tail(double *x, int64_t n, int64_t npad)
{
    const int64_t a = n + (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (a < npad)
        x[a] = 0.0;
}

void launch_solve_sigma(hipStream_t s, double *x, const double *L, int64_t ld, int64_t n,
                        int64_t npad, const double *Linv)
{
    launch_trsv(s, x, L, ld, npad, Linv, 0);
    hipLaunchKernelGGL(k_zero_tail, dim3((unsigned)((npad - n + 255) / 256)), dim3(256), 0, s, x, n,
                       npad);
    launch_trsv(s, x, L, ld, npad, Linv, 1);
}

// x[a] += d[a] (a < npad); out[0] = sum_a z[a] x[a] over a < n when out is set
// (one workgroup, fixed order)
__global__ __launch_bounds__(256) void k_axpy_dot(double *x, const double *d, const double *z,
                                                  int64_t n, int64_t npad, double *out)
{
    __shared__ double sh[4];
    double v = 0.0;
    for (int64_t a = threadIdx.x; a < npad; a += 256) {
        const double xa = d ? x[a] + d[a] : x[a];
        x[a] = xa;
        if (a < n)
            v = fma(z[a], xa, v);
    }
    v = block_sum(v, sh);
    if (out && threadIdx.x == 0)
        out[0] = v;
}

void launch_axpy_dot(hipStream_t s, double *x, const double *d, const double *z, int64_t n,
                     int64_t npad, double *out)
{
    hipLaunchKernelGGL(k_axpy_dot, dim3(1), dim3(256), 0, s, x, d, z, n, npad, out);
}

// ---------------------------------------------------------------------------
// Adjoint gradient (score without the W matrices).  With w = Sigma^{-1} Z,
//   dl/dtheta_i = 1/2 w^T Sigma_i w - 1/2 tr(Sigma^{-1} Sigma_i)
//               = sum_ab (1/2 w_a w_b - 1/2 (Sigma^{-1})_ab) (Sigma_i)_ab,
// the Frobenius product of Sigma_i with 1/2 (w w^T - Sigma^{-1}) (Eq. (2)
// with tr(A B) = <A, B^T>_F), so Sigma_i is regenerated entry by entry and is
// never stored.  Sigma^{-1} comes from X = L'^{-1}: the bordered factor
// [[L, 0], [y^T, 1]] has the inverse [[L^{-1}, 0], [-w^T, 1]] (row n is
// -(L^{-T} y)^T), so P = X^T X restricted to a, b < n is Sigma^{-1} + w w^T
// and the weight of entry (a, b) is w_a w_b - P_ab / 2.
// ---------------------------------------------------------------------------

// X[0:rows, 0:ncols] = identity
__global__ __launch_bounds__(256) void k_fill_identity(double *X, int64_t ld, int64_t rows,
                                                       int64_t ncols)
{
    const int64_t total = rows * ncols;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * 256) {
        const int64_t r = i % rows, c = i / rows;
        X[r + c * ld] = (r == c) ? 1.0 : 0.0;
    }
}

void launch_fill_identity(hipStream_t s, double *X, int64_t ld, int64_t rows, int64_t ncols)
{
    if (rows <= 0 || ncols <= 0)
        return;
    hipLaunchKernelGGL(k_fill_identity, dim3(4096), dim3(256), 0, s, X, ld, rows, ncols);
}

// P = X^T X on the block-lower 128 x 128 tiles of the leading ncols x ncols
// part, X lower triangular (npad x ncols):
//   P[m0 + i][n0 + j] = sum_{k >= m0} X[k][m0 + i] X[k][n0 + j],
// rows k < m0 being zero in column m0 + i.  Tiles starting at or beyond ncols
// and the strictly upper 128-tile of each diagonal block are skipped.  Tile
// pairs are enumerated with the block row ascending, so the longest sums
// start first.
__global__ __launch_bounds__(256) void k_lauum(double *P, const double *X, int64_t ld,
                                               int64_t npad, int64_t ncols)
{
    using TL = Tile<2, 2, true, false, true>;
    __shared__ double lds[TL::LDS];
    const int64_t p = blockIdx.x >> 2;
    const int s = blockIdx.x & 3;
    int64_t I = (int64_t)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= p)
        ++I;
    while (I * (I + 1) / 2 > p)
        --I;
    const int64_t J = p - I * (I + 1) / 2;
    const int64_t m0 = I * NB + 128 * (s >> 1), n0 = J * NB + 128 * (s & 1);
    if (m0 >= ncols || n0 >= ncols || n0 > m0)
        return;
    d4 acc[4][4];
    TL::zero(acc);
    TL::run(acc, X + m0 + m0 * ld, ld, X + m0 + n0 * ld, ld, (int)(npad - m0), lds);
    TL::store_c(acc, P + m0 + n0 * ld, ld);
}

void launch_lauum(hipStream_t s, double *P, const double *X, int64_t ld, int64_t npad,
                  int64_t ncols)
{
    const int64_t T = npad / NB;
    const int64_t pairs = T * (T + 1) / 2;
    hipLaunchKernelGGL(k_lauum, dim3((unsigned)(4 * pairs)), dim3(256), 0, s, P, X, ld, npad,
                       ncols);
}

// w[a] = -X[n][a] = (Sigma^{-1} Z)_a for a < n
__global__ __launch_bounds__(256) void k_extract_w(const double *X, int64_t ld, int64_t n,
                                                   double *w)
{
    const int64_t a = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (a < n)
        w[a] = -X[n + a * ld];
}

void launch_extract_w(hipStream_t s, const double *X, int64_t ld, int64_t n, double *w)
{
    hipLaunchKernelGGL(k_extract_w, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, X, ld,
                       n, w);
}

// Per 64 x 64 tile pair (ti >= tj) of the strictly lower triangle a > b
// (a, b < n): 2 sum (w_a w_b - P_ab / 2) (Sigma_alpha)_ab and the same with
// Sigma_nu, with the derivative entries regenerated as in k_gen.  The factor 2
// counts the mirrored entry; the diagonal contributes nothing (both
// derivatives vanish at distance 0).  Two partials per workgroup.
__global__ __launch_bounds__(256) void k_adjoint(GenParams gp, const double *__restrict__ xs,
                                                 const double *__restrict__ ys,
                                                 const Node *__restrict__ gtab,
                                                 const double *__restrict__ P,
                                                 const double *__restrict__ w,
                                                 double *__restrict__ part)
{
    __shared__ Node tab[TAB_MAX];
    __shared__ double sh[4];
    const int t = threadIdx.x;
    const int ntab = gp.off[NLEV - 1] + gp.len[NLEV - 1];
    for (int i = t; i < ntab; i += 256)
        tab[i] = gtab[i];
    const int64_t p = blockIdx.x;
    int64_t ti = (int64_t)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= p)
        ++ti;
    while (ti * (ti + 1) / 2 > p)
        --ti;
    const int64_t tj = p - ti * (ti + 1) / 2;
    const bool diag = (ti == tj);
    const int al = t & 63;
    const int64_t a = ti * GT + al;
    const int64_t n = gp.n, ld = gp.ld;
    const double xa = a < n ? xs[a] : 0.0, ya = a < n ? ys[a] : 0.0, wa = a < n ? w[a] : 0.0;
    const double inv_alpha = 1.0 / gp.alpha;
    __syncthreads();
    double sa = 0.0, sn = 0.0;
#pragma unroll 1
    for (int e = 0; e < 16; ++e) {
        const int bl = (t >> 6) * 16 + e;
        const int64_t b = tj * GT + bl;
        if (a >= n || b >= n || (diag && al <= bl))
            continue;
        const double dx = xa - xs[b], dy = ya - ys[b];
        double c, ca, cn;
        matern3(gp, tab, sqrt(dx * dx + dy * dy) * inv_alpha, GEN_DERIV, c, ca, cn);
        const double g = fma(wa, w[b], -0.5 * P[a + b * ld]);
        sa = fma(g, ca, sa);
        sn = fma(g, cn, sn);
    }
    sa = block_sum(sa, sh);
    sn = block_sum(sn, sh);
    if (t == 0) {
        part[2 * p] = 2.0 * sa;
        part[2 * p + 1] = 2.0 * sn;
    }
}

void launch_adjoint(hipStream_t s, const GenParams &gp, const double *xs, const double *ys,
                    const Node *tab, const double *P, const double *w, double *part)
{
    const int64_t nt = (gp.n + GT - 1) / GT;
    const int64_t pairs = nt * (nt + 1) / 2;
    hipLaunchKernelGGL(k_adjoint, dim3((unsigned)pairs), dim3(256), 0, s, gp, xs, ys, tab, P, w,
                       part);
}

// out[0..1] = sums of the `count` partial pairs, in a fixed order
__global__ __launch_bounds__(256) void k_reduce_pairs(const double *part, int64_t count,
                                                      double *out)
{
    __shared__ double sh[4];
    const int t = threadIdx.x;
    for (int q = 0; q < 2; ++q) {
        double v = 0.0;
        for (int64_t g = t; g < count; g += 256)
            v += part[2 * g + q];
        v = block_sum(v, sh);
        if (t == 0)
            out[q] = v;
    }
}

void launch_reduce_pairs(hipStream_t s, const double *part, int64_t count, double *out)
{
    hipLaunchKernelGGL(k_reduce_pairs, dim3(1), dim3(256), 0, s, part, count, out);
}

}  // namespace fbt
