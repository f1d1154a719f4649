// Task graph of one batched round: every field's evaluation (Algorithm 2 or 3)
// as tile tasks of one persistent kernel.  Plain C++ shared by the kernel and
// the host planner (and its host-only tests): task encoding, the dependency
// counters each task waits on and the counters it advances.
//
// Per field with T tiles of BT rows (bordered order npad = T BT, Section 2's
// covariance plus the observation row, as in the single-field path):
//   GEN(i, j)     i >= j: tile (i, j) of Sigma' and, for Algorithm 3, tiles
//                 (i, j) and (j, i) of Sigma_alpha and Sigma_nu
//   CHOL(i, j)    i >= j: tile (i, j) of the factor L' (left-looking: the
//                 tile minus the product of the finished block columns < j,
//                 then the diagonal factorisation and its inverse for i = j,
//                 or the product with the inverse of L_jj^T for i > j)
//   LSOLVE(k, c)  tile (k, c) of X = L'^{-1} [Sigma_alpha' | Sigma_nu'],
//                 c < 2T (forward substitution down tile column c)
//   RSOLVE(i, j)  i >= j: tile (i, j) of W_alpha and W_nu = X L'^{-T}
//                 (in place of X), with its share of tr W, y^T W y and the
//                 Frobenius products (Eqs. (2), (3), (5))
//   REDUCE        the field's nine terms in a fixed order
// A task waits until counters of its field reach given values; every counter
// only grows and is advanced by the tasks listed in the comments below.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define FBT_HD __host__ __device__
#else
#define FBT_HD
#endif

namespace fbt {

enum RType { R_GEN = 0, R_CHOL = 1, R_LSOLVE = 2, R_RSOLVE = 3, R_REDUCE = 4 };

struct RTask {
    int32_t ft; // field << 3 | type
    int32_t ij; // i << 16 | j
};

FBT_HD inline RTask rtask(int field, int type, int i, int j)
{
    RTask t;
    t.ft = (field << 3) | type;
    t.ij = (i << 16) | j;
    return t;
}
FBT_HD inline int rt_field(RTask t) { return t.ft >> 3; }
FBT_HD inline int rt_type(RTask t) { return t.ft & 7; }
FBT_HD inline int rt_i(RTask t) { return t.ij >> 16; }
FBT_HD inline int rt_j(RTask t) { return t.ij & 0xffff; }

// index of tile pair (i, j), i >= j, in the lower triangle
FBT_HD inline int rpair(int i, int j) { return i * (i + 1) / 2 + j; }

// Offsets of a field's counters (int32) for T tiles.
struct RCount {
    int gen;  // T(T+1)/2: 1 once GEN(i, j) is done
    int col;  // T: finished CHOL tiles of tile column j (complete at T - j)
    int diag; // T: 1 once CHOL(j, j) (factor and inverse of L_jj) is done
    int xd;   // 2T: finished LSOLVE tiles of column c (they finish in row order)
    int wd;   // T: finished RSOLVE tiles of tile row i (they finish in column order)
    int wtot; // 1: finished RSOLVE tiles
    int info; // 1: 0, or 1 + the first row whose pivot failed (not a counter)
    int size;
};

FBT_HD inline RCount rcount(int T)
{
    RCount c;
    c.gen = 0;
    c.col = c.gen + T * (T + 1) / 2;
    c.diag = c.col + T;
    c.xd = c.diag + T;
    c.wd = c.xd + 2 * T;
    c.wtot = c.wd + T;
    c.info = c.wtot + 1;
    c.size = (c.info + 1 + 63) / 64 * 64;
    return c;
}

// What task t of a field (T tiles, mode 1 = Algorithm 2, 2 = Algorithm 3)
// waits for: counter off[k] >= need[k], k < return value.  CHOL(i, j), i > j,
// takes its last wait (the diagonal tile) only before the product with the
// inverse; the order of the waits is the order of the arrays.
FBT_HD inline int rdeps(RTask t, int T, int mode, int *off, int *need)
{
    const RCount c = rcount(T);
    const int i = rt_i(t), j = rt_j(t);
    int k = 0;
    switch (rt_type(t)) {
    case R_GEN:
        break;
    case R_CHOL:
        off[k] = c.gen + rpair(i, j), need[k++] = 1;
        if (j > 0)
            off[k] = c.col + j - 1, need[k++] = T - j + 1; // block columns < j finished
        if (i > j)
            off[k] = c.diag + j, need[k++] = 1;
        break;
    case R_LSOLVE: {
        const int cc = j % T; // tile column of Sigma_alpha or Sigma_nu
        off[k] = c.gen + (i >= cc ? rpair(i, cc) : rpair(cc, i)), need[k++] = 1;
        off[k] = c.diag + i, need[k++] = 1; // L' rows of tile row i and L_ii^{-1}
        if (i > 0)
            off[k] = c.xd + j, need[k++] = i; // X tiles above in column j
        break;
    }
    case R_RSOLVE:
        // X columns j of both matrices solved (this tile's input, and every
        // reader of the X tiles that the W tiles overwrite is done)
        off[k] = c.xd + j, need[k++] = T;
        off[k] = c.xd + T + j, need[k++] = T;
        if (j > 0)
            off[k] = c.wd + i, need[k++] = j; // W tiles left of it in row i
        break;
    case R_REDUCE:
        if (mode == 2)
            off[k] = c.wtot, need[k++] = T * (T + 1) / 2;
        else
            off[k] = c.diag + T - 1, need[k++] = 1;
        break;
    }
    return k;
}

// Counters task t advances by one when it is done.
FBT_HD inline int rpublish(RTask t, int T, int *off)
{
    const RCount c = rcount(T);
    const int i = rt_i(t), j = rt_j(t);
    int k = 0;
    switch (rt_type(t)) {
    case R_GEN:
        off[k++] = c.gen + rpair(i, j);
        break;
    case R_CHOL:
        off[k++] = c.col + j;
        if (i == j)
            off[k++] = c.diag + j;
        break;
    case R_LSOLVE:
        off[k++] = c.xd + j;
        break;
    case R_RSOLVE:
        off[k++] = c.wd + i;
        off[k++] = c.wtot;
        break;
    default:
        break;
    }
    return k;
}

// Slots of a field's partial sums (doubles, one 128-byte line per slot, since
// different workgroups write neighbouring slots): the log-det partial of each
// diagonal tile, then seven per RSOLVE tile (tr_a, tr_n, u_a, u_n, F_aa, F_an,
// F_nn).
struct RPart {
    int logdet; // 16 T
    int wpart;  // 16 T(T+1)/2
    int size;
};

FBT_HD inline RPart rpart(int T)
{
    RPart p;
    p.logdet = 0;
    p.wpart = 16 * T;
    p.size = p.wpart + 16 * (T * (T + 1) / 2);
    return p;
}

} // namespace fbt
