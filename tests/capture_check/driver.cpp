// Drives the library, linked against the recording stand-in of the HIP
// runtime (hip_record.cpp), through the calls whose stream, event, copy and
// graph usage is to be checked, and prints the stand-in's report.  Exit code:
// the number of violations (0: none), 100 + k for a library call that failed.
//
//   batch graph   fbt_batch_eval with the graph execution: groups of several
//                 padded orders in all modes, captured once, replayed with new
//                 theta, re-captured when the modes change, then destroyed;
//   batch workers the same fields with the worker pool (no capture);
//   context       fbt_eval, fbt_loglik, fbt_grad and fbt_eval_noalloc on one
//                 context, in FP64 and in each mixed precision.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "fisherbt.h"

extern "C" int hiprec_report(FILE *f);
extern "C" long hiprec_captures(void);
extern "C" long hiprec_graph_launches(void);

static void fields(int nf, std::vector<int64_t> &n, std::vector<std::vector<double>> &locs,
                   std::vector<std::vector<double>> &z)
{
    // padded orders 256, 512, 768, 1024 and 3072 (n + 1 rounded up to a
    // multiple of 256), including n + 1 = 256 exactly; 3,000 gives twelve
    // block steps (six pairs) in every phase
    const int64_t sizes[] = {200, 300, 600, 255, 256, 900, 3000, 520};
    uint64_t s = 12345;
    auto u = [&]() {
        s = s * 6364136223846793005ull + 1442695040888963407ull;
        return (double)(s >> 11) * (1.0 / 9007199254740992.0);
    };
    n.resize(nf);
    locs.resize(nf);
    z.resize(nf);
    for (int f = 0; f < nf; ++f) {
        n[f] = sizes[f % 8];
        locs[f].resize(2 * n[f]);
        z[f].resize(n[f]);
        for (int64_t i = 0; i < n[f]; ++i) {
            locs[f][2 * i] = u();
            locs[f][2 * i + 1] = u();
            z[f][i] = u() - 0.5;
        }
    }
}

#define CALL(k, expr)                                                                              \
    do {                                                                                           \
        const fbt_status st_ = (expr);                                                             \
        if (st_ != FBT_OK) {                                                                       \
            std::fprintf(stderr, "call failed (%d): %s\n", (int)st_, #expr);                      \
            hiprec_report(stderr);                                                                 \
            return 100 + (k);                                                                      \
        }                                                                                          \
    } while (0)

static int batch(int exec)
{
    const int nf = 16;
    std::vector<int64_t> n;
    std::vector<std::vector<double>> locs, z;
    fields(nf, n, locs, z);
    std::vector<const double *> pl(nf), pz(nf);
    for (int f = 0; f < nf; ++f) {
        pl[f] = locs[f].data();
        pz[f] = z[f].data();
    }
    fbt_config cfg;
    std::memset(&cfg, 0, sizeof(cfg));
    fbt_batch *b = nullptr;
    CALL(1, fbt_batch_create(&cfg, 3, &b));
    CALL(2, fbt_batch_set_fields(b, nf, n.data(), pl.data(), pz.data()));
    CALL(3, fbt_batch_set_exec(b, exec));
    std::vector<double> th(3 * nf), ll(nf), sc(3 * nf), fi(9 * nf);
    std::vector<int32_t> mode(nf), st(nf);
    for (int f = 0; f < nf; ++f)
        mode[f] = f % 4; // skip, loglik, eval, adjoint
    for (int call = 0; call < 4; ++call) {
        for (int f = 0; f < nf; ++f) {
            th[3 * f] = 1.0 + 0.1 * call;
            th[3 * f + 1] = 0.05 + 0.01 * f;
            th[3 * f + 2] = 0.5 + 0.05 * call;
        }
        if (call == 2) // new modes: the graph is captured again
            for (int f = 0; f < nf; ++f)
                mode[f] = 1 + (f % 2);
        CALL(4, fbt_batch_eval(b, th.data(), mode.data(), ll.data(), sc.data(), fi.data(),
                               st.data()));
    }
    // a group limit change also rebuilds
    CALL(5, fbt_batch_set_group_limit(b, 512, 1));
    CALL(6, fbt_batch_eval(b, th.data(), mode.data(), ll.data(), sc.data(), fi.data(), st.data()));
    fbt_batch_destroy(b);
    return 0;
}

static int context()
{
    std::vector<int64_t> n;
    std::vector<std::vector<double>> locs, z;
    fields(3, n, locs, z);
    const double th[3] = {1.0, 0.1, 0.5};
    const int precisions[] = {FBT_FP64, FBT_MIXED_FP32, FBT_MIXED_BF16, FBT_MIXED_FP32_ALL};
    for (int p : precisions) {
        fbt_config cfg;
        std::memset(&cfg, 0, sizeof(cfg));
        cfg.precision = p;
        fbt_ctx *c = nullptr;
        CALL(10, fbt_create(&cfg, &c));
        for (int f = 0; f < 3; ++f) {
            double ll, sc[3], fi[9], g[3];
            CALL(11, fbt_set_data(c, n[f], locs[f].data(), z[f].data()));
            CALL(12, fbt_eval(c, th, &ll, sc, fi));
            CALL(13, fbt_loglik(c, th, &ll));
            CALL(14, fbt_eval(c, th, &ll, sc, fi)); // on the log-likelihood's factor
            CALL(15, fbt_grad(c, th, &ll, g, nullptr));
        }
        fbt_destroy(c);
    }
    // the allocation-free entry point on a stream of the caller's
    hipStream_t s;
    double *dl = nullptr, *dz = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
        hipMalloc((void **)&dl, 2 * n[1] * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&dz, n[1] * sizeof(double)) != hipSuccess ||
        hipMemcpyAsync(dl, locs[1].data(), 2 * n[1] * sizeof(double), hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipMemcpyAsync(dz, z[1].data(), n[1] * sizeof(double), hipMemcpyHostToDevice, s) !=
            hipSuccess)
        return 120;
    double ll, sc[3], fi[9];
    for (int rep = 0; rep < 2; ++rep) {
        // its scratch is a device variable, not filled like allocated memory:
        // the factorisation reads as failed, which ends the call normally
        const fbt_status st = fbt_eval_noalloc(0, s, n[1] - 50 * rep, dl, dz, th, &ll, sc, fi);
        if (st != FBT_OK && st != FBT_ENOTPD)
            return 116;
    }
    (void)hipFree(dl);
    (void)hipFree(dz);
    (void)hipStreamDestroy(s);
    return 0;
}

// The persistent execution with its round graph: captured at the first call
// for a field set and modes, replayed by the next, captured again for new
// modes.  The round kernel does not run under the stand-in, so the calls
// report the undrained round (FBT_EDEVICE); the calls themselves are checked.
static int persistent()
{
    const int nf = 6;
    std::vector<int64_t> n;
    std::vector<std::vector<double>> locs, z;
    fields(nf, n, locs, z);
    std::vector<const double *> pl(nf), pz(nf);
    for (int f = 0; f < nf; ++f) {
        pl[f] = locs[f].data();
        pz[f] = z[f].data();
    }
    fbt_config cfg;
    std::memset(&cfg, 0, sizeof(cfg));
    fbt_batch *b = nullptr;
    CALL(30, fbt_batch_create(&cfg, 1, &b));
    CALL(31, fbt_batch_set_fields(b, nf, n.data(), pl.data(), pz.data()));
    CALL(32, fbt_batch_set_exec(b, FBT_BATCH_PERSISTENT));
    CALL(33, fbt_batch_set_round_graph(b, 1));
    std::vector<double> th(3 * nf), ll(nf), sc(3 * nf), fi(9 * nf);
    std::vector<int32_t> mode(nf), st(nf);
    for (int call = 0; call < 3; ++call) {
        for (int f = 0; f < nf; ++f) {
            th[3 * f] = 1.0 + 0.1 * call;
            th[3 * f + 1] = 0.05 + 0.01 * f;
            th[3 * f + 2] = 0.5;
            mode[f] = call < 2 ? 1 + (f % 2) : 2;
        }
        const fbt_status r =
            fbt_batch_eval(b, th.data(), mode.data(), ll.data(), sc.data(), fi.data(), st.data());
        if (r != FBT_OK && r != FBT_EDEVICE)
            return 34;
    }
    fbt_batch_destroy(b);
    return 0;
}

int main()
{
    int r;
    if ((r = batch(FBT_BATCH_GRAPH)) != 0)
        return r;
    const long captures = hiprec_captures(), launches = hiprec_graph_launches();
    std::printf("batch graph: %ld captures, %ld graph launches\n", captures, launches);
    if (captures < 3 || launches < 5) {
        std::printf("the graph execution did not run as expected\n");
        return 99;
    }
    if ((r = batch(FBT_BATCH_WORKERS)) != 0)
        return r;
    if ((r = persistent()) != 0)
        return r;
    std::printf("persistent round graph: %ld captures, %ld graph launches\n",
                hiprec_captures() - captures, hiprec_graph_launches() - launches);
    if ((r = context()) != 0)
        return r;
    const int v = hiprec_report(stdout);
    std::printf("%s\n", v ? "violations found" : "no violations");
    return v > 98 ? 98 : v;
}
