// Batched evaluation over many independent fields.  Fields of the same padded
// order and mode are grouped so that every kernel launch advances one block
// step of all of them (the latency-bound diagonal-block steps are shared).
// Two executions:
//  - workers: groups are spread over a pool of worker contexts (each with its
//    own HIP streams and device buffers) driven by host threads, largest work
//    first;
//  - graph: every group owns a context, and the whole call (all groups, each
//    on its own streams) is captured once in a HIP graph that later calls with
//    the same fields, modes and precision replay with new theta.
// Group sizes can be limited per padded order, by hand or by the autotuner,
// which times the candidates on the caller's workload and keeps the fastest.
// Every field's arithmetic is exactly the single-context evaluation (the
// group only offsets each field's buffers), so results do not depend on the
// grouping, the execution, the number of workers or which worker took a field.
#include "fisherbt.h"
#include "fbt_internal.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <map>
#include <atomic>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

// device memory one batched group may hold (its three matrices per field)
constexpr size_t GROUP_BYTES = (size_t)8 << 30;
// tile size of the persistent execution when none is set or tuned
constexpr int DEFAULT_TILE = 128;

namespace {

struct Task {
    int mode;
    std::vector<int32_t> fields;
    double cost;
};

} // namespace

struct fbt_batch {
    fbt_config cfg{};
    std::vector<fbt_ctx *> ctx;
    std::vector<int64_t> n;
    std::vector<std::vector<double>> locs, z;
    std::vector<int32_t> order; // fields by decreasing n
    std::string err;
    int exec = FBT_BATCH_WORKERS;
    std::map<int64_t, int32_t> limit; // padded order -> most fields per group (absent: no limit)
    // graph execution: contexts, tasks and the instantiated graph of the last call
    std::vector<fbt_ctx *> gctx;
    std::vector<Task> gtasks;
    std::vector<int32_t> gmodes;
    uint64_t fields_version = 0, graph_fields_version = ~(uint64_t)0;
    uint64_t limit_version = 0, graph_limit_version = ~(uint64_t)0;
    hipStream_t gs = nullptr;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    // persistent execution: one launch per call (fbt_round.hip)
    fbt::RoundExec *round = nullptr;
    int tile = 0;   // 0: default (DEFAULT_TILE)
    int queues = 0; // 0: default (8)
    int round_graph = 1; // the persistent round replayed from a HIP graph
    int fit_threads = 0; // fbt_batch_fit: fits running at once (0: FIT_THREADS)
};

namespace {

void drop_graph(fbt_batch *b)
{
    if (b->graph_exec)
        (void)hipGraphExecDestroy(b->graph_exec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    b->graph_exec = nullptr;
    b->graph = nullptr;
    b->gmodes.clear();
}

// Groups of one call: fields of the same padded order and mode (1, 2), at
// most GROUP_BYTES of matrices and the padded order's limit per group;
// adjoint-mode fields (3) one by one.  Largest work first.
std::vector<Task> make_tasks(const fbt_batch *b, const int32_t *mode)
{
    std::map<std::pair<int, int64_t>, std::vector<int32_t>> buckets;
    std::vector<Task> tasks;
    for (int32_t f : b->order) {
        if (mode[f] == 0)
            continue;
        const int64_t npad = 256 * ((b->n[f] + 1 + 255) / 256);
        if (mode[f] == 3)
            tasks.push_back({3, {f}, (double)npad * npad * npad});
        else
            buckets[{mode[f], npad}].push_back(f);
    }
    for (auto &kv : buckets) {
        const int64_t npad = kv.first.second;
        const size_t per = (size_t)npad * npad * 24;
        size_t gmax = std::max<size_t>(1, GROUP_BYTES / per);
        const auto lim = b->limit.find(npad);
        if (lim != b->limit.end() && lim->second > 0)
            gmax = std::min<size_t>(gmax, (size_t)lim->second);
        const double unit = (double)npad * npad * npad * (kv.first.first == 2 ? 9.0 : 1.0);
        for (size_t i = 0; i < kv.second.size(); i += gmax) {
            Task t{kv.first.first, {}, 0.0};
            for (size_t j = i; j < std::min(kv.second.size(), i + gmax); ++j)
                t.fields.push_back(kv.second[j]);
            t.cost = unit * (double)t.fields.size();
            tasks.push_back(std::move(t));
        }
    }
    std::stable_sort(tasks.begin(), tasks.end(),
                     [](const Task &a, const Task &c) { return a.cost > c.cost; });
    return tasks;
}

// Outputs of one group (gll/gsc/gfi/gst indexed by the group's fields).
void scatter(const Task &t, const double *gll, const double *gsc, const double *gfi,
             const int32_t *gst, double *loglik, double *score, double *fisher, int32_t *status)
{
    for (size_t k = 0; k < t.fields.size(); ++k) {
        const int32_t f = t.fields[k];
        status[f] = gst[k];
        if (gst[k] != FBT_OK)
            continue;
        loglik[f] = gll[k];
        if (t.mode == 2) {
            std::memcpy(score + 3 * f, &gsc[3 * k], 3 * sizeof(double));
            std::memcpy(fisher + 9 * f, &gfi[9 * k], 9 * sizeof(double));
        }
    }
}

fbt_status graph_eval(fbt_batch *b, const double *thetas, const int32_t *mode, double *loglik,
                      double *score, double *fisher, int32_t *status);

// Persistent execution: the log-likelihood and derivative fields of the call
// in one launch of the round kernel; adjoint-mode fields after it, one by
// one on the first worker context.
fbt_status persistent_eval(fbt_batch *b, const double *thetas, const int32_t *mode,
                           double *loglik, double *score, double *fisher, int32_t *status)
{
    const int32_t nf = (int32_t)b->n.size();
    if (!b->round) {
        b->round = fbt::round_create(b->cfg.device);
        if (!b->round) {
            b->err = "batch: cannot create the persistent execution's stream";
            return FBT_EDEVICE;
        }
    }
    std::vector<const double *> lp(nf), zp(nf);
    for (int32_t f = 0; f < nf; ++f) {
        lp[f] = b->locs[f].data();
        zp[f] = b->z[f].data();
    }
    std::vector<int32_t> m12(nf);
    bool any = false;
    for (int32_t f = 0; f < nf; ++f) {
        m12[f] = (mode[f] == 1 || mode[f] == 2) ? mode[f] : 0;
        any = any || m12[f] != 0;
    }
    if (any) {
        fbt::round_set_queues(b->round, b->queues ? b->queues : 8);
        fbt::round_set_graph(b->round, b->round_graph != 0);
        std::string err;
        const fbt_status st = fbt::round_eval(b->round, b->tile ? b->tile : DEFAULT_TILE, nf,
                                              b->n.data(), lp.data(), zp.data(),
                                              b->fields_version, thetas, m12.data(), loglik,
                                              score, fisher, status, &err);
        if (st != FBT_OK) {
            b->err = "batch: " + err;
            return st;
        }
    }
    for (int32_t f : b->order) {
        if (mode[f] != 3)
            continue;
        fbt_ctx *c = b->ctx[0];
        fbt_status st = fbt_set_data(c, b->n[f], b->locs[f].data(), b->z[f].data());
        if (st == FBT_OK)
            st = fbt_grad(c, thetas + 3 * f, loglik + f, score + 3 * f, nullptr);
        status[f] = st;
        if (st == FBT_EDEVICE || st == FBT_ENOMEM) {
            b->err = std::string("batch: ") + fbt_last_error(c);
            return st;
        }
    }
    return FBT_OK;
}

} // namespace

extern "C" {

fbt_status fbt_batch_create(const fbt_config *cfg, int32_t workers, fbt_batch **out)
{
    if (!cfg || !out || workers < 1 || workers > 64)
        return FBT_EINVAL;
    *out = nullptr;
    fbt_batch *b = new fbt_batch();
    b->cfg = *cfg;
    b->cfg.hip_stream = nullptr;
    fbt_config wc = *cfg;
    wc.hip_stream = nullptr; // every worker needs streams of its own
    for (int w = 0; w < workers; ++w) {
        fbt_ctx *c = nullptr;
        const fbt_status st = fbt_create(&wc, &c);
        if (st != FBT_OK) {
            fbt_batch_destroy(b);
            return st;
        }
        b->ctx.push_back(c);
    }
    *out = b;
    return FBT_OK;
}

void fbt_batch_destroy(fbt_batch *b)
{
    if (!b)
        return;
    drop_graph(b);
    fbt::round_destroy(b->round);
    for (fbt_ctx *c : b->ctx)
        fbt_destroy(c);
    for (fbt_ctx *c : b->gctx)
        fbt_destroy(c);
    for (hipEvent_t e : b->join)
        (void)hipEventDestroy(e);
    if (b->fork)
        (void)hipEventDestroy(b->fork);
    if (b->gs)
        (void)hipStreamDestroy(b->gs);
    delete b;
}

fbt_status fbt_batch_set_fields(fbt_batch *b, int32_t nf, const int64_t *n,
                                const double *const *locs, const double *const *z)
{
    if (!b || nf < 0 || (nf > 0 && (!n || !locs || !z)))
        return FBT_EINVAL;
    for (int32_t f = 0; f < nf; ++f)
        if (n[f] < 1 || n[f] > ((int64_t)1 << 20) || !locs[f] || !z[f])
            return FBT_EINVAL;
    b->n.assign(n, n + nf);
    b->locs.assign(nf, {});
    b->z.assign(nf, {});
    for (int32_t f = 0; f < nf; ++f) {
        b->locs[f].assign(locs[f], locs[f] + 2 * n[f]);
        b->z[f].assign(z[f], z[f] + n[f]);
    }
    b->order.resize(nf);
    std::iota(b->order.begin(), b->order.end(), 0);
    std::stable_sort(b->order.begin(), b->order.end(),
                     [&](int32_t a, int32_t c) { return b->n[a] > b->n[c]; });
    ++b->fields_version;
    return FBT_OK;
}

fbt_status fbt_batch_eval(fbt_batch *b, const double *thetas, const int32_t *mode,
                          double *loglik, double *score, double *fisher, int32_t *status)
{
    if (!b || !thetas || !mode || !status)
        return FBT_EINVAL;
    const int32_t nf = (int32_t)b->n.size();
    for (int32_t f = 0; f < nf; ++f) {
        if (mode[f] < 0 || mode[f] > 3)
            return FBT_EINVAL;
        if (mode[f] >= 1 && !loglik)
            return FBT_EINVAL;
        if ((mode[f] == 2 || mode[f] == 3) && !score)
            return FBT_EINVAL;
        if (mode[f] == 2 && !fisher)
            return FBT_EINVAL;
    }
    for (int32_t f = 0; f < nf; ++f)
        status[f] = FBT_OK;
    if (b->exec == FBT_BATCH_GRAPH)
        return graph_eval(b, thetas, mode, loglik, score, fisher, status);
    if (b->exec == FBT_BATCH_PERSISTENT)
        return persistent_eval(b, thetas, mode, loglik, score, fisher, status);
    const std::vector<Task> tasks = make_tasks(b, mode);
    std::atomic<size_t> next(0);
    std::mutex mu;
    fbt_status fatal = FBT_OK;
    auto work = [&](fbt_ctx *c) {
        for (;;) {
            const size_t i = next.fetch_add(1);
            if (i >= tasks.size())
                return;
            const Task &t = tasks[i];
            fbt_status st = FBT_OK;
            if (t.mode == 3) {
                const int32_t f = t.fields[0];
                st = fbt_set_data(c, b->n[f], b->locs[f].data(), b->z[f].data());
                if (st == FBT_OK)
                    st = fbt_grad(c, thetas + 3 * f, loglik + f, score + 3 * f, nullptr);
                status[f] = st;
            } else {
                const int G = (int)t.fields.size();
                std::vector<int64_t> gn(G);
                std::vector<const double *> gl(G), gz(G);
                std::vector<double> gth(3 * G), gll(G), gsc(3 * G), gfi(9 * G);
                std::vector<int32_t> gst(G);
                for (int k = 0; k < G; ++k) {
                    const int32_t f = t.fields[k];
                    gn[k] = b->n[f];
                    gl[k] = b->locs[f].data();
                    gz[k] = b->z[f].data();
                    std::memcpy(&gth[3 * k], thetas + 3 * f, 3 * sizeof(double));
                }
                st = fbt::group_run(c, G, gn.data(), gl.data(), gz.data(), gth.data(), t.mode,
                                    gll.data(), gsc.data(), gfi.data(), gst.data());
                if (st == FBT_OK)
                    scatter(t, gll.data(), gsc.data(), gfi.data(), gst.data(), loglik, score,
                            fisher, status);
                if (st != FBT_OK)
                    for (int32_t f : t.fields)
                        status[f] = st;
            }
            if (st == FBT_EDEVICE || st == FBT_ENOMEM) {
                std::lock_guard<std::mutex> g(mu);
                if (fatal == FBT_OK) {
                    fatal = st;
                    b->err = std::string("batch: ") + fbt_last_error(c);
                }
                next.store(tasks.size()); // stop handing out tasks
                return;
            }
        }
    };
    std::vector<std::thread> pool;
    for (size_t w = 1; w < b->ctx.size(); ++w)
        pool.emplace_back(work, b->ctx[w]);
    work(b->ctx[0]);
    for (std::thread &t : pool)
        t.join();
    return fatal;
}

const char *fbt_batch_last_error(const fbt_batch *b) { return b ? b->err.c_str() : ""; }

} // extern "C"

namespace {

// Batched Fisher-BT: every field runs the library's driver (fbt_fit_evaluator,
// Algorithm 1) on a host thread, with an evaluator that posts the request and
// sleeps; once every running driver has posted, the calling thread evaluates
// all posted requests in one fbt_batch_eval call (a round: one launch of the
// round kernel in the persistent execution) and wakes the drivers with their
// results.  At most FIT_THREADS fits run at once: a thread whose fit ends
// takes the next field (counted as running throughout, so that no round
// starts in between with fewer fields).  Each driver sees exactly the
// evaluations a single-field fit over the batch's evaluator would see.
constexpr int FIT_THREADS = 512; // default of fbt_batch_set_fit_threads

struct FitShared {
    std::mutex mu;
    std::condition_variable coord, field;
    int posted = 0;  // drivers waiting for their request's result
    int running = 0; // drivers inside a fit
    size_t next = 0; // next field of the run list
};

struct FitSlot {
    FitShared *S = nullptr;
    int mode = 0; // 1 log-likelihood, 2 derivatives
    double th[3] = {0, 0, 0};
    double ll = 0, sc[3] = {0, 0, 0}, fi[9] = {0};
    fbt_status st = FBT_OK;
    bool posted = false, ready = false;
};

fbt_status fit_post(FitSlot *sl, int mode, const double *th, double *ll, double *sc, double *fi)
{
    FitShared &S = *sl->S;
    std::unique_lock<std::mutex> lk(S.mu);
    sl->mode = mode;
    std::memcpy(sl->th, th, 3 * sizeof(double));
    sl->ready = false;
    sl->posted = true;
    ++S.posted;
    S.coord.notify_one();
    S.field.wait(lk, [&] { return sl->ready; });
    if (sl->st == FBT_OK) {
        *ll = sl->ll;
        if (mode == 2) {
            std::memcpy(sc, sl->sc, 3 * sizeof(double));
            std::memcpy(fi, sl->fi, 9 * sizeof(double));
        }
    }
    return sl->st;
}

fbt_status fit_loglik(void *user, const double theta[3], double *ll)
{
    return fit_post(static_cast<FitSlot *>(user), 1, theta, ll, nullptr, nullptr);
}

fbt_status fit_eval(void *user, const double theta[3], double *ll, double score[3],
                    double fisher[9])
{
    return fit_post(static_cast<FitSlot *>(user), 2, theta, ll, score, fisher);
}

} // namespace

extern "C" {

fbt_status fbt_batch_fit(fbt_batch *b, const fbt_fit_options *opt, const double *theta0,
                         const int32_t *active, fbt_fit_result *res, int32_t *status,
                         int32_t *rounds)
{
    if (!b || !opt || !res || !status)
        return FBT_EINVAL;
    // as fbt_fit: the acceptance tests of Eq. (4) take FP64 log-likelihoods
    if (b->cfg.precision == FBT_MIXED_FP32_ALL || b->cfg.precision == FBT_MIXED_BF16_ALL) {
        b->err = "batch fit: the FP32 and bfloat16 Cholesky forms change the log-likelihood that "
                 "the acceptance tests of Eq. (4) take";
        return FBT_EINVAL;
    }
    const int32_t nf = (int32_t)b->n.size();
    FitShared S;
    std::vector<FitSlot> slot(nf);
    std::vector<fbt_fit_options> o(nf, *opt);
    std::vector<int32_t> run;
    for (int32_t f = 0; f < nf; ++f) {
        slot[f].S = &S;
        o[f].theta0 = theta0 ? theta0 + 3 * f : nullptr;
        status[f] = FBT_OK;
        if (!active || active[f])
            run.push_back(f);
    }
    if (rounds)
        *rounds = 0;
    const int nrun = (int)run.size();
    const int nthreads = std::min(nrun, b->fit_threads > 0 ? b->fit_threads : FIT_THREADS);
    S.running = nthreads; // each thread starts inside its first fit
    S.next = (size_t)nthreads;
    std::vector<std::thread> th;
    th.reserve(nthreads);
    for (int w = 0; w < nthreads; ++w)
        th.emplace_back([&, w] {
            size_t k = (size_t)w;
            for (;;) {
                const int32_t f = run[k];
                fbt_evaluator ev{&slot[f], fit_loglik, fit_eval};
                std::memset(&res[f], 0, sizeof(fbt_fit_result));
                status[f] = fbt_fit_evaluator(&ev, &o[f], &res[f]);
                std::lock_guard<std::mutex> g(S.mu);
                if (S.next < run.size()) {
                    k = S.next++; // stays running: the next field's fit starts at once
                    continue;
                }
                --S.running;
                S.coord.notify_one();
                return;
            }
        });
    std::vector<double> thetas(3 * (size_t)nf, 1.0), ll(nf), sc(3 * (size_t)nf), fi(9 * (size_t)nf);
    std::vector<int32_t> mode(nf), st(nf);
    fbt_status fatal = FBT_OK;
    std::unique_lock<std::mutex> lk(S.mu);
    for (;;) {
        S.coord.wait(lk, [&] { return S.posted == S.running; });
        if (S.running == 0)
            break;
        for (int32_t f = 0; f < nf; ++f) {
            mode[f] = slot[f].posted ? slot[f].mode : 0;
            if (slot[f].posted)
                std::memcpy(&thetas[3 * f], slot[f].th, 3 * sizeof(double));
        }
        lk.unlock();
        const fbt_status r = fbt_batch_eval(b, thetas.data(), mode.data(), ll.data(), sc.data(),
                                            fi.data(), st.data());
        lk.lock();
        if (r != FBT_OK && fatal == FBT_OK)
            fatal = r;
        for (int32_t f = 0; f < nf; ++f) {
            FitSlot &sl = slot[f];
            if (!sl.posted)
                continue;
            sl.st = r != FBT_OK ? r : (fbt_status)st[f];
            sl.ll = ll[f];
            std::memcpy(sl.sc, &sc[3 * f], 3 * sizeof(double));
            std::memcpy(sl.fi, &fi[9 * f], 9 * sizeof(double));
            sl.posted = false;
            sl.ready = true;
        }
        S.posted = 0;
        if (rounds)
            ++*rounds;
        S.field.notify_all();
    }
    lk.unlock();
    for (std::thread &t : th)
        t.join();
    return fatal;
}

// The graph execution is switched off: its first capture and replay ended the
// host process with a segmentation fault inside the capture / instantiate /
// launch sequence, the cause is not identified, and the path stays closed
// until it is.  Asking for it is an error; the code is kept for that work
// (FBT_GRAPH_EXEC=1 builds it in, for the host-only check of its capture
// sequence against a recording stand-in of the runtime).
#ifndef FBT_GRAPH_EXEC
#define FBT_GRAPH_EXEC 0
#endif
constexpr bool GRAPH_EXEC_ENABLED = FBT_GRAPH_EXEC != 0;

fbt_status fbt_batch_set_exec(fbt_batch *b, int32_t exec)
{
    if (!b || (exec != FBT_BATCH_WORKERS && exec != FBT_BATCH_GRAPH &&
               exec != FBT_BATCH_PERSISTENT))
        return FBT_EINVAL;
    if (exec == FBT_BATCH_PERSISTENT && b->cfg.precision != FBT_FP64) {
        b->err = "batch: the persistent execution computes in FP64 only";
        return FBT_EINVAL;
    }
    if (exec == FBT_BATCH_GRAPH && !GRAPH_EXEC_ENABLED) {
        b->err = "batch: the graph execution is disabled (its capture crashed the host process; "
                 "cause not identified)";
        return FBT_EINVAL;
    }
    b->exec = exec;
    return FBT_OK;
}

fbt_status fbt_batch_set_group_limit(fbt_batch *b, int64_t npad, int32_t max_fields)
{
    if (!b || npad < 256 || npad % 256 != 0 || max_fields < 0)
        return FBT_EINVAL;
    if (max_fields == 0)
        b->limit.erase(npad);
    else
        b->limit[npad] = max_fields;
    ++b->limit_version;
    return FBT_OK;
}

int32_t fbt_batch_group_limit(const fbt_batch *b, int64_t npad)
{
    if (!b)
        return -1;
    const auto it = b->limit.find(npad);
    return it == b->limit.end() ? 0 : it->second;
}

int32_t fbt_batch_get_exec(const fbt_batch *b) { return b ? b->exec : -1; }

fbt_status fbt_batch_set_tile(fbt_batch *b, int32_t tile)
{
    if (!b || (tile != 0 && tile != 64 && tile != 128))
        return FBT_EINVAL;
    b->tile = tile;
    return FBT_OK;
}

int32_t fbt_batch_get_tile(const fbt_batch *b) { return b ? (b->tile ? b->tile : DEFAULT_TILE) : -1; }

fbt_status fbt_batch_set_fit_threads(fbt_batch *b, int32_t threads)
{
    if (!b || threads < 0 || threads > 4096)
        return FBT_EINVAL;
    b->fit_threads = threads;
    return FBT_OK;
}

fbt_status fbt_batch_set_queues(fbt_batch *b, int32_t queues)
{
    if (!b || (queues != 0 && queues != 1 && queues != 2 && queues != 4 && queues != 8))
        return FBT_EINVAL;
    b->queues = queues;
    return FBT_OK;
}

int32_t fbt_batch_get_queues(const fbt_batch *b) { return b ? (b->queues ? b->queues : 8) : -1; }

fbt_status fbt_batch_set_round_graph(fbt_batch *b, int32_t on)
{
    if (!b)
        return FBT_EINVAL;
    b->round_graph = on != 0;
    return FBT_OK;
}

fbt_status fbt_batch_set_round_trace(fbt_batch *b, int32_t on)
{
    if (!b)
        return FBT_EINVAL;
    if (!b->round) {
        b->round = fbt::round_create(b->cfg.device);
        if (!b->round)
            return FBT_EDEVICE;
    }
    fbt::round_set_trace(b->round, on != 0);
    return FBT_OK;
}

int64_t fbt_batch_round_trace(const fbt_batch *b, int64_t *out, int64_t cap)
{
    return (b && out && cap > 0) ? fbt::round_trace(b->round, out, cap) : 0;
}

fbt_status fbt_batch_round_stats(const fbt_batch *b, int64_t *ntasks, double *plan_us,
                                 double *kernel_ms)
{
    if (!b)
        return FBT_EINVAL;
    if (ntasks)
        *ntasks = fbt::round_task_count(b->round);
    if (plan_us)
        *plan_us = fbt::round_plan_estimate_us(b->round);
    if (kernel_ms)
        *kernel_ms = fbt::round_last_ms(b->round);
    return FBT_OK;
}

fbt_status fbt_batch_autotune(fbt_batch *b, const double *thetas, const int32_t *mode,
                              const char *path)
{
    if (!b || !thetas || !mode)
        return FBT_EINVAL;
    const int32_t nf = (int32_t)b->n.size();
    std::map<int64_t, int> count;
    for (int32_t f = 0; f < nf; ++f) {
        if (mode[f] < 0 || mode[f] > 3)
            return FBT_EINVAL;
        if (mode[f] == 1 || mode[f] == 2)
            ++count[256 * ((b->n[f] + 1 + 255) / 256)];
    }
    std::vector<double> ll(nf), sc(3 * (size_t)nf), fi(9 * (size_t)nf);
    std::vector<int32_t> st(nf);
    using clk = std::chrono::steady_clock;
    // best of two timed calls after one untimed call (which builds a graph)
    auto time_call = [&](const int32_t *m, double *secs) -> fbt_status {
        fbt_status r = fbt_batch_eval(b, thetas, m, ll.data(), sc.data(), fi.data(), st.data());
        if (r != FBT_OK)
            return r;
        double best = 1e300;
        for (int rep = 0; rep < 2; ++rep) {
            const auto t0 = clk::now();
            if ((r = fbt_batch_eval(b, thetas, m, ll.data(), sc.data(), fi.data(), st.data())) !=
                FBT_OK)
                return r;
            best = std::min(best, std::chrono::duration<double>(clk::now() - t0).count());
        }
        *secs = best;
        return FBT_OK;
    };
    for (const auto &kv : count) {
        const int64_t npad = kv.first;
        std::vector<int32_t> sub(nf, 0);
        for (int32_t f = 0; f < nf; ++f)
            if ((mode[f] == 1 || mode[f] == 2) && 256 * ((b->n[f] + 1 + 255) / 256) == npad)
                sub[f] = mode[f];
        int32_t best_lim = 0;
        double best = 1e300;
        for (int32_t lim : {1, 2, 4, 8, 16, 32, 0}) {
            if (lim >= kv.second)
                lim = 0; // no limit
            if (lim == 0 && best_lim == 0 && best < 1e300)
                break;   // "no limit" timed already
            fbt_batch_set_group_limit(b, npad, lim);
            double t;
            const fbt_status r = time_call(sub.data(), &t);
            if (r != FBT_OK)
                return r;
            if (t < best) {
                best = t;
                best_lim = lim;
            }
            if (lim == 0)
                break;
        }
        fbt_batch_set_group_limit(b, npad, best_lim);
    }
    // The buckets were timed alone; in the whole call their groups share the
    // workers, so the per-order choices compete with no limits and with one
    // limit for every order, timed on the whole call.
    const std::map<int64_t, int32_t> per_order = b->limit;
    auto set_all = [&](const std::map<int64_t, int32_t> &m) {
        b->limit = m;
        ++b->limit_version;
    };
    const int32_t keep = b->exec;
    b->exec = FBT_BATCH_WORKERS;
    fbt_status r;
    double tw = 1e300;
    std::map<int64_t, int32_t> best_map;
    std::string chosen;
    for (int cand = 0; cand < 5; ++cand) {
        std::map<int64_t, int32_t> m;
        std::string name;
        if (cand == 0) {
            m = per_order;
            name = "per_order";
        } else if (cand == 1) {
            name = "none";
        } else {
            const int32_t u = 4 << (2 * (cand - 2)); // 4, 16, 64
            for (const auto &kv : count)
                m[kv.first] = u;
            name = "all_" + std::to_string(u);
        }
        set_all(m);
        double t;
        if ((r = time_call(mode, &t)) != FBT_OK)
            return r;
        if (t < tw) {
            tw = t;
            best_map = m;
            chosen = name;
        }
    }
    set_all(best_map);
    std::string js = "{\n  \"limits\": {";
    bool first = true;
    for (const auto &kv : b->limit) {
        char lb[96];
        std::snprintf(lb, sizeof(lb), "%s\n    \"%lld\": %d", first ? "" : ",", (long long)kv.first,
                      kv.second);
        js += lb;
        first = false;
    }
    js += "\n  },\n  \"chosen\": \"" + chosen + "\",";
    double tg = -1;
    double best_t = tw;
    b->exec = FBT_BATCH_WORKERS;
    if (GRAPH_EXEC_ENABLED) {
        b->exec = FBT_BATCH_GRAPH;
        if ((r = time_call(mode, &tg)) != FBT_OK) {
            b->exec = keep;
            return r;
        }
        b->exec = tg < tw ? FBT_BATCH_GRAPH : FBT_BATCH_WORKERS;
        best_t = std::min(tw, tg);
    }
    // the persistent execution (FP64 only) with each tile size
    double tp[2] = {-1.0, -1.0};
    const int keep_tile = b->tile;
    int best_tile = keep_tile;
    if (b->cfg.precision == FBT_FP64) {
        const int exec_now = b->exec;
        b->exec = FBT_BATCH_PERSISTENT;
        bool won = false;
        for (int q = 0; q < 2; ++q) {
            b->tile = q == 0 ? 64 : 128;
            if ((r = time_call(mode, &tp[q])) != FBT_OK) {
                b->exec = keep;
                b->tile = keep_tile;
                return r;
            }
            if (tp[q] < best_t) {
                best_t = tp[q];
                best_tile = b->tile;
                won = true;
            }
        }
        b->exec = won ? FBT_BATCH_PERSISTENT : exec_now;
        b->tile = won ? best_tile : keep_tile;
    }
    char buf[384];
    std::snprintf(buf, sizeof(buf),
                  "\n  \"exec\": %d,\n  \"tile\": %d,\n  \"seconds_workers\": %.6f,\n  "
                  "\"seconds_graph\": %.6f,\n  \"seconds_persistent_64\": %.6f,\n  "
                  "\"seconds_persistent_128\": %.6f,\n  \"precision\": %d\n}\n",
                  b->exec, b->tile, tw, tg, tp[0], tp[1], (int)b->cfg.precision);
    js += buf;
    if (path) {
        FILE *fp = std::fopen(path, "w");
        if (!fp) {
            b->err = std::string("autotune: cannot write ") + path;
            return FBT_EINVAL;
        }
        std::fputs(js.c_str(), fp);
        std::fclose(fp);
    }
    return FBT_OK;
}

fbt_status fbt_batch_load_tuning(fbt_batch *b, const char *path)
{
    if (!b || !path)
        return FBT_EINVAL;
    FILE *fp = std::fopen(path, "r");
    if (!fp)
        return FBT_EINVAL;
    std::string txt;
    char buf[4096];
    size_t k;
    while ((k = std::fread(buf, 1, sizeof(buf), fp)) > 0)
        txt.append(buf, k);
    std::fclose(fp);
    // the file fbt_batch_autotune writes: "limits": {"npad": n, ...}, "exec": e
    const size_t lp = txt.find("\"limits\"");
    const size_t ep = txt.find("\"exec\"");
    if (lp == std::string::npos || ep == std::string::npos)
        return FBT_EINVAL;
    const size_t open = txt.find('{', lp), close = txt.find('}', lp);
    if (open == std::string::npos || close == std::string::npos)
        return FBT_EINVAL;
    std::map<int64_t, int32_t> lim;
    size_t pos = open + 1;
    while (pos < close) {
        const size_t q1 = txt.find('"', pos);
        if (q1 == std::string::npos || q1 > close)
            break;
        const size_t q2 = txt.find('"', q1 + 1);
        const size_t colon = txt.find(':', q2);
        if (q2 == std::string::npos || colon == std::string::npos || colon > close)
            return FBT_EINVAL;
        const long long npad = std::atoll(txt.substr(q1 + 1, q2 - q1 - 1).c_str());
        const int v = std::atoi(txt.c_str() + colon + 1);
        if (npad < 256 || npad % 256 != 0 || v < 0)
            return FBT_EINVAL;
        lim[npad] = v;
        const size_t comma = txt.find(',', colon);
        pos = (comma == std::string::npos || comma > close) ? close : comma + 1;
    }
    const int e = std::atoi(txt.c_str() + txt.find(':', ep) + 1);
    if (e != FBT_BATCH_WORKERS && !(e == FBT_BATCH_GRAPH && GRAPH_EXEC_ENABLED) &&
        !(e == FBT_BATCH_PERSISTENT && b->cfg.precision == FBT_FP64))
        return FBT_EINVAL;
    int tile = 0;
    const size_t tp = txt.find("\"tile\"");
    if (tp != std::string::npos) {
        tile = std::atoi(txt.c_str() + txt.find(':', tp) + 1);
        if (tile != 0 && tile != 64 && tile != 128)
            return FBT_EINVAL;
    }
    b->tile = tile;
    b->limit.clear();
    for (const auto &kv : lim)
        if (kv.second > 0)
            b->limit[kv.first] = kv.second;
    ++b->limit_version;
    b->exec = e;
    return FBT_OK;
}

} // extern "C"

namespace {

#define GCHK(expr)                                                                                 \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) {                                                                    \
            b->err = std::string("batch graph: " #expr ": ") + hipGetErrorString(e_);             \
            return FBT_EDEVICE;                                                                    \
        }                                                                                          \
    } while (0)

// Graph execution: the groups of the call, each on a context of its own,
// captured once (fields, modes, limits and precision fixed) and replayed.
fbt_status graph_eval(fbt_batch *b, const double *thetas, const int32_t *mode, double *loglik,
                      double *score, double *fisher, int32_t *status)
{
    const int32_t nf = (int32_t)b->n.size();
    std::vector<int32_t> modes(mode, mode + nf);
    for (int32_t &m : modes)
        if (m == 3)
            m = 0; // adjoint-mode fields run after the graph
    auto gth = [&](const Task &t) {
        std::vector<double> th(3 * t.fields.size());
        for (size_t k = 0; k < t.fields.size(); ++k)
            std::memcpy(&th[3 * k], thetas + 3 * t.fields[k], 3 * sizeof(double));
        return th;
    };
    std::vector<std::vector<int>> bad;
    const bool rebuild = !b->graph_exec || modes != b->gmodes ||
                         b->graph_fields_version != b->fields_version ||
                         b->graph_limit_version != b->limit_version;
    if (rebuild) {
        drop_graph(b);
        b->gtasks = make_tasks(b, modes.data());
        while (b->gctx.size() < b->gtasks.size()) {
            fbt_ctx *c = nullptr;
            const fbt_status st = fbt_create(&b->cfg, &c);
            if (st != FBT_OK) {
                b->err = "batch graph: context creation failed";
                return st;
            }
            fbt::ctx_set_capturable(c, true);
            b->gctx.push_back(c);
        }
        if (!b->gs)
            GCHK(hipStreamCreateWithFlags(&b->gs, hipStreamNonBlocking));
        if (!b->fork)
            GCHK(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
        while (b->join.size() < b->gtasks.size()) {
            hipEvent_t e;
            GCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            b->join.push_back(e);
        }
    }
    const size_t ng = b->gtasks.size();
    bad.resize(ng);
    for (size_t g = 0; g < ng; ++g) {
        const Task &t = b->gtasks[g];
        fbt_ctx *c = b->gctx[g];
        const int G = (int)t.fields.size();
        if (rebuild) {
            std::vector<int64_t> gn(G);
            std::vector<const double *> gl(G), gz(G);
            for (int k = 0; k < G; ++k) {
                gn[k] = b->n[t.fields[k]];
                gl[k] = b->locs[t.fields[k]].data();
                gz[k] = b->z[t.fields[k]].data();
            }
            const fbt_status st = fbt::group_prepare(c, G, gn.data(), gl.data(), gz.data());
            if (st != FBT_OK) {
                b->err = std::string("batch graph: ") + fbt_last_error(c);
                return st;
            }
        }
        bad[g].assign(G, 0);
        const std::vector<double> th = gth(t);
        fbt::group_stage(c, th.data(), bad[g].data());
    }
    if (rebuild && ng > 0) {
        GCHK(hipStreamBeginCapture(b->gs, hipStreamCaptureModeThreadLocal));
        fbt_status st = FBT_OK;
        hipError_t he = hipEventRecord(b->fork, b->gs);
        for (size_t g = 0; g < ng && st == FBT_OK && he == hipSuccess; ++g) {
            hipStream_t cs = fbt::ctx_stream(b->gctx[g]);
            if ((he = hipStreamWaitEvent(cs, b->fork, 0)) != hipSuccess)
                break;
            if ((st = fbt::group_enqueue(b->gctx[g], b->gtasks[g].mode)) != FBT_OK)
                break;
            if ((he = hipEventRecord(b->join[g], cs)) == hipSuccess)
                he = hipStreamWaitEvent(b->gs, b->join[g], 0);
        }
        hipGraph_t graph = nullptr;
        const hipError_t ee = hipStreamEndCapture(b->gs, &graph);
        if (st != FBT_OK || he != hipSuccess || ee != hipSuccess) {
            if (graph)
                (void)hipGraphDestroy(graph);
            b->err = std::string("batch graph: capture failed: ") +
                     hipGetErrorString(he != hipSuccess ? he : ee);
            return st != FBT_OK ? st : FBT_EDEVICE;
        }
        b->graph = graph;
        GCHK(hipGraphInstantiate(&b->graph_exec, b->graph, nullptr, nullptr, 0));
        b->gmodes = modes;
        b->graph_fields_version = b->fields_version;
        b->graph_limit_version = b->limit_version;
    }
    if (ng > 0) {
        GCHK(hipGraphLaunch(b->graph_exec, b->gs));
        GCHK(hipStreamSynchronize(b->gs));
    }
    for (size_t g = 0; g < ng; ++g) {
        const Task &t = b->gtasks[g];
        const size_t G = t.fields.size();
        std::vector<double> gll(G), gsc(3 * G), gfi(9 * G);
        std::vector<int32_t> gst(G);
        const std::vector<double> th = gth(t);
        fbt::group_results(b->gctx[g], t.mode, th.data(), bad[g].data(), gll.data(), gsc.data(),
                           gfi.data(), gst.data());
        scatter(t, gll.data(), gsc.data(), gfi.data(), gst.data(), loglik, score, fisher, status);
    }
    // adjoint-mode fields, one by one on the first worker context
    for (int32_t f = 0; f < nf; ++f) {
        if (mode[f] != 3)
            continue;
        fbt_ctx *c = b->ctx[0];
        fbt_status st = fbt_set_data(c, b->n[f], b->locs[f].data(), b->z[f].data());
        if (st == FBT_OK)
            st = fbt_grad(c, thetas + 3 * f, loglik + f, score + 3 * f, nullptr);
        status[f] = st;
        if (st == FBT_EDEVICE || st == FBT_ENOMEM) {
            b->err = std::string("batch: ") + fbt_last_error(c);
            return st;
        }
    }
    return FBT_OK;
}

} // namespace
