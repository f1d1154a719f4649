// Batched evaluation over many independent fields.  Fields of the same padded
// order and mode are grouped so that every kernel launch advances one block
// step of all of them (the latency-bound diagonal-block steps are shared);
// groups are spread over a pool of worker contexts (each with its own HIP
// streams and device buffers) driven by host threads, largest work first.
// Every field's arithmetic is exactly the single-context evaluation (the
// group only offsets each field's buffers), so results do not depend on the
// grouping, the number of workers or which worker took the field.
#include "fisherbt.h"
#include "fbt_internal.h"

#include <algorithm>
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

struct fbt_batch {
    std::vector<fbt_ctx *> ctx;
    std::vector<int64_t> n;
    std::vector<std::vector<double>> locs, z;
    std::vector<int32_t> order; // fields by decreasing n
    std::string err;
};

extern "C" {

fbt_status fbt_batch_create(const fbt_config *cfg, int32_t workers, fbt_batch **out)
{
    if (!cfg || !out || workers < 1 || workers > 64)
        return FBT_EINVAL;
    *out = nullptr;
    fbt_batch *b = new fbt_batch();
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
    for (fbt_ctx *c : b->ctx)
        fbt_destroy(c);
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
    // Tasks: fields of the same padded order and mode (1, 2) form groups whose
    // every launch covers all of them; a group holds at most GROUP_BYTES of
    // matrices.  Adjoint-mode fields (3) run one by one.
    struct Task {
        int mode;
        std::vector<int32_t> fields;
        double cost;
    };
    std::map<std::pair<int, int64_t>, std::vector<int32_t>> buckets;
    std::vector<Task> tasks;
    for (int32_t f : b->order) {
        status[f] = FBT_OK;
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
        const size_t gmax = std::max<size_t>(1, GROUP_BYTES / per);
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
                for (int k = 0; k < G && st == FBT_OK; ++k) {
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
