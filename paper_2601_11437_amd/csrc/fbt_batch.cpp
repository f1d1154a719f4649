// Batched evaluation over many independent fields: a pool of contexts (each
// with its own pair of HIP streams and its own device buffers, sized once for
// the largest field) driven by host worker threads.  Workers take fields from
// one shared queue ordered by decreasing n (longest processing time first), so
// the evaluations of different fields overlap on the device.  Every field's
// evaluation is exactly the single-context one (same kernels, same fixed
// reduction order), so results do not depend on the number of workers or on
// which worker took the field.
#include "fisherbt.h"

#include <algorithm>
#include <atomic>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

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
    std::atomic<int32_t> next(0);
    std::mutex mu;
    fbt_status fatal = FBT_OK;
    auto work = [&](fbt_ctx *c) {
        for (;;) {
            const int32_t i = next.fetch_add(1);
            if (i >= nf)
                return;
            const int32_t f = b->order[i];
            if (mode[f] == 0) {
                status[f] = FBT_OK;
                continue;
            }
            fbt_status st = fbt_set_data(c, b->n[f], b->locs[f].data(), b->z[f].data());
            const double *th = thetas + 3 * f;
            if (st == FBT_OK) {
                if (mode[f] == 1)
                    st = fbt_loglik(c, th, loglik + f);
                else if (mode[f] == 2)
                    st = fbt_eval(c, th, loglik + f, score + 3 * f, fisher + 9 * f);
                else
                    st = fbt_grad(c, th, loglik + f, score + 3 * f, nullptr);
            }
            status[f] = st;
            if (st == FBT_EDEVICE || st == FBT_ENOMEM) {
                std::lock_guard<std::mutex> g(mu);
                if (fatal == FBT_OK) {
                    fatal = st;
                    b->err = "field " + std::to_string(f) + ": " + fbt_last_error(c);
                }
                next.store(nf); // stop handing out fields
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
