// Host planner of the persistent round kernel: list scheduling of the tile
// tasks of all fields onto the kernel's workgroups, and the check that the
// resulting ticket order can never make a workgroup wait on a task that no
// workgroup holds.
#include "fbt_plan.h"
#include "fisherbt.h"

#include <algorithm>
#include <cstdio>
#include <queue>
#include <utility>

namespace fbt {

int64_t rtask_count(int T, int mode)
{
    if (mode != 1 && mode != 2)
        return 0;
    const int64_t P = (int64_t)T * (T + 1) / 2;
    return mode == 1 ? 2 * P + 1 : 3 * P + 2 * (int64_t)T * T + 1;
}

namespace {

// Local task ids of one field: GEN, CHOL, LSOLVE, RSOLVE, REDUCE, then one
// zero-cost node per block column that stands for "column finished".
struct Ids {
    int T, mode;
    int64_t P, gen, chol, ls, rs, red, coln, total;
    Ids(int T_, int mode_) : T(T_), mode(mode_)
    {
        P = (int64_t)T * (T + 1) / 2;
        gen = 0;
        chol = gen + P;
        ls = chol + P;
        rs = ls + (mode == 2 ? 2 * (int64_t)T * T : 0);
        red = rs + (mode == 2 ? P : 0);
        coln = red + 1;
        total = coln + T;
    }
    int64_t g(int i, int j) const { return gen + rpair(i, j); }
    int64_t c(int i, int j) const { return chol + rpair(i, j); }
    int64_t l(int k, int col) const { return ls + (int64_t)k * 2 * T + col; }
    int64_t r(int i, int j) const { return rs + rpair(i, j); }
};

RTask task_of(const Ids &d, int field, int64_t id)
{
    if (id < d.chol) {
        int i = 0;
        while ((int64_t)(i + 1) * (i + 2) / 2 <= id - d.gen)
            ++i;
        return rtask(field, R_GEN, i, (int)(id - d.gen - (int64_t)i * (i + 1) / 2));
    }
    if (id < d.ls) {
        int i = 0;
        while ((int64_t)(i + 1) * (i + 2) / 2 <= id - d.chol)
            ++i;
        return rtask(field, R_CHOL, i, (int)(id - d.chol - (int64_t)i * (i + 1) / 2));
    }
    if (id < d.rs) {
        const int64_t q = id - d.ls;
        return rtask(field, R_LSOLVE, (int)(q / (2 * d.T)), (int)(q % (2 * d.T)));
    }
    if (id < d.red) {
        int i = 0;
        while ((int64_t)(i + 1) * (i + 2) / 2 <= id - d.rs)
            ++i;
        return rtask(field, R_RSOLVE, i, (int)(id - d.rs - (int64_t)i * (i + 1) / 2));
    }
    return rtask(field, R_REDUCE, 0, 0);
}

// Cost model (microseconds on one workgroup slot, two slots per CU): FP64
// MFMA products at 0.12 TFLOP/s per slot, generation per entry, a fixed cost
// per task (ticket, waits, release), and the diagonal factorisation.
struct Cost {
    double bt;
    double gemm(double K) const { return 2.0 * bt * bt * K / 0.12e6; }
    double task(const RTask &t, int mode) const
    {
        const int i = rt_i(t), j = rt_j(t);
        const double b3 = 2.0 * bt * bt * bt / 0.12e6;
        switch (rt_type(t)) {
        case R_GEN: {
            const double e = (i == j) ? bt * (bt + 1) / 2 : bt * bt;
            return 4.0 + e * (mode == 2 ? 0.026 : 0.019);
        }
        case R_CHOL:
            return 4.0 + gemm(j * bt) + (i == j ? (bt > 64 ? 40.0 : 15.0) : b3);
        case R_LSOLVE:
            return 4.0 + gemm(i * bt) + b3;
        case R_RSOLVE:
            return 6.0 + 2.0 * (gemm(j * bt) + b3);
        default:
            return 10.0;
        }
    }
};

} // namespace

RPlan rplan(const std::vector<RPlanField> &fields, int bt, int slots, std::string *err)
{
    RPlan plan;
    const int nf = (int)fields.size();
    std::vector<int64_t> base(nf + 1, 0);
    std::vector<Ids> ids;
    ids.reserve(nf);
    for (int f = 0; f < nf; ++f) {
        const int m = (fields[f].mode == 1 || fields[f].mode == 2) ? fields[f].mode : 0;
        ids.emplace_back(fields[f].T, m);
        base[f + 1] = base[f] + (m ? ids[f].total : 0);
    }
    const int64_t N = base[nf];
    std::vector<int64_t> head(N + 1, 0);
    std::vector<std::pair<int64_t, int64_t>> edges; // (pred, succ), global ids
    std::vector<double> cost(N, 0.0);
    std::vector<char> real(N, 0);
    const Cost cm{(double)bt};
    for (int f = 0; f < nf; ++f) {
        const Ids &d = ids[f];
        if (!d.mode)
            continue;
        const int T = d.T;
        const int64_t o = base[f];
        auto E = [&](int64_t a, int64_t b) { edges.emplace_back(o + a, o + b); };
        for (int64_t id = 0; id < d.coln; ++id) {
            cost[o + id] = cm.task(task_of(d, f, id), d.mode);
            real[o + id] = 1;
        }
        for (int j = 0; j < T; ++j)
            for (int i = j; i < T; ++i) {
                E(d.g(i, j), d.c(i, j));
                E(d.c(i, j), d.coln + j);
                if (j > 0)
                    E(d.coln + j - 1, d.c(i, j));
                if (i > j)
                    E(d.c(j, j), d.c(i, j));
            }
        if (d.mode == 2) {
            for (int k = 0; k < T; ++k)
                for (int col = 0; col < 2 * T; ++col) {
                    const int cc = col % T;
                    E(k >= cc ? d.g(k, cc) : d.g(cc, k), d.l(k, col));
                    E(d.c(k, k), d.l(k, col));
                    if (k > 0)
                        E(d.l(k - 1, col), d.l(k, col));
                }
            for (int i = 0; i < T; ++i)
                for (int j = 0; j <= i; ++j) {
                    E(d.l(T - 1, j), d.r(i, j));
                    E(d.l(T - 1, T + j), d.r(i, j));
                    if (j > 0)
                        E(d.r(i, j - 1), d.r(i, j));
                }
            for (int i = 0; i < T; ++i)
                E(d.r(i, i), d.red);
        } else {
            E(d.c(T - 1, T - 1), d.red);
        }
    }
    // adjacency (CSR) and in-degrees
    std::vector<int32_t> indeg(N, 0);
    for (const auto &e : edges)
        ++head[e.first + 1], ++indeg[e.second];
    for (int64_t v = 0; v < N; ++v)
        head[v + 1] += head[v];
    std::vector<int64_t> adj(edges.size());
    {
        std::vector<int64_t> fill(head.begin(), head.end() - 1);
        for (const auto &e : edges)
            adj[fill[e.first]++] = e.second;
    }
    edges.clear();
    edges.shrink_to_fit();
    // topological order (Kahn), then upward ranks in reverse
    std::vector<int64_t> topo;
    topo.reserve(N);
    {
        std::vector<int32_t> deg(indeg);
        for (int64_t v = 0; v < N; ++v)
            if (!deg[v])
                topo.push_back(v);
        for (size_t q = 0; q < topo.size(); ++q)
            for (int64_t e = head[topo[q]]; e < head[topo[q] + 1]; ++e)
                if (--deg[adj[e]] == 0)
                    topo.push_back(adj[e]);
        if ((int64_t)topo.size() != N) {
            if (err)
                *err = "round plan: the task graph has a cycle";
            return RPlan();
        }
    }
    std::vector<double> rank(N, 0.0);
    for (int64_t q = N - 1; q >= 0; --q) {
        const int64_t v = topo[q];
        double m = 0.0;
        for (int64_t e = head[v]; e < head[v + 1]; ++e)
            m = std::max(m, rank[adj[e]]);
        rank[v] = cost[v] + m;
    }
    // list schedule: `slots` workers; the ready task of highest rank starts
    // whenever a worker is free; the start order is the ticket order
    auto field_of = [&](int64_t v) {
        return (int)(std::upper_bound(base.begin(), base.end(), v) - base.begin()) - 1;
    };
    typedef std::pair<double, int64_t> Item;
    std::priority_queue<Item> ready; // max rank (ties: smaller id first)
    std::priority_queue<Item, std::vector<Item>, std::greater<Item>> running; // min finish
    std::vector<int32_t> deg(indeg);
    std::vector<int64_t> stack;
    double now = 0.0;
    int freew = std::max(1, slots);
    plan.order.reserve(N);
    // a node becomes ready; zero-cost column nodes finish at once
    auto release = [&](int64_t v) {
        stack.push_back(v);
        while (!stack.empty()) {
            const int64_t u = stack.back();
            stack.pop_back();
            if (real[u]) {
                ready.push({rank[u], -u});
                continue;
            }
            for (int64_t e = head[u]; e < head[u + 1]; ++e)
                if (--deg[adj[e]] == 0)
                    stack.push_back(adj[e]);
        }
    };
    for (int64_t v = 0; v < N; ++v)
        if (!indeg[v])
            release(v);
    while (!ready.empty() || !running.empty()) {
        while (freew > 0 && !ready.empty()) {
            const int64_t v = -ready.top().second;
            ready.pop();
            const int f = field_of(v);
            plan.order.push_back(task_of(ids[f], f, v - base[f]));
            plan.busy_us += cost[v];
            running.push({now + cost[v], v});
            --freew;
        }
        if (running.empty())
            break;
        const Item it = running.top();
        running.pop();
        now = it.first;
        ++freew;
        for (int64_t e = head[it.second]; e < head[it.second + 1]; ++e)
            if (--deg[adj[e]] == 0)
                release(adj[e]);
    }
    plan.est_us = now;
    plan.qoff = {0, (int64_t)plan.order.size()};
    const std::string chk = rplan_check(plan.order, fields);
    if (!chk.empty()) {
        if (err)
            *err = "round plan: " + chk;
        return RPlan();
    }
    return plan;
}

RPlan rplan_queues(const std::vector<RPlanField> &fields, int bt, int slots, int nq,
                   std::string *err)
{
    const int nf = (int)fields.size();
    nq = std::max(1, std::min(nq, std::max(1, slots)));
    // estimated work of each field: its tasks under the cost model
    const Cost cm{(double)bt};
    std::vector<double> work(nf, 0.0);
    for (int f = 0; f < nf; ++f) {
        const int m = fields[f].mode;
        if (m != 1 && m != 2)
            continue;
        const Ids d(fields[f].T, m);
        for (int64_t id = 0; id < d.coln; ++id)
            work[f] += cm.task(task_of(d, f, id), m);
    }
    std::vector<int> byw(nf);
    for (int f = 0; f < nf; ++f)
        byw[f] = f;
    std::stable_sort(byw.begin(), byw.end(), [&](int a, int b) { return work[a] > work[b]; });
    std::vector<double> load(nq, 0.0);
    std::vector<int> queue_of(nf, 0);
    for (int f : byw) {
        const int q = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        queue_of[f] = q;
        load[q] += work[f];
    }
    RPlan plan;
    plan.qoff.assign(1, 0);
    for (int q = 0; q < nq; ++q) {
        std::vector<RPlanField> sub(fields);
        for (int f = 0; f < nf; ++f)
            if (queue_of[f] != q)
                sub[f].mode = 0;
        std::string e;
        const RPlan p = rplan(sub, bt, std::max(1, slots / nq), &e);
        if (!e.empty()) {
            if (err)
                *err = e;
            return RPlan();
        }
        plan.order.insert(plan.order.end(), p.order.begin(), p.order.end());
        plan.qoff.push_back((int64_t)plan.order.size());
        plan.est_us = std::max(plan.est_us, p.est_us);
        plan.busy_us += p.busy_us;
    }
    return plan;
}

std::string rplan_check(const std::vector<RTask> &order, const std::vector<RPlanField> &fields)
{
    const int nf = (int)fields.size();
    std::vector<std::vector<int>> cnt(nf);
    std::vector<std::vector<char>> seen(nf);
    std::vector<int64_t> count(nf, 0);
    for (int f = 0; f < nf; ++f) {
        const int T = fields[f].T;
        if (T < 1 || T > 4096)
            return "field " + std::to_string(f) + ": tile count out of range";
        cnt[f].assign(rcount(T).size, 0);
        seen[f].assign((size_t)5 * 2 * T * T + 1, 0);
    }
    char buf[160];
    for (size_t q = 0; q < order.size(); ++q) {
        const RTask t = order[q];
        const int f = rt_field(t), ty = rt_type(t), i = rt_i(t), j = rt_j(t);
        if (f < 0 || f >= nf || ty > R_REDUCE) {
            std::snprintf(buf, sizeof buf, "ticket %zu: bad task", q);
            return buf;
        }
        const int T = fields[f].T, mode = fields[f].mode;
        bool ok = mode == 1 || mode == 2;
        if (ty == R_GEN || ty == R_CHOL || ty == R_RSOLVE)
            ok = ok && j >= 0 && j <= i && i < T;
        if (ty == R_RSOLVE || ty == R_LSOLVE)
            ok = ok && mode == 2;
        if (ty == R_LSOLVE)
            ok = ok && i >= 0 && i < T && j >= 0 && j < 2 * T;
        if (ty == R_REDUCE)
            ok = ok && i == 0 && j == 0;
        if (!ok) {
            std::snprintf(buf, sizeof buf, "ticket %zu: task (%d, %d, %d) not in field %d", q, ty, i,
                          j, f);
            return buf;
        }
        const size_t key = (size_t)ty * 2 * T * T + (size_t)i * 2 * T + j;
        if (seen[f][key]) {
            std::snprintf(buf, sizeof buf, "ticket %zu: task (%d, %d, %d) of field %d repeated", q,
                          ty, i, j, f);
            return buf;
        }
        seen[f][key] = 1;
        ++count[f];
        int off[4], need[4];
        const int k = rdeps(t, T, mode, off, need);
        for (int a = 0; a < k; ++a)
            if (cnt[f][off[a]] < need[a]) {
                std::snprintf(buf, sizeof buf,
                              "ticket %zu: task (%d, %d, %d) of field %d waits for counter %d >= "
                              "%d, which is %d",
                              q, ty, i, j, f, off[a], need[a], cnt[f][off[a]]);
                return buf;
            }
        const int kp = rpublish(t, T, off);
        for (int a = 0; a < kp; ++a)
            ++cnt[f][off[a]];
    }
    for (int f = 0; f < nf; ++f)
        if (count[f] != rtask_count(fields[f].T, fields[f].mode)) {
            std::snprintf(buf, sizeof buf, "field %d: %lld tasks, expected %lld", f,
                          (long long)count[f], (long long)rtask_count(fields[f].T, fields[f].mode));
            return buf;
        }
    return "";
}

} // namespace fbt

extern "C" {

fbt_status fbt_round_plan(int32_t nf, const int64_t *n, const int32_t *mode, int32_t tile,
                          int32_t slots, int32_t queues, int64_t *ntasks, int32_t *tasks,
                          int64_t *qoff, double *est_us)
{
    if (nf < 0 || (nf > 0 && (!n || !mode)) || (tile != 64 && tile != 128) || slots < 1 ||
        queues < 1 || queues > 8 || !ntasks)
        return FBT_EINVAL;
    std::vector<fbt::RPlanField> pf(nf);
    for (int32_t f = 0; f < nf; ++f) {
        if (n[f] < 1 || n[f] > ((int64_t)1 << 20))
            return FBT_EINVAL;
        pf[f] = {n[f], (int)((n[f] + 1 + tile - 1) / tile),
                 (mode[f] == 1 || mode[f] == 2) ? mode[f] : 0};
    }
    std::string err;
    const fbt::RPlan plan = fbt::rplan_queues(pf, tile, slots, queues, &err);
    if (!err.empty())
        return FBT_EINVAL;
    *ntasks = (int64_t)plan.order.size();
    if (qoff)
        for (size_t q = 0; q < plan.qoff.size(); ++q)
            qoff[q] = plan.qoff[q];
    if (tasks)
        for (size_t q = 0; q < plan.order.size(); ++q) {
            tasks[2 * q] = plan.order[q].ft;
            tasks[2 * q + 1] = plan.order[q].ij;
        }
    if (est_us)
        *est_us = plan.est_us;
    return FBT_OK;
}

int32_t fbt_round_task_deps(int32_t T, int32_t mode, int32_t ft, int32_t ij, int32_t *off,
                            int32_t *need, int32_t *pub, int32_t *npub)
{
    fbt::RTask t;
    t.ft = ft;
    t.ij = ij;
    int o[4], nd[4], p[4];
    const int k = fbt::rdeps(t, T, mode, o, nd);
    const int kp = fbt::rpublish(t, T, p);
    for (int a = 0; a < k; ++a) {
        if (off)
            off[a] = o[a];
        if (need)
            need[a] = nd[a];
    }
    for (int a = 0; a < kp; ++a)
        if (pub)
            pub[a] = p[a];
    if (npub)
        *npub = kp;
    return k;
}

} // extern "C"
