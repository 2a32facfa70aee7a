// Batched Gauss-Newton solves of many independent instances of uneven size
// (different grids, row counts and regularisation weights): a native executor
// that overlaps the instances on the GPU, and a small autotuner.
//
// Executor: the instances are sorted by decreasing work (N * (m + 1)) and
// pulled from a shared queue by nworkers host threads. Each thread drives one
// worker: a HIP stream (default priority) and one context per (grid,
// precision, smoother schedule, beta, graph replay) it has met, so the
// hierarchy, the coarsest inverse and the device workspace are set up once
// per key and reused by later instances. Workers are kept for the process
// (per device, at most kMaxCtxPerWorker contexts each, the least recently
// used one dropped beyond that) and handed to later batches, so a batch on
// grids seen before allocates and frees no device memory. A worker's two
// streams (its work stream and the stream its contexts capture V-cycle graphs
// on) are created once, one thread at a time, and never destroyed, so no
// stream is created or destroyed while other workers synchronise theirs. The
// solve of one instance is the library's own h1w_gn_solve path; the workers'
// streams let the small kernels and host round trips of different instances
// overlap.
//
// Autotuner: it picks the smoother schedule of the V-cycle, i.e. the lower
// end of the Chebyshev interval for eig(D^-1 A) at the batch's number of
// smoothing steps (the upper end stays 2, a bound of that spectrum), per
// (grid, precision) key: the schedule changes B, not J, so the rows and alpha
// of an instance do not enter, and one context per grid serves every instance
// of it. The worker that meets a key first solves that instance with each
// candidate interval and then the default, back to back on its own stream.
// The candidates differ only in the smoother's Chebyshev weights (the same
// kernels and launches per CG iteration), so the one with the fewest CG
// iterations has the shortest time to solution; the tuner compares iteration
// counts, which, unlike the wall time of one small solve while other workers
// share the GPU, do not depend on timing; a tie keeps the default. On the 2D
// grids of the batch workload [0.4, 2] and [0.5, 2] need 6 iterations where
// the default [0.3, 2] needs 7; on 3D grids all three need 7. The losing
// candidates' contexts are dropped at once, so that they do not push the
// contexts later batches use out of the worker's cache. The default's solve
// is the instance's result; while a key is being tuned, other workers solve
// its instances with the default. Tuned keys are kept for the process: a
// later batch reuses them (autotune = 1) or tunes them again (autotune = 2).
// In the grouped mode the tuning worker solves the whole group with each
// candidate and the default, and keeps the schedule with the least work (the
// instances' iterations weighted by m + 1): one instance's iterations need
// not show what a schedule does to the rest of its group.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <vector>

#include "context.h"

namespace h1w {

namespace {

// smoother schedules tried by the tuner (lower Chebyshev bound with the
// upper bound kChebHiDefault; 0 = the default interval, last: its solution
// is kept)
constexpr double kTuneLo[] = {0.4, 0.5, 0.0};
constexpr int kNumCandidates = 3;

struct GridKey {
    int dim, n0, n1, n2, precision, nu;
    double cheb_lo;  // 0: the default interval
    double beta;
    bool graphs;
    bool operator<(const GridKey& o) const {
        return std::tie(dim, n0, n1, n2, precision, nu, cheb_lo, beta, graphs) <
               std::tie(o.dim, o.n0, o.n1, o.n2, o.precision, o.nu, o.cheb_lo, o.beta, o.graphs);
    }
};

// a grid within one batch (its items must share beta)
struct ShapeKey {
    int dim, n0, n1, n2;
    bool operator<(const ShapeKey& o) const {
        return std::tie(dim, n0, n1, n2) < std::tie(o.dim, o.n0, o.n1, o.n2);
    }
};

constexpr int kMaxCtxPerWorker = 24;

struct TuneKey {
    int dim, n0, n1, n2, precision, nu;  // nu: the batch's smoothing steps, which the interval goes with
    bool grouped;                        // chosen for the grouped mode (by a whole group's steps)
    bool operator<(const TuneKey& o) const {
        return std::tie(dim, n0, n1, n2, precision, nu, grouped) <
               std::tie(o.dim, o.n0, o.n1, o.n2, o.precision, o.nu, o.grouped);
    }
};

int row_bucket(int m) {
    int b = 0;
    while ((1 << b) < std::max(1, m)) ++b;
    return b;
}

// Candidate choice for one tuning key, shared by all workers.
struct TuneState {
    bool claimed = false;                    // a worker is tuning (or has tuned) the key
    bool done = false;
    bool reused = false;                     // taken from an earlier batch of the process
    double best = -1.0;                      // wall time per N (m + 1) of the chosen candidate
    double best_lo = 0.0;                    // its lower Chebyshev bound (0: the default)
    int best_iters = 0, def_iters = 0;       // CG iterations of the chosen candidate and the default
    int bucket = 0;                          // ceil(log2 m) of the instance it was tuned on
};

// tuning results of earlier batches in this process
std::mutex g_tuned_mu;
std::map<TuneKey, TuneState> g_tuned;

// The tuning keys met by one batch call, shared by its workers.
struct BatchTuner {
    int autotune = 0;
    std::mutex mu;
    std::map<TuneKey, TuneState> keys;

    // schedule (lower Chebyshev bound, 0 = the default) for key tk; tuning:
    // the caller tunes the key now (and runs the default meanwhile)
    double choose(const TuneKey& tk, bool& tuning) {
        tuning = false;
        if (!autotune) return 0.0;
        std::lock_guard<std::mutex> lk(mu);
        TuneState& ts = keys[tk];
        if (!ts.claimed && autotune == 1) {  // a choice of an earlier batch
            std::lock_guard<std::mutex> lg(g_tuned_mu);
            auto f = g_tuned.find(tk);
            if (f != g_tuned.end()) {
                ts = f->second;
                ts.reused = true;
            }
        }
        if (!ts.claimed) {
            ts.claimed = true;
            tuning = true;
            return 0.0;
        }
        return ts.done ? ts.best_lo : 0.0;
    }

    void finish(const TuneKey& tk, double lo, double t_norm, int its, int its_def, int bucket) {
        std::lock_guard<std::mutex> lk(mu);
        TuneState& ts = keys[tk];
        ts.best = t_norm;
        ts.best_lo = lo;
        ts.best_iters = its;
        ts.def_iters = its_def;
        ts.bucket = bucket;
        ts.done = true;
    }

    // keeps the choices made by this batch for later ones and lists the
    // batch's keys in the report
    void publish(h1w_batch_report* report) {
        if (autotune) {
            std::lock_guard<std::mutex> lk(g_tuned_mu);
            for (const auto& [tk, ts] : keys)
                if (ts.done && !ts.reused) g_tuned[tk] = ts;
        }
        if (!report) return;
        int k = 0;
        for (const auto& [tk, ts] : keys) {
            if (k >= H1W_BATCH_MAX_KEYS) break;
            h1w_batch_tuned& r = report->tuned[k++];
            r.dim = tk.dim;
            r.n[0] = tk.n0;
            r.n[1] = tk.n1;
            r.n[2] = tk.n2;
            r.m_bucket = ts.bucket;
            r.nu = tk.nu;
            r.cheb_lo = ts.best_lo > 0.0 ? ts.best_lo : kChebLoDefault;
            r.iters = ts.best_iters;
            r.iters_default = ts.def_iters;
            r.ms_per_unit = ts.best;
            r.reused = ts.reused ? 1 : 0;
            r.grouped = tk.grouped ? 1 : 0;
        }
        report->ntuned = k;
    }
};

// the default schedule is the last candidate: in the per-instance mode its
// solve is the instance's result
constexpr int kDefaultCandidate = kNumCandidates - 1;
static_assert(kTuneLo[kDefaultCandidate] == 0.0, "the default schedule is tried last");

// The schedule to keep, from a cost per candidate (CG iterations, or a
// weighted sum of them; negative: the candidate failed): another candidate
// replaces the default only with a lower cost (or when the default failed).
// Returns its index into kTuneLo, or -1 when every candidate failed.
template <typename T>
int pick_candidate(const T* cost) {
    int best = -1;
    for (int c = 0; c < kDefaultCandidate; ++c)
        if (cost[c] >= 0 && (best < 0 || cost[c] < cost[best])) best = c;
    if (cost[kDefaultCandidate] >= 0 && (best < 0 || cost[best] >= cost[kDefaultCandidate]))
        return kDefaultCandidate;
    return best;
}

struct Worker {
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;  // lent to its contexts for V-cycle graph captures
    std::map<GridKey, std::unique_ptr<Ctx>> ctxs;
    std::map<GridKey, uint64_t> last_use;
    uint64_t clock = 0;
};

// Idle workers per device. Never destroyed: the workers' streams and device
// buffers are reclaimed with the process, so no HIP call runs during exit.
struct WorkerPool {
    std::mutex mu;
    std::map<int, std::vector<Worker*>> idle;
};

WorkerPool& worker_pool() {
    static WorkerPool* p = new WorkerPool();
    return *p;
}

}  // namespace

namespace {

// Grouped (lock-step) mode: the items of one grid form a group solved by
// Ctx::gn_group_solve on one worker; the groups are spread over the workers.
void batch_solve_grouped(int count, const h1w_batch_item* items, const h1w_batch_opts& o, h1w_info* infos,
                         h1w_status* status, h1w_batch_report* report, std::vector<std::string>& item_err,
                         int device) {
    constexpr int kMaxGroup = 256;  // items per lock-step group (larger grids' groups are cut)
    const int nu_fixed = o.nu > 0 ? o.nu : 2;
    item_err.assign(count, std::string());
    // groups of item indices per grid, in first-seen order, cut at kMaxGroup
    std::map<std::tuple<int, int, int, int, double>, std::vector<int>> by_grid;
    std::vector<std::vector<int>> groups;
    for (int i = 0; i < count; ++i) {
        const h1w_batch_item& it = items[i];
        if (status) status[i] = H1W_OK;
        if (infos) infos[i] = h1w_info{};
        if ((it.dim != 2 && it.dim != 3) || it.m < 0 || it.m > Ctx::kGroupMaxRows || !std::isfinite(it.beta)) {
            if (status) status[i] = H1W_EINVAL;
            item_err[i] = "grouped items need dim 2 or 3, 0 <= m <= 128 and a finite beta";
            continue;
        }
        const int n2 = it.dim == 3 ? it.n[2] : 1;
        auto& v = by_grid[{it.dim, it.n[0], it.n[1], n2, it.beta}];
        v.push_back(i);
        if ((int)v.size() == kMaxGroup) {
            groups.push_back(std::move(v));
            v.clear();
        }
    }
    for (auto& [key, v] : by_grid)
        if (!v.empty()) groups.push_back(std::move(v));
    // larger groups (by work) first
    auto gwork = [&](const std::vector<int>& v) {
        double w = 0.0;
        for (int i : v) {
            double nn = 1.0;
            for (int a = 0; a < items[i].dim; ++a) nn *= items[i].n[a];
            w += nn * (items[i].m + 1);
        }
        return w;
    };
    std::stable_sort(groups.begin(), groups.end(),
                     [&](const std::vector<int>& a, const std::vector<int>& b) { return gwork(a) > gwork(b); });

    const int nworkers = std::clamp(o.nworkers > 0 ? o.nworkers : 8, 1, 16);
    const int nw = std::max(1, std::min(nworkers, (int)groups.size()));
    std::vector<Worker*> workers(nw, nullptr);
    {
        std::lock_guard<std::mutex> lk(worker_pool().mu);
        auto& idle = worker_pool().idle[device];
        for (int w = 0; w < nw; ++w) {
            if (!idle.empty()) {
                workers[w] = idle.back();
                idle.pop_back();
            } else {
                workers[w] = new Worker();
            }
        }
    }
    BatchTuner tuner;
    tuner.autotune = o.autotune;
    std::atomic<int> next{0};
    std::vector<std::string> worker_err(nw);
    auto run = [&](int w) {
        Worker& me = *workers[w];
        try {
            H1W_HIP(hipSetDevice(device));
            if (!me.stream) {
                std::lock_guard<std::recursive_mutex> lk(capture_lock());
                H1W_HIP(hipStreamCreateWithFlags(&me.stream, hipStreamNonBlocking));
            }
        } catch (const Error& e) {
            worker_err[w] = e.msg;
            return;
        }
        for (;;) {
            const int q = next.fetch_add(1);
            if (q >= (int)groups.size()) break;
            const std::vector<int>& grp = groups[q];
            const h1w_batch_item& i0 = items[grp[0]];
            const int n2 = i0.dim == 3 ? i0.n[2] : 1;
            const TuneKey tk{i0.dim, i0.n[0], i0.n[1], n2, o.precision, nu_fixed, true};
            bool tuning = false;
            const double lo0 = tuner.choose(tk, tuning);
            auto gkey = [&](double lo_c) {
                return GridKey{i0.dim, i0.n[0], i0.n[1], n2, o.precision, nu_fixed, lo_c, i0.beta, false};
            };
            std::vector<GridKey> used;  // contexts this group ran on (dropped if it fails)
            auto drop = [&](const GridKey& gk) {
                me.ctxs.erase(gk);
                me.last_use.erase(gk);
            };
            auto ctx_for = [&](double lo_c) -> Ctx& {
                const GridKey gk = gkey(lo_c);
                me.last_use[gk] = ++me.clock;
                used.push_back(gk);
                auto& slot = me.ctxs[gk];
                if (!slot) {
                    while ((int)me.ctxs.size() > kMaxCtxPerWorker) {
                        auto victim = me.ctxs.end();
                        uint64_t oldest = UINT64_MAX;
                        for (auto c = me.ctxs.begin(); c != me.ctxs.end(); ++c)
                            if (c->second && me.last_use[c->first] < oldest) {
                                oldest = me.last_use[c->first];
                                victim = c;
                            }
                        if (victim == me.ctxs.end()) break;
                        me.last_use.erase(victim->first);
                        me.ctxs.erase(victim);
                    }
                    h1w_grid_desc d{};
                    d.dim = i0.dim;
                    d.n[0] = i0.n[0];
                    d.n[1] = i0.n[1];
                    d.n[2] = n2;
                    d.beta = i0.beta;
                    d.precision = o.precision;
                    d.nu = nu_fixed;
                    if (lo_c > 0.0) {
                        d.cheb_lo = lo_c;
                        d.cheb_hi = kChebHiDefault;
                    }
                    auto c = std::make_unique<Ctx>();
                    c->init(d, me.stream);
                    me.ctxs[gk] = std::move(c);
                }
                return *me.ctxs[gk];
            };
            std::vector<h1w_info> ginf(grp.size(), h1w_info{});
            std::vector<h1w_status> gst(grp.size(), H1W_OK);  // each item's own outcome
            h1w_status st = H1W_OK;                            // a failure of the whole group
            std::string msg;
            try {
                std::vector<Ctx::GroupItem> gi(grp.size());
                for (size_t k = 0; k < grp.size(); ++k) {
                    const h1w_batch_item& it = items[grp[k]];
                    gi[k] = Ctx::GroupItem{it.m, it.J, it.ldj, it.alpha, it.b, it.x};
                }
                h1w_solve_opts so{};
                so.rtol = o.rtol;
                so.maxit = o.maxit;
                double lo = lo0;
                bool have_result = false;  // ginf and the items' x hold the chosen schedule's solve
                double ms = 0.0;
                if (tuning) {
                    // the whole group with each candidate and then the default
                    // (its solve stays the result if it is kept); the choice
                    // is the schedule with the least work: the items' CG
                    // iterations weighted by m + 1 (a converged item drops out
                    // of the group's passes). A candidate counts only if it
                    // solved every item.
                    double cost[kNumCandidates], tms[kNumCandidates];
                    int sum_it[kNumCandidates];
                    Error def_err{H1W_OK, ""};
                    bool def_ran = false;
                    std::vector<h1w_status> cst(grp.size());
                    for (int c = 0; c < kNumCandidates; ++c) {
                        cost[c] = -1.0;
                        Ctx& cx = ctx_for(kTuneLo[c]);
                        cx.sync();
                        const auto t0 = std::chrono::steady_clock::now();
                        try {  // a candidate that fails (e.g. no convergence) is skipped
                            cx.gn_group_solve((int)grp.size(), gi.data(), so, ginf.data(), cst.data());
                        } catch (const Error& e) {
                            used.pop_back();
                            drop(gkey(kTuneLo[c]));
                            if (c == kDefaultCandidate) def_err = e;
                            continue;
                        }
                        tms[c] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
                        if (c == kDefaultCandidate) {
                            def_ran = true;
                            gst = cst;
                        }
                        if (std::any_of(cst.begin(), cst.end(), [](h1w_status v) { return v != H1W_OK; })) continue;
                        cost[c] = 0.0;
                        sum_it[c] = 0;
                        for (size_t k = 0; k < gi.size(); ++k) {
                            cost[c] += (double)ginf[k].iters * (gi[k].m + 1);
                            sum_it[c] += ginf[k].iters;
                        }
                    }
                    int pick = pick_candidate(cost);
                    if (pick < 0) {
                        // no schedule solved every item: the default's solve
                        // (the last one) is the result, its failures the items'
                        if (!def_ran) throw def_err;
                        pick = kDefaultCandidate;
                        sum_it[pick] = -1;
                    }
                    double nn = 1.0, work = 0.0;
                    for (int a = 0; a < i0.dim; ++a) nn *= i0.n[a];
                    for (const auto& g : gi) work += nn * (g.m + 1);
                    lo = kTuneLo[pick];
                    tuner.finish(tk, lo, tms[pick] / work, sum_it[pick],
                                 cost[kDefaultCandidate] >= 0.0 ? sum_it[kDefaultCandidate] : -1, row_bucket(i0.m));
                    for (int c = 0; c < kDefaultCandidate; ++c)
                        if (c != pick && cost[c] >= 0.0) drop(gkey(kTuneLo[c]));
                    if (pick == kDefaultCandidate) {
                        have_result = true;
                        ms = tms[pick];
                    } else {
                        drop(gkey(0.0));
                    }
                }
                if (!have_result) {
                    Ctx& cx = ctx_for(lo);
                    const auto t0 = std::chrono::steady_clock::now();
                    cx.gn_group_solve((int)grp.size(), gi.data(), so, ginf.data(), gst.data());
                    ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
                }
                for (auto& f : ginf) f.t_total_ms = ms;
            } catch (const Error& e) {
                st = e.st;
                msg = e.msg;
            } catch (const std::bad_alloc&) {
                st = H1W_ENOMEM;
                msg = "host allocation failed";
            } catch (const std::exception& e) {
                st = H1W_EINVAL;
                msg = e.what();
            }
            if (st != H1W_OK)  // a context left by a failed group is not reused
                for (const GridKey& gk : used) drop(gk);
            for (size_t k = 0; k < grp.size(); ++k) {
                const h1w_status sk = st != H1W_OK ? st : gst[k];
                if (infos) infos[grp[k]] = ginf[k];
                if (status) status[grp[k]] = sk;
                if (st != H1W_OK)
                    item_err[grp[k]] = msg;
                else if (sk == H1W_ENOCONV)
                    item_err[grp[k]] = "grouped GN-CG: missed rtol on its true residual within maxit iterations";
                else if (sk != H1W_OK)
                    item_err[grp[k]] = "grouped GN-CG: non-finite values or a breakdown in this instance";
            }
        }
    };
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<std::thread> threads;
    threads.reserve(nw);
    for (int w = 0; w < nw; ++w) threads.emplace_back(run, w);
    for (auto& t : threads) t.join();
    const double total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    {
        std::lock_guard<std::mutex> lk(worker_pool().mu);
        auto& idle = worker_pool().idle[device];
        for (Worker* w : workers) idle.push_back(w);
    }
    for (const auto& e : worker_err)
        if (!e.empty()) throw Error{H1W_EHIP, "batch worker setup failed: " + e};
    if (report) {
        *report = h1w_batch_report{};
        report->t_total_ms = total_ms;
        report->nworkers = nw;
    }
    tuner.publish(report);
}

// One solve per item on the workers' streams.
void batch_solve_each(int count, const h1w_batch_item* items, const h1w_batch_opts& o, h1w_info* infos,
                      h1w_status* status, h1w_batch_report* report, std::vector<std::string>& item_err,
                      int device) {
    const int nworkers = std::clamp(o.nworkers > 0 ? o.nworkers : 8, 1, 16);
    const int nu_fixed = o.nu > 0 ? o.nu : 2;

    // decreasing work first, so the long solves do not finish last
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    auto work = [&](int i) {
        const h1w_batch_item& it = items[i];
        double nn = 1.0;
        for (int a = 0; a < it.dim; ++a) nn *= it.n[a];
        return nn * (it.m + 1);
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work(a) > work(b); });

    BatchTuner tuner;
    tuner.autotune = o.autotune;
    std::atomic<int> next{0};
    std::vector<Worker*> workers(nworkers, nullptr);
    {
        std::lock_guard<std::mutex> lk(worker_pool().mu);
        auto& idle = worker_pool().idle[device];
        for (int w = 0; w < nworkers; ++w) {
            if (!idle.empty()) {
                workers[w] = idle.back();
                idle.pop_back();
            } else {
                workers[w] = new Worker();
            }
        }
    }
    // each item's grid must keep the beta of the first item of that grid
    std::map<ShapeKey, double> grid_beta;
    for (int i = 0; i < count; ++i) {
        const h1w_batch_item& it = items[i];
        if (it.dim != 2 && it.dim != 3) continue;  // reported per item below
        grid_beta.emplace(ShapeKey{it.dim, it.n[0], it.n[1], it.dim == 3 ? it.n[2] : 1}, it.beta);
    }
    std::vector<std::string> worker_err(nworkers);
    item_err.assign(count, std::string());

    auto run = [&](int w) {
        Worker& me = *workers[w];
        try {
            H1W_HIP(hipSetDevice(device));
            if (!me.stream) {
                std::lock_guard<std::recursive_mutex> lk(capture_lock());
                H1W_HIP(hipStreamCreateWithFlags(&me.stream, hipStreamNonBlocking));
            }
            if (o.graphs && !me.cap_stream) {
                std::lock_guard<std::recursive_mutex> lk(capture_lock());
                H1W_HIP(hipStreamCreateWithFlags(&me.cap_stream, hipStreamNonBlocking));
            }
        } catch (const Error& e) {
            worker_err[w] = e.msg;
            return;
        }
        for (;;) {
            const int q = next.fetch_add(1);
            if (q >= count) break;
            const int i = order[q];
            const h1w_batch_item& it = items[i];
            h1w_info inf{};
            h1w_status st = H1W_OK;
            std::vector<GridKey> used;  // contexts this item ran on (dropped if it fails)
            auto drop = [&](const GridKey& gk) {
                me.ctxs.erase(gk);
                me.last_use.erase(gk);
            };
            try {
                require(it.dim == 2 || it.dim == 3, "item dim must be 2 or 3");
                require(it.m >= 0, "item m must be >= 0");
                require(it.b != nullptr && it.x != nullptr && (it.m == 0 || it.J != nullptr),
                        "item b, x (and J when m > 0) must not be NULL");
                const int n2 = it.dim == 3 ? it.n[2] : 1;
                TuneKey tk{it.dim, it.n[0], it.n[1], n2, o.precision, nu_fixed, false};
                bool tuning = false;
                const double lo = tuner.choose(tk, tuning);
                require(std::isfinite(it.beta) && it.beta == grid_beta[ShapeKey{it.dim, it.n[0], it.n[1], n2}],
                        "items of one grid must share beta within a batch");
                auto gkey = [&](double lo_c) {
                    return GridKey{it.dim, it.n[0], it.n[1], n2, o.precision, nu_fixed, lo_c, it.beta, o.graphs != 0};
                };
                auto ctx_for = [&](double lo_c) -> Ctx& {
                    const GridKey gk = gkey(lo_c);
                    me.last_use[gk] = ++me.clock;
                    used.push_back(gk);
                    auto& slot = me.ctxs[gk];
                    if (!slot) {
                        // beyond the cap, drop the least recently used context
                        while ((int)me.ctxs.size() > kMaxCtxPerWorker) {
                            auto victim = me.ctxs.end();
                            uint64_t oldest = UINT64_MAX;
                            for (auto c = me.ctxs.begin(); c != me.ctxs.end(); ++c)
                                if (c->second && me.last_use[c->first] < oldest) {
                                    oldest = me.last_use[c->first];
                                    victim = c;
                                }
                            if (victim == me.ctxs.end()) break;
                            me.last_use.erase(victim->first);
                            me.ctxs.erase(victim);
                        }
                        h1w_grid_desc d{};
                        d.dim = it.dim;
                        d.n[0] = it.n[0];
                        d.n[1] = it.n[1];
                        d.n[2] = n2;
                        d.beta = it.beta;
                        d.precision = o.precision;
                        d.nu = nu_fixed;
                        if (lo_c > 0.0) {
                            d.cheb_lo = lo_c;
                            d.cheb_hi = kChebHiDefault;
                        }
                        d.flags = o.graphs ? H1W_FLAG_GRAPH_VCYCLE : 0u;
                        auto c = std::make_unique<Ctx>();
                        c->init(d, me.stream);
                        if (o.graphs) {  // no stream is created or destroyed with a batch context
                            c->cap_stream = me.cap_stream;
                            c->own_cap_stream = false;
                        }
                        me.ctxs[gk] = std::move(c);
                    }
                    return *me.ctxs[gk];
                };
                require(std::isfinite(it.alpha) && it.alpha > 0.0, "item alpha must be finite and > 0");
                require(it.m == 0 || it.ldj >= ctx_for(lo).N(), "item ldj must be >= N");
                h1w_solve_opts so{};
                so.rtol = o.rtol;
                so.maxit = o.maxit;
                if (!tuning) {
                    ctx_for(lo).gn_solve(it.m, it.J, it.ldj, it.alpha, it.b, nullptr, nullptr, it.x, so, &inf);
                } else {
                    // the candidates on this instance, the default last (its x is the result)
                    int its[kNumCandidates];
                    double tms[kNumCandidates];
                    for (int c = 0; c < kNumCandidates; ++c) {
                        its[c] = -1;
                        const double lo_c = kTuneLo[c];
                        Ctx& cx = ctx_for(lo_c);
                        cx.sync();
                        const auto t0 = std::chrono::steady_clock::now();
                        if (c == kDefaultCandidate) {
                            cx.gn_solve(it.m, it.J, it.ldj, it.alpha, it.b, nullptr, nullptr, it.x, so, &inf);
                        } else {
                            try {  // a candidate that fails (e.g. no convergence) is skipped
                                cx.gn_solve(it.m, it.J, it.ldj, it.alpha, it.b, nullptr, nullptr, it.x, so, &inf);
                            } catch (const Error&) {
                                used.pop_back();
                                drop(gkey(lo_c));
                                continue;
                            }
                        }
                        tms[c] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
                        its[c] = inf.iters;
                    }
                    const int pick = pick_candidate(its);  // the default ran, so pick >= 0
                    tuner.finish(tk, kTuneLo[pick], tms[pick] / work(i), its[pick], its[kDefaultCandidate],
                                 row_bucket(it.m));
                    // the losing candidates' contexts are not used again by
                    // this key: dropped now (in the tuning call) rather than
                    // by the LRU cap later, when a timed batch would pay for
                    // re-creating what they pushed out
                    for (int c = 0; c < kDefaultCandidate; ++c)
                        if (c != pick && its[c] >= 0) drop(gkey(kTuneLo[c]));
                }
            } catch (const Error& e) {
                st = e.st;
                item_err[i] = e.msg;
            } catch (const std::bad_alloc&) {
                st = H1W_ENOMEM;
                item_err[i] = "host allocation failed";
            } catch (const std::exception& e) {
                st = H1W_EINVAL;
                item_err[i] = e.what();
            }
            if (st != H1W_OK)  // a context left by a failed solve is not reused
                for (const GridKey& gk : used) drop(gk);
            if (infos) infos[i] = inf;
            if (status) status[i] = st;
        }
    };

    const auto t0 = std::chrono::steady_clock::now();
    std::vector<std::thread> threads;
    threads.reserve(nworkers);
    for (int w = 0; w < nworkers; ++w) threads.emplace_back(run, w);
    for (auto& t : threads) t.join();
    const double total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();

    // the workers go back to the pool with their streams and contexts
    {
        std::lock_guard<std::mutex> lk(worker_pool().mu);
        auto& idle = worker_pool().idle[device];
        for (Worker* w : workers) idle.push_back(w);
    }
    for (const auto& e : worker_err)
        if (!e.empty()) throw Error{H1W_EHIP, "batch worker setup failed: " + e};
    if (report) {
        *report = h1w_batch_report{};
        report->t_total_ms = total_ms;
        report->nworkers = nworkers;
    }
    tuner.publish(report);
}

}  // namespace

void batch_solve(int count, const h1w_batch_item* items, const h1w_batch_opts& o, h1w_info* infos,
                 h1w_status* status, h1w_batch_report* report, std::string* first_err) {
    int device = 0;
    H1W_HIP(hipGetDevice(&device));
    std::vector<std::string> item_err;
    // grouped mode: items with more rows than a group's instance may hold are
    // solved one at a time after the groups
    std::vector<int> big;
    if (o.grouped)
        for (int i = 0; i < count; ++i)
            if (items[i].m > Ctx::kGroupMaxRows) big.push_back(i);
    if (!o.grouped) {
        batch_solve_each(count, items, o, infos, status, report, item_err, device);
    } else if (big.empty()) {
        batch_solve_grouped(count, items, o, infos, status, report, item_err, device);
    } else {
        std::vector<int> small;
        for (int i = 0, b = 0; i < count; ++i) {
            if (b < (int)big.size() && big[b] == i) ++b;
            else small.push_back(i);
        }
        item_err.assign(count, std::string());
        h1w_batch_report reps[2];
        int nrep = 0;
        auto run = [&](const std::vector<int>& idx, bool grouped) {
            if (idx.empty()) return;
            const int n = (int)idx.size();
            std::vector<h1w_batch_item> sub(n);
            for (int k = 0; k < n; ++k) sub[k] = items[idx[k]];
            std::vector<h1w_info> sinf(n);
            std::vector<h1w_status> sst(n, H1W_OK);
            std::vector<std::string> serr;
            h1w_batch_report& rep = reps[nrep++];
            rep = h1w_batch_report{};
            h1w_batch_opts so = o;
            so.grouped = grouped ? 1 : 0;
            if (grouped) batch_solve_grouped(n, sub.data(), so, sinf.data(), sst.data(), &rep, serr, device);
            else batch_solve_each(n, sub.data(), so, sinf.data(), sst.data(), &rep, serr, device);
            for (int k = 0; k < n; ++k) {
                if (infos) infos[idx[k]] = sinf[k];
                if (status) status[idx[k]] = sst[k];
                item_err[idx[k]] = serr[k];
            }
        };
        run(small, true);
        run(big, false);
        if (report) {
            *report = h1w_batch_report{};
            for (int r = 0; r < nrep; ++r) {
                report->t_total_ms += reps[r].t_total_ms;
                report->nworkers = std::max(report->nworkers, reps[r].nworkers);
                for (int k = 0; k < reps[r].ntuned && report->ntuned < H1W_BATCH_MAX_KEYS; ++k)
                    report->tuned[report->ntuned++] = reps[r].tuned[k];
            }
        }
    }
    if (first_err) {
        first_err->clear();
        for (int i = 0; i < count && first_err->empty(); ++i)
            if (!item_err[i].empty()) *first_err = "item " + std::to_string(i) + ": " + item_err[i];
    }
}

}  // namespace h1w
