// Continuous-batching query server (the interactive feedback loop of Section 5.2.2 at scale).
//
// A request is a graph handle plus evidence clamps and run parameters. One host thread runs the
// loop: admit waiting requests in arrival order while the number of active runs stays within
// max_active and the device state of the server's graphs within the memory budget (a graph with a
// request in flight is not admitted twice: its messages are one state), advance every active run
// by step_iters iterations in one persistent launch (one workgroup per run, so the runs overlap on
// the device; runs whose levels are too wide for one workgroup take the LEVELS executor on their
// own stream, concurrently with that launch), then retire the runs that finished and copy their
// marginals out. Requests that arrive while a step runs join at the next step.
//
// Device memory. Every graph submitted to the server is managed by it: the server counts the
// device state (messages, beliefs, potentials, marginals, run state) of those that are resident.
// Admitting a request whose graph is evicted allocates its state again and restores its messages;
// when that, or the graphs already resident, would exceed the budget, the server first evicts idle
// graphs (no request in flight), least recently used first: their messages go to host memory
// (exact bytes) and their device state is freed. A re-query after new evidence therefore starts
// warm whether its graph stayed resident or was evicted in between.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "fastlbp.h"
#include "internal.h"

using namespace fastlbp;
using Clock = std::chrono::steady_clock;

// Most iterations a wide run (LEVELS executor) advances per step when steps are sized in levels.
constexpr int32_t kWideStepIters = 32;
// Steps sized in levels grow by this factor while no request arrives: a request can only join at a
// step's end, so short steps keep admission and retirement prompt while requests come in, and long
// steps cut the launches (and host round trips) per iteration of the runs still going once they stop.
constexpr int32_t kQuietStepFactor = 4;

namespace {

struct Request {
    uint64_t ticket = 0;
    fastlbp_graph *g = nullptr;
    std::vector<int32_t> ev_vars;
    std::vector<int8_t> ev_vals;
    int32_t max_iters = 0;
    double tol = 0.0, damping = 0.0;
    Clock::time_point t_submit, t_start, t_done;
    int status = 1;  // 1 pending, 0 done, < 0 failed with that code
    std::string error;
    std::vector<double> p1;
    fastlbp_run_stats stats{};
    bool warm = false;
};

}  // namespace

struct fastlbp_server {
    fastlbp_server_options opts{};
    Launcher *launcher = nullptr;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> pending;
    std::vector<std::shared_ptr<Request>> active;
    std::unordered_map<uint64_t, std::shared_ptr<Request>> by_ticket;
    std::unordered_map<fastlbp_graph *, int> runs_of_graph;  // completed runs per handle (warm starts)
    std::unordered_set<fastlbp_graph *> managed;             // graphs submitted here (residency managed)
    uint64_t clock = 0;                                       // least-recently-used stamps
    uint64_t next_ticket = 1;
    uint64_t submitted = 0;  // requests submitted so far
    bool stop = false;
    std::thread th;
    // statistics
    std::vector<double> lat_ms;
    int64_t completed = 0, updates = 0, steps = 0, evictions = 0, restores = 0;
    size_t peak_resident = 0;
    int64_t persistent_launches = 0;
    double busy_ms = 0.0, kernel_ms = 0.0, method_bytes = 0.0, persistent_ms = 0.0, persistent_bytes = 0.0;
    Clock::time_point t0 = Clock::now();

    void loop();
    size_t resident_bytes() const {
        size_t t = 0;
        for (auto *g : managed)
            if (graph_resident(g)) t += graph_state_bytes(g);
        return t;
    }
    bool is_active(const fastlbp_graph *g) const {
        for (auto &a : active)
            if (a->g == g) return true;
        return false;
    }
    // Evicts idle managed graphs, least recently used first, until `need` more bytes fit the
    // budget or none is left; a graph whose handle is in use by the caller (lock held) is skipped.
    void make_room(size_t need, const fastlbp_graph *keep) {
        size_t cur = resident_bytes();
        if (cur + need <= opts.memory_budget) return;
        std::vector<fastlbp_graph *> idle;
        for (auto *g : managed)
            if (g != keep && graph_resident(g) && !is_active(g)) idle.push_back(g);
        std::sort(idle.begin(), idle.end(),
                  [](fastlbp_graph *a, fastlbp_graph *b) { return graph_last_use(a) < graph_last_use(b); });
        for (auto *g : idle) {
            if (cur + need <= opts.memory_budget) break;
            std::unique_lock<std::recursive_mutex> lk(graph_mutex(g), std::try_to_lock);
            if (!lk.owns_lock()) continue;
            const size_t b = graph_state_bytes(g);
            graph_evict(g);
            cur -= b;
            ++evictions;
        }
    }
};

namespace fastlbp {
void server_forget(fastlbp_server *s, fastlbp_graph *g) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->managed.erase(g);
    s->runs_of_graph.erase(g);
}
}  // namespace fastlbp

void fastlbp_server::loop() {
    (void)hipSetDevice(opts.device);
    std::vector<fastlbp_graph *> gs, narrow, wide;
    std::vector<double> damp, narrow_damp;
    std::vector<int32_t> narrow_step, maxit;
    // levels per step of the narrow runs: step_levels, or kQuietStepFactor times more when no
    // request arrived during the previous step and none waits (wide runs keep step_levels: each
    // captures its step's iterations in a hipGraph, which a changing step length would re-capture)
    uint64_t seen = 0;
    int64_t step_levels = opts.step_levels;
    // iterations a run advances per step: about `levels` levels (so a step costs about the same for
    // every run and small graphs are not held back by large ones), or step_iters
    auto iters_of = [&](int64_t levels, int32_t units, int32_t max_iters) {
        if (opts.step_levels <= 0) return opts.step_iters;
        const int64_t it = levels / std::max(1, units);
        return int32_t(std::max<int64_t>(1, std::min<int64_t>(std::max<int32_t>(1, max_iters), it)));
    };
    while (true) {
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return stop || !pending.empty() || !active.empty(); });
            if (stop && active.empty()) break;
            // admission: FIFO, skipping requests whose graph is busy; stop at the first request
            // that does not fit the memory budget
            for (auto it = pending.begin(); it != pending.end() && int(active.size()) < opts.max_active;) {
                auto r = *it;
                bool busy = false;
                for (auto &a : active) busy = busy || a->g == r->g;
                if (busy) {
                    ++it;
                    continue;
                }
                // device memory: make room by evicting idle graphs, then restore this one
                const size_t need = graph_resident(r->g) ? 0 : graph_state_bytes(r->g);
                try {
                    make_room(need, r->g);
                } catch (DeviceError &) {
                }
                if (!active.empty() && resident_bytes() + need > opts.memory_budget) break;
                it = pending.erase(it);
                try {
                    if (!graph_resident(r->g)) {
                        graph_restore(r->g);
                        ++restores;
                    }
                    int rc = set_evidence(r->g, int32_t(r->ev_vars.size()), r->ev_vars.data(), r->ev_vals.data());
                    if (rc) {
                        r->status = rc;
                        r->error = fastlbp_last_error();
                        cv_done.notify_all();
                        continue;
                    }
                    step_begin(r->g, r->max_iters, r->tol, 0);
                } catch (OomError &) {
                    r->status = FASTLBP_E_OOM;
                    r->error = "device allocation failed";
                    cv_done.notify_all();
                    continue;
                } catch (DeviceError &e) {
                    r->status = FASTLBP_E_DEVICE;
                    r->error = e.msg;
                    cv_done.notify_all();
                    continue;
                }
                r->warm = runs_of_graph[r->g] > 0;
                r->t_start = Clock::now();
                graph_last_use(r->g) = ++clock;
                active.push_back(r);
            }
            peak_resident = std::max(peak_resident, resident_bytes());
            const bool quiet = submitted == seen && pending.empty();
            seen = submitted;
            step_levels = int64_t(opts.step_levels) * (quiet ? kQuietStepFactor : 1);
            gs.clear();
            damp.clear();
            maxit.clear();
            for (auto &a : active) {
                gs.push_back(a->g);
                damp.push_back(a->damping);
                maxit.push_back(a->max_iters);
            }
        }
        if (gs.empty()) continue;
        // one step: every active run advances by up to step_iters iterations
        auto ts = Clock::now();
        std::vector<std::shared_ptr<Request>> finished;
        std::string err;
        float dev_ms = 0.f;
        double launch_bytes = -1.0;
        try {
            // wide runs first (asynchronous, each on its own stream), then the persistent launch of
            // the narrow runs, which overlaps them
            narrow.clear();
            wide.clear();
            narrow_damp.clear();
            narrow_step.clear();
            for (size_t i = 0; i < gs.size(); ++i) {
                if (graph_wide(gs[i])) {
                    wide.push_back(gs[i]);
                    // (at most kWideStepIters: each handle captures its step's iterations in a hipGraph)
                    step_levels_enqueue(gs[i], damp[i],
                                        std::min(kWideStepIters, iters_of(opts.step_levels, graph_launches_per_iter(gs[i]), maxit[i])));
                } else {
                    narrow.push_back(gs[i]);
                    narrow_damp.push_back(damp[i]);
                    narrow_step.push_back(iters_of(step_levels, graph_exec_levels(gs[i]), maxit[i]));
                }
            }
            if (!narrow.empty()) {
                std::vector<int32_t> it0(narrow.size());
                for (size_t i = 0; i < narrow.size(); ++i) it0[i] = graph_host_state(narrow[i]).iter;
                step_run(*launcher, int(narrow.size()), narrow.data(), narrow_damp.data(), narrow_step.data());
                dev_ms = launcher_kernel_ms(launcher);
                // method bytes of this persistent launch: each run's iterations in it
                double bytes = 0.0;
                for (size_t i = 0; i < narrow.size(); ++i)
                    bytes += graph_method_bytes_per_iter(narrow[i], graph_host_state(narrow[i]).tol, narrow_damp[i]) *
                             double(graph_host_state(narrow[i]).iter - it0[i]);
                launch_bytes = bytes;
            }
            for (auto *g : wide) dev_ms = std::max(dev_ms, step_levels_finish(g));
            // the persistent launch refreshed the narrow runs' host state; the wide ones are read
            for (auto *g : wide) read_state(g, launcher_stream(launcher));
        } catch (DeviceError &e) {
            err = e.msg;
            for (auto *g : wide) {
                try {
                    graph_sync(g);
                } catch (DeviceError &) {
                }
            }
        }
        double step_ms = std::chrono::duration<double, std::milli>(Clock::now() - ts).count();
        std::unique_lock<std::mutex> lk(mu);
        ++steps;
        busy_ms += step_ms;
        if (err.empty()) kernel_ms += dev_ms;
        if (err.empty() && launch_bytes >= 0.0) {
            ++persistent_launches;
            persistent_ms += launcher_kernel_ms(launcher);
            persistent_bytes += launch_bytes;
        }
        for (auto it = active.begin(); it != active.end();) {
            auto r = *it;
            const RunState &hs = graph_host_state(r->g);
            if (err.empty() && !hs.done) {
                ++it;
                continue;
            }
            if (!err.empty()) {
                r->status = FASTLBP_E_DEVICE;
                r->error = err;
            } else {
                try {
                    r->p1.resize(graph_num_vars(r->g));
                    marginals_into(r->g, r->p1.data());
                    fill_stats_public(r->g, r->stats, 0.f, r->damping);
                    r->status = 0;
                } catch (DeviceError &e) {
                    r->status = FASTLBP_E_DEVICE;
                    r->error = e.msg;
                }
            }
            r->t_done = Clock::now();
            runs_of_graph[r->g] += 1;
            graph_last_use(r->g) = ++clock;
            if (r->status == 0) {
                lat_ms.push_back(std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count());
                ++completed;
                updates += r->stats.message_updates;
                method_bytes += r->stats.method_bytes_per_iter * double(r->stats.iterations);
            }
            it = active.erase(it);
        }
        cv_done.notify_all();
    }
}

extern "C" {

void fastlbp_server_options_default(fastlbp_server_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->device = 0;
    o->precision = FASTLBP_FP32;
    o->max_active = 256;
    o->step_iters = 2;
    o->memory_budget = 0;
    o->step_levels = 2048;
}

int fastlbp_server_create(const fastlbp_server_options *opts, fastlbp_server_t *out) {
    clear_error();
    if (!out) {
        set_error("out is NULL");
        return FASTLBP_E_INVALID_ARG;
    }
    *out = nullptr;
    fastlbp_server_options o;
    fastlbp_server_options_default(&o);
    if (opts) o = *opts;
    if (o.max_active < 1 || o.step_iters < 1 || o.step_levels < 0 ||
        (o.precision != FASTLBP_FP32 && o.precision != FASTLBP_FP64)) {
        set_error("need max_active >= 1, step_iters >= 1, step_levels >= 0 and a valid precision");
        return FASTLBP_E_INVALID_ARG;
    }
    std::unique_ptr<fastlbp_server> s(new fastlbp_server());
    try {
        if (hipSetDevice(o.device) != hipSuccess) throw DeviceError{"hipSetDevice failed"};
        if (o.memory_budget == 0) {
            size_t free_b = 0, total_b = 0;
            if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) throw DeviceError{"hipMemGetInfo failed"};
            o.memory_budget = free_b / 10 * 8;
        }
        s->opts = o;
        s->launcher = launcher_create(o.device, nullptr, Alloc{});
    } catch (DeviceError &e) {
        (void)hipGetLastError();
        set_error(e.msg);
        return FASTLBP_E_DEVICE;
    } catch (OomError &) {
        set_error("device allocation failed");
        return FASTLBP_E_OOM;
    }
    s->th = std::thread([srv = s.get()] { srv->loop(); });
    *out = s.release();
    return FASTLBP_OK;
}

int fastlbp_server_submit(fastlbp_server_t s, fastlbp_graph_t g, int32_t n_ev, const int32_t *ev_vars,
                          const int8_t *ev_vals, int32_t max_iters, double tol, double damping, uint64_t *ticket) {
    clear_error();
    if (!s || !g || !ticket || n_ev < 0 || (n_ev > 0 && (!ev_vars || !ev_vals))) {
        set_error("invalid argument");
        return FASTLBP_E_INVALID_ARG;
    }
    if (max_iters < 0 || !(tol >= 0.0) || !(damping >= 0.0 && damping < 1.0)) {
        set_error("need max_iters >= 0, tol >= 0, 0 <= damping < 1");
        return FASTLBP_E_INVALID_ARG;
    }
    if (graph_device(g) != s->opts.device || graph_precision(g) != s->opts.precision) {
        set_error("graph device or precision differs from the server's");
        return FASTLBP_E_INVALID_ARG;
    }
    if (graph_state_bytes(g) > s->opts.memory_budget) {
        set_error("graph state exceeds the server's memory budget");
        return FASTLBP_E_TOO_LARGE;
    }
    auto r = std::make_shared<Request>();
    r->g = g;
    r->ev_vars.assign(ev_vars, ev_vars + n_ev);
    r->ev_vals.assign(ev_vals, ev_vals + n_ev);
    r->max_iters = max_iters;
    r->tol = tol;
    r->damping = damping;
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        ++s->submitted;
        if (s->stop) {
            set_error("server is shutting down");
            return FASTLBP_E_STATE;
        }
        if (graph_manager(g) && graph_manager(g) != s) {
            set_error("graph is managed by another server");
            return FASTLBP_E_STATE;
        }
        graph_set_manager(g, s);
        s->managed.insert(g);
        r->ticket = s->next_ticket++;
        s->by_ticket[r->ticket] = r;
        s->pending.push_back(r);
    }
    s->cv_work.notify_one();
    *ticket = r->ticket;
    return FASTLBP_OK;
}

static int collect(fastlbp_server_t s, std::shared_ptr<Request> r, double *p1, fastlbp_run_stats *st,
                   double *latency_ms) {
    s->by_ticket.erase(r->ticket);
    if (r->status < 0) {
        set_error(r->error);
        return r->status;
    }
    if (p1 && !r->p1.empty()) std::memcpy(p1, r->p1.data(), sizeof(double) * r->p1.size());
    if (st) *st = r->stats;
    if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
    return FASTLBP_OK;
}

int fastlbp_server_poll(fastlbp_server_t s, uint64_t ticket, double *p1, fastlbp_run_stats *st, double *latency_ms) {
    clear_error();
    if (!s) {
        set_error("server is NULL");
        return FASTLBP_E_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->by_ticket.find(ticket);
    if (it == s->by_ticket.end()) {
        set_error("unknown ticket");
        return FASTLBP_E_INVALID_ARG;
    }
    if (it->second->status == 1) return 1;
    return collect(s, it->second, p1, st, latency_ms);
}

int fastlbp_server_wait(fastlbp_server_t s, uint64_t ticket, double *p1, fastlbp_run_stats *st, double *latency_ms) {
    clear_error();
    if (!s) {
        set_error("server is NULL");
        return FASTLBP_E_INVALID_ARG;
    }
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->by_ticket.find(ticket);
    if (it == s->by_ticket.end()) {
        set_error("unknown ticket");
        return FASTLBP_E_INVALID_ARG;
    }
    auto r = it->second;
    s->cv_done.wait(lk, [&] { return r->status != 1; });
    return collect(s, r, p1, st, latency_ms);
}

int fastlbp_server_get_stats(fastlbp_server_t s, fastlbp_server_stats *out) {
    clear_error();
    if (!s || !out) {
        set_error("invalid argument");
        return FASTLBP_E_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(out, 0, sizeof(*out));
    out->completed = s->completed;
    out->message_updates = s->updates;
    out->steps = s->steps;
    out->busy_ms = s->busy_ms;
    out->kernel_ms = s->kernel_ms;
    out->method_bytes = s->method_bytes;
    out->evictions = s->evictions;
    out->restores = s->restores;
    out->resident_bytes = s->resident_bytes();
    out->peak_resident_bytes = s->peak_resident;
    out->persistent_launches = s->persistent_launches;
    out->persistent_ms = s->persistent_ms;
    out->persistent_method_bytes = s->persistent_bytes;
    out->pending = int32_t(s->pending.size());
    out->active = int32_t(s->active.size());
    if (!s->lat_ms.empty()) {
        std::vector<double> v = s->lat_ms;
        std::sort(v.begin(), v.end());
        auto pct = [&](double q) {
            size_t k = size_t(q * double(v.size() - 1) + 0.5);
            return v[std::min(k, v.size() - 1)];
        };
        out->p50_ms = pct(0.50);
        out->p99_ms = pct(0.99);
    }
    return FASTLBP_OK;
}

void fastlbp_server_destroy(fastlbp_server_t s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (auto &r : s->pending) {
            r->status = FASTLBP_E_STATE;
            r->error = "server destroyed before the request ran";
        }
        s->pending.clear();
    }
    s->cv_work.notify_all();
    if (s->th.joinable()) s->th.join();
    s->cv_done.notify_all();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (auto *g : s->managed) graph_set_manager(g, nullptr);
        s->managed.clear();
    }
    launcher_destroy(s->launcher);
    delete s;
}

}  // extern "C"
