// Autotuner of the launch choices of a graph handle: executor, degree-bucket cut-offs (which
// factors run one per thread, per wavefront or per workgroup, which variables one per thread or per
// wavefront), iterations per hipGraph replay and the persistent executor's workgroup size.
//
// The small graphs of the evaluation (Section 5.2) lack parallelism and the large ones are bound by
// memory, so no one setting suits every shape: fastlbp_autotune times a few candidates on the
// handle's own graph and schedule (a few iterations each, from the handle's current messages, which
// are restored afterwards) and keeps the fastest. The choice is cached in a text file under a key
// of the graph's shape (sizes, degree histogram, level widths per bucket), so a later handle of the
// same shape takes it without timing: given the cache, the result is deterministic.
//
// Cache file: one line per key, "<key hex> <executor> <thread max> <wave max> <var thread max>
// <graph iters> <persistent threads> <best ms/iter> <default ms/iter>"; a later line for a key
// replaces an earlier one; malformed lines are skipped.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "exec.h"

namespace fastlbp {

namespace {

struct Cand {
    int exec;
    PlanParams pp;
    int graph_iters;
    int threads;
};

uint64_t fnv(uint64_t h, uint64_t x) {
    for (int i = 0; i < 8; ++i) {
        h ^= (x >> (8 * i)) & 0xff;
        h *= 1099511628211ull;
    }
    return h;
}

// Shape key: precision, sizes, schedule kind and depth, the degree histogram of the factors (per
// type, log2 bins) and of the variables, and the width of every executed level per default bucket.
uint64_t shape_key(const fastlbp_graph *g) {
    const HostGraph &hg = g->hg();
    const HostPlan &hp = g->P->hp;
    uint64_t h = 1469598103934665603ull;
    h = fnv(h, uint64_t(g->precision()));
    h = fnv(h, uint64_t(hg.V));
    h = fnv(h, uint64_t(hg.F));
    h = fnv(h, uint64_t(hg.E));
    h = fnv(h, uint64_t(g->P->kind));
    h = fnv(h, uint64_t(hp.exec_levels));
    std::vector<uint64_t> hist(7 * 32, 0), vhist(32, 0);
    for (int32_t a = 0; a < hg.F; ++a) {
        const int64_t d = hg.fac_off[a + 1] - hg.fac_off[a];
        int b = 0;
        while ((int64_t(1) << b) < d && b < 31) ++b;
        hist[size_t(hg.fac_type[a]) * 32 + size_t(b)]++;
    }
    for (int32_t v = 0; v < hg.V; ++v) {
        int b = 0;
        while ((1 << b) < hg.var_deg[v] && b < 31) ++b;
        vhist[size_t(b)]++;
    }
    for (uint64_t x : hist) h = fnv(h, x);
    for (uint64_t x : vhist) h = fnv(h, x);
    for (int32_t L = 0; L < hp.exec_levels; ++L) {
        for (int b = 0; b < FB_COUNT; ++b) h = fnv(h, uint64_t(hp.fac_lvl_off[b][L + 1] - hp.fac_lvl_off[b][L]));
        for (int b = 0; b < VB_COUNT; ++b) h = fnv(h, uint64_t(hp.var_lvl_off[b][L + 1] - hp.var_lvl_off[b][L]));
    }
    return h;
}

bool cache_read(const std::string &path, uint64_t key, fastlbp_tune_result &r) {
    std::ifstream in(path);
    if (!in) return false;
    std::string line;
    bool found = false;
    while (std::getline(in, line)) {
        std::istringstream ss(line);
        std::string khex;
        fastlbp_tune_result t{};
        if (!(ss >> khex >> t.executor >> t.thread_max_degree >> t.wave_max_degree >> t.var_thread_max_degree >>
              t.graph_iters >> t.persistent_threads >> t.best_ms_per_iter >> t.default_ms_per_iter))
            continue;
        char *end = nullptr;
        const unsigned long long k = std::strtoull(khex.c_str(), &end, 16);
        if (!end || *end != '\0' || k != key) continue;
        PlanParams pp;
        pp.thread_max_deg = t.thread_max_degree;
        pp.wave_max_deg = t.wave_max_degree;
        pp.var_thread_max_deg = t.var_thread_max_degree;
        if (!pp.valid() || t.executor < FASTLBP_EXEC_LEVELS || t.executor > FASTLBP_EXEC_HYBRID ||
            t.graph_iters < 0 || t.graph_iters > 1024 ||
            (t.persistent_threads != 0 && t.persistent_threads != 512 && t.persistent_threads != 1024))
            continue;
        t.key = key;
        t.from_cache = 1;
        t.candidates = 0;
        r = t;
        found = true;  // keep reading: the last line for a key wins
    }
    return found;
}

bool cache_append(const std::string &path, const fastlbp_tune_result &r) {
    FILE *f = std::fopen(path.c_str(), "a");
    if (!f) return false;
    std::fprintf(f, "%016llx %d %d %d %d %d %d %.6f %.6f\n", (unsigned long long)r.key, r.executor,
                 r.thread_max_degree, r.wave_max_degree, r.var_thread_max_degree, r.graph_iters,
                 r.persistent_threads, r.best_ms_per_iter, r.default_ms_per_iter);
    std::fclose(f);
    return true;
}

std::string cache_path_of(const char *p) {
    if (p && *p) return p;
    const char *e = std::getenv("FASTLBP_AUTOTUNE_CACHE");
    return e ? std::string(e) : std::string();
}

int default_exec(const fastlbp_graph *g) {
    // what choose_executor picks with the executor option left on AUTO
    fastlbp_graph *m = const_cast<fastlbp_graph *>(g);
    const int saved = m->opts.executor;
    m->opts.executor = FASTLBP_EXEC_AUTO;
    const int e = choose_executor(m);
    m->opts.executor = saved;
    return e;
}

// Puts the handle on candidate c (plan for its cut-offs, executor and launch sizes).
void apply(fastlbp_graph *g, const Cand &c, std::shared_ptr<Plan> plan) {
    g->drop_graph();
    g->P = std::move(plan);
    g->pparams = c.pp;
    g->opts.executor = c.exec;
    g->tune_graph_iters = c.graph_iters;
    g->tune_threads = c.threads;
    g->tuned = true;
}

}  // namespace

}  // namespace fastlbp

using namespace fastlbp;

extern "C" {

int fastlbp_autotune_cache_get(const char *cache_path, uint64_t key, fastlbp_tune_result *out) {
    clear_error();
    if (!out) {
        set_error("out is NULL");
        return FASTLBP_E_INVALID_ARG;
    }
    const std::string path = cache_path_of(cache_path);
    if (path.empty()) {
        set_error("no cache path (argument or FASTLBP_AUTOTUNE_CACHE)");
        return FASTLBP_E_INVALID_ARG;
    }
    fastlbp_tune_result r{};
    if (!cache_read(path, key, r)) return 1;
    *out = r;
    return FASTLBP_OK;
}

int fastlbp_autotune_cache_put(const char *cache_path, const fastlbp_tune_result *r) {
    clear_error();
    if (!r) {
        set_error("result is NULL");
        return FASTLBP_E_INVALID_ARG;
    }
    const std::string path = cache_path_of(cache_path);
    if (path.empty()) {
        set_error("no cache path (argument or FASTLBP_AUTOTUNE_CACHE)");
        return FASTLBP_E_INVALID_ARG;
    }
    PlanParams pp;
    pp.thread_max_deg = r->thread_max_degree;
    pp.wave_max_deg = r->wave_max_degree;
    pp.var_thread_max_deg = r->var_thread_max_degree;
    if (!pp.valid() || r->executor < FASTLBP_EXEC_LEVELS || r->executor > FASTLBP_EXEC_HYBRID) {
        set_error("invalid tuning result");
        return FASTLBP_E_INVALID_ARG;
    }
    if (!cache_append(path, *r)) {
        set_error("cannot write " + path);
        return FASTLBP_E_INVALID_ARG;
    }
    return FASTLBP_OK;
}

int fastlbp_autotune(fastlbp_graph_t g, int32_t probe_iters, double damping, const char *cache_path,
                     fastlbp_tune_result *out) {
    clear_error();
    if (!g || probe_iters < 1 || !(damping >= 0.0 && damping < 1.0)) {
        set_error("need a graph, probe_iters >= 1 and 0 <= damping < 1");
        return FASTLBP_E_INVALID_ARG;
    }
    std::lock_guard<std::recursive_mutex> lk(g->mu);
    const std::string path = cache_path_of(cache_path);
    // the key of the default plan's shape
    std::shared_ptr<Plan> orig = g->P;
    const Cand orig_c = {g->opts.executor, g->pparams, g->tune_graph_iters, g->tune_threads};
    const bool was_tuned = g->tuned;
    void *saved = nullptr;
    size_t saved_bytes = 0;
    // on failure: the handle's messages and launch choices as they were
    auto undo = [&]() {
        if (saved) {
            (void)hipMemcpyAsync(g->msg, saved, saved_bytes, hipMemcpyDeviceToDevice, g->L.stream);
            (void)hipStreamSynchronize(g->L.stream);
            g->alloc.put(saved);
            saved = nullptr;
        }
        apply(g, orig_c, orig);
        g->tuned = was_tuned;
    };
    try {
        HIPCHK(hipSetDevice(g->opts.device));
        graph_restore(g);
        std::shared_ptr<Plan> base = orig;
        const PlanParams defaults;
        const std::vector<int32_t> &level = orig->hp.level_of_edge;
        const int32_t nlev = orig->hp.num_levels;
        if (g->pparams.thread_max_deg != defaults.thread_max_deg || g->pparams.wave_max_deg != defaults.wave_max_deg ||
            g->pparams.var_thread_max_deg != defaults.var_thread_max_deg)
            base = plan_from_levels(*g->S, g->alloc, g->L.stream, orig->kind, level, nlev, defaults);
        apply(g, Cand{orig_c.exec, defaults, 0, 0}, base);
        fastlbp_tune_result res{};
        res.key = shape_key(g);
        if (!path.empty() && cache_read(path, res.key, res)) {
            PlanParams pp;
            pp.thread_max_deg = res.thread_max_degree;
            pp.wave_max_deg = res.wave_max_degree;
            pp.var_thread_max_deg = res.var_thread_max_degree;
            std::shared_ptr<Plan> plan = base;
            if (pp.thread_max_deg != defaults.thread_max_deg || pp.wave_max_deg != defaults.wave_max_deg ||
                pp.var_thread_max_deg != defaults.var_thread_max_deg)
                plan = plan_from_levels(*g->S, g->alloc, g->L.stream, orig->kind, level, nlev, pp);
            apply(g, Cand{res.executor, pp, res.graph_iters, res.persistent_threads}, plan);
            if (out) *out = res;
            return FASTLBP_OK;
        }
        // candidates
        const int dex = default_exec(g);
        const bool f32 = g->precision() == FASTLBP_FP32;
        std::vector<int> execs = {FASTLBP_EXEC_LEVELS};
        if (base->hp.fused_levels > 0) execs.push_back(FASTLBP_EXEC_HYBRID);
        if (g->hg().nonprior_edges <= (int64_t(4) << 20) && base->hp.max_level_edges <= 65536)
            execs.push_back(FASTLBP_EXEC_PERSISTENT);
        std::vector<PlanParams> pps(1, defaults);
        {
            PlanParams p = defaults;
            p.thread_max_deg = 4;
            pps.push_back(p);
            p = defaults;
            p.wave_max_deg = 65;
            pps.push_back(p);
            p = defaults;
            p.var_thread_max_deg = 16;
            pps.push_back(p);
        }
        std::vector<Cand> cands;
        cands.push_back(Cand{dex, defaults, 0, 0});  // the default first: its time is the reference
        for (int e : execs)
            for (const PlanParams &pp : pps) {
                if (e == FASTLBP_EXEC_PERSISTENT) {
                    cands.push_back(Cand{e, pp, 0, 512});
                    if (f32) cands.push_back(Cand{e, pp, 0, 1024});
                } else {
                    cands.push_back(Cand{e, pp, 0, 0});
                    cands.push_back(Cand{e, pp, 4, 0});
                }
            }
        // the handle's messages are restored before every probe and at the end
        const size_t mb = g->S->msg_bytes() * std::max<int64_t>(g->hg().E, 1);
        saved = g->alloc.get(mb);
        if (!saved) throw OomError{};
        saved_bytes = mb;
        HIPCHK(hipMemcpyAsync(saved, g->msg, mb, hipMemcpyDeviceToDevice, g->L.stream));
        HIPCHK(hipStreamSynchronize(g->L.stream));
        std::vector<std::shared_ptr<Plan>> plans(pps.size());
        plans[0] = base;
        auto plan_of = [&](const PlanParams &pp) {
            for (size_t i = 0; i < pps.size(); ++i)
                if (pps[i].thread_max_deg == pp.thread_max_deg && pps[i].wave_max_deg == pp.wave_max_deg &&
                    pps[i].var_thread_max_deg == pp.var_thread_max_deg) {
                    if (!plans[i])
                        plans[i] = plan_from_levels(*g->S, g->alloc, g->L.stream, orig->kind, level, nlev, pp);
                    return plans[i];
                }
            return base;
        };
        double best = 1e300;
        Cand best_c = cands[0];
        int timed = 0;
        for (size_t ci = 0; ci < cands.size(); ++ci) {
            const Cand &c = cands[ci];
            if (ci > 0 && c.exec == cands[0].exec && c.pp.thread_max_deg == defaults.thread_max_deg &&
                c.pp.wave_max_deg == defaults.wave_max_deg && c.pp.var_thread_max_deg == defaults.var_thread_max_deg &&
                c.graph_iters == 0 && c.threads == 0)
                continue;  // the default again
            apply(g, c, plan_of(c.pp));
            float ms = 0.f;
            for (int rep = 0; rep < 2; ++rep) {  // the first run warms up (plans, captured graphs)
                HIPCHK(hipMemcpyAsync(g->msg, saved, mb, hipMemcpyDeviceToDevice, g->L.stream));
                HIPCHK(hipEventRecord(g->L.ev0, g->L.stream));
                run_any(g, probe_iters, 0.0, damping, c.exec);
                HIPCHK(hipEventRecord(g->L.ev1, g->L.stream));
                HIPCHK(hipStreamSynchronize(g->L.stream));
                HIPCHK(hipEventElapsedTime(&ms, g->L.ev0, g->L.ev1));
            }
            ++timed;
            const double per = double(ms) / probe_iters;
            if (ci == 0) res.default_ms_per_iter = per;
            if (per < best) {
                best = per;
                best_c = c;
            }
        }
        apply(g, best_c, plan_of(best_c.pp));
        HIPCHK(hipMemcpyAsync(g->msg, saved, mb, hipMemcpyDeviceToDevice, g->L.stream));
        HIPCHK(hipStreamSynchronize(g->L.stream));
        g->alloc.put(saved);
        saved = nullptr;
        res.executor = best_c.exec;
        res.thread_max_degree = best_c.pp.thread_max_deg;
        res.wave_max_degree = best_c.pp.wave_max_deg;
        res.var_thread_max_degree = best_c.pp.var_thread_max_deg;
        res.graph_iters = best_c.graph_iters;
        res.persistent_threads = best_c.threads;
        res.candidates = timed;
        res.from_cache = 0;
        res.best_ms_per_iter = best;
        if (!path.empty() && !cache_append(path, res)) {
            set_error("cannot write " + path);
            if (out) *out = res;
            return FASTLBP_E_INVALID_ARG;
        }
        if (out) *out = res;
    } catch (OomError &) {
        undo();
        set_error("device allocation failed");
        return FASTLBP_E_OOM;
    } catch (DeviceError &e) {
        undo();
        set_error(e.msg);
        return FASTLBP_E_DEVICE;
    }
    return FASTLBP_OK;
}

}  // extern "C"
