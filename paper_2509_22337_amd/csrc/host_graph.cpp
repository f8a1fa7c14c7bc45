// Host-side graph preparation (the Initialization and Dependency Analysis stages of Section 4.1).
#include <algorithm>
#include <array>
#include <functional>
#include <queue>
#include <cmath>
#include <cstring>
#include <numeric>

#include "fastlbp.h"
#include "host.h"

namespace fastlbp {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

}  // namespace fastlbp

extern "C" const char *fastlbp_last_error(void) { return fastlbp::g_last_error.c_str(); }

namespace fastlbp {

static bool bad_prob(double p) { return !(p >= 0.0 && p <= 1.0); }

int validate_graph(int32_t V, int32_t F, const int64_t *off, const int32_t *ev, const uint8_t *ft, const double *fp,
                   const double *ep, const int64_t *toff, const double *tw, const int8_t *tind) {
    if (V < 0 || F < 0) {
        set_error("negative size");
        return FASTLBP_E_INVALID_ARG;
    }
    if (!off || (F > 0 && !ft)) {
        set_error("factor_offsets and factor_types are required");
        return FASTLBP_E_INVALID_ARG;
    }
    if (off[0] != 0) {
        set_error("factor_offsets[0] must be 0");
        return FASTLBP_E_BAD_GRAPH;
    }
    for (int32_t a = 0; a < F; ++a)
        if (off[a + 1] < off[a]) {
            set_error("factor_offsets must be non-decreasing (factor " + std::to_string(a) + ")");
            return FASTLBP_E_BAD_GRAPH;
        }
    int64_t E = off[F];
    if (E >= (int64_t(1) << 31)) {
        set_error("more than 2^31-1 edges");
        return FASTLBP_E_TOO_LARGE;
    }
    if (E > 0 && !ev) {
        set_error("edge_vars is required");
        return FASTLBP_E_INVALID_ARG;
    }
    for (int64_t e = 0; e < E; ++e)
        if (ev[e] < 0 || ev[e] >= V) {
            set_error("edge " + std::to_string(e) + " has variable id out of range");
            return FASTLBP_E_BAD_GRAPH;
        }
    std::vector<int32_t> seen(V > 0 ? V : 1, -1);
    for (int32_t a = 0; a < F; ++a) {
        int64_t d = off[a + 1] - off[a];
        int t = ft[a];
        std::string where = " (factor " + std::to_string(a) + ")";
        if (t > FASTLBP_TERMS) {
            set_error("unknown factor type" + where);
            return FASTLBP_E_BAD_GRAPH;
        }
        const int64_t nt = toff ? toff[a + 1] - toff[a] : 0;
        if (t == FASTLBP_TERMS) {
            if (!toff) {
                set_error("TERMS factors need term data (fastlbp_graph_create_terms)" + where);
                return FASTLBP_E_BAD_GRAPH;
            }
            if (d < 1 || nt < 1) {
                set_error("TERMS needs degree >= 1 and at least one term" + where);
                return FASTLBP_E_BAD_GRAPH;
            }
            if (d > FASTLBP_MAX_TERM_DEGREE || nt > FASTLBP_MAX_TERMS) {
                set_error("TERMS factor above FASTLBP_MAX_TERM_DEGREE or FASTLBP_MAX_TERMS" + where);
                return FASTLBP_E_TOO_LARGE;
            }
        } else if (nt != 0) {
            set_error("only TERMS factors take terms" + where);
            return FASTLBP_E_BAD_GRAPH;
        }
        if (t == FASTLBP_PRIOR && d != 1) {
            set_error("PRIOR needs degree 1" + where);
            return FASTLBP_E_BAD_GRAPH;
        }
        if (t == FASTLBP_NOT && d != 2) {
            set_error("NOT needs degree 2" + where);
            return FASTLBP_E_BAD_GRAPH;
        }
        if (t != FASTLBP_PRIOR && t != FASTLBP_NOT && t != FASTLBP_TERMS && d < 2) {
            set_error("AND/OR/IMPLIES/NOISY_OR need degree >= 2" + where);
            return FASTLBP_E_BAD_GRAPH;
        }
        if (d > FASTLBP_MAX_DEGREE) {
            set_error("factor degree above FASTLBP_MAX_DEGREE" + where);
            return FASTLBP_E_TOO_LARGE;
        }
        for (int64_t e = off[a]; e < off[a + 1]; ++e) {
            if (seen[ev[e]] == a) {
                set_error("variable " + std::to_string(ev[e]) + " appears twice" + where);
                return FASTLBP_E_BAD_GRAPH;
            }
            seen[ev[e]] = a;
        }
        if (fp) {
            double p = fp[a];
            if ((t == FASTLBP_PRIOR || t == FASTLBP_IMPLIES) && bad_prob(p)) {
                set_error("parameter outside [0,1]" + where);
                return FASTLBP_E_BAD_GRAPH;
            }
            if (t == FASTLBP_NOISY_OR && !(p >= 0.0 && p < 1.0)) {
                set_error("noisy-or leak outside [0,1)" + where);
                return FASTLBP_E_BAD_GRAPH;
            }
        }
        if (ep && t == FASTLBP_NOISY_OR)
            for (int64_t e = off[a]; e + 1 < off[a + 1]; ++e)
                if (bad_prob(ep[e])) {
                    set_error("noisy-or activation outside [0,1]" + where);
                    return FASTLBP_E_BAD_GRAPH;
                }
    }
    if (toff) {
        if (toff[0] != 0) {
            set_error("term_offsets[0] must be 0");
            return FASTLBP_E_BAD_GRAPH;
        }
        for (int32_t a = 0; a < F; ++a)
            if (toff[a + 1] < toff[a]) {
                set_error("term_offsets must be non-decreasing");
                return FASTLBP_E_BAD_GRAPH;
            }
        const int64_t T = toff[F];
        if (T > 0 && (!tw || !tind)) {
            set_error("term_weights and term_indicators are required");
            return FASTLBP_E_INVALID_ARG;
        }
        for (int64_t t = 0; t < T; ++t)
            if (!(tw[t] >= 0.0 && tw[t] < __builtin_inf())) {
                set_error("term weight " + std::to_string(t) + " not finite and >= 0");
                return FASTLBP_E_BAD_GRAPH;
            }
        int64_t k = 0;
        for (int32_t a = 0; a < F; ++a)
            for (int64_t q = 0; q < (toff[a + 1] - toff[a]) * (off[a + 1] - off[a]); ++q, ++k)
                if (tind[k] < -1 || tind[k] > 1) {
                    set_error("term indicator outside {-1, 0, 1} (factor " + std::to_string(a) + ")");
                    return FASTLBP_E_BAD_GRAPH;
                }
    }
    return FASTLBP_OK;
}

// Class-atomic Algorithm 2. Edges are visited in (rank, edge id) order, one rank class at a time.
// A class joins the current level unless one of its edges e = (a, v) has a neighbour of
// Definition 1 in the level: an edge (a*, v*) with v* adjacent to a, v* != v and a* != a. Such a
// neighbour precedes e strictly (it belongs to an earlier class), so the class opens a new level.
// Per variable we remember whether the current level holds an edge at it and from which factor
// (or "several"), which makes the test O(degree of a) per factor touched by the class.
int32_t analyze_levels(int32_t V, int32_t F, const int64_t *off, const int32_t *ev, const int32_t *rank,
                       std::vector<int32_t> &level) {
    int64_t E = off[F];
    level.assign(E, 0);
    if (E == 0) return 0;
    if (!rank) return 1;
    std::vector<int32_t> edge_fac(E);
    for (int32_t a = 0; a < F; ++a)
        for (int64_t e = off[a]; e < off[a + 1]; ++e) edge_fac[e] = a;
    std::vector<int32_t> order(E);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return rank[x] < rank[y]; });
    std::vector<int32_t> mark_level(V, -1), mark_fac(V, -1);
    int32_t cur = 0;
    bool first = true;
    int64_t i = 0;
    while (i < E) {
        int64_t j = i;
        while (j < E && rank[order[j]] == rank[order[i]]) ++j;
        bool cut = false;
        if (!first) {
            // factors of the class are contiguous runs because ids ascend inside a class
            int64_t k = i;
            while (k < j && !cut) {
                int32_t a = edge_fac[order[k]];
                int64_t k2 = k;
                while (k2 < j && edge_fac[order[k2]] == a) ++k2;
                int32_t only_v = (k2 - k == 1) ? ev[order[k]] : -1;
                for (int64_t q = off[a]; q < off[a + 1]; ++q) {
                    int32_t vs = ev[q];
                    if (vs == only_v) continue;
                    if (mark_level[vs] == cur && mark_fac[vs] != a) {
                        cut = true;
                        break;
                    }
                }
                k = k2;
            }
        }
        if (cut) ++cur;
        first = false;
        for (int64_t k = i; k < j; ++k) {
            int32_t e = order[k];
            int32_t v = ev[e], a = edge_fac[e];
            level[e] = cur;
            if (mark_level[v] != cur) {
                mark_level[v] = cur;
                mark_fac[v] = a;
            } else if (mark_fac[v] != a) {
                mark_fac[v] = -2;
            }
        }
        i = j;
    }
    return cur + 1;
}

void HostGraph::build(int32_t V_, int32_t F_, const int64_t *off, const int32_t *ev, const uint8_t *ft,
                      const double *fp, const double *ep) {
    V = V_;
    F = F_;
    E = off[F];
    fac_off.assign(off, off + F + 1);
    edge_var.assign(ev, ev + E);
    fac_type.assign(ft, ft + F);
    fac_param.resize(F);
    edge_param.assign(E, 0.0);
    edge_fac.resize(E);
    max_deg = 0;
    for (int32_t a = 0; a < F; ++a) {
        int t = ft[a];
        double def = (t == FASTLBP_PRIOR) ? 0.5 : (t == FASTLBP_IMPLIES ? 1.0 : 0.0);
        fac_param[a] = fp ? fp[a] : def;
        for (int64_t e = off[a]; e < off[a + 1]; ++e) {
            edge_fac[e] = a;
            if (t == FASTLBP_NOISY_OR && e + 1 < off[a + 1]) edge_param[e] = ep ? ep[e] : 1.0;
        }
        if (t != FASTLBP_PRIOR) max_deg = std::max<int32_t>(max_deg, int32_t(off[a + 1] - off[a]));
    }
    // variable-major transpose of the non-PRIOR edges (stable: ascending edge id per variable)
    var_off.assign(V + 1, 0);
    nonprior_edges = 0;
    for (int64_t e = 0; e < E; ++e)
        if (fac_type[edge_fac[e]] != FASTLBP_PRIOR) {
            var_off[ev[e] + 1]++;
            ++nonprior_edges;
        }
    for (int32_t v = 0; v < V; ++v) var_off[v + 1] += var_off[v];
    var_edge.resize(nonprior_edges);
    std::vector<int32_t> fill(var_off.begin(), var_off.end() - 1);
    for (int64_t e = 0; e < E; ++e)
        if (fac_type[edge_fac[e]] != FASTLBP_PRIOR) var_edge[fill[ev[e]]++] = int32_t(e);
    var_deg.resize(V);
    for (int32_t v = 0; v < V; ++v) var_deg[v] = var_off[v + 1] - var_off[v];
    // PRIOR folding: LLR in bits, p = 1 and p = 0 become infinite terms
    prior_fin.assign(V, 0.0);
    prior_pos.assign(V, 0);
    prior_neg.assign(V, 0);
    for (int32_t a = 0; a < F; ++a)
        if (fac_type[a] == FASTLBP_PRIOR) {
            int32_t v = ev[off[a]];
            double p = fac_param[a];
            if (p >= 1.0)
                prior_pos[v]++;
            else if (p <= 0.0)
                prior_neg[v]++;
            else
                prior_fin[v] += std::log2(p) - std::log2(1.0 - p);
        }
}

// A general preorder as classes and strict arcs between them (Definition 2): checks that the arcs
// form a DAG and that every edge is comparable with every edge of its N_E (Definition 1) that is
// not a PRIOR edge, then ranks the classes by a deterministic topological order (Kahn's algorithm,
// smallest class first). Returns 0 or an error code (message set).
int classes_to_ranks(int32_t V, int32_t F, const int64_t *off, const int32_t *ev, const uint8_t *ft, int32_t C,
                     const int32_t *edge_class, int32_t A, const int32_t *arcs, std::vector<int32_t> &rank) {
    const int64_t E = off[F];
    if (C < 1 || C > kMaxClasses || A < 0 || (E > 0 && !edge_class) || (A > 0 && !arcs)) {
        set_error("need 1 <= num_classes <= " + std::to_string(kMaxClasses) + " and the class and arc arrays");
        return C > kMaxClasses ? FASTLBP_E_TOO_LARGE : FASTLBP_E_INVALID_ARG;
    }
    for (int64_t e = 0; e < E; ++e)
        if (edge_class[e] < 0 || edge_class[e] >= C) {
            set_error("edge " + std::to_string(e) + " has a class out of range");
            return FASTLBP_E_INVALID_ARG;
        }
    std::vector<std::vector<int32_t>> succ(C);
    std::vector<int32_t> indeg(C, 0);
    for (int32_t i = 0; i < A; ++i) {
        const int32_t x = arcs[2 * i], y = arcs[2 * i + 1];
        if (x < 0 || x >= C || y < 0 || y >= C) {
            set_error("arc " + std::to_string(i) + " names a class out of range");
            return FASTLBP_E_INVALID_ARG;
        }
        if (x == y) {
            set_error("arc " + std::to_string(i) + " puts a class strictly before itself");
            return FASTLBP_E_BAD_SCHEDULE;
        }
        succ[x].push_back(y);
        indeg[y]++;
    }
    // topological order, smallest available class first
    std::vector<int32_t> order, pos(C, -1);
    order.reserve(C);
    std::priority_queue<int32_t, std::vector<int32_t>, std::greater<int32_t>> ready;
    for (int32_t c = 0; c < C; ++c)
        if (indeg[c] == 0) ready.push(c);
    while (!ready.empty()) {
        const int32_t c = ready.top();
        ready.pop();
        pos[c] = int32_t(order.size());
        order.push_back(c);
        for (int32_t y : succ[c])
            if (--indeg[y] == 0) ready.push(y);
    }
    if (int32_t(order.size()) != C) {
        set_error("the class arcs contain a cycle");
        return FASTLBP_E_BAD_SCHEDULE;
    }
    // reachability (class x strictly before class y), in reverse topological order
    const size_t W = (size_t(C) + 63) / 64;
    std::vector<uint64_t> reach(size_t(C) * W, 0);
    for (int32_t i = C - 1; i >= 0; --i) {
        const int32_t c = order[i];
        uint64_t *rc = &reach[size_t(c) * W];
        for (int32_t y : succ[c]) {
            rc[y >> 6] |= uint64_t(1) << (y & 63);
            const uint64_t *ry = &reach[size_t(y) * W];
            for (size_t k = 0; k < W; ++k) rc[k] |= ry[k];
        }
    }
    auto before = [&](int32_t x, int32_t y) { return (reach[size_t(x) * W + (y >> 6)] >> (y & 63)) & 1; };
    auto comparable = [&](int32_t x, int32_t y) { return x == y || before(x, y) || before(y, x); };
    // Definition 2: e1 = (a, v), e2 = (a2, u) with u in N(a) \ v and a2 in N(u) \ a. Per variable u,
    // the distinct classes of its non-PRIOR edges; per factor, those of its other edges.
    std::vector<int32_t> edge_fac(E);
    for (int32_t a = 0; a < F; ++a)
        for (int64_t e = off[a]; e < off[a + 1]; ++e) edge_fac[e] = a;
    auto is_prior = [&](int64_t e) { return ft && ft[edge_fac[e]] == FASTLBP_PRIOR; };
    std::vector<int32_t> voff(size_t(V) + 1, 0), vedge(E);
    for (int64_t e = 0; e < E; ++e) voff[ev[e] + 1]++;
    for (int32_t v = 0; v < V; ++v) voff[v + 1] += voff[v];
    {
        std::vector<int32_t> fill(voff.begin(), voff.end() - 1);
        for (int64_t e = 0; e < E; ++e) vedge[fill[ev[e]]++] = int32_t(e);
    }
    // distinct classes (with counts) of each variable's non-PRIOR edges
    std::vector<int32_t> vcls_off(size_t(V) + 1, 0), vcls, vcnt;
    {
        std::vector<int32_t> tmp;
        for (int32_t v = 0; v < V; ++v) {
            tmp.clear();
            for (int32_t q = voff[v]; q < voff[v + 1]; ++q)
                if (!is_prior(vedge[q])) tmp.push_back(edge_class[vedge[q]]);
            std::sort(tmp.begin(), tmp.end());
            for (size_t i = 0; i < tmp.size();) {
                size_t j = i;
                while (j < tmp.size() && tmp[j] == tmp[i]) ++j;
                vcls.push_back(tmp[i]);
                vcnt.push_back(int32_t(j - i));
                i = j;
            }
            vcls_off[v + 1] = int32_t(vcls.size());
        }
    }
    std::vector<int32_t> fcls, fcnt;
    std::vector<uint8_t> checked;
    for (int32_t a = 0; a < F; ++a) {
        if (ft && ft[a] == FASTLBP_PRIOR) continue;
        // distinct classes of a's edges, with counts
        fcls.clear();
        fcnt.clear();
        {
            std::vector<int32_t> tmp(edge_class + off[a], edge_class + off[a + 1]);
            std::sort(tmp.begin(), tmp.end());
            for (size_t i = 0; i < tmp.size();) {
                size_t j = i;
                while (j < tmp.size() && tmp[j] == tmp[i]) ++j;
                fcls.push_back(tmp[i]);
                fcnt.push_back(int32_t(j - i));
                i = j;
            }
        }
        for (int64_t eu = off[a]; eu < off[a + 1]; ++eu) {
            const int32_t u = ev[eu], cu = edge_class[eu];
            // e1 ranges over a's edges other than (a, u): a's classes, less cu if only (a, u) has it;
            // e2 over u's non-PRIOR edges outside a: u's classes, less cu if only (a, u) has it
            for (size_t i = 0; i < fcls.size(); ++i) {
                const int32_t x = fcls[i];
                if (x == cu && fcnt[i] == 1) continue;
                for (int32_t q = vcls_off[u]; q < vcls_off[u + 1]; ++q) {
                    const int32_t y = vcls[q];
                    if (y == cu && vcnt[q] == 1) continue;
                    if (!comparable(x, y)) {
                        set_error("classes " + std::to_string(x) + " and " + std::to_string(y) +
                                  " are incomparable but hold dependent edges (Definition 2)");
                        return FASTLBP_E_BAD_SCHEDULE;
                    }
                }
            }
        }
    }
    rank.resize(E);
    for (int64_t e = 0; e < E; ++e) rank[e] = pos[edge_class[e]];
    return FASTLBP_OK;
}

void HostGraph::set_terms(const int64_t *toff, const double *tw, const int8_t *tind) {
    term_off.clear();
    term_weight.clear();
    term_ind.clear();
    term_base.clear();
    term_mask.clear();
    if (!toff || toff[F] == 0) return;
    term_off.resize(size_t(F) + 1);
    for (int32_t a = 0; a <= F; ++a) term_off[a] = int32_t(toff[a]);
    term_weight.assign(tw, tw + toff[F]);
    term_base.resize(size_t(F) + 1);
    int64_t n = 0;
    for (int32_t a = 0; a < F; ++a) {
        term_base[a] = int32_t(n);
        n += (toff[a + 1] - toff[a]) * (fac_off[a + 1] - fac_off[a]);
    }
    term_base[F] = int32_t(n);
    term_ind.assign(tind, tind + n);
    term_mask.assign(term_weight.size(), 0);
    for (int32_t a = 0; a < F; ++a) {
        const int64_t d = fac_off[a + 1] - fac_off[a];
        if (d > kThreadMaxDeg) continue;
        for (int32_t t = term_off[a]; t < term_off[a + 1]; ++t)
            for (int64_t k = 0; k < d; ++k) {
                const int8_t c = term_ind[term_base[a] + (t - term_off[a]) * d + k];
                if (c >= 0) term_mask[t] |= uint16_t((1u << k) | (unsigned(c) << (8 + k)));
            }
    }
}

namespace {

// Stable reordering of v by an integer key in [0, nkeys): a counting sort.
template <class K>
void counting_sort(std::vector<int32_t> &v, int64_t nkeys, K key, std::vector<int32_t> &tmp) {
    std::vector<int64_t> cnt(size_t(nkeys) + 1, 0);
    for (int32_t x : v) cnt[size_t(key(x)) + 1]++;
    for (int64_t k = 0; k < nkeys; ++k) cnt[size_t(k) + 1] += cnt[size_t(k)];
    tmp.resize(v.size());
    for (int32_t x : v) tmp[size_t(cnt[size_t(key(x))]++)] = x;
    v.swap(tmp);
}

}  // namespace

int factor_bucket(int deg, const PlanParams &pp) {
    if (deg <= pp.thread_max_deg) return FB_THREAD;
    if (deg <= pp.wave_max_deg) return FB_WAVE;
    return FB_BLOCK;
}

void HostPlan::build(const HostGraph &g, const std::vector<int32_t> &level, int32_t nlevels, bool flooding,
                     int msg_bytes, int param_bytes, const PlanParams &pp) {
    params = pp;
    num_levels = nlevels;
    level_of_edge = level;
    all_active = flooding ? 1 : 0;
    // executed levels: those holding at least one non-PRIOR edge
    std::vector<int32_t> exec_of(std::max(nlevels, 1), -1);
    std::vector<int64_t> level_np(std::max(nlevels, 1), 0);
    for (int64_t e = 0; e < g.E; ++e)
        if (g.fac_type[g.edge_fac[e]] != FASTLBP_PRIOR) level_np[level[e]]++;
    exec_levels = 0;
    max_level_edges = 0;
    for (int32_t L = 0; L < nlevels; ++L)
        if (level_np[L] > 0) {
            exec_of[L] = exec_levels++;
            max_level_edges = std::max<int32_t>(max_level_edges, int32_t(level_np[L]));
        }
    edge_exec_level.assign(g.E, -1);
    for (int64_t e = 0; e < g.E; ++e)
        if (g.fac_type[g.edge_fac[e]] != FASTLBP_PRIOR) edge_exec_level[e] = exec_of[level[e]];
    // factor tasks per executed level: a factor joins level L if one of its edges is active in L
    std::vector<std::vector<int32_t>> fac_by_level(FB_COUNT * std::max(exec_levels, 1));
    std::vector<std::vector<int32_t>> var_by_level(VB_COUNT * std::max(exec_levels, 1));
    bytes_per_iter = 0.0;
    updates_per_iter = 0;
    touched_edges_per_iter = noisy_params_per_iter = term_weights_per_iter = term_entries_per_iter = 0;
    std::vector<int32_t> lv;
    for (int32_t a = 0; a < g.F; ++a) {
        if (g.fac_type[a] == FASTLBP_PRIOR) continue;
        int64_t b = g.fac_off[a], d = g.fac_off[a + 1] - b;
        const bool terms = g.fac_type[a] == FASTLBP_TERMS;
        int bucket = terms ? (d <= kThreadMaxDeg ? FB_TERMS_THREAD : FB_TERMS_WAVE) : factor_bucket(int(d), pp);
        int32_t prev = -1;
        // levels of a factor's edges in ascending order of level, each level once
        lv.clear();
        for (int64_t e = b; e < b + d; ++e) lv.push_back(edge_exec_level[e]);
        std::sort(lv.begin(), lv.end());
        for (int32_t L : lv) {
            if (L == prev) continue;
            prev = L;
            fac_by_level[L * FB_COUNT + bucket].push_back(a);
            touched_edges_per_iter += d;
            if (g.fac_type[a] == FASTLBP_NOISY_OR) noisy_params_per_iter += d - 1;
            if (terms) {
                term_weights_per_iter += g.term_off[a + 1] - g.term_off[a];
                term_entries_per_iter += int64_t(g.term_off[a + 1] - g.term_off[a]) * d;
            }
            // bytes of a factor task: offsets, type, parameters, list entry; per edge: variable id,
            // belief, old message, (level tag unless flooding), NOISY_OR activation
            double per_edge = 4.0 + sizeof(Belief) + msg_bytes + (flooding ? 0 : 4) +
                              (g.fac_type[a] == FASTLBP_NOISY_OR ? param_bytes : 0);
            bytes_per_iter += 4 + 8 + 1 + param_bytes + per_edge * double(d);
            if (terms) {  // term range; per term its weight and indicators: a 16-bit mask pair
                          // (thread path) or indicator base plus one byte per edge (wavefront path)
                const double l = double(g.term_off[a + 1] - g.term_off[a]);
                bytes_per_iter += bucket == FB_TERMS_THREAD ? 8 + l * (param_bytes / 2 + 2)
                                                             : 8 + 4 + l * (param_bytes / 2 + double(d));
            }
        }
    }
    // variables whose incoming messages a level writes: their beliefs are refreshed after it. Built
    // from the variable-major rows, so every level's list comes out sorted and without repeats.
    for (int64_t e = 0; e < g.E; ++e)
        if (edge_exec_level[e] >= 0) {
            ++updates_per_iter;
            bytes_per_iter += msg_bytes;  // written message
        }
    for (int32_t v = 0; v < g.V; ++v) {
        lv.clear();
        for (int32_t q = g.var_off[v]; q < g.var_off[v + 1]; ++q) lv.push_back(edge_exec_level[g.var_edge[q]]);
        std::sort(lv.begin(), lv.end());
        const int vb = g.var_deg[v] <= pp.var_thread_max_deg ? VB_THREAD : VB_WAVE;
        for (size_t i = 0; i < lv.size(); ++i) {
            if (lv[i] < 0 || (i > 0 && lv[i] == lv[i - 1])) continue;
            var_by_level[size_t(lv[i]) * VB_COUNT + vb].push_back(v);
            // list entry, offsets, phi, belief write; per edge: edge id and message
            bytes_per_iter += 4 + 8 + 2 * sizeof(Belief) + double(g.var_deg[v]) * (4 + msg_bytes);
        }
    }
    auto fdeg = [&](int32_t a) { return int32_t(g.fac_off[a + 1] - g.fac_off[a]); };
    std::vector<int32_t> sort_tmp;
    for (int b = 0; b < FB_COUNT; ++b) {
        fac_list[b].clear();
        fac_lvl_off[b].assign(1, 0);
        for (int32_t L = 0; L < exec_levels; ++L) {
            auto &src = fac_by_level[L * FB_COUNT + b];
            // thread bucket: by degree, then type (a wavefront follows one code path), then factor
            // id, so neighbouring threads read neighbouring messages and, where the caller numbers
            // variables in factor order, neighbouring beliefs (ordering by first variable instead
            // costs the 19M-edge BINGO-shaped graph 11% per iteration). A narrow level (one
            // workgroup runs it) puts the highest degrees first: its time is that of its slowest
            // wavefront, the one holding the largest factors, and the lowest wavefronts of a
            // workgroup get their loads issued first (SmartFL-shaped graph: 5% per level). Wider
            // buckets: largest first, so the longest tasks start early
            // (lists are built in factor order, and the sorts below are stable)
            if (b == FB_THREAD) {
                const bool narrow = int64_t(src.size()) <= kFuseMaxRecs;
                counting_sort(src, int64_t(kThreadMaxDeg + 1) * 8, [&](int32_t x) {
                    return int64_t(narrow ? kThreadMaxDeg - fdeg(x) : fdeg(x)) * 8 + g.fac_type[x];
                }, sort_tmp);
            } else if (b == FB_TERMS_THREAD)  // by degree, then term count: a wavefront's loops agree
                std::sort(src.begin(), src.end(), [&](int32_t x, int32_t y) {
                    int dx = fdeg(x), dy = fdeg(y);
                    if (dx != dy) return dx < dy;
                    int lx = g.term_off[x + 1] - g.term_off[x], ly = g.term_off[y + 1] - g.term_off[y];
                    return lx != ly ? lx < ly : x < y;
                });
            else
                counting_sort(src, kBlockMaxDeg + 1, [&](int32_t x) { return int64_t(kBlockMaxDeg - std::min(fdeg(x), kBlockMaxDeg)); },
                              sort_tmp);
            fac_list[b].insert(fac_list[b].end(), src.begin(), src.end());
            fac_lvl_off[b].push_back(int32_t(fac_list[b].size()));
        }
    }
    auto vkey = [&](int32_t v) { return std::min<int32_t>(g.var_deg[v], kVarRecEdges); };
    for (int b = 0; b < VB_COUNT; ++b) {
        var_list[b].clear();
        var_lvl_off[b].assign(1, 0);
        for (int32_t L = 0; L < exec_levels; ++L) {
            auto &src = var_by_level[L * VB_COUNT + b];
            if (b == VB_THREAD) {  // by degree; on a narrow level the highest first, as for factors
                const bool narrow = int64_t(src.size()) <= kFuseMaxRecs;
                counting_sort(src, kVarRecEdges + 1,
                              [&](int32_t v) { return narrow ? int64_t(kVarRecEdges - vkey(v)) : int64_t(vkey(v)); },
                              sort_tmp);
            }
            var_list[b].insert(var_list[b].end(), src.begin(), src.end());
            var_lvl_off[b].push_back(int32_t(var_list[b].size()));
        }
        init_var[b].clear();
    }
    for (int32_t v = 0; v < g.V; ++v) init_var[g.var_deg[v] <= pp.var_thread_max_deg ? VB_THREAD : VB_WAVE].push_back(v);
    // records: factor {b, d | type << 8 | active << 16, id, u0..u7, 0}; variable {v, row, degree,
    // e0..e4}. A degree group is padded to a multiple of 64 with copies of its first record that
    // write nothing (factor: no active edge; variable: padding flag).
    frec.clear();
    frec.reserve(size_t(fac_lvl_off[FB_THREAD].back() + 64 * std::max(exec_levels, 1) * 8) * 12);
    frec_off.assign(1, 0);
    for (int32_t L = 0; L < exec_levels; ++L) {
        const int32_t i0 = fac_lvl_off[FB_THREAD][L], i1 = fac_lvl_off[FB_THREAD][L + 1];
        for (int32_t i = i0; i < i1;) {
            const int32_t d = fdeg(fac_list[FB_THREAD][i]);
            int32_t j = i;
            for (; j < i1 && fdeg(fac_list[FB_THREAD][j]) == d; ++j) {
                int32_t a = fac_list[FB_THREAD][j];
                int64_t b = g.fac_off[a];
                int32_t r[12] = {0};
                unsigned mask = 0;
                for (int64_t k = 0; k < d; ++k)
                    if (edge_exec_level[b + k] == L) mask |= 1u << k;
                r[0] = int32_t(b);
                r[1] = d | (int32_t(g.fac_type[a]) << 8) | int32_t(mask << 16);
                r[2] = a;
                for (int k = 0; k < 8; ++k) r[3 + k] = k < d ? g.edge_var[b + k] : 0;
                frec.insert(frec.end(), r, r + 12);
            }
            const size_t first = frec.size() - size_t(j - i) * 12;
            int32_t pad[12];
            std::copy(frec.begin() + first, frec.begin() + first + 12, pad);
            pad[1] &= 0xffff;  // no active edge
            while ((frec.size() / 12) % 64) frec.insert(frec.end(), pad, pad + 12);
            i = j;
        }
        frec_off.push_back(int32_t(frec.size() / 12));
    }
    vrec.clear();
    vrec.reserve(size_t(var_lvl_off[VB_THREAD].back() + 64 * std::max(exec_levels, 1) * 6) * 8);
    vrec_off.assign(1, 0);
    for (int32_t L = 0; L < exec_levels; ++L) {
        const int32_t i0 = var_lvl_off[VB_THREAD][L], i1 = var_lvl_off[VB_THREAD][L + 1];
        for (int32_t i = i0; i < i1;) {
            const int32_t key = vkey(var_list[VB_THREAD][i]);
            int32_t j = i;
            for (; j < i1 && vkey(var_list[VB_THREAD][j]) == key; ++j) {
                int32_t v = var_list[VB_THREAD][j];
                int32_t r[8] = {0};
                r[0] = v;
                r[1] = g.var_off[v];
                r[2] = g.var_deg[v];
                for (int q = 0; q < kVarRecEdges; ++q) r[3 + q] = q < g.var_deg[v] ? g.var_edge[g.var_off[v] + q] : 0;
                vrec.insert(vrec.end(), r, r + 8);
            }
            const size_t first = vrec.size() - size_t(j - i) * 8;
            int32_t pad[8];
            std::copy(vrec.begin() + first, vrec.begin() + first + 8, pad);
            pad[2] |= 1 << 30;  // padding: computes, stores nothing
            while ((vrec.size() / 8) % 64) vrec.insert(vrec.end(), pad, pad + 8);
            i = j;
        }
        vrec_off.push_back(int32_t(vrec.size() / 8));
    }
    // weighted-term records: {b, d | terms << 8 | written-edge mask << 16, first term, variables}
    trec.clear();
    trec_off.assign(1, 0);
    for (int32_t L = 0; L < exec_levels; ++L) {
        for (int32_t i = fac_lvl_off[FB_TERMS_THREAD][L]; i < fac_lvl_off[FB_TERMS_THREAD][L + 1]; ++i) {
            const int32_t a = fac_list[FB_TERMS_THREAD][i];
            const int64_t b = g.fac_off[a], d = g.fac_off[a + 1] - b;
            int32_t r[12] = {0};
            unsigned mask = 0;
            for (int64_t k = 0; k < d; ++k)
                if (edge_exec_level[b + k] == L) mask |= 1u << k;
            r[0] = int32_t(b);
            r[1] = int32_t(d) | ((g.term_off[a + 1] - g.term_off[a]) << 8) | int32_t(mask << 16);
            r[2] = g.term_off[a];
            for (int64_t k = 0; k < d; ++k) r[3 + k] = g.edge_var[b + k];
            trec.insert(trec.end(), r, r + 12);
        }
        trec_off.push_back(int32_t(trec.size() / 12));
    }
    // incremental variable phase (LEVELS executor): which (level, variable) tasks write only part
    // of the variable's edges; the written edges of every level grouped by variable, in variable
    // order (filled from the variable-major rows, so no sort is needed). Flooding writes every edge
    // of every variable in its one level: nothing to do there.
    drec.clear();
    dedge.clear();
    dwave.clear();
    drec_off.assign(1, 0);
    dwave_off.assign(1, 0);
    has_delta = 0;
    if (!flooding) {
        std::vector<int64_t> lcnt(size_t(exec_levels) + 1, 0);
        for (int64_t e = 0; e < g.E; ++e)
            if (edge_exec_level[e] >= 0) lcnt[size_t(edge_exec_level[e]) + 1]++;
        for (int32_t L = 0; L < exec_levels; ++L) lcnt[size_t(L) + 1] += lcnt[size_t(L)];
        std::vector<int64_t> pos(lcnt.begin(), lcnt.end() - 1);
        std::vector<int32_t> by_level(static_cast<size_t>(lcnt[size_t(exec_levels)]));
        for (int32_t v = 0; v < g.V; ++v)
            for (int32_t q = g.var_off[v]; q < g.var_off[v + 1]; ++q) {
                const int32_t e = g.var_edge[q];
                const int32_t L = edge_exec_level[e];
                if (L >= 0) by_level[size_t(pos[size_t(L)]++)] = e;
            }
        for (int32_t L = 0; L < exec_levels && !has_delta; ++L) {
            const int64_t b = lcnt[size_t(L)], en = lcnt[size_t(L) + 1];
            for (int64_t i = b; i < en && !has_delta;) {
                int64_t j = i;
                while (j < en && g.edge_var[by_level[size_t(j)]] == g.edge_var[by_level[size_t(i)]]) ++j;
                if (int32_t(j - i) < g.var_deg[g.edge_var[by_level[size_t(i)]]]) has_delta = 1;
                i = j;
            }
        }
        std::vector<std::array<int32_t, 8>> recs;
        for (int32_t L = 0; has_delta && L < exec_levels; ++L) {
            const int64_t b = lcnt[size_t(L)], en = lcnt[size_t(L) + 1];
            // records of the level, then sorted by (kind, edges held) so a wavefront runs one shape
            recs.clear();
            for (int64_t i = b; i < en;) {
                const int32_t v = g.edge_var[by_level[size_t(i)]];
                int64_t j = i;
                while (j < en && g.edge_var[by_level[size_t(j)]] == v) ++j;
                const int32_t w = int32_t(j - i), deg = g.var_deg[v];
                std::array<int32_t, 8> r{};
                r[0] = v;
                if (w == deg && deg <= pp.var_thread_max_deg) {  // rebuild from the row
                    r[1] = g.var_off[v];
                    r[2] = deg;
                    for (int q = 0; q < kVarRecEdges; ++q) r[3 + q] = q < deg ? g.var_edge[g.var_off[v] + q] : 0;
                    recs.push_back(r);
                } else if (w <= kVarThreadMaxDeg && w < deg) {  // add new - old of the written edges
                    r[1] = int32_t(dedge.size());
                    r[2] = w | (1 << 29);
                    for (int q = 0; q < w; ++q) {
                        if (q < kVarRecEdges) r[3 + q] = by_level[size_t(i + q)];
                        dedge.push_back(by_level[size_t(i + q)]);
                    }
                    recs.push_back(r);
                } else {
                    dwave.push_back(v);  // many written edges of a high-degree variable: rebuild by wavefront
                }
                i = j;
            }
            auto key = [](const std::array<int32_t, 8> &r) {
                return ((r[2] >> 29) & 1) * 16 + std::min<int32_t>(r[2] & 0xffff, kVarRecEdges);
            };
            {  // stable by key (32 kinds)
                std::vector<std::array<int32_t, 8>> byk[32];
                for (auto &r : recs) byk[key(r)].push_back(r);
                recs.clear();
                for (auto &bk : byk) recs.insert(recs.end(), bk.begin(), bk.end());
            }
            for (size_t i = 0; i < recs.size();) {
                size_t j = i;
                while (j < recs.size() && key(recs[j]) == key(recs[i])) ++j;
                for (size_t k = i; k < j; ++k) drec.insert(drec.end(), recs[k].begin(), recs[k].end());
                std::array<int32_t, 8> p = recs[i];  // padding copies of the group's first record
                p[2] |= 1 << 30;
                for (size_t k = j - i; k % 64; ++k) drec.insert(drec.end(), p.begin(), p.end());
                i = j;
            }
            drec_off.push_back(int32_t(drec.size() / 8));
            dwave_off.push_back(int32_t(dwave.size()));
        }
        if (!has_delta) {
            drec_off.assign(1, 0);
            dwave_off.assign(1, 0);
        }
    }
    // staging in LDS: a level qualifies when all of its written edges come from thread-bucket
    // factors, its variables have at most kStagedEdges written edges each and none takes the
    // wavefront path, and its written edges fit kMaxStageSlots
    level_lds.assign(exec_levels, 0);
    prec.clear();
    stage_slots = 0;
    // a level may be staged only if it is narrow: no level of a wide plan is (and its variable
    // records are not built)
    bool any_narrow = false;
    for (int32_t L = 0; L < exec_levels && !any_narrow; ++L)
        any_narrow = frec_off[L + 1] - frec_off[L] <= kMaxStageSlots;
    if (any_narrow) prec.assign(vrec.size() / 8 * 4, 0);
    std::vector<int32_t> edge_slot(any_narrow ? g.E : 0, -1);
    for (int32_t L = 0; any_narrow && L < exec_levels; ++L) {
        bool ok = fac_lvl_off[FB_WAVE][L + 1] == fac_lvl_off[FB_WAVE][L] &&
                  fac_lvl_off[FB_BLOCK][L + 1] == fac_lvl_off[FB_BLOCK][L] &&
                  fac_lvl_off[FB_TERMS_WAVE][L + 1] == fac_lvl_off[FB_TERMS_WAVE][L] &&
                  fac_lvl_off[FB_TERMS_THREAD][L + 1] == fac_lvl_off[FB_TERMS_THREAD][L] &&
                  var_lvl_off[VB_WAVE][L + 1] == var_lvl_off[VB_WAVE][L];
        int32_t slots = 0;
        for (int32_t i = frec_off[L]; i < frec_off[L + 1]; ++i) {
            int32_t *r = &frec[size_t(i) * 12];
            const int32_t b = r[0], d = r[1] & 0xff;
            const unsigned active = (unsigned)(r[1] >> 16) & 0xffu;
            r[11] = slots;
            for (int k = 0; k < d; ++k)
                if ((active >> k) & 1u) edge_slot[b + k] = slots++;
        }
        ok = ok && slots <= kMaxStageSlots;
        for (int32_t i = vrec_off[L]; ok && i < vrec_off[L + 1]; ++i) {
            const int32_t *r = &vrec[size_t(i) * 8];
            const int32_t v = r[0];
            int32_t *q = &prec[size_t(i) * 4];
            q[0] = v;
            int32_t n = 0, sl[kStagedEdges] = {0, 0, 0, 0, 0, 0};
            for (int32_t p = g.var_off[v]; p < g.var_off[v + 1]; ++p) {
                const int32_t e = g.var_edge[p];
                if (edge_exec_level[e] != L) continue;
                if (n == kStagedEdges || edge_slot[e] < 0) {
                    ok = false;
                    break;
                }
                sl[n++] = edge_slot[e];
            }
            if (n == 0) ok = false;  // a staged task reads its belief from its first slot
            const uint32_t pad = (r[2] >> 30) & 1;  // keeps the padding flag
            q[1] = int32_t(uint32_t(n) | pad << 3 | uint32_t(sl[0]) << 4 | uint32_t(sl[1]) << 18);
            q[2] = int32_t(uint32_t(sl[2]) | uint32_t(sl[3]) << 16);
            q[3] = int32_t(uint32_t(sl[4]) | uint32_t(sl[5]) << 16);
        }
        level_lds[L] = ok ? 1 : 0;
        if (ok) stage_slots = std::max(stage_slots, slots);
    }
    // narrow levels and the fused segments of the HYBRID executor; launches per iteration
    seg_end.assign(exec_levels, -1);
    seg_teams.assign(exec_levels, 0);
    fused_levels = 0;
    launches_levels = launches_hybrid = 1;  // the end-of-iteration kernel
    auto cnt = [](const std::vector<int32_t> &off, int32_t L) { return off[L + 1] - off[L]; };
    std::vector<uint8_t> narrow(exec_levels, 0);
    for (int32_t L = 0; L < exec_levels; ++L) {
        int launches = 0;
        for (int b = 0; b < FB_COUNT; ++b) launches += cnt(fac_lvl_off[b], L) > 0 && b != FB_THREAD ? 1 : 0;
        launches += cnt(frec_off, L) > 0 ? 1 : 0;
        launches += cnt(vrec_off, L) > 0 ? 1 : 0;
        launches += cnt(var_lvl_off[VB_WAVE], L) > 0 ? 1 : 0;
        launches_levels += launches;
        narrow[L] = cnt(frec_off, L) <= kFuseMaxRecs && cnt(vrec_off, L) <= kFuseMaxRecs &&
                    cnt(fac_lvl_off[FB_TERMS_THREAD], L) <= kFuseMaxRecs && cnt(fac_lvl_off[FB_BLOCK], L) == 0 &&
                    cnt(fac_lvl_off[FB_WAVE], L) + cnt(fac_lvl_off[FB_TERMS_WAVE], L) +
                            cnt(var_lvl_off[VB_WAVE], L) <= kFuseMaxWaveTasks;
    }
    for (int32_t L = 0; L < exec_levels;) {
        if (!narrow[L]) {
            int launches = 0;
            for (int b = 0; b < FB_COUNT; ++b) launches += cnt(fac_lvl_off[b], L) > 0 && b != FB_THREAD ? 1 : 0;
            launches += (cnt(frec_off, L) > 0) + (cnt(vrec_off, L) > 0) + (cnt(var_lvl_off[VB_WAVE], L) > 0);
            launches_hybrid += launches;
            ++L;
            continue;
        }
        int32_t e = L;
        bool teams = false;
        while (e < exec_levels && narrow[e] && e - L < kFuseMaxLevels) {
            teams = teams || cnt(fac_lvl_off[FB_WAVE], e) + cnt(fac_lvl_off[FB_TERMS_WAVE], e) +
                                     cnt(fac_lvl_off[FB_TERMS_THREAD], e) + cnt(var_lvl_off[VB_WAVE], e) > 0;
            ++e;
        }
        seg_end[L] = e;
        seg_teams[L] = teams ? 1 : 0;
        fused_levels += e - L;
        launches_hybrid += 1;
        L = e;
    }
}

}  // namespace fastlbp

extern "C" int fastlbp_graph_validate(int32_t num_vars, int32_t num_factors, const int64_t *factor_offsets,
                                      const int32_t *edge_vars, const uint8_t *factor_types,
                                      const double *factor_params, const double *edge_params) {
    fastlbp::clear_error();
    return fastlbp::validate_graph(num_vars, num_factors, factor_offsets, edge_vars, factor_types, factor_params,
                                   edge_params);
}

extern "C" int fastlbp_analyze_levels(int32_t num_vars, int32_t num_factors, const int64_t *factor_offsets,
                                      const int32_t *edge_vars, const int32_t *edge_rank, int32_t *level_of_edge,
                                      int32_t *num_levels_out) {
    fastlbp::clear_error();
    if (num_vars < 0 || num_factors < 0 || !factor_offsets || !level_of_edge) {
        fastlbp::set_error("invalid argument");
        return FASTLBP_E_INVALID_ARG;
    }
    if (factor_offsets[0] != 0) {
        fastlbp::set_error("factor_offsets[0] must be 0");
        return FASTLBP_E_BAD_GRAPH;
    }
    for (int32_t a = 0; a < num_factors; ++a)
        if (factor_offsets[a + 1] < factor_offsets[a]) {
            fastlbp::set_error("factor_offsets must be non-decreasing");
            return FASTLBP_E_BAD_GRAPH;
        }
    int64_t E = factor_offsets[num_factors];
    for (int64_t e = 0; e < E; ++e)
        if (edge_vars[e] < 0 || edge_vars[e] >= num_vars) {
            fastlbp::set_error("variable id out of range");
            return FASTLBP_E_BAD_GRAPH;
        }
    std::vector<int32_t> level;
    int32_t n = fastlbp::analyze_levels(num_vars, num_factors, factor_offsets, edge_vars, edge_rank, level);
    if (E) std::memcpy(level_of_edge, level.data(), sizeof(int32_t) * E);
    if (num_levels_out) *num_levels_out = n;
    return FASTLBP_OK;
}

extern "C" int fastlbp_classes_to_ranks(int32_t num_vars, int32_t num_factors, const int64_t *factor_offsets,
                                        const int32_t *edge_vars, const uint8_t *factor_types, int32_t num_classes,
                                        const int32_t *edge_class, int32_t num_arcs, const int32_t *arcs,
                                        int32_t *edge_rank) {
    fastlbp::clear_error();
    if (num_vars < 0 || num_factors < 0 || !factor_offsets || (factor_offsets[num_factors] > 0 && !edge_rank)) {
        fastlbp::set_error("invalid argument");
        return FASTLBP_E_INVALID_ARG;
    }
    if (factor_offsets[0] != 0) {
        fastlbp::set_error("factor_offsets[0] must be 0");
        return FASTLBP_E_BAD_GRAPH;
    }
    for (int32_t a = 0; a < num_factors; ++a)
        if (factor_offsets[a + 1] < factor_offsets[a]) {
            fastlbp::set_error("factor_offsets must be non-decreasing");
            return FASTLBP_E_BAD_GRAPH;
        }
    for (int64_t e = 0; e < factor_offsets[num_factors]; ++e)
        if (edge_vars[e] < 0 || edge_vars[e] >= num_vars) {
            fastlbp::set_error("variable id out of range");
            return FASTLBP_E_BAD_GRAPH;
        }
    std::vector<int32_t> rank;
    int rc = fastlbp::classes_to_ranks(num_vars, num_factors, factor_offsets, edge_vars, factor_types, num_classes,
                                   edge_class, num_arcs, arcs, rank);
    if (rc) return rc;
    if (!rank.empty()) std::memcpy(edge_rank, rank.data(), sizeof(int32_t) * rank.size());
    return FASTLBP_OK;
}

// ------------------------------------------------------------------------------------------------
// Rank generators of adaptive update strategies (randomized and residual-driven BP, Section 6)
// ------------------------------------------------------------------------------------------------

namespace fastlbp {

// SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number generators", 2014): the
// value for counter x of a stream is the output mix of seed + (x + 1) * golden gamma.
uint64_t splitmix64_at(uint64_t seed, uint64_t x) {
    uint64_t z = seed + (x + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

void ranks_random(int32_t F, const int64_t *off, int32_t groups, uint64_t seed, int32_t block, int32_t *rank) {
    for (int32_t a = 0; a < F; ++a) {
        const uint64_t x = (uint64_t(uint32_t(block)) << 32) | uint64_t(uint32_t(a));
        const int32_t r = int32_t(splitmix64_at(seed, x) % uint64_t(groups));
        for (int64_t e = off[a]; e < off[a + 1]; ++e) rank[e] = r;
    }
}

void ranks_residual(int64_t E, const double *before, const double *after, int32_t groups, int32_t *rank) {
    double rmax = 0.0;
    for (int64_t e = 0; e < E; ++e) rmax = std::max(rmax, std::fabs(after[e] - before[e]));
    for (int64_t e = 0; e < E; ++e) {
        if (!(rmax > 0.0)) {
            rank[e] = 0;
            continue;
        }
        const double q = double(groups) * (std::fabs(after[e] - before[e]) / rmax);
        const int32_t bucket = std::min<int32_t>(groups - 1, int32_t(std::floor(q)));
        rank[e] = groups - 1 - bucket;  // the largest changes go first
    }
}

}  // namespace fastlbp

extern "C" int fastlbp_ranks_random(int32_t num_factors, const int64_t *factor_offsets, int32_t groups, uint64_t seed,
                                    int32_t block, int32_t *edge_rank) {
    fastlbp::clear_error();
    if (num_factors < 0 || !factor_offsets || groups < 1 || block < 0 ||
        (factor_offsets[num_factors] > 0 && !edge_rank)) {
        fastlbp::set_error("invalid argument");
        return FASTLBP_E_INVALID_ARG;
    }
    for (int32_t a = 0; a < num_factors; ++a)
        if (factor_offsets[a + 1] < factor_offsets[a]) {
            fastlbp::set_error("factor_offsets must be non-decreasing");
            return FASTLBP_E_BAD_GRAPH;
        }
    fastlbp::ranks_random(num_factors, factor_offsets, groups, seed, block, edge_rank);
    return FASTLBP_OK;
}

extern "C" int fastlbp_ranks_residual(int64_t num_edges, const double *p_before, const double *p_after, int32_t groups,
                                      int32_t *edge_rank) {
    fastlbp::clear_error();
    if (num_edges < 0 || groups < 1 || (num_edges > 0 && (!p_before || !p_after || !edge_rank))) {
        fastlbp::set_error("invalid argument");
        return FASTLBP_E_INVALID_ARG;
    }
    for (int64_t e = 0; e < num_edges; ++e)
        if (!(p_before[e] >= 0.0 && p_before[e] <= 1.0) || !(p_after[e] >= 0.0 && p_after[e] <= 1.0)) {
            fastlbp::set_error("message " + std::to_string(e) + " outside [0,1]");
            return FASTLBP_E_INVALID_ARG;
        }
    fastlbp::ranks_residual(num_edges, p_before, p_after, groups, edge_rank);
    return FASTLBP_OK;
}
