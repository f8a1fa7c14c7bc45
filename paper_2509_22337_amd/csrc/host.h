// Host-side graph preparation: validation, variable-major transpose, prior folding, the
// dependency analysis (Algorithm 2) and per-level work lists. No device code here.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "layout.h"

namespace fastlbp {

void set_error(const std::string &msg);
void clear_error();

int validate_graph(int32_t V, int32_t F, const int64_t *fac_off, const int32_t *edge_var, const uint8_t *fac_type,
                   const double *fac_param, const double *edge_param, const int64_t *term_off = nullptr,
                   const double *term_weight = nullptr, const int8_t *term_ind = nullptr);

// Class-atomic Algorithm 2 over the preorder given by `rank` (nullptr = one class).
// level[e] receives the level of every edge; returns the number of levels.
int32_t analyze_levels(int32_t V, int32_t F, const int64_t *fac_off, const int32_t *edge_var, const int32_t *rank,
                       std::vector<int32_t> &level);

// Largest number of classes of a general preorder (the comparability check keeps a C x C bit matrix).
constexpr int32_t kMaxClasses = 16384;
int classes_to_ranks(int32_t V, int32_t F, const int64_t *off, const int32_t *ev, const uint8_t *ft, int32_t C,
                     const int32_t *edge_class, int32_t A, const int32_t *arcs, std::vector<int32_t> &rank);

struct HostGraph {
    int32_t V = 0, F = 0;
    int64_t E = 0;
    std::vector<int64_t> fac_off;
    std::vector<int32_t> edge_var;
    std::vector<uint8_t> fac_type;
    std::vector<double> fac_param;   // defaults applied
    std::vector<double> edge_param;  // defaults applied
    std::vector<int32_t> edge_fac;
    std::vector<int32_t> var_off;    // [V+1] non-PRIOR edges
    std::vector<int32_t> var_edge;
    std::vector<int32_t> var_deg;    // non-PRIOR degree
    // PRIOR factors folded per variable: finite LLR sum (bits) and counts of p = 1 / p = 0
    std::vector<double> prior_fin;
    std::vector<int32_t> prior_pos, prior_neg;
    int32_t max_deg = 0;
    int64_t nonprior_edges = 0;
    // TERMS factors: term range per factor, weights, and indicator rows (term t of factor a fixes
    // edge k to term_ind[term_base[a] + (t - term_off[a]) * d_a + k], -1 = any value)
    std::vector<int32_t> term_off;   // [F+1] (empty when the graph has no TERMS factor)
    std::vector<double> term_weight; // [T]
    std::vector<int8_t> term_ind;
    std::vector<int32_t> term_base;  // [F+1]
    std::vector<uint16_t> term_mask; // [T] factors of degree <= 8: fixed-edge bits | value bits << 8

    void build(int32_t V, int32_t F, const int64_t *off, const int32_t *ev, const uint8_t *ft, const double *fp,
               const double *ep);
    void set_terms(const int64_t *toff, const double *tw, const int8_t *tind);
};

// Degree cut-offs of the task buckets (defaults from layout.h; the autotuner may pick others).
struct PlanParams {
    int32_t thread_max_deg = kThreadMaxDeg;         // factors of degree <= this: one thread (2..8)
    int32_t wave_max_deg = kWaveMaxDeg;             // then one wavefront up to this (<= 257), then a workgroup
    int32_t var_thread_max_deg = kVarThreadMaxDeg;  // variables of degree <= this: one thread, else a wavefront
    bool valid() const {
        return thread_max_deg >= 1 && thread_max_deg <= kThreadMaxDeg && wave_max_deg > thread_max_deg &&
               wave_max_deg <= kWaveMaxDeg && var_thread_max_deg >= 1 && var_thread_max_deg <= kVarThreadMaxDeg;
    }
};

// Work lists for one schedule. Levels without any non-PRIOR edge are not executed.
struct HostPlan {
    int32_t num_levels = 0;       // levels of the dependency analysis (all edges)
    int32_t exec_levels = 0;      // levels with work on the device
    int32_t all_active = 0;
    int32_t max_level_edges = 0;  // widest executed level (active non-PRIOR edges)
    std::vector<int32_t> level_of_edge;
    std::vector<int32_t> edge_exec_level;  // [E], -1 for PRIOR
    std::vector<int32_t> fac_list[FB_COUNT];
    std::vector<int32_t> fac_lvl_off[FB_COUNT];
    std::vector<int32_t> var_list[VB_COUNT];
    std::vector<int32_t> var_lvl_off[VB_COUNT];
    std::vector<int32_t> init_var[VB_COUNT];
    // task records of the thread buckets (12 / 8 int32 each): per level sorted by degree, each
    // degree group padded to a multiple of 64 records; frec_off / vrec_off delimit the levels
    std::vector<int32_t> frec, vrec;
    std::vector<int32_t> frec_off, vrec_off;
    // task records of the weighted-term thread bucket (12 int32 each, TermRec), per level
    std::vector<int32_t> trec, trec_off;
    // levels whose new messages the persistent executor stages in LDS: flag per level, variable
    // tasks with staging slots (4 int32 each, in vrec's order), most slots of a staged level
    std::vector<int32_t> level_lds;
    std::vector<int32_t> prec;
    int32_t stage_slots = 0;
    // incremental variable phase of the LEVELS executor (plans where some level writes only part of
    // a variable's edges): per level, records {v, start, count | kind, e0..e4} (8 int32 each) that
    // either rebuild the belief from the whole row (kind 0: the level writes every edge of v) or
    // add new - old of the written edges (kind 1: edges e0..e4, the rest at dedge[start..]);
    // variables above the thread bucket with many written edges rebuild by wavefront (dwave)
    int32_t has_delta = 0;
    std::vector<int32_t> drec, drec_off, dedge, dwave, dwave_off;
    // fused segments of the HYBRID executor: seg_end[L] > L when level L starts a run of narrow
    // levels [L, seg_end[L]) executed by one workgroup (seg_teams[L]: the run has wavefront tasks)
    std::vector<int32_t> seg_end;
    std::vector<uint8_t> seg_teams;
    int32_t fused_levels = 0;      // levels inside fused segments
    int32_t launches_levels = 0;   // kernel launches of one LEVELS iteration
    int32_t launches_hybrid = 0;   // kernel launches of one HYBRID iteration
    double bytes_per_iter = 0.0;   // bytes one iteration of this implementation moves (its structures)
    int64_t updates_per_iter = 0;  // non-PRIOR edges written per iteration
    // counts behind the method's own bytes of one iteration (method_bytes_per_iter)
    int64_t touched_edges_per_iter = 0;  // edges of the factors a level touches, summed over levels
    int64_t noisy_params_per_iter = 0;   // NOISY_OR activations read (inputs of touched NOISY_OR factors)
    int64_t term_weights_per_iter = 0;   // weights of touched weighted-term factors
    int64_t term_entries_per_iter = 0;   // indicator entries (terms x degree) of touched term factors

    // Bytes one iteration of the method moves at minimum, with s-byte messages (the message
    // representation of the precision: a 4- or 8-byte log-likelihood ratio). Each touched factor
    // edge costs 4 (the variable-major position of the edge) + s (gather f->v for Eq.(1)) + s
    // (v->f written) + s (v->f read by the factor); each written edge costs s (the new f->v) and,
    // when the old value is needed (damping or a convergence test), s more; each NOISY_OR
    // activation and each term weight s; each term indicator 2 bits (fixed, value). Under flooding
    // every edge is touched and written once: 4 + 5s per edge (+ s per activation).
    double method_bytes_per_iter(int s, bool needs_old) const {
        return double(touched_edges_per_iter) * (4.0 + 3.0 * s) + double(updates_per_iter) * (needs_old ? 2.0 * s : s) +
               double(noisy_params_per_iter + term_weights_per_iter) * s + double(term_entries_per_iter) * 0.25;
    }

    PlanParams params;

    void build(const HostGraph &g, const std::vector<int32_t> &level, int32_t nlevels, bool flooding,
               int msg_bytes, int param_bytes, const PlanParams &pp = PlanParams());
};

int factor_bucket(int deg, const PlanParams &pp = PlanParams());

// Rank generators of adaptive update strategies: random ordered groups (every factor's edges share
// a rank drawn from a counter-based generator of seed, block and factor) and residual-driven ranks
// (the edges whose messages changed most go first, in `groups` classes of equal width of the change).
uint64_t splitmix64_at(uint64_t seed, uint64_t x);
void ranks_random(int32_t F, const int64_t *off, int32_t groups, uint64_t seed, int32_t block, int32_t *rank);
void ranks_residual(int64_t E, const double *before, const double *after, int32_t groups, int32_t *rank);

}  // namespace fastlbp
