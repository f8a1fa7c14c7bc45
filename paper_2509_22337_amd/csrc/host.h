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
    // tasks with staging slots (8 int32 each, in vrec's order), most slots of a staged level
    std::vector<int32_t> level_lds;
    std::vector<int32_t> prec;
    int32_t stage_slots = 0;
    // fused segments of the HYBRID executor: seg_end[L] > L when level L starts a run of narrow
    // levels [L, seg_end[L]) executed by one workgroup (seg_teams[L]: the run has wavefront tasks)
    std::vector<int32_t> seg_end;
    std::vector<uint8_t> seg_teams;
    int32_t fused_levels = 0;      // levels inside fused segments
    int32_t launches_levels = 0;   // kernel launches of one LEVELS iteration
    int32_t launches_hybrid = 0;   // kernel launches of one HYBRID iteration
    double bytes_per_iter = 0.0;   // algorithmic bytes of one iteration
    int64_t updates_per_iter = 0;  // non-PRIOR edges written per iteration

    void build(const HostGraph &g, const std::vector<int32_t> &level, int32_t nlevels, bool flooding,
               int msg_bytes, int param_bytes);
};

int factor_bucket(int deg);

}  // namespace fastlbp
