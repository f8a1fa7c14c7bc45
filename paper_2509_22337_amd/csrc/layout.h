// Device data layout shared by the host planner and the HIP kernels.
//
// Edges keep the caller's factor-major numbering. Messages f->v live in one array indexed by
// edge id (stored as log-likelihood ratios in log2 units, "bits": l = log2 mu(1) - log2 mu(0)),
// so the factor phase reads and writes each factor's messages contiguously. Every variable keeps a
// belief record B_v = phi_v + sum over its non-PRIOR edges of l, accumulated in float64 with
// separate counts of +inf and -inf terms; the variable-to-factor message of Eq.(1) is then
// B_v minus the factor's own incoming message, which the factor phase forms on the fly. PRIOR
// factors are folded into phi_v together with evidence, so they never occupy message slots on the
// device.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <type_traits>

namespace fastlbp {

// Pointer to global memory. Indexing goes through an address_space(1) pointer, so device code
// uses global (not flat) memory instructions even when the pointer itself was loaded from memory
// (as in the per-workgroup run descriptors of the persistent executor).
template <class T>
struct GPtr {
    typedef __attribute__((address_space(1))) T gT;
    typedef __attribute__((address_space(1))) int gint;
    T *p;
    __host__ __device__ GPtr() : p(nullptr) {}
    __host__ __device__ GPtr(T *q) : p(q) {}
    // scalar element access
    __device__ __forceinline__ gT &operator[](int64_t i) const { return ((gT *)p)[i]; }
    __device__ __forceinline__ gT *operator->() const { return (gT *)p; }
    // whole-struct load and store, moved as dwords
    __device__ __forceinline__ typename std::remove_const<T>::type ld(int64_t i) const {
        static_assert(sizeof(T) % 4 == 0, "dword-sized structs only");
        const gint *q = (const gint *)(p + i);
        int tmp[sizeof(T) / 4];
#pragma unroll
        for (int k = 0; k < int(sizeof(T) / 4); ++k) tmp[k] = q[k];
        typename std::remove_const<T>::type out;
        __builtin_memcpy(&out, tmp, sizeof(T));
        return out;
    }
    // the same, streaming past the caches (data read once per iteration)
    __device__ __forceinline__ typename std::remove_const<T>::type ld_stream(int64_t i) const {
        static_assert(sizeof(T) % 4 == 0, "dword-sized structs only");
        const gint *q = (const gint *)(p + i);
        int tmp[sizeof(T) / 4];
#pragma unroll
        for (int k = 0; k < int(sizeof(T) / 4); ++k) tmp[k] = __builtin_nontemporal_load(q + k);
        typename std::remove_const<T>::type out;
        __builtin_memcpy(&out, tmp, sizeof(T));
        return out;
    }
    __device__ __forceinline__ void st(int64_t i, const T &v) const {
        static_assert(sizeof(T) % 4 == 0, "dword-sized structs only");
        int tmp[sizeof(T) / 4];
        __builtin_memcpy(tmp, &v, sizeof(T));
        gint *q = (gint *)(p + i);
#pragma unroll
        for (int k = 0; k < int(sizeof(T) / 4); ++k) q[k] = tmp[k];
    }
    __host__ __device__ T *get() const { return p; }
};

// Finite part plus counts of infinite terms of a sum of LLRs. A sum with both +inf and -inf
// terms is the product of two exactly-zero entries: the "null" message (0, 0).
struct Belief {
    double fin;
    int32_t npos;
    int32_t nneg;
};

template <typename V>
struct Pair {
    V a;  // parameter p (NOISY_OR activation / leak, IMPLIES weight) in the precision's value domain
    V b;  // 1 - p in the same domain
};

// Per-run state in device memory. Every kernel of a captured iteration returns immediately once
// `done` is set, so replaying more iterations than needed is harmless. The LEVELS executor's
// kernels fold their residual and contradiction partials into kRedSlots slots (one per 64-byte
// line, picked by workgroup index) rather than one word: device-scope atomics to a single address
// from all XCDs serialise, and at one per workgroup they would dominate a wide level. The
// end-of-iteration kernel reduces and clears the slots. Only the header (up to `rpart`) is copied
// to the host.
constexpr int kRedSlots = 64;
constexpr int kRedStride = 8;  // 64 bytes between slots
struct alignas(64) RunState {
    unsigned long long contra;  // messages replaced by uniform during the run
    int32_t iter;               // iterations completed
    int32_t done;               // 1 once converged or max_iters reached
    double last_r;              // residual of the last completed iteration
    int32_t max_iters;
    int32_t converged;
    double tol;
    int32_t step_end;           // a launch of the persistent executor returns once iter reaches this
    int32_t pad;
    alignas(64) unsigned long long rpart[kRedSlots * kRedStride];  // max |dP(x=1)| as double bits
    unsigned long long cpart[kRedSlots * kRedStride];              // contradictions
};
constexpr size_t kRunStateHeader = offsetof(RunState, rpart);

// Degree buckets. Factor degree d = inputs + head.
constexpr int kThreadMaxDeg = 8;     // one thread per factor
constexpr int kWaveMaxDeg = 257;     // one wavefront per factor: 64 lanes x up to 4 inputs + head
constexpr int kBlockMaxDeg = 16385;  // one 1024-thread workgroup per factor: 1024 x 16 + head
constexpr int kVarThreadMaxDeg = 64; // one thread per variable, else one wavefront
constexpr int kVarRecEdges = 5;      // edge ids held in a variable task record (VarRec::e)
// A level is narrow (one workgroup runs it in the HYBRID executor) with at most this many factor
// records and variable records, no workgroup-per-factor task and few wavefront tasks.
constexpr int kFuseMaxRecs = 2048;
constexpr int kFuseMaxWaveTasks = 128;
constexpr int kFuseMaxLevels = 2048;  // levels of one fused launch (their offsets go to LDS)

// Factors given as weighted terms: FB_TERMS_THREAD one thread per factor (degree <= kThreadMaxDeg),
// FB_TERMS_WAVE one wavefront per factor (degree up to 64)
enum { FB_THREAD = 0, FB_WAVE = 1, FB_BLOCK = 2, FB_TERMS_WAVE = 3, FB_TERMS_THREAD = 4, FB_COUNT = 5 };
enum { VB_THREAD = 0, VB_WAVE = 1, VB_COUNT = 2 };

template <typename S, typename V>
struct DevGraph {
    int32_t num_vars;
    int32_t num_edges;
    GPtr<const int32_t> fac_off;    // [F+1]
    GPtr<const int32_t> edge_var;   // [E]
    GPtr<const uint8_t> fac_type;   // [F]
    GPtr<const Pair<V>> fpar;       // [F]
    GPtr<const Pair<V>> epar;       // [E]
    GPtr<const int32_t> var_off;    // [V+1] over non-PRIOR edges
    GPtr<const int32_t> var_edge;   // [E_np] edge ids, variable-major
    GPtr<const Belief> phi;         // [V] priors + evidence
    GPtr<Belief> bel;               // [V]
    GPtr<S> msg;                    // [E]
    GPtr<S> prev;                   // [2E] (new, old) of each message a level wrote, side by side
                                    // (plans with incremental variable tasks), else null
    GPtr<const int32_t> edge_level; // [E] executed level of each edge (-1 for PRIOR edges)
    // weighted-term factors: term range per factor [F+1], weights in the value domain [T], start of
    // each factor's indicator rows [F+1], indicators (row t of factor a: one entry per edge, -1 any)
    GPtr<const int32_t> term_off;
    GPtr<const V> term_w;
    GPtr<const int32_t> term_base;
    GPtr<const int8_t> term_ind;
    // per term of a factor of degree <= 8: bit k = the term fixes edge k, bit 8 + k = to value 1
    GPtr<const uint16_t> term_mask;
    V damp_old;                // lambda in the value domain
    V damp_new;                // 1 - lambda in the value domain
    int32_t damped;            // lambda > 0 (a damped kernel leaves undamped runs' messages as computed)
};

// Work lists of one schedule, concatenated over the executed levels. Level L owns
// fac_list[b][fac_lvl_off[b][L] .. fac_lvl_off[b][L+1]) for every factor bucket b, and the same for
// variables. init_var lists every variable (all levels' beliefs are rebuilt from it at run start).
// Task records of the persistent executor: everything static about a task resolved on the host.
struct alignas(16) FacRec {
    int32_t b;     // first edge
    int32_t meta;  // degree | type << 8 | (edges the level writes, bit k = edge b + k) << 16
    int32_t fac;   // factor id (for its parameters)
    int32_t u[9];  // variable of edge b + k, k < degree (<= 8); u[8]: first staging slot of the
                   // record's written edges (persistent executor, levels staged in LDS)
};

// Task record of a weighted-term factor of degree <= 8 (thread path, both executors).
struct alignas(16) TermRec {
    int32_t b;     // first edge
    int32_t meta;  // degree | term count << 8 | (edges the level writes, bit k = edge b + k) << 16
    int32_t t0;    // first term
    int32_t u[9];  // variable of edge b + k, k < degree; u[8] unused
};

struct alignas(16) VarRec {
    int32_t v, start, cnt;  // variable, first position in var_edge, degree | (padding record) << 30
    int32_t e[5];           // its first edges (the rest from var_edge)
};

// Variable task of a level staged in LDS (persistent executor), 16 bytes so that two fit the
// registers of one prefetch: the variable, how many of its messages the level writes, a padding
// flag and their staging slots (n | pad << 3 | s0 << 4 | s1 << 18, then s2 | s3 << 16 and
// s4 | s5 << 16). Its belief is updated from the value before the level plus (new - old) of those
// messages.
constexpr int kStagedEdges = 6;
constexpr int kMaxStageSlots = 2048;  // written edges of a level that may be staged in LDS (< 2^14)
struct alignas(16) VarRecP {
    int32_t v;
    uint32_t a, b, c;
    __host__ __device__ int n() const { return int(a & 7u); }
    __host__ __device__ bool pad() const { return ((a >> 3) & 1u) != 0; }
    __host__ __device__ int32_t slot(int j) const {
        const uint32_t w = j < 2 ? (a >> (4 + 14 * j)) & 0x3fffu : ((j < 4 ? b : c) >> (16 * (j & 1))) & 0xffffu;
        return int32_t(w);
    }
};

struct DevPlan {
    int32_t num_levels;
    int32_t all_active;  // 1: every listed factor writes all of its edges (flooding)
    GPtr<const int32_t> fac_list[FB_COUNT];
    GPtr<const int32_t> fac_lvl_off[FB_COUNT];  // [num_levels+1]
    GPtr<const int32_t> var_list[VB_COUNT];
    GPtr<const int32_t> var_lvl_off[VB_COUNT];  // [num_levels+1]
    GPtr<const int32_t> init_var[VB_COUNT];
    int32_t init_var_count[VB_COUNT];
    // per-level task records of the thread buckets, sorted by degree, each degree group padded to
    // a multiple of 64 records (so every level starts at a multiple of 64)
    GPtr<const FacRec> frec;
    GPtr<const int32_t> frec_off;  // [num_levels+1]
    GPtr<const VarRec> vrec;
    GPtr<const int32_t> vrec_off;  // [num_levels+1]
    // levels staged in LDS (persistent executor): per level 1 if its variable phase reads the
    // level's new messages from LDS (then prec holds its variable tasks, in vrec's order)
    GPtr<const VarRecP> prec;
    GPtr<const int32_t> level_lds;  // [num_levels]
    // weighted-term factors of degree <= 8, per level (sorted by degree, then term count)
    GPtr<const TermRec> trec;
    GPtr<const int32_t> trec_off;   // [num_levels+1]
    int32_t stage_slots;            // most slots any staged level uses (0: none staged)
    // incremental variable tasks of the LEVELS executor (has_delta): per level records and the
    // wavefront rebuilds of high-degree variables
    int32_t has_delta;
    GPtr<const VarRec> drec;
    GPtr<const int32_t> drec_off;   // [num_levels+1]
    GPtr<const int32_t> dedge;      // written edges of the delta records beyond the fifth
    GPtr<const int32_t> dwave;
    GPtr<const int32_t> dwave_off;  // [num_levels+1]
};

}  // namespace fastlbp
