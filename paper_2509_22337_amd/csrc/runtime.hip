// Kernels, iteration driver and the C ABI of libfastlbp (the Kernel Launch and Message Passing
// stages of Section 4.1, executed as described in Section 4.3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <type_traits>
#include <vector>

#include "fastlbp.h"
#include "host.h"
#include "internal.h"
#include "kernels.h"

namespace fastlbp {

// ------------------------------------------------------------------------------------------------
// Kernels
// ------------------------------------------------------------------------------------------------

// Workgroup-wide residual (max) and contradiction count (sum), then one atomic per workgroup into
// the slot of its index. Every thread of the workgroup must call it.
template <int NT>
__device__ __forceinline__ void flush_acc(Acc acc, RunState *st) {
    constexpr int NW = NT / 64;
    __shared__ double s_r[NW];
    __shared__ unsigned int s_c[NW];
    double r = acc.r;
    unsigned int c = acc.contra;
#pragma unroll
    for (int k = 32; k >= 1; k >>= 1) {
        r = fmax(r, __shfl_xor(r, k, 64));
        c += __shfl_xor(c, k, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        s_r[threadIdx.x >> 6] = r;
        s_c[threadIdx.x >> 6] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < NW; ++i) {
            r = fmax(r, s_r[i]);
            c += s_c[i];
        }
        const int slot = int(blockIdx.x % kRedSlots) * kRedStride;
        if (r > 0.0) atomicMax(&st->rpart[slot], (unsigned long long)__double_as_longlong(r));
        if (c) atomicAdd(&st->cpart[slot], (unsigned long long)c);
    }
}

// Factors of degree <= 8 from the level's task records (records of a level start at a multiple of
// 64 and the grid stride is a multiple of 64, so a wavefront's records share one degree).
template <class P, bool DAMP>
__global__ __launch_bounds__(256) void k_fac_rec(DevGraph<typename P::S, typename P::V> g, const FacRec *recs,
                                                 int32_t count, RunState *st) {
    if (st->done) return;
    Acc acc = {0.0, 0u};
    const GPtr<const FacRec> R(recs);
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        factor_rec<P, DAMP>(g, R.ld_stream(i), acc);
    flush_acc<256>(acc, st);
}

template <class P, bool ALL, bool DAMP>
__global__ __launch_bounds__(256) void k_fac_wave(DevGraph<typename P::S, typename P::V> g, const int32_t *list,
                                                  int32_t count, int32_t level, RunState *st) {
    if (st->done) return;
    Acc acc = {0.0, 0u};
    const int lane = threadIdx.x & 63;
    const int waves = gridDim.x * (blockDim.x >> 6);
    for (int32_t i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); i < count; i += waves)
        factor_wave<P, ALL, DAMP>(g, list[i], lane, level, acc);
    flush_acc<256>(acc, st);
}

// Weighted-term factors, one wavefront each.
template <class P, bool ALL, bool DAMP>
__global__ __launch_bounds__(256) void k_fac_terms(DevGraph<typename P::S, typename P::V> g, const int32_t *list,
                                                   int32_t count, int32_t level, RunState *st) {
    if (st->done) return;
    Acc acc = {0.0, 0u};
    const int lane = threadIdx.x & 63;
    const int waves = gridDim.x * (blockDim.x >> 6);
    for (int32_t i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); i < count; i += waves)
        factor_terms<P, ALL, DAMP>(g, list[i], lane, level, acc);
    flush_acc<256>(acc, st);
}

// Weighted-term factors of degree <= 8, one thread per task record.
template <class P, bool DAMP>
__global__ __launch_bounds__(256) void k_fac_terms_rec(DevGraph<typename P::S, typename P::V> g, const TermRec *recs,
                                                       int32_t count, RunState *st) {
    if (st->done) return;
    Acc acc = {0.0, 0u};
    const GPtr<const TermRec> R(recs);
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        factor_terms_rec<P, DAMP>(g, R.ld_stream(i), acc);
    flush_acc<256>(acc, st);
}

// One workgroup of NT threads per factor (1024 for float32; 512 for float64, whose factor code
// needs more than the 128 registers a 1024-thread workgroup allows).
template <class P, bool ALL, bool DAMP, int NT>
__global__ __launch_bounds__(NT) void k_fac_block(DevGraph<typename P::S, typename P::V> g, const int32_t *list,
                                                  int32_t count, int32_t level, RunState *st) {
    if (st->done) return;
    __shared__ TeamLds<typename P::V> lds;
    Acc acc = {0.0, 0u};
    for (int32_t i = blockIdx.x; i < count; i += gridDim.x)
        factor_team<P, NT, (kBlockMaxDeg - 1) / NT, ALL, DAMP>(g, list[i], threadIdx.x, level, acc, &lds);
    flush_acc<NT>(acc, st);
}

template <class P>
constexpr int block_threads() {
    return sizeof(typename P::V) == 8 ? 512 : 1024;
}

template <class P>
__global__ __launch_bounds__(256) void k_var_thread(DevGraph<typename P::S, typename P::V> g, const int32_t *list,
                                                    int32_t count, const RunState *st) {
    if (st && st->done) return;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        var_thread<P>(g, list[i]);
}

template <class P>
__global__ __launch_bounds__(256) void k_var_rec(DevGraph<typename P::S, typename P::V> g, const VarRec *recs,
                                                 int32_t count, const RunState *st) {
    if (st->done) return;
    const GPtr<const VarRec> R(recs);
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        var_rec<P>(g, R.ld_stream(i));
}

template <class P>
__global__ __launch_bounds__(256) void k_var_wave(DevGraph<typename P::S, typename P::V> g, const int32_t *list,
                                                  int32_t count, const RunState *st) {
    if (st && st->done) return;
    const int waves = gridDim.x * (blockDim.x >> 6);
    for (int32_t i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); i < count; i += waves)
        var_wave<P>(g, list[i], threadIdx.x & 63);
}

// Resets the residual slots (one 64-thread workgroup).
__device__ __forceinline__ void clear_slots(RunState *st) {
    for (int i = threadIdx.x; i < kRedSlots; i += blockDim.x) {
        st->rpart[i * kRedStride] = 0ull;
        st->cpart[i * kRedStride] = 0ull;
    }
}

__global__ void k_run_init(RunState *st, int32_t max_iters, double tol) {
    clear_slots(st);
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->contra = 0ull;
        st->iter = 0;
        st->done = max_iters <= 0 ? 1 : 0;
        st->last_r = 0.0;
        st->max_iters = max_iters;
        st->converged = 0;
        st->tol = tol;
        st->step_end = max_iters;
    }
}

static_assert(kRedSlots == 64, "k_finalize reduces the slots with one wavefront");

// End of one iteration (one 64-thread workgroup): reduce and clear the residual slots, publish
// the residual, decide whether to stop.
__global__ void k_finalize(RunState *st) {
    if (st->done) return;
    const int t = threadIdx.x;
    double r = __longlong_as_double((long long)st->rpart[t * kRedStride]);
    unsigned long long c = st->cpart[t * kRedStride];
    st->rpart[t * kRedStride] = 0ull;
    st->cpart[t * kRedStride] = 0ull;
#pragma unroll
    for (int k = 32; k >= 1; k >>= 1) {
        r = fmax(r, __shfl_xor(r, k, 64));
        c += __shfl_xor(c, k, 64);
    }
    if (t != 0) return;
    st->contra += c;
    st->iter += 1;
    st->last_r = r;
    if (r < st->tol) {
        st->converged = 1;
        st->done = 1;
    } else if (st->iter >= st->max_iters) {
        st->done = 1;
    }
}

// Eq.(3) from the beliefs: P(x=1) = 1 / (1 + 2^-B); contradictory beliefs give 1/2.
__global__ void k_marginals(const Belief *bel, int32_t V, double *out) {
    int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    out[v] = belief_p1(bel[v]);
}

// Descriptor of one run for the persistent executor: the graph view (structure + state pointers,
// damping), the level plan and the run's state. A launch handles one descriptor per workgroup, so
// many graphs (or many queries of one graph) run side by side in one launch.
template <class P>
struct RunDesc {
    DevGraph<typename P::S, typename P::V> g;
    DevPlan plan;
    GPtr<RunState> st;
    GPtr<int32_t> status;  // receives a copy of the run's state header when the launch ends
    int32_t step;          // > 0: this launch stops the run after `step` more iterations
};

// Dynamic LDS of a level staged in LDS, for `cap` slots: the (new, old) message pairs (padded to
// 16 bytes), then one belief per slot.
template <class S>
__host__ __device__ constexpr size_t stage_pair_bytes(int32_t cap) {
    return (sizeof(S) * 2 * size_t(cap) + 15) & ~size_t(15);
}
template <class S>
__host__ __device__ constexpr size_t stage_bytes(int32_t cap) {
    return stage_pair_bytes<S>(cap) + sizeof(Belief) * size_t(cap);
}

// Levels [L0, L1) of one run in one workgroup of NT threads, with workgroup barriers between
// phases. Thread tasks come as records whose loads are issued one phase ahead (the variable records
// of a level while its factor phase runs, the factor records of the next level while the variable
// phase runs), so each phase waits for one round of dependent loads. On entry `fr` / `pr` hold this
// thread's first factor record of L0 and, if L0 is staged, its first staged variable record; on
// exit they hold those of level `Lnext` (none when Lnext < 0). TEAMS adds the wavefront- and
// workgroup-per-factor paths and the weighted-term paths. foff / voff / staged give each level's
// record offsets and staging flag.
template <class P, bool DAMP, bool TEAMS, int NT, bool UNCOND, class FOff, class VOff, class Staged>
__device__ __forceinline__ void level_range(const DevGraph<typename P::S, typename P::V> &g, const DevPlan &plan,
                                            int32_t L0, int32_t L1, int32_t Lnext, FOff foff, VOff voff,
                                            Staged staged, typename P::S *s_slot, Belief *b_slot,
                                            TeamLds<typename P::V> *lds, Acc &acc, FacRec &fr, VarRecP &pr) {
    using S = typename P::S;
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const GPtr<const FacRec> frec = plan.frec;
    const GPtr<const VarRec> vrec = plan.vrec;
    const GPtr<const VarRecP> prec = plan.prec;
    for (int32_t L = L0; L < L1; ++L) {
        const int32_t f0 = foff(L), f1 = foff(L + 1);
        const int32_t v0 = voff(L), v1 = voff(L + 1);
        const bool stg = staged(L);
        // variable phase input of an unstaged level, issued now (a staged level's variable phase
        // reads LDS only: its records were prefetched, its beliefs come from the factor phase)
        VarRec vr = {};
        const VarRecP pc = pr;
        if (v0 + tid < v1 && !stg) vr = vrec.ld_stream(v0 + tid);
        S *const slots = stg ? s_slot : nullptr;
        if (f0 + tid < f1) factor_rec<P, DAMP>(g, fr, acc, slots, b_slot);
        for (int32_t i = f0 + tid + NT; i < f1; i += NT)
            factor_rec<P, DAMP>(g, frec.ld_stream(i), acc, slots, b_slot);
        if (TEAMS) {
            const GPtr<const int32_t> lst = plan.fac_list[FB_WAVE];
            int32_t o0 = plan.fac_lvl_off[FB_WAVE][L], o1 = plan.fac_lvl_off[FB_WAVE][L + 1];
            for (int32_t i = o0 + w; i < o1; i += NW) factor_wave<P, false, DAMP>(g, lst[i], lane, L, acc);
        }
        if (TEAMS) {
            const int32_t o0 = plan.trec_off[L], o1 = plan.trec_off[L + 1];
            for (int32_t i = o0 + tid; i < o1; i += NT) factor_terms_rec<P, DAMP>(g, plan.trec.ld_stream(i), acc);
        }
        if (TEAMS) {
            const GPtr<const int32_t> lst = plan.fac_list[FB_TERMS_WAVE];
            int32_t o0 = plan.fac_lvl_off[FB_TERMS_WAVE][L], o1 = plan.fac_lvl_off[FB_TERMS_WAVE][L + 1];
            for (int32_t i = o0 + w; i < o1; i += NW) factor_terms<P, false, DAMP>(g, lst[i], lane, L, acc);
        }
        if (TEAMS) {
            const GPtr<const int32_t> lst = plan.fac_list[FB_BLOCK];
            int32_t o0 = plan.fac_lvl_off[FB_BLOCK][L], o1 = plan.fac_lvl_off[FB_BLOCK][L + 1];
            for (int32_t i = o0; i < o1; ++i)
                factor_team<P, NT, (kBlockMaxDeg - 1) / NT, false, DAMP>(g, lst[i], tid, L, acc, lds);
        }
        if (stg) {
            // the variable phase reads only the staging slots and beliefs loaded before the
            // level: wait for LDS, not for the messages' global stores
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
            __builtin_amdgcn_s_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
        } else {
            __syncthreads();
        }
        {
            // records of the next level (Lnext after the last level of the range)
            // UNCOND: unconditional loads, record 0 for threads without one (never used: the phases
            // check the index again), since a conditional load makes the compiler wait for it at
            // once; the conditional form needs fewer registers
            const int32_t Ln = (L + 1 < L1) ? L + 1 : Lnext;
            if (UNCOND) {
                if (Ln >= 0) {
                    const int32_t n0 = foff(Ln), n1 = foff(Ln + 1);
                    fr = frec.ld_stream(n0 + tid < n1 ? n0 + tid : 0);
                    const int32_t m0 = voff(Ln), m1 = voff(Ln + 1);
                    pr = prec.ld_stream(staged(Ln) && m0 + tid < m1 ? m0 + tid : 0);
                }
            } else {
                fr = FacRec{};
                pr = VarRecP{};
                if (Ln >= 0) {
                    const int32_t n0 = foff(Ln), n1 = foff(Ln + 1);
                    if (n0 + tid < n1) fr = frec.ld_stream(n0 + tid);
                    const int32_t m0 = voff(Ln), m1 = voff(Ln + 1);
                    if (staged(Ln) && m0 + tid < m1) pr = prec.ld_stream(m0 + tid);
                }
            }
        }
        if (stg) {
            if (v0 + tid < v1) var_staged<P>(g, pc, s_slot, b_slot);
            for (int32_t i = v0 + tid + NT; i < v1; i += NT) var_staged<P>(g, prec.ld_stream(i), s_slot, b_slot);
        } else {
            if (v0 + tid < v1) var_rec<P>(g, vr);
            for (int32_t i = v0 + tid + NT; i < v1; i += NT) var_rec<P>(g, vrec.ld_stream(i));
            const GPtr<const int32_t> lst = plan.var_list[VB_WAVE];
            int32_t o0 = plan.var_lvl_off[VB_WAVE][L], o1 = plan.var_lvl_off[VB_WAVE][L + 1];
            for (int32_t i = o0 + w; i < o1; i += NW) var_wave<P>(g, lst[i], lane);
        }
        // the next level reads these beliefs and messages from memory
        __syncthreads();
    }
}

// One workgroup of NT threads runs every level and iteration of one run. Used when the levels are
// too narrow to fill the GPU. A launch returns when the run is done or its iteration count reaches
// st->step_end, so a caller can advance many runs in steps. OFFL: every run's per-level offsets and
// flags fit the launch's LDS table (else they are read from memory); a compile-time choice, so the
// level loop has one path and the compiler's memory waits stay precise.
template <class P, bool DAMP, bool TEAMS, int NT, bool OFFL>
__global__ __launch_bounds__(NT) void k_persistent(const RunDesc<P> *descs, int32_t lds_levels, int32_t stage_cap) {
    using S = typename P::S;
    using V = typename P::V;
    constexpr int NW = NT / 64;
    __shared__ TeamLds<V> lds;
    __shared__ double red_r[NW];
    __shared__ unsigned int red_c[NW];
    __shared__ int s_done;
    // dynamic LDS: staging slots (new, old message pairs of a staged level's written edges), the
    // beliefs before the level of those edges' variables, then the per-level factor record
    // offsets, variable record offsets and staging flags
    extern __shared__ __align__(16) unsigned char s_dyn[];
    S *const s_slot = (S *)s_dyn;
    Belief *const b_slot = (Belief *)(s_dyn + stage_pair_bytes<S>(stage_cap));
    int32_t *const s_off = (int32_t *)(s_dyn + stage_bytes<S>(stage_cap));
    const RunDesc<P> &D = descs[blockIdx.x];
    const DevGraph<typename P::S, typename P::V> g = D.g;
    const DevPlan plan = D.plan;
    GPtr<RunState> st = D.st;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const GPtr<const FacRec> frec = plan.frec;
    const GPtr<const VarRecP> prec = plan.prec;
    const int32_t NL = plan.num_levels;
    // staged levels need the launch's slot area to hold this plan's largest staged level
    const bool staging = plan.stage_slots > 0 && plan.stage_slots <= stage_cap;
    // per-level offsets and flags: staged once in LDS so that a level does not start with a round
    // trip to memory (schedules deeper than the launch's LDS allowance read them from memory)
    if (OFFL)
        for (int32_t i = tid; i <= NL; i += NT) {
            s_off[i] = plan.frec_off[i];
            s_off[lds_levels + 1 + i] = plan.vrec_off[i];
            s_off[2 * (lds_levels + 1) + i] = (staging && i < NL) ? (int32_t)plan.level_lds[i] : 0;
        }
    auto foff = [&](int32_t L) { return OFFL ? s_off[L] : (int32_t)plan.frec_off[L]; };
    auto voff = [&](int32_t L) { return OFFL ? s_off[lds_levels + 1 + L] : (int32_t)plan.vrec_off[L]; };
    auto staged = [&](int32_t L) {
        return OFFL ? s_off[2 * (lds_levels + 1) + L] != 0 : (staging && plan.level_lds[L] != 0);
    };
    for (int32_t i = tid; i < plan.init_var_count[VB_THREAD]; i += NT) var_thread<P>(g, plan.init_var[VB_THREAD][i]);
    for (int32_t i = w; i < plan.init_var_count[VB_WAVE]; i += NW) var_wave<P>(g, plan.init_var[VB_WAVE][i], lane);
    if (tid == 0) {
        if (D.step > 0) st->step_end = st->iter + D.step;
        s_done = st->done || st->iter >= st->step_end;
    }
    __syncthreads();
    // records of level 0: the factor record, and the staged variable record when level 0 is staged
    FacRec fr = {};
    VarRecP pr = {};
    if (NL > 0) {
        fr = frec.ld_stream(foff(0) + tid < foff(1) ? foff(0) + tid : 0);
        pr = prec.ld_stream(staged(0) && voff(0) + tid < voff(1) ? voff(0) + tid : 0);
    }
    while (!s_done) {
        Acc acc = {0.0, 0u};
        level_range<P, DAMP, TEAMS, NT, true>(g, plan, 0, NL, 0, foff, voff, staged, s_slot, b_slot, &lds, acc, fr, pr);
        // end of iteration: block-wide residual and contradiction count
        double r = acc.r;
        unsigned int c = acc.contra;
#pragma unroll
        for (int k = 32; k >= 1; k >>= 1) {
            r = fmax(r, __shfl_xor(r, k, 64));
            c += __shfl_xor(c, k, 64);
        }
        if (lane == 0) {
            red_r[w] = r;
            red_c[w] = c;
        }
        __syncthreads();
        if (tid == 0) {
            double rr = 0.0;
            unsigned long long cc = 0;
            for (int i = 0; i < NW; ++i) {
                rr = fmax(rr, red_r[i]);
                cc += red_c[i];
            }
            st->contra += cc;
            st->iter += 1;
            st->last_r = rr;
            if (rr < st->tol) {
                st->converged = 1;
                st->done = 1;
            } else if (st->iter >= st->max_iters) {
                st->done = 1;
            }
            s_done = st->done || st->iter >= st->step_end;
        }
        __syncthreads();
    }
    // state header for the host, gathered with the other runs' into one array
    if (tid == 0) {
        const __attribute__((address_space(1))) int32_t *src = (const __attribute__((address_space(1))) int32_t *)st.get();
        for (int k = 0; k < int(kRunStateHeader / 4); ++k) D.status[k] = src[k];
    }
}

// Levels [L0, L1) of one iteration of the LEVELS executor in one workgroup: a run of narrow
// levels that would otherwise cost a few launches each. The residual and contradiction count go
// into the run state's slots like those of the other factor kernels.
template <class P, bool DAMP, bool TEAMS, int NT>
__global__ __launch_bounds__(NT) void k_levels_fused(DevGraph<typename P::S, typename P::V> g, DevPlan plan,
                                                     RunState *st, int32_t L0, int32_t L1, int32_t stage_cap) {
    using S = typename P::S;
    using V = typename P::V;
    __shared__ TeamLds<V> lds;
    extern __shared__ __align__(16) unsigned char s_dyn[];
    if (st->done) return;
    S *const s_slot = (S *)s_dyn;
    Belief *const b_slot = (Belief *)(s_dyn + stage_pair_bytes<S>(stage_cap));
    const int tid = threadIdx.x;
    const bool staging = plan.stage_slots > 0 && plan.stage_slots <= stage_cap;
    auto foff = [&](int32_t L) { return (int32_t)plan.frec_off[L]; };
    auto voff = [&](int32_t L) { return (int32_t)plan.vrec_off[L]; };
    auto staged = [&](int32_t L) { return staging && plan.level_lds[L] != 0; };
    FacRec fr = {};
    VarRecP pr = {};
    if (foff(L0) + tid < foff(L0 + 1)) fr = plan.frec.ld_stream(foff(L0) + tid);
    if (staged(L0) && voff(L0) + tid < voff(L0 + 1)) pr = plan.prec.ld_stream(voff(L0) + tid);
    Acc acc = {0.0, 0u};
    level_range<P, DAMP, TEAMS, NT, false>(g, plan, L0, L1, -1, foff, voff, staged, s_slot, b_slot, &lds, acc, fr, pr);
    flush_acc<NT>(acc, st);
}

// ------------------------------------------------------------------------------------------------
// Device memory
// ------------------------------------------------------------------------------------------------

#define HIPCHK(x)                                                                                          \
    do {                                                                                                   \
        hipError_t _e = (x);                                                                               \
        if (_e != hipSuccess) throw DeviceError{std::string(#x) + ": " + hipGetErrorString(_e)};           \
    } while (0)

// A set of device allocations freed together.
struct DevPool {
    Alloc alloc;
    std::vector<void *> owned;
    size_t bytes = 0;
    void *get(size_t n) {
        void *p = alloc.get(n);
        if (!p) throw OomError{};
        owned.push_back(p);
        bytes += n;
        return p;
    }
    template <class T>
    T *upload(const std::vector<T> &v, hipStream_t s) {
        T *p = (T *)get(sizeof(T) * std::max<size_t>(v.size(), 1));
        if (!v.empty()) {
            HIPCHK(hipMemcpyAsync(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s));
            HIPCHK(hipStreamSynchronize(s));  // the host vector may die after return
        }
        return p;
    }
    void release() {
        for (void *p : owned) alloc.put(p);
        owned.clear();
        bytes = 0;
    }
    ~DevPool() { release(); }
};

// Graph structure on the device: immutable after creation, shared by clones.
struct Structure {
    int device = 0;
    int precision = FASTLBP_FP64;
    HostGraph hg;
    DevPool pool;
    int32_t *fac_off = nullptr, *edge_var = nullptr, *var_off = nullptr, *var_edge = nullptr;
    uint8_t *fac_type = nullptr;
    void *fpar = nullptr, *epar = nullptr;
    int32_t *term_off = nullptr, *term_base = nullptr;
    void *term_w = nullptr;
    int8_t *term_ind = nullptr;
    uint16_t *term_mask = nullptr;
    size_t msg_bytes() const { return precision == FASTLBP_FP32 ? 4 : 8; }
    size_t val_bytes() const { return precision == FASTLBP_FP32 ? 4 : 8; }
};

// Level plan of one schedule on the device: immutable after schedule_set, shared by clones.
struct Plan {
    int kind = FASTLBP_SCHED_FLOODING;
    HostPlan hp;
    DevPool pool;
    int32_t *edge_level = nullptr;
    int32_t *fac_list[FB_COUNT] = {}, *fac_lvl_off[FB_COUNT] = {};
    int32_t *var_list[VB_COUNT] = {}, *var_lvl_off[VB_COUNT] = {}, *init_var[VB_COUNT] = {};
    int32_t *frec = nullptr, *vrec = nullptr, *frec_off = nullptr, *vrec_off = nullptr;
    int32_t *prec = nullptr, *level_lds = nullptr;
    int32_t *trec = nullptr, *trec_off = nullptr;
    bool teams() const {
        return !hp.fac_list[FB_WAVE].empty() || !hp.fac_list[FB_BLOCK].empty() ||
               !hp.fac_list[FB_TERMS_WAVE].empty() || !hp.fac_list[FB_TERMS_THREAD].empty();
    }
    DevPlan view() const {
        DevPlan p;
        p.num_levels = hp.exec_levels;
        p.all_active = hp.all_active;
        for (int b = 0; b < FB_COUNT; ++b) {
            p.fac_list[b] = fac_list[b];
            p.fac_lvl_off[b] = fac_lvl_off[b];
        }
        for (int b = 0; b < VB_COUNT; ++b) {
            p.var_list[b] = var_list[b];
            p.var_lvl_off[b] = var_lvl_off[b];
            p.init_var[b] = init_var[b];
            p.init_var_count[b] = int32_t(hp.init_var[b].size());
        }
        p.frec = (const FacRec *)frec;
        p.frec_off = frec_off;
        p.vrec = (const VarRec *)vrec;
        p.vrec_off = vrec_off;
        p.prec = (const VarRecP *)prec;
        p.level_lds = level_lds;
        p.trec = (const TermRec *)trec;
        p.trec_off = trec_off;
        p.stage_slots = hp.stage_slots;
        return p;
    }
};

// Stream, descriptor buffer and events for persistent launches (one per handle, one per server).
struct Launcher {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    DevPool pool;
    void *desc = nullptr;
    size_t desc_cap = 0;
    std::vector<unsigned char> hdesc;
    unsigned char *hstatus = nullptr;  // pinned copy of the runs' state headers after a launch
    size_t hstatus_cap = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t k0 = nullptr, k1 = nullptr;  // around the last persistent kernel
    float last_kernel_ms = 0.f;
    void init(hipStream_t s, const Alloc &a) {
        pool.alloc = a;
        if (s) {
            stream = s;
        } else {
            HIPCHK(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
            own_stream = true;
        }
        HIPCHK(hipEventCreate(&ev0));
        HIPCHK(hipEventCreate(&ev1));
        HIPCHK(hipEventCreate(&k0));
        HIPCHK(hipEventCreate(&k1));
    }
    void *descs(size_t bytes) {
        if (bytes > desc_cap) {
            pool.release();
            desc_cap = std::max<size_t>(bytes, 4096);
            desc = pool.get(desc_cap);
        }
        return desc;
    }
    unsigned char *status_host(size_t bytes) {
        if (bytes > hstatus_cap) {
            if (hstatus) (void)hipHostFree(hstatus);
            hstatus = nullptr;
            hstatus_cap = 0;
            HIPCHK(hipHostMalloc((void **)&hstatus, bytes, hipHostMallocDefault));
            hstatus_cap = bytes;
        }
        return hstatus;
    }
    ~Launcher() {
        if (stream) (void)hipStreamSynchronize(stream);
        if (hstatus) (void)hipHostFree(hstatus);
        pool.release();
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        if (k0) (void)hipEventDestroy(k0);
        if (k1) (void)hipEventDestroy(k1);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
};

}  // namespace fastlbp

using namespace fastlbp;

// A graph handle: shared structure and plan, and its own message state, evidence and stream.
struct fastlbp_graph {
    fastlbp_options opts;
    Alloc alloc;
    std::shared_ptr<Structure> S;
    std::shared_ptr<Plan> P;
    std::vector<int8_t> evidence;
    DevPool state;
    Belief *phi = nullptr, *bel = nullptr;
    void *msg = nullptr;
    RunState *st = nullptr;
    double *marg = nullptr;
    Launcher L;
    RunState *h_state = nullptr;  // pinned copy
    void *ev_buf = nullptr;       // staging for evidence updates (indices + potentials)
    size_t ev_cap = 0;
    // captured iterations of the LEVELS executor
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    int graph_iters = 0;
    double graph_damping = -1.0;
    bool graph_fused = false;
    const Plan *graph_plan = nullptr;
    fastlbp_run_stats last{};

    const HostGraph &hg() const { return S->hg; }
    int precision() const { return S->precision; }
    size_t state_bytes() const { return state.bytes; }
    void drop_graph() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        gexec = nullptr;
        graph = nullptr;
        graph_iters = 0;
        graph_plan = nullptr;
    }
    ~fastlbp_graph() {
        if (L.stream) (void)hipStreamSynchronize(L.stream);
        drop_graph();
        state.release();
        alloc.put(ev_buf);
        if (h_state) (void)hipHostFree(h_state);
    }
    template <class PP>
    DevGraph<typename PP::S, typename PP::V> view(double damping) const {
        DevGraph<typename PP::S, typename PP::V> g;
        g.num_vars = S->hg.V;
        g.num_edges = int32_t(S->hg.E);
        g.fac_off = S->fac_off;
        g.edge_var = S->edge_var;
        g.fac_type = S->fac_type;
        g.fpar = (const Pair<typename PP::V> *)S->fpar;
        g.epar = (const Pair<typename PP::V> *)S->epar;
        g.var_off = S->var_off;
        g.var_edge = S->var_edge;
        g.phi = phi;
        g.bel = bel;
        g.msg = (typename PP::S *)msg;
        g.edge_level = P->edge_level;
        g.term_off = S->term_off;
        g.term_w = (const typename PP::V *)S->term_w;
        g.term_base = S->term_base;
        g.term_ind = S->term_ind;
        g.term_mask = S->term_mask;
        g.damped = damping > 0.0 ? 1 : 0;
        if (precision() == FASTLBP_FP32) {
            g.damp_old = (typename PP::V)(damping > 0 ? std::log2(damping) : -INFINITY);
            g.damp_new = (typename PP::V)std::log2(1.0 - damping);
        } else {
            g.damp_old = (typename PP::V)damping;
            g.damp_new = (typename PP::V)(1.0 - damping);
        }
        return g;
    }
};

namespace fastlbp {

static int grid_for(int64_t items, int per_block) {
    int64_t b = (items + per_block - 1) / per_block;
    return int(std::max<int64_t>(1, std::min<int64_t>(b, 65535 * 8)));
}

// Grid of the factor kernels: at most 8 workgroups per compute unit (enough to reach their
// occupancy); the workgroups loop over the rest, which bounds the residual atomics per launch.
static int fac_grid(int64_t items, int per_block) { return std::min(grid_for(items, per_block), 256 * 8); }

// parameters in the value domain of the precision: (p, 1-p) as log2 (FP32) or linear (FP64)
template <class V>
static Pair<V> param_pair(double p, bool logd) {
    Pair<V> q;
    if (logd) {
        q.a = (V)(p > 0 ? std::log2(p) : -INFINITY);
        q.b = (V)(p < 1 ? std::log2(1.0 - p) : -INFINITY);
    } else {
        q.a = (V)p;
        q.b = (V)(1.0 - p);
    }
    return q;
}

template <class V>
static void upload_params(Structure &S, hipStream_t s, bool logd) {
    std::vector<Pair<V>> fp(std::max(S.hg.F, 1)), ep(std::max<int64_t>(S.hg.E, 1));
    for (int32_t a = 0; a < S.hg.F; ++a) fp[a] = param_pair<V>(S.hg.fac_param[a], logd);
    for (int64_t e = 0; e < S.hg.E; ++e) ep[e] = param_pair<V>(S.hg.edge_param[e], logd);
    S.fpar = S.pool.upload(fp, s);
    S.epar = S.pool.upload(ep, s);
    if (!S.hg.term_off.empty()) {
        std::vector<V> tw(S.hg.term_weight.size());
        for (size_t t = 0; t < tw.size(); ++t) {
            const double x = S.hg.term_weight[t];
            tw[t] = logd ? (V)(x > 0 ? std::log2(x) : -INFINITY) : (V)x;
        }
        S.term_w = S.pool.upload(tw, s);
    }
}

static std::shared_ptr<Plan> make_plan(const Structure &S, const Alloc &alloc, hipStream_t s, int kind,
                                       const int32_t *rank) {
    auto P = std::make_shared<Plan>();
    P->pool.alloc = alloc;
    P->kind = kind;
    std::vector<int32_t> level;
    int32_t n = analyze_levels(S.hg.V, S.hg.F, S.hg.fac_off.data(), S.hg.edge_var.data(),
                               kind == FASTLBP_SCHED_FLOODING ? nullptr : rank, level);
    P->hp.build(S.hg, level, n, kind == FASTLBP_SCHED_FLOODING, int(S.msg_bytes()), int(2 * S.val_bytes()));
    P->edge_level = P->pool.upload(P->hp.edge_exec_level, s);
    for (int b = 0; b < FB_COUNT; ++b) {
        P->fac_list[b] = P->pool.upload(P->hp.fac_list[b], s);
        P->fac_lvl_off[b] = P->pool.upload(P->hp.fac_lvl_off[b], s);
    }
    for (int b = 0; b < VB_COUNT; ++b) {
        P->var_list[b] = P->pool.upload(P->hp.var_list[b], s);
        P->var_lvl_off[b] = P->pool.upload(P->hp.var_lvl_off[b], s);
        P->init_var[b] = P->pool.upload(P->hp.init_var[b], s);
    }
    P->frec = P->pool.upload(P->hp.frec, s);
    P->vrec = P->pool.upload(P->hp.vrec, s);
    P->frec_off = P->pool.upload(P->hp.frec_off, s);
    P->vrec_off = P->pool.upload(P->hp.vrec_off, s);
    P->prec = P->pool.upload(P->hp.prec, s);
    P->level_lds = P->pool.upload(P->hp.level_lds, s);
    P->trec = P->pool.upload(P->hp.trec, s);
    P->trec_off = P->pool.upload(P->hp.trec_off, s);
    return P;
}

__global__ void k_phi_scatter(Belief *phi, const int32_t *idx, const Belief *val, int32_t n) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) phi[idx[i]] = val[i];
}

static Belief phi_of(const fastlbp_graph *g, int32_t v);
static void upload_phi(fastlbp_graph *g);

// Refreshes phi for the variables in `changed` (any order, repeats allowed): a small scatter when
// few change, the whole array otherwise. Evidence updates thus cost O(clamps), not O(V).
static void update_phi(fastlbp_graph *g, std::vector<int32_t> &changed) {
    std::sort(changed.begin(), changed.end());
    changed.erase(std::unique(changed.begin(), changed.end()), changed.end());
    const int32_t n = int32_t(changed.size());
    if (n == 0) return;
    if (int64_t(n) * 16 > g->hg().V) {
        upload_phi(g);
        return;
    }
    const size_t ib = (sizeof(int32_t) * size_t(n) + 15) & ~size_t(15);
    const size_t bytes = ib + sizeof(Belief) * size_t(n);
    if (bytes > g->ev_cap) {
        g->alloc.put(g->ev_buf);
        g->ev_buf = nullptr;
        g->ev_cap = 0;
        g->ev_buf = g->alloc.get(bytes);
        if (!g->ev_buf) throw OomError{};
        g->ev_cap = bytes;
    }
    std::vector<unsigned char> host(bytes);
    std::memcpy(host.data(), changed.data(), sizeof(int32_t) * size_t(n));
    Belief *hv = (Belief *)(host.data() + ib);
    for (int32_t i = 0; i < n; ++i) hv[i] = phi_of(g, changed[i]);
    HIPCHK(hipMemcpyAsync(g->ev_buf, host.data(), bytes, hipMemcpyHostToDevice, g->L.stream));
    k_phi_scatter<<<(n + 255) / 256, 256, 0, g->L.stream>>>(g->phi, (const int32_t *)g->ev_buf,
                                                            (const Belief *)((unsigned char *)g->ev_buf + ib), n);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(g->L.stream));  // `host` dies on return
}

static Belief phi_of(const fastlbp_graph *g, int32_t v) {
    const HostGraph &hg = g->hg();
    Belief b;
    b.fin = hg.prior_fin[v];
    b.npos = hg.prior_pos[v] + (g->evidence[v] == 1 ? 1 : 0);
    b.nneg = hg.prior_neg[v] + (g->evidence[v] == 0 ? 1 : 0);
    return b;
}

static void upload_phi(fastlbp_graph *g) {
    std::vector<Belief> phi(g->hg().V);
    for (int32_t v = 0; v < g->hg().V; ++v) phi[v] = phi_of(g, v);
    if (phi.empty()) return;
    HIPCHK(hipMemcpyAsync(g->phi, phi.data(), sizeof(Belief) * phi.size(), hipMemcpyHostToDevice, g->L.stream));
    HIPCHK(hipStreamSynchronize(g->L.stream));
}

// Allocates the handle's state (messages uniform, beliefs, phi from its evidence, run state).
static void alloc_state(fastlbp_graph *g) {
    const HostGraph &hg = g->hg();
    g->state.alloc = g->alloc;
    size_t mb = g->S->msg_bytes() * std::max<int64_t>(hg.E, 1);
    g->phi = (Belief *)g->state.get(sizeof(Belief) * std::max(hg.V, 1));
    g->bel = (Belief *)g->state.get(sizeof(Belief) * std::max(hg.V, 1));
    g->msg = g->state.get(mb);
    g->st = (RunState *)g->state.get(sizeof(RunState));
    g->marg = (double *)g->state.get(sizeof(double) * std::max(hg.V, 1));
    HIPCHK(hipMemsetAsync(g->msg, 0, mb, g->L.stream));
    HIPCHK(hipMemsetAsync(g->bel, 0, sizeof(Belief) * std::max(hg.V, 1), g->L.stream));
    HIPCHK(hipMemsetAsync(g->st, 0, sizeof(RunState), g->L.stream));
    upload_phi(g);
}

// Recompute every belief from phi and the current messages.
template <class PP>
static void launch_init_beliefs(fastlbp_graph *g, const DevGraph<typename PP::S, typename PP::V> &dg) {
    const HostPlan &hp = g->P->hp;
    int32_t n0 = int32_t(hp.init_var[VB_THREAD].size()), n1 = int32_t(hp.init_var[VB_WAVE].size());
    if (n0) k_var_thread<PP><<<grid_for(n0, 256), 256, 0, g->L.stream>>>(dg, g->P->init_var[VB_THREAD], n0, nullptr);
    if (n1) k_var_wave<PP><<<grid_for(n1, 4), 256, 0, g->L.stream>>>(dg, g->P->init_var[VB_WAVE], n1, nullptr);
    HIPCHK(hipGetLastError());
}

static int persistent_threads(int precision, bool teams, int runs);

// One launch of k_levels_fused for levels [L0, L1).
template <class PP, bool DAMP>
static void launch_fused(fastlbp_graph *g, const DevGraph<typename PP::S, typename PP::V> &dg, const DevPlan &dp,
                         int32_t L0, int32_t L1, bool teams, hipStream_t s) {
    const int32_t cap = g->P->hp.stage_slots;
    const size_t lds = stage_bytes<typename PP::S>(std::max(cap, 1));
    const int nt = persistent_threads(g->precision(), teams, 1);
    if constexpr (std::is_same<PP, PolLog32>::value) {
        if (nt == 1024) {
            k_levels_fused<PP, DAMP, false, 1024><<<1, 1024, lds, s>>>(dg, dp, g->st, L0, L1, cap);
            return;
        }
    }
    if (teams)
        k_levels_fused<PP, DAMP, true, 512><<<1, 512, lds, s>>>(dg, dp, g->st, L0, L1, cap);
    else
        k_levels_fused<PP, DAMP, false, 512><<<1, 512, lds, s>>>(dg, dp, g->st, L0, L1, cap);
}

// One iteration of the LEVELS executor: for every level, the factor phase then the variable phase.
// fuse (HYBRID executor): each run of narrow levels goes to one single-workgroup launch.
template <class PP, bool ALL, bool DAMP>
static void enqueue_iteration(fastlbp_graph *g, const DevGraph<typename PP::S, typename PP::V> &dg, bool fuse) {
    const HostPlan &pl = g->P->hp;
    const Plan &P = *g->P;
    hipStream_t s = g->L.stream;
    const DevPlan dp = P.view();
    for (int32_t L = 0; L < pl.exec_levels; ++L) {
        if (fuse && pl.seg_end[L] > L) {
            launch_fused<PP, DAMP>(g, dg, dp, L, pl.seg_end[L], pl.seg_teams[L] != 0, s);
            L = pl.seg_end[L] - 1;
            continue;
        }
        int32_t o, n;
        o = pl.frec_off[L];
        n = pl.frec_off[L + 1] - o;
        if (n) k_fac_rec<PP, DAMP><<<fac_grid(n, 256), 256, 0, s>>>(dg, (const FacRec *)P.frec + o, n, g->st);
        o = pl.fac_lvl_off[FB_WAVE][L];
        n = pl.fac_lvl_off[FB_WAVE][L + 1] - o;
        if (n) k_fac_wave<PP, ALL, DAMP><<<fac_grid(n, 4), 256, 0, s>>>(dg, P.fac_list[FB_WAVE] + o, n, L, g->st);
        o = pl.fac_lvl_off[FB_TERMS_WAVE][L];
        n = pl.fac_lvl_off[FB_TERMS_WAVE][L + 1] - o;
        if (n) k_fac_terms<PP, ALL, DAMP><<<fac_grid(n, 4), 256, 0, s>>>(dg, P.fac_list[FB_TERMS_WAVE] + o, n, L, g->st);
        o = pl.trec_off[L];
        n = pl.trec_off[L + 1] - o;
        if (n) k_fac_terms_rec<PP, DAMP><<<fac_grid(n, 256), 256, 0, s>>>(dg, (const TermRec *)P.trec + o, n, g->st);
        o = pl.fac_lvl_off[FB_BLOCK][L];
        n = pl.fac_lvl_off[FB_BLOCK][L + 1] - o;
        if (n)
            k_fac_block<PP, ALL, DAMP, block_threads<PP>()><<<std::min(n, 4096), block_threads<PP>(), 0, s>>>(
                dg, P.fac_list[FB_BLOCK] + o, n, L, g->st);
        o = pl.vrec_off[L];
        n = pl.vrec_off[L + 1] - o;
        if (n) k_var_rec<PP><<<grid_for(n, 256), 256, 0, s>>>(dg, (const VarRec *)P.vrec + o, n, g->st);
        o = pl.var_lvl_off[VB_WAVE][L];
        n = pl.var_lvl_off[VB_WAVE][L + 1] - o;
        if (n) k_var_wave<PP><<<grid_for(n, 4), 256, 0, s>>>(dg, P.var_list[VB_WAVE] + o, n, g->st);
    }
    k_finalize<<<1, 64, 0, s>>>(g->st);
}

// Workgroup size of the persistent executor. 512 threads in general (float64 factor code and the
// team paths need more than the 128 registers a 1024-thread workgroup allows). A launch of at most
// as many runs as compute units, all float32 with thread tasks only, takes 1024 threads: each run
// has a compute unit to itself, and levels of up to 1024 tasks finish in one pass. With more runs,
// two 512-thread workgroups share a compute unit, so twice as many runs are in flight.
static int persistent_threads(int precision, bool teams, int runs) {
    return (precision == FASTLBP_FP32 && !teams && runs <= 256) ? 1024 : 512;
}

static int choose_executor(const fastlbp_graph *g) {
    int ex = g->opts.executor;
    if (ex != FASTLBP_EXEC_AUTO) return ex;
    // one workgroup keeps up with a level of a few thousand edges; wider levels need the GPU.
    // A plan with a few wide levels among many narrow ones runs the narrow ones fused.
    const HostPlan &hp = g->P->hp;
    const bool small = g->hg().nonprior_edges <= (int64_t(4) << 20);
    if (small && hp.fused_levels == hp.exec_levels) return FASTLBP_EXEC_PERSISTENT;  // every level narrow
    if (hp.fused_levels >= 4 && hp.launches_hybrid * 2 <= hp.launches_levels) return FASTLBP_EXEC_HYBRID;
    if (small && hp.max_level_edges <= 8192) return FASTLBP_EXEC_PERSISTENT;
    return FASTLBP_EXEC_LEVELS;
}

// The handle's hipGraph of K captured iterations, re-captured when K, damping or the plan changed.
template <class PP, bool ALL, bool DAMP>
static void ensure_iteration_graph(fastlbp_graph *g, const DevGraph<typename PP::S, typename PP::V> &dg, int K,
                                   double damping, bool fuse) {
    if (g->gexec && g->graph_iters == K && g->graph_damping == damping && g->graph_plan == g->P.get() &&
        g->graph_fused == fuse)
        return;
    g->drop_graph();
    hipStream_t s = g->L.stream;
    HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < K; ++k) enqueue_iteration<PP, ALL, DAMP>(g, dg, fuse);
    HIPCHK(hipStreamEndCapture(s, &g->graph));
    HIPCHK(hipGraphInstantiate(&g->gexec, g->graph, nullptr, nullptr, 0));
    g->graph_iters = K;
    g->graph_damping = damping;
    g->graph_plan = g->P.get();
    g->graph_fused = fuse;
}

template <class PP, bool ALL, bool DAMP>
static void run_levels(fastlbp_graph *g, int32_t max_iters, double tol, double damping, bool fuse) {
    auto dg = g->view<PP>(damping);
    hipStream_t s = g->L.stream;
    k_run_init<<<1, 64, 0, s>>>(g->st, max_iters, tol);
    HIPCHK(hipGetLastError());
    launch_init_beliefs<PP>(g, dg);
    if (max_iters <= 0) return;
    // iterations per replay: enough to amortise the launch, few enough to stop soon after
    // convergence (kernels of finished iterations return at once)
    int per_iter_kernels = std::max(1, fuse ? g->P->hp.launches_hybrid : g->P->hp.launches_levels);
    int K = std::max(1, std::min(32, 2048 / per_iter_kernels));
    K = std::min(K, max_iters);
    bool use_graph = g->opts.use_graph != 0;
    if (use_graph) ensure_iteration_graph<PP, ALL, DAMP>(g, dg, K, damping, fuse);
    int done_iters = 0;
    while (true) {
        if (use_graph)
            HIPCHK(hipGraphLaunch(g->gexec, s));
        else
            for (int k = 0; k < K; ++k) enqueue_iteration<PP, ALL, DAMP>(g, dg, fuse);
        HIPCHK(hipGetLastError());
        done_iters += K;
        if (done_iters >= max_iters) break;
        HIPCHK(hipMemcpyAsync(g->h_state, g->st, kRunStateHeader, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (g->h_state->done) break;
    }
}

// One persistent launch over n runs (one workgroup each) on `lc`'s stream. Every run advances
// until it is done or its iteration count reaches its step_end (with step > 0, first set to
// step iterations past the current count). On return every run's host state header is current.
template <class PP>
static void launch_persistent(Launcher &lc, int n, fastlbp_graph *const *gs, const double *damping,
                              int32_t step = 0) {
    if (n <= 0) return;
    bool teams = false, damp = false;
    for (int i = 0; i < n; ++i) {
        teams = teams || gs[i]->P->teams();
        damp = damp || damping[i] > 0.0;
    }
    const size_t dbytes = sizeof(RunDesc<PP>) * size_t(n);
    const size_t sbytes = kRunStateHeader * size_t(n);
    const size_t bytes = dbytes + sbytes;
    void *d = lc.descs(bytes);
    int32_t *dstatus = (int32_t *)((unsigned char *)d + dbytes);
    lc.hdesc.resize(dbytes);
    RunDesc<PP> *h = (RunDesc<PP> *)lc.hdesc.data();
    for (int i = 0; i < n; ++i) {
        h[i].g = gs[i]->view<PP>(damping[i]);
        h[i].plan = gs[i]->P->view();
        h[i].st = GPtr<RunState>(gs[i]->st);
        h[i].status = GPtr<int32_t>(dstatus + i * int(kRunStateHeader / 4));
        h[i].step = step;
    }
    unsigned char *hs = lc.status_host(sbytes);
    HIPCHK(hipMemcpyAsync(d, h, dbytes, hipMemcpyHostToDevice, lc.stream));
    const RunDesc<PP> *dd = (const RunDesc<PP> *)d;
    int nt = persistent_threads(gs[0]->precision(), teams, n);
    hipStream_t s = lc.stream;
    // dynamic LDS: staging slots for the largest staged level in the launch, then per-level
    // offsets and flags of the deepest schedule (up to 4096 levels; deeper schedules read them
    // from memory). Kept within 64 KiB so two 512-thread workgroups fit a compute unit.
    int32_t max_levels = 0, stage_cap = 0;
    for (int i = 0; i < n; ++i) {
        max_levels = std::max(max_levels, gs[i]->P->hp.exec_levels);
        stage_cap = std::max(stage_cap, gs[i]->P->hp.stage_slots);
    }
    const size_t slot_bytes = stage_bytes<typename PP::S>(stage_cap);
    int32_t lds_levels = std::min<int32_t>(max_levels, 4095);
    if (slot_bytes + sizeof(int32_t) * 3 * size_t(lds_levels + 1) > (size_t(64) << 10)) lds_levels = 0;
    const size_t lds_bytes = slot_bytes + sizeof(int32_t) * 3 * size_t(lds_levels + 1);
    HIPCHK(hipEventRecord(lc.k0, s));
    const bool offl = max_levels <= lds_levels;
#define FASTLBP_LAUNCH(DA, TE, NT_)                                                        \
    do {                                                                                   \
        if (offl)                                                                          \
            k_persistent<PP, DA, TE, NT_, true><<<n, NT_, lds_bytes, s>>>(dd, lds_levels, stage_cap);  \
        else                                                                               \
            k_persistent<PP, DA, TE, NT_, false><<<n, NT_, lds_bytes, s>>>(dd, lds_levels, stage_cap); \
    } while (0)
    bool launched = false;
    if constexpr (std::is_same<PP, PolLog32>::value) {
        if (nt == 1024) {
            if (damp) FASTLBP_LAUNCH(true, false, 1024);
            else FASTLBP_LAUNCH(false, false, 1024);
            launched = true;
        }
    }
    if (!launched) {
        if (damp && teams) FASTLBP_LAUNCH(true, true, 512);
        else if (damp) FASTLBP_LAUNCH(true, false, 512);
        else if (teams) FASTLBP_LAUNCH(false, true, 512);
        else FASTLBP_LAUNCH(false, false, 512);
    }
#undef FASTLBP_LAUNCH
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(lc.k1, s));
    HIPCHK(hipMemcpyAsync(hs, dstatus, sbytes, hipMemcpyDeviceToHost, s));
    // (the descriptor staging buffer may be rewritten by the next call only after this)
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipEventElapsedTime(&lc.last_kernel_ms, lc.k0, lc.k1));
    for (int i = 0; i < n; ++i) std::memcpy(gs[i]->h_state, hs + kRunStateHeader * size_t(i), kRunStateHeader);
}

__global__ void k_run_init_step(RunState *st, int32_t max_iters, double tol, int32_t step) {
    clear_slots(st);
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->contra = 0ull;
        st->iter = 0;
        st->done = max_iters <= 0 ? 1 : 0;
        st->last_r = 0.0;
        st->max_iters = max_iters;
        st->converged = 0;
        st->tol = tol;
        st->step_end = step;
    }
}

template <class PP, bool ALL, bool DAMP>
static void run_single(fastlbp_graph *g, int32_t max_iters, double tol, double damping, int exec) {
    if (exec == FASTLBP_EXEC_LEVELS || exec == FASTLBP_EXEC_HYBRID) {
        run_levels<PP, ALL, DAMP>(g, max_iters, tol, damping, exec == FASTLBP_EXEC_HYBRID);
        return;
    }
    k_run_init_step<<<1, 64, 0, g->L.stream>>>(g->st, max_iters, tol, max_iters);
    HIPCHK(hipGetLastError());
    fastlbp_graph *one[1] = {g};
    launch_persistent<PP>(g->L, 1, one, &damping);
}

template <class PP>
static void run_dispatch(fastlbp_graph *g, int32_t max_iters, double tol, double damping, int exec) {
    bool all = g->P->hp.all_active != 0, damp = damping > 0.0;
    if (all && damp) run_single<PP, true, true>(g, max_iters, tol, damping, exec);
    if (all && !damp) run_single<PP, true, false>(g, max_iters, tol, damping, exec);
    if (!all && damp) run_single<PP, false, true>(g, max_iters, tol, damping, exec);
    if (!all && !damp) run_single<PP, false, false>(g, max_iters, tol, damping, exec);
}

static int device_error(const DeviceError &e) {
    set_error(e.msg);
    return FASTLBP_E_DEVICE;
}

static void fill_stats(fastlbp_graph *g, int exec, float ms, fastlbp_run_stats &s) {
    s = fastlbp_run_stats{};
    s.iterations = g->h_state->iter;
    s.converged = g->h_state->converged;
    s.residual = g->h_state->last_r;
    s.contradictions = (int64_t)g->h_state->contra;
    s.levels = g->P->hp.num_levels;
    s.executor = exec;
    s.algorithmic_bytes_per_iter = g->P->hp.bytes_per_iter;
    s.device_ms = ms;
    s.message_updates = g->P->hp.updates_per_iter * int64_t(s.iterations);
    g->last = s;
}

// ---- used by the server ----------------------------------------------------------------------

void step_begin(fastlbp_graph *g, int32_t max_iters, double tol, int32_t step) {
    k_run_init_step<<<1, 64, 0, g->L.stream>>>(g->st, max_iters, tol, step);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(g->L.stream));
}

void step_run(Launcher &lc, int n, fastlbp_graph *const *gs, const double *damping, int32_t step) {
    if (gs[0]->precision() == FASTLBP_FP32)
        launch_persistent<PolLog32>(lc, n, gs, damping, step);
    else
        launch_persistent<PolLin64>(lc, n, gs, damping, step);
}

// A server step of a run on the LEVELS executor: beliefs rebuilt (the evidence may be new), then
// `iters` iterations on the handle's own stream, so the step overlaps the persistent launch of the
// narrow runs. Iterations after the run is done return at once.
template <class PP, bool ALL, bool DAMP>
static void step_levels_t(fastlbp_graph *g, double damping, int32_t iters) {
    auto dg = g->view<PP>(damping);
    hipStream_t s = g->L.stream;
    HIPCHK(hipEventRecord(g->L.k0, s));
    launch_init_beliefs<PP>(g, dg);
    const bool fuse = choose_executor(g) == FASTLBP_EXEC_HYBRID;
    if (g->opts.use_graph) {
        ensure_iteration_graph<PP, ALL, DAMP>(g, dg, iters, damping, fuse);
        HIPCHK(hipGraphLaunch(g->gexec, s));
    } else {
        for (int k = 0; k < iters; ++k) enqueue_iteration<PP, ALL, DAMP>(g, dg, fuse);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(g->L.k1, s));
}

template <class PP>
static void step_levels_p(fastlbp_graph *g, double damping, int32_t iters) {
    bool all = g->P->hp.all_active != 0, damp = damping > 0.0;
    if (all && damp) step_levels_t<PP, true, true>(g, damping, iters);
    if (all && !damp) step_levels_t<PP, true, false>(g, damping, iters);
    if (!all && damp) step_levels_t<PP, false, true>(g, damping, iters);
    if (!all && !damp) step_levels_t<PP, false, false>(g, damping, iters);
}

bool graph_wide(fastlbp_graph *g) { return choose_executor(g) != FASTLBP_EXEC_PERSISTENT; }

void step_levels_enqueue(fastlbp_graph *g, double damping, int32_t iters) {
    if (g->precision() == FASTLBP_FP32)
        step_levels_p<PolLog32>(g, damping, iters);
    else
        step_levels_p<PolLin64>(g, damping, iters);
}

float step_levels_finish(fastlbp_graph *g) {
    HIPCHK(hipStreamSynchronize(g->L.stream));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, g->L.k0, g->L.k1));
    return ms;
}

void read_state(fastlbp_graph *g, hipStream_t s) {
    HIPCHK(hipMemcpyAsync(g->h_state, g->st, kRunStateHeader, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
}

void refresh_beliefs(fastlbp_graph *g) {
    if (g->hg().V == 0) return;
    if (g->precision() == FASTLBP_FP32)
        launch_init_beliefs<PolLog32>(g, g->view<PolLog32>(0.0));
    else
        launch_init_beliefs<PolLin64>(g, g->view<PolLin64>(0.0));
}

void marginals_into(fastlbp_graph *g, double *p1) {
    if (g->hg().V == 0) return;
    refresh_beliefs(g);
    k_marginals<<<grid_for(g->hg().V, 256), 256, 0, g->L.stream>>>(g->bel, g->hg().V, g->marg);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(p1, g->marg, sizeof(double) * g->hg().V, hipMemcpyDeviceToHost, g->L.stream));
    HIPCHK(hipStreamSynchronize(g->L.stream));
}

void fill_stats_public(fastlbp_graph *g, fastlbp_run_stats &s, float ms) { fill_stats(g, choose_executor(g), ms, s); }

int set_evidence(fastlbp_graph *g, int32_t n, const int32_t *vars, const int8_t *values) {
    for (int32_t i = 0; i < n; ++i)
        if (vars[i] < 0 || vars[i] >= g->hg().V || values[i] < -1 || values[i] > 1) {
            set_error("evidence entry " + std::to_string(i) + " out of range");
            return FASTLBP_E_INVALID_ARG;
        }
    std::vector<int32_t> changed;
    std::vector<int8_t> before;
    for (int32_t i = 0; i < n; ++i)
        if (g->evidence[vars[i]] != values[i]) {
            changed.push_back(vars[i]);
            before.push_back(g->evidence[vars[i]]);
            g->evidence[vars[i]] = values[i];
        }
    try {
        update_phi(g, changed);
    } catch (...) {  // leave the handle's evidence as it was
        for (size_t i = changed.size(); i-- > 0;) g->evidence[changed[i]] = before[i];
        throw;
    }
    return FASTLBP_OK;
}

Launcher *launcher_create(int device, hipStream_t s, const Alloc &a) {
    HIPCHK(hipSetDevice(device));
    auto *l = new Launcher();
    l->init(s, a);
    return l;
}
void launcher_destroy(Launcher *l) { delete l; }
hipStream_t launcher_stream(Launcher *l) { return l->stream; }
float launcher_kernel_ms(Launcher *l) { return l->last_kernel_ms; }
int graph_device(fastlbp_graph *g) { return g->opts.device; }
int graph_precision(fastlbp_graph *g) { return g->precision(); }
size_t graph_state_bytes(fastlbp_graph *g) { return g->state_bytes(); }
int32_t graph_num_vars(fastlbp_graph *g) { return g->hg().V; }
const RunState &graph_host_state(fastlbp_graph *g) { return *g->h_state; }
void graph_sync(fastlbp_graph *g) { HIPCHK(hipStreamSynchronize(g->L.stream)); }
hipStream_t graph_stream(fastlbp_graph *g) { return g->L.stream; }
const Belief *graph_beliefs(fastlbp_graph *g) { return g->bel; }
const Alloc &graph_alloc(fastlbp_graph *g) { return g->alloc; }

}  // namespace fastlbp

// ------------------------------------------------------------------------------------------------
// C ABI
// ------------------------------------------------------------------------------------------------

extern "C" {

void fastlbp_options_default(fastlbp_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->precision = FASTLBP_FP64;
    o->device = 0;
    o->stream = nullptr;
    o->executor = FASTLBP_EXEC_AUTO;
    o->use_graph = 1;
}

const char *fastlbp_version(void) { return "fastlbp-mi355x 0.2 (gfx950)"; }

static int check_options(const fastlbp_options &o) {
    if (o.precision != FASTLBP_FP64 && o.precision != FASTLBP_FP32) {
        set_error("precision must be FASTLBP_FP64 or FASTLBP_FP32");
        return FASTLBP_E_INVALID_ARG;
    }
    if (o.executor < FASTLBP_EXEC_AUTO || o.executor > FASTLBP_EXEC_HYBRID) {
        set_error("unknown executor");
        return FASTLBP_E_INVALID_ARG;
    }
    if ((o.alloc == nullptr) != (o.free == nullptr)) {
        set_error("alloc and free must be given together");
        return FASTLBP_E_INVALID_ARG;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        set_error("no HIP device");
        return FASTLBP_E_DEVICE;
    }
    if (o.device < 0 || o.device >= ndev) {
        set_error("device ordinal out of range");
        return FASTLBP_E_INVALID_ARG;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, o.device) != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipGetDeviceProperties failed");
        return FASTLBP_E_DEVICE;
    }
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        set_error(std::string("device is ") + prop.gcnArchName + ", library is built for gfx950");
        return FASTLBP_E_DEVICE;
    }
    return FASTLBP_OK;
}

// Common tail of create and clone: launcher, pinned state, device state.
static int finish_handle(fastlbp_graph *g) {
    HIPCHK(hipSetDevice(g->opts.device));
    g->L.init((hipStream_t)g->opts.stream, g->alloc);
    HIPCHK(hipHostMalloc((void **)&g->h_state, sizeof(RunState), hipHostMallocDefault));
    alloc_state(g);
    return FASTLBP_OK;
}

int fastlbp_graph_create(int32_t num_vars, int32_t num_factors, const int64_t *factor_offsets,
                         const int32_t *edge_vars, const uint8_t *factor_types, const double *factor_params,
                         const double *edge_params, const fastlbp_options *opts, fastlbp_graph_t *out) {
    return fastlbp_graph_create_terms(num_vars, num_factors, factor_offsets, edge_vars, factor_types, factor_params,
                                      edge_params, nullptr, nullptr, nullptr, opts, out);
}

int fastlbp_graph_create_terms(int32_t num_vars, int32_t num_factors, const int64_t *factor_offsets,
                               const int32_t *edge_vars, const uint8_t *factor_types, const double *factor_params,
                               const double *edge_params, const int64_t *term_offsets, const double *term_weights,
                               const int8_t *term_indicators, const fastlbp_options *opts, fastlbp_graph_t *out) {
    clear_error();
    if (!out) {
        set_error("out is NULL");
        return FASTLBP_E_INVALID_ARG;
    }
    *out = nullptr;
    int rc = validate_graph(num_vars, num_factors, factor_offsets, edge_vars, factor_types, factor_params, edge_params,
                            term_offsets, term_weights, term_indicators);
    if (rc) return rc;
    fastlbp_options o;
    fastlbp_options_default(&o);
    if (opts) o = *opts;
    rc = check_options(o);
    if (rc) return rc;
    std::unique_ptr<fastlbp_graph> g(new fastlbp_graph());
    g->opts = o;
    g->alloc.fn_alloc = o.alloc;
    g->alloc.fn_free = o.free;
    g->alloc.ctx = o.alloc_ctx;
    try {
        HIPCHK(hipSetDevice(o.device));
        g->L.init((hipStream_t)o.stream, g->alloc);
        hipStream_t s = g->L.stream;
        auto S = std::make_shared<Structure>();
        S->device = o.device;
        S->precision = o.precision;
        S->pool.alloc = g->alloc;
        S->hg.build(num_vars, num_factors, factor_offsets, edge_vars, factor_types, factor_params, edge_params);
        S->hg.set_terms(term_offsets, term_weights, term_indicators);
        const HostGraph &hg = S->hg;
        std::vector<int32_t> off32(hg.fac_off.begin(), hg.fac_off.end());
        S->fac_off = S->pool.upload(off32, s);
        S->edge_var = S->pool.upload(hg.edge_var, s);
        S->fac_type = S->pool.upload(hg.fac_type, s);
        S->var_off = S->pool.upload(hg.var_off, s);
        S->var_edge = S->pool.upload(hg.var_edge, s);
        if (!hg.term_off.empty()) {
            S->term_off = S->pool.upload(hg.term_off, s);
            S->term_base = S->pool.upload(hg.term_base, s);
            S->term_ind = S->pool.upload(hg.term_ind, s);
            S->term_mask = S->pool.upload(hg.term_mask, s);
        }
        if (o.precision == FASTLBP_FP32)
            upload_params<float>(*S, s, true);
        else
            upload_params<double>(*S, s, false);
        g->S = S;
        g->P = make_plan(*S, g->alloc, s, FASTLBP_SCHED_FLOODING, nullptr);
        g->evidence.assign(hg.V, -1);
        HIPCHK(hipHostMalloc((void **)&g->h_state, sizeof(RunState), hipHostMallocDefault));
        alloc_state(g.get());
    } catch (OomError &) {
        set_error("device allocation failed");
        return FASTLBP_E_OOM;
    } catch (DeviceError &e) {
        return device_error(e);
    } catch (std::bad_alloc &) {
        set_error("host allocation failed");
        return FASTLBP_E_OOM;
    }
    *out = g.release();
    return FASTLBP_OK;
}

int fastlbp_graph_clone(fastlbp_graph_t src, fastlbp_graph_t *out) {
    clear_error();
    if (!src || !out) {
        set_error("invalid argument");
        return FASTLBP_E_INVALID_ARG;
    }
    *out = nullptr;
    std::unique_ptr<fastlbp_graph> g(new fastlbp_graph());
    g->opts = src->opts;
    g->opts.stream = nullptr;  // every handle gets its own stream
    g->alloc = src->alloc;
    g->S = src->S;
    g->P = src->P;
    g->evidence.assign(src->hg().V, -1);
    try {
        finish_handle(g.get());
    } catch (OomError &) {
        set_error("device allocation failed");
        return FASTLBP_E_OOM;
    } catch (DeviceError &e) {
        return device_error(e);
    }
    *out = g.release();
    return FASTLBP_OK;
}

void fastlbp_graph_destroy(fastlbp_graph_t g) { delete g; }

int fastlbp_schedule_set(fastlbp_graph_t g, int32_t kind, const int32_t *edge_rank, int32_t *num_levels_out) {
    clear_error();
    if (!g) {
        set_error("graph is NULL");
        return FASTLBP_E_INVALID_ARG;
    }
    if (kind != FASTLBP_SCHED_FLOODING && kind != FASTLBP_SCHED_RANKED) {
        set_error("unknown schedule kind");
        return FASTLBP_E_INVALID_ARG;
    }
    if (kind == FASTLBP_SCHED_RANKED && !edge_rank && g->hg().E > 0) {
        set_error("RANKED needs edge_rank");
        return FASTLBP_E_BAD_SCHEDULE;
    }
    try {
        HIPCHK(hipSetDevice(g->opts.device));
        HIPCHK(hipStreamSynchronize(g->L.stream));
        auto P = make_plan(*g->S, g->alloc, g->L.stream, kind, edge_rank);
        g->drop_graph();
        g->P = P;  // other handles sharing the old plan keep it
    } catch (OomError &) {
        set_error("device allocation failed");
        return FASTLBP_E_OOM;
    } catch (DeviceError &e) {
        return device_error(e);
    }
    if (num_levels_out) *num_levels_out = g->P->hp.num_levels;
    return FASTLBP_OK;
}

int fastlbp_schedule_set_classes(fastlbp_graph_t g, int32_t num_classes, const int32_t *edge_class, int32_t num_arcs,
                                 const int32_t *arcs, int32_t *num_levels_out) {
    clear_error();
    if (!g) {
        set_error("graph is NULL");
        return FASTLBP_E_INVALID_ARG;
    }
    std::vector<int32_t> rank;
    const HostGraph &hg = g->hg();
    int rc = classes_to_ranks(hg.V, hg.F, hg.fac_off.data(), hg.edge_var.data(), hg.fac_type.data(), num_classes,
                              edge_class, num_arcs, arcs, rank);
    if (rc) return rc;
    return fastlbp_schedule_set(g, FASTLBP_SCHED_RANKED, rank.data(), num_levels_out);
}

int fastlbp_schedule_levels(fastlbp_graph_t g, int32_t *level_of_edge) {
    clear_error();
    if (!g || (!level_of_edge && g->hg().E > 0)) {
        set_error("invalid argument");
        return FASTLBP_E_INVALID_ARG;
    }
    if (g->hg().E) std::memcpy(level_of_edge, g->P->hp.level_of_edge.data(), sizeof(int32_t) * g->hg().E);
    return FASTLBP_OK;
}

int fastlbp_evidence_set(fastlbp_graph_t g, int32_t n, const int32_t *vars, const int8_t *values) {
    clear_error();
    if (!g || n < 0 || (n > 0 && (!vars || !values))) {
        set_error("invalid argument");
        return FASTLBP_E_INVALID_ARG;
    }
    try {
        return set_evidence(g, n, vars, values);
    } catch (OomError &) {
        set_error("device allocation failed");
        return FASTLBP_E_OOM;
    } catch (DeviceError &e) {
        return device_error(e);
    }
}

int fastlbp_evidence_clear(fastlbp_graph_t g) {
    clear_error();
    if (!g) {
        set_error("graph is NULL");
        return FASTLBP_E_INVALID_ARG;
    }
    std::vector<int8_t> saved = g->evidence;
    try {
        std::vector<int32_t> changed;
        for (int32_t v = 0; v < int32_t(g->evidence.size()); ++v)
            if (g->evidence[v] != -1) {
                g->evidence[v] = -1;
                changed.push_back(v);
            }
        update_phi(g, changed);
    } catch (OomError &) {
        g->evidence = saved;
        set_error("device allocation failed");
        return FASTLBP_E_OOM;
    } catch (DeviceError &e) {
        g->evidence = saved;
        return device_error(e);
    }
    return FASTLBP_OK;
}

static int check_run_args(int32_t max_iters, double tol, double damping) {
    if (max_iters < 0 || !(tol >= 0.0) || !(damping >= 0.0 && damping < 1.0)) {
        set_error("need max_iters >= 0, tol >= 0, 0 <= damping < 1");
        return FASTLBP_E_INVALID_ARG;
    }
    return FASTLBP_OK;
}

int fastlbp_run(fastlbp_graph_t g, int32_t max_iters, double tol, double damping, fastlbp_run_stats *stats) {
    clear_error();
    if (!g) {
        set_error("graph is NULL");
        return FASTLBP_E_INVALID_ARG;
    }
    int rc = check_run_args(max_iters, tol, damping);
    if (rc) return rc;
    int exec = choose_executor(g);
    try {
        HIPCHK(hipSetDevice(g->opts.device));
        hipStream_t s = g->L.stream;
        HIPCHK(hipEventRecord(g->L.ev0, s));
        if (g->precision() == FASTLBP_FP32)
            run_dispatch<PolLog32>(g, max_iters, tol, damping, exec);
        else
            run_dispatch<PolLin64>(g, max_iters, tol, damping, exec);
        HIPCHK(hipEventRecord(g->L.ev1, s));
        HIPCHK(hipMemcpyAsync(g->h_state, g->st, kRunStateHeader, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, g->L.ev0, g->L.ev1));
        fastlbp_run_stats st;
        fill_stats(g, exec, ms, st);
        if (stats) *stats = st;
    } catch (OomError &) {
        set_error("device allocation failed");
        return FASTLBP_E_OOM;
    } catch (DeviceError &e) {
        return device_error(e);
    }
    return FASTLBP_OK;
}

int fastlbp_run_batch(int32_t n, fastlbp_graph_t *graphs, int32_t max_iters, double tol, double damping,
                      fastlbp_run_stats *stats) {
    clear_error();
    if (n < 0 || (n > 0 && !graphs)) {
        set_error("invalid argument");
        return FASTLBP_E_INVALID_ARG;
    }
    if (n == 0) return FASTLBP_OK;
    int rc = check_run_args(max_iters, tol, damping);
    if (rc) return rc;
    for (int32_t i = 0; i < n; ++i) {
        if (!graphs[i]) {
            set_error("graph is NULL");
            return FASTLBP_E_INVALID_ARG;
        }
        if (graphs[i]->precision() != graphs[0]->precision() || graphs[i]->opts.device != graphs[0]->opts.device) {
            set_error("a batch needs one precision and one device");
            return FASTLBP_E_INVALID_ARG;
        }
        for (int32_t j = 0; j < i; ++j)
            if (graphs[j] == graphs[i]) {
                set_error("a handle appears twice in the batch");
                return FASTLBP_E_INVALID_ARG;
            }
    }
    fastlbp_graph *g0 = graphs[0];
    try {
        HIPCHK(hipSetDevice(g0->opts.device));
        for (int32_t i = 0; i < n; ++i) HIPCHK(hipStreamSynchronize(graphs[i]->L.stream));
        hipStream_t s = g0->L.stream;
        for (int32_t i = 0; i < n; ++i) k_run_init_step<<<1, 64, 0, s>>>(graphs[i]->st, max_iters, tol, max_iters);
        HIPCHK(hipGetLastError());
        HIPCHK(hipEventRecord(g0->L.ev0, s));
        std::vector<double> damps(n, damping);
        if (g0->precision() == FASTLBP_FP32)
            launch_persistent<PolLog32>(g0->L, n, graphs, damps.data());
        else
            launch_persistent<PolLin64>(g0->L, n, graphs, damps.data());
        HIPCHK(hipEventRecord(g0->L.ev1, s));
        HIPCHK(hipStreamSynchronize(s));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, g0->L.ev0, g0->L.ev1));
        for (int32_t i = 0; i < n; ++i) {  // host state headers were refreshed by the launch
            fastlbp_run_stats st;
            fill_stats(graphs[i], FASTLBP_EXEC_PERSISTENT, ms, st);
            if (stats) stats[i] = st;
        }
    } catch (OomError &) {
        set_error("device allocation failed");
        return FASTLBP_E_OOM;
    } catch (DeviceError &e) {
        return device_error(e);
    }
    return FASTLBP_OK;
}

int fastlbp_marginals(fastlbp_graph_t g, double *p1) {
    clear_error();
    if (!g || (!p1 && g->hg().V > 0)) {
        set_error("invalid argument");
        return FASTLBP_E_INVALID_ARG;
    }
    try {
        HIPCHK(hipSetDevice(g->opts.device));
        marginals_into(g, p1);
    } catch (DeviceError &e) {
        return device_error(e);
    }
    return FASTLBP_OK;
}

int fastlbp_messages_get(fastlbp_graph_t g, double *f2v_p1) {
    clear_error();
    if (!g || (!f2v_p1 && g->hg().E > 0)) {
        set_error("invalid argument");
        return FASTLBP_E_INVALID_ARG;
    }
    const HostGraph &hg = g->hg();
    int64_t E = hg.E;
    if (!E) return FASTLBP_OK;
    try {
        std::vector<double> l(E);
        hipStream_t s = g->L.stream;
        if (g->precision() == FASTLBP_FP32) {
            std::vector<float> f(E);
            HIPCHK(hipMemcpyAsync(f.data(), g->msg, 4 * E, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            for (int64_t e = 0; e < E; ++e) l[e] = f[e];
        } else {
            HIPCHK(hipMemcpyAsync(l.data(), g->msg, 8 * E, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
        }
        for (int64_t e = 0; e < E; ++e) {
            if (hg.fac_type[hg.edge_fac[e]] == FASTLBP_PRIOR)
                f2v_p1[e] = hg.fac_param[hg.edge_fac[e]];
            else
                f2v_p1[e] = 1.0 / (1.0 + std::exp2(-l[e]));
        }
    } catch (DeviceError &e) {
        return device_error(e);
    }
    return FASTLBP_OK;
}

int fastlbp_messages_set(fastlbp_graph_t g, const double *f2v_p1) {
    clear_error();
    if (!g || (!f2v_p1 && g->hg().E > 0)) {
        set_error("invalid argument");
        return FASTLBP_E_INVALID_ARG;
    }
    const HostGraph &hg = g->hg();
    int64_t E = hg.E;
    for (int64_t e = 0; e < E; ++e)
        if (!(f2v_p1[e] >= 0.0 && f2v_p1[e] <= 1.0)) {
            set_error("message " + std::to_string(e) + " outside [0,1]");
            return FASTLBP_E_INVALID_ARG;
        }
    if (!E) return FASTLBP_OK;
    try {
        std::vector<double> l(E, 0.0);
        for (int64_t e = 0; e < E; ++e) {
            if (hg.fac_type[hg.edge_fac[e]] == FASTLBP_PRIOR) continue;
            double p = f2v_p1[e];
            l[e] = (p >= 1.0) ? INFINITY : (p <= 0.0 ? -INFINITY : std::log2(p) - std::log2(1.0 - p));
        }
        hipStream_t s = g->L.stream;
        if (g->precision() == FASTLBP_FP32) {
            std::vector<float> f(l.begin(), l.end());
            HIPCHK(hipMemcpyAsync(g->msg, f.data(), 4 * E, hipMemcpyHostToDevice, s));
            HIPCHK(hipStreamSynchronize(s));
        } else {
            HIPCHK(hipMemcpyAsync(g->msg, l.data(), 8 * E, hipMemcpyHostToDevice, s));
            HIPCHK(hipStreamSynchronize(s));
        }
    } catch (DeviceError &e) {
        return device_error(e);
    }
    return FASTLBP_OK;
}

int fastlbp_messages_reset(fastlbp_graph_t g) {
    clear_error();
    if (!g) {
        set_error("graph is NULL");
        return FASTLBP_E_INVALID_ARG;
    }
    try {
        HIPCHK(hipMemsetAsync(g->msg, 0, g->S->msg_bytes() * std::max<int64_t>(g->hg().E, 1), g->L.stream));
        HIPCHK(hipStreamSynchronize(g->L.stream));
    } catch (DeviceError &e) {
        return device_error(e);
    }
    return FASTLBP_OK;
}

}  // extern "C"
