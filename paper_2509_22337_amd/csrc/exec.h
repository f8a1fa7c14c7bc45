// Kernels and launch code of the executors. Shared by the translation units that instantiate them
// (one per precision and executor, compiled in parallel) and by the C ABI in runtime.hip.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
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

// Incremental variable tasks of a level (plans with has_delta), one thread per record.
template <class P>
__global__ __launch_bounds__(256) void k_var_drec(DevGraph<typename P::S, typename P::V> g, DevPlan plan,
                                                  const VarRec *recs, int32_t count, const RunState *st) {
    if (st->done) return;
    const GPtr<const VarRec> R(recs);
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        var_delta<P>(g, plan, R.ld_stream(i));
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

// Small kernels of the run state and the marginals, defined once in runtime.hip.
__global__ void k_run_init(RunState *st, int32_t max_iters, double tol);
__global__ void k_run_init_step(RunState *st, int32_t max_iters, double tol, int32_t step);
__global__ void k_finalize(RunState *st);
__global__ void k_marginals(const Belief *bel, int32_t V, double *out);

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
// phases. Thread tasks come as records whose loads are issued ahead: a staged level's variable
// records before its factor phase, the next level's records as soon as this level's factor phase
// has issued its work, so their latency overlaps the barrier and the variable phase. Records are
// read through the caches: a narrow run reads the same records every iteration, and its plan is
// small enough to stay in the MALL (the wide-level kernels stream theirs). On entry `fr` / `pr` hold this
// thread's first factor record of L0 and, if L0 is staged, its first two staged variable records
// (tid and tid + NT); on exit they hold those of level `Lnext` (none when Lnext < 0). TEAMS adds the wavefront- and
// workgroup-per-factor paths and the weighted-term paths. foff / voff / staged give each level's
// record offsets and staging flag.
template <class P, bool DAMP, bool TEAMS, int NT, bool UNCOND, class FOff, class VOff, class Staged>
__device__ __forceinline__ void level_range(const DevGraph<typename P::S, typename P::V> &g, const DevPlan &plan,
                                            int32_t L0, int32_t L1, int32_t Lnext, FOff foff, VOff voff,
                                            Staged staged, typename P::S *s_slot, Belief *b_slot,
                                            TeamLds<typename P::V> *lds, Acc &acc, FacRec &fr, VarRecP (&pr)[2]) {
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
        const VarRecP pc0 = pr[0], pc1 = pr[1];
        if (v0 + tid < v1 && !stg) vr = vrec.ld(v0 + tid);
        S *const slots = stg ? s_slot : nullptr;
        // (the variable phase here rebuilds or stages beliefs, never reads (new, old) pairs)
        if (f0 + tid < f1) factor_rec<P, DAMP, false>(g, fr, acc, slots, b_slot);
        for (int32_t i = f0 + tid + NT; i < f1; i += NT)
            factor_rec<P, DAMP, false>(g, frec.ld(i), acc, slots, b_slot);
        if (TEAMS) {
            const GPtr<const int32_t> lst = plan.fac_list[FB_WAVE];
            int32_t o0 = plan.fac_lvl_off[FB_WAVE][L], o1 = plan.fac_lvl_off[FB_WAVE][L + 1];
            for (int32_t i = o0 + w; i < o1; i += NW) factor_wave<P, false, DAMP>(g, lst[i], lane, L, acc);
        }
        if (TEAMS) {
            const int32_t o0 = plan.trec_off[L], o1 = plan.trec_off[L + 1];
            for (int32_t i = o0 + tid; i < o1; i += NT) factor_terms_rec<P, DAMP>(g, plan.trec.ld(i), acc);
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
        {
            // records of the next level (Lnext after the last level of the range)
            // UNCOND: unconditional loads, record 0 for threads without one (never used: the phases
            // check the index again), since a conditional load makes the compiler wait for it at
            // once; the conditional form needs fewer registers
            const int32_t Ln = (L + 1 < L1) ? L + 1 : Lnext;
            if (UNCOND) {
                if (Ln >= 0) {
                    const int32_t n0 = foff(Ln), n1 = foff(Ln + 1);
                    fr = frec.ld(n0 + tid < n1 ? n0 + tid : 0);
                    const int32_t m0 = voff(Ln), m1 = voff(Ln + 1);
                    pr[0] = prec.ld(staged(Ln) && m0 + tid < m1 ? m0 + tid : 0);
                    pr[1] = prec.ld(staged(Ln) && m0 + tid + NT < m1 ? m0 + tid + NT : 0);
                }
            } else {
                fr = FacRec{};
                pr[0] = pr[1] = VarRecP{};
                if (Ln >= 0) {
                    const int32_t n0 = foff(Ln), n1 = foff(Ln + 1);
                    if (n0 + tid < n1) fr = frec.ld(n0 + tid);
                    const int32_t m0 = voff(Ln), m1 = voff(Ln + 1);
                    if (staged(Ln) && m0 + tid < m1) pr[0] = prec.ld(m0 + tid);
                    if (staged(Ln) && m0 + tid + NT < m1) pr[1] = prec.ld(m0 + tid + NT);
                }
            }
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
        if (stg) {
            if (v0 + tid < v1) var_staged<P>(g, pc0, s_slot, b_slot);
            if (v0 + tid + NT < v1) var_staged<P>(g, pc1, s_slot, b_slot);
            for (int32_t i = v0 + tid + 2 * NT; i < v1; i += NT) var_staged<P>(g, prec.ld(i), s_slot, b_slot);
        } else {
            if (v0 + tid < v1) var_rec<P>(g, vr);
            for (int32_t i = v0 + tid + NT; i < v1; i += NT) var_rec<P>(g, vrec.ld(i));
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
    // beliefs from the messages when the run starts; a later step of the same run continues from the
    // beliefs the previous launch left, so a run's result does not depend on how it is cut into steps
    if (st->iter == 0) {
        for (int32_t i = tid; i < plan.init_var_count[VB_THREAD]; i += NT) var_thread<P>(g, plan.init_var[VB_THREAD][i]);
        for (int32_t i = w; i < plan.init_var_count[VB_WAVE]; i += NW) var_wave<P>(g, plan.init_var[VB_WAVE][i], lane);
    }
    if (tid == 0) {
        if (D.step > 0) st->step_end = st->iter + D.step;
        s_done = st->done || st->iter >= st->step_end;
    }
    __syncthreads();
    // records of level 0: the factor record, and the staged variable record when level 0 is staged
    FacRec fr = {};
    VarRecP pr[2] = {};
    if (NL > 0) {
        fr = frec.ld(foff(0) + tid < foff(1) ? foff(0) + tid : 0);
        pr[0] = prec.ld(staged(0) && voff(0) + tid < voff(1) ? voff(0) + tid : 0);
        pr[1] = prec.ld(staged(0) && voff(0) + tid + NT < voff(1) ? voff(0) + tid + NT : 0);
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
    VarRecP pr[2] = {};
    if (foff(L0) + tid < foff(L0 + 1)) fr = plan.frec.ld(foff(L0) + tid);
    if (staged(L0) && voff(L0) + tid < voff(L0 + 1)) pr[0] = plan.prec.ld(voff(L0) + tid);
    if (staged(L0) && voff(L0) + tid + NT < voff(L0 + 1)) pr[1] = plan.prec.ld(voff(L0) + tid + NT);
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

// Pinned host bytes per handle for staging one launch descriptor and one state header.
constexpr size_t kFixedHostBytes = 2048;

// Descriptor and state-header areas provided by the caller of a persistent launch (a device area
// and a pinned host area of at least the launch's descriptor and header bytes).
struct FixedArea {
    void *dev;
    size_t dev_bytes;
    unsigned char *host;
    size_t host_bytes;
};

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
    // Copies v to a new allocation of at least min_elems elements; elements past v are zero (task
    // record arrays are read from index 0 by prefetches even when a plan has no record of a kind).
    template <class T>
    T *upload(const std::vector<T> &v, hipStream_t s, size_t min_elems = 1) {
        const size_t n = std::max<size_t>(v.size(), std::max<size_t>(min_elems, 1));
        T *p = (T *)get(sizeof(T) * n);
        if (n > v.size()) HIPCHK(hipMemsetAsync(p + v.size(), 0, sizeof(T) * (n - v.size()), s));
        if (!v.empty()) HIPCHK(hipMemcpyAsync(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));  // the host vector may die after return
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
    int32_t *drec = nullptr, *drec_off = nullptr, *dedge = nullptr, *dwave = nullptr, *dwave_off = nullptr;
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
        p.has_delta = hp.has_delta;
        p.drec = (const VarRec *)drec;
        p.drec_off = drec_off;
        p.dedge = dedge;
        p.dwave = dwave;
        p.dwave_off = dwave_off;
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
    // a second stream for the workgroup-per-factor launch of a level, which then overlaps the
    // level's other factor launches (fork and join through the two events)
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
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
    // creates the side stream and its events on first need (never while a capture is open)
    void ensure_side() {
        if (side) return;
        HIPCHK(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&join, hipEventDisableTiming));
        HIPCHK(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
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
        if (side) {
            (void)hipStreamSynchronize(side);
            (void)hipStreamDestroy(side);
        }
        if (fork) (void)hipEventDestroy(fork);
        if (join) (void)hipEventDestroy(join);
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
    void *prev = nullptr;  // (new, old) pairs of written messages (plans with incremental variable tasks)
    RunState *st = nullptr;
    double *marg = nullptr;
    Launcher L;
    RunState *h_state = nullptr;  // pinned copy
    unsigned char *h_fixed = nullptr;  // pinned staging of fastlbp_run_noalloc's launch descriptor
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
    // Residency of the device state, managed by a serving loop under a memory budget. While the
    // handle is evicted its messages are held in host_msg (their exact bytes), the device state is
    // freed and every call that needs it restores it first (graph_restore).
    std::atomic<bool> resident{true};
    size_t state_nominal = 0;            // device bytes of the state when resident
    std::vector<unsigned char> host_msg;
    std::recursive_mutex mu;             // held by every public call on the handle and by an eviction
    fastlbp_server *mgr = nullptr;       // the server managing the residency (at most one)
    uint64_t last_use = 0;               // the server's least-recently-used stamp
    // launch choices (the autotuner's; defaults: bucket cut-offs of layout.h, the rules below)
    PlanParams pparams;                  // bucket cut-offs of the plans built for this handle
    int32_t tune_graph_iters = 0;        // iterations per hipGraph replay (0: from the plan's launches)
    int32_t tune_threads = 0;            // persistent workgroup size (0: by rule)
    bool tuned = false;                  // the choices came from fastlbp_autotune

    const HostGraph &hg() const { return S->hg; }
    int precision() const { return S->precision; }
    size_t state_bytes() const { return state_nominal; }
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
        if (h_fixed) (void)hipHostFree(h_fixed);
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
        g.prev = (typename PP::S *)(P->hp.has_delta ? prev : nullptr);
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

static inline int grid_for(int64_t items, int per_block) {
    int64_t b = (items + per_block - 1) / per_block;
    return int(std::max<int64_t>(1, std::min<int64_t>(b, 65535 * 8)));
}

// Grid of the factor kernels: at most 8 workgroups per compute unit (enough to reach their
// occupancy); the workgroups loop over the rest, which bounds the residual atomics per launch.
static inline int fac_grid(int64_t items, int per_block) { return std::min(grid_for(items, per_block), 256 * 8); }

// Recompute every belief from phi and the current messages.
template <class PP>
static void launch_init_beliefs(fastlbp_graph *g, const DevGraph<typename PP::S, typename PP::V> &dg) {
    const HostPlan &hp = g->P->hp;
    int32_t n0 = int32_t(hp.init_var[VB_THREAD].size()), n1 = int32_t(hp.init_var[VB_WAVE].size());
    if (n0) k_var_thread<PP><<<grid_for(n0, 256), 256, 0, g->L.stream>>>(dg, g->P->init_var[VB_THREAD], n0, nullptr);
    if (n1) k_var_wave<PP><<<grid_for(n1, 4), 256, 0, g->L.stream>>>(dg, g->P->init_var[VB_WAVE], n1, nullptr);
    HIPCHK(hipGetLastError());
}

static inline int persistent_threads(int precision, bool teams, int runs);

// One launch of k_levels_fused for levels [L0, L1).
template <class PP, bool DAMP>
static void launch_fused(fastlbp_graph *g, const DevGraph<typename PP::S, typename PP::V> &dg_in, const DevPlan &dp,
                         int32_t L0, int32_t L1, bool teams, hipStream_t s) {
    // fused levels keep their beliefs themselves: no old values to record
    DevGraph<typename PP::S, typename PP::V> dg = dg_in;
    dg.prev = GPtr<typename PP::S>();
    const int32_t cap = g->P->hp.stage_slots;
    const size_t lds = stage_bytes<typename PP::S>(std::max(cap, 1));
    int nt = persistent_threads(g->precision(), teams, 1);
    if (g->tune_threads == 512 || (g->tune_threads == 1024 && g->precision() == FASTLBP_FP32 && !teams))
        nt = g->tune_threads;
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
static void enqueue_iteration(fastlbp_graph *g, const DevGraph<typename PP::S, typename PP::V> &dg, bool fuse,
                              bool side_ok = true) {
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
        // the level's workgroup-per-factor tasks (few, long: a hub factor with thousands of inputs)
        // run on the side stream beside its other factor launches; the variable phase waits for both
        const int32_t ob = pl.fac_lvl_off[FB_BLOCK][L], nb = pl.fac_lvl_off[FB_BLOCK][L + 1] - ob;
        const bool others = pl.frec_off[L + 1] > pl.frec_off[L] ||
                            pl.fac_lvl_off[FB_WAVE][L + 1] > pl.fac_lvl_off[FB_WAVE][L] ||
                            pl.fac_lvl_off[FB_TERMS_WAVE][L + 1] > pl.fac_lvl_off[FB_TERMS_WAVE][L] ||
                            pl.trec_off[L + 1] > pl.trec_off[L];
        const bool fork = nb > 0 && others && side_ok && g->L.side;
        if (fork) {
            HIPCHK(hipEventRecord(g->L.fork, s));
            HIPCHK(hipStreamWaitEvent(g->L.side, g->L.fork, 0));
            k_fac_block<PP, ALL, DAMP, block_threads<PP>()><<<std::min(nb, 4096), block_threads<PP>(), 0, g->L.side>>>(
                dg, P.fac_list[FB_BLOCK] + ob, nb, L, g->st);
            HIPCHK(hipEventRecord(g->L.join, g->L.side));
        }
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
        if (fork)
            HIPCHK(hipStreamWaitEvent(s, g->L.join, 0));
        else if (nb)
            k_fac_block<PP, ALL, DAMP, block_threads<PP>()><<<std::min(nb, 4096), block_threads<PP>(), 0, s>>>(
                dg, P.fac_list[FB_BLOCK] + ob, nb, L, g->st);
        if (pl.has_delta && dg.prev.p) {  // incremental variable tasks
            o = pl.drec_off[L];
            n = pl.drec_off[L + 1] - o;
            if (n) k_var_drec<PP><<<grid_for(n, 256), 256, 0, s>>>(dg, dp, (const VarRec *)P.drec + o, n, g->st);
            o = pl.dwave_off[L];
            n = pl.dwave_off[L + 1] - o;
            if (n) k_var_wave<PP><<<grid_for(n, 4), 256, 0, s>>>(dg, P.dwave + o, n, g->st);
            continue;
        }
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
static inline int persistent_threads(int precision, bool teams, int runs) {
    return (precision == FASTLBP_FP32 && !teams && runs <= 256) ? 1024 : 512;
}

static inline int choose_executor(const fastlbp_graph *g) {
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
// plain: launch every iteration's kernels directly instead of replaying a captured hipGraph (whose
// instantiation allocates).
static void run_levels(fastlbp_graph *g, int32_t max_iters, double tol, double damping, bool fuse, bool plain) {
    auto dg = g->view<PP>(damping);
    hipStream_t s = g->L.stream;
    k_run_init<<<1, 64, 0, s>>>(g->st, max_iters, tol);
    HIPCHK(hipGetLastError());
    launch_init_beliefs<PP>(g, dg);
    if (max_iters <= 0) return;
    // iterations per replay: enough to amortise the launch, few enough to stop soon after
    // convergence (kernels of finished iterations return at once)
    int per_iter_kernels = std::max(1, fuse ? g->P->hp.launches_hybrid : g->P->hp.launches_levels);
    int K = g->tune_graph_iters > 0 ? g->tune_graph_iters : std::max(1, std::min(32, 2048 / per_iter_kernels));
    K = std::min(K, max_iters);
    bool use_graph = g->opts.use_graph != 0 && !plain;
    // (the allocation-free path keeps every launch on the caller's stream)
    if (!plain && !g->P->hp.fac_list[FB_BLOCK].empty()) g->L.ensure_side();
    if (use_graph) ensure_iteration_graph<PP, ALL, DAMP>(g, dg, K, damping, fuse);
    int done_iters = 0;
    while (true) {
        if (use_graph)
            HIPCHK(hipGraphLaunch(g->gexec, s));
        else
            for (int k = 0; k < K; ++k) enqueue_iteration<PP, ALL, DAMP>(g, dg, fuse, !plain);
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
// fixed (optional): a caller-provided device area for the descriptors and state headers and a
// pinned host area for their staging, used instead of the launcher's own buffers (which are
// allocated on first use).
// steps (optional): each run's own step, replacing `step`.
static void launch_persistent(Launcher &lc, int n, fastlbp_graph *const *gs, const double *damping,
                              int32_t step = 0, const FixedArea *fixed = nullptr, const int32_t *steps = nullptr) {
    if (n <= 0) return;
    bool teams = false, damp = false;
    for (int i = 0; i < n; ++i) {
        teams = teams || gs[i]->P->teams();
        damp = damp || damping[i] > 0.0;
    }
    const size_t dbytes = sizeof(RunDesc<PP>) * size_t(n);
    const size_t sbytes = kRunStateHeader * size_t(n);
    const size_t bytes = dbytes + sbytes;
    if (fixed && (bytes > fixed->dev_bytes || bytes > fixed->host_bytes))
        throw DeviceError{"launch descriptors exceed the fixed area"};
    void *d = fixed ? fixed->dev : lc.descs(bytes);
    int32_t *dstatus = (int32_t *)((unsigned char *)d + dbytes);
    if (!fixed) lc.hdesc.resize(dbytes);
    RunDesc<PP> *h = (RunDesc<PP> *)(fixed ? fixed->host : lc.hdesc.data());
    for (int i = 0; i < n; ++i) {
        h[i].g = gs[i]->view<PP>(damping[i]);
        h[i].g.prev = GPtr<typename PP::S>();  // the persistent level loop keeps its beliefs itself
        h[i].plan = gs[i]->P->view();
        h[i].st = GPtr<RunState>(gs[i]->st);
        h[i].status = GPtr<int32_t>(dstatus + i * int(kRunStateHeader / 4));
        h[i].step = steps ? steps[i] : step;
    }
    unsigned char *hs = fixed ? fixed->host + dbytes : lc.status_host(sbytes);
    HIPCHK(hipMemcpyAsync(d, h, dbytes, hipMemcpyHostToDevice, lc.stream));
    const RunDesc<PP> *dd = (const RunDesc<PP> *)d;
    int nt = persistent_threads(gs[0]->precision(), teams, n);
    {  // a size the autotuner chose, when every run of the launch has the same choice
        const int want = gs[0]->tune_threads;
        bool same = want > 0;
        for (int i = 1; i < n && same; ++i) same = gs[i]->tune_threads == want;
        if (same && (want == 512 || (want == 1024 && gs[0]->precision() == FASTLBP_FP32 && !teams))) nt = want;
    }
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
// A server step of a run on the LEVELS executor: beliefs rebuilt (the evidence may be new), then
// `iters` iterations on the handle's own stream, so the step overlaps the persistent launch of the
// narrow runs. Iterations after the run is done return at once.
template <class PP, bool ALL, bool DAMP>
static void step_levels_t(fastlbp_graph *g, double damping, int32_t iters) {
    auto dg = g->view<PP>(damping);
    hipStream_t s = g->L.stream;
    if (!g->P->hp.fac_list[FB_BLOCK].empty()) g->L.ensure_side();
    HIPCHK(hipEventRecord(g->L.k0, s));
    // beliefs from the messages at the run's first step only (later steps continue from the
    // beliefs the last one left, as one longer launch would)
    if (g->h_state->iter == 0) launch_init_beliefs<PP>(g, dg);
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

// Runs of the LEVELS or HYBRID executor, dispatched over the plan's activity and damping.
template <class PP>
static void levels_run(fastlbp_graph *g, int32_t max_iters, double tol, double damping, bool fuse, bool plain) {
    bool all = g->P->hp.all_active != 0, damp = damping > 0.0;
    if (all && damp) run_levels<PP, true, true>(g, max_iters, tol, damping, fuse, plain);
    if (all && !damp) run_levels<PP, true, false>(g, max_iters, tol, damping, fuse, plain);
    if (!all && damp) run_levels<PP, false, true>(g, max_iters, tol, damping, fuse, plain);
    if (!all && !damp) run_levels<PP, false, false>(g, max_iters, tol, damping, fuse, plain);
}

// Plan of a schedule with known levels (runtime.hip), and one run on an executor.
std::shared_ptr<Plan> plan_from_levels(const Structure &S, const Alloc &alloc, hipStream_t s, int kind,
                                       const std::vector<int32_t> &level, int32_t n, const PlanParams &pp);
void run_any(fastlbp_graph *g, int32_t max_iters, double tol, double damping, int exec);

// Instantiations, one translation unit per precision and executor (exec_*.hip).
void levels_run_f32(fastlbp_graph *g, int32_t max_iters, double tol, double damping, bool fuse, bool plain);
void levels_run_f64(fastlbp_graph *g, int32_t max_iters, double tol, double damping, bool fuse, bool plain);
void levels_step_f32(fastlbp_graph *g, double damping, int32_t iters);
void levels_step_f64(fastlbp_graph *g, double damping, int32_t iters);
void init_beliefs_f32(fastlbp_graph *g);
void init_beliefs_f64(fastlbp_graph *g);
void persistent_launch_f32(Launcher &lc, int n, fastlbp_graph *const *gs, const double *damping, int32_t step,
                           const FixedArea *fixed = nullptr, const int32_t *steps = nullptr);
void persistent_launch_f64(Launcher &lc, int n, fastlbp_graph *const *gs, const double *damping, int32_t step,
                           const FixedArea *fixed = nullptr, const int32_t *steps = nullptr);

}  // namespace fastlbp
