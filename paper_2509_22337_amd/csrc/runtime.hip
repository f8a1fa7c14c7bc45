// Kernels, iteration driver and the C ABI of libfastlbp (the Kernel Launch and Message Passing
// stages of Section 4.1, executed as described in Section 4.3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "fastlbp.h"
#include "host.h"
#include "kernels.h"

namespace fastlbp {

// ------------------------------------------------------------------------------------------------
// Kernels
// ------------------------------------------------------------------------------------------------

__device__ __forceinline__ void flush_acc(Acc acc, RunState *st) {
    double r = acc.r;
    unsigned int c = acc.contra;
#pragma unroll
    for (int k = 32; k >= 1; k >>= 1) {
        r = fmax(r, __shfl_xor(r, k, 64));
        c += __shfl_xor(c, k, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        if (r > 0.0) atomicMax(&st->rbits, (unsigned long long)__double_as_longlong(r));
        if (c) atomicAdd(&st->contra, (unsigned long long)c);
    }
}

template <class P, bool ALL, bool DAMP>
__global__ __launch_bounds__(256) void k_fac_thread(DevGraph<typename P::S, typename P::V> g, const int32_t *list,
                                                    int32_t count, int32_t level, RunState *st) {
    if (st->done) return;
    Acc acc = {0.0, 0u};
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        factor_team<P, 1, kThreadMaxDeg - 1, ALL, DAMP>(g, list[i], 0, level, acc, nullptr);
    flush_acc(acc, st);
}

template <class P, bool ALL, bool DAMP>
__global__ __launch_bounds__(256) void k_fac_wave(DevGraph<typename P::S, typename P::V> g, const int32_t *list,
                                                  int32_t count, int32_t level, RunState *st) {
    if (st->done) return;
    Acc acc = {0.0, 0u};
    const int lane = threadIdx.x & 63;
    const int waves = gridDim.x * (blockDim.x >> 6);
    for (int32_t i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); i < count; i += waves)
        factor_team<P, 64, 16, ALL, DAMP>(g, list[i], lane, level, acc, nullptr);
    flush_acc(acc, st);
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
    flush_acc(acc, st);
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
__global__ __launch_bounds__(256) void k_var_wave(DevGraph<typename P::S, typename P::V> g, const int32_t *list,
                                                  int32_t count, const RunState *st) {
    if (st && st->done) return;
    const int waves = gridDim.x * (blockDim.x >> 6);
    for (int32_t i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); i < count; i += waves)
        var_wave<P>(g, list[i], threadIdx.x & 63);
}

__global__ void k_run_init(RunState *st, int32_t max_iters, double tol) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->rbits = 0ull;
        st->contra = 0ull;
        st->iter = 0;
        st->done = max_iters <= 0 ? 1 : 0;
        st->last_r = 0.0;
        st->max_iters = max_iters;
        st->converged = 0;
        st->tol = tol;
    }
}

// End of one iteration: publish the residual, decide whether to stop.
__global__ void k_finalize(RunState *st) {
    if (threadIdx.x != 0 || blockIdx.x != 0 || st->done) return;
    double r = __longlong_as_double((long long)st->rbits);
    st->rbits = 0ull;
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
    Belief B = bel[v];
    double p;
    if (B.npos > 0 && B.nneg > 0)
        p = 0.5;
    else if (B.npos > 0)
        p = 1.0;
    else if (B.nneg > 0)
        p = 0.0;
    else
        p = 1.0 / (1.0 + exp2(-B.fin));
    out[v] = p;
}

// One workgroup of NT threads runs the whole run: every iteration, every level, both phases, with
// workgroup barriers between phases. Used when the levels are too narrow to fill the GPU. TEAMS
// adds the wavefront- and workgroup-per-factor paths (plans with factors of degree > 8).
template <class P, bool ALL, bool DAMP, bool TEAMS, int NT>
__global__ __launch_bounds__(NT) void k_persistent(DevGraph<typename P::S, typename P::V> g, DevPlan plan,
                                                   RunState *st) {
    using V = typename P::V;
    constexpr int NW = NT / 64;
    __shared__ TeamLds<V> lds;
    __shared__ double red_r[NW];
    __shared__ unsigned int red_c[NW];
    __shared__ int s_done;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int32_t i = tid; i < plan.init_var_count[VB_THREAD]; i += NT) var_thread<P>(g, plan.init_var[VB_THREAD][i]);
    for (int32_t i = w; i < plan.init_var_count[VB_WAVE]; i += NW) var_wave<P>(g, plan.init_var[VB_WAVE][i], lane);
    if (tid == 0) s_done = st->done;
    __syncthreads();
    while (!s_done) {
        Acc acc = {0.0, 0u};
        for (int32_t L = 0; L < plan.num_levels; ++L) {
            {
                const int32_t *lst = plan.fac_list[FB_THREAD];
                int32_t o0 = plan.fac_lvl_off[FB_THREAD][L], o1 = plan.fac_lvl_off[FB_THREAD][L + 1];
                for (int32_t i = o0 + tid; i < o1; i += NT)
                    factor_team<P, 1, kThreadMaxDeg - 1, ALL, DAMP>(g, lst[i], 0, L, acc, nullptr);
            }
            if (TEAMS) {
                const int32_t *lst = plan.fac_list[FB_WAVE];
                int32_t o0 = plan.fac_lvl_off[FB_WAVE][L], o1 = plan.fac_lvl_off[FB_WAVE][L + 1];
                for (int32_t i = o0 + w; i < o1; i += NW) factor_team<P, 64, 16, ALL, DAMP>(g, lst[i], lane, L, acc, nullptr);
            }
            if (TEAMS) {
                const int32_t *lst = plan.fac_list[FB_BLOCK];
                int32_t o0 = plan.fac_lvl_off[FB_BLOCK][L], o1 = plan.fac_lvl_off[FB_BLOCK][L + 1];
                for (int32_t i = o0; i < o1; ++i)
                    factor_team<P, NT, (kBlockMaxDeg - 1) / NT, ALL, DAMP>(g, lst[i], tid, L, acc, &lds);
            }
            __syncthreads();
            {
                const int32_t *lst = plan.var_list[VB_THREAD];
                int32_t o0 = plan.var_lvl_off[VB_THREAD][L], o1 = plan.var_lvl_off[VB_THREAD][L + 1];
                for (int32_t i = o0 + tid; i < o1; i += NT) var_thread<P>(g, lst[i]);
            }
            {
                const int32_t *lst = plan.var_list[VB_WAVE];
                int32_t o0 = plan.var_lvl_off[VB_WAVE][L], o1 = plan.var_lvl_off[VB_WAVE][L + 1];
                for (int32_t i = o0 + w; i < o1; i += NW) var_wave<P>(g, lst[i], lane);
            }
            __syncthreads();
        }
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
            s_done = st->done;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------------------
// Device memory
// ------------------------------------------------------------------------------------------------

struct Alloc {
    void *(*fn_alloc)(size_t, void *) = nullptr;
    void (*fn_free)(void *, void *) = nullptr;
    void *ctx = nullptr;
    void *get(size_t bytes) {
        if (bytes == 0) bytes = 16;
        if (fn_alloc) return fn_alloc(bytes, ctx);
        void *p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
        return p;
    }
    void put(void *p) {
        if (!p) return;
        if (fn_free)
            fn_free(p, ctx);
        else
            (void)hipFree(p);
    }
};

struct OomError {};
struct DeviceError {
    std::string msg;
};

#define HIPCHK(x)                                                                                          \
    do {                                                                                                   \
        hipError_t _e = (x);                                                                               \
        if (_e != hipSuccess) throw DeviceError{std::string(#x) + ": " + hipGetErrorString(_e)};           \
    } while (0)

}  // namespace fastlbp

using namespace fastlbp;

struct DevArrays {
    // structure
    int32_t *fac_off = nullptr, *edge_var = nullptr, *var_off = nullptr, *var_edge = nullptr, *edge_level = nullptr;
    uint8_t *fac_type = nullptr;
    void *fpar = nullptr, *epar = nullptr;
    Belief *phi = nullptr, *bel = nullptr;
    void *msg = nullptr;
    RunState *state = nullptr;
    double *marg = nullptr;
    // plan
    int32_t *fac_list[FB_COUNT] = {}, *fac_lvl_off[FB_COUNT] = {};
    int32_t *var_list[VB_COUNT] = {}, *var_lvl_off[VB_COUNT] = {}, *init_var[VB_COUNT] = {};
};

struct fastlbp_graph {
    fastlbp_options opts;
    Alloc alloc;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int precision = FASTLBP_FP64;
    HostGraph hg;
    HostPlan plan;
    int sched_kind = FASTLBP_SCHED_FLOODING;
    DevArrays d;
    std::vector<void *> owned;  // every device allocation
    std::vector<void *> plan_owned;
    // captured iterations for the LEVELS executor
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    int graph_iters = 0;
    double graph_damping = -1.0;
    RunState *h_state = nullptr;  // pinned copy
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    fastlbp_run_stats last{};
    size_t msg_bytes() const { return precision == FASTLBP_FP32 ? 4 : 8; }
    size_t val_bytes() const { return precision == FASTLBP_FP32 ? 4 : 8; }

    void *dev(size_t bytes, bool plan_buf = false) {
        void *p = alloc.get(bytes);
        if (!p) throw OomError{};
        (plan_buf ? plan_owned : owned).push_back(p);
        return p;
    }
    template <class T>
    T *upload(const std::vector<T> &v, bool plan_buf = false) {
        T *p = (T *)dev(sizeof(T) * std::max<size_t>(v.size(), 1), plan_buf);
        if (!v.empty()) {
            HIPCHK(hipMemcpyAsync(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, stream));
            HIPCHK(hipStreamSynchronize(stream));  // the host vector may die after return
        }
        return p;
    }
    void drop_graph() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        gexec = nullptr;
        graph = nullptr;
        graph_iters = 0;
    }
    ~fastlbp_graph() {
        if (stream) (void)hipStreamSynchronize(stream);
        drop_graph();
        for (void *p : owned) alloc.put(p);
        for (void *p : plan_owned) alloc.put(p);
        if (h_state) (void)hipHostFree(h_state);
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }

    template <class P>
    DevGraph<typename P::S, typename P::V> view(double damping) const {
        DevGraph<typename P::S, typename P::V> g;
        g.num_vars = hg.V;
        g.num_edges = int32_t(hg.E);
        g.fac_off = d.fac_off;
        g.edge_var = d.edge_var;
        g.fac_type = d.fac_type;
        g.fpar = (const Pair<typename P::V> *)d.fpar;
        g.epar = (const Pair<typename P::V> *)d.epar;
        g.var_off = d.var_off;
        g.var_edge = d.var_edge;
        g.phi = d.phi;
        g.bel = d.bel;
        g.msg = (typename P::S *)d.msg;
        g.edge_level = d.edge_level;
        if (precision == FASTLBP_FP32) {
            g.damp_old = (typename P::V)(damping > 0 ? std::log2(damping) : -INFINITY);
            g.damp_new = (typename P::V)std::log2(1.0 - damping);
        } else {
            g.damp_old = (typename P::V)damping;
            g.damp_new = (typename P::V)(1.0 - damping);
        }
        return g;
    }
    DevPlan dplan() const {
        DevPlan p;
        p.num_levels = plan.exec_levels;
        p.all_active = plan.all_active;
        for (int b = 0; b < FB_COUNT; ++b) {
            p.fac_list[b] = d.fac_list[b];
            p.fac_lvl_off[b] = d.fac_lvl_off[b];
        }
        for (int b = 0; b < VB_COUNT; ++b) {
            p.var_list[b] = d.var_list[b];
            p.var_lvl_off[b] = d.var_lvl_off[b];
            p.init_var[b] = d.init_var[b];
            p.init_var_count[b] = int32_t(plan.init_var[b].size());
        }
        return p;
    }
};

namespace fastlbp {

static int grid_for(int64_t items, int per_block) {
    int64_t b = (items + per_block - 1) / per_block;
    return int(std::max<int64_t>(1, std::min<int64_t>(b, 65535 * 8)));
}

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
static void upload_params(fastlbp_graph *g, bool logd) {
    std::vector<Pair<V>> fp(std::max(g->hg.F, 1)), ep(std::max<int64_t>(g->hg.E, 1));
    for (int32_t a = 0; a < g->hg.F; ++a) fp[a] = param_pair<V>(g->hg.fac_param[a], logd);
    for (int64_t e = 0; e < g->hg.E; ++e) ep[e] = param_pair<V>(g->hg.edge_param[e], logd);
    g->d.fpar = g->upload(fp);
    g->d.epar = g->upload(ep);
}

static void upload_plan(fastlbp_graph *g) {
    HIPCHK(hipStreamSynchronize(g->stream));
    for (void *p : g->plan_owned) g->alloc.put(p);
    g->plan_owned.clear();
    g->drop_graph();
    g->d.edge_level = g->upload(g->plan.edge_exec_level, true);
    for (int b = 0; b < FB_COUNT; ++b) {
        g->d.fac_list[b] = g->upload(g->plan.fac_list[b], true);
        g->d.fac_lvl_off[b] = g->upload(g->plan.fac_lvl_off[b], true);
    }
    for (int b = 0; b < VB_COUNT; ++b) {
        g->d.var_list[b] = g->upload(g->plan.var_list[b], true);
        g->d.var_lvl_off[b] = g->upload(g->plan.var_lvl_off[b], true);
        g->d.init_var[b] = g->upload(g->plan.init_var[b], true);
    }
    HIPCHK(hipStreamSynchronize(g->stream));
}

static void upload_phi(fastlbp_graph *g) {
    std::vector<Belief> phi;
    g->hg.phi(phi);
    if (phi.empty()) return;
    HIPCHK(hipMemcpyAsync(g->d.phi, phi.data(), sizeof(Belief) * phi.size(), hipMemcpyHostToDevice, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
}

// Recompute every belief from phi and the current messages.
template <class P>
static void launch_init_beliefs(fastlbp_graph *g, const DevGraph<typename P::S, typename P::V> &dg) {
    int32_t n0 = int32_t(g->plan.init_var[VB_THREAD].size()), n1 = int32_t(g->plan.init_var[VB_WAVE].size());
    if (n0) k_var_thread<P><<<grid_for(n0, 256), 256, 0, g->stream>>>(dg, g->d.init_var[VB_THREAD], n0, nullptr);
    if (n1) k_var_wave<P><<<grid_for(n1, 4), 256, 0, g->stream>>>(dg, g->d.init_var[VB_WAVE], n1, nullptr);
    HIPCHK(hipGetLastError());
}

// One iteration of the LEVELS executor: for every level, the factor phase then the variable phase.
template <class P, bool ALL, bool DAMP>
static void enqueue_iteration(fastlbp_graph *g, const DevGraph<typename P::S, typename P::V> &dg) {
    const HostPlan &pl = g->plan;
    for (int32_t L = 0; L < pl.exec_levels; ++L) {
        int32_t o, n;
        o = pl.fac_lvl_off[FB_THREAD][L];
        n = pl.fac_lvl_off[FB_THREAD][L + 1] - o;
        if (n) k_fac_thread<P, ALL, DAMP><<<grid_for(n, 256), 256, 0, g->stream>>>(dg, g->d.fac_list[FB_THREAD] + o, n, L, g->d.state);
        o = pl.fac_lvl_off[FB_WAVE][L];
        n = pl.fac_lvl_off[FB_WAVE][L + 1] - o;
        if (n) k_fac_wave<P, ALL, DAMP><<<grid_for(n, 4), 256, 0, g->stream>>>(dg, g->d.fac_list[FB_WAVE] + o, n, L, g->d.state);
        o = pl.fac_lvl_off[FB_BLOCK][L];
        n = pl.fac_lvl_off[FB_BLOCK][L + 1] - o;
        if (n)
            k_fac_block<P, ALL, DAMP, block_threads<P>()><<<std::min(n, 4096), block_threads<P>(), 0, g->stream>>>(
                dg, g->d.fac_list[FB_BLOCK] + o, n, L, g->d.state);
        o = pl.var_lvl_off[VB_THREAD][L];
        n = pl.var_lvl_off[VB_THREAD][L + 1] - o;
        if (n) k_var_thread<P><<<grid_for(n, 256), 256, 0, g->stream>>>(dg, g->d.var_list[VB_THREAD] + o, n, g->d.state);
        o = pl.var_lvl_off[VB_WAVE][L];
        n = pl.var_lvl_off[VB_WAVE][L + 1] - o;
        if (n) k_var_wave<P><<<grid_for(n, 4), 256, 0, g->stream>>>(dg, g->d.var_list[VB_WAVE] + o, n, g->d.state);
    }
    k_finalize<<<1, 64, 0, g->stream>>>(g->d.state);
}

// Workgroup size of the persistent executor: 1024 threads for float32, 512 for float64 (whose
// factor code needs up to 256 registers). FASTLBP_PERSISTENT_THREADS=512|1024 overrides.
static int persistent_threads(int precision) {
    const char *e = std::getenv("FASTLBP_PERSISTENT_THREADS");
    if (e && (std::atoi(e) == 512 || std::atoi(e) == 1024)) return std::atoi(e);
    return precision == FASTLBP_FP32 ? 1024 : 512;
}

static int choose_executor(const fastlbp_graph *g) {
    int ex = g->opts.executor;
    if (ex == FASTLBP_EXEC_LEVELS || ex == FASTLBP_EXEC_PERSISTENT) return ex;
    // one workgroup keeps up with a level of a few thousand edges; wider levels need the GPU
    if (g->plan.max_level_edges <= 8192 && g->hg.nonprior_edges <= (int64_t(4) << 20)) return FASTLBP_EXEC_PERSISTENT;
    return FASTLBP_EXEC_LEVELS;
}

template <class P, bool ALL, bool DAMP>
static void run_impl(fastlbp_graph *g, int32_t max_iters, double tol, double damping, int exec) {
    auto dg = g->view<P>(damping);
    k_run_init<<<1, 64, 0, g->stream>>>(g->d.state, max_iters, tol);
    HIPCHK(hipGetLastError());
    if (exec == FASTLBP_EXEC_PERSISTENT) {
        // the variant without wavefront/workgroup factor code needs fewer registers
        bool teams = !g->plan.fac_list[FB_WAVE].empty() || !g->plan.fac_list[FB_BLOCK].empty();
        // float64 factor code needs more than the 128 registers a 1024-thread workgroup allows
        int nt = persistent_threads(g->precision);
        if (teams && nt == 1024)
            k_persistent<P, ALL, DAMP, true, 1024><<<1, 1024, 0, g->stream>>>(dg, g->dplan(), g->d.state);
        else if (teams)
            k_persistent<P, ALL, DAMP, true, 512><<<1, 512, 0, g->stream>>>(dg, g->dplan(), g->d.state);
        else if (nt == 1024)
            k_persistent<P, ALL, DAMP, false, 1024><<<1, 1024, 0, g->stream>>>(dg, g->dplan(), g->d.state);
        else
            k_persistent<P, ALL, DAMP, false, 512><<<1, 512, 0, g->stream>>>(dg, g->dplan(), g->d.state);
        HIPCHK(hipGetLastError());
        return;
    }
    launch_init_beliefs<P>(g, dg);
    if (max_iters <= 0) return;
    // iterations per replay: enough to amortise the launch, few enough to stop soon after
    // convergence (kernels of finished iterations return at once)
    int per_iter_kernels = 1 + 2 * std::max(1, g->plan.exec_levels);
    int K = std::max(1, std::min(32, 2048 / per_iter_kernels));
    K = std::min(K, max_iters);
    bool use_graph = g->opts.use_graph != 0;
    if (use_graph && (!g->gexec || g->graph_iters != K || g->graph_damping != damping)) {
        g->drop_graph();
        HIPCHK(hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal));
        for (int k = 0; k < K; ++k) enqueue_iteration<P, ALL, DAMP>(g, dg);
        HIPCHK(hipStreamEndCapture(g->stream, &g->graph));
        HIPCHK(hipGraphInstantiate(&g->gexec, g->graph, nullptr, nullptr, 0));
        g->graph_iters = K;
        g->graph_damping = damping;
    }
    int done_iters = 0;
    while (true) {
        if (use_graph)
            HIPCHK(hipGraphLaunch(g->gexec, g->stream));
        else
            for (int k = 0; k < K; ++k) enqueue_iteration<P, ALL, DAMP>(g, dg);
        HIPCHK(hipGetLastError());
        done_iters += K;
        if (done_iters >= max_iters) break;
        HIPCHK(hipMemcpyAsync(g->h_state, g->d.state, sizeof(RunState), hipMemcpyDeviceToHost, g->stream));
        HIPCHK(hipStreamSynchronize(g->stream));
        if (g->h_state->done) break;
    }
}

template <class P>
static void run_dispatch(fastlbp_graph *g, int32_t max_iters, double tol, double damping, int exec) {
    bool all = g->plan.all_active != 0, damp = damping > 0.0;
    if (all && damp) run_impl<P, true, true>(g, max_iters, tol, damping, exec);
    if (all && !damp) run_impl<P, true, false>(g, max_iters, tol, damping, exec);
    if (!all && damp) run_impl<P, false, true>(g, max_iters, tol, damping, exec);
    if (!all && !damp) run_impl<P, false, false>(g, max_iters, tol, damping, exec);
}

static int device_error(const DeviceError &e) {
    set_error(e.msg);
    return FASTLBP_E_DEVICE;
}

static int set_schedule(fastlbp_graph *g, int kind, const int32_t *rank) {
    std::vector<int32_t> level;
    int32_t n = analyze_levels(g->hg.V, g->hg.F, g->hg.fac_off.data(), g->hg.edge_var.data(),
                               kind == FASTLBP_SCHED_FLOODING ? nullptr : rank, level);
    HostPlan p;
    p.build(g->hg, level, n, kind == FASTLBP_SCHED_FLOODING, int(g->msg_bytes()), int(2 * g->val_bytes()));
    g->plan = std::move(p);
    g->sched_kind = kind;
    upload_plan(g);
    return FASTLBP_OK;
}

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

const char *fastlbp_version(void) { return "fastlbp-mi355x 0.1 (gfx950)"; }

int fastlbp_graph_create(int32_t num_vars, int32_t num_factors, const int64_t *factor_offsets,
                         const int32_t *edge_vars, const uint8_t *factor_types, const double *factor_params,
                         const double *edge_params, const fastlbp_options *opts, fastlbp_graph_t *out) {
    clear_error();
    if (!out) {
        set_error("out is NULL");
        return FASTLBP_E_INVALID_ARG;
    }
    *out = nullptr;
    int rc = validate_graph(num_vars, num_factors, factor_offsets, edge_vars, factor_types, factor_params, edge_params);
    if (rc) return rc;
    fastlbp_options o;
    fastlbp_options_default(&o);
    if (opts) o = *opts;
    if (o.precision != FASTLBP_FP64 && o.precision != FASTLBP_FP32) {
        set_error("precision must be FASTLBP_FP64 or FASTLBP_FP32");
        return FASTLBP_E_INVALID_ARG;
    }
    if (o.executor < FASTLBP_EXEC_AUTO || o.executor > FASTLBP_EXEC_PERSISTENT) {
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
    std::unique_ptr<fastlbp_graph> g(new fastlbp_graph());
    g->opts = o;
    g->precision = o.precision;
    g->alloc.fn_alloc = o.alloc;
    g->alloc.fn_free = o.free;
    g->alloc.ctx = o.alloc_ctx;
    try {
        HIPCHK(hipSetDevice(o.device));
        hipDeviceProp_t prop;
        HIPCHK(hipGetDeviceProperties(&prop, o.device));
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
            set_error(std::string("device is ") + prop.gcnArchName + ", library is built for gfx950");
            return FASTLBP_E_DEVICE;
        }
        if (o.stream) {
            g->stream = (hipStream_t)o.stream;
        } else {
            HIPCHK(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking));
            g->own_stream = true;
        }
        HIPCHK(hipEventCreate(&g->ev0));
        HIPCHK(hipEventCreate(&g->ev1));
        HIPCHK(hipHostMalloc((void **)&g->h_state, sizeof(RunState), hipHostMallocDefault));
        g->hg.build(num_vars, num_factors, factor_offsets, edge_vars, factor_types, factor_params, edge_params);
        HostGraph &hg = g->hg;
        std::vector<int32_t> off32(hg.fac_off.begin(), hg.fac_off.end());
        g->d.fac_off = g->upload(off32);
        g->d.edge_var = g->upload(hg.edge_var);
        g->d.fac_type = g->upload(hg.fac_type);
        g->d.var_off = g->upload(hg.var_off);
        g->d.var_edge = g->upload(hg.var_edge);
        if (g->precision == FASTLBP_FP32)
            upload_params<float>(g.get(), true);
        else
            upload_params<double>(g.get(), false);
        g->d.phi = (Belief *)g->dev(sizeof(Belief) * std::max(hg.V, 1));
        g->d.bel = (Belief *)g->dev(sizeof(Belief) * std::max(hg.V, 1));
        g->d.msg = g->dev(g->msg_bytes() * std::max<int64_t>(hg.E, 1));
        g->d.state = (RunState *)g->dev(sizeof(RunState));
        g->d.marg = (double *)g->dev(sizeof(double) * std::max(hg.V, 1));
        HIPCHK(hipMemsetAsync(g->d.msg, 0, g->msg_bytes() * std::max<int64_t>(hg.E, 1), g->stream));
        HIPCHK(hipMemsetAsync(g->d.bel, 0, sizeof(Belief) * std::max(hg.V, 1), g->stream));
        HIPCHK(hipMemsetAsync(g->d.state, 0, sizeof(RunState), g->stream));
        upload_phi(g.get());
        set_schedule(g.get(), FASTLBP_SCHED_FLOODING, nullptr);
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
    if (kind == FASTLBP_SCHED_RANKED && !edge_rank && g->hg.E > 0) {
        set_error("RANKED needs edge_rank");
        return FASTLBP_E_BAD_SCHEDULE;
    }
    HostPlan keep = g->plan;
    int keep_kind = g->sched_kind;
    try {
        set_schedule(g, kind, edge_rank);
    } catch (OomError &) {
        g->plan = keep;
        g->sched_kind = keep_kind;
        try {
            upload_plan(g);
        } catch (...) {
        }
        set_error("device allocation failed");
        return FASTLBP_E_OOM;
    } catch (DeviceError &e) {
        return device_error(e);
    }
    if (num_levels_out) *num_levels_out = g->plan.num_levels;
    return FASTLBP_OK;
}

int fastlbp_schedule_levels(fastlbp_graph_t g, int32_t *level_of_edge) {
    clear_error();
    if (!g || (!level_of_edge && g->hg.E > 0)) {
        set_error("invalid argument");
        return FASTLBP_E_INVALID_ARG;
    }
    if (g->hg.E) std::memcpy(level_of_edge, g->plan.level_of_edge.data(), sizeof(int32_t) * g->hg.E);
    return FASTLBP_OK;
}

int fastlbp_evidence_set(fastlbp_graph_t g, int32_t n, const int32_t *vars, const int8_t *values) {
    clear_error();
    if (!g || n < 0 || (n > 0 && (!vars || !values))) {
        set_error("invalid argument");
        return FASTLBP_E_INVALID_ARG;
    }
    for (int32_t i = 0; i < n; ++i)
        if (vars[i] < 0 || vars[i] >= g->hg.V || values[i] < -1 || values[i] > 1) {
            set_error("evidence entry " + std::to_string(i) + " out of range");
            return FASTLBP_E_INVALID_ARG;
        }
    for (int32_t i = 0; i < n; ++i) g->hg.evidence[vars[i]] = values[i];
    try {
        upload_phi(g);
    } catch (DeviceError &e) {
        return device_error(e);
    }
    return FASTLBP_OK;
}

int fastlbp_evidence_clear(fastlbp_graph_t g) {
    clear_error();
    if (!g) {
        set_error("graph is NULL");
        return FASTLBP_E_INVALID_ARG;
    }
    std::fill(g->hg.evidence.begin(), g->hg.evidence.end(), int8_t(-1));
    try {
        upload_phi(g);
    } catch (DeviceError &e) {
        return device_error(e);
    }
    return FASTLBP_OK;
}

int fastlbp_run(fastlbp_graph_t g, int32_t max_iters, double tol, double damping, fastlbp_run_stats *stats) {
    clear_error();
    if (!g) {
        set_error("graph is NULL");
        return FASTLBP_E_INVALID_ARG;
    }
    if (max_iters < 0 || !(tol >= 0.0) || !(damping >= 0.0 && damping < 1.0)) {
        set_error("need max_iters >= 0, tol >= 0, 0 <= damping < 1");
        return FASTLBP_E_INVALID_ARG;
    }
    int exec = choose_executor(g);
    try {
        HIPCHK(hipSetDevice(g->opts.device));
        HIPCHK(hipEventRecord(g->ev0, g->stream));
        if (g->precision == FASTLBP_FP32)
            run_dispatch<PolLog32>(g, max_iters, tol, damping, exec);
        else
            run_dispatch<PolLin64>(g, max_iters, tol, damping, exec);
        HIPCHK(hipEventRecord(g->ev1, g->stream));
        HIPCHK(hipMemcpyAsync(g->h_state, g->d.state, sizeof(RunState), hipMemcpyDeviceToHost, g->stream));
        HIPCHK(hipStreamSynchronize(g->stream));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, g->ev0, g->ev1));
        fastlbp_run_stats s{};
        s.iterations = g->h_state->iter;
        s.converged = g->h_state->converged;
        s.residual = g->h_state->last_r;
        s.contradictions = (int64_t)g->h_state->contra;
        s.levels = g->plan.num_levels;
        s.executor = exec;
        s.algorithmic_bytes_per_iter = g->plan.bytes_per_iter;
        s.device_ms = ms;
        s.message_updates = g->plan.updates_per_iter * int64_t(s.iterations);
        g->last = s;
        if (stats) *stats = s;
    } catch (DeviceError &e) {
        return device_error(e);
    }
    return FASTLBP_OK;
}

int fastlbp_marginals(fastlbp_graph_t g, double *p1) {
    clear_error();
    if (!g || (!p1 && g->hg.V > 0)) {
        set_error("invalid argument");
        return FASTLBP_E_INVALID_ARG;
    }
    if (g->hg.V == 0) return FASTLBP_OK;
    try {
        HIPCHK(hipSetDevice(g->opts.device));
        if (g->precision == FASTLBP_FP32)
            launch_init_beliefs<PolLog32>(g, g->view<PolLog32>(0.0));
        else
            launch_init_beliefs<PolLin64>(g, g->view<PolLin64>(0.0));
        k_marginals<<<grid_for(g->hg.V, 256), 256, 0, g->stream>>>(g->d.bel, g->hg.V, g->d.marg);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(p1, g->d.marg, sizeof(double) * g->hg.V, hipMemcpyDeviceToHost, g->stream));
        HIPCHK(hipStreamSynchronize(g->stream));
    } catch (DeviceError &e) {
        return device_error(e);
    }
    return FASTLBP_OK;
}

int fastlbp_messages_get(fastlbp_graph_t g, double *f2v_p1) {
    clear_error();
    if (!g || (!f2v_p1 && g->hg.E > 0)) {
        set_error("invalid argument");
        return FASTLBP_E_INVALID_ARG;
    }
    int64_t E = g->hg.E;
    if (!E) return FASTLBP_OK;
    try {
        std::vector<double> l(E);
        if (g->precision == FASTLBP_FP32) {
            std::vector<float> f(E);
            HIPCHK(hipMemcpyAsync(f.data(), g->d.msg, 4 * E, hipMemcpyDeviceToHost, g->stream));
            HIPCHK(hipStreamSynchronize(g->stream));
            for (int64_t e = 0; e < E; ++e) l[e] = f[e];
        } else {
            HIPCHK(hipMemcpyAsync(l.data(), g->d.msg, 8 * E, hipMemcpyDeviceToHost, g->stream));
            HIPCHK(hipStreamSynchronize(g->stream));
        }
        for (int64_t e = 0; e < E; ++e) {
            if (g->hg.fac_type[g->hg.edge_fac[e]] == FASTLBP_PRIOR)
                f2v_p1[e] = g->hg.fac_param[g->hg.edge_fac[e]];
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
    if (!g || (!f2v_p1 && g->hg.E > 0)) {
        set_error("invalid argument");
        return FASTLBP_E_INVALID_ARG;
    }
    int64_t E = g->hg.E;
    for (int64_t e = 0; e < E; ++e)
        if (!(f2v_p1[e] >= 0.0 && f2v_p1[e] <= 1.0)) {
            set_error("message " + std::to_string(e) + " outside [0,1]");
            return FASTLBP_E_INVALID_ARG;
        }
    if (!E) return FASTLBP_OK;
    try {
        std::vector<double> l(E, 0.0);
        for (int64_t e = 0; e < E; ++e) {
            if (g->hg.fac_type[g->hg.edge_fac[e]] == FASTLBP_PRIOR) continue;
            double p = f2v_p1[e];
            l[e] = (p >= 1.0) ? INFINITY : (p <= 0.0 ? -INFINITY : std::log2(p) - std::log2(1.0 - p));
        }
        if (g->precision == FASTLBP_FP32) {
            std::vector<float> f(l.begin(), l.end());
            HIPCHK(hipMemcpyAsync(g->d.msg, f.data(), 4 * E, hipMemcpyHostToDevice, g->stream));
            HIPCHK(hipStreamSynchronize(g->stream));
        } else {
            HIPCHK(hipMemcpyAsync(g->d.msg, l.data(), 8 * E, hipMemcpyHostToDevice, g->stream));
            HIPCHK(hipStreamSynchronize(g->stream));
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
        HIPCHK(hipMemsetAsync(g->d.msg, 0, g->msg_bytes() * std::max<int64_t>(g->hg.E, 1), g->stream));
        HIPCHK(hipStreamSynchronize(g->stream));
    } catch (DeviceError &e) {
        return device_error(e);
    }
    return FASTLBP_OK;
}

}  // extern "C"
