// Kernels, iteration driver and the C ABI of libfastlbp (the Kernel Launch and Message Passing
// stages of Section 4.1, executed as described in Section 4.3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "exec.h"
#include "fastlbp.h"
#include "host.h"
#include "internal.h"

namespace fastlbp {


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

// The device plan of a schedule whose levels are known (the task lists and records for the given
// bucket cut-offs).
std::shared_ptr<Plan> plan_from_levels(const Structure &S, const Alloc &alloc, hipStream_t s, int kind,
                                       const std::vector<int32_t> &level, int32_t n, const PlanParams &pp) {
    auto P = std::make_shared<Plan>();
    P->pool.alloc = alloc;
    P->kind = kind;
    P->hp.build(S.hg, level, n, kind == FASTLBP_SCHED_FLOODING, int(S.msg_bytes()), int(2 * S.val_bytes()), pp);
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
    P->frec = P->pool.upload(P->hp.frec, s, sizeof(FacRec) / 4);
    P->vrec = P->pool.upload(P->hp.vrec, s, sizeof(VarRec) / 4);
    P->frec_off = P->pool.upload(P->hp.frec_off, s);
    P->vrec_off = P->pool.upload(P->hp.vrec_off, s);
    P->prec = P->pool.upload(P->hp.prec, s, sizeof(VarRecP) / 4);
    P->level_lds = P->pool.upload(P->hp.level_lds, s);
    P->trec = P->pool.upload(P->hp.trec, s, sizeof(TermRec) / 4);
    P->trec_off = P->pool.upload(P->hp.trec_off, s);
    P->drec = P->pool.upload(P->hp.drec, s, sizeof(VarRec) / 4);
    P->drec_off = P->pool.upload(P->hp.drec_off, s);
    P->dedge = P->pool.upload(P->hp.dedge, s);
    P->dwave = P->pool.upload(P->hp.dwave, s);
    P->dwave_off = P->pool.upload(P->hp.dwave_off, s);
    return P;
}

static std::shared_ptr<Plan> make_plan(const Structure &S, const Alloc &alloc, hipStream_t s, int kind,
                                       const int32_t *rank, const PlanParams &pp) {
    std::vector<int32_t> level;
    int32_t n = analyze_levels(S.hg.V, S.hg.F, S.hg.fac_off.data(), S.hg.edge_var.data(),
                               kind == FASTLBP_SCHED_FLOODING ? nullptr : rank, level);
    return plan_from_levels(S, alloc, s, kind, level, n, pp);
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
    g->prev = g->P->hp.has_delta ? g->state.get(2 * mb) : nullptr;  // (new, old) pairs
    HIPCHK(hipMemsetAsync(g->msg, 0, mb, g->L.stream));
    HIPCHK(hipMemsetAsync(g->bel, 0, sizeof(Belief) * std::max(hg.V, 1), g->L.stream));
    HIPCHK(hipMemsetAsync(g->st, 0, sizeof(RunState), g->L.stream));
    upload_phi(g);
    g->state_nominal = g->state.bytes;
}

// Frees the handle's device state after copying its messages (exact bytes) to host memory. The
// captured iterations hold the old addresses and go too.
void graph_evict(fastlbp_graph *g) {
    if (!g->resident) return;
    hipStream_t s = g->L.stream;
    HIPCHK(hipStreamSynchronize(s));
    const size_t mb = g->S->msg_bytes() * std::max<int64_t>(g->hg().E, 1);
    g->host_msg.resize(mb);
    HIPCHK(hipMemcpyAsync(g->host_msg.data(), g->msg, mb, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    g->drop_graph();
    g->state.release();
    g->phi = g->bel = nullptr;
    g->msg = nullptr;
    g->prev = nullptr;
    g->st = nullptr;
    g->marg = nullptr;
    g->resident = false;
}

// Allocates the device state again and puts the evicted messages back; the potentials come from
// the handle's evidence, the beliefs are rebuilt by the next run. On failure the handle stays
// evicted.
void graph_restore(fastlbp_graph *g) {
    if (g->resident) return;
    try {
        alloc_state(g);
        HIPCHK(hipMemcpyAsync(g->msg, g->host_msg.data(), g->host_msg.size(), hipMemcpyHostToDevice, g->L.stream));
        HIPCHK(hipStreamSynchronize(g->L.stream));
    } catch (...) {
        g->state.release();
        g->phi = g->bel = nullptr;
        g->msg = nullptr;
        g->prev = nullptr;
        g->st = nullptr;
        g->marg = nullptr;
        throw;
    }
    std::vector<unsigned char>().swap(g->host_msg);
    g->resident = true;
}

bool graph_resident(fastlbp_graph *g) { return g->resident; }
void graph_set_manager(fastlbp_graph *g, fastlbp_server *s) { g->mgr = s; }
fastlbp_server *graph_manager(fastlbp_graph *g) { return g->mgr; }
uint64_t &graph_last_use(fastlbp_graph *g) { return g->last_use; }
std::recursive_mutex &graph_mutex(fastlbp_graph *g) { return g->mu; }


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

// Fixed device area of fastlbp_run_noalloc, one copy per device, held until the process ends:
// the run state at offset 0, then the persistent executor's launch descriptor and state header.
// Host code reaches it only through the address hipGetSymbolAddress returns for the device.
constexpr size_t kScratchStateOffset = 0;
constexpr size_t kScratchDescOffset = (sizeof(RunState) + 255) & ~size_t(255);
constexpr size_t kScratchDescBytes = FASTLBP_NOALLOC_SCRATCH_BYTES - kScratchDescOffset;
static_assert(kScratchDescBytes >= sizeof(RunDesc<PolLin64>) + kRunStateHeader &&
                  kScratchDescBytes >= sizeof(RunDesc<PolLog32>) + kRunStateHeader,
              "the scratch area holds one run state, one descriptor and one state header");
static_assert(kFixedHostBytes >= sizeof(RunDesc<PolLin64>) + kRunStateHeader &&
                  kFixedHostBytes >= sizeof(RunDesc<PolLog32>) + kRunStateHeader,
              "the pinned staging holds one descriptor and one state header");
static __device__ __align__(256) unsigned char scratch[FASTLBP_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on `device` (current), looked up once per device.
static void *noalloc_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) throw DeviceError{"device ordinal beyond the scratch table"};
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            throw DeviceError{std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
        }
        g_scratch_ptr[device] = p;
    }
    return g_scratch_ptr[device];
}

// One run on the executor `exec` (the run state is reset first).
void run_any(fastlbp_graph *g, int32_t max_iters, double tol, double damping, int exec) {
    const bool f32 = g->precision() == FASTLBP_FP32;
    if (exec == FASTLBP_EXEC_LEVELS || exec == FASTLBP_EXEC_HYBRID) {
        const bool fuse = exec == FASTLBP_EXEC_HYBRID;
        if (f32)
            levels_run_f32(g, max_iters, tol, damping, fuse, false);
        else
            levels_run_f64(g, max_iters, tol, damping, fuse, false);
        return;
    }
    k_run_init_step<<<1, 64, 0, g->L.stream>>>(g->st, max_iters, tol, max_iters);
    HIPCHK(hipGetLastError());
    fastlbp_graph *one[1] = {g};
    if (f32)
        persistent_launch_f32(g->L, 1, one, &damping, 0);
    else
        persistent_launch_f64(g->L, 1, one, &damping, 0);
}

static int device_error(const DeviceError &e) {
    set_error(e.msg);
    return FASTLBP_E_DEVICE;
}

static void fill_stats(fastlbp_graph *g, int exec, float ms, double damping, fastlbp_run_stats &s) {
    s = fastlbp_run_stats{};
    s.iterations = g->h_state->iter;
    s.converged = g->h_state->converged;
    s.residual = g->h_state->last_r;
    s.contradictions = (int64_t)g->h_state->contra;
    s.levels = g->P->hp.num_levels;
    s.executor = exec;
    s.impl_bytes_per_iter = g->P->hp.bytes_per_iter;
    s.method_bytes_per_iter =
        g->P->hp.method_bytes_per_iter(int(g->S->msg_bytes()), g->h_state->tol > 0.0 || damping > 0.0);
    s.device_ms = ms;
    s.message_updates = g->P->hp.updates_per_iter * int64_t(s.iterations);
    s.thread_max_degree = g->P->hp.params.thread_max_deg;
    s.wave_max_degree = g->P->hp.params.wave_max_deg;
    s.var_thread_max_degree = g->P->hp.params.var_thread_max_deg;
    s.graph_iters = g->tune_graph_iters;
    s.persistent_threads = g->tune_threads;
    s.tuned = g->tuned ? 1 : 0;
    g->last = s;
}

// ---- used by the server ----------------------------------------------------------------------

void step_begin(fastlbp_graph *g, int32_t max_iters, double tol, int32_t step) {
    k_run_init_step<<<1, 64, 0, g->L.stream>>>(g->st, max_iters, tol, step);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(g->L.stream));
    g->h_state->iter = 0;
    g->h_state->done = max_iters <= 0 ? 1 : 0;
    g->h_state->converged = 0;
}

double graph_method_bytes_per_iter(fastlbp_graph *g, double tol, double damping) {
    return g->P->hp.method_bytes_per_iter(int(g->S->msg_bytes()), tol > 0.0 || damping > 0.0);
}

void step_run(Launcher &lc, int n, fastlbp_graph *const *gs, const double *damping, const int32_t *steps) {
    if (gs[0]->precision() == FASTLBP_FP32)
        persistent_launch_f32(lc, n, gs, damping, 0, nullptr, steps);
    else
        persistent_launch_f64(lc, n, gs, damping, 0, nullptr, steps);
}

int32_t graph_exec_levels(fastlbp_graph *g) { return g->P->hp.exec_levels; }
int32_t graph_launches_per_iter(fastlbp_graph *g) {
    return choose_executor(g) == FASTLBP_EXEC_HYBRID ? g->P->hp.launches_hybrid : g->P->hp.launches_levels;
}

bool graph_wide(fastlbp_graph *g) { return choose_executor(g) != FASTLBP_EXEC_PERSISTENT; }

void step_levels_enqueue(fastlbp_graph *g, double damping, int32_t iters) {
    if (g->precision() == FASTLBP_FP32)
        levels_step_f32(g, damping, iters);
    else
        levels_step_f64(g, damping, iters);
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
        init_beliefs_f32(g);
    else
        init_beliefs_f64(g);
}

void marginals_into(fastlbp_graph *g, double *p1) {
    if (g->hg().V == 0) return;
    refresh_beliefs(g);
    k_marginals<<<grid_for(g->hg().V, 256), 256, 0, g->L.stream>>>(g->bel, g->hg().V, g->marg);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(p1, g->marg, sizeof(double) * g->hg().V, hipMemcpyDeviceToHost, g->L.stream));
    HIPCHK(hipStreamSynchronize(g->L.stream));
}

void fill_stats_public(fastlbp_graph *g, fastlbp_run_stats &s, float ms, double damping) {
    fill_stats(g, choose_executor(g), ms, damping, s);
}

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
    if (!g->resident) return FASTLBP_OK;  // the potentials are rebuilt from the evidence on restore
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
    HIPCHK(hipHostMalloc((void **)&g->h_fixed, kFixedHostBytes, hipHostMallocDefault));
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
        g->P = make_plan(*S, g->alloc, s, FASTLBP_SCHED_FLOODING, nullptr, g->pparams);
        g->evidence.assign(hg.V, -1);
        HIPCHK(hipHostMalloc((void **)&g->h_state, sizeof(RunState), hipHostMallocDefault));
        HIPCHK(hipHostMalloc((void **)&g->h_fixed, kFixedHostBytes, hipHostMallocDefault));
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
    g->pparams = src->pparams;
    g->tune_graph_iters = src->tune_graph_iters;
    g->tune_threads = src->tune_threads;
    g->tuned = src->tuned;
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

int fastlbp_graph_get_info(fastlbp_graph_t g, fastlbp_graph_info *out) {
    clear_error();
    if (!g || !out) {
        set_error("invalid argument");
        return FASTLBP_E_INVALID_ARG;
    }
    std::lock_guard<std::recursive_mutex> lk(g->mu);
    std::memset(out, 0, sizeof(*out));
    out->num_vars = g->hg().V;
    out->num_factors = g->hg().F;
    out->num_edges = g->hg().E;
    out->precision = g->precision();
    out->resident = g->resident ? 1 : 0;
    out->state_bytes = g->state_nominal;
    out->structure_bytes = g->S->pool.bytes;
    out->plan_bytes = g->P->pool.bytes;
    out->levels = g->P->hp.num_levels;
    out->executed_levels = g->P->hp.exec_levels;
    return FASTLBP_OK;
}

void fastlbp_graph_destroy(fastlbp_graph_t g) {
    if (!g) return;
    if (g->mgr) server_forget(g->mgr, g);
    delete g;
}

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
    std::lock_guard<std::recursive_mutex> lk(g->mu);
    try {
        HIPCHK(hipSetDevice(g->opts.device));
        HIPCHK(hipStreamSynchronize(g->L.stream));
        auto P = make_plan(*g->S, g->alloc, g->L.stream, kind, edge_rank, g->pparams);
        if (P->hp.has_delta && !g->prev && g->resident) {  // old values for the incremental variable tasks
            g->prev = g->state.get(2 * g->S->msg_bytes() * std::max<int64_t>(g->hg().E, 1));  // (new, old) pairs
            g->state_nominal = g->state.bytes;
        }
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
    std::lock_guard<std::recursive_mutex> lk(g->mu);
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
    std::lock_guard<std::recursive_mutex> lk(g->mu);
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
    std::lock_guard<std::recursive_mutex> lk(g->mu);
    try {
        graph_restore(g);
        HIPCHK(hipSetDevice(g->opts.device));
        hipStream_t s = g->L.stream;
        HIPCHK(hipEventRecord(g->L.ev0, s));
        run_any(g, max_iters, tol, damping, exec);
        HIPCHK(hipEventRecord(g->L.ev1, s));
        HIPCHK(hipMemcpyAsync(g->h_state, g->st, kRunStateHeader, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, g->L.ev0, g->L.ev1));
        fastlbp_run_stats st;
        fill_stats(g, exec, ms, damping, st);
        if (stats) *stats = st;
    } catch (OomError &) {
        set_error("device allocation failed");
        return FASTLBP_E_OOM;
    } catch (DeviceError &e) {
        return device_error(e);
    }
    return FASTLBP_OK;
}

// Runs like fastlbp_run without allocating: the run state (iteration counters, residual and
// contradiction partials) and the persistent executor's launch descriptor live in the device's
// fixed scratch area, the descriptor is staged through the handle's pinned buffer allocated at
// creation, and the LEVELS and HYBRID executors launch their kernels directly instead of replaying
// a captured hipGraph. The handle's own run state is left untouched.
int fastlbp_run_noalloc(fastlbp_graph_t g, int32_t max_iters, double tol, double damping, fastlbp_run_stats *stats) {
    clear_error();
    if (!g) {
        set_error("graph is NULL");
        return FASTLBP_E_INVALID_ARG;
    }
    int rc = check_run_args(max_iters, tol, damping);
    if (rc) return rc;
    std::lock_guard<std::recursive_mutex> lk(g->mu);
    if (!g->resident) {  // restoring would allocate
        set_error("the handle's device state is evicted; any other call on it restores it");
        return FASTLBP_E_STATE;
    }
    const int exec = choose_executor(g);
    RunState *const own = g->st;
    try {
        HIPCHK(hipSetDevice(g->opts.device));
        unsigned char *area = (unsigned char *)noalloc_scratch(g->opts.device);
        hipStream_t s = g->L.stream;
        HIPCHK(hipEventRecord(g->L.ev0, s));
        g->st = (RunState *)(area + kScratchStateOffset);
        const bool f32 = g->precision() == FASTLBP_FP32;
        if (exec == FASTLBP_EXEC_LEVELS || exec == FASTLBP_EXEC_HYBRID) {
            const bool fuse = exec == FASTLBP_EXEC_HYBRID;
            if (f32)
                levels_run_f32(g, max_iters, tol, damping, fuse, true);
            else
                levels_run_f64(g, max_iters, tol, damping, fuse, true);
        } else {
            k_run_init_step<<<1, 64, 0, s>>>(g->st, max_iters, tol, max_iters);
            HIPCHK(hipGetLastError());
            const FixedArea fa = {area + kScratchDescOffset, kScratchDescBytes, g->h_fixed, kFixedHostBytes};
            fastlbp_graph *one[1] = {g};
            if (f32)
                persistent_launch_f32(g->L, 1, one, &damping, 0, &fa);
            else
                persistent_launch_f64(g->L, 1, one, &damping, 0, &fa);
        }
        HIPCHK(hipEventRecord(g->L.ev1, s));
        HIPCHK(hipMemcpyAsync(g->h_state, g->st, kRunStateHeader, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        g->st = own;
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, g->L.ev0, g->L.ev1));
        fastlbp_run_stats st;
        fill_stats(g, exec, ms, damping, st);
        if (stats) *stats = st;
    } catch (OomError &) {
        g->st = own;
        set_error("allocation attempted by fastlbp_run_noalloc");
        return FASTLBP_E_OOM;
    } catch (DeviceError &e) {
        g->st = own;
        return device_error(e);
    }
    return FASTLBP_OK;
}

int fastlbp_run_adaptive(fastlbp_graph_t g, int32_t generator, int32_t groups, int32_t every, uint64_t seed,
                         int32_t max_iters, double tol, double damping, fastlbp_run_stats *stats) {
    clear_error();
    if (!g || (generator != FASTLBP_RANKS_RANDOM && generator != FASTLBP_RANKS_RESIDUAL) || groups < 1 ||
        every < 1) {
        set_error("need a graph, a known generator, groups >= 1 and every >= 1");
        return FASTLBP_E_INVALID_ARG;
    }
    int rc = check_run_args(max_iters, tol, damping);
    if (rc) return rc;
    std::lock_guard<std::recursive_mutex> lk(g->mu);
    const HostGraph &hg = g->hg();
    std::vector<int32_t> rank(size_t(std::max<int64_t>(hg.E, 1)), 0);
    std::vector<double> before, after;
    fastlbp_run_stats total{};
    int32_t done = 0;
    for (int32_t block = 0; done < max_iters || (max_iters == 0 && block == 0); ++block) {
        if (generator == FASTLBP_RANKS_RANDOM) {
            ranks_random(hg.F, hg.fac_off.data(), groups, seed, block, rank.data());
        } else if (block == 0) {
            std::fill(rank.begin(), rank.end(), 0);  // no change measured yet: one class (flooding)
        } else {
            ranks_residual(hg.E, before.data(), after.data(), groups, rank.data());
        }
        rc = fastlbp_schedule_set(g, FASTLBP_SCHED_RANKED, rank.data(), nullptr);
        if (rc) return rc;
        if (generator == FASTLBP_RANKS_RESIDUAL) {
            before.resize(size_t(std::max<int64_t>(hg.E, 1)));
            rc = fastlbp_messages_get(g, before.data());
            if (rc) return rc;
        }
        fastlbp_run_stats st;
        rc = fastlbp_run(g, std::min(every, max_iters - done), tol, damping, &st);
        if (rc) return rc;
        if (generator == FASTLBP_RANKS_RESIDUAL) {
            after.resize(size_t(std::max<int64_t>(hg.E, 1)));
            rc = fastlbp_messages_get(g, after.data());
            if (rc) return rc;
        }
        const int32_t its = total.iterations + st.iterations;
        const int64_t contra = total.contradictions + st.contradictions, upd = total.message_updates + st.message_updates;
        const double ms = total.device_ms + st.device_ms;
        total = st;
        total.iterations = its;
        total.contradictions = contra;
        total.message_updates = upd;
        total.device_ms = ms;
        done += st.iterations;
        if (st.converged || max_iters == 0) break;
    }
    if (stats) *stats = total;
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
    std::vector<std::unique_lock<std::recursive_mutex>> locks;
    for (int32_t i = 0; i < n; ++i) locks.emplace_back(graphs[i]->mu);
    try {
        HIPCHK(hipSetDevice(g0->opts.device));
        for (int32_t i = 0; i < n; ++i) graph_restore(graphs[i]);
        for (int32_t i = 0; i < n; ++i) HIPCHK(hipStreamSynchronize(graphs[i]->L.stream));
        hipStream_t s = g0->L.stream;
        for (int32_t i = 0; i < n; ++i) k_run_init_step<<<1, 64, 0, s>>>(graphs[i]->st, max_iters, tol, max_iters);
        HIPCHK(hipGetLastError());
        HIPCHK(hipEventRecord(g0->L.ev0, s));
        std::vector<double> damps(n, damping);
        if (g0->precision() == FASTLBP_FP32)
            persistent_launch_f32(g0->L, n, graphs, damps.data(), 0);
        else
            persistent_launch_f64(g0->L, n, graphs, damps.data(), 0);
        HIPCHK(hipEventRecord(g0->L.ev1, s));
        HIPCHK(hipStreamSynchronize(s));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, g0->L.ev0, g0->L.ev1));
        for (int32_t i = 0; i < n; ++i) {  // host state headers were refreshed by the launch
            fastlbp_run_stats st;
            fill_stats(graphs[i], FASTLBP_EXEC_PERSISTENT, ms, damping, st);
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
    std::lock_guard<std::recursive_mutex> lk(g->mu);
    try {
        graph_restore(g);
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
    std::lock_guard<std::recursive_mutex> lk(g->mu);
    try {
        graph_restore(g);
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
    std::lock_guard<std::recursive_mutex> lk(g->mu);
    try {
        graph_restore(g);
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
    std::lock_guard<std::recursive_mutex> lk(g->mu);
    try {
        graph_restore(g);
        HIPCHK(hipMemsetAsync(g->msg, 0, g->S->msg_bytes() * std::max<int64_t>(g->hg().E, 1), g->L.stream));
        HIPCHK(hipStreamSynchronize(g->L.stream));
    } catch (DeviceError &e) {
        return device_error(e);
    }
    return FASTLBP_OK;
}

}  // extern "C"
