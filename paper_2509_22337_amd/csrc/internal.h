// Internal interface between the runtime (kernels, graph handles) and the serving loop.
#pragma once
#include <hip/hip_runtime_api.h>

#include <cstddef>
#include <cstdint>
#include <mutex>
#include <string>

#include "fastlbp.h"
#include "layout.h"

namespace fastlbp {

// Device allocator: the caller's callbacks (e.g. a framework's caching allocator) or hipMalloc.
struct Alloc {
    void *(*fn_alloc)(size_t, void *) = nullptr;
    void (*fn_free)(void *, void *) = nullptr;
    void *ctx = nullptr;
    void *get(size_t bytes) const {
        if (bytes == 0) bytes = 16;
        if (fn_alloc) return fn_alloc(bytes, ctx);
        void *p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return p;
    }
    void put(void *p) const {
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

struct Launcher;

void set_error(const std::string &msg);
void clear_error();

// The server drives runs in steps: step_begin resets a handle's run state (iteration 0) for a
// run of max_iters; step_run advances n handles by up to `step` iterations in one persistent
// launch (one workgroup per handle), waits for it and refreshes their pinned host state mirrors
// (graph_host_state); read_state refreshes one handle's mirror (runs stepped elsewhere).
Launcher *launcher_create(int device, hipStream_t s, const Alloc &a);
void launcher_destroy(Launcher *l);
hipStream_t launcher_stream(Launcher *l);
float launcher_kernel_ms(Launcher *l);  // duration of the last persistent launch (HIP events)
void step_begin(fastlbp_graph *g, int32_t max_iters, double tol, int32_t step);
void step_run(Launcher &lc, int n, fastlbp_graph *const *gs, const double *damping, const int32_t *steps);
// Levels one iteration of the handle's schedule executes, and kernel launches of one iteration on
// the LEVELS executor (the server sizes each run's step by them).
int32_t graph_exec_levels(fastlbp_graph *g);
int32_t graph_launches_per_iter(fastlbp_graph *g);
void read_state(fastlbp_graph *g, hipStream_t s);
// Runs whose levels are too wide for one workgroup (the LEVELS executor) are stepped on their own
// stream instead: step_levels_enqueue queues `iters` iterations without waiting, step_levels_finish
// waits for them and returns their device time in ms.
bool graph_wide(fastlbp_graph *g);
void step_levels_enqueue(fastlbp_graph *g, double damping, int32_t iters);
float step_levels_finish(fastlbp_graph *g);
const RunState &graph_host_state(fastlbp_graph *g);
void marginals_into(fastlbp_graph *g, double *p1);
// Rebuilds every belief from phi and the current messages (the executors may leave beliefs that
// were updated incrementally during the last level), on the handle's stream, without waiting.
void refresh_beliefs(fastlbp_graph *g);
void fill_stats_public(fastlbp_graph *g, fastlbp_run_stats &s, float ms, double damping);
int set_evidence(fastlbp_graph *g, int32_t n, const int32_t *vars, const int8_t *values);
int graph_device(fastlbp_graph *g);
int graph_precision(fastlbp_graph *g);
size_t graph_state_bytes(fastlbp_graph *g);
int32_t graph_num_vars(fastlbp_graph *g);
void graph_sync(fastlbp_graph *g);
hipStream_t graph_stream(fastlbp_graph *g);
const Belief *graph_beliefs(fastlbp_graph *g);
const Alloc &graph_alloc(fastlbp_graph *g);
// Residency of a handle's device state (messages, beliefs, potentials, run state): graph_evict
// copies the messages to host memory and frees the state, graph_restore allocates it again and
// puts the messages back (exact bytes, so a warm start survives). graph_mutex is held by every
// public call on the handle; a server evicting an idle handle takes it with try_lock.
void graph_evict(fastlbp_graph *g);
void graph_restore(fastlbp_graph *g);
bool graph_resident(fastlbp_graph *g);
std::recursive_mutex &graph_mutex(fastlbp_graph *g);
// Called by fastlbp_graph_destroy for a handle a server manages: the server drops it from its set.
void server_forget(fastlbp_server *s, fastlbp_graph *g);
void graph_set_manager(fastlbp_graph *g, fastlbp_server *s);
fastlbp_server *graph_manager(fastlbp_graph *g);
uint64_t &graph_last_use(fastlbp_graph *g);
// Method bytes of one iteration of the handle's schedule (fastlbp_run_stats.method_bytes_per_iter).
double graph_method_bytes_per_iter(fastlbp_graph *g, double tol, double damping);

}  // namespace fastlbp
