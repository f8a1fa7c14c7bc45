// BINGO's alarm-ranking loop (Section 5.2.2, Section 5.3): belief propagation, pick the most likely
// uninspected alarm on the device, clamp the user's answer, repeat.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <string>
#include <vector>

#include "fastlbp.h"
#include "host.h"
#include "internal.h"
#include "kernels.h"

namespace fastlbp {

#define ALCHK(x)                                                                                           \
    do {                                                                                                   \
        hipError_t _e = (x);                                                                               \
        if (_e != hipSuccess) throw DeviceError{std::string(#x) + ": " + hipGetErrorString(_e)};           \
    } while (0)

struct AlarmPick {
    int32_t pos;  // position in the alarm list, -1 when every alarm is inspected
    int32_t pad;
    double p1;    // its marginal
};

// better(a, b): higher marginal first, then the lower position
__device__ __forceinline__ bool pick_better(double pa, int32_t ia, double pb, int32_t ib) {
    return pa > pb || (pa == pb && ia < ib);
}

// One workgroup: the uninspected alarm with the highest marginal (Eq.(3) from the beliefs), marked
// inspected. Thread t scans positions t, t + NT, ... in ascending order, so within a thread a tie
// keeps the lower position; the reduction orders (marginal, position) the same way.
constexpr int kPickThreads = 1024;
__global__ __launch_bounds__(kPickThreads) void k_alarm_pick(const Belief *bel, const int32_t *alarm_vars,
                                                             int8_t *inspected, int32_t A, AlarmPick *out) {
    __shared__ double s_p[kPickThreads / 64];
    __shared__ int32_t s_i[kPickThreads / 64];
    double bp = -1.0;
    int32_t bi = 0x7fffffff;
    for (int32_t i = threadIdx.x; i < A; i += kPickThreads) {
        if (inspected[i]) continue;
        const double p = belief_p1(bel[alarm_vars[i]]);
        if (pick_better(p, i, bp, bi)) {
            bp = p;
            bi = i;
        }
    }
#pragma unroll
    for (int k = 32; k >= 1; k >>= 1) {
        const double op = __shfl_xor(bp, k, 64);
        const int32_t oi = __shfl_xor(bi, k, 64);
        if (pick_better(op, oi, bp, bi)) {
            bp = op;
            bi = oi;
        }
    }
    if ((threadIdx.x & 63) == 0) {
        s_p[threadIdx.x >> 6] = bp;
        s_i[threadIdx.x >> 6] = bi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kPickThreads / 64; ++w)
            if (pick_better(s_p[w], s_i[w], bp, bi)) {
                bp = s_p[w];
                bi = s_i[w];
            }
        const bool found = bi < A;
        out->pos = found ? bi : -1;
        out->p1 = found ? bp : 0.0;
        if (found) inspected[bi] = 1;
    }
}

}  // namespace fastlbp

using namespace fastlbp;

int fastlbp_alarm_loop(fastlbp_graph_t g, int32_t A, const int32_t *alarm_vars, const int8_t *labels,
                       int32_t max_rounds, int32_t max_iters, double tol, double damping, int32_t *out_order,
                       double *out_prob, fastlbp_alarm_stats *stats) {
    clear_error();
    if (!g || A < 1 || !alarm_vars || !labels || max_rounds < 0 || (max_rounds > 0 && !out_order)) {
        set_error("need a graph, num_alarms >= 1, alarm_vars, labels, max_rounds >= 0 and out_order");
        return FASTLBP_E_INVALID_ARG;
    }
    const int32_t V = graph_num_vars(g);
    std::vector<uint8_t> seen(size_t(V > 0 ? V : 1), 0);
    int32_t total_true = 0;
    for (int32_t i = 0; i < A; ++i) {
        if (alarm_vars[i] < 0 || alarm_vars[i] >= V || seen[alarm_vars[i]]) {
            set_error("alarm " + std::to_string(i) + ": variable out of range or repeated");
            return FASTLBP_E_INVALID_ARG;
        }
        seen[alarm_vars[i]] = 1;
        if (labels[i] != 0 && labels[i] != 1) {
            set_error("alarm " + std::to_string(i) + ": label outside {0, 1}");
            return FASTLBP_E_INVALID_ARG;
        }
        total_true += labels[i];
    }
    if (max_iters < 0 || !(tol >= 0.0) || !(damping >= 0.0 && damping < 1.0)) {
        set_error("need max_iters >= 0, tol >= 0, 0 <= damping < 1");
        return FASTLBP_E_INVALID_ARG;
    }
    std::lock_guard<std::recursive_mutex> lk(graph_mutex(g));
    const auto t0 = std::chrono::steady_clock::now();
    fastlbp_alarm_stats st{};
    const Alloc &al = graph_alloc(g);
    int32_t *d_vars = nullptr;
    int8_t *d_insp = nullptr;
    AlarmPick *d_pick = nullptr, *h_pick = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = FASTLBP_OK;
    try {
        ALCHK(hipSetDevice(graph_device(g)));
        graph_restore(g);
        hipStream_t s = graph_stream(g);
        d_vars = (int32_t *)al.get(sizeof(int32_t) * size_t(A));
        d_insp = (int8_t *)al.get(size_t(A));
        d_pick = (AlarmPick *)al.get(sizeof(AlarmPick));
        if (!d_vars || !d_insp || !d_pick) throw OomError{};
        ALCHK(hipHostMalloc((void **)&h_pick, sizeof(AlarmPick), hipHostMallocDefault));
        ALCHK(hipEventCreate(&e0));
        ALCHK(hipEventCreate(&e1));
        ALCHK(hipMemcpyAsync(d_vars, alarm_vars, sizeof(int32_t) * size_t(A), hipMemcpyHostToDevice, s));
        ALCHK(hipMemsetAsync(d_insp, 0, size_t(A), s));
        ALCHK(hipStreamSynchronize(s));
        while (st.rounds < max_rounds && st.true_found < total_true) {
            fastlbp_run_stats rs;
            rc = fastlbp_run(g, max_iters, tol, damping, &rs);
            if (rc) break;
            st.iterations += rs.iterations;
            st.message_updates += rs.message_updates;
            st.device_ms += rs.device_ms;
            st.method_bytes += rs.method_bytes_per_iter * double(rs.iterations);
            ALCHK(hipEventRecord(e0, s));
            refresh_beliefs(g);  // the marginals of Eq.(3) exactly as fastlbp_marginals reports them
            k_alarm_pick<<<1, kPickThreads, 0, s>>>(graph_beliefs(g), d_vars, d_insp, A, d_pick);
            ALCHK(hipGetLastError());
            ALCHK(hipEventRecord(e1, s));
            ALCHK(hipMemcpyAsync(h_pick, d_pick, sizeof(AlarmPick), hipMemcpyDeviceToHost, s));
            ALCHK(hipStreamSynchronize(s));
            float ms = 0.f;
            ALCHK(hipEventElapsedTime(&ms, e0, e1));
            st.device_ms += ms;
            const int32_t pos = h_pick->pos;
            if (pos < 0 || pos >= A) break;  // every alarm inspected
            out_order[st.rounds] = pos;
            if (out_prob) out_prob[st.rounds] = h_pick->p1;
            const int8_t lab = labels[pos];
            rc = set_evidence(g, 1, &alarm_vars[pos], &lab);
            if (rc) break;
            st.rounds++;
            st.true_found += lab;
        }
    } catch (OomError &) {
        set_error("device allocation failed");
        rc = FASTLBP_E_OOM;
    } catch (DeviceError &e) {
        set_error(e.msg);
        rc = FASTLBP_E_DEVICE;
    }
    if (graph_stream(g)) (void)hipStreamSynchronize(graph_stream(g));
    al.put(d_vars);
    al.put(d_insp);
    al.put(d_pick);
    if (h_pick) (void)hipHostFree(h_pick);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    st.wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = st;
    return rc;
}
