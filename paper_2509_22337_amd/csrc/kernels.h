// Device code for the two phases of one level (Section 4.3.1): the factor phase computes the
// factor-to-variable messages of the level's active edges (Eq.(2) through the local structure of
// each factor type, Section 3.3), the variable phase refreshes the beliefs that Eq.(1) reads.
//
// Factor algebra. Every non-NOT type is an "any input fires" structure: input j carries weights
// (h_j(x), a_j(x)) for not firing / firing given its value x, and the factor depends on its inputs
// only through s = [some input fired]:
//     OR        h = (1, 0), a = (0, 1)          f(x, y) = [y = s]
//     AND       h = (0, 1), a = (1, 0)          f(x, y) = [y = !s]
//     IMPLIES   h = (0, 1), a = (1, 0)          f = 1 if s; p if !s and y; 1-p if !s and !y
//     NOISY_OR  h = (1, 1-p), a = (0, p)        f = P(y | s): cause-level OR, leak = extra cause
// With normalised input messages m_j, each input contributes a leaf (H_j, F_j) = (sum_x m_j h_j,
// sum_x m_j a_j) with H_j + F_j = 1. Segments combine associatively as
//     (H_L, F_L) * (H_R, F_R) = (H_L H_R, F_L + H_L F_R),
// i.e. "no cause fired in either" and "the first firing cause lies left, or none left and one
// right". All terms are non-negative, so the same scan runs in the log domain without subtraction.
// The message to the head needs the total (H, F); the message to input i needs the product of all
// other leaves, prefix_i * suffix_i, which a forward and a backward scan give in O(degree).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "layout.h"

namespace fastlbp {

enum { T_PRIOR = 0, T_AND = 1, T_OR = 2, T_NOT = 3, T_IMPLIES = 4, T_NOISY_OR = 5 };

// ------------------------------------------------------------------------------------------------
// Precision policies. S: stored message type (LLR in bits). V: value of the factor algebra.
// ------------------------------------------------------------------------------------------------

// float32, log2 domain: V holds log2 of a non-negative real.
struct PolLog32 {
    using S = float;
    using V = float;
    static __device__ __forceinline__ V zero() { return -__builtin_huge_valf(); }
    static __device__ __forceinline__ V one() { return 0.0f; }
    static __device__ __forceinline__ V mul(V a, V b) { return a + b; }
    // log2(2^a + 2^b) without subtraction of large values
    static __device__ __forceinline__ V add(V a, V b) {
        V m = fmaxf(a, b), n = fminf(a, b);
        if (m == -__builtin_huge_valf()) return m;
        return m + __builtin_amdgcn_logf(1.0f + __builtin_amdgcn_exp2f(n - m));
    }
    // normalised pair (log2 mu(0), log2 mu(1)) from an LLR l (bits); exact at l = +-inf
    static __device__ __forceinline__ void leaf(S l, V &m0, V &m1) {
        float t = __builtin_amdgcn_logf(1.0f + __builtin_amdgcn_exp2f(-fabsf(l)));
        m0 = -(fmaxf(l, 0.0f) + t);
        m1 = -(fmaxf(-l, 0.0f) + t);
    }
    static __device__ __forceinline__ S llr(V v0, V v1, bool &contra) {
        contra = (v0 == -__builtin_huge_valf()) && (v1 == -__builtin_huge_valf());
        return contra ? 0.0f : v1 - v0;
    }
    static __device__ __forceinline__ S from_double(double x) { return (float)x; }
    // |P(x=1) under a - P(x=1) under b| for the residual, in float32. With hi >= lo and
    // s(x) = 1 / (1 + 2^-x), s(hi) - s(lo) = s(lo) s(-hi) (2^(hi-lo) - 1): three factors, each to
    // a few ulp, so the difference keeps a relative error of about 1e-6 instead of the absolute
    // 1e-7 of subtracting two rounded probabilities (which would blur a tol of 1e-6).
    static __device__ __forceinline__ double delta_p1(S a, S b) {
        const float hi = fmaxf(a, b), lo = fminf(a, b);
        const float d = hi - lo;
        if (!(d > 0.0f)) return 0.0;
        if (d < 32.0f) {  // both finite here
            const float sl = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-lo));
            const float sh = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(hi));
            float em;
            if (d < 0.25f) {  // 2^d - 1 by its series in x = d ln 2 (x < 0.18, truncation < 3e-7 relative)
                const float x = d * 0.69314718f;
                em = x * (1.0f + x * (0.5f + x * (1.0f / 6.0f + x * (1.0f / 24.0f + x * (1.0f / 120.0f)))));
            } else {
                em = __builtin_amdgcn_exp2f(d) - 1.0f;
            }
            return (double)(sl * sh * em);
        }
        // far apart (or infinite): no cancellation to fear
        const float ph = hi == INFINITY ? 1.0f : __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-hi));
        const float pl = lo == -INFINITY ? 0.0f : __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-lo));
        return (double)(ph - pl);
    }
    // An upper bound of delta_p1(a, b) that costs no transcendental: the slope of P(x=1) in the LLR
    // (bits) is ln2 P (1 - P) <= ln2 / 4 = 0.1732868; 0.1734 leaves room for delta_p1's own rounding
    // (a few ulp relative). Equal infinities (a - b = NaN) give 0, as delta_p1 does.
    static __device__ __forceinline__ double delta_bound(S a, S b) {
        const float d = fabsf(a - b);
        return d > 0.0f ? (double)(d * 0.1734f) : 0.0;
    }
};

// float64, linear domain.
struct PolLin64 {
    using S = double;
    using V = double;
    static __device__ __forceinline__ V zero() { return 0.0; }
    static __device__ __forceinline__ V one() { return 1.0; }
    static __device__ __forceinline__ V mul(V a, V b) { return a * b; }
    static __device__ __forceinline__ V add(V a, V b) { return a + b; }
    static __device__ __forceinline__ void leaf(S l, V &m0, V &m1) {
        double e = exp2(-fabs(l));
        double r = 1.0 / (1.0 + e);
        if (l >= 0.0) {
            m1 = r;
            m0 = e * r;
        } else {
            m0 = r;
            m1 = e * r;
        }
    }
    static __device__ __forceinline__ S llr(V v0, V v1, bool &contra) {
        contra = (v0 == 0.0) && (v1 == 0.0);
        return contra ? 0.0 : log2(v1) - log2(v0);
    }
    static __device__ __forceinline__ S from_double(double x) { return x; }
    static __device__ __forceinline__ double delta_p1(S a, S b) {
        return fabs(1.0 / (1.0 + exp2(-a)) - 1.0 / (1.0 + exp2(-b)));
    }
    // Upper bound of delta_p1(a, b) (slope of P(x=1) in the LLR at most ln2 / 4), with an absolute
    // margin for the rounding of the difference of two probabilities.
    static __device__ __forceinline__ double delta_bound(S a, S b) {
        const double d = fabs(a - b);
        return d > 0.0 ? d * 0.1734 + 1e-15 : 0.0;
    }
};

// P(x = 1) of an LLR in bits, in float64 (used for the residual).
__device__ __forceinline__ double prob1(double l) { return 1.0 / (1.0 + exp2(-l)); }

// Marginal P(x = 1) of Eq.(3) from a belief; a belief with both infinite kinds (0/0) gives 1/2.
__device__ __forceinline__ double belief_p1(const Belief &B) {
    if (B.npos > 0 && B.nneg > 0) return 0.5;
    if (B.npos > 0) return 1.0;
    if (B.nneg > 0) return 0.0;
    return 1.0 / (1.0 + exp2(-B.fin));
}

// Variable-to-factor message of Eq.(1) from the variable's belief minus the factor's own incoming
// message. `null` marks the product of two exact zeros (0, 0).
template <class P>
__device__ __forceinline__ typename P::S v2f(const Belief &B, typename P::S own, bool &null) {
    using S = typename P::S;
    const S inf = (S)__builtin_huge_val();
    int np = B.npos - (own == inf ? 1 : 0);
    int nn = B.nneg - (own == -inf ? 1 : 0);
    null = (np > 0) && (nn > 0);
    if (null) return (S)0;
    if (np > 0) return inf;
    if (nn > 0) return -inf;
    double f = B.fin - ((own == inf || own == -inf) ? 0.0 : (double)own);
    return P::from_double(f);
}

template <class V>
struct HF {
    V h, f;
};

template <class P>
__device__ __forceinline__ HF<typename P::V> combine(HF<typename P::V> L, HF<typename P::V> R) {
    return {P::mul(L.h, R.h), P::add(L.f, P::mul(L.h, R.f))};
}

template <class P>
__device__ __forceinline__ HF<typename P::V> identity() {
    return {P::one(), P::zero()};
}

// Leaf of input j from its normalised message (m0, m1).
template <class P>
__device__ __forceinline__ HF<typename P::V> make_leaf(int type, typename P::V m0, typename P::V m1,
                                                       const Pair<typename P::V> &ep) {
    if (type == T_OR) return {m0, m1};
    if (type == T_NOISY_OR) return {P::add(m0, P::mul(m1, ep.b)), P::mul(m1, ep.a)};
    return {m1, m0};  // AND, IMPLIES: an input fires when it is 0
}

// Unnormalised message to the head from the total (H, F) of all inputs (leak included).
template <class P>
__device__ __forceinline__ void head_msg(int type, HF<typename P::V> t, const Pair<typename P::V> &fp,
                                         typename P::V &o0, typename P::V &o1) {
    if (type == T_OR || type == T_NOISY_OR) {
        o0 = t.h;
        o1 = t.f;
    } else if (type == T_AND) {
        o0 = t.f;
        o1 = t.h;
    } else {  // IMPLIES: fp = (p, 1-p)
        o0 = P::add(P::mul(fp.b, t.h), t.f);
        o1 = P::add(P::mul(fp.a, t.h), t.f);
    }
}

// Unnormalised message to input i from the product x of the other inputs' leaves (leak included),
// the head's normalised message (my0, my1) and the input's own parameters.
template <class P>
__device__ __forceinline__ void input_msg(int type, HF<typename P::V> x, typename P::V my0, typename P::V my1,
                                          const Pair<typename P::V> &fp, const Pair<typename P::V> &ep,
                                          typename P::V &o0, typename P::V &o1) {
    using V = typename P::V;
    if (type == T_OR || type == T_NOISY_OR) {
        V base = P::add(P::mul(my0, x.h), P::mul(my1, x.f));  // input i does not fire
        o0 = base;
        o1 = (type == T_OR) ? my1 : P::add(P::mul(ep.b, base), P::mul(ep.a, my1));
    } else if (type == T_AND) {
        o0 = my0;
        o1 = P::add(P::mul(my1, x.h), P::mul(my0, x.f));
    } else {  // IMPLIES
        V s = P::add(my0, my1);
        V wy = P::add(P::mul(my0, fp.b), P::mul(my1, fp.a));
        o0 = s;
        o1 = P::add(P::mul(wy, x.h), P::mul(s, x.f));
    }
}

// Per-thread accumulators of the residual and the contradiction count.
struct Acc {
    double r;
    unsigned int contra;
};

// New stored value of a message from its unnormalised entries (o0, o1): contradiction handling,
// damping against the old value, residual.
template <class P, bool DAMP>
__device__ __forceinline__ typename P::S finish_msg(const DevGraph<typename P::S, typename P::V> &g, typename P::S old,
                                                    typename P::V o0, typename P::V o1, bool force_contra, Acc &acc) {
    using S = typename P::S;
    using V = typename P::V;
    bool contra;
    S l = P::llr(o0, o1, contra);
    if (force_contra) {
        contra = true;
        l = (S)0;
    }
    if (contra) acc.contra++;
    if (DAMP && g.damped) {
        V a0, a1, b0, b1;
        P::leaf(old, a0, a1);
        P::leaf(l, b0, b1);
        bool c2;
        l = P::llr(P::add(P::mul(g.damp_old, a0), P::mul(g.damp_new, b0)),
                   P::add(P::mul(g.damp_old, a1), P::mul(g.damp_new, b1)), c2);
    }
    // the residual is a maximum: a change whose bound cannot raise it needs no exact value
    if (P::delta_bound(l, old) > acc.r) acc.r = fmax(acc.r, P::delta_p1(l, old));
    return l;
}

// The (new, old) pair of a written message, side by side so that an incremental variable task
// fetches both with one request.
template <class S>
struct alignas(2 * sizeof(S)) MsgPair {
    S nw, od;
};

// Stores a new message, and the (new, old) pair where the plan's variable tasks add new - old
// (PAIRS = false: the caller's variable phase never reads pairs, as in the single-workgroup level
// loop, so the code for them is left out).
template <class S, class V, bool PAIRS = true>
__device__ __forceinline__ void put_msg(const DevGraph<S, V> &g, int32_t e, S nw, S old) {
    g.msg[e] = nw;
    if (PAIRS && g.prev.p) GPtr<MsgPair<S>>((MsgPair<S> *)g.prev.p).st(e, MsgPair<S>{nw, old});
}

template <class P, bool DAMP>
__device__ __forceinline__ void store_msg(const DevGraph<typename P::S, typename P::V> &g, int32_t e,
                                          typename P::S old, typename P::V o0, typename P::V o1, bool force_contra,
                                          Acc &acc) {
    put_msg(g, e, finish_msg<P, DAMP>(g, old, o0, o1, force_contra, acc), old);
}

template <bool ALL_ACTIVE>
__device__ __forceinline__ bool is_active(const GPtr<const int32_t> &edge_level, int32_t e, int level) {
    return ALL_ACTIVE || edge_level[e] == level;
}

// NOT factor: the message to y is the input's message reversed, and vice versa.
template <class P, bool ALL_ACTIVE, bool DAMP>
__device__ __forceinline__ void factor_not(const DevGraph<typename P::S, typename P::V> &g, int32_t b, int level, Acc &acc) {
    using S = typename P::S;
    using V = typename P::V;
    S lo[2], vf[2];
    bool nl[2];
    for (int k = 0; k < 2; ++k) {
        lo[k] = g.msg[b + k];
        vf[k] = v2f<P>(g.bel.ld(g.edge_var[b + k]), lo[k], nl[k]);
    }
    for (int k = 0; k < 2; ++k) {
        if (!is_active<ALL_ACTIVE>(g.edge_level, b + k, level)) continue;
        V m0, m1;
        P::leaf(-vf[1 - k], m0, m1);
        store_msg<P, DAMP>(g, b + k, lo[k], m0, m1, nl[1 - k], acc);
    }
}

// ------------------------------------------------------------------------------------------------
// One factor processed by a team of TEAM lanes (TEAM = 1: a single thread; 64: a wavefront;
// > 64: a whole workgroup using `lds`). Lane `lane` owns a contiguous chunk of at most CMAX inputs.
// ------------------------------------------------------------------------------------------------

template <class V>
struct TeamLds {
    HF<V> wave_tot[16];
    HF<V> wave_pre[16];
    HF<V> wave_suf[16];
    int wave_null[16];
    int null_total;
    HF<V> total;
};

template <class P, int TEAM>
struct TeamScan;

// Exclusive prefix and suffix of per-lane aggregates across the team; also the team-wide total and
// the number of null inputs. `init` is the leftmost element (the NOISY_OR leak, else identity).
template <class P>
struct TeamScan<P, 1> {
    using V = typename P::V;
    static __device__ __forceinline__ void run(HF<V> agg, int nnull, HF<V> init, HF<V> &pre, HF<V> &suf, HF<V> &tot, int &ntot,
                               TeamLds<V> *) {
        pre = init;
        suf = identity<P>();
        tot = combine<P>(init, agg);
        ntot = nnull;
    }
};

template <class P>
__device__ __forceinline__ void wave_scans(HF<typename P::V> x, int lane, HF<typename P::V> &incl_pre,
                                           HF<typename P::V> &incl_suf) {
    using V = typename P::V;
    HF<V> p = x, s = x;
#pragma unroll
    for (int k = 1; k < 64; k <<= 1) {
        V ph = __shfl_up(p.h, k, 64), pf = __shfl_up(p.f, k, 64);
        if (lane >= k) p = combine<P>({ph, pf}, p);
        V sh = __shfl_down(s.h, k, 64), sf = __shfl_down(s.f, k, 64);
        if (lane + k < 64) s = combine<P>(s, {sh, sf});
    }
    incl_pre = p;
    incl_suf = s;
}

__device__ __forceinline__ int wave_sum(int x) {
#pragma unroll
    for (int k = 32; k >= 1; k >>= 1) x += __shfl_xor(x, k, 64);
    return x;
}

template <class P>
struct TeamScan<P, 64> {
    using V = typename P::V;
    static __device__ __forceinline__ void run(HF<V> agg, int nnull, HF<V> init, HF<V> &pre, HF<V> &suf, HF<V> &tot, int &ntot,
                               TeamLds<V> *) {
        int lane = threadIdx.x & 63;
        HF<V> ip, is;
        wave_scans<P>(agg, lane, ip, is);
        HF<V> ep = {__shfl_up(ip.h, 1, 64), __shfl_up(ip.f, 1, 64)};
        HF<V> es = {__shfl_down(is.h, 1, 64), __shfl_down(is.f, 1, 64)};
        pre = (lane == 0) ? init : combine<P>(init, ep);
        suf = (lane == 63) ? identity<P>() : es;
        HF<V> all = {__shfl(ip.h, 63, 64), __shfl(ip.f, 63, 64)};
        tot = combine<P>(init, all);
        ntot = wave_sum(nnull);
    }
};

template <class P, int TEAM>
struct TeamScan {
    using V = typename P::V;
    static_assert(TEAM % 64 == 0 && TEAM / 64 <= 16, "team is up to 16 wavefronts");
    static __device__ __forceinline__ void run(HF<V> agg, int nnull, HF<V> init, HF<V> &pre, HF<V> &suf, HF<V> &tot, int &ntot,
                               TeamLds<V> *lds) {
        constexpr int NW = TEAM / 64;
        int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        HF<V> ip, is;
        wave_scans<P>(agg, lane, ip, is);
        HF<V> ep = {__shfl_up(ip.h, 1, 64), __shfl_up(ip.f, 1, 64)};
        HF<V> es = {__shfl_down(is.h, 1, 64), __shfl_down(is.f, 1, 64)};
        int wn = wave_sum(nnull);
        if (lane == 63) lds->wave_tot[w] = ip;
        if (lane == 0) lds->wave_null[w] = wn;
        __syncthreads();
        if (threadIdx.x == 0) {
            HF<V> run = init;
            int nt = 0;
            for (int i = 0; i < NW; ++i) {
                lds->wave_pre[i] = run;
                run = combine<P>(run, lds->wave_tot[i]);
                nt += lds->wave_null[i];
            }
            lds->total = run;
            lds->null_total = nt;
            HF<V> r = identity<P>();
            for (int i = NW - 1; i >= 0; --i) {
                lds->wave_suf[i] = r;
                r = combine<P>(lds->wave_tot[i], r);
            }
        }
        __syncthreads();
        HF<V> wp = lds->wave_pre[w], ws = lds->wave_suf[w];
        pre = (lane == 0) ? wp : combine<P>(wp, ep);
        suf = (lane == 63) ? ws : combine<P>(es, ws);
        tot = lds->total;
        ntot = lds->null_total;
        __syncthreads();  // lds is reused by the next factor
    }
};

// The leaves of SB consecutive inputs of a factor (positions i0 + k0 .. of the edge range starting at
// b, those before i1 valid), with every load issued before any is used: positions past the chunk
// load the lane's first edge instead (b + i0 <= the head edge, always valid) and are masked. ok[j]
// marks the valid positions; x[j] is the identity leaf where a position is invalid or its v->f
// message is null.
template <class P, int SB, int CMAX>
__device__ __forceinline__ void load_leaves(const DevGraph<typename P::S, typename P::V> &g, int type, int32_t b,
                                            int32_t i0, int32_t i1, int k0, HF<typename P::V> (&x)[SB],
                                            typename P::S (&o)[SB], bool (&nl)[SB], bool (&ok)[SB]) {
    using V = typename P::V;
    int32_t v[SB];
    Pair<V> ep[SB];
#pragma unroll
    for (int j = 0; j < SB; ++j) {
        ok[j] = (k0 + j < CMAX) && (i0 + k0 + j < i1);
        const int32_t e = b + (ok[j] ? i0 + k0 + j : i0);
        o[j] = g.msg[e];
        v[j] = g.edge_var[e];
        ep[j] = {P::zero(), P::one()};
        if (type == T_NOISY_OR) ep[j] = g.epar.ld(e);
    }
    Belief B[SB];
#pragma unroll
    for (int j = 0; j < SB; ++j) B[j] = g.bel.ld(v[j]);
#pragma unroll
    for (int j = 0; j < SB; ++j) {
        bool n;
        const typename P::S vf = v2f<P>(B[j], o[j], n);
        V m0, m1;
        P::leaf(vf, m0, m1);
        const HF<V> t = make_leaf<P>(type, m0, m1, ep[j]);
        nl[j] = ok[j] && n;
        const bool id = !ok[j] || n;
        x[j].h = id ? P::one() : t.h;
        x[j].f = id ? P::zero() : t.f;
    }
}

// Writes the messages of the head and of every active input of factor a, NT lanes working together:
// each lane owns a chunk of at most CMAX consecutive inputs, taken in sub-chunks of 4 whose loads are
// issued together. A first pass combines each sub-chunk; the scan across the lanes gives the prefix
// before and the suffix after each lane's chunk; a second pass, over the sub-chunks from last to
// first, reloads each sub-chunk (cache hits) and forms its suffix and exclusive products. Leaves are
// reloaded instead of held so that a 1024-lane workgroup stays within its 128-register budget.
template <class P, int TEAM, int CMAX, bool ALL_ACTIVE, bool DAMP>
__device__ __forceinline__ void factor_team(const DevGraph<typename P::S, typename P::V> &g, int32_t a, int lane, int level,
                            Acc &acc, TeamLds<typename P::V> *lds) {
    using S = typename P::S;
    using V = typename P::V;
    constexpr int SB = 4;                       // sub-chunk length
    constexpr int NS = (CMAX + SB - 1) / SB;    // sub-chunks per lane
    const int32_t b = g.fac_off[a];
    const int32_t d = g.fac_off[a + 1] - b;
    const int type = g.fac_type[a];
    if (type == T_NOT) {
        if (lane == 0) factor_not<P, ALL_ACTIVE, DAMP>(g, b, level, acc);
        return;
    }
    const int32_t n = d - 1;
    const Pair<V> fp = g.fpar.ld(a);
    // head (last edge): its v->f message weights the messages to the inputs
    const int32_t eh = b + n;
    S lh_old = g.msg[eh];
    bool null_h;
    S vfh = v2f<P>(g.bel.ld(g.edge_var[eh]), lh_old, null_h);
    V my0 = P::zero(), my1 = P::zero();
    if (!null_h) P::leaf(vfh, my0, my1);
    // chunk of inputs owned by this lane
    const int32_t c = (n + TEAM - 1) / TEAM;
    const int32_t i0 = min(n, lane * c), i1 = min(n, i0 + c);
    HF<V> sub[NS];  // aggregate of each sub-chunk, later the prefix before it
    int nnull = 0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        sub[s] = identity<P>();
        if (i0 + s * SB < i1) {
            HF<V> x[SB];
            S o[SB];
            bool nl[SB], ok[SB];
            load_leaves<P, SB, CMAX>(g, type, b, i0, i1, s * SB, x, o, nl, ok);
#pragma unroll
            for (int j = 0; j < SB; ++j) {
                nnull += nl[j] ? 1 : 0;
                if (ok[j]) sub[s] = combine<P>(sub[s], x[j]);
            }
        }
    }
    HF<V> agg = sub[0];
#pragma unroll
    for (int s = 1; s < NS; ++s) agg = combine<P>(agg, sub[s]);
    HF<V> init = identity<P>();
    if (type == T_NOISY_OR) init = {fp.b, fp.a};  // the leak: fires with probability leak
    HF<V> pre, suf, tot;
    int ntot;
    TeamScan<P, TEAM>::run(agg, nnull, init, pre, suf, tot, ntot, lds);
    if (lane == 0 && is_active<ALL_ACTIVE>(g.edge_level, eh, level)) {
        V o0, o1;
        head_msg<P>(type, tot, fp, o0, o1);
        store_msg<P, DAMP>(g, eh, lh_old, o0, o1, ntot > 0, acc);
    }
    // prefix before each sub-chunk
    {
        HF<V> run = pre;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            HF<V> t = sub[s];
            sub[s] = run;
            run = combine<P>(run, t);
        }
    }
    // sub-chunks from last to first: suffix inside the sub-chunk, then the exclusive products
    HF<V> rsuf = suf;
#pragma unroll
    for (int s = NS - 1; s >= 0; --s) {
        if (i0 + s * SB >= i1) continue;
        HF<V> x[SB];
        S o[SB];
        bool nl[SB], ok[SB];
        load_leaves<P, SB, CMAX>(g, type, b, i0, i1, s * SB, x, o, nl, ok);
        HF<V> sx[SB];
        HF<V> run = rsuf;
#pragma unroll
        for (int j = SB - 1; j >= 0; --j) {
            sx[j] = run;
            if (ok[j]) run = combine<P>(x[j], run);
        }
        rsuf = run;
        run = sub[s];
#pragma unroll
        for (int j = 0; j < SB; ++j) {
            if (ok[j]) {
                const int32_t e = b + i0 + s * SB + j;
                if (is_active<ALL_ACTIVE>(g.edge_level, e, level)) {
                    HF<V> xo = combine<P>(run, sx[j]);
                    Pair<V> ep = {P::zero(), P::one()};
                    if (type == T_NOISY_OR) ep = g.epar.ld(e);
                    V o0, o1;
                    input_msg<P>(type, xo, my0, my1, fp, ep, o0, o1);
                    int others_null = ntot - (nl[j] ? 1 : 0) + (null_h ? 1 : 0);
                    store_msg<P, DAMP>(g, e, o[j], o0, o1, others_null > 0, acc);
                }
                run = combine<P>(run, x[j]);
            }
        }
    }
}

// Factor given as weighted terms (Eq.(4)): one wavefront per factor, lane k owning edge k (degree
// <= 64). The message to edge k at value x sums, over the terms that admit x at k, the term's
// weight times the product over the other edges of their v->f message at the value the term fixes
// (1 where the term leaves the edge free, the messages being normalised). For each term the product
// over the other edges is the exclusive prefix times the exclusive suffix across the lanes, so it
// costs O(log degree) steps and no division. A null v->f message (two exact zeros) makes every
// other edge's message a contradiction, as in the typed factors.
template <class P, bool ALL_ACTIVE, bool DAMP>
__device__ __forceinline__ void factor_terms(const DevGraph<typename P::S, typename P::V> &g, int32_t a, int lane,
                                             int level, Acc &acc) {
    using S = typename P::S;
    using V = typename P::V;
    const int32_t b = g.fac_off[a];
    const int32_t d = g.fac_off[a + 1] - b;
    const int32_t t0 = g.term_off[a], t1 = g.term_off[a + 1];
    const int32_t ib = g.term_base[a];
    const bool mine = lane < d;
    S old = (S)0;
    bool nl = false;
    V m0 = P::one(), m1 = P::one();
    if (mine) {
        old = g.msg[b + lane];
        const S vf = v2f<P>(g.bel.ld(g.edge_var[b + lane]), old, nl);
        if (!nl) P::leaf(vf, m0, m1);
    }
    const int nnull = wave_sum(nl ? 1 : 0);
    V acc0 = P::zero(), acc1 = P::zero();
    for (int32_t t = t0; t < t1; ++t) {
        const int c = mine ? (int)g.term_ind[ib + int64_t(t - t0) * d + lane] : -1;
        const V f = c < 0 ? P::one() : (c ? m1 : m0);
        // inclusive prefix and suffix products over lanes 0..d-1 (lanes >= d hold the identity)
        V p = f, q = f;
        for (int k = 1; k < d; k <<= 1) {
            const V pu = __shfl_up(p, k, 64);
            const V qd = __shfl_down(q, k, 64);
            if (lane >= k) p = P::mul(pu, p);
            if (lane + k < 64) q = P::mul(q, qd);
        }
        V xp = __shfl_up(p, 1, 64), xq = __shfl_down(q, 1, 64);
        if (lane == 0) xp = P::one();
        if (lane == 63) xq = P::one();
        const V x = P::mul(g.term_w[t], P::mul(xp, xq));
        if (c != 1) acc0 = P::add(acc0, x);
        if (c != 0) acc1 = P::add(acc1, x);
    }
    if (mine && is_active<ALL_ACTIVE>(g.edge_level, b + lane, level))
        store_msg<P, DAMP>(g, b + lane, old, acc0, acc1, nnull - (nl ? 1 : 0) > 0, acc);
}

// Weighted-term factor of degree <= kThreadMaxDeg in one thread, from its task record: for every
// term, a forward pass gives the weight times the product over the edges before k and a backward
// pass the product over the edges after k, so each term costs O(degree) and the factor
// O(terms x degree). Term t's indicators come as the mask pair term_mask[t] (fixed edges, their
// values); the record's mask selects the edges the level writes.
template <class P, bool DAMP>
__device__ __forceinline__ void factor_terms_rec(const DevGraph<typename P::S, typename P::V> &g, const TermRec &r,
                                                 Acc &acc) {
    using S = typename P::S;
    using V = typename P::V;
    constexpr int K = kThreadMaxDeg;
    const int32_t b = r.b;
    const int32_t d = r.meta & 0xff;
    const int32_t t0 = r.t0, t1 = r.t0 + ((r.meta >> 8) & 0xff);
    const unsigned act = ((unsigned)r.meta >> 16) & 0xffu;
    S old[K];
    V m0[K], m1[K], a0[K], a1[K];
    bool nl[K];
    int nnull = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        m0[k] = P::one();
        m1[k] = P::one();
        a0[k] = P::zero();
        a1[k] = P::zero();
        old[k] = (S)0;
        nl[k] = false;
        if (k < d) {
            old[k] = g.msg[b + k];
            const S vf = v2f<P>(g.bel.ld(r.u[k]), old[k], nl[k]);
            if (!nl[k]) P::leaf(vf, m0[k], m1[k]);
            nnull += nl[k] ? 1 : 0;
        }
    }
    for (int32_t t = t0; t < t1; ++t) {
        const unsigned mk = g.term_mask[t];
        V pre[K];
        V run = g.term_w[t];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            pre[k] = run;
            if (k < d && ((mk >> k) & 1u)) run = P::mul(run, ((mk >> (8 + k)) & 1u) ? m1[k] : m0[k]);
        }
        V suf = P::one();
#pragma unroll
        for (int k = K - 1; k >= 0; --k) {
            if (k < d) {
                const bool fix = (mk >> k) & 1u, val = (mk >> (8 + k)) & 1u;
                const V x = P::mul(pre[k], suf);
                if (!fix || !val) a0[k] = P::add(a0[k], x);
                if (!fix || val) a1[k] = P::add(a1[k], x);
                if (fix) suf = P::mul(suf, val ? m1[k] : m0[k]);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (k < d && ((act >> k) & 1u))
            store_msg<P, DAMP>(g, b + k, old[k], a0[k], a1[k], nnull - (nl[k] ? 1 : 0) > 0, acc);
}

// Variable phase: B_v = phi_v + sum of the v's incoming non-PRIOR messages (float64, with counts).
// Branch-free (a wavefront's lanes disagree on which terms are infinite): an infinite term adds to
// its count and 0 to the finite part.
template <class P>
__device__ __forceinline__ void belief_add(Belief &B, typename P::S l) {
    using S = typename P::S;
    const S inf = (S)__builtin_huge_val();
    const bool pi = l == inf, ni = l == -inf;
    B.npos += pi ? 1 : 0;
    B.nneg += ni ? 1 : 0;
    B.fin += (pi || ni) ? 0.0 : (double)l;
}

template <class P>
__device__ __forceinline__ void var_thread(const DevGraph<typename P::S, typename P::V> &g, int32_t v) {
    Belief B = g.phi.ld(v);
    for (int32_t q = g.var_off[v]; q < g.var_off[v + 1]; ++q) belief_add<P>(B, g.msg[g.var_edge[q]]);
    g.bel.st(v, B);
}

// One wavefront per variable (high degree); fixed-shape reduction, so the result is deterministic.
template <class P>
__device__ __forceinline__ void var_wave(const DevGraph<typename P::S, typename P::V> &g, int32_t v, int lane) {
    Belief B = {0.0, 0, 0};
    for (int32_t q = g.var_off[v] + lane; q < g.var_off[v + 1]; q += 64) belief_add<P>(B, g.msg[g.var_edge[q]]);
#pragma unroll
    for (int k = 32; k >= 1; k >>= 1) {
        B.fin += __shfl_xor(B.fin, k, 64);
        B.npos += __shfl_xor(B.npos, k, 64);
        B.nneg += __shfl_xor(B.nneg, k, 64);
    }
    if (lane == 0) {
        Belief p = g.phi.ld(v);
        p.fin += B.fin;
        p.npos += B.npos;
        p.nneg += B.nneg;
        g.bel.st(v, p);
    }
}

// ------------------------------------------------------------------------------------------------
// Record-based thread tasks (both executors). The host packs, per level, one record per factor of
// degree <= 8 and one per variable of degree <= 64 with everything static already resolved (edge
// range, degree, type, the level's active edges, variable ids, first edge ids), so that a thread
// issues all of a task's dynamic loads (messages, beliefs) at once. Records of a level are sorted
// by degree and every degree group is padded to a multiple of 64, so the 64 records a wavefront
// takes share one degree: the degree switch below is then uniform and each case loads exactly its
// degree's operands. (Without the padding, a wavefront straddling two degrees runs both cases one
// after the other, which doubles its chain of dependent loads; on narrow levels the slowest
// wavefront sets the level's time.)
// ------------------------------------------------------------------------------------------------

// One factor of degree D from values in registers: lo[k] the old message of edge b + k, vf[k] its
// variable-to-factor message, nl[k] whether that is the null message. Bit k of `active` selects
// the edges the level writes.
// Puts the new and the old message of active edge k into the level's staging slots (when given).
template <class P>
__device__ __forceinline__ void stage_slot(typename P::S *slots, int32_t slot0, unsigned active, int k,
                                           typename P::S nw, typename P::S old) {
    if (slots) {
        const int32_t i = slot0 + __builtin_popcount(active & ((1u << k) - 1u));
        slots[2 * i] = nw;
        slots[2 * i + 1] = old;
    }
}

// Factor families of the thread path, fixed at compile time so that a wavefront (whose records
// share degree and type) runs straight-line code. FAM_OR covers OR, AND and NOT: AND is OR on the
// negated edges (y = AND(x) iff not y = OR(not x)) and NOT is a one-input OR on its negated input,
// so those edges enter as negated LLRs and their two message entries leave swapped. Swapping the
// pair is exactly the negation the AND and NOT formulas perform, so every stored value equals the
// one the type's own formula gives.
enum { FAM_OR = 0, FAM_IMPLIES = 1, FAM_NOISY = 2 };

template <class P, bool DAMP, int D, int FAM, bool PAIRS>
__device__ __forceinline__ void factor_local(const DevGraph<typename P::S, typename P::V> &g, int type, int32_t b,
                                             unsigned active, const Pair<typename P::V> &fp,
                                             const typename P::S (&lo)[D], const typename P::S (&vf)[D],
                                             const bool (&nl)[D], const Pair<typename P::V> (&ep)[D], Acc &acc,
                                             typename P::S *slots, int32_t slot0) {
    using S = typename P::S;
    using V = typename P::V;
    constexpr int n = D - 1;
    // edges entering negated (FAM_OR only): AND every edge, NOT its input
    const unsigned flip = FAM != FAM_OR ? 0u : type == T_AND ? (1u << D) - 1u : type == T_NOT ? 1u : 0u;
    HF<V> lf[n];
    int nnull = 0;
#pragma unroll
    for (int k = 0; k < n; ++k) {
        V m0, m1;
        P::leaf(((flip >> k) & 1u) ? -vf[k] : vf[k], m0, m1);
        HF<V> x;
        if constexpr (FAM == FAM_OR) x = {m0, m1};
        else if constexpr (FAM == FAM_NOISY) x = {P::add(m0, P::mul(m1, ep[k].b)), P::mul(m1, ep[k].a)};
        else x = {m1, m0};  // IMPLIES: an input fires when it is 0
        // a null incoming message contributes the identity leaf
        lf[k].h = nl[k] ? P::one() : x.h;
        lf[k].f = nl[k] ? P::zero() : x.f;
        nnull += nl[k] ? 1 : 0;
    }
    // Products with the identity leaf are skipped: combining with (1, 0) returns the other operand
    // exactly (log domain: x + 0 and log2(2^x + 0) = x), so only the NOISY_OR leak (the leftmost
    // leaf) costs a combine at the ends of the prefix and suffix products.
    HF<V> pre = identity<P>();
    if constexpr (FAM == FAM_NOISY) pre = {fp.b, fp.a};  // leak
    HF<V> l0 = lf[0];  // prefix product through input 0, leak included
    if constexpr (FAM == FAM_NOISY) l0 = combine<P>(pre, lf[0]);
    // Each part below runs only when the task writes an edge that needs it. Under a ranked
    // schedule a task usually writes either the head (forward) or the inputs (backward), and the
    // records of a level mostly agree, so the wavefront skips the other part.
    if ((active >> n) & 1u) {
        HF<V> t = l0;
#pragma unroll
        for (int k = 1; k < n; ++k) t = combine<P>(t, lf[k]);
        V o0, o1;
        if constexpr (FAM == FAM_IMPLIES) {  // fp = (p, 1-p)
            o0 = P::add(P::mul(fp.b, t.h), t.f);
            o1 = P::add(P::mul(fp.a, t.h), t.f);
        } else {
            o0 = t.h;
            o1 = t.f;
        }
        if ((flip >> n) & 1u) {
            const V tmp = o0;
            o0 = o1;
            o1 = tmp;
        }
        const S l = finish_msg<P, DAMP>(g, lo[n], o0, o1, nnull > 0, acc);
        put_msg<S, V, PAIRS>(g, b + n, l, lo[n]);
        stage_slot<P>(slots, slot0, active, n, l, lo[n]);
    }
    if (active & ((1u << n) - 1u)) {
        // the head's normalised incoming message (zero when null)
        V my0, my1;
        P::leaf(((flip >> n) & 1u) ? -vf[n] : vf[n], my0, my1);
        my0 = nl[n] ? P::zero() : my0;
        my1 = nl[n] ? P::zero() : my1;
        // sx[k] = product of the leaves after input k (k <= n - 2; after the last one: identity)
        HF<V> sx[n];
        if constexpr (n >= 2) {
            sx[n - 2] = lf[n - 1];
#pragma unroll
            for (int k = n - 3; k >= 0; --k) sx[k] = combine<P>(lf[k + 1], sx[k + 1]);
        }
        HF<V> run = l0;  // prefix product through input k - 1 (for k >= 1)
#pragma unroll
        for (int k = 0; k < n; ++k) {
            if ((active >> k) & 1u) {
                HF<V> x;  // product of the other inputs' leaves, leak included
                if (k == 0) {
                    if constexpr (n == 1) {
                        x = pre;
                    } else {
                        x = sx[0];
                        if constexpr (FAM == FAM_NOISY) x = combine<P>(pre, sx[0]);
                    }
                } else if (k == n - 1) {
                    x = run;
                } else {
                    x = combine<P>(run, sx[k]);
                }
                V o0, o1;
                if constexpr (FAM == FAM_IMPLIES) {
                    const V s2 = P::add(my0, my1);
                    const V wy = P::add(P::mul(my0, fp.b), P::mul(my1, fp.a));
                    o0 = s2;
                    o1 = P::add(P::mul(wy, x.h), P::mul(s2, x.f));
                } else {
                    const V base = P::add(P::mul(my0, x.h), P::mul(my1, x.f));  // input k does not fire
                    o0 = base;
                    if constexpr (FAM == FAM_NOISY) o1 = P::add(P::mul(ep[k].b, base), P::mul(ep[k].a, my1));
                    else o1 = my1;
                }
                if ((flip >> k) & 1u) {
                    const V tmp = o0;
                    o0 = o1;
                    o1 = tmp;
                }
                const int others_null = nnull - (nl[k] ? 1 : 0) + (nl[n] ? 1 : 0);
                const S l = finish_msg<P, DAMP>(g, lo[k], o0, o1, others_null > 0, acc);
                put_msg<S, V, PAIRS>(g, b + k, l, lo[k]);
                stage_slot<P>(slots, slot0, active, k, l, lo[k]);
            }
            if (k >= 1 && k + 1 < n) run = combine<P>(run, lf[k]);
        }
    }
}

// N consecutive values from p (global memory, 4-byte aligned) in as few loads as possible: 16-byte
// loads, then one of 4, 8 or 12 bytes for the rest. A factor's messages are contiguous, so a thread
// fetches them with one or two requests instead of one per edge.
template <class S, int N>
__device__ __forceinline__ void load_run(const S *p, S (&out)[N]) {
    typedef int iv4 __attribute__((ext_vector_type(4), aligned(4)));
    typedef int iv3 __attribute__((ext_vector_type(3), aligned(4)));
    typedef int iv2 __attribute__((ext_vector_type(2), aligned(4)));
    typedef __attribute__((address_space(1))) const int gint;
    typedef __attribute__((address_space(1))) const iv4 giv4;
    typedef __attribute__((address_space(1))) const iv3 giv3;
    typedef __attribute__((address_space(1))) const iv2 giv2;
    static_assert(sizeof(S) % 4 == 0, "dword-sized values only");
    constexpr int NW = N * int(sizeof(S) / 4);
    int w[NW];
    gint *q = (gint *)p;
#pragma unroll
    for (int i = 0; i + 4 <= NW; i += 4) {
        const iv4 x = *(giv4 *)(q + i);
#pragma unroll
        for (int j = 0; j < 4; ++j) w[i + j] = x[j];
    }
    constexpr int R = NW % 4, B0 = NW - R;
    if constexpr (R == 3) {
        const iv3 x = *(giv3 *)(q + B0);
        w[B0] = x[0];
        w[B0 + 1] = x[1];
        w[B0 + 2] = x[2];
    } else if constexpr (R == 2) {
        const iv2 x = *(giv2 *)(q + B0);
        w[B0] = x[0];
        w[B0 + 1] = x[1];
    } else if constexpr (R == 1) {
        w[B0] = q[B0];
    }
    __builtin_memcpy(out, w, sizeof(out));
}

// Loads of one factor of degree D (edges b .. b+D-1, variables u[]), all issued before any is used,
// then the family's arithmetic. On a level staged in LDS, the belief of each written edge's
// variable (as the factor read it, the value before the level) also goes to the edge's slot in
// bslots, for the variable phase.
template <class P, bool DAMP, int D, bool PAIRS>
__device__ __forceinline__ void factor_fetch_compute(const DevGraph<typename P::S, typename P::V> &g, int32_t b,
                                                     int type, int32_t fac, unsigned active, const int32_t *u,
                                                     Acc &acc, typename P::S *slots, Belief *bslots, int32_t slot0) {
    using S = typename P::S;
    using V = typename P::V;
    S lo[D];
    Belief B[D];
    load_run<S, D>(g.msg.get() + b, lo);
#pragma unroll
    for (int k = 0; k < D; ++k) B[k] = g.bel.ld(u[k]);
    Pair<V> ep[D];
#pragma unroll
    for (int k = 0; k < D; ++k) ep[k] = {P::zero(), P::one()};
    Pair<V> fp = {P::zero(), P::one()};
    if (type == T_NOISY_OR || type == T_IMPLIES) {
        fp = g.fpar.ld(fac);
        if (type == T_NOISY_OR) {
#pragma unroll
            for (int k = 0; k < D - 1; ++k) ep[k] = g.epar.ld(b + k);
        }
    }
    S vf[D];
    bool nl[D];
#pragma unroll
    for (int k = 0; k < D; ++k) vf[k] = v2f<P>(B[k], lo[k], nl[k]);
    if (slots) {
#pragma unroll
        for (int k = 0; k < D; ++k)
            if ((active >> k) & 1u) bslots[slot0 + __builtin_popcount(active & ((1u << k) - 1u))] = B[k];
    }
    if (type == T_NOISY_OR)
        factor_local<P, DAMP, D, FAM_NOISY, PAIRS>(g, type, b, active, fp, lo, vf, nl, ep, acc, slots, slot0);
    else if (type == T_IMPLIES)
        factor_local<P, DAMP, D, FAM_IMPLIES, PAIRS>(g, type, b, active, fp, lo, vf, nl, ep, acc, slots, slot0);
    else
        factor_local<P, DAMP, D, FAM_OR, PAIRS>(g, type, b, active, fp, lo, vf, nl, ep, acc, slots, slot0);
}

// `slots`: the level's LDS staging area (persistent executor, staged levels), else nullptr.
// PAIRS: keep the (new, old) pairs for incremental variable tasks when the plan has them.
template <class P, bool DAMP, bool PAIRS = true>
__device__ __forceinline__ void factor_rec(const DevGraph<typename P::S, typename P::V> &g, const FacRec &r, Acc &acc,
                                           typename P::S *slots = nullptr, Belief *bslots = nullptr) {
    const int d = r.meta & 0xff, type = (r.meta >> 8) & 0xff;
    const unsigned active = (unsigned)(r.meta >> 16) & 0xffu;
    const int32_t slot0 = r.u[8];
    switch (d) {
    case 2: factor_fetch_compute<P, DAMP, 2, PAIRS>(g, r.b, type, r.fac, active, r.u, acc, slots, bslots, slot0); break;
    case 3: factor_fetch_compute<P, DAMP, 3, PAIRS>(g, r.b, type, r.fac, active, r.u, acc, slots, bslots, slot0); break;
    case 4: factor_fetch_compute<P, DAMP, 4, PAIRS>(g, r.b, type, r.fac, active, r.u, acc, slots, bslots, slot0); break;
    case 5: factor_fetch_compute<P, DAMP, 5, PAIRS>(g, r.b, type, r.fac, active, r.u, acc, slots, bslots, slot0); break;
    case 6: factor_fetch_compute<P, DAMP, 6, PAIRS>(g, r.b, type, r.fac, active, r.u, acc, slots, bslots, slot0); break;
    case 7: factor_fetch_compute<P, DAMP, 7, PAIRS>(g, r.b, type, r.fac, active, r.u, acc, slots, bslots, slot0); break;
    case 8: factor_fetch_compute<P, DAMP, 8, PAIRS>(g, r.b, type, r.fac, active, r.u, acc, slots, bslots, slot0); break;
    default: break;
    }
}

// A variable record with C edge ids in the record (C = min(degree, 5)); edges past the fifth come
// from var_edge. Padding records (bit 30 of cnt) recompute their group's first belief and do not
// store it.
template <class P, int C>
__device__ __forceinline__ void var_rec_c(const DevGraph<typename P::S, typename P::V> &g, const VarRec &r, int cnt,
                                          bool pad) {
    using S = typename P::S;
    Belief B = g.phi.ld(r.v);
    S m[C > 0 ? C : 1];
#pragma unroll
    for (int j = 0; j < C; ++j) m[j] = g.msg[r.e[j]];
#pragma unroll
    for (int j = 0; j < C; ++j) belief_add<P>(B, m[j]);
    if (C == kVarRecEdges)
        for (int32_t j = kVarRecEdges; j < cnt; ++j) belief_add<P>(B, g.msg[g.var_edge[r.start + j]]);
    if (!pad) g.bel.st(r.v, B);
}

template <class P>
__device__ __forceinline__ void var_rec(const DevGraph<typename P::S, typename P::V> &g, const VarRec &r) {
    const int cnt = r.cnt & 0xffff;
    const bool pad = (r.cnt >> 30) & 1;
    switch (cnt < kVarRecEdges ? cnt : kVarRecEdges) {
    case 0: var_rec_c<P, 0>(g, r, cnt, pad); break;
    case 1: var_rec_c<P, 1>(g, r, cnt, pad); break;
    case 2: var_rec_c<P, 2>(g, r, cnt, pad); break;
    case 3: var_rec_c<P, 3>(g, r, cnt, pad); break;
    case 4: var_rec_c<P, 4>(g, r, cnt, pad); break;
    default: var_rec_c<P, kVarRecEdges>(g, r, cnt, pad); break;
    }
}

template <class P>
__device__ __forceinline__ void belief_sub(Belief &B, typename P::S l) {
    using S = typename P::S;
    const S inf = (S)__builtin_huge_val();
    const bool pi = l == inf, ni = l == -inf;
    B.npos -= pi ? 1 : 0;
    B.nneg -= ni ? 1 : 0;
    B.fin -= (pi || ni) ? 0.0 : (double)l;
}

// Incremental variable task (LEVELS executor), from a record of the level's delta list: kind 0
// rebuilds the belief from the whole row as var_rec does; kind 1 takes the belief before the level
// and, for each message the level wrote, subtracts its old value and adds the new one (both from the
// message's (new, old) pair in prev). The counts of infinite terms stay exact; the finite part is
// updated in float64 (beliefs are rebuilt from the messages at the start of every run). Padding
// records (bit 30) store nothing.
template <class P>
__device__ __forceinline__ void var_delta(const DevGraph<typename P::S, typename P::V> &g, const DevPlan &plan,
                                          const VarRec &r) {
    if (!((r.cnt >> 29) & 1)) {
        var_rec<P>(g, r);
        return;
    }
    using S = typename P::S;
    const int n = r.cnt & 0xffff;
    const bool pad = (r.cnt >> 30) & 1;
    Belief B = g.bel.ld(r.v);
    const GPtr<const MsgPair<S>> pairs((const MsgPair<S> *)g.prev.p);
    MsgPair<S> m[kVarRecEdges];
#pragma unroll
    for (int j = 0; j < kVarRecEdges; ++j) m[j] = pairs.ld(r.e[j < n ? j : 0]);
#pragma unroll
    for (int j = 0; j < kVarRecEdges; ++j)
        if (j < n) {
            belief_sub<P>(B, m[j].od);
            belief_add<P>(B, m[j].nw);
        }
    for (int32_t j = kVarRecEdges; j < n; ++j) {
        const MsgPair<S> x = pairs.ld(plan.dedge[r.start + j]);
        belief_sub<P>(B, x.od);
        belief_add<P>(B, x.nw);
    }
    if (!pad) g.bel.st(r.v, B);
}

// Variable task of a staged level: its belief before the level (left in bslots by the factor that
// wrote its first staged message) plus, for each message the level wrote, new minus old, read from
// the staging slots. The variable phase thus reads LDS only. The counts of infinite terms stay
// exact; the finite part is updated in float64 (the whole belief is rebuilt from the messages when
// a run starts and before marginals are read). A staged task has at least one written message (the host stages a
// level only then).
template <class P>
__device__ __forceinline__ void var_staged(const DevGraph<typename P::S, typename P::V> &g, const VarRecP &r,
                                           const typename P::S *slots, const Belief *bslots) {
    const int n = r.n();
    Belief B = bslots[r.slot(0)];
#pragma unroll
    for (int j = 0; j < kStagedEdges; ++j)
        if (j < n) {
            const int32_t s = r.slot(j);
            belief_sub<P>(B, slots[2 * s + 1]);
            belief_add<P>(B, slots[2 * s]);
        }
    if (!r.pad()) g.bel.st(r.v, B);
}

// ------------------------------------------------------------------------------------------------
// One factor of n = d - 1 inputs (8 < d <= 257) by one wavefront. Lane j owns the contiguous inputs
// [j c, j c + c) with c = ceil(n / 64) <= C, keeps their leaves in registers, and issues every load
// (its inputs, clamped to the last one so each address is valid, and the head) before the scan.
// ------------------------------------------------------------------------------------------------
template <class P, int C, bool ALL_ACTIVE, bool DAMP>
__device__ __forceinline__ void factor_wave_c(const DevGraph<typename P::S, typename P::V> &g, int32_t a, int32_t b,
                                              int32_t d, int type, int lane, int level, Acc &acc) {
    using S = typename P::S;
    using V = typename P::V;
    const int32_t n = d - 1;
    const int32_t c = (n + 63) >> 6;
    const int32_t i0 = min(n, lane * c), i1 = min(n, i0 + c);
    const int32_t eh = b + n;
    S lo[C];
    int32_t u[C];
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const int32_t e = b + min(i0 + k, n - 1);
        lo[k] = g.msg[e];
        u[k] = g.edge_var[e];
    }
    const S loh = g.msg[eh];
    const int32_t uh = g.edge_var[eh];
    Belief B[C];
#pragma unroll
    for (int k = 0; k < C; ++k) B[k] = g.bel.ld(u[k]);
    const Belief Bh = g.bel.ld(uh);
    Pair<V> fp = {P::zero(), P::one()};
    if (type == T_NOISY_OR || type == T_IMPLIES) fp = g.fpar.ld(a);
    Pair<V> ep[C];
#pragma unroll
    for (int k = 0; k < C; ++k) ep[k] = {P::zero(), P::one()};
    if (type == T_NOISY_OR) {
#pragma unroll
        for (int k = 0; k < C; ++k) ep[k] = g.epar.ld(b + min(i0 + k, n - 1));
    }
    bool null_h;
    const S vfh = v2f<P>(Bh, loh, null_h);
    V my0 = P::zero(), my1 = P::zero();
    if (!null_h) P::leaf(vfh, my0, my1);
    HF<V> lf[C];
    bool ln[C];
    int nnull = 0;
    HF<V> agg = identity<P>();
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const bool mine = i0 + k < i1;
        const S vf = v2f<P>(B[k], lo[k], ln[k]);
        lf[k] = identity<P>();
        if (mine && !ln[k]) {
            V m0, m1;
            P::leaf(vf, m0, m1);
            lf[k] = make_leaf<P>(type, m0, m1, ep[k]);
        }
        nnull += (mine && ln[k]) ? 1 : 0;
        agg = combine<P>(agg, lf[k]);
    }
    HF<V> init = identity<P>();
    if (type == T_NOISY_OR) init = {fp.b, fp.a};  // the leak: fires with probability leak
    HF<V> pre, suf, tot;
    int ntot;
    TeamScan<P, 64>::run(agg, nnull, init, pre, suf, tot, ntot, nullptr);
    if (lane == 0 && is_active<ALL_ACTIVE>(g.edge_level, eh, level)) {
        V o0, o1;
        head_msg<P>(type, tot, fp, o0, o1);
        store_msg<P, DAMP>(g, eh, loh, o0, o1, ntot > 0, acc);
    }
    HF<V> sx[C];
    HF<V> run = suf;
#pragma unroll
    for (int k = C - 1; k >= 0; --k) {
        sx[k] = run;
        run = combine<P>(lf[k], run);
    }
    run = pre;
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const int32_t e = b + i0 + k;
        if (i0 + k < i1 && is_active<ALL_ACTIVE>(g.edge_level, e, level)) {
            HF<V> xo = combine<P>(run, sx[k]);
            V o0, o1;
            input_msg<P>(type, xo, my0, my1, fp, ep[k], o0, o1);
            int others_null = ntot - (ln[k] ? 1 : 0) + (null_h ? 1 : 0);
            store_msg<P, DAMP>(g, e, lo[k], o0, o1, others_null > 0, acc);
        }
        run = combine<P>(run, lf[k]);
    }
}

template <class P, bool ALL_ACTIVE, bool DAMP>
__device__ __forceinline__ void factor_wave(const DevGraph<typename P::S, typename P::V> &g, int32_t a, int lane,
                                            int level, Acc &acc) {
    const int32_t b = g.fac_off[a];
    const int32_t d = g.fac_off[a + 1] - b;
    const int type = g.fac_type[a];
    if (type == T_NOT) {  // degree 2: never in this bucket, kept for safety
        if (lane == 0) factor_not<P, ALL_ACTIVE, DAMP>(g, b, level, acc);
        return;
    }
    const int32_t c = (d - 1 + 63) >> 6;
    if (c <= 1)
        factor_wave_c<P, 1, ALL_ACTIVE, DAMP>(g, a, b, d, type, lane, level, acc);
    else if (c <= 2)
        factor_wave_c<P, 2, ALL_ACTIVE, DAMP>(g, a, b, d, type, lane, level, acc);
    else
        factor_wave_c<P, 4, ALL_ACTIVE, DAMP>(g, a, b, d, type, lane, level, acc);
}

}  // namespace fastlbp
