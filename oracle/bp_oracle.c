/*
 * Plain FP64 CPU oracle for loopy belief propagation on binary factor graphs with local-structure
 * factors, scheduled by an update strategy given as edge ranks.
 *
 * TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the benchmark's CPU-baseline leg
 * may load this library. It shares no code with the GPU path and is deliberately slow and direct:
 *   - factor-to-variable messages are Eq.(2) (Section 3.2) evaluated per factor type by summing
 *     the factor's disjoint cubes (the grouping of assignments that Eq.(4) / Section 3.3 relies on);
 *     a message to an input variable conditions that input on each value and reuses the head sum,
 *     so every message costs O(degree) and a factor O(degree^2);
 *   - variable-to-factor messages are Eq.(1) as a plain product over the variable's other factors;
 *   - the schedule is Eq.(5) with delta from Definition 2, executed class by class in ascending
 *     rank: every message of a class is computed from the state before the class, then all are
 *     written. No dependency analysis is involved;
 *   - marginals are Eq.(3).
 *
 * Readings where the paper is silent (all listed in the design notes):
 *   initial messages uniform; every stored message normalised to sum 1; a message whose two
 *   entries are both 0 is replaced by (1/2, 1/2) and counted as a contradiction; damping mixes the
 *   normalised old and new message as lambda*old + (1-lambda)*new; a PRIOR factor is an ordinary
 *   unary factor whose message is the constant prior, and an evidence clamp is a unary indicator
 *   potential of the variable (Eq.(1) and Eq.(3) then include it); the residual is the largest change of
 *   P(x=1) over the messages written in an iteration, and a run stops after the first iteration
 *   whose residual is below tol (tol = 0 runs every iteration).
 *
 * Factor catalogue (head = last edge; inputs x_1..x_n are the edges before it):
 *   AND      f = [y = x_1 & ... & x_n]
 *   OR       f = [y = x_1 | ... | x_n]
 *   NOT      f = [y = !x_1]                      (n = 1)
 *   IMPLIES  probabilistic Horn rule p: x_1 & ... & x_n -> y  (Section 1, Section 2.2):
 *            f = p if all inputs are 1 and y = 1, 1-p if all inputs are 1 and y = 0, else 1
 *            (p = 1 is the hard implication)
 *   NOISY_OR P(y=0 | x) = (1-leak) * prod_{j: x_j=1} (1-p_j)
 *   PRIOR    unary, f(1) = p, f(0) = 1-p
 *
 * Floating point: built with -ffp-contract=off so results do not depend on FMA contraction.
 * Products are plain linear-domain products; for huge deterministic fan-in they can underflow
 * (the design notes list this limit).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { T_PRIOR = 0, T_AND = 1, T_OR = 2, T_NOT = 3, T_IMPLIES = 4, T_NOISY_OR = 5, T_TERMS = 6 };

/* ------------------------------------------------------------------------------------------ */
/* Eq.(2) summed over the head for every head value, given the inputs' incoming messages.       */
/* g[y] = sum over input assignments x of f(x, y) * prod_j m_j(x_j).                            */
/* ------------------------------------------------------------------------------------------ */

/* sum_k fire_k * prod_{j<k} nofire_j * prod_{j>k} tot_j: the cube "input k is the first one that
 * fires" summed over k. `suf` is scratch of length n+1. */
static double first_fire_cubes(int n, const double *nofire, const double *fire, const double *tot, double *suf) {
    suf[n] = 1.0;
    for (int j = n - 1; j >= 0; --j) suf[j] = suf[j + 1] * tot[j];
    double pre = 1.0, s = 0.0;
    for (int k = 0; k < n; ++k) {
        s += fire[k] * pre * suf[k + 1];
        pre *= nofire[k];
    }
    return s;
}

static double product(int n, const double *a) {
    double p = 1.0;
    for (int j = 0; j < n; ++j) p *= a[j];
    return p;
}

/* Work arrays for one factor, sized by the caller for the largest degree (+2). */
typedef struct {
    double *nofire, *fire, *tot, *suf, *c0, *c1;
} fwork;

/* n inputs with messages (m0[j], m1[j]); p_in[j] is the NOISY_OR activation of input j. */
static void head_sum(int type, int n, double fparam, const double *p_in, const double *m0, const double *m1,
                     fwork *w, double g[2]) {
    switch (type) {
    case T_NOT:
        /* y = !x */
        g[0] = m1[0];
        g[1] = m0[0];
        return;
    case T_OR:
        for (int j = 0; j < n; ++j) { w->nofire[j] = m0[j]; w->fire[j] = m1[j]; w->tot[j] = m0[j] + m1[j]; }
        g[0] = product(n, w->nofire);                                    /* all inputs 0 */
        g[1] = first_fire_cubes(n, w->nofire, w->fire, w->tot, w->suf);  /* first 1 at k */
        return;
    case T_AND:
        for (int j = 0; j < n; ++j) { w->nofire[j] = m1[j]; w->fire[j] = m0[j]; w->tot[j] = m0[j] + m1[j]; }
        g[1] = product(n, w->nofire);                                    /* all inputs 1 */
        g[0] = first_fire_cubes(n, w->nofire, w->fire, w->tot, w->suf);  /* first 0 at k */
        return;
    case T_IMPLIES: {
        for (int j = 0; j < n; ++j) { w->nofire[j] = m1[j]; w->fire[j] = m0[j]; w->tot[j] = m0[j] + m1[j]; }
        double all1 = product(n, w->nofire);
        double some0 = first_fire_cubes(n, w->nofire, w->fire, w->tot, w->suf); /* f = 1 for either y */
        g[0] = (1.0 - fparam) * all1 + some0;
        g[1] = fparam * all1 + some0;
        return;
    }
    case T_NOISY_OR: {
        /* Latent causes: the leak fires with prob. leak; input j fires with prob. p_j if x_j = 1.
         * y = 0 iff no cause fires. Summing each input over its value gives, per cause,
         * no-fire weight m0 + m1*(1-p), fire weight m1*p, total m0 + m1. The leak is cause 0. */
        w->nofire[0] = 1.0 - fparam; w->fire[0] = fparam; w->tot[0] = 1.0;
        for (int j = 0; j < n; ++j) {
            w->nofire[j + 1] = m0[j] + m1[j] * (1.0 - p_in[j]);
            w->fire[j + 1] = m1[j] * p_in[j];
            w->tot[j + 1] = m0[j] + m1[j];
        }
        g[0] = product(n + 1, w->nofire);
        g[1] = first_fire_cubes(n + 1, w->nofire, w->fire, w->tot, w->suf);
        return;
    }
    default:
        g[0] = g[1] = 0.0;
        return;
    }
}

/* Unnormalised Eq.(2) message of a factor to each of its d edges (head = edge d-1), from the
 * incoming variable-to-factor messages (m0[k], m1[k]) of all d edges.
 *   to the head:     out(y)   = g(y)
 *   to input i:      out(x_i) = sum_y m_y(y) * g(y | input i fixed to x_i)
 * Fixing input i to value c is done by replacing its message by the indicator of c. */
void oracle_factor_messages(int type, int d, double fparam, const double *eparam, const double *m0,
                            const double *m1, double *out0, double *out1) {
    if (type == T_PRIOR) {
        out0[0] = 1.0 - fparam;
        out1[0] = fparam;
        return;
    }
    int n = d - 1;
    fwork w;
    double *buf = (double *)malloc(sizeof(double) * 6 * (size_t)(d + 2));
    w.nofire = buf; w.fire = buf + (d + 2); w.tot = buf + 2 * (d + 2); w.suf = buf + 3 * (d + 2);
    w.c0 = buf + 4 * (d + 2); w.c1 = buf + 5 * (d + 2);
    double g[2];
    head_sum(type, n, fparam, eparam, m0, m1, &w, g);
    out0[n] = g[0];
    out1[n] = g[1];
    double my0 = m0[n], my1 = m1[n];
    for (int i = 0; i < n; ++i) {
        memcpy(w.c0, m0, sizeof(double) * n);
        memcpy(w.c1, m1, sizeof(double) * n);
        double res[2];
        for (int c = 0; c < 2; ++c) {
            w.c0[i] = (c == 0) ? 1.0 : 0.0;
            w.c1[i] = (c == 1) ? 1.0 : 0.0;
            head_sum(type, n, fparam, eparam, w.c0, w.c1, &w, g);
            res[c] = my0 * g[0] + my1 * g[1];
        }
        out0[i] = res[0];
        out1[i] = res[1];
    }
    free(buf);
}

/* Eq.(4) for a factor given as l weighted terms over its d edges: ind[t*d + k] is the value edge k
 * is fixed to in term t, or -1 (any value). The message to edge v at value x sums, over the terms
 * that allow x at v, the term's weight times the product over the other edges of the incoming
 * message at the fixed value, or of the message's total for a wildcard. Written as the definition
 * reads: O(l d^2). */
void oracle_terms_messages(int d, int l, const double *weight, const int8_t *ind, const double *m0,
                           const double *m1, double *out0, double *out1) {
    for (int v = 0; v < d; ++v) {
        double acc[2] = {0.0, 0.0};
        for (int x = 0; x < 2; ++x)
            for (int t = 0; t < l; ++t) {
                int cv = ind[t * d + v];
                if (cv != -1 && cv != x) continue;
                double sm = weight[t];
                for (int j = 0; j < d; ++j) {
                    if (j == v) continue;
                    int c = ind[t * d + j];
                    sm *= (c == -1) ? (m0[j] + m1[j]) : (c == 1 ? m1[j] : m0[j]);
                }
                acc[x] += sm;
            }
        out0[v] = acc[0];
        out1[v] = acc[1];
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Loopy BP driver                                                                            */
/* ------------------------------------------------------------------------------------------ */

typedef struct {
    int32_t iterations;
    int32_t converged;
    double residual;
    int64_t contradictions;
    int64_t marginal_contradictions;
    int64_t message_updates;
} oracle_stats;

static void normalise(double *a0, double *a1) {
    double s = *a0 + *a1;
    if (s > 0.0) { *a0 /= s; *a1 /= s; }
}

/* Unnormalised outputs (o0, o1) [d] of factor a in the state (msg0, msg1): the incoming
 * variable-to-factor messages by Eq.(1), as a plain product over each variable's other edges
 * (unary potential phi included), then Eq.(2) by factor type, or Eq.(4) for a TERMS factor. */
static void factor_outputs(int32_t a, const int64_t *fac_off, const int32_t *edge_var, const uint8_t *fac_type,
                           const double *fac_param, const double *edge_param, const int64_t *var_off,
                           const int64_t *var_edges, const int32_t *edge_fac, const double *phi0, const double *phi1,
                           const double *msg0, const double *msg1, const int64_t *term_off, const double *term_weight,
                           const int8_t *term_ind, const int64_t *ind_base, double *vf0, double *vf1, double *ep,
                           double *o0, double *o1) {
    int64_t b = fac_off[a];
    int d = (int)(fac_off[a + 1] - b);
    for (int k = 0; k < d; ++k) {
        int32_t u = edge_var[b + k];
        double p0 = phi0[u], p1 = phi1[u];
        for (int64_t q = var_off[u]; q < var_off[u + 1]; ++q) {
            int64_t e2 = var_edges[q];
            if (edge_fac[e2] == a) continue;
            p0 *= msg0[e2];
            p1 *= msg1[e2];
            normalise(&p0, &p1); /* keeps the running product in range */
        }
        vf0[k] = p0; vf1[k] = p1;
        ep[k] = edge_param ? edge_param[b + k] : 0.0;
    }
    if (fac_type[a] == T_TERMS)
        oracle_terms_messages(d, (int)(term_off[a + 1] - term_off[a]), term_weight + term_off[a],
                              term_ind + ind_base[a], vf0, vf1, o0, o1);
    else
        oracle_factor_messages(fac_type[a], d, fac_param[a], ep, vf0, vf1, o0, o1);
}

/* rank_of_edge: NULL = one class (flooding). group_of_edge: optional; when given, the groups it
 * defines replace the rank classes (used to check that executing the dependency-analysis levels
 * reproduces the class-by-class semantics). Messages msg0/msg1 [E] are read as the start state
 * and hold the final state on return; marg1 [V] receives P(x=1). Returns 0 on success. */
int oracle_bp(int32_t V, int32_t F, const int64_t *fac_off, const int32_t *edge_var, const uint8_t *fac_type,
              const double *fac_param, const double *edge_param, const int32_t *rank_of_edge,
              const int32_t *group_of_edge, const int8_t *evidence, int32_t max_iters, double tol, double damping,
              double *msg0, double *msg1, double *marg1, oracle_stats *st, const int64_t *term_off,
              const double *term_weight, const int8_t *term_ind) {
    int64_t E = fac_off[F];
    memset(st, 0, sizeof(*st));
    /* start of each factor's indicator rows (TERMS factors), term-major */
    int64_t *ind_base = (int64_t *)calloc((size_t)F + 1, sizeof(int64_t));
    for (int32_t a = 0; a < F; ++a) {
        int64_t l = term_off ? term_off[a + 1] - term_off[a] : 0;
        ind_base[a + 1] = ind_base[a] + l * (fac_off[a + 1] - fac_off[a]);
    }
    /* edge -> factor */
    int32_t *edge_fac = (int32_t *)malloc(sizeof(int32_t) * (size_t)(E > 0 ? E : 1));
    int dmax = 1;
    for (int32_t a = 0; a < F; ++a) {
        for (int64_t e = fac_off[a]; e < fac_off[a + 1]; ++e) edge_fac[e] = a;
        int d = (int)(fac_off[a + 1] - fac_off[a]);
        if (d > dmax) dmax = d;
    }
    /* variable -> incident edges (ascending edge id) */
    int64_t *var_off = (int64_t *)calloc((size_t)V + 1, sizeof(int64_t));
    int64_t *var_edges = (int64_t *)malloc(sizeof(int64_t) * (size_t)(E > 0 ? E : 1));
    for (int64_t e = 0; e < E; ++e) var_off[edge_var[e] + 1]++;
    for (int32_t v = 0; v < V; ++v) var_off[v + 1] += var_off[v];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)V + 1));
    memcpy(fill, var_off, sizeof(int64_t) * ((size_t)V + 1));
    for (int64_t e = 0; e < E; ++e) var_edges[fill[edge_var[e]]++] = e;
    free(fill);
    /* unary potential: evidence indicator only; PRIOR factors stay ordinary edges whose message
     * is the constant prior, which is the same product in Eq.(1) and Eq.(3). */
    double *phi0 = (double *)malloc(sizeof(double) * ((size_t)V + 1));
    double *phi1 = (double *)malloc(sizeof(double) * ((size_t)V + 1));
    for (int32_t v = 0; v < V; ++v) {
        phi0[v] = 1.0; phi1[v] = 1.0;
        if (evidence && evidence[v] == 0) phi1[v] = 0.0;
        if (evidence && evidence[v] == 1) phi0[v] = 0.0;
    }
    /* PRIOR messages are constants */
    for (int32_t a = 0; a < F; ++a)
        if (fac_type[a] == T_PRIOR) {
            int64_t e = fac_off[a];
            msg0[e] = 1.0 - fac_param[a];
            msg1[e] = fac_param[a];
        }
    /* groups: sort edges by (key, edge id) */
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(E > 0 ? E : 1));
    int64_t n_order = 0;
    const int32_t *key = group_of_edge ? group_of_edge : rank_of_edge;
    for (int64_t e = 0; e < E; ++e)
        if (fac_type[edge_fac[e]] != T_PRIOR) order[n_order++] = e;
    if (key) {
        /* insertion-free stable counting sort on the key */
        int32_t kmin = 0, kmax = 0;
        for (int64_t i = 0; i < n_order; ++i) {
            int32_t k = key[order[i]];
            if (i == 0 || k < kmin) kmin = k;
            if (i == 0 || k > kmax) kmax = k;
        }
        int64_t nk = (int64_t)kmax - kmin + 1;
        int64_t *cnt = (int64_t *)calloc((size_t)nk + 1, sizeof(int64_t));
        for (int64_t i = 0; i < n_order; ++i) cnt[key[order[i]] - kmin + 1]++;
        for (int64_t k = 0; k < nk; ++k) cnt[k + 1] += cnt[k];
        int64_t *sorted = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_order > 0 ? n_order : 1));
        for (int64_t i = 0; i < n_order; ++i) sorted[cnt[key[order[i]] - kmin]++] = order[i];
        memcpy(order, sorted, sizeof(int64_t) * (size_t)n_order);
        free(sorted);
        free(cnt);
    }
    /* scratch */
    double *vf0 = (double *)malloc(sizeof(double) * (size_t)(dmax + 1));
    double *vf1 = (double *)malloc(sizeof(double) * (size_t)(dmax + 1));
    double *ep = (double *)malloc(sizeof(double) * (size_t)(dmax + 1));
    double *o0 = (double *)malloc(sizeof(double) * (size_t)(dmax + 1));
    double *o1 = (double *)malloc(sizeof(double) * (size_t)(dmax + 1));
    double *new0 = (double *)malloc(sizeof(double) * (size_t)(E > 0 ? E : 1));
    double *new1 = (double *)malloc(sizeof(double) * (size_t)(E > 0 ? E : 1));

    int32_t it = 0;
    double r = 0.0;
    for (it = 0; it < max_iters;) {
        r = 0.0;
        int64_t cs = 0;
        while (cs < n_order) {
            int64_t ce = cs + 1;
            if (key)
                while (ce < n_order && key[order[ce]] == key[order[cs]]) ++ce;
            else
                ce = n_order;
            /* compute every message of the class from the state before the class */
            int64_t i = cs;
            while (i < ce) {
                int32_t a = edge_fac[order[i]];
                int64_t b = fac_off[a];
                factor_outputs(a, fac_off, edge_var, fac_type, fac_param, edge_param, var_off, var_edges, edge_fac,
                               phi0, phi1, msg0, msg1, term_off, term_weight, term_ind, ind_base, vf0, vf1, ep, o0,
                               o1);
                /* keep the outputs of the class's edges of this factor */
                while (i < ce && edge_fac[order[i]] == a) {
                    int64_t e = order[i];
                    new0[e] = o0[e - b];
                    new1[e] = o1[e - b];
                    ++i;
                }
                /* within a class, edges are in ascending id, so one factor's edges are adjacent */
            }
            /* write the class */
            for (int64_t j = cs; j < ce; ++j) {
                int64_t e = order[j];
                double n0 = new0[e], n1 = new1[e];
                if (n0 + n1 > 0.0) {
                    normalise(&n0, &n1);
                } else {
                    n0 = n1 = 0.5;
                    st->contradictions++;
                }
                double s0 = damping * msg0[e] + (1.0 - damping) * n0;
                double s1 = damping * msg1[e] + (1.0 - damping) * n1;
                normalise(&s0, &s1);
                double dlt = fabs(s1 - msg1[e]);
                if (dlt > r) r = dlt;
                msg0[e] = s0;
                msg1[e] = s1;
            }
            st->message_updates += ce - cs;
            cs = ce;
        }
        ++it;
        if (r < tol) { st->converged = 1; break; }
    }
    st->iterations = it;
    st->residual = r;
    /* Eq.(3) */
    for (int32_t v = 0; v < V; ++v) {
        double p0 = phi0[v], p1 = phi1[v];
        normalise(&p0, &p1);
        for (int64_t q = var_off[v]; q < var_off[v + 1]; ++q) {
            int64_t e2 = var_edges[q];
            p0 *= msg0[e2];
            p1 *= msg1[e2];
            normalise(&p0, &p1);
        }
        if (p0 + p1 > 0.0) {
            marg1[v] = p1 / (p0 + p1);
        } else {
            marg1[v] = 0.5;
            st->marginal_contradictions++;
        }
    }
    free(ind_base);
    free(edge_fac); free(var_off); free(var_edges); free(phi0); free(phi1); free(order);
    free(vf0); free(vf1); free(ep); free(o0); free(o1); free(new0); free(new1);
    return 0;
}

/* One flooding update of a sample of factors, computed one factor at a time from the state
 * (msg0, msg1) [E] without running the whole iteration: for each factor in `sample` [n], the new
 * normalised messages of its edges (a message whose two entries are both 0 becomes (1/2, 1/2) and
 * sets its entry of `contra`), written to out1 (P(x=1)) from position out_off[i]. No damping. This
 * is the same Eq.(1)-(2) / Eq.(4) arithmetic as an iteration of oracle_bp, restricted to the
 * sampled factors, for graphs too large for the whole iteration. Returns 0 on success. */
int oracle_factor_sample(int32_t V, int32_t F, const int64_t *fac_off, const int32_t *edge_var, const uint8_t *fac_type,
                         const double *fac_param, const double *edge_param, const int8_t *evidence,
                         const double *msg0_in, const double *msg1_in, const int64_t *term_off,
                         const double *term_weight, const int8_t *term_ind, int32_t n, const int32_t *sample,
                         const int64_t *out_off, double *out1, int8_t *contra) {
    int64_t E = fac_off[F];
    int64_t *ind_base = (int64_t *)calloc((size_t)F + 1, sizeof(int64_t));
    for (int32_t a = 0; a < F; ++a) {
        int64_t l = term_off ? term_off[a + 1] - term_off[a] : 0;
        ind_base[a + 1] = ind_base[a] + l * (fac_off[a + 1] - fac_off[a]);
    }
    int32_t *edge_fac = (int32_t *)malloc(sizeof(int32_t) * (size_t)(E > 0 ? E : 1));
    int dmax = 1;
    for (int32_t a = 0; a < F; ++a) {
        for (int64_t e = fac_off[a]; e < fac_off[a + 1]; ++e) edge_fac[e] = a;
        int d = (int)(fac_off[a + 1] - fac_off[a]);
        if (d > dmax) dmax = d;
    }
    int64_t *var_off = (int64_t *)calloc((size_t)V + 1, sizeof(int64_t));
    int64_t *var_edges = (int64_t *)malloc(sizeof(int64_t) * (size_t)(E > 0 ? E : 1));
    for (int64_t e = 0; e < E; ++e) var_off[edge_var[e] + 1]++;
    for (int32_t v = 0; v < V; ++v) var_off[v + 1] += var_off[v];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)V + 1));
    memcpy(fill, var_off, sizeof(int64_t) * ((size_t)V + 1));
    for (int64_t e = 0; e < E; ++e) var_edges[fill[edge_var[e]]++] = e;
    free(fill);
    double *phi0 = (double *)malloc(sizeof(double) * ((size_t)V + 1));
    double *phi1 = (double *)malloc(sizeof(double) * ((size_t)V + 1));
    for (int32_t v = 0; v < V; ++v) {
        phi0[v] = 1.0; phi1[v] = 1.0;
        if (evidence && evidence[v] == 0) phi1[v] = 0.0;
        if (evidence && evidence[v] == 1) phi0[v] = 0.0;
    }
    /* PRIOR messages are the constant prior, whatever the state holds */
    double *msg0 = (double *)malloc(sizeof(double) * (size_t)(E > 0 ? E : 1));
    double *msg1 = (double *)malloc(sizeof(double) * (size_t)(E > 0 ? E : 1));
    memcpy(msg0, msg0_in, sizeof(double) * (size_t)E);
    memcpy(msg1, msg1_in, sizeof(double) * (size_t)E);
    for (int32_t a = 0; a < F; ++a)
        if (fac_type[a] == T_PRIOR) {
            msg0[fac_off[a]] = 1.0 - fac_param[a];
            msg1[fac_off[a]] = fac_param[a];
        }
    double *vf0 = (double *)malloc(sizeof(double) * (size_t)(dmax + 1));
    double *vf1 = (double *)malloc(sizeof(double) * (size_t)(dmax + 1));
    double *ep = (double *)malloc(sizeof(double) * (size_t)(dmax + 1));
    double *o0 = (double *)malloc(sizeof(double) * (size_t)(dmax + 1));
    double *o1 = (double *)malloc(sizeof(double) * (size_t)(dmax + 1));
    int rc = 0;
    for (int32_t i = 0; i < n; ++i) {
        int32_t a = sample[i];
        if (a < 0 || a >= F || fac_type[a] == T_PRIOR) { rc = -1; break; }
        factor_outputs(a, fac_off, edge_var, fac_type, fac_param, edge_param, var_off, var_edges, edge_fac, phi0,
                       phi1, msg0, msg1, term_off, term_weight, term_ind, ind_base, vf0, vf1, ep, o0, o1);
        int d = (int)(fac_off[a + 1] - fac_off[a]);
        for (int k = 0; k < d; ++k) {
            double n0 = o0[k], n1 = o1[k];
            int c = !(n0 + n1 > 0.0);
            if (c) { n0 = n1 = 0.5; } else normalise(&n0, &n1);
            out1[out_off[i] + k] = n1;
            contra[out_off[i] + k] = (int8_t)c;
        }
    }
    free(ind_base); free(edge_fac); free(var_off); free(var_edges); free(phi0); free(phi1); free(msg0); free(msg1);
    free(vf0); free(vf1); free(ep); free(o0); free(o1);
    return rc;
}
