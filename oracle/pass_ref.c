/*
 * Oracle compiler pass: the permutation-inserting pass of the paper's Section 3
 * (Algorithm 1), written plainly: no pruning of candidate swaps, no incremental
 * bookkeeping.  Every candidate permutation is scored by a full scan.
 *
 * TEST INFRASTRUCTURE ONLY (see sim.c): the product pass is a separate
 * implementation whose output is compared against this one instruction by
 * instruction.
 *
 * Readings of points the paper leaves open:
 *  - A permutation sigma maps qubit q to position sigma(q); q is local iff
 *    sigma(q) < m (Section 2).
 *  - A gate "acts on local qubits" iff each qubit on which it acts
 *    non-diagonally is local: the target of CX/CU (unless U is diagonal) and
 *    the qubit of a non-diagonal U.  Controls and CZ are diagonal, so a CNOT
 *    with a global control and local target needs no communication
 *    (Sections 2 and 4; Appendix C for diagonal gates).
 *  - The DAG has an edge h -> v (h before v in program order) for every pair
 *    sharing a qubit that does not commute exactly.  Two gates commute when on
 *    every shared qubit both act as Z-type (diagonal: control, CZ, diagonal
 *    matrix) or both as X-type (matrix in span{I, X}: CX target), or when they
 *    are identical gates (Section 3 uses commutation to drop edges).
 *  - sigma o (l g) exchanges the positions of qubits l and g.
 *  - The count a' for a candidate sigma' is the number of not yet scheduled
 *    gates that would become schedulable under sigma': gates local under
 *    sigma' whose predecessors are all scheduled or themselves counted
 *    (a closure taken in program order).
 *  - Loops: l runs over local qubits in ascending qubit index, g over global
 *    qubits in ascending qubit index, and the first strict maximum wins.
 *  - The scheduling sweep runs in program order, which reaches the fixed point
 *    in one sweep because every predecessor has a lower index.
 *  - The fallback "vertex without incoming edges" is the lowest-index gate
 *    whose predecessors are all scheduled.
 *
 * Two optional parameters extend the pass for the tiled device executor; with
 * r = 1 and pinned = 0 the pass is the paper's algorithm:
 *  - r: up to r swaps are chained into one PermuteQubits; each further swap is
 *    taken only if it strictly raises the count reached by the previous ones.
 *  - pinned: qubits at positions < pinned are never chosen as l.
 *
 * Output: an int32 instruction stream,
 *   0 v          ApplyGate(v) on local qubits
 *   1 s_0..s_n-1 PermuteQubits(s)
 *   2 v          ApplyGate(v) requiring communication (fallback branch)
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t kind, q0, q1, pad;
    double u[8];
} orc_gate;

enum { K_U = 0, K_CX = 1, K_CZ = 2, K_CU = 3 };
enum { T_NONE = 0, T_Z = 1, T_X = 2, T_G = 3 };

/* action type of a 2x2 matrix (interleaved re, im) */
static int matrix_type(const double *m)
{
    if (m[2] == 0 && m[3] == 0 && m[4] == 0 && m[5] == 0)
        return T_Z;
    if (m[0] == m[6] && m[1] == m[7] && m[2] == m[4] && m[3] == m[5])
        return T_X;
    return T_G;
}

/* how gate g acts on qubit q */
static int action_on(const orc_gate *g, int q)
{
    switch (g->kind) {
    case K_U:  return q == g->q0 ? matrix_type(g->u) : T_NONE;
    case K_CX: return q == g->q0 ? T_Z : (q == g->q1 ? T_X : T_NONE);
    case K_CZ: return (q == g->q0 || q == g->q1) ? T_Z : T_NONE;
    case K_CU: return q == g->q0 ? T_Z : (q == g->q1 ? matrix_type(g->u) : T_NONE);
    }
    return T_NONE;
}

static int n_qubits_of(const orc_gate *g) { return g->kind == K_U ? 1 : 2; }

static int identical(const orc_gate *a, const orc_gate *b)
{
    return a->kind == b->kind && a->q0 == b->q0 && a->q1 == b->q1 && memcmp(a->u, b->u, sizeof a->u) == 0;
}

static int commute(const orc_gate *a, const orc_gate *b)
{
    if (identical(a, b))
        return 1;
    int qa[2] = {a->q0, a->q1};
    for (int k = 0; k < n_qubits_of(a); ++k) {
        int q = qa[k];
        int ta = action_on(a, q), tb = action_on(b, q);
        if (tb == T_NONE)
            continue;                              /* not shared */
        if (!(ta == tb && (ta == T_Z || ta == T_X)))
            return 0;
    }
    return 1;
}

/* g is local under sigma iff every qubit it acts on non-diagonally is local */
static int is_local(const orc_gate *g, const int *sigma, int m)
{
    int qs[2] = {g->q0, g->q1};
    for (int k = 0; k < n_qubits_of(g); ++k) {
        int t = action_on(g, qs[k]);
        if (t != T_Z && sigma[qs[k]] >= m)
            return 0;
    }
    return 1;
}

typedef struct {
    int64_t ng;
    int64_t *pred_start, *pred;    /* CSR list of predecessors */
} dag_t;

static int build_dag(const orc_gate *g, int64_t ng, dag_t *d)
{
    d->ng = ng;
    d->pred_start = (int64_t *)calloc((size_t)ng + 1, sizeof(int64_t));
    int64_t cap = 1024, cnt = 0;
    d->pred = (int64_t *)malloc(sizeof(int64_t) * cap);
    if (!d->pred_start || !d->pred)
        return -1;
    for (int64_t v = 0; v < ng; ++v) {
        d->pred_start[v] = cnt;
        for (int64_t h = 0; h < v; ++h) {
            int shares = 0;
            int qh[2] = {g[h].q0, g[h].q1};
            for (int k = 0; k < n_qubits_of(&g[h]); ++k)
                if (action_on(&g[v], qh[k]) != T_NONE)
                    shares = 1;
            if (shares && !commute(&g[h], &g[v])) {
                if (cnt == cap) {
                    cap *= 2;
                    d->pred = (int64_t *)realloc(d->pred, sizeof(int64_t) * cap);
                    if (!d->pred)
                        return -1;
                }
                d->pred[cnt++] = h;
            }
        }
    }
    d->pred_start[ng] = cnt;
    return 0;
}

static void free_dag(dag_t *d)
{
    free(d->pred_start);
    free(d->pred);
}

/* Number of edges of the DAG (exported for tests). */
int64_t orc_dag_edges(const orc_gate *g, int64_t ng, int64_t *pred_out, int64_t cap)
{
    dag_t d;
    if (build_dag(g, ng, &d))
        return -1;
    int64_t e = d.pred_start[ng];
    /* pairs (h, v) flattened */
    for (int64_t v = 0, k = 0; v < ng && pred_out; ++v)
        for (int64_t p = d.pred_start[v]; p < d.pred_start[v + 1]; ++p, ++k)
            if (2 * k + 1 < cap) {
                pred_out[2 * k] = d.pred[p];
                pred_out[2 * k + 1] = v;
            }
    free_dag(&d);
    return e;
}

static int preds_in(const dag_t *d, int64_t v, const char *set_a, const char *set_b)
{
    for (int64_t p = d->pred_start[v]; p < d->pred_start[v + 1]; ++p) {
        int64_t h = d->pred[p];
        if (!set_a[h] && !(set_b && set_b[h]))
            return 0;
    }
    return 1;
}

/* count of gates that become schedulable under sigma (closure in program order) */
static int64_t closure_count(const orc_gate *g, const dag_t *d, const char *done, char *mark,
                             const int *sigma, int m)
{
    int64_t cnt = 0;
    memset(mark, 0, (size_t)d->ng);
    for (int64_t v = 0; v < d->ng; ++v) {
        if (done[v])
            continue;
        if (is_local(&g[v], sigma, m) && preds_in(d, v, done, mark)) {
            mark[v] = 1;
            ++cnt;
        }
    }
    return cnt;
}

/*
 * Returns the number of int32 words written to out (or -1 on error, -2 if cap
 * is too small).  stats (may be NULL): [n_apply, n_perm, n_global, n_swaps].
 */
int64_t orc_pass(const orc_gate *g, int64_t ng, int n, int m, int r, int pinned,
                 int32_t *out, int64_t cap, int64_t *stats)
{
    if (m < 1 || m > n || r < 1 || pinned < 0 || pinned > m)
        return -1;
    dag_t d;
    if (build_dag(g, ng, &d))
        return -1;
    char *done = (char *)calloc((size_t)ng + 1, 1);
    char *mark = (char *)calloc((size_t)ng + 1, 1);
    int *sigma = (int *)malloc(sizeof(int) * n);
    int *cur = (int *)malloc(sizeof(int) * n);
    int *cand = (int *)malloc(sizeof(int) * n);
    int *best = (int *)malloc(sizeof(int) * n);
    int64_t w = 0, remaining = ng, n_apply = 0, n_perm = 0, n_global = 0, n_swaps = 0;
    int64_t rc = 0;
    for (int q = 0; q < n; ++q)
        sigma[q] = q;

#define EMIT(x)                         \
    do {                                \
        if (w >= cap) { rc = -2; goto end; } \
        out[w++] = (int32_t)(x);        \
    } while (0)

    while (remaining > 0) {
        /* schedule every local gate without unscheduled predecessors */
        for (int64_t v = 0; v < ng; ++v) {
            if (done[v])
                continue;
            if (preds_in(&d, v, done, NULL) && is_local(&g[v], sigma, m)) {
                EMIT(0);
                EMIT(v);
                done[v] = 1;
                --remaining;
                ++n_apply;
            }
        }
        if (remaining == 0)
            break;

        /* try single local<->global exchanges, chained up to r times */
        memcpy(cur, sigma, sizeof(int) * n);
        int64_t base = 0;
        int swaps = 0;
        for (int step = 0; step < r; ++step) {
            int64_t best_a = base;
            int found = 0;
            for (int l = 0; l < n; ++l) {
                if (!(cur[l] < m && cur[l] >= pinned))
                    continue;
                for (int gq = 0; gq < n; ++gq) {
                    if (cur[gq] < m)
                        continue;
                    memcpy(cand, cur, sizeof(int) * n);
                    cand[l] = cur[gq];
                    cand[gq] = cur[l];
                    int64_t a = closure_count(g, &d, done, mark, cand, m);
                    if (a > best_a) {
                        best_a = a;
                        memcpy(best, cand, sizeof(int) * n);
                        found = 1;
                    }
                }
            }
            if (!found)
                break;
            memcpy(cur, best, sizeof(int) * n);
            base = best_a;
            ++swaps;
        }
        if (swaps > 0) {
            memcpy(sigma, cur, sizeof(int) * n);
            EMIT(1);
            for (int q = 0; q < n; ++q)
                EMIT(sigma[q]);
            ++n_perm;
            n_swaps += swaps;
        } else {
            for (int64_t v = 0; v < ng; ++v)
                if (!done[v] && preds_in(&d, v, done, NULL)) {
                    EMIT(2);
                    EMIT(v);
                    done[v] = 1;
                    --remaining;
                    ++n_global;
                    break;
                }
        }
    }
    rc = w;
end:
#undef EMIT
    if (stats) {
        stats[0] = n_apply;
        stats[1] = n_perm;
        stats[2] = n_global;
        stats[3] = n_swaps;
    }
    free(done);
    free(mark);
    free(sigma);
    free(cur);
    free(cand);
    free(best);
    free_dag(&d);
    return rc;
}

/* 1 if gate v of g is local under sigma with m local positions (for tests) */
int orc_gate_is_local(const orc_gate *g, const int *sigma, int m)
{
    return is_local(g, sigma, m);
}

int orc_commute(const orc_gate *a, const orc_gate *b)
{
    return commute(a, b);
}
