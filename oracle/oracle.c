/*
 * oracle.c - plain, sequential CPU oracle for the LLP sweep.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The GPU product path
 * never links, loads or calls it, and it shares no code, header, table or
 * helper with the GPU path.
 *
 * Every solver here is Algorithm LLP of the paper's Background section
 * (start from the bottom of the lattice, repeatedly advance each forbidden
 * index j to alpha(G, j), return null when alpha exceeds the bound T[j]),
 * written as the paper's single-threaded cyclic solver (Section 4.3, "A
 * simple cyclic solver": sweep every index in order, stop after a pass that
 * advances nothing) or as its bag solver (Section 4.3, "A simple bag-based
 * solver": process indices taken from a FIFO bag of candidates, push the
 * indices an advance may make forbidden).
 *
 * Values are kept in the problem's natural domain with 64-bit integers
 * (distances, levels, start times, DP values), never in an encoded form, so
 * nothing here mirrors the GPU's state representation.
 *
 * Status codes returned (numeric values chosen to line up with the library's
 * documented status codes): 0 ok, 1 bad argument, 2 bad input,
 * 3 infeasible (alpha > T), 4 int32 overflow of a result,
 * 5 not converged within max_passes, 8 cycle in a job DAG.
 *
 * Build: gcc -O2 -shared -fPIC oracle.c -o liboracle.so   (single-threaded)
 */
#define _POSIX_C_SOURCE 199309L
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define OR_OK 0
#define OR_E_ARG 1
#define OR_E_INPUT 2
#define OR_E_INFEASIBLE 3
#define OR_E_OVERFLOW 4
#define OR_E_NOT_CONVERGED 5
#define OR_E_CYCLE 8

#define INF64 INT64_MAX
#define I32MAX 2147483647LL

/* ------------------------------------------------------------------ */
/* Adjacency lists built by the oracle itself from an arc list.         */
/* rows[v] .. rows[v+1] index the arcs whose `key` endpoint is v.        */
/* ------------------------------------------------------------------ */
typedef struct { int64_t* rows; int64_t* arc; } adj_t;

static int adj_build(int64_t n, int64_t m, const int32_t* key, adj_t* A) {
    A->rows = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    A->arc = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    if (!A->rows || !A->arc) return -1;
    for (int64_t e = 0; e < m; ++e) A->rows[key[e] + 1]++;
    for (int64_t v = 0; v < n; ++v) A->rows[v + 1] += A->rows[v];
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!fill) return -1;
    memcpy(fill, A->rows, sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t e = 0; e < m; ++e) A->arc[fill[key[e]]++] = e;
    free(fill);
    return 0;
}

static void adj_free(adj_t* A) { free(A->rows); free(A->arc); }

static int check_graph(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                       const int32_t* w) {
    for (int64_t e = 0; e < m; ++e) {
        if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return OR_E_INPUT;
        if (w && w[e] < 0) return OR_E_INPUT;   /* Section 5.2: weights are non-negative */
    }
    return OR_OK;
}

/* ================================================================== */
/* Single-source shortest paths, Section 5.2 (and BFS, Section 5.3,    */
/* which is the same predicate with every weight equal to 1).          */
/*                                                                      */
/* State d(v): d(s) = 0, d(v) = infinity otherwise.  The lattice order  */
/* is ">=" on distances (Section 4.2, monotonicity requirement): an     */
/* advance lowers d.  Index v != s is forbidden iff some arc (u, v) has */
/* d(v) > d(u) + w(u, v); the advance sets                              */
/*     d(v) := min{ d(v), d(u) + w(u, v) : (u, v) in E }.              */
/* The source is never forbidden (Section 5.2 implementation).          */
/* ================================================================== */
static int64_t sssp_alpha(const adj_t* in, const int32_t* src, const int32_t* w,
                          const int64_t* d, int64_t v) {
    int64_t best = d[v];
    for (int64_t k = in->rows[v]; k < in->rows[v + 1]; ++k) {
        int64_t e = in->arc[k];
        int64_t du = d[src[e]];
        if (du == INF64) continue;
        int64_t cand = du + (w ? w[e] : 1);
        if (cand < best) best = cand;
    }
    return best;
}

static int sssp_output(int32_t n, const int64_t* d, int32_t* out) {
    int status = OR_OK;
    for (int64_t v = 0; v < n; ++v) {
        if (d[v] == INF64) out[v] = (int32_t)I32MAX;
        else if (d[v] >= I32MAX) { out[v] = (int32_t)I32MAX; status = OR_E_OVERFLOW; }
        else out[v] = (int32_t)d[v];
    }
    return status;
}

/* Cyclic solver.  order (nullable) gives the index visiting order of every
   pass; jacobi != 0 evaluates every alpha of a pass against the state at the
   start of that pass (all forbidden indices advanced "simultaneously", as in
   Algorithm LLP's inner loop) instead of the latest state. */
int oracle_sssp_cyclic(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                       const int32_t* w, int32_t source, int64_t max_passes,
                       const int32_t* order, int32_t jacobi,
                       int32_t* dist_out, int64_t* passes_out) {
    if (n <= 0 || m < 0 || source < 0 || source >= n) return OR_E_ARG;
    int st = check_graph(n, m, src, dst, w);
    if (st) return st;
    adj_t in;
    if (adj_build(n, m, dst, &in)) return OR_E_ARG;
    int64_t* d = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t* snap = jacobi ? (int64_t*)malloc(sizeof(int64_t) * (size_t)n) : NULL;
    for (int64_t v = 0; v < n; ++v) d[v] = INF64;
    d[source] = 0;
    int64_t passes = 0;
    int status = OR_OK;
    for (;;) {
        int changed = 0;
        const int64_t* rd = d;
        if (jacobi) { memcpy(snap, d, sizeof(int64_t) * (size_t)n); rd = snap; }
        for (int64_t i = 0; i < n; ++i) {
            int64_t v = order ? order[i] : i;
            if (v == source) continue;
            int64_t a = sssp_alpha(&in, src, w, rd, v);
            if (a < d[v]) { d[v] = a; changed = 1; }
        }
        ++passes;
        if (!changed) break;
        if (max_passes > 0 && passes >= max_passes) { status = OR_E_NOT_CONVERGED; break; }
    }
    int st2 = sssp_output(n, d, dist_out);
    if (status == OR_OK) status = st2;
    if (passes_out) *passes_out = passes;
    free(d); free(snap); adj_free(&in);
    return status;
}

/* Bag solver (FIFO bag with membership flags).  The bag starts with the
   source's out-neighbours; an advance of v pushes v's out-neighbours, the
   indices whose predicate reads d(v) (Section 4.2, problem-specific state
   selection).  sssp_bag_run works on adjacency lists built beforehand. */
static void sssp_bag_run(int32_t n, const adj_t* in, const adj_t* out, const int32_t* src,
                         const int32_t* dst, const int32_t* w, int32_t source, int64_t* d,
                         int32_t* q, uint8_t* inq, int64_t* evals_out) {
    for (int64_t v = 0; v < n; ++v) { d[v] = INF64; inq[v] = 0; }
    d[source] = 0;
    int64_t head = 0, size = 0, evals = 0;
#define PUSH_OUT(u)                                                        \
    for (int64_t k = out->rows[u]; k < out->rows[(u) + 1]; ++k) {          \
        int32_t x = dst[out->arc[k]];                                      \
        if (!inq[x] && x != source) { inq[x] = 1; q[(head + size) % n] = x; ++size; } \
    }
    PUSH_OUT(source);
    while (size > 0) {
        int32_t v = q[head]; head = (head + 1) % n; --size; inq[v] = 0;
        ++evals;
        int64_t a = sssp_alpha(in, src, w, d, v);
        if (a < d[v]) { d[v] = a; PUSH_OUT(v); }
    }
#undef PUSH_OUT
    *evals_out = evals;
}

static double now_s(void) {
    struct timespec t;
    clock_gettime(CLOCK_MONOTONIC, &t);
    return (double)t.tv_sec + 1e-9 * (double)t.tv_nsec;
}

/* solve_s (nullable) receives the time of the solve alone: the adjacency
   lists are built before the clock starts. */
int oracle_sssp_bag_timed(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                          const int32_t* w, int32_t source, int32_t* dist_out, int64_t* evals_out,
                          double* solve_s) {
    if (n <= 0 || m < 0 || source < 0 || source >= n) return OR_E_ARG;
    int st = check_graph(n, m, src, dst, w);
    if (st) return st;
    adj_t in, out;
    if (adj_build(n, m, dst, &in) || adj_build(n, m, src, &out)) return OR_E_ARG;
    int64_t* d = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int32_t* q = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    uint8_t* inq = (uint8_t*)malloc((size_t)n);
    int64_t evals = 0;
    double t0 = now_s();
    sssp_bag_run(n, &in, &out, src, dst, w, source, d, q, inq, &evals);
    if (solve_s) *solve_s = now_s() - t0;
    int status = sssp_output(n, d, dist_out);
    if (evals_out) *evals_out = evals;
    free(d); free(q); free(inq); adj_free(&in); adj_free(&out);
    return status;
}

int oracle_sssp_bag(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                    const int32_t* w, int32_t source, int32_t* dist_out, int64_t* evals_out) {
    return oracle_sssp_bag_timed(n, m, src, dst, w, source, dist_out, evals_out, NULL);
}

/* Cross-checks timed beside the oracle (textbook algorithms, not LLP):
   Dijkstra with a binary heap of (distance, vertex) entries and lazy
   deletion, and a FIFO-queue BFS, each over out-adjacency lists built
   before the clock starts.  w == NULL: unit weights. */
int oracle_dijkstra_timed(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                          const int32_t* w, int32_t source, int32_t* dist_out, double* solve_s) {
    if (n <= 0 || m < 0 || source < 0 || source >= n) return OR_E_ARG;
    int st = check_graph(n, m, src, dst, w);
    if (st) return st;
    adj_t out;
    if (adj_build(n, m, src, &out)) return OR_E_ARG;
    int64_t* d = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t cap = m + 1, size = 0;
    int64_t* hk = (int64_t*)malloc(sizeof(int64_t) * (size_t)cap);
    int32_t* hv = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
    double t0 = now_s();
    for (int64_t v = 0; v < n; ++v) d[v] = INF64;
    d[source] = 0;
    hk[0] = 0; hv[0] = source; size = 1;
    while (size > 0) {
        int64_t k = hk[0];
        int32_t u = hv[0];
        --size;                                  /* pop: move the last entry down from the root */
        int64_t i = 0;
        while (size > 0) {
            int64_t c = 2 * i + 1;
            if (c >= size) break;
            if (c + 1 < size && hk[c + 1] < hk[c]) ++c;
            if (hk[c] >= hk[size]) break;
            hk[i] = hk[c]; hv[i] = hv[c]; i = c;
        }
        if (size > 0) { hk[i] = hk[size]; hv[i] = hv[size]; }
        if (k > d[u]) continue;                  /* stale entry */
        for (int64_t a = out.rows[u]; a < out.rows[u + 1]; ++a) {
            int64_t e = out.arc[a];
            int64_t nd = k + (w ? w[e] : 1);
            int32_t x = dst[e];
            if (nd < d[x]) {
                d[x] = nd;
                int64_t j = size++;              /* push: sift up */
                while (j > 0 && hk[(j - 1) / 2] > nd) { hk[j] = hk[(j - 1) / 2]; hv[j] = hv[(j - 1) / 2]; j = (j - 1) / 2; }
                hk[j] = nd; hv[j] = x;
            }
        }
    }
    if (solve_s) *solve_s = now_s() - t0;
    int status = sssp_output(n, d, dist_out);
    free(d); free(hk); free(hv); adj_free(&out);
    return status;
}

int oracle_bfs_queue_timed(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                           int32_t source, int32_t* level_out, double* solve_s) {
    if (n <= 0 || m < 0 || source < 0 || source >= n) return OR_E_ARG;
    int st = check_graph(n, m, src, dst, NULL);
    if (st) return st;
    adj_t out;
    if (adj_build(n, m, src, &out)) return OR_E_ARG;
    int64_t* d = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int32_t* q = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    double t0 = now_s();
    for (int64_t v = 0; v < n; ++v) d[v] = INF64;
    d[source] = 0;
    int64_t head = 0, tail = 0;
    q[tail++] = source;
    while (head < tail) {
        int32_t u = q[head++];
        for (int64_t a = out.rows[u]; a < out.rows[u + 1]; ++a) {
            int32_t x = dst[out.arc[a]];
            if (d[x] == INF64) { d[x] = d[u] + 1; q[tail++] = x; }
        }
    }
    if (solve_s) *solve_s = now_s() - t0;
    int status = sssp_output(n, d, level_out);
    free(d); free(q); adj_free(&out);
    return status;
}

/* ================================================================== */
/* Stable marriage, Section 5.4.                                        */
/*                                                                      */
/* G[m] = index into man m's preference list, from 0 (men propose).     */
/* target(m) = mpref[m][G[m]].  Man m is forbidden iff the woman he      */
/* targets prefers another man who also currently targets her; the      */
/* advance moves him one step down his list, alpha = G[m] + 1, bounded   */
/* by T[m] = n - 1.  Ranks: wrank[w][m] = position of m on w's list,     */
/* 0 = most preferred.                                                   */
/* ================================================================== */
static int sm_check(int32_t n, const int16_t* mpref, const int16_t* wrank) {
    for (int64_t i = 0; i < (int64_t)n * n; ++i) {
        if (mpref[i] < 0 || mpref[i] >= n) return OR_E_INPUT;
        if (wrank[i] < 0 || wrank[i] >= n) return OR_E_INPUT;
    }
    return OR_OK;
}

static void sm_output(int32_t n, const int16_t* mpref, const int64_t* G, int32_t* wife,
                      int32_t* prop) {
    for (int64_t m = 0; m < n; ++m) {
        wife[m] = mpref[m * n + G[m]];
        if (prop) prop[m] = (int32_t)G[m];
    }
}

/* Literal predicate: scan every other man (O(n) per evaluation, as the
   paper's implementation does).  Cyclic solver. */
int oracle_sm_scan(int32_t n, const int16_t* mpref, const int16_t* wrank, int64_t max_passes,
                   int32_t* wife, int32_t* prop, int64_t* passes_out) {
    if (n <= 0) return OR_E_ARG;
    int st = sm_check(n, mpref, wrank);
    if (st) return st;
    int64_t* G = (int64_t*)calloc((size_t)n, sizeof(int64_t));
    int64_t passes = 0;
    int status = OR_OK;
    for (;;) {
        int changed = 0;
        for (int64_t m = 0; m < n && status == OR_OK; ++m) {
            int64_t w = mpref[m * n + G[m]];
            int forbidden = 0;
            for (int64_t o = 0; o < n; ++o) {
                if (o == m) continue;
                if (mpref[o * n + G[o]] == w && wrank[w * n + o] < wrank[w * n + m]) { forbidden = 1; break; }
            }
            if (forbidden) {
                int64_t a = G[m] + 1;
                if (a > n - 1) { status = OR_E_INFEASIBLE; break; }
                G[m] = a;
                changed = 1;
            }
        }
        ++passes;
        if (status != OR_OK || !changed) break;
        if (max_passes > 0 && passes >= max_passes) { status = OR_E_NOT_CONVERGED; break; }
    }
    sm_output(n, mpref, G, wife, prop);
    if (passes_out) *passes_out = passes;
    free(G);
    return status;
}

/* Bag solver with a per-woman table best[w] = smallest rank of any man that
   has ever targeted w.  The man holding that rank is never forbidden at w
   (no better man can target w), so he never leaves, and best[w] equals the
   smallest rank among the men currently targeting w; the predicate
   "some man currently targeting w is ranked better than m" is therefore
   best[w] < wrank[w][m].  This is the per-woman shortcut the paper suggests
   in place of the O(n) scan; the test suite checks it against the scan.
   An advance of m pushes m and the man who held w' (the affected men). */
int oracle_sm_bag(int32_t n, const int16_t* mpref, const int16_t* wrank,
                  int32_t* wife, int32_t* prop, int64_t* evals_out) {
    if (n <= 0) return OR_E_ARG;
    int st = sm_check(n, mpref, wrank);
    if (st) return st;
    int64_t* G = (int64_t*)calloc((size_t)n, sizeof(int64_t));
    int64_t* best = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t* holder = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t* q = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    uint8_t* inq = (uint8_t*)calloc((size_t)n, 1);
    for (int64_t w = 0; w < n; ++w) { best[w] = n; holder[w] = -1; }
    int64_t head = 0, size = 0, evals = 0;
    for (int64_t m = 0; m < n; ++m) {
        int64_t w = mpref[m * n];
        int64_t r = wrank[w * n + m];
        if (r < best[w]) { best[w] = r; holder[w] = m; }
        q[size++] = m; inq[m] = 1;
    }
    int status = OR_OK;
    while (size > 0) {
        int64_t m = q[head]; head = (head + 1) % n; --size; inq[m] = 0;
        ++evals;
        int64_t w = mpref[m * n + G[m]];
        if (best[w] < wrank[w * n + m]) {                 /* forbidden */
            int64_t a = G[m] + 1;
            if (a > n - 1) { status = OR_E_INFEASIBLE; break; }
            G[m] = a;
            int64_t w2 = mpref[m * n + a];
            int64_t r2 = wrank[w2 * n + m];
            if (r2 < best[w2]) {
                int64_t prev = holder[w2];
                best[w2] = r2; holder[w2] = m;
                if (prev >= 0 && !inq[prev]) { inq[prev] = 1; q[(head + size) % n] = prev; ++size; }
            }
            if (!inq[m]) { inq[m] = 1; q[(head + size) % n] = m; ++size; }
        }
    }
    sm_output(n, mpref, G, wife, prop);
    if (evals_out) *evals_out = evals;
    free(G); free(best); free(holder); free(q); free(inq);
    return status;
}

/* ================================================================== */
/* Job scheduling, Section 5.5.                                         */
/*                                                                      */
/* The paper's state is the completion time C[j] with                   */
/* C[j] >= max_{p in P(j)} C[p] + t_j.  The oracle keeps the earliest   */
/* start time S[j] = C[j] - t_j, so the bottom is S = 0 and             */
/*     alpha(S, j) = max_{p in P(j)} (S[p] + t_p),  max over {} = 0.    */
/* Bound T[j] = 2^31 - 1 - t_j (the completion time must fit int32).    */
/* The READY conjunct of the paper's predicate only restricts which      */
/* indices a schedule may look at, not the least fixpoint, so the cyclic */
/* solver uses the plain inequality; the bag solver below follows the    */
/* paper's ready-counter implementation.  A cycle is reported up front   */
/* (Kahn's algorithm): on a cycle of positive duration the least         */
/* fixpoint does not exist.                                              */
/* ================================================================== */
static int jobs_check(int32_t n, const int32_t* pp, const int32_t* pi, const int32_t* dur) {
    if (pp[0] != 0) return OR_E_INPUT;
    for (int64_t j = 0; j < n; ++j) {
        if (pp[j + 1] < pp[j]) return OR_E_INPUT;
        if (dur[j] < 0) return OR_E_INPUT;
    }
    for (int64_t k = 0; k < pp[n]; ++k) if (pi[k] < 0 || pi[k] >= n) return OR_E_INPUT;
    return OR_OK;
}

static int jobs_is_dag(int32_t n, const int32_t* pp, const int32_t* pi) {
    int64_t E = pp[n];
    int64_t* indeg = (int64_t*)calloc((size_t)n, sizeof(int64_t));
    adj_t succ;
    int32_t* parent = (int32_t*)malloc(sizeof(int32_t) * (size_t)(E > 0 ? E : 1));
    for (int64_t j = 0; j < n; ++j)
        for (int64_t k = pp[j]; k < pp[j + 1]; ++k) { indeg[j]++; parent[k] = pi[k]; }
    adj_build(n, E, parent, &succ);
    /* child of arc k */
    int32_t* child = (int32_t*)malloc(sizeof(int32_t) * (size_t)(E > 0 ? E : 1));
    for (int64_t j = 0; j < n; ++j) for (int64_t k = pp[j]; k < pp[j + 1]; ++k) child[k] = (int32_t)j;
    int64_t* q = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t qh = 0, qt = 0;
    for (int64_t j = 0; j < n; ++j) if (indeg[j] == 0) q[qt++] = j;
    while (qh < qt) {
        int64_t p = q[qh++];
        for (int64_t k = succ.rows[p]; k < succ.rows[p + 1]; ++k) {
            int64_t c = child[succ.arc[k]];
            if (--indeg[c] == 0) q[qt++] = c;
        }
    }
    free(indeg); free(parent); free(child); free(q); adj_free(&succ);
    return qt == n;
}

int oracle_jobs_cyclic(int32_t n, const int32_t* pred_ptr, const int32_t* pred_idx,
                       const int32_t* dur, int64_t max_passes, int32_t* start,
                       int64_t* passes_out) {
    if (n <= 0) return OR_E_ARG;
    int st = jobs_check(n, pred_ptr, pred_idx, dur);
    if (st) return st;
    if (!jobs_is_dag(n, pred_ptr, pred_idx)) return OR_E_CYCLE;
    int64_t* S = (int64_t*)calloc((size_t)n, sizeof(int64_t));
    int64_t passes = 0;
    int status = OR_OK;
    for (;;) {
        int changed = 0;
        for (int64_t j = 0; j < n && status == OR_OK; ++j) {
            int64_t a = 0;
            for (int64_t k = pred_ptr[j]; k < pred_ptr[j + 1]; ++k) {
                int64_t p = pred_idx[k];
                if (S[p] + dur[p] > a) a = S[p] + dur[p];
            }
            if (a > S[j]) {
                if (a > I32MAX - dur[j]) { status = OR_E_OVERFLOW; break; }
                S[j] = a;
                changed = 1;
            }
        }
        ++passes;
        if (status != OR_OK || !changed) break;
        if (max_passes > 0 && passes >= max_passes) { status = OR_E_NOT_CONVERGED; break; }
    }
    for (int64_t j = 0; j < n; ++j) start[j] = (int32_t)(S[j] > I32MAX ? I32MAX : S[j]);
    if (passes_out) *passes_out = passes;
    free(S);
    return status;
}

/* Bag solver with the paper's readiness counters: a job enters the bag when
   its last predecessor has been fixed; it is then advanced to the maximum
   its predecessors published and fixed, exactly once. */
int oracle_jobs_bag(int32_t n, const int32_t* pred_ptr, const int32_t* pred_idx,
                    const int32_t* dur, int32_t* start) {
    if (n <= 0) return OR_E_ARG;
    int st = jobs_check(n, pred_ptr, pred_idx, dur);
    if (st) return st;
    int64_t E = pred_ptr[n];
    int32_t* parent = (int32_t*)malloc(sizeof(int32_t) * (size_t)(E > 0 ? E : 1));
    int32_t* child = (int32_t*)malloc(sizeof(int32_t) * (size_t)(E > 0 ? E : 1));
    for (int64_t j = 0; j < n; ++j)
        for (int64_t k = pred_ptr[j]; k < pred_ptr[j + 1]; ++k) { parent[k] = pred_idx[k]; child[k] = (int32_t)j; }
    adj_t succ;
    adj_build(n, E, parent, &succ);
    int64_t* remaining = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t* mfp = (int64_t*)calloc((size_t)n, sizeof(int64_t));
    int64_t* S = (int64_t*)calloc((size_t)n, sizeof(int64_t));
    int64_t* q = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t qh = 0, qt = 0;
    for (int64_t j = 0; j < n; ++j) {
        remaining[j] = pred_ptr[j + 1] - pred_ptr[j];
        if (remaining[j] == 0) q[qt++] = j;
    }
    int status = OR_OK;
    while (qh < qt) {
        int64_t j = q[qh++];
        S[j] = mfp[j];
        if (S[j] > I32MAX - dur[j]) { status = OR_E_OVERFLOW; break; }
        int64_t c_j = S[j] + dur[j];
        for (int64_t k = succ.rows[j]; k < succ.rows[j + 1]; ++k) {
            int64_t c = child[succ.arc[k]];
            if (c_j > mfp[c]) mfp[c] = c_j;
            if (--remaining[c] == 0) q[qt++] = c;
        }
    }
    if (status == OR_OK && qt != n) status = OR_E_CYCLE;
    for (int64_t j = 0; j < n; ++j) start[j] = (int32_t)(S[j] > I32MAX ? I32MAX : S[j]);
    free(parent); free(child); free(remaining); free(mfp); free(S); free(q); adj_free(&succ);
    return status;
}

/* ================================================================== */
/* 0-1 knapsack, Section 5.8.                                           */
/*                                                                      */
/* Cells G[k][c], k = 0..n items, c = 0..W capacity (inclusive), all 0   */
/* at the bottom; row 0 has no item and stays 0.  Cell (k, c), k >= 1,  */
/* is forbidden iff it is below the recurrence                          */
/*     alpha = max( G[k-1][c], v_k + G[k-1][c - w_k] if c >= w_k ).     */
/* The answer is G[n][W]; the whole last row is returned on request.    */
/* Cyclic solver over the cells in row-major order.                     */
/* ================================================================== */
int oracle_knapsack(int32_t items, int32_t W, const int32_t* wt, const int32_t* val,
                    int64_t max_passes, int32_t* best, int32_t* last_row, int64_t* passes_out) {
    if (items < 0 || W < 0) return OR_E_ARG;
    for (int64_t k = 0; k < items; ++k) if (wt[k] < 0 || val[k] < 0) return OR_E_INPUT;
    int64_t cols = (int64_t)W + 1;
    int64_t* G = (int64_t*)calloc((size_t)((items + 1) * cols), sizeof(int64_t));
    int64_t passes = 0;
    int status = OR_OK;
    for (;;) {
        int changed = 0;
        for (int64_t k = 1; k <= items; ++k) {
            int64_t wk = wt[k - 1], vk = val[k - 1];
            for (int64_t c = 0; c <= W; ++c) {
                int64_t a = G[(k - 1) * cols + c];
                if (c >= wk && G[(k - 1) * cols + c - wk] + vk > a) a = G[(k - 1) * cols + c - wk] + vk;
                if (a > G[k * cols + c]) {
                    if (a > I32MAX) status = OR_E_OVERFLOW;
                    G[k * cols + c] = a;
                    changed = 1;
                }
            }
        }
        ++passes;
        if (!changed || status != OR_OK) break;
        if (max_passes > 0 && passes >= max_passes) { status = OR_E_NOT_CONVERGED; break; }
    }
    int64_t b = G[items * cols + W];
    *best = (int32_t)(b > I32MAX ? I32MAX : b);
    if (last_row)
        for (int64_t c = 0; c <= W; ++c) {
            int64_t x = G[items * cols + c];
            last_row[c] = (int32_t)(x > I32MAX ? I32MAX : x);
        }
    if (passes_out) *passes_out = passes;
    free(G);
    return status;
}

/* ================================================================== */
/* Transitive closure, Section 5.7.                                     */
/*                                                                      */
/* Boolean state G[u][v] (reachable by a path of length >= 1), bottom   */
/* all false.  Pair (u, v) is forbidden iff G[u][v] is false and either  */
/* (u, v) is an arc or some w has G[u][w] and G[w][v]; the advance sets  */
/* G[u][v] = true.  Output rows of ceil(n/32) uint32 words, bit v & 31   */
/* of word v >> 5 (least significant bit = lowest column).               */
/* Cyclic solver over pairs in row-major order.                          */
/* ================================================================== */
int oracle_tc(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
              uint32_t* bits_out, int64_t* passes_out) {
    if (n <= 0 || m < 0) return OR_E_ARG;
    int st = check_graph(n, m, src, dst, NULL);
    if (st) return st;
    uint8_t* A = (uint8_t*)calloc((size_t)n * n, 1);
    uint8_t* G = (uint8_t*)calloc((size_t)n * n, 1);
    for (int64_t e = 0; e < m; ++e) A[(int64_t)src[e] * n + dst[e]] = 1;
    int64_t passes = 0;
    for (;;) {
        int changed = 0;
        for (int64_t u = 0; u < n; ++u)
            for (int64_t v = 0; v < n; ++v) {
                if (G[u * n + v]) continue;
                int forbidden = A[u * n + v];
                for (int64_t x = 0; x < n && !forbidden; ++x)
                    if (G[u * n + x] && G[x * n + v]) forbidden = 1;
                if (forbidden) { G[u * n + v] = 1; changed = 1; }
            }
        ++passes;
        if (!changed) break;
    }
    int64_t words = (n + 31) / 32;
    memset(bits_out, 0, sizeof(uint32_t) * (size_t)(n * words));
    for (int64_t u = 0; u < n; ++u)
        for (int64_t v = 0; v < n; ++v)
            if (G[u * n + v]) bits_out[u * words + (v >> 5)] |= 1u << (v & 31);
    if (passes_out) *passes_out = passes;
    free(A); free(G);
    return OR_OK;
}

/* ================================================================== */
/* Parallel reduction, Section 5.6: the root of the combine tree holds   */
/* the sum of the inputs under 64-bit integer addition (wrap-around),    */
/* whatever the tree shape.  The oracle is that definition.              */
/* ================================================================== */
uint64_t oracle_reduce(int64_t n, const uint64_t* x) {
    uint64_t s = 0;
    for (int64_t i = 0; i < n; ++i) s += x[i];
    return s;
}
