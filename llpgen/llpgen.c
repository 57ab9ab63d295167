/*
 * llpgen.c - seeded synthetic input generators for the LLP sweep.
 *
 * This file only draws random numbers and lays inputs out (edge lists,
 * compressed sparse rows, preference tables, DAGs, item lists).  It holds
 * none of the method's arithmetic: no forbidden test, no advance, no
 * fixpoint.  Both the CPU oracle tests and the GPU path consume its output.
 *
 * Random numbers: counter-based splitmix64 (Steele, Lea and Flood, "Fast
 * splittable pseudorandom number generators", OOPSLA 2014).  Draw i of a
 * stream with key k is mix64(k + (i + 1) * GAMMA), i.e. the i-th output of a
 * splitmix64 generator seeded with k, so every draw is independent of thread
 * count and loop order.  A stream key is mix64(seed * GAMMA ^ tag) for a
 * fixed per-purpose tag.
 *
 * Integer ranges use the multiply-shift map ((hi32 * span) >> 32).
 * Poisson variates use sequential inversion; permutations use Fisher-Yates.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC llpgen.c -o libllpgen.so
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t llpgen_mix64(uint64_t z) { return mix64(z); }

uint64_t llpgen_key(uint64_t seed, uint64_t tag) { return mix64(seed * GAMMA ^ tag); }

static inline uint64_t draw(uint64_t key, uint64_t i) { return mix64(key + (i + 1) * GAMMA); }

uint64_t llpgen_draw(uint64_t key, uint64_t i) { return draw(key, i); }

/* uniform integer in [lo, hi] from the high 32 bits of a draw */
static inline int64_t urange(uint64_t d, int64_t lo, int64_t hi) {
    uint64_t span = (uint64_t)(hi - lo + 1);
    return lo + (int64_t)(((d >> 32) * span) >> 32);
}

/* Stream tags (arbitrary distinct constants). */
enum {
    TAG_U = 0x11, TAG_V = 0x12, TAG_W = 0x13, TAG_CYCW = 0x14,
    TAG_RMAT = 0x21, TAG_PERM = 0x22,
    TAG_GRIDW = 0x31,
    TAG_MPREF = 0x41, TAG_WPREF = 0x42,
    TAG_DAGK = 0x51, TAG_DAGP = 0x52, TAG_DAGT = 0x53,
    TAG_KN = 0x61, TAG_KW = 0x62, TAG_KWT = 0x63, TAG_KVAL = 0x64,
    TAG_U64 = 0x71
};

/* ------------------------------------------------------------------ */
/* Uniform random directed graph with an appended Hamiltonian cycle.    */
/* Arc e < m_rand: u ~ U[0,n), v uniform over the n-1 vertices != u.    */
/* Arcs m_rand .. m_rand+n-1: i -> (i+1) mod n (only when cycle != 0).  */
/* Weights U[wlo, whi] on every arc.                                    */
/* ------------------------------------------------------------------ */
void llpgen_uniform(int32_t n, int64_t m_rand, int32_t cycle, int32_t wlo, int32_t whi,
                    uint64_t seed, int32_t* src, int32_t* dst, int32_t* w) {
    uint64_t ku = llpgen_key(seed, TAG_U), kv = llpgen_key(seed, TAG_V), kw = llpgen_key(seed, TAG_W);
    #pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m_rand; ++e) {
        int32_t u = (int32_t)urange(draw(ku, e), 0, n - 1);
        int32_t off = (int32_t)urange(draw(kv, e), 1, n - 1);
        src[e] = u;
        dst[e] = (int32_t)(((int64_t)u + off) % n);
        w[e] = (int32_t)urange(draw(kw, e), wlo, whi);
    }
    if (cycle) {
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            src[m_rand + i] = (int32_t)i;
            dst[m_rand + i] = (int32_t)((i + 1) % n);
            w[m_rand + i] = (int32_t)urange(draw(kw, m_rand + i), wlo, whi);
        }
    }
}

/* ------------------------------------------------------------------ */
/* Fisher-Yates permutation of [0, n) from stream key k.               */
/* ------------------------------------------------------------------ */
static void fy_perm(int64_t n, uint64_t k, int32_t* p) {
    for (int64_t i = 0; i < n; ++i) p[i] = (int32_t)i;
    for (int64_t i = n - 1; i > 0; --i) {
        int64_t j = urange(draw(k, (uint64_t)i), 0, i);
        int32_t t = p[i]; p[i] = p[j]; p[j] = t;
    }
}

void llpgen_perm(int64_t n, uint64_t seed, uint64_t tag, int32_t* p) {
    fy_perm(n, llpgen_key(seed, tag), p);
}

/* ------------------------------------------------------------------ */
/* R-MAT graph (Chakrabarti, Zhan and Faloutsos 2004), scale s,         */
/* edge factor ef: 2^s * ef arcs; at each of the s bit levels the       */
/* (row, col) quadrant is chosen with probabilities (a, b, c, d).       */
/* Self-loops and duplicates are kept.  If relabel != 0, vertex ids are */
/* mapped through a seeded random permutation.  If cycle != 0, the arcs */
/* i -> (i+1) mod n are appended after the R-MAT arcs.                  */
/* Weights U[wlo, whi] on every arc.                                    */
/* ------------------------------------------------------------------ */
void llpgen_rmat(int32_t scale, int32_t ef, double a, double b, double c,
                 int32_t relabel, int32_t cycle, int32_t wlo, int32_t whi, uint64_t seed,
                 int32_t* src, int32_t* dst, int32_t* w) {
    const int64_t n = (int64_t)1 << scale;
    const int64_t m_r = n * ef;
    const uint64_t kr = llpgen_key(seed, TAG_RMAT), kw = llpgen_key(seed, TAG_W);
    const uint64_t ta = (uint64_t)(a * 4294967296.0);
    const uint64_t tb = (uint64_t)((a + b) * 4294967296.0);
    const uint64_t tc = (uint64_t)((a + b + c) * 4294967296.0);
    const int64_t words = (scale + 1) / 2;  /* two 32-bit levels per 64-bit draw */
    int32_t* perm = NULL;
    if (relabel) {
        perm = (int32_t*)malloc(sizeof(int32_t) * n);
        fy_perm(n, llpgen_key(seed, TAG_PERM), perm);
    }
    #pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m_r; ++e) {
        uint32_t u = 0, v = 0;
        for (int64_t k = 0; k < words; ++k) {
            uint64_t d = draw(kr, (uint64_t)(e * words + k));
            for (int h = 0; h < 2; ++h) {
                int level = (int)(2 * k + h);
                if (level >= scale) break;
                uint64_t r = h ? (d >> 32) : (d & 0xFFFFFFFFULL);
                uint32_t ub, vb;
                if (r < ta) { ub = 0; vb = 0; }
                else if (r < tb) { ub = 0; vb = 1; }
                else if (r < tc) { ub = 1; vb = 0; }
                else { ub = 1; vb = 1; }
                u |= ub << level;
                v |= vb << level;
            }
        }
        src[e] = relabel ? perm[u] : (int32_t)u;
        dst[e] = relabel ? perm[v] : (int32_t)v;
        w[e] = (int32_t)urange(draw(kw, (uint64_t)e), wlo, whi);
    }
    if (cycle) {
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            src[m_r + i] = (int32_t)i;
            dst[m_r + i] = (int32_t)((i + 1) % n);
            w[m_r + i] = (int32_t)urange(draw(kw, (uint64_t)(m_r + i)), wlo, whi);
        }
    }
    free(perm);
}

/* ------------------------------------------------------------------ */
/* 2-D grid, rows x cols, 4-neighbour, both arc directions, weights     */
/* U[wlo, whi] drawn independently per arc.  Vertex id = r * cols + c.  */
/* Arcs are emitted per vertex in id order, neighbours in the order     */
/* up, left, right, down.  Returns the arc count.                        */
/* ------------------------------------------------------------------ */
int64_t llpgen_grid_arcs(int32_t rows, int32_t cols) {
    return 2 * ((int64_t)rows * (cols - 1) + (int64_t)(rows - 1) * cols);
}

void llpgen_grid(int32_t rows, int32_t cols, int32_t wlo, int32_t whi, uint64_t seed,
                 int32_t* src, int32_t* dst, int32_t* w) {
    const uint64_t kw = llpgen_key(seed, TAG_GRIDW);
    #pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < rows; ++r) {
        /* arcs emitted before row r: 2(cols-1) horizontal arcs per row, plus one
           vertical arc per vertex for each of "has a row above" / "has a row below" */
        int64_t above = r > 0 ? r - 1 : 0;                 /* rows rr in [1, r) */
        int64_t below = r < rows - 1 ? r : rows - 1;       /* rows rr in [0, min(r, rows-1)) */
        int64_t base = r * 2 * (int64_t)(cols - 1) + (above + below) * cols;
        int64_t e = base;
        for (int64_t c = 0; c < cols; ++c) {
            int32_t v = (int32_t)(r * cols + c);
            if (r > 0) { src[e] = v; dst[e] = v - cols; w[e] = (int32_t)urange(draw(kw, e), wlo, whi); ++e; }
            if (c > 0) { src[e] = v; dst[e] = v - 1; w[e] = (int32_t)urange(draw(kw, e), wlo, whi); ++e; }
            if (c < cols - 1) { src[e] = v; dst[e] = v + 1; w[e] = (int32_t)urange(draw(kw, e), wlo, whi); ++e; }
            if (r < rows - 1) { src[e] = v; dst[e] = v + cols; w[e] = (int32_t)urange(draw(kw, e), wlo, whi); ++e; }
        }
    }
}

/* ------------------------------------------------------------------ */
/* Stable-marriage preferences: every man's list and every woman's list */
/* is an independent uniform permutation.  mpref[m*n + i] = i-th woman  */
/* on man m's list (0 = most preferred).  wrank[w*n + m] = rank of man  */
/* m on woman w's list (0 = most preferred).                             */
/* ------------------------------------------------------------------ */
void llpgen_sm(int32_t n, uint64_t seed, int16_t* mpref, int16_t* wrank) {
    const uint64_t km = llpgen_key(seed, TAG_MPREF), kf = llpgen_key(seed, TAG_WPREF);
    #pragma omp parallel
    {
        int32_t* p = (int32_t*)malloc(sizeof(int32_t) * n);
        #pragma omp for schedule(static)
        for (int64_t m = 0; m < n; ++m) {
            fy_perm(n, mix64(km ^ (uint64_t)m * GAMMA), p);
            for (int64_t i = 0; i < n; ++i) mpref[m * n + i] = (int16_t)p[i];
        }
        #pragma omp for schedule(static)
        for (int64_t wmn = 0; wmn < n; ++wmn) {
            fy_perm(n, mix64(kf ^ (uint64_t)wmn * GAMMA), p);   /* p[i] = i-th man on her list */
            for (int64_t i = 0; i < n; ++i) wrank[wmn * n + p[i]] = (int16_t)i;
        }
        free(p);
    }
}

/* ------------------------------------------------------------------ */
/* Random job DAG.  Job j draws k_j = min(Poisson(lam), j) distinct     */
/* parents uniformly from [0, j) and a duration U[dlo, dhi].             */
/* Pass pred_idx == NULL to get only the in-degree counts (pred_ptr).    */
/* ------------------------------------------------------------------ */
static int32_t poisson_inv(double lam, uint64_t d) {
    double u = (double)(d >> 11) * (1.0 / 9007199254740992.0);
    double p = exp(-lam), s = p;
    int32_t k = 0;
    while (u > s && k < 1000) { ++k; p *= lam / k; s += p; }
    return k;
}

void llpgen_dag(int32_t n, double lam, int32_t dlo, int32_t dhi, uint64_t seed,
                int32_t* pred_ptr, int32_t* pred_idx, int32_t* dur) {
    const uint64_t kk = llpgen_key(seed, TAG_DAGK), kp = llpgen_key(seed, TAG_DAGP), kt = llpgen_key(seed, TAG_DAGT);
    if (pred_idx == NULL) {
        pred_ptr[0] = 0;
        for (int64_t j = 0; j < n; ++j) {
            int32_t k = poisson_inv(lam, draw(kk, j));
            if (k > j) k = (int32_t)j;
            pred_ptr[j + 1] = pred_ptr[j] + k;
        }
        return;
    }
    #pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t j = 0; j < n; ++j) {
        int32_t b = pred_ptr[j], k = pred_ptr[j + 1] - b;
        dur[j] = (int32_t)urange(draw(kt, j), dlo, dhi);
        if (k == j) { for (int32_t i = 0; i < k; ++i) pred_idx[b + i] = i; continue; }
        uint64_t t = 0;
        for (int32_t i = 0; i < k;) {
            int32_t cand = (int32_t)urange(draw(kp, (uint64_t)j * 4096 + t), 0, j - 1);
            ++t;
            int dup = 0;
            for (int32_t q = 0; q < i; ++q) if (pred_idx[b + q] == cand) { dup = 1; break; }
            if (!dup) pred_idx[b + i++] = cand;
        }
    }
}

/* ------------------------------------------------------------------ */
/* 0-1 knapsack instance i of a family: item count U[nlo, nhi],          */
/* capacity U[wlo, whi], weights U[1, floor(W/4)], values U[1, vmax].    */
/* First call with wt == NULL returns (items, W) via out2.               */
/* ------------------------------------------------------------------ */
void llpgen_knapsack(uint64_t seed, int64_t inst, int32_t nlo, int32_t nhi, int32_t Wlo, int32_t Whi,
                     int32_t vmax, int32_t* out2, int32_t* wt, int32_t* val) {
    const uint64_t kn = llpgen_key(seed, TAG_KN), kW = llpgen_key(seed, TAG_KW);
    int32_t items = (int32_t)urange(draw(kn, inst), nlo, nhi);
    int32_t W = (int32_t)urange(draw(kW, inst), Wlo, Whi);
    out2[0] = items; out2[1] = W;
    if (wt == NULL) return;
    const uint64_t kwt = mix64(llpgen_key(seed, TAG_KWT) ^ (uint64_t)inst * GAMMA);
    const uint64_t kv = mix64(llpgen_key(seed, TAG_KVAL) ^ (uint64_t)inst * GAMMA);
    int32_t wmax = W / 4 < 1 ? 1 : W / 4;
    for (int32_t i = 0; i < items; ++i) {
        wt[i] = (int32_t)urange(draw(kwt, i), 1, wmax);
        val[i] = (int32_t)urange(draw(kv, i), 1, vmax);
    }
}

/* ------------------------------------------------------------------ */
/* n uniform 64-bit words.                                              */
/* ------------------------------------------------------------------ */
void llpgen_u64(int64_t n, uint64_t seed, uint64_t* x) {
    const uint64_t k = llpgen_key(seed, TAG_U64);
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) x[i] = draw(k, (uint64_t)i);
}

/* ------------------------------------------------------------------ */
/* Stable counting sort of m items by key in [0, n): ptr[n+1] gets the  */
/* row offsets; a_out/b_out receive a/b in sorted order (b may be NULL).*/
/* Used to lay edge lists out as compressed sparse rows.                 */
/* ------------------------------------------------------------------ */
void llpgen_csr(int32_t n, int64_t m, const int32_t* key, const int32_t* a, const int32_t* b,
                int32_t* ptr, int32_t* a_out, int32_t* b_out) {
    int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t e = 0; e < m; ++e) cnt[key[e] + 1]++;
    for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    for (int64_t i = 0; i <= n; ++i) ptr[i] = (int32_t)cnt[i];
    for (int64_t e = 0; e < m; ++e) {
        int64_t pos = cnt[key[e]]++;
        a_out[pos] = a[e];
        if (b) b_out[pos] = b[e];
    }
    free(cnt);
}
