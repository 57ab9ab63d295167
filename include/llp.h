/*
 * llp.h - C ABI of libllp, the MI355X (gfx950) lattice-linear-predicate sweep.
 *
 * The library computes the least vector G of a lattice of bounded int32
 * vectors that satisfies a lattice-linear predicate B (paper, Background:
 * Definitions 1-3 and Algorithm LLP): starting from the bottom, every
 * forbidden index j is advanced to alpha(G, j) in parallel, without locks,
 * until no index is forbidden.  Advances are monotone atomic maxima, so any
 * schedule reaches the same least fixpoint and every output is bit-exact
 * whatever schedule, option, tile size or replay produced it.
 *
 * Conventions for every entry point
 *  - Pointers marked [device] are HIP device memory (for instance the data
 *    pointer of a torch CUDA tensor); all others are host memory.
 *  - The caller owns every input, output and workspace buffer; the library
 *    never frees caller memory.  The library owns only its lazily created
 *    per-device state (kernel occupancy table, learned-scheduler weights,
 *    instantiated hipGraphs, a fallback workspace), released by llp_shutdown().
 *  - All device work is enqueued on opts->stream (a hipStream_t; NULL = the
 *    default stream).  Unless LLP_ASYNC is set, the call waits for its own
 *    work and returns the final status.  With LLP_ASYNC it returns LLP_OK once
 *    the work is enqueued and the device writes the status to
 *    opts->status_dev (required with LLP_ASYNC).
 *  - A nonzero return is an llp_status; llp_last_error() gives a
 *    thread-local message.  No exception crosses the ABI.
 *  - Outputs are defined for LLP_OK and LLP_E_NOT_CONVERGED (the partial
 *    state, decoded); undefined for every other status.
 *  - opts may be NULL (defaults).  Calls on distinct streams with distinct
 *    workspaces may run concurrently.
 */
#ifndef LLP_H
#define LLP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LLP_OK = 0,
    LLP_E_ARG = 1,           /* bad host argument (size, null pointer, option) */
    LLP_E_INPUT = 2,         /* device validation failed (id out of range, negative weight, ...) */
    LLP_E_INFEASIBLE = 3,    /* Algorithm LLP returns null: alpha exceeded the bound T[j] */
    LLP_E_OVERFLOW = 4,      /* a result does not fit int32 */
    LLP_E_NOT_CONVERGED = 5, /* max_rounds reached; the partial state is decoded into the output */
    LLP_E_WORKSPACE = 6,     /* workspace too small */
    LLP_E_HIP = 7,           /* HIP runtime error or device watchdog */
    LLP_E_CYCLE = 8,         /* job graph has a cycle */
    LLP_E_ABORTED = 9        /* host abort flag observed */
} llp_status;

/* Schedules.  Every schedule reaches the same least fixpoint. */
#define LLP_SCHED_PLAIN   0u  /* pull over the in-CSR on a compacted candidate worklist */
#define LLP_SCHED_FIXED   1u  /* the mode given by flags (LLP_PUSH / LLP_DENSE) and delta, every round */
#define LLP_SCHED_LEARNED 2u  /* per round, the loaded MLP picks push/pull, dense/worklist and delta; rounds
                                 of fewer than m/256 frontier arcs take the HYBRID code instead */
#define LLP_SCHED_HYBRID  3u  /* per round, a frontier-width threshold: dense when the changed vertices'
                                 out-arcs exceed a fraction of all arcs (SSSP 1/3, BFS 1/14, jobs 1/2),
                                 push otherwise (pull without out_w); on weighted graphs of 2 to 8
                                 arcs per vertex the push rounds use the wide delta buckets */
#define LLP_SCHED_RANDOM  4u  /* per round, a seeded random mode and delta class (schedule-independence tests) */
#define LLP_SCHED_SCRIPT  5u  /* per round, the code opts->plan[r-1] (plain after the plan ends); used to
                                 measure what a decision at a given round costs when training the scheduler */

/* Round codes (llp_trace_rec.mode, opts->plan): bits 0-1 the mode (0 pull over
   the candidate worklist, 1 dense pull, 2 push), bits 8-9 the delta class:
   0 = the base width (2^floor(log2 of the mean arc weight), estimated from a
   sample of the arcs; 1 for BFS), 1 = 64 x the base width, 2 = no buckets,
   3 = opts->delta.  In LLP_SCHED_SCRIPT plans, mode 3 means "the round the
   frontier-width hybrid would run".  With a delta width D, a round only expands (or pushes
   from) the changed vertices whose distance lies below floor(dmin / D) * D + D,
   dmin the smallest distance among them; the others are carried to the next
   round (delta-stepping buckets, paper Section 4.2).  Dense rounds ignore
   the buckets. */
#define LLP_ROUND_CODE(mode, dclass) ((int32_t)((mode) | ((dclass) << 8)))

/* Flags. */
#define LLP_PUSH      (1u << 0)  /* FIXED: push single-arc partial advances along out-arcs */
#define LLP_DENSE     (1u << 1)  /* FIXED: evaluate every index each round (no worklist) */
#define LLP_VALIDATE  (1u << 2)  /* validate inputs on the device first (LLP_E_INPUT) */
#define LLP_ASYNC     (1u << 3)  /* return after enqueueing; status goes to status_dev */
#define LLP_VERIFY    (1u << 4)  /* after convergence, one dense round must change nothing */
#define LLP_TRACE     (1u << 5)  /* write one llp_trace_rec per round to trace_dev */
#define LLP_TIMING    (1u << 6)  /* fill stats->device_ms / kernel_ms with hipEvent times */
#define LLP_JOBS_PULL (1u << 7)  /* jobs: pull over predecessors instead of readiness counters */

/* Per-solve counters (host struct, filled when opts->stats != NULL). */
typedef struct {
    int64_t rounds;           /* sweep rounds executed */
    int64_t candidates;       /* indices evaluated by pull rounds (every index in a dense round) */
    int64_t edges_inspected;  /* in-arcs read by pull rounds */
    int64_t advances;         /* entries of the changed lists consumed (indices advanced) */
    int64_t expand_edges;     /* out-arcs read by successor expansion */
    int64_t eval_launches;    /* step launches that evaluated a pull or dense round (LLP_TIMING; a dense
                                 round is decided and evaluated in one launch, a bitmap round in two) */
    float device_ms;          /* whole solve on the stream (LLP_TIMING) */
    float kernel_ms;          /* summed duration of the evaluation (MAIN) kernel launches (LLP_TIMING) */
    int64_t push_edges;       /* out-arcs read by push rounds */
    int64_t pre_launches;     /* step launches that only expanded or pushed (LLP_TIMING) */
    float pre_ms;             /* summed duration of the PRE kernel launches (LLP_TIMING) */
    float pad;
    int64_t states_gathered;  /* tail states read by pull rounds: edges_inspected less the arcs a dense
                                 round proves unable to improve their row (not gathered), and less
                                 every arc of a bitmap round */
    int64_t bitmap_rounds;    /* BFS dense rounds that looked their tails up in a bitmap of n bits
                                 (marked: distance <= the smallest of the input list), built from the
                                 state array by a step launch of the round's own, instead of gathering
                                 tail states; such a round takes two step launches */
} llp_stats;

/* One record per round when LLP_TRACE is set (device buffer of trace_cap records). */
typedef struct {
    int32_t round;
    int32_t mode;             /* round code (LLP_ROUND_CODE): bits 0-1 mode, bits 8-9 delta class */
    int32_t in_count;         /* changed indices the round consumed (its input list) */
    int32_t out_count;        /* pull rounds: candidates evaluated; 0 for dense and push rounds */
    int64_t in_edges;         /* out-arcs of the input list */
    int64_t out_edges;        /* pull rounds: in-arcs of the candidates */
    int32_t bucket;           /* delta-bucket floor (distance) or -1 */
    int32_t pending;          /* changed vertices carried to the next round by the delta filter (and by a
                                 BFS bitmap round) */
    int32_t bitmap;           /* 1: a BFS dense round evaluated with the bitmap (two step launches;
                                 see llp_stats.bitmap_rounds) */
    int32_t pad;
} llp_trace_rec;

typedef struct {
    uint32_t size;              /* sizeof(llp_opts), for ABI evolution; 0 = treat as current */
    uint32_t sched;             /* LLP_SCHED_* */
    uint32_t flags;             /* LLP_* flags */
    int32_t delta;              /* FIXED: delta-bucket width in distance units, 0 = none */
    int64_t max_rounds;         /* watchdog; 0 = problem default (4n + 64 rounds for graphs, n + 2 for jobs) */
    void* workspace;            /* [device] caller scratch, >= llp_workspace_bytes(); NULL = library-owned */
    size_t workspace_bytes;
    void* stream;               /* hipStream_t */
    const int32_t* warm_start;  /* [device] optional: a previous output (<= the fixpoint in the lattice order) */
    int32_t* status_dev;        /* [device] optional status word (required with LLP_ASYNC) */
    volatile int32_t* abort_host; /* [host, pinned] optional: a nonzero value aborts at the next round */
    llp_stats* stats;           /* [host] optional */
    int32_t chunk;              /* launch knob, 0 = default: graph sweeps: workgroups (list segments) per CU
                                   (default 2, at most 8; pass the same opts to llp_workspace_bytes);
                                   stable marriage: proposals per thread per launch; batch: instances per
                                   queue claim; jobs readiness: widest level, in arcs, run by one
                                   workgroup in LDS (default and most 1024; -1 = none) */
    int32_t block;              /* threads per workgroup; 0 = default (256) */
    llp_trace_rec* trace_dev;   /* [device] LLP_TRACE output */
    int64_t trace_cap;
    uint64_t seed;              /* LLP_SCHED_RANDOM seed */
    const int32_t* plan;        /* [device] LLP_SCHED_SCRIPT: round codes for rounds 1..plan_len */
    int64_t plan_len;
} llp_opts;

/* Directed graph as compressed sparse rows, int32 ids, m < 2^31.
   In-CSR (arcs grouped by head v): in_ptr[n+1], in_src[m] (tail u), in_w[m].
   Out-CSR (arcs grouped by tail u): out_ptr[n+1], out_dst[m], out_w[m].
   The pull sweep needs the in-CSR; successor expansion needs out_ptr/out_dst;
   push rounds need out_w.  in_w / out_w are NULL for BFS. */
typedef struct {
    int32_t n;
    int64_t m;
    const int32_t* in_ptr;   /* [device] */
    const int32_t* in_src;   /* [device] */
    const int32_t* in_w;     /* [device] weights >= 0, or NULL */
    const int32_t* out_ptr;  /* [device] */
    const int32_t* out_dst;  /* [device] */
    const int32_t* out_w;    /* [device] or NULL (push rounds are then unavailable for SSSP) */
} llp_graph;

/* Scratch bytes a solve of this kind and size needs in opts->workspace.
   kind: LLP_KIND_* below; n = vertices/men/jobs/items/elements, m = arcs (or
   knapsack capacity W, or batch instance count). */
#define LLP_KIND_SSSP     1
#define LLP_KIND_BFS      2
#define LLP_KIND_SM       3
#define LLP_KIND_JOBS     4
#define LLP_KIND_KNAPSACK 5
#define LLP_KIND_TC       6
#define LLP_KIND_REDUCE   7
#define LLP_KIND_BATCH    8
size_t llp_workspace_bytes(int kind, int64_t n, int64_t m, const llp_opts* opts);

/* Single-source shortest paths (paper Section 5.2).  State G[v] = 2^31-1 - d(v)
   (0 = not reached), advanced by atomicMax; alpha(G, v) is the largest
   G[u] - w(u, v) over in-arcs with G[u] > 0, and 2^31-1 for the source.
   dist[n] [device, output]: d(v), 2^31-1 for unreachable v.
   Errors: LLP_E_ARG (n <= 0, source out of range, null CSR), LLP_E_INPUT
   (LLP_VALIDATE: id out of range, negative weight, bad row offsets),
   LLP_E_OVERFLOW (a reachable vertex has d(v) >= 2^31-1),
   LLP_E_NOT_CONVERGED, LLP_E_ABORTED, LLP_E_HIP. */
int llp_solve_sssp(const llp_graph* g, int32_t source, int32_t* dist, const llp_opts* opts);

/* Breadth-first levels (paper Section 5.3): SSSP with every weight 1
   (in_w / out_w ignored).  level[n] [device, output], 2^31-1 = unreachable. */
int llp_solve_bfs(const llp_graph* g, int32_t source, int32_t* level, const llp_opts* opts);

/* Man-optimal stable matching (paper Section 5.4).  G[m] = man m's proposal
   index (0 = first choice); m is forbidden iff the woman he targets is also
   targeted by a man she ranks better; alpha = G[m] + 1, bound n - 1.
   men_pref [device] int16[n*n]: men_pref[m*n + i] = i-th woman on m's list.
   women_rank [device] int16[n*n]: women_rank[w*n + m] = rank of m for w (0 = best).
   wife [device, output] int32[n]; proposal_idx [device, output, nullable] int32[n].
   n <= 32767.  Errors: LLP_E_ARG, LLP_E_INPUT (LLP_VALIDATE: ids out of
   range), LLP_E_INFEASIBLE (a man exhausts his list: malformed lists).
   With the default schedule, no warm start and no chunk, n <= 12288 runs in
   one workgroup with the matching state in LDS, from a per-solve table of
   (woman, her rank of the man) for the first 64 positions of every list
   (later positions read both arrays); the workspace then holds 64 n int32
   for it (llp_workspace_bytes(LLP_KIND_SM, n, 0, opts)). */
int llp_solve_sm(int32_t n, const int16_t* men_pref, const int16_t* women_rank, int32_t* wife,
                 int32_t* proposal_idx, const llp_opts* opts);

/* Earliest start times of a job DAG (paper Section 5.5).  S[j] = max over
   predecessors p of S[p] + dur[p] (0 without predecessors); the paper's
   completion time is S[j] + dur[j].  pred_ptr[n+1], pred_idx[E] [device]:
   predecessor lists; succ_ptr[n+1], succ_idx[E] [device]: the same arcs
   grouped by predecessor.  dur[n] [device] >= 0.  start[n] [device, output].
   Default schedule: the paper's readiness counters (each job fixed once),
   one launch per wide level; consecutive levels of at most 1024 arcs
   (opts->chunk) run in one launch, by one workgroup with the level lists in
   LDS, up to 64 levels per launch.  LLP_JOBS_PULL: pull rounds over
   predecessors with successor worklists.
   Errors: LLP_E_ARG, LLP_E_INPUT, LLP_E_CYCLE (the arcs contain a cycle),
   LLP_E_OVERFLOW (a completion time exceeds 2^31-1). */
int llp_solve_jobs(int32_t n, const int32_t* pred_ptr, const int32_t* pred_idx, const int32_t* dur,
                   const int32_t* succ_ptr, const int32_t* succ_idx, int32_t* start,
                   const llp_opts* opts);

/* 0-1 knapsack (paper Section 5.8): DP cells G[k][c], k = 0..items,
   c = 0..W, advanced to max(G[k-1][c], v_k + G[k-1][c - w_k]).  One
   workgroup sweeps the table a row at a time (every cell of row k is
   forbidden once row k-1 is final), rows resident in LDS.  wt, val [device]
   int32[items] >= 0; best [device, output] int32[1] = G[items][W];
   last_row [device, output, nullable] int32[W+1] = G[items][.].
   Limits: items >= 0, 0 <= W <= 16383.  Errors: LLP_E_ARG, LLP_E_INPUT
   (negative weight or value), LLP_E_OVERFLOW (a value beyond int32). */
int llp_solve_knapsack(int32_t items, int32_t W, const int32_t* wt, const int32_t* val,
                       int32_t* best, int32_t* last_row, const llp_opts* opts);

/* Transitive closure (paper Section 5.7): boolean G[u][v], bottom all false;
   (u, v) is forbidden iff false and either an arc or G[u][w] and G[w][v] for
   some w.  Input: arcs as in-order out-CSR out_ptr[n+1], out_dst[m] [device].
   bits [device, output] uint32[n * ceil(n/32)]: row u, bit (v & 31) of word
   v >> 5.  Limits: n <= 65536. */
int llp_solve_tc(int32_t n, int64_t m, const int32_t* out_ptr, const int32_t* out_dst,
                 uint32_t* bits, const llp_opts* opts);

/* Parallel reduction (paper Section 5.6): a tree of tiles whose node is
   forbidden once its children have published; the root is the sum of x[n]
   [device] modulo 2^64.  result [device, output] uint64[1]. */
int llp_solve_reduce(int64_t n, const uint64_t* x, uint64_t* result, const llp_opts* opts);

/* For callers that cannot allocate device memory (code under hipGraph
   capture, tight serving loops, harnesses that forbid allocation): the same
   reduction as llp_solve_reduce with the same arguments and result, calling
   no allocator.  Its scratch (a counter and one partial per tile, at most
   2048 tiles: 16,640 bytes) is a static array that each GPU holds until the
   process ends; opts->workspace is ignored.  Every call on a GPU uses that
   GPU's one array, so calls that overlap on one GPU (other streams, other
   threads) race and must be serialised by the caller.  LLP_E_ARG when the
   launch would need more tiles than the array holds (only on a device of
   more than 256 compute units) or with LLP_TIMING. */
int llp_solve_reduce_noalloc(int64_t n, const uint64_t* x, uint64_t* result, const llp_opts* opts);

/* Batched persistent solve: count independent instances in one launch of a
   persistent kernel; each workgroup takes `chunk` instances at a time from a
   device queue and solves each one on its own (workgroup-local sweep, state in
   LDS).  desc [device] llp_instance[count]; pool [device] int32[pool_words]
   input words; out_pool [device] int32[out_words] output words.
   LLP_KIND_KNAPSACK instance: n = items, cap_or_source = W (0 <= W <= 16383),
     pool[in_off ..] = wt[n], val[n]; out_pool[out_off] = best.
   LLP_KIND_SSSP instance: n vertices (1 <= n <= 8192), m arcs,
     cap_or_source = source, pool[in_off ..] = out_ptr[n+1], out_dst[m],
     out_w[m] (arcs grouped by tail, weights >= 0); out_pool[out_off ..] =
     dist[n] (2^31-1 = unreachable).
   Per-instance status words go to out_status [device, nullable]
   int32[count]; an instance whose ranges fall outside pool / out_pool, or
   whose arrays are malformed, gets LLP_E_INPUT without being read further.
   The return value is the first nonzero instance status.
   A first call measures the largest W and n in desc (one small readback) to
   size the LDS; opts->block / opts->chunk = 0 take the autotuned values (or
   512 threads, 1 instance). */
typedef struct {
    int32_t kind;
    int32_t n;
    int32_t cap_or_source;
    int32_t pad;
    int64_t m;
    int64_t in_off;
    int64_t out_off;
} llp_instance;

int llp_solve_batch(int32_t count, const llp_instance* desc, const int32_t* pool, int64_t pool_words,
                    int32_t* out_pool, int64_t out_words, int32_t* out_status, const llp_opts* opts);

/* Batched solve replayed from an instantiated hipGraph cached by the library,
   keyed by (desc, pool, out_pool, out_status, workspace, count, pool and out
   sizes, stream, block, chunk); the first call measures, captures and
   instantiates, later calls only launch the graph.  Every replay measures
   the instance limits and rebuilds the claim order inside the graph, so the
   workspace may be used by other solves between replays and the table at
   desc may change: when it then holds a larger knapsack W or SSSP n than
   the captured launch was sized for, a synchronous call drops the graph,
   captures a new one and solves again (with LLP_ASYNC those instances get
   LLP_E_INPUT instead).  With LLP_ASYNC a replay returns once enqueued and
   the batch status goes to opts->status_dev.  Same arguments and results as
   llp_solve_batch.  Released by llp_shutdown(). */
int llp_solve_batch_graph(int32_t count, const llp_instance* desc, const int32_t* pool, int64_t pool_words,
                          int32_t* out_pool, int64_t out_words, int32_t* out_status, const llp_opts* opts);

/* ---------------------------------------------------------------- autotuner
   Times each candidate (threads per workgroup in {256, 512, 1024} x
   instances per queue claim in {1, 2, 4, 8}) of the batch kernel on the given
   batch (median of 3 timed launches after one warm-up) and records the
   fastest for the current device and the batch's size class (see below);
   llp_solve_batch uses it when opts->block and opts->chunk are 0.  Writes one "block chunk ms" line per
   candidate to report (nullable, host) as text, up to report_bytes.
   Outputs of the batch are left as computed by the last candidate. */
int llp_autotune_batch(int32_t count, const llp_instance* desc, const int32_t* pool, int64_t pool_words,
                       int32_t* out_pool, int64_t out_words, char* report, size_t report_bytes,
                       const llp_opts* opts);
/* Times the graph sweep at 1, 2, 3 and 4 workgroups per CU (opts->chunk) on
   this graph for kind LLP_KIND_SSSP or LLP_KIND_BFS from source, with the
   schedule and flags of opts (median of 3 timed solves after one warm-up)
   and records the fastest for the kind and the size class of g->m; solves
   with opts->chunk = 0 use it.  out [device, n] receives the fixpoint, which
   the shape does not change.  One "chunk ms" line per candidate goes to report
   (nullable, host).  A caller-provided workspace must hold
   llp_workspace_bytes(kind, n, m, opts with chunk 0). */
int llp_autotune_graph(const llp_graph* g, int32_t source, int32_t kind, int32_t* out, char* report,
                       size_t report_bytes, const llp_opts* opts);
/* The most recently recorded choice for kind (LLP_KIND_BATCH: block and
   chunk; LLP_KIND_SSSP / LLP_KIND_BFS: block 0 and the workgroups per CU) on
   the current device; LLP_E_ARG if none has been recorded. */
int llp_autotune_get(int kind, int32_t* block, int32_t* chunk);
/* Records are kept per (GPU architecture, CU count, kind, size class), the
   size class being floor(log2(size)) with size the instance count of a batch
   or the arc count m of a graph.  A solve that leaves its shape to the
   library takes the record of its class on the current device, else that of
   the nearest class of the same kind (the larger on a tie), else the default.
   llp_autotune_lookup returns that choice for a size (LLP_E_ARG if none).
   llp_autotune_save writes every record, of every architecture, to a JSON
   file (host path; written to path.tmp, then renamed); llp_autotune_load adds
   the records of such a file (LLP_E_INPUT if it is malformed or out of range,
   in which case none is taken) and stores their number in *loaded (nullable).
   Neither needs a GPU.  llp_shutdown forgets every record. */
int llp_autotune_lookup(int32_t kind, int64_t size, int32_t* block, int32_t* chunk);
int llp_autotune_save(const char* path);
int llp_autotune_load(const char* path, int32_t* loaded);

/* ---------------------------------------------------------------- learned scheduler
   Network: 12 round features -> 64 -> 64 -> 5 outputs (ReLU hidden layers),
   BF16 weights and activations, FP32 accumulation.  Parameter block layout
   (LLP_MLP_PARAMS floats, row-major): W1[64][12], b1[64], W2[64][64], b2[64],
   W3[5][64], b3[5].  Outputs: [push logit, dense logit, delta logits x3]. */
#define LLP_MLP_IN 12
#define LLP_MLP_HID 64
#define LLP_MLP_OUT 5
#define LLP_MLP_PARAMS (64 * 12 + 64 + 64 * 64 + 64 + 5 * 64 + 5)

/* Load FP32 master weights (host array of LLP_MLP_PARAMS floats); the library
   keeps a BF16 copy on the current device for LLP_SCHED_LEARNED. */
int llp_sched_set_weights(const float* params);

/* Training kernels over a batch of B rows, all buffers [device]:
   forward: x[B][12] fp32 -> logits[B][5] fp32 (activations saved in act,
     act[B][2*64] bf16 hidden activations);
   backward: given dlogits[B][5] fp32, accumulate grad[LLP_MLP_PARAMS] fp32;
   loss: BCE on outputs 0-1 against label bits, softmax cross-entropy on 2..4
     against the delta class; writes dlogits and loss[1];
   step: Adam on fp32 master params (and refreshes their bf16 copy).
   Forward products run on the matrix cores in BF16 with FP32 accumulation
   (the network's own arithmetic); backward products in FP32, since the
   straight-through gradients stay unrounded.  Results agree with a
   sequential FP32 evaluation up to the order of the FP32 sums. */
int llp_mlp_forward(int32_t B, const float* params, const float* x, float* logits, uint16_t* act,
                    void* stream);
int llp_mlp_loss(int32_t B, const float* logits, const int32_t* labels, float* dlogits, float* loss,
                 void* stream);
int llp_mlp_backward(int32_t B, const float* params, const float* x, const uint16_t* act,
                     const float* dlogits, float* grad, void* stream);
int llp_mlp_adam(const float* grad, float* params, float* m1, float* m2, int32_t step, float lr,
                 void* stream);

/* Per-round feature vector the sweep feeds the network (for trace-driven
   training): 12 fp32 values per llp_trace_rec of a solve of the given kind
   (LLP_KIND_SSSP, LLP_KIND_BFS or LLP_KIND_JOBS, with push rounds
   available) on n indices and m arcs.  Features: frontier size and arcs
   (log and linear, relative to n and m), the frontier's mean degree
   relative to the graph's, the frontier-width hybrid's code for the round
   (0 push, 0.5 push with wide buckets, 0.25 pull, 1 dense), log2(1 + m/n)/8,
   the change of the frontier size, the previous round's mode, r/(r + 16),
   and the changed indices so far over n; each rounded to bf16. */
int llp_trace_features(int64_t rounds, const llp_trace_rec* trace, int32_t n, int64_t m, int32_t kind,
                       float* features /* [device, output] [rounds][12] */, void* stream);

const char* llp_last_error(void);
const char* llp_version(void);
void llp_shutdown(void);

#ifdef __cplusplus
}
#endif

#endif /* LLP_H */
