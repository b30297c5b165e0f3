/*
 * mce.h -- exact maximal clique enumeration on one AMD Instinct MI355X (gfx950).
 *
 * The operation (paper: "Parallelizing Maximal Clique Enumeration on GPUs",
 * Section II-A): for a simple undirected graph G, enumerate every maximal
 * clique -- a vertex set that is pairwise adjacent and is contained in no
 * larger such set -- exactly, with no approximation.  The library returns the
 * number of maximal cliques, their histogram by size, an order-independent
 * 64-bit hash of the set of cliques, and optionally the cliques themselves.
 *
 * The method (Sections II-B..II-D and III): Bron-Kerbosch with Tomita
 * pivoting (Algorithm 2) over independent first-level subtrees (Algorithm 3)
 * in a degeneracy order; each subtree is explored depth-first by one
 * wavefront over a partial induced subgraph (Section III-D) held as bitmaps,
 * with the compact excluded-set representation of Section III-E and the
 * worker list of Section III-C for load balancing.
 *
 * Clique hash (a fixed definition, not from the paper): fmix is the
 * SplitMix64 output finaliser (Steele, Lea and Flood, OOPSLA 2014),
 * gamma = 0x9E3779B97F4A7C15, key(v) = fmix((v + 1) * gamma) for input vertex
 * id v, h(C) = fmix(sum_{v in C} key(v) + |C| * gamma), and the reported hash
 * is the sum of h(C) over all reported cliques, modulo 2^64.
 *
 * Core window: with max_root_core = c the library reports exactly the maximal
 * cliques whose smallest core number is <= c (all of them when c >= the
 * degeneracy).  Isolated vertices are maximal cliques of size 1.
 *
 * Conventions for every entry point:
 *   - every function returns mce_status; nothing throws or aborts across the ABI;
 *   - on error a thread-local message is available from mce_last_error();
 *   - pointers documented as "device" must be device (HBM) memory of the
 *     current HIP device; "host" pointers are ordinary host memory;
 *   - the library never takes ownership of caller memory.
 */
#ifndef MCE_H
#define MCE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MCE_OK = 0,
    MCE_WARN_STREAM_TRUNCATED = 1,   /* clique stream buffer full; totals still exact */
    MCE_ERR_INVALID_ARG = -1,        /* NULL pointer, bad struct_size, bad option */
    MCE_ERR_INVALID_GRAPH = -2,      /* CSR violates the graph rules below */
    MCE_ERR_OUT_OF_MEMORY = -3,      /* device allocation failed */
    MCE_ERR_DEVICE = -4,             /* HIP runtime error or no usable device */
    MCE_ERR_BUFFER_TOO_SMALL = -5,   /* hist shorter than max_clique_size + 1 */
    MCE_ERR_TIMEOUT = -6,            /* enumeration exceeded timeout_ms; results invalid */
    MCE_ERR_UNSUPPORTED = -7         /* graph exceeds a built-in limit (see mce_graph_info) */
} mce_status;

/* Opaque graph handle: library-owned device state (oriented CSR in degeneracy
 * order, core numbers, per-vertex keys, enumeration scratch). */
typedef struct mce_graph mce_graph;

typedef struct {
    uint32_t n;              /* vertices */
    uint64_t nnz;            /* stored arcs (2 x edges) */
    uint32_t max_degree;     /* Delta */
    uint32_t degeneracy;     /* d = largest core number */
    uint64_t n_isolated;     /* vertices of degree 0 */
    uint32_t peel_rounds;    /* rounds of the synchronous peel */
    uint32_t max_out_degree; /* largest |P| of a first-level subtree (<= d) */
    uint32_t max_in_degree;  /* largest |X| of a first-level subtree (<= Delta) */
    uint32_t n_graphs;       /* graphs in the handle (1 unless batch-loaded) */
    uint32_t peel_mode;      /* how the peel ran: 1 = one cooperative launch with grid
                                barriers, 2 = step kernels replayed from a captured graph,
                                3 = a batch whose member graphs each peeled on their own
                                (one workgroup per member; members of at most 8192 vertices) */
} mce_graph_info;

/* ---- load flags */
#define MCE_LOAD_DEVICE_PTRS 0x1u  /* row_ptr/col_idx are device pointers */
#define MCE_LOAD_NO_VALIDATE 0x2u  /* skip the graph-rule checks (caller vouches) */
#define MCE_LOAD_PEEL_STEPS 0x4u   /* run the peel as step kernels replayed from a captured
                                      graph instead of one cooperative launch (same result;
                                      the library also falls back to it by itself when the
                                      device cannot run the single launch) */

/*
 * Load an undirected simple graph given as CSR with both arc directions stored
 * (Section III-D: the original graph is kept in CSR form).
 *
 * row_ptr: uint32[n+1]; col_idx: uint32[nnz].  Graph rules: row_ptr[0] = 0,
 * row_ptr non-decreasing, row_ptr[n] = nnz, every col < n, each row strictly
 * increasing (sorted, no duplicates), no self-loops, symmetric.  Any violation
 * gives MCE_ERR_INVALID_GRAPH and mce_last_error() names the first offending
 * row and position.
 *
 * The arrays are only read during the call (copied to the device when they are
 * host pointers; read in place with MCE_LOAD_DEVICE_PTRS) and never retained.
 * Loading computes the synchronous-round peel (core numbers; vertices ordered
 * by (core, round, id)), and orients every row into the later (P) and earlier
 * (X) neighbour lists of Algorithm 3.  stream: hipStream_t or NULL (default
 * stream); the call synchronises before returning.  *out receives a handle to
 * release with mce_free().
 */
mce_status mce_load_csr(const uint32_t* row_ptr, const uint32_t* col_idx, uint32_t n,
                        uint64_t nnz, uint32_t flags, void* stream, mce_graph** out);

/*
 * Load n_graphs independent graphs for batched enumeration.  row_ptr_cat holds
 * each graph's row_ptr (starting at 0, length n_i + 1) end to end; col_idx_cat
 * holds each graph's col_idx end to end.  row_off[i] / col_off[i] (uint64,
 * length n_graphs + 1, host memory) give where graph i starts in each array,
 * so n_i = row_off[i+1] - row_off[i] - 1 and nnz_i = col_off[i+1] - col_off[i].
 * Every graph obeys the rules of mce_load_csr.  Vertex ids in results are
 * per-graph input ids.  Same flags, ownership and stream rules; with
 * MCE_LOAD_DEVICE_PTRS the two concatenated arrays are device pointers (the
 * offsets stay in host memory) and the per-graph end checks run on the device.
 */
mce_status mce_load_csr_batch(const uint32_t* row_ptr_cat, const uint32_t* col_idx_cat,
                              const uint64_t* row_off, const uint64_t* col_off,
                              uint32_t n_graphs, uint32_t flags, void* stream, mce_graph** out);

/* Describe graph graph_idx of the handle (0 for a single graph), or with
 * graph_idx = MCE_GRAPH_WHOLE the whole handle: for a batch, the disjoint union
 * of its graphs (n and nnz summed, degrees and degeneracy the largest of any
 * member), e.g. to size one histogram length that serves every member. */
#define MCE_GRAPH_WHOLE 0xFFFFFFFFu
mce_status mce_graph_get_info(const mce_graph* g, uint32_t graph_idx, mce_graph_info* out);

/*
 * Copy the degeneracy data of graph graph_idx to caller-owned host arrays of
 * n entries each (any may be NULL): core[v] = core number of input vertex v,
 * peel_round[v] = round of the synchronous peel that removed v (Section II-D;
 * round r removes every remaining vertex whose remaining degree is at most the
 * current level k, and the level rises to the minimum remaining degree when
 * no vertex qualifies), order[i] = input id of the i-th vertex of the
 * degeneracy order (sorted by round, then id).
 */
mce_status mce_graph_copy_order(const mce_graph* g, uint32_t graph_idx, uint32_t* core, uint32_t* peel_round,
                                uint32_t* order);

/* ---- enumeration flags */
#define MCE_F_WORKER_LIST   0x01u  /* donate branches to idle wavefronts (Section III-C) */
#define MCE_F_LEARNED_ORDER 0x02u  /* order the roots with the most later neighbours (at least 16;
                                      about 8 per workgroup at most) by descending cost predicted
                                      by opt->model, then the rest in degeneracy order */
#define MCE_F_SPLIT         0x04u  /* with LEARNED_ORDER: split the costliest roots into groups of
                                      level-1 branches (group c of C takes branches t, t % C == c) */
#define MCE_F_STATS         0x08u  /* fill mce_result.stats */
#define MCE_F_STREAM        0x10u  /* write cliques to the stream buffers */
#define MCE_F_ROOT_STATS    0x20u  /* per-root counters into opt->root_* (device arrays) */
#define MCE_F_REVERSE_ORDER 0x40u  /* process roots in reverse degeneracy order */
#define MCE_F_CUSTOM_ORDER  0x80u  /* process roots in the order given by opt->root_order */
#define MCE_F_TASK_LOG      0x100u /* record tasks slower than opt->task_log_min_us in opt->task_log */
#define MCE_F_L2_ROOTS      0x200u /* independent second-level subtrees (Algorithm 4): one task per edge
                                      {v, w} with v a root of the window and w a later neighbour of v;
                                      R = {v, w}, P = common neighbours after w, X = common neighbours
                                      before w.  Same results; excludes MCE_F_LEARNED_ORDER */

#define MCE_OPTIONS_VERSION 1u

typedef struct {
    uint32_t struct_size;       /* sizeof(mce_options) */
    uint32_t flags;             /* MCE_F_* */
    uint32_t max_root_core;     /* core window c; UINT32_MAX = full enumeration */
    uint32_t wg_per_cu;         /* persistent workgroups per compute unit; 0 = occupancy limit */
    uint32_t bitmap_max_p;      /* largest subtree universe whose bitmap rows live in LDS;
                                   larger ones use HBM rows; 0 = the largest up to 128 whose
                                   LDS still lets the register-limited number of workgroups
                                   per compute unit be resident */
    uint32_t donate_min_p;      /* donate a branch only if its |P| >= this; 0 = 24 (Section III-C
                                   uses 10; a donated branch here is rebuilt from the CSR by
                                   its receiver, so smaller ones cost more than they save) */
    uint32_t donate_max_depth;  /* donate only at depth <= this; 0 = unlimited */
    uint32_t split_top;         /* MCE_F_SPLIT: a root predicted above 1/workgroups of the total
                                   predicted cost is split in proportion (at most 64 groups);
                                   besides, the split_top costliest roots by predicted rank are
                                   split into 64 groups if predicted at least 4x the mean cost
                                   (0 = none) */
    const void* model;          /* MCE_F_LEARNED_ORDER: device pointer to mce_model weights */
    void* stream;               /* hipStream_t or NULL */
    uint64_t timeout_ms;        /* watchdog; 0 = 600000 */
    const uint32_t* root_order; /* MCE_F_CUSTOM_ORDER: device uint32[n], a permutation of input ids */
    uint64_t* root_count;       /* MCE_F_ROOT_STATS: device uint64[n] by input id, accumulated into */
    uint64_t* root_hash;        /* MCE_F_ROOT_STATS: device uint64[n] */
    uint64_t* root_nodes;       /* MCE_F_ROOT_STATS: device uint64[n] (search-tree nodes) */
    uint32_t xrow_ratio;        /* build X bitmap rows for a task when |X| <= ratio * max(|P u X_P|, 64);
                                   0 = default 32; larger X uses lookups in the original graph */
    uint32_t xrow_min_u;        /* ... and only when |P u X_P| >= xrow_min_u; 0 = default 16 */
    uint64_t xrow_budget_words; /* X bitmap rows per workgroup, 64-bit words; 0 = default 2^18 */
    uint32_t donate_every;      /* offer every k-th eligible branch to the worker list; 0 = 1 */
    uint32_t task_log_min_us;   /* MCE_F_TASK_LOG: record tasks that ran at least this long */
    uint64_t* task_log;         /* MCE_F_TASK_LOG: device uint64[task_log_cap * 8], one record of 8
                                   words per task, in completion order:
                                   [0] root input id, [1] |R| << 32 | universe |P u X_P|,
                                   [2] split group c << 48 | C << 32 | initial |X_X|,
                                   [3] search-tree nodes, [4] task time (ns), [5] bitmap build
                                   time (ns), [6] branches donated by the task,
                                   [7] workgroup << 48 | start time (ns, device clock) */
    uint64_t task_log_cap;      /* records that fit; MCE_STAT_TASK_LOG counts all qualifying tasks */
} mce_options;

/* indices into mce_result.stats */
enum {
    MCE_STAT_NODES = 0,        /* search-tree nodes expanded */
    MCE_STAT_DONATIONS = 1,    /* branches handed to idle workgroups */
    MCE_STAT_TASKS = 2,        /* tasks run (roots + donated + split) */
    MCE_STAT_ROOTS = 3,        /* first-level subtrees in the window with |P| > 0 */
    MCE_STAT_WORKGROUPS = 4,   /* persistent workgroups launched */
    MCE_STAT_KERNEL_NS = 5,    /* enumeration kernel time (ns) */
    MCE_STAT_SETUP_NS = 6,     /* root-queue setup time (ns) */
    MCE_STAT_XTESTS = 7,       /* X_X adjacency tests */
    MCE_STAT_BUILD_EDGES = 8,  /* adjacency entries scanned to build bitmaps */
    MCE_STAT_HBM_ROWS = 9,     /* tasks whose bitmap rows lived in HBM */
    MCE_STAT_IDLE_NS = 10,     /* summed workgroup idle time in the worker list (ns) */
    MCE_STAT_LDS_BYTES = 11,   /* LDS bytes per workgroup */
    MCE_STAT_PROBES = 12,      /* adjacency-list entries read by X_X binary searches */
    MCE_STAT_ROOT_WORDS = 13,  /* P and X ids staged from the oriented CSR for roots */
    MCE_STAT_BUSY_NS = 14,     /* summed task time over workgroups (ns) */
    MCE_STAT_MAX_TASK_NS = 15, /* longest single task (ns) */
    MCE_STAT_XROW_TASKS = 16,  /* tasks that built X bitmap rows */
    MCE_STAT_BUILD_NS = 17,    /* summed bitmap-construction time over workgroups (ns) */
    MCE_STAT_TASK_LOG = 18,    /* tasks that qualified for the task log (may exceed its capacity) */
    MCE_STAT_DONATE_NS = 19,   /* summed time spent offering branches to the worker list (ns) */
    MCE_STAT_POP_FAILS = 20,   /* offers that found no idle workgroup */
    MCE_STAT_XCOL_WORDS = 21,  /* X-column words read for bitmap X_X children */
    MCE_STAT_FOLD_DONATIONS = 22 /* donations sent as register frames (no rebuild by the receiver) */
};

typedef struct {
    uint64_t count;                   /* out: number of maximal cliques */
    uint64_t hash;                    /* out: sum of h(C) mod 2^64 */
    uint32_t max_clique_size;         /* out: largest clique size (0 if none) */
    uint32_t hist_len;                /* in: length of hist */
    uint64_t* hist;                   /* in/out, host, caller-owned: hist[k] = #cliques of size k */
    uint32_t* stream_vertices;        /* MCE_F_STREAM: device uint32[stream_vcap] */
    uint64_t stream_vcap;
    uint64_t* stream_offsets;         /* MCE_F_STREAM: device uint64[stream_ocap]; entry i is
                                         (start << 16) | size of clique i in stream_vertices, or
                                         UINT64_MAX if its vertices did not fit */
    uint64_t stream_ocap;
    uint64_t stream_vertices_written; /* out */
    uint64_t stream_cliques_written;  /* out */
    uint64_t stats[24];               /* out (MCE_F_STATS): see MCE_STAT_* */
} mce_result;

/*
 * Enumerate the maximal cliques of a single-graph handle (Algorithms 2 and 3).
 * opt may be NULL (defaults: worker list on, full enumeration).  res must not
 * be NULL; res->hist may be NULL (hist_len 0) only if the histogram is not
 * wanted -- otherwise a hist shorter than max_clique_size + 1 gives
 * MCE_ERR_BUFFER_TOO_SMALL with count, hash and max_clique_size still valid
 * (degeneracy + 2 always suffices).  Stream: cliques in unspecified order,
 * vertex ids are input ids; when a buffer fills, writing stops and the call
 * returns MCE_WARN_STREAM_TRUNCATED with totals still exact.  One call per
 * handle at a time; the call synchronises its stream before returning.
 */
mce_status mce_enumerate(mce_graph* g, const mce_options* opt, mce_result* res);

/*
 * Enumerate every graph of a batch-loaded handle in one persistent launch.
 * The batch is held as one disjoint union (its maximal cliques are exactly
 * those of the member graphs), peeled and oriented once; the work queue holds
 * (root) entries of all graphs and every result is attributed to the graph of
 * its root.  res is an array of n_res >= n_graphs results (res[i] for graph i,
 * same field rules as mce_enumerate).  Streams, per-root statistics and custom
 * orders are single-graph only.  For a batch handle, peel_round and order of
 * mce_graph_copy_order refer to the union's peel restricted to the graph.
 */
mce_status mce_enumerate_batch(mce_graph* g, const mce_options* opt, mce_result* res,
                               uint32_t n_res);

/* ---- learned root ordering (all arrays are device memory) */

/* Floats in a cost model: W1[64][4], b1[64], W2[64][64], b2[64], W3[64][64],
 * b3[64], W4[64], b4, then the per-feature mean[4] and std[4] used to
 * normalise inputs.  Hidden layers use ReLU; the output predicts
 * log(1 + search-tree nodes) of a first-level subtree. */
#define MCE_MODEL_FLOATS 8713

/*
 * Cheap features of first-level subtrees, 4 floats per root: log(1+degree),
 * log(1+core number), log(1+2-hop count) (sum of neighbour degrees), and the
 * edge density of the root's later-neighbour set P.  root_ids: device
 * uint32[n_roots] input vertex ids of a single-graph handle; feat: device
 * float[n_roots * 4].
 */
mce_status mce_root_features(const mce_graph* g, const uint32_t* root_ids, uint32_t n_roots, float* feat,
                             void* stream);

/* BF16 inference (weights and activations rounded to bfloat16, FP32 sums):
 * out[i] = predicted log(1 + nodes) for feat[i*4 .. i*4+3]. */
mce_status mce_model_predict(const float* model, const float* feat, uint32_t n, float* out, void* stream);

typedef struct {
    uint32_t struct_size;  /* sizeof(mce_train_options) */
    uint32_t epochs;       /* full-batch Adam steps */
    float lr, beta1, beta2, eps;
    uint32_t fit_norm;     /* 1: set mean/std of the model from feat before training */
    uint32_t reserved;
} mce_train_options;

/* Train a model in place with FP32 forward/backward kernels and Adam
 * (Kingma and Ba, 2015) on mean squared error; model holds the initial
 * weights.  loss_history: host float[epochs] or NULL. */
mce_status mce_model_train(float* model, const float* feat, const float* target, uint32_t n,
                           const mce_train_options* opt, float* loss_history, void* stream);

/* One FP32 forward and backward pass: grad (device float[MCE_MODEL_FLOATS],
 * zero for mean/std) of the mean squared error, and the loss (host). */
mce_status mce_model_loss_grad(const float* model, const float* feat, const float* target, uint32_t n,
                               float* grad, float* loss, void* stream);

/*
 * mce_model_loss_grad for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same results, with the activations
 * and partial sums in a fixed device array of the library (about 24.5 MiB,
 * held on every device the library runs on until the process ends) instead
 * of per-call buffers.  Allocates nothing, device or host.
 *
 * n: 1 .. MCE_NOALLOC_MAX_SAMPLES, else MCE_ERR_INVALID_ARG (larger sets go
 * through mce_model_loss_grad).  model, feat (float[n*4]), target (float[n])
 * and grad (float[MCE_MODEL_FLOATS]) are device pointers as there; loss: host
 * float or NULL.  stream: hipStream_t of the current device, or NULL.  Calls
 * on one device share the array: calls that overlap on one device (other host
 * threads, other streams) race and must be serialised by the caller.
 */
#define MCE_NOALLOC_MAX_SAMPLES 16384u
mce_status mce_model_loss_grad_noalloc(const float* model, const float* feat, const float* target, uint32_t n,
                                       float* grad, float* loss, void* stream);

/*
 * Autotuner for the performance knobs (none of them changes the result):
 * coordinate descent over donate_min_p, bitmap_max_p, wg_per_cu,
 * donate_max_depth and xrow_ratio, timing setup + kernel with device events on
 * this handle (single graph or batch).  base: the options to start from
 * (MCE_F_STREAM, MCE_F_ROOT_STATS and MCE_F_TASK_LOG are rejected); tuned:
 * receives base with the best knob values.  Every trial must reproduce the
 * base run's count, hash and histogram for every graph, else MCE_ERR_DEVICE.
 * report may be NULL; its struct_size must be set when given.
 */
typedef struct {
    uint32_t struct_size; /* sizeof(mce_tune_report) */
    uint32_t passes;      /* in: coordinate-descent passes; 0 = 1 */
    uint32_t repeats;     /* in: timed runs per setting (the minimum counts); 0 = 1 */
    uint32_t trials;      /* out: enumerations run */
    double base_ms;       /* out: time with the base options */
    double best_ms;       /* out: time with the tuned options */
} mce_tune_report;

mce_status mce_autotune(mce_graph* g, const mce_options* base, mce_options* tuned, mce_tune_report* report);

/* Release a handle (NULL is a no-op). */
void mce_free(mce_graph* g);

/* Static description of a status code. */
const char* mce_status_string(mce_status s);

/* Detail of the last error on the calling thread ("" if none). */
const char* mce_last_error(void);

/* Library version string. */
const char* mce_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MCE_H */
