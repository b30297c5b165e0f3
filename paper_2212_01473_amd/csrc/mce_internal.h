// Internal declarations shared by the library's own sources (never by the
// CPU oracle).  All device code targets gfx950: wave64, 160 KB LDS per CU.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>

#include "../../include/mce.h"

namespace mce {

constexpr int kWave = 64;
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ULL;

// Error plumbing ---------------------------------------------------------------
void set_error(const std::string& msg);
const char* get_error();

struct Status {
    mce_status code = MCE_OK;
    bool ok() const { return code == MCE_OK; }
};

#define MCE_HIP_TRY(expr)                                                         \
    do {                                                                          \
        hipError_t _e = (expr);                                                   \
        if (_e != hipSuccess) {                                                   \
            ::mce::set_error(std::string(#expr) + ": " + hipGetErrorString(_e));  \
            return _e == hipErrorOutOfMemory ? MCE_ERR_OUT_OF_MEMORY : MCE_ERR_DEVICE; \
        }                                                                         \
    } while (0)

// Device buffer owned by the library ------------------------------------------
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    mce_status alloc(size_t b) {
        if (b <= bytes && p) return MCE_OK;
        release();
        if (b == 0) b = 8;
        hipError_t e = hipMalloc(&p, b);
        if (e != hipSuccess) {
            p = nullptr;
            set_error(std::string("hipMalloc(") + std::to_string(b) + "): " + hipGetErrorString(e));
            return e == hipErrorOutOfMemory ? MCE_ERR_OUT_OF_MEMORY : MCE_ERR_DEVICE;
        }
        bytes = b;
        return MCE_OK;
    }
    template <class T> T* as() const { return reinterpret_cast<T*>(p); }
};

// Primitives (prim.hip) ------------------------------------------------------------
// Exclusive prefix sum of n uint32 values into out (out may alias in); the total
// is written to *total_dev (device) when non-null.  tmp must hold
// scan_tmp_words(n) uint64 words.
size_t scan_tmp_words(size_t n);
mce_status exclusive_scan_u32(const uint32_t* in, uint32_t* out, size_t n, uint32_t* total_dev,
                              uint64_t* tmp, hipStream_t s);
mce_status exclusive_scan_u64(const uint64_t* in, uint64_t* out, size_t n, uint64_t* total_dev,
                              uint64_t* tmp, hipStream_t s);
void fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s);
void fill_u64(uint64_t* p, uint64_t v, size_t n, hipStream_t s);
void iota_u32(uint32_t* p, size_t n, hipStream_t s);

// Stable sort of (key, value) pairs by the low `key_bits` bits of key (LSD radix,
// 8-bit digits).  keys/vals are permuted in place using the alt buffers.
struct RadixTmp {
    DevBuf keys_alt, vals_alt, hist, scan_tmp;
};
mce_status stable_sort_pairs_u32(uint32_t* keys, uint32_t* vals, size_t n, int key_bits,
                                 RadixTmp& tmp, hipStream_t s);

// Preprocessing (preprocess.hip) ---------------------------------------------------
struct GraphMeta {
    uint32_t n = 0;
    uint64_t nnz = 0;
    uint32_t max_degree = 0, degeneracy = 0, max_out = 0, max_in = 0;
    uint64_t n_isolated = 0;
    uint32_t voff = 0;  // first union vertex of this graph
};

struct Oriented {
    uint32_t ngraphs = 1;             // > 1: a batch enumerated as one disjoint union
    std::vector<GraphMeta> meta;      // per graph (batch) or one entry
    DevBuf gid;                       // graph of each rank (batch only)
    uint32_t n = 0;
    uint64_t nnz = 0;
    uint32_t max_degree = 0, degeneracy = 0, rounds = 0;
    uint32_t max_out = 0, max_in = 0;
    uint64_t n_isolated = 0;
    bool peel_steps = false;  // in: run the peel as step kernels replayed from a graph
    uint32_t peel_mode = 0;   // out: 1 = one cooperative launch, 2 = step kernels, 3 = per member
    // rank space
    DevBuf op, oc;    // out CSR: later neighbours, sorted ascending by rank
    DevBuf ip, ic;    // in CSR: earlier neighbours (unsorted)
    DevBuf perm;      // input id of each rank
    DevBuf vkey;      // key(input id) of each rank
    DevBuf core_r;    // core number of each rank
    DevBuf rank;      // rank of each input id
    // input space
    DevBuf core, round; // by input id
};

// rp/ci are device pointers (input space).  validate: run the graph-rule checks.
// gid_in / voff (device, optional): graph of each input vertex and first vertex
// of each graph, for a batch loaded as one disjoint union (keys then use the
// vertex id local to its graph).  max_member_n: the largest member's vertex
// count (a batch whose members are all small peels each member on its own).
mce_status preprocess_graph(const uint32_t* rp, const uint32_t* ci, uint32_t n, uint64_t nnz,
                            bool validate, hipStream_t s, Oriented& g, const uint32_t* gid_in = nullptr,
                            const uint32_t* voff = nullptr, uint32_t ngraphs = 1, uint32_t max_member_n = 0);

// Build the union CSR of a batch on the device (host inputs) and preprocess it.
mce_status preprocess_batch(const uint32_t* rp_cat, const uint32_t* ci_cat, const uint64_t* row_off,
                            const uint64_t* col_off, uint32_t ng, bool validate, bool on_dev, hipStream_t s,
                            Oriented& g);

// Enumeration (enumerate.hip) ----------------------------------------------------------
// Default knobs (measured on gfx950; see the options in mce.h)
constexpr uint32_t kDefaultDonateMinP = 24;
constexpr uint32_t kDefaultBitmapMaxP = 128;

struct EnumConfig {
    uint32_t flags = MCE_F_WORKER_LIST;
    uint32_t max_root_core = 0xFFFFFFFFu;
    uint32_t wg_per_cu = 0;
    uint32_t bitmap_max_p = 0;
    uint32_t donate_min_p = kDefaultDonateMinP;
    uint32_t donate_max_depth = 0;
    uint32_t donate_every = 1;
    uint32_t task_log_min_us = 0;
    uint64_t* task_log = nullptr;
    uint64_t task_log_cap = 0;
    uint64_t timeout_ms = 600000;
    const uint32_t* root_order = nullptr;  // device, input ids
    uint64_t* root_count = nullptr;
    uint64_t* root_hash = nullptr;
    uint64_t* root_nodes = nullptr;
    uint32_t* stream_vertices = nullptr;
    uint64_t stream_vcap = 0;
    uint64_t* stream_offsets = nullptr;
    uint64_t stream_ocap = 0;
    uint64_t xrow_budget_words = 1ull << 18;  // X rows per workgroup (words)
    uint32_t xrow_ratio = 32;                // X rows when |X| <= ratio * max(|U|, 64)
    uint32_t xrow_min_u = 16;                // ... and |U| >= xrow_min_u
    const void* model = nullptr;             // MLP weights (device) for MCE_F_LEARNED_ORDER
    uint32_t split_top = 0;
    // explicit work queue (learned order / split); otherwise built from the window
};

struct EnumOutput {
    struct PerGraph {
        uint64_t count = 0, hash = 0;
        std::vector<uint64_t> hist;
        uint32_t max_size = 0;
    };
    std::vector<PerGraph> graphs;
    uint64_t xrow_tasks = 0, build_ns = 0;
    uint64_t count = 0, hash = 0;
    std::vector<uint64_t> hist;  // index = size
    uint32_t max_size = 0;
    uint64_t stats[24] = {0};
    uint64_t stream_v = 0, stream_c = 0;
    bool stream_truncated = false;
    bool timed_out = false;
};

// Work queue built from the learned model.
struct LearnedQueue {
    DevBuf feat, score, keys, sorted, roots, score_sorted, groups, pos, gpos, scan_tmp, total, sroots, ssplits, psum;
    DevBuf flag, heavy, light, phist;
    const uint32_t* qroots = nullptr;
    const uint32_t* qsplits = nullptr;
    uint32_t n = 0, len = 0, scored = 0, min_p = 0;
};

// One graph's enumeration state kept across calls (scratch sized to the graph).
struct EnumState {
    LearnedQueue lq;
    DevBuf roots, ctrl, acc, gacc, hist, scratch, idle, flags, small;
    DevBuf l2v, l2e;  // second-level tasks: root rank and edge index in the later-neighbour CSR
    DevBuf tmp_a, tmp_b, tmp_c, scan_tmp;
    size_t scratch_stride = 0;
    uint32_t grid = 0;
    uint32_t lds_cap = 0;
};

// raw tick counter slot of the build time
constexpr int MCE_STAT_BUILD_TICKS = MCE_STAT_BUILD_NS;

mce_status build_root_queue(const Oriented& g, const EnumConfig& cfg, EnumState& st, hipStream_t s,
                            uint32_t* nroots_out);
mce_status enumerate_graph(const Oriented& g, const EnumConfig& cfg, EnumState& st, hipStream_t s,
                           EnumOutput& out);

// Learned part (learned.hip) ------------------------------------------------------------
mce_status root_features(const Oriented& g, const uint32_t* roots_rank, uint32_t nr, float* feat, hipStream_t s);
mce_status ids_to_ranks(const Oriented& g, const uint32_t* ids, uint32_t n, uint32_t* out, hipStream_t s);
mce_status model_predict(const float* model, const float* feat, uint32_t n, float* out, hipStream_t s);
mce_status model_loss_grad(const float* model, const float* feat, const float* target, uint32_t n, float* grad,
                           float* loss, hipStream_t s);
mce_status model_loss_grad_noalloc(const float* model, const float* feat, const float* target, uint32_t n,
                                   float* grad, float* loss, hipStream_t s);
mce_status model_fit_norm(float* model, const float* feat, uint32_t n, hipStream_t s);
mce_status model_train(float* model, const float* feat, const float* target, uint32_t n, uint32_t epochs, float lr,
                       float b1, float b2, float eps, bool fit_norm, float* loss_hist, hipStream_t s);
// The learned queue in st.lq.  built_n: the plain queue's length when
// build_root_queue has already filled st.roots (degeneracy order, no custom or
// reverse order), else kQueueNotBuilt.
constexpr uint32_t kQueueNotBuilt = 0xFFFFFFFFu;
mce_status learned_queue(const Oriented& g, const EnumConfig& cfg, EnumState& st, hipStream_t s, uint32_t grid,
                         LearnedQueue& q, uint32_t built_n = kQueueNotBuilt);

}  // namespace mce
