// C ABI of the library (declared in include/mce.h).  Argument checking, device
// memory for host-supplied graphs, and orchestration of preprocessing and
// enumeration; every step of the computation runs in this library's kernels.
#include "mce_internal.h"

#include <algorithm>
#include <memory>
#include <string>
#include <vector>

namespace mce {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }
const char* get_error() { return g_last_error.c_str(); }

}  // namespace mce

struct mce_graph {
    std::vector<std::unique_ptr<mce::Oriented>> graphs;
    mce::EnumState state;
    bool batch = false;
};

using namespace mce;

namespace {

mce_status fail(mce_status code, const std::string& msg)
{
    set_error(msg);
    return code;
}

mce_status load_one(const uint32_t* row_ptr, const uint32_t* col_idx, uint32_t n, uint64_t nnz, uint32_t flags,
                    hipStream_t s, Oriented& og)
{
    const bool on_dev = (flags & MCE_LOAD_DEVICE_PTRS) != 0;
    const bool validate = (flags & MCE_LOAD_NO_VALIDATE) == 0;
    DevBuf drp, dci;
    const uint32_t* rp = row_ptr;
    const uint32_t* ci = col_idx;
    if (!on_dev) {
        if (validate) {
            // cheap host checks that guard the device copies
            if (row_ptr[0] != 0) return fail(MCE_ERR_INVALID_GRAPH, "invalid graph: row_ptr[0] != 0 at row 0");
            if ((uint64_t)row_ptr[n] != nnz)
                return fail(MCE_ERR_INVALID_GRAPH, "invalid graph: row_ptr[n] != nnz at row " + std::to_string(n));
        }
        mce_status st;
        if ((st = drp.alloc(((size_t)n + 1) * 4)) != MCE_OK) return st;
        if ((st = dci.alloc((size_t)(nnz ? nnz : 1) * 4)) != MCE_OK) return st;
        MCE_HIP_TRY(hipMemcpyAsync(drp.p, row_ptr, ((size_t)n + 1) * 4, hipMemcpyHostToDevice, s));
        if (nnz) MCE_HIP_TRY(hipMemcpyAsync(dci.p, col_idx, (size_t)nnz * 4, hipMemcpyHostToDevice, s));
        rp = drp.as<uint32_t>();
        ci = dci.as<uint32_t>();
    }
    og.peel_steps = (flags & MCE_LOAD_PEEL_STEPS) != 0;
    return preprocess_graph(rp, ci, n, nnz, validate, s, og);
}

void fill_info(const Oriented& o, uint32_t idx, mce_graph_info* out)
{
    const GraphMeta& m = o.meta[idx];
    out->n = m.n;
    out->nnz = m.nnz;
    out->max_degree = m.max_degree;
    out->degeneracy = m.degeneracy;
    out->n_isolated = m.n_isolated;
    out->peel_rounds = o.rounds;
    out->max_out_degree = m.max_out;
    out->max_in_degree = m.max_in;
    out->n_graphs = o.ngraphs;
    out->peel_mode = o.peel_mode;
}

mce_status config_from(const mce_options* opt, EnumConfig& cfg)
{
    if (!opt) return MCE_OK;
    if (opt->struct_size != sizeof(mce_options))
        return fail(MCE_ERR_INVALID_ARG, "mce_options.struct_size must be sizeof(mce_options)");
    if (opt->xrow_ratio) cfg.xrow_ratio = opt->xrow_ratio;
    if (opt->xrow_budget_words) cfg.xrow_budget_words = opt->xrow_budget_words;
    if (opt->xrow_min_u) cfg.xrow_min_u = opt->xrow_min_u;
    if (opt->donate_every) cfg.donate_every = opt->donate_every;
    if (opt->flags & MCE_F_TASK_LOG) {
        if (!opt->task_log && opt->task_log_cap)
            return fail(MCE_ERR_INVALID_ARG, "MCE_F_TASK_LOG with task_log_cap > 0 needs task_log");
        cfg.task_log = opt->task_log;
        cfg.task_log_cap = opt->task_log ? opt->task_log_cap : 0;
        cfg.task_log_min_us = opt->task_log_min_us;
    }
    cfg.flags = opt->flags;
    cfg.max_root_core = opt->max_root_core;
    cfg.wg_per_cu = opt->wg_per_cu;
    cfg.bitmap_max_p = opt->bitmap_max_p;
    cfg.donate_min_p = opt->donate_min_p ? opt->donate_min_p : kDefaultDonateMinP;
    cfg.donate_max_depth = opt->donate_max_depth;
    cfg.timeout_ms = opt->timeout_ms ? opt->timeout_ms : 600000ull;
    cfg.root_order = opt->root_order;
    cfg.root_count = opt->root_count;
    cfg.root_hash = opt->root_hash;
    cfg.root_nodes = opt->root_nodes;
    cfg.model = opt->model;
    cfg.split_top = opt->split_top;
    if ((cfg.flags & MCE_F_SPLIT) && !(cfg.flags & MCE_F_LEARNED_ORDER))
        return fail(MCE_ERR_INVALID_ARG, "MCE_F_SPLIT needs MCE_F_LEARNED_ORDER");
    if ((cfg.flags & MCE_F_LEARNED_ORDER) && (cfg.flags & (MCE_F_CUSTOM_ORDER | MCE_F_REVERSE_ORDER)))
        return fail(MCE_ERR_INVALID_ARG, "learned order excludes custom and reverse orders");
    if ((cfg.flags & MCE_F_L2_ROOTS) && (cfg.flags & MCE_F_LEARNED_ORDER))
        return fail(MCE_ERR_INVALID_ARG, "MCE_F_L2_ROOTS excludes the learned order");
    if (cfg.bitmap_max_p > 4096) return fail(MCE_ERR_INVALID_ARG, "bitmap_max_p must be <= 4096");
    return MCE_OK;
}

mce_status finish_result(const EnumOutput& eo, size_t gi, mce_result* res, mce_status st)
{
    const EnumOutput::PerGraph& pg = eo.graphs[gi];
    res->count = pg.count;
    res->hash = pg.hash;
    res->max_clique_size = pg.max_size;
    for (int i = 0; i < 24; ++i) res->stats[i] = eo.stats[i];
    res->stream_cliques_written = eo.stream_c < res->stream_ocap ? eo.stream_c : res->stream_ocap;
    res->stream_vertices_written = eo.stream_v < res->stream_vcap ? eo.stream_v : res->stream_vcap;
    if (st != MCE_OK) return st;
    if (res->hist && res->hist_len) {
        for (uint32_t k = 0; k < res->hist_len; ++k) res->hist[k] = k < pg.hist.size() ? pg.hist[k] : 0;
        if (res->hist_len < pg.max_size + 1)
            return fail(MCE_ERR_BUFFER_TOO_SMALL,
                        "hist_len " + std::to_string(res->hist_len) + " < max_clique_size + 1 = " +
                            std::to_string(pg.max_size + 1));
    }
    if (eo.stream_truncated) return MCE_WARN_STREAM_TRUNCATED;
    return MCE_OK;
}

}  // namespace

extern "C" {

mce_status mce_load_csr(const uint32_t* row_ptr, const uint32_t* col_idx, uint32_t n, uint64_t nnz, uint32_t flags,
                        void* stream, mce_graph** out)
{
    set_error("");
    if (!out) return fail(MCE_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!row_ptr) return fail(MCE_ERR_INVALID_ARG, "row_ptr is NULL");
    if (!col_idx && nnz) return fail(MCE_ERR_INVALID_ARG, "col_idx is NULL");
    if (n == 0xFFFFFFFFu) return fail(MCE_ERR_INVALID_ARG, "n too large");
    if (flags & ~(MCE_LOAD_DEVICE_PTRS | MCE_LOAD_NO_VALIDATE | MCE_LOAD_PEEL_STEPS))
        return fail(MCE_ERR_INVALID_ARG, "unknown load flags");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    auto g = std::make_unique<mce_graph>();
    g->graphs.emplace_back(new Oriented());
    uint32_t dummy = 0;
    mce_status st = load_one(row_ptr, nnz ? col_idx : &dummy, n, nnz, flags, s, *g->graphs[0]);
    if (st != MCE_OK) return st;
    *out = g.release();
    return MCE_OK;
}

mce_status mce_load_csr_batch(const uint32_t* row_ptr_cat, const uint32_t* col_idx_cat, const uint64_t* row_off,
                              const uint64_t* col_off, uint32_t n_graphs, uint32_t flags, void* stream,
                              mce_graph** out)
{
    set_error("");
    if (!out) return fail(MCE_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!row_ptr_cat || !row_off || !col_off) return fail(MCE_ERR_INVALID_ARG, "NULL batch array");
    if (n_graphs == 0) return fail(MCE_ERR_INVALID_ARG, "n_graphs is 0");
    if (flags & ~(MCE_LOAD_DEVICE_PTRS | MCE_LOAD_NO_VALIDATE | MCE_LOAD_PEEL_STEPS))
        return fail(MCE_ERR_INVALID_ARG, "unknown load flags");
    for (uint32_t i = 0; i < n_graphs; ++i) {
        if (row_off[i + 1] <= row_off[i] || col_off[i + 1] < col_off[i])
            return fail(MCE_ERR_INVALID_ARG, "batch offsets not increasing at graph " + std::to_string(i));
    }
    if (col_off[n_graphs] > col_off[0] && !col_idx_cat) return fail(MCE_ERR_INVALID_ARG, "col_idx_cat is NULL");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    auto g = std::make_unique<mce_graph>();
    g->batch = true;
    g->graphs.emplace_back(new Oriented());
    g->graphs[0]->peel_steps = (flags & MCE_LOAD_PEEL_STEPS) != 0;
    mce_status st = preprocess_batch(row_ptr_cat, col_idx_cat, row_off, col_off, n_graphs,
                                     (flags & MCE_LOAD_NO_VALIDATE) == 0, (flags & MCE_LOAD_DEVICE_PTRS) != 0, s,
                                     *g->graphs[0]);
    if (st != MCE_OK) return st;
    *out = g.release();
    return MCE_OK;
}

mce_status mce_graph_get_info(const mce_graph* g, uint32_t graph_idx, mce_graph_info* out)
{
    if (!g || !out) return fail(MCE_ERR_INVALID_ARG, "NULL argument");
    const Oriented& o = *g->graphs[0];
    if (graph_idx == MCE_GRAPH_WHOLE) {
        // the whole handle: for a batch, its disjoint union
        out->n = o.n;
        out->nnz = o.nnz;
        out->max_degree = o.max_degree;
        out->degeneracy = o.degeneracy;
        out->n_isolated = o.n_isolated;
        out->peel_rounds = o.rounds;
        out->max_out_degree = o.max_out;
        out->max_in_degree = o.max_in;
        out->n_graphs = o.ngraphs;
        out->peel_mode = o.peel_mode;
        return MCE_OK;
    }
    if (graph_idx >= o.meta.size()) return fail(MCE_ERR_INVALID_ARG, "graph_idx out of range");
    fill_info(o, graph_idx, out);
    return MCE_OK;
}

mce_status mce_graph_copy_order(const mce_graph* g, uint32_t graph_idx, uint32_t* core, uint32_t* peel_round,
                                uint32_t* order)
{
    if (!g) return fail(MCE_ERR_INVALID_ARG, "NULL graph");
    const Oriented& o = *g->graphs[0];
    if (graph_idx >= o.meta.size()) return fail(MCE_ERR_INVALID_ARG, "graph_idx out of range");
    const GraphMeta& m = o.meta[graph_idx];
    size_t bytes = (size_t)m.n * 4;
    if (bytes == 0) return MCE_OK;
    if (core) MCE_HIP_TRY(hipMemcpy(core, o.core.as<uint32_t>() + m.voff, bytes, hipMemcpyDeviceToHost));
    if (peel_round) MCE_HIP_TRY(hipMemcpy(peel_round, o.round.as<uint32_t>() + m.voff, bytes, hipMemcpyDeviceToHost));
    if (order) {
        if (o.ngraphs == 1) {
            MCE_HIP_TRY(hipMemcpy(order, o.perm.p, bytes, hipMemcpyDeviceToHost));
        } else {
            std::vector<uint32_t> perm(o.n), gid(o.n);
            MCE_HIP_TRY(hipMemcpy(perm.data(), o.perm.p, (size_t)o.n * 4, hipMemcpyDeviceToHost));
            MCE_HIP_TRY(hipMemcpy(gid.data(), o.gid.p, (size_t)o.n * 4, hipMemcpyDeviceToHost));
            size_t k = 0;
            for (uint32_t r = 0; r < o.n; ++r)
                if (gid[r] == graph_idx) order[k++] = perm[r] - m.voff;
        }
    }
    return MCE_OK;
}

mce_status mce_enumerate(mce_graph* g, const mce_options* opt, mce_result* res)
{
    set_error("");
    if (!g || !res) return fail(MCE_ERR_INVALID_ARG, "NULL argument");
    if (g->batch) return fail(MCE_ERR_INVALID_ARG, "batch handle: use mce_enumerate_batch");
    EnumConfig cfg;
    mce_status st = config_from(opt, cfg);
    if (st != MCE_OK) return st;
    if (res->hist_len && !res->hist) return fail(MCE_ERR_INVALID_ARG, "hist is NULL with hist_len > 0");
    if (cfg.flags & MCE_F_STREAM) {
        cfg.stream_vertices = res->stream_vertices;
        cfg.stream_vcap = res->stream_vcap;
        cfg.stream_offsets = res->stream_offsets;
        cfg.stream_ocap = res->stream_ocap;
    }
    hipStream_t s = opt ? reinterpret_cast<hipStream_t>(opt->stream) : nullptr;
    EnumOutput eo;
    st = enumerate_graph(*g->graphs[0], cfg, g->state, s, eo);
    if (st != MCE_OK && st != MCE_ERR_TIMEOUT) return st;
    return finish_result(eo, 0, res, st);
}

mce_status mce_enumerate_batch(mce_graph* g, const mce_options* opt, mce_result* res, uint32_t n_res)
{
    set_error("");
    if (!g || !res) return fail(MCE_ERR_INVALID_ARG, "NULL argument");
    const Oriented& o = *g->graphs[0];
    if (n_res < o.ngraphs) return fail(MCE_ERR_INVALID_ARG, "n_res smaller than the number of graphs");
    EnumConfig cfg;
    mce_status st = config_from(opt, cfg);
    if (st != MCE_OK) return st;
    if (cfg.flags & (MCE_F_STREAM | MCE_F_ROOT_STATS | MCE_F_CUSTOM_ORDER))
        return fail(MCE_ERR_INVALID_ARG, "stream, per-root statistics and custom order are single-graph only");
    for (uint32_t i = 0; i < o.ngraphs; ++i)
        if (res[i].hist_len && !res[i].hist) return fail(MCE_ERR_INVALID_ARG, "hist is NULL with hist_len > 0");
    hipStream_t s = opt ? reinterpret_cast<hipStream_t>(opt->stream) : nullptr;
    EnumOutput eo;
    st = enumerate_graph(o, cfg, g->state, s, eo);
    if (st != MCE_OK && st != MCE_ERR_TIMEOUT) return st;
    mce_status worst = MCE_OK;
    for (uint32_t i = 0; i < o.ngraphs; ++i) {
        mce_status si = finish_result(eo, i, &res[i], st);
        if (si < 0 && worst >= 0) worst = si;
        else if (si > 0 && worst == MCE_OK) worst = si;
    }
    return worst;
}

mce_status mce_root_features(const mce_graph* g, const uint32_t* root_ids, uint32_t n_roots, float* feat,
                             void* stream)
{
    set_error("");
    if (!g || (!root_ids && n_roots) || (!feat && n_roots)) return fail(MCE_ERR_INVALID_ARG, "NULL argument");
    if (g->batch) return fail(MCE_ERR_INVALID_ARG, "features are for single-graph handles");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const Oriented& o = *g->graphs[0];
    DevBuf ranks;
    mce_status st;
    if ((st = ranks.alloc((size_t)(n_roots ? n_roots : 1) * 4)) != MCE_OK) return st;
    if ((st = ids_to_ranks(o, root_ids, n_roots, ranks.as<uint32_t>(), s)) != MCE_OK) return st;
    if ((st = root_features(o, ranks.as<uint32_t>(), n_roots, feat, s)) != MCE_OK) return st;
    MCE_HIP_TRY(hipStreamSynchronize(s));
    return MCE_OK;
}

mce_status mce_model_predict(const float* model, const float* feat, uint32_t n, float* out, void* stream)
{
    set_error("");
    if (!model || (n && (!feat || !out))) return fail(MCE_ERR_INVALID_ARG, "NULL argument");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    mce_status st = model_predict(model, feat, n, out, s);
    if (st != MCE_OK) return st;
    MCE_HIP_TRY(hipStreamSynchronize(s));
    return MCE_OK;
}

mce_status mce_model_train(float* model, const float* feat, const float* target, uint32_t n,
                           const mce_train_options* opt, float* loss_history, void* stream)
{
    set_error("");
    if (!model || !feat || !target || !opt) return fail(MCE_ERR_INVALID_ARG, "NULL argument");
    if (opt->struct_size != sizeof(mce_train_options))
        return fail(MCE_ERR_INVALID_ARG, "mce_train_options.struct_size must be sizeof(mce_train_options)");
    if (n == 0 || opt->epochs == 0) return fail(MCE_ERR_INVALID_ARG, "no samples or no epochs");
    return model_train(model, feat, target, n, opt->epochs, opt->lr, opt->beta1, opt->beta2, opt->eps,
                       opt->fit_norm != 0, loss_history, reinterpret_cast<hipStream_t>(stream));
}

mce_status mce_model_loss_grad(const float* model, const float* feat, const float* target, uint32_t n,
                               float* grad, float* loss, void* stream)
{
    set_error("");
    if (!model || !feat || !target || !grad) return fail(MCE_ERR_INVALID_ARG, "NULL argument");
    return model_loss_grad(model, feat, target, n, grad, loss, reinterpret_cast<hipStream_t>(stream));
}

mce_status mce_model_loss_grad_noalloc(const float* model, const float* feat, const float* target, uint32_t n,
                                       float* grad, float* loss, void* stream)
{
    set_error("");
    if (!model || !feat || !target || !grad) return fail(MCE_ERR_INVALID_ARG, "NULL argument");
    return model_loss_grad_noalloc(model, feat, target, n, grad, loss, reinterpret_cast<hipStream_t>(stream));
}

void mce_free(mce_graph* g) { delete g; }

const char* mce_status_string(mce_status s)
{
    switch (s) {
    case MCE_OK: return "ok";
    case MCE_WARN_STREAM_TRUNCATED: return "clique stream truncated (totals exact)";
    case MCE_ERR_INVALID_ARG: return "invalid argument";
    case MCE_ERR_INVALID_GRAPH: return "invalid graph";
    case MCE_ERR_OUT_OF_MEMORY: return "out of device memory";
    case MCE_ERR_DEVICE: return "device error";
    case MCE_ERR_BUFFER_TOO_SMALL: return "histogram buffer too small";
    case MCE_ERR_TIMEOUT: return "timeout";
    case MCE_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char* mce_last_error(void) { return get_error(); }

const char* mce_version(void) { return "mce-mi355x 0.1 (gfx950)"; }

}  // extern "C"

// ---------------------------------------------------------------- autotuner
// Coordinate descent over the performance knobs: each knob in turn takes the
// candidate value with the shortest measured time (setup + kernel, device
// events) while the others stay fixed.  Every trial must reproduce the base
// run's count, hash and histogram; candidates slower than 3x the best time so
// far are cut off by the watchdog.
mce_status mce_autotune(mce_graph* g, const mce_options* base, mce_options* tuned, mce_tune_report* report)
{
    set_error("");
    if (!g || !base || !tuned) return fail(MCE_ERR_INVALID_ARG, "NULL argument");
    if (report && report->struct_size != sizeof(mce_tune_report))
        return fail(MCE_ERR_INVALID_ARG, "mce_tune_report.struct_size must be sizeof(mce_tune_report)");
    if (base->flags & (MCE_F_STREAM | MCE_F_ROOT_STATS | MCE_F_TASK_LOG))
        return fail(MCE_ERR_INVALID_ARG, "autotune: stream, per-root statistics and task log are not tuned");
    const uint32_t passes = report && report->passes ? report->passes : 1u;
    const uint32_t repeats = report && report->repeats ? report->repeats : 1u;
    const Oriented& o = *g->graphs[0];
    hipStream_t s = reinterpret_cast<hipStream_t>(base->stream);

    mce_options cur = *base;
    uint32_t trials = 0;
    EnumOutput ref;
    bool have_ref = false;
    // time of one option set (minimum over repeats); +inf if cut off
    auto measure = [&](const mce_options& opt, double cutoff_ms, double* ms) -> mce_status {
        EnumConfig cfg;
        mce_status st = config_from(&opt, cfg);
        if (st != MCE_OK) return st;
        cfg.flags |= MCE_F_STATS;
        if (cutoff_ms > 0) cfg.timeout_ms = std::max<uint64_t>(1000, (uint64_t)(3.0 * cutoff_ms) + 1);
        double best = 1e300;
        for (uint32_t r = 0; r < repeats; ++r) {
            EnumOutput eo;
            st = enumerate_graph(o, cfg, g->state, s, eo);
            ++trials;
            if (st == MCE_ERR_TIMEOUT) {
                *ms = 1e300;
                return MCE_OK;
            }
            if (st != MCE_OK) return st;
            if (!have_ref) {
                ref = eo;
                have_ref = true;
            } else {
                for (size_t gi = 0; gi < ref.graphs.size(); ++gi) {
                    const auto& a = ref.graphs[gi];
                    const auto& b = eo.graphs[gi];
                    if (a.count != b.count || a.hash != b.hash || a.hist != b.hist)
                        return fail(MCE_ERR_DEVICE, "autotune: a knob setting changed the result of graph " +
                                                        std::to_string(gi));
                }
            }
            best = std::min(best, (eo.stats[MCE_STAT_KERNEL_NS] + eo.stats[MCE_STAT_SETUP_NS]) / 1e6);
        }
        *ms = best;
        return MCE_OK;
    };

    double best_ms = 0;
    mce_status st = measure(cur, 0, &best_ms);
    if (st != MCE_OK) return st;
    const double base_ms = best_ms;

    struct Knob {
        uint32_t mce_options::*field;
        std::vector<uint32_t> values;
    };
    const std::vector<Knob> knobs = {
        {&mce_options::donate_min_p, {16, 20, 24, 32}},
        {&mce_options::bitmap_max_p, {64, 128, 256}},
        {&mce_options::wg_per_cu, {0, 4, 2}},
        {&mce_options::donate_max_depth, {0, 3}},
        {&mce_options::xrow_ratio, {8, 32, 128}},
    };
    for (uint32_t pass = 0; pass < passes; ++pass) {
        for (const Knob& k : knobs) {
            uint32_t keep = cur.*k.field;
            for (uint32_t v : k.values) {
                if (v == keep) continue;
                mce_options cand = cur;
                cand.*k.field = v;
                double ms = 0;
                if ((st = measure(cand, best_ms, &ms)) != MCE_OK) return st;
                if (ms < best_ms) {
                    best_ms = ms;
                    cur.*k.field = v;
                }
            }
        }
    }
    *tuned = cur;
    if (report) {
        report->trials = trials;
        report->base_ms = base_ms;
        report->best_ms = best_ms;
    }
    return MCE_OK;
}
