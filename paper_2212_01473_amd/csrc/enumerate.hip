// Persistent maximal-clique enumeration kernel for gfx950.
//
// One wavefront (64 lanes) owns one task at a time and explores it depth-first
// (Section III-A): Bron-Kerbosch with pivoting (Algorithm 2) below a
// first-level subtree of Algorithm 3.  A task is (R, P, X_P, X_X):
//   * U = P u X_P, the vertices whose adjacency is kept as bitmap rows over U --
//     the partial induced subgraph of Section III-D (edges among P; for a
//     root task U = P = the later neighbours of the root);
//   * X_X, the part of X that came from the root's earlier neighbours, kept as
//     one array shrunk in place across levels with per-level end pointers
//     (Section III-E, Fig. 2); adjacency of an X_X vertex x to a branch vertex
//     b is looked up in the original graph (x precedes b, so b is searched in
//     the sorted later-neighbour list of x);
//   * the pivot maximises |P n N(u)| over u in P u X_P (Section III-E, last
//     paragraph: X_X vertices are not pivot candidates under partial induced
//     subgraphs).
// Work distribution (Section III-C): phase 1 pops roots from a shared counter;
// in phase 2 idle wavefronts enter a worker list (MPMC ring of workgroup ids)
// and busy ones donate branches to them.
//
// Two representations of the bitmap state:
//   * mid mode (|U| > 64): W = ceil(|U|/64) words per set, lane w holds word w
//     of P, X_P and the remaining-branch set B; rows live in LDS when |U| fits
//     the launch's LDS budget, otherwise in per-workgroup HBM scratch; the
//     per-level stack lives in HBM scratch;
//   * small mode (|U'| <= 64, reached by re-indexing P u X_P of a node): lane k
//     holds the 64-bit row of local vertex k in registers and P, X_P, B are
//     single wave-uniform words; the stack is in LDS.
#include "mce_internal.h"

#include <chrono>

namespace mce {

namespace {

constexpr uint32_t kFlagIdle = 0u, kFlagTask = 1u, kFlagTerm = 2u;
constexpr uint32_t kEmptySlot = 0xFFFFFFFFu;
constexpr int kHistLds = 256;
constexpr int kSmallDepth = 66;
constexpr uint32_t kMaxUniverse = 4096;  // W <= 64 words per bitmap row

struct Ctrl {
    unsigned long long packed;     // started << 32 | idle
    unsigned long long ring_head;
    unsigned long long ring_tail;
    unsigned long long stream_v;
    unsigned long long stream_c;
    unsigned int root_cursor;
    unsigned int err;              // 1 = timeout, 2 = internal limit
    unsigned int stream_trunc;
    unsigned int waiting;          // workgroups currently in the worker list
    unsigned int pad[4];
};

struct MboxHdr {
    uint32_t root;     // root rank (per-root statistics)
    uint32_t rsize;    // |R|
    uint64_t keysum;   // sum of keys of R (mod 2^64)
    uint32_t np, nxp, nxx, anc;
};

struct Params {
    const uint32_t* op;
    const uint32_t* oc;
    const uint32_t* ip;
    const uint32_t* ic;
    const uint64_t* vkey;
    const uint32_t* perm;
    const uint32_t* roots;
    uint32_t nroots;
    Ctrl* ctrl;
    unsigned long long* acc;
    unsigned long long* hist;
    uint32_t hist_len;
    uint8_t* scratch;
    uint64_t stride;
    uint64_t off_P, off_XP, off_R, off_xx, off_flag, off_hpos, off_spos, off_rows, off_stack, off_meta;
    uint32_t* ring;
    uint32_t ring_mask;
    uint32_t* wflags;
    uint32_t ucap, lds_cap, wg, xcap, rcap;
    uint32_t flags;
    uint32_t donate_min_p, donate_max_depth;
    uint32_t nwg;
    uint64_t timeout_ticks;
    unsigned long long* root_count;
    unsigned long long* root_hash;
    unsigned long long* root_nodes;
    uint32_t* s_verts;
    uint64_t s_vcap;
    unsigned long long* s_offs;
    uint64_t s_ocap;
};

// ---------------------------------------------------------------- wave helpers
__device__ inline uint32_t lane_id() { return __lane_id(); }

__device__ inline uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline uint64_t uni64(uint64_t v)
{
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}
__device__ inline uint64_t rl64(uint64_t v, uint32_t l)
{
    uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, l);
    uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}
__device__ inline uint32_t rl32(uint32_t v, uint32_t l) { return __builtin_amdgcn_readlane(v, l); }
__device__ inline uint64_t shfl64(uint64_t v, uint32_t src)
{
    uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, (int)src, 64);
    uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), (int)src, 64);
    return ((uint64_t)hi << 32) | lo;
}
__device__ inline uint32_t prefix_popc(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
// Row rotation through DPP (row_ror:N, N = 1..15, rows of 16 lanes).
template <int N>
__device__ inline uint32_t row_ror(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x120 + N, 0xF, 0xF, false);
}
// Wave-wide sum / max: reduce each 16-lane row with DPP rotations, then
// combine the four rows through readlane (no LDS round trips).
__device__ inline uint32_t wave_sum(uint32_t v)
{
    v += row_ror<1>(v);
    v += row_ror<2>(v);
    v += row_ror<4>(v);
    v += row_ror<8>(v);
    return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) +
           __builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48);
}
__device__ inline uint32_t wave_max(uint32_t v)
{
    v = max(v, row_ror<1>(v));
    v = max(v, row_ror<2>(v));
    v = max(v, row_ror<4>(v));
    v = max(v, row_ror<8>(v));
    return max(max(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
               max(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}
__device__ inline uint32_t wave_excl_scan(uint32_t v)
{
    uint32_t x = v;
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = (uint32_t)__shfl_up((int)x, off, 64);
        if (lane_id() >= (uint32_t)off) x += y;
    }
    return x - v;
}
// Cross-lane visibility of global/LDS stores within the (single-wave) workgroup.
__device__ inline void wave_mem_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_s_barrier();
}
__device__ inline uint64_t now_ticks() { return __builtin_amdgcn_s_memrealtime(); }

__device__ inline uint64_t fmix64(uint64_t z)
{
    // SplitMix64 output finaliser (Steele, Lea and Flood, OOPSLA 2014).
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// ---------------------------------------------------------------- per-workgroup context
struct Wg {
    // global scratch
    MboxHdr* mbox;
    uint32_t* mP;
    uint32_t* mXP;
    uint32_t* R;
    uint32_t* xx;
    uint64_t* xflag;
    uint32_t* hpos;
    uint32_t* spos;
    uint64_t* grows;
    uint64_t* gstack;
    uint64_t* gmeta;
    // LDS
    uint32_t* hist;   // kHistLds
    uint32_t* sidx;   // 64
    uint64_t* pw;     // 64
    uint64_t* xw;     // 64
    uint64_t* sP;     // kSmallDepth
    uint64_t* sXP;
    uint64_t* sB;
    uint64_t* sK;
    uint32_t* sL;
    uint32_t* sA;
    uint32_t* uarr;   // ucap
    uint64_t* ukey;   // ucap: key of each universe vertex
    uint64_t* lrows;  // lds_cap * ws_lds
    // accumulators (wave-uniform)
    uint64_t count, hash, nodes, donations, tasks, xtests, edges, hbm_tasks, idle_ticks, root_list_words;
    uint64_t busy_ticks, max_task_ticks, task_t0;
    uint32_t probes;  // per lane
    uint32_t hmax;
    uint32_t wl_tick;
    uint32_t wl_seen;
    uint32_t poll;
    uint64_t deadline;
    uint32_t me;
    bool abort;
};

// Is b among the later neighbours of x?  (x precedes b in the order.)
// probes counts the list entries read.
__device__ inline bool has_later(const Params& p, uint32_t x, uint32_t b, uint32_t& probes)
{
    uint32_t lo = p.op[x], hi = p.op[x + 1];
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        uint32_t w = p.oc[mid];
        ++probes;
        if (w == b) return true;
        if (w < b) lo = mid + 1;
        else hi = mid;
    }
    return false;
}

// Any X_X vertex in xx[0, L) adjacent to b?
__device__ bool xx_any(const Params& p, Wg& w, uint32_t L, uint32_t b)
{
    const uint32_t lane = lane_id();
    for (uint32_t base = 0; base < L; base += 64) {
        uint32_t i = base + lane;
        bool hit = i < L && has_later(p, w.xx[i], b, w.probes);
        w.xtests += min(64u, L - base);
        if (__ballot(hit)) return true;
    }
    return false;
}

// Partition xx[0, L): vertices adjacent to b move to [0, K), the rest to
// [K, L) (Section III-E: the array keeps every level's X_X as a prefix).
// Returns K.  Only the misplaced elements move (holes in [0,K) are swapped
// with kept elements in [K,L)).
__device__ uint32_t xx_partition(const Params& p, Wg& w, uint32_t L, uint32_t b)
{
    const uint32_t lane = lane_id();
    uint32_t K = 0;
    for (uint32_t base = 0; base < L; base += 64) {
        uint32_t i = base + lane;
        bool keep = i < L && has_later(p, w.xx[i], b, w.probes);
        uint64_t m = __ballot(keep);
        if (lane == 0) w.xflag[base >> 6] = m;
        K += (uint32_t)__popcll(m);
    }
    w.xtests += L;
    if (K == 0 || K == L) return K;
    wave_mem_sync();
    uint32_t nh = 0;
    for (uint32_t base = 0; base < K; base += 64) {
        uint64_t m = w.xflag[base >> 6];
        uint32_t i = base + lane;
        bool hole = i < K && !((m >> lane) & 1ull);
        uint64_t hm = __ballot(hole);
        if (hole) w.hpos[nh + prefix_popc(hm)] = i;
        nh += (uint32_t)__popcll(hm);
    }
    uint32_t ns = 0;
    for (uint32_t base = K & ~63u; base < L; base += 64) {
        uint64_t m = w.xflag[base >> 6];
        uint32_t i = base + lane;
        bool stray = i >= K && i < L && ((m >> lane) & 1ull);
        uint64_t sm = __ballot(stray);
        if (stray) w.spos[ns + prefix_popc(sm)] = i;
        ns += (uint32_t)__popcll(sm);
    }
    wave_mem_sync();
    for (uint32_t k = lane; k < nh; k += 64) {
        uint32_t a = w.hpos[k], s = w.spos[k];
        uint32_t va = w.xx[a], vs = w.xx[s];
        w.xx[a] = vs;
        w.xx[s] = va;
    }
    wave_mem_sync();
    return K;
}

__device__ void report(const Params& p, Wg& w, uint32_t rsize, uint64_t ks)
{
    w.count += 1;
    w.hash += fmix64(ks + (uint64_t)rsize * kGamma);
    w.hmax = max(w.hmax, rsize);
    const uint32_t lane = lane_id();
    if (lane == 0) {
        if (rsize < (uint32_t)kHistLds) w.hist[rsize] += 1;
        else atomicAdd(&p.hist[rsize < p.hist_len ? rsize : p.hist_len - 1], 1ull);
    }
    if (p.flags & MCE_F_STREAM) {
        unsigned long long c = 0, v = 0;
        if (lane == 0) {
            c = atomicAdd(&p.ctrl->stream_c, 1ull);
            v = atomicAdd(&p.ctrl->stream_v, (unsigned long long)rsize);
        }
        c = uni64(c);
        v = uni64(v);
        bool fits = v + rsize <= p.s_vcap;
        if (fits) {
            for (uint32_t j = lane; j < rsize; j += 64) p.s_verts[v + j] = p.perm[w.R[j]];
        }
        if (lane == 0) {
            if (c < p.s_ocap) p.s_offs[c] = fits ? ((v << 16) | rsize) : ~0ull;
            if (!fits || c >= p.s_ocap) p.ctrl->stream_trunc = 1;
        }
    }
}

__device__ inline void flush_hist(const Params& p, Wg& w)
{
    uint32_t top = min(w.hmax + 1, (uint32_t)kHistLds);
    __syncthreads();
    for (uint32_t k = lane_id(); k < top; k += 64) {
        uint32_t c = w.hist[k];
        if (c) {
            atomicAdd(&p.hist[k], (unsigned long long)c);
            w.hist[k] = 0;
        }
    }
    __syncthreads();
    w.hmax = 0;
}

__device__ inline bool check_deadline(const Params& p, Wg& w)
{
    if (w.abort) return true;
    if (now_ticks() > w.deadline) {
        if (lane_id() == 0) atomicOr(&p.ctrl->err, 1u);
        w.abort = true;
    }
    return w.abort;
}

// ---------------------------------------------------------------- worker list
// Pop an idle workgroup id (or kEmptySlot).  Lane 0 acts; result broadcast.
__device__ uint32_t wl_try_pop(const Params& p, Wg& w)
{
    uint32_t r = kEmptySlot;
    if (lane_id() == 0) {
        // The ring carries only workgroup ids, so every access here is relaxed;
        // the task itself is published with release/acquire on the receiver's flag.
        unsigned long long h = __hip_atomic_load(&p.ctrl->ring_head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned long long t = __hip_atomic_load(&p.ctrl->ring_tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (h < t) {
            if (__hip_atomic_compare_exchange_strong(&p.ctrl->ring_head, &h, h + 1, __ATOMIC_RELAXED,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                uint32_t* slot = &p.ring[h & p.ring_mask];
                uint32_t v;
                // the pusher has claimed this slot and stores its id imminently
                while ((v = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == kEmptySlot) {
                    if (now_ticks() > w.deadline) break;
                    __builtin_amdgcn_s_sleep(1);
                }
                if (v != kEmptySlot) {
                    __hip_atomic_store(slot, kEmptySlot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_fetch_add(&p.ctrl->waiting, ~0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                r = v;
            }
        }
    }
    return uni(r);
}

// Number of waiting workgroups as read at the previous check: the load issued
// now is consumed at the next check, so its latency overlaps the search.
__device__ inline bool wl_has_waiting(const Params& p, Wg& w)
{
    uint32_t prev = w.wl_seen;
    w.wl_seen = __hip_atomic_load(&p.ctrl->waiting, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return uni(prev) != 0;
}

__device__ inline Wg wg_view(const Params& p, uint32_t g)
{
    Wg w;
    uint8_t* base = p.scratch + (uint64_t)g * p.stride;
    w.mbox = reinterpret_cast<MboxHdr*>(base);
    w.mP = reinterpret_cast<uint32_t*>(base + p.off_P);
    w.mXP = reinterpret_cast<uint32_t*>(base + p.off_XP);
    w.R = reinterpret_cast<uint32_t*>(base + p.off_R);
    w.xx = reinterpret_cast<uint32_t*>(base + p.off_xx);
    return w;
}

// Should this branch be handed to an idle workgroup (Section III-C)?
__device__ inline bool donation_wanted(const Params& p, Wg& w, uint32_t np_child, bool more_here, bool anc,
                                       uint32_t depth)
{
    if (!(p.flags & MCE_F_WORKER_LIST)) return false;
    if (np_child < p.donate_min_p || !more_here || !anc) return false;
    if (p.donate_max_depth && depth > p.donate_max_depth) return false;
    if ((++w.wl_tick & 3u) != 0) return false;
    return wl_has_waiting(p, w);
}

// Write a task into receiver r's mailbox.  P / X_P given as (id list writer)
// callbacks are replaced by explicit arrays filled by the caller before.
__device__ void send_task(const Params& p, Wg& w, uint32_t r, uint32_t root, uint32_t rsize, uint64_t ks,
                          uint32_t np, uint32_t nxp, uint32_t nxx, uint32_t vb)
{
    const uint32_t lane = lane_id();
    Wg d = wg_view(p, r);
    // P and X_P ids were staged in this workgroup's own mailbox arrays (free while busy)
    for (uint32_t i = lane; i < np; i += 64) d.mP[i] = w.mP[i];
    for (uint32_t i = lane; i < nxp; i += 64) d.mXP[i] = w.mXP[i];
    for (uint32_t i = lane; i < nxx; i += 64) d.xx[i] = w.xx[i];
    for (uint32_t i = lane; i + 1 < rsize; i += 64) d.R[i] = w.R[i];
    if (lane == 0) {
        d.R[rsize - 1] = vb;
        MboxHdr h;
        h.root = root;
        h.rsize = rsize;
        h.keysum = ks;
        h.np = np;
        h.nxp = nxp;
        h.nxx = nxx;
        h.anc = 0;
        *d.mbox = h;
    }
    // publish the mailbox: one release fence, then the flag
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (lane == 0) __hip_atomic_store(&p.wflags[r], kFlagTask, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    w.donations += 1;
}

// Try to donate; returns true when the branch was handed over.  The caller has
// already partitioned X_X for the child (its first nxx entries of xx).
__device__ bool try_donate(const Params& p, Wg& w, uint32_t root, uint32_t rsize, uint64_t ks, uint32_t np,
                           uint32_t nxp, uint32_t nxx, uint32_t vb)
{
    uint32_t r = wl_try_pop(p, w);
    if (r == kEmptySlot) return false;
    // the receiver stops counting as idle before it is handed work
    if (lane_id() == 0) __hip_atomic_fetch_add(&p.ctrl->packed, ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    send_task(p, w, r, root, rsize, ks, np, nxp, nxx, vb);
    return true;
}

// ---------------------------------------------------------------- small mode
// Universe of m <= 64 vertices; lane k holds its rank su and its row.
__device__ void run_small(const Params& p, Wg& w, uint32_t root, uint32_t m, uint32_t su, uint64_t skey,
                          uint64_t row, uint64_t P, uint64_t XP, uint32_t L, uint64_t ks, uint32_t rs, bool anc0)
{
    const uint32_t lane = lane_id();
    const bool valid = lane < m;
    uint32_t depth = 0;
    uint64_t B;
    bool anc = anc0;
    // enter node (P != 0)
enter : {
    w.nodes += 1;
    uint64_t cand = P | XP;
    uint32_t key = 0;
    if (valid && ((cand >> lane) & 1ull)) key = ((uint32_t)__popcll(P & row) << 8) | (255u - lane);
    uint32_t best = wave_max(key);
    uint32_t piv = 255u - (best & 255u);
    B = P & ~rl64(row, piv);
}
    while (true) {
        if (B == 0) {
            if (depth == 0) return;
            --depth;
            P = w.sP[depth];
            XP = w.sXP[depth];
            B = w.sB[depth];
            ks = w.sK[depth];
            L = w.sL[depth];
            anc = w.sA[depth] != 0;
            --rs;
            continue;
        }
        if ((++w.poll & 1023u) == 0 && check_deadline(p, w)) return;
        uint32_t bb = (uint32_t)__builtin_ctzll(B);
        B &= B - 1;
        uint64_t rowb = rl64(row, bb);
        uint64_t Pc = P & rowb;
        uint64_t XPc = XP & rowb;
        P &= ~(1ull << bb);
        XP |= 1ull << bb;
        uint32_t vb = rl32(su, bb);
        uint64_t ksc = ks + rl64(skey, bb);
        if (Pc == 0) {
            w.nodes += 1;
            if (XPc == 0 && !xx_any(p, w, L, vb)) {
                if (p.flags & MCE_F_STREAM) {
                    if (lane == 0) w.R[rs] = vb;
                    wave_mem_sync();
                }
                report(p, w, rs + 1, ksc);
            }
            continue;
        }
        uint32_t Lc = xx_partition(p, w, L, vb);
        uint32_t npc = (uint32_t)__popcll(Pc);
        if (donation_wanted(p, w, npc, B != 0, anc || depth > 0, depth)) {
            // stage ids of P' and X_P' in the own mailbox arrays
            uint32_t nxc = (uint32_t)__popcll(XPc);
            if (valid && ((Pc >> lane) & 1ull)) w.mP[prefix_popc(Pc)] = su;
            if (valid && ((XPc >> lane) & 1ull)) w.mXP[prefix_popc(XPc)] = su;
            wave_mem_sync();
            if (try_donate(p, w, root, rs + 1, ksc, npc, nxc, Lc, vb)) continue;
        }
        // push current level, descend
        if (lane == 0) {
            w.sP[depth] = P;
            w.sXP[depth] = XP;
            w.sB[depth] = B;
            w.sK[depth] = ks;
            w.sL[depth] = L;
            w.sA[depth] = anc ? 1u : 0u;
            w.R[rs] = vb;
        }
        anc = anc || (B != 0);
        ++depth;
        ++rs;
        P = Pc;
        XP = XPc;
        L = Lc;
        ks = ksc;
        goto enter;
    }
}

// ---------------------------------------------------------------- bitmap rows
// Build rows over U[0, nu) (sorted ranks) at row stride ws words: bit j of row i
// is set iff U[i] and U[j] are adjacent.  rows is LDS or HBM.
__device__ void build_rows(const Params& p, Wg& w, const uint32_t* U, uint32_t nu, uint32_t ws, uint64_t* rows)
{
    const uint32_t lane = lane_id();
    for (uint32_t i = lane; i < nu * ws; i += 64) rows[i] = 0;
    wave_mem_sync();
    const uint32_t umax = U[nu - 1];
    for (uint32_t i = 0; i + 1 < nu; ++i) {
        uint32_t u = U[i];
        uint32_t beg = p.op[u], end = p.op[u + 1];
        w.edges += end - beg;
        for (uint32_t e0 = beg; e0 < end; e0 += 64) {
            uint32_t e = e0 + lane;
            uint32_t x = e < end ? p.oc[e] : 0xFFFFFFFFu;
            if (x <= umax) {
                // binary search x in U[i+1, nu)
                uint32_t lo = i + 1, hi = nu;
                while (lo < hi) {
                    uint32_t mid = (lo + hi) >> 1;
                    uint32_t y = U[mid];
                    if (y < x) lo = mid + 1;
                    else hi = mid;
                }
                if (lo < nu && U[lo] == x) {
                    atomicOr((unsigned long long*)&rows[(uint64_t)i * ws + (lo >> 6)], 1ull << (lo & 63));
                    atomicOr((unsigned long long*)&rows[(uint64_t)lo * ws + (i >> 6)], 1ull << (i & 63));
                }
            }
            // rows are sorted: once a chunk ends beyond U's largest rank, stop
            if (p.oc[min(e0 + 63, end - 1)] > umax) break;
        }
    }
    __threadfence();
    wave_mem_sync();
}

// Small-universe rows directly in registers (nu <= 64): lane k gets row k.
__device__ uint64_t build_small_rows(const Params& p, Wg& w, const uint32_t* U, uint32_t nu)
{
    const uint32_t lane = lane_id();
    uint64_t up = 0;
    if (lane < nu) {
        uint32_t u = U[lane];
        uint32_t beg = p.op[u], end = p.op[u + 1];
        uint32_t umax = U[nu - 1];
        uint32_t j = lane + 1;
        // merge N+(u) (sorted) with U[lane+1, nu) (sorted)
        for (uint32_t e = beg; e < end && j < nu; ++e) {
            uint32_t x = p.oc[e];
            if (x > umax) break;
            while (j < nu && U[j] < x) ++j;
            if (j < nu && U[j] == x) up |= 1ull << j;
        }
    }
    w.edges += wave_sum(lane < nu ? (p.op[U[lane] + 1] - p.op[U[lane]]) : 0u);
    uint64_t row = up;
    for (uint32_t j = 0; j < nu; ++j) {
        uint64_t upj = rl64(up, j);
        if ((upj >> lane) & 1ull) row |= 1ull << j;
    }
    return lane < nu ? row : 0ull;
}

// Re-index the node (P u X_P, at most 64 vertices) into small mode and run it.
__device__ void compact_and_run_small(const Params& p, Wg& w, uint32_t root, const uint32_t* U, const uint64_t* rows,
                                      uint32_t ws, uint32_t W, uint64_t Pc, uint64_t XPc, uint32_t L, uint64_t ks,
                                      uint32_t rs, bool anc)
{
    const uint32_t lane = lane_id();
    uint64_t cand = lane < W ? (Pc | XPc) : 0ull;
    uint32_t cnt = (uint32_t)__popcll(cand);
    uint32_t pre = wave_excl_scan(cnt);
    uint32_t m = wave_sum(cnt);
    uint64_t c = cand;
    uint32_t t = pre;
    while (c) {
        uint32_t bit = (uint32_t)__builtin_ctzll(c);
        c &= c - 1;
        w.sidx[t++] = lane * 64 + bit;
    }
    __syncthreads();
    bool valid = lane < m;
    uint32_t o = valid ? w.sidx[lane] : 0u;
    uint32_t su = valid ? U[o] : 0u;
    uint64_t skey = valid ? w.ukey[o] : 0ull;
    uint64_t row = 0;
    for (uint32_t k2 = 0; k2 < m; ++k2) {
        uint32_t o2 = w.sidx[k2];
        if (valid && ((rows[(uint64_t)o * ws + (o2 >> 6)] >> (o2 & 63)) & 1ull)) row |= 1ull << k2;
    }
    uint64_t pword = shfl64(Pc, o >> 6);
    uint64_t xword = shfl64(XPc, o >> 6);
    uint64_t Ps = __ballot(valid && ((pword >> (o & 63)) & 1ull));
    uint64_t XPs = __ballot(valid && ((xword >> (o & 63)) & 1ull));
    __syncthreads();
    run_small(p, w, root, m, su, skey, row, Ps, XPs, L, ks, rs, anc);
}

// ---------------------------------------------------------------- mid mode
__device__ void run_mid(const Params& p, Wg& w, uint32_t root, const uint32_t* U, uint32_t nu, uint64_t* rows,
                        uint32_t ws, uint64_t P, uint64_t XP, uint32_t L, uint64_t ks, uint32_t rs)
{
    const uint32_t lane = lane_id();
    const uint32_t W = (nu + 63) >> 6;
    const uint32_t gws = p.wg;  // stack stride in words
    uint32_t depth = 0;
    uint64_t B = 0;
    bool anc = false;
enter : {
    w.nodes += 1;
    uint32_t best = 0;
    uint64_t cand = P | XP;
    for (uint32_t t = 0; t < W; ++t) {
        uint64_t cw = rl64(cand, t);
        if (cw == 0) continue;
        uint32_t i = t * 64 + lane;
        if ((cw >> lane) & 1ull) {
            uint32_t sc = 0;
            const uint64_t* ri = rows + (uint64_t)i * ws;
            for (uint32_t q = 0; q < W; ++q) sc += (uint32_t)__popcll(rl64(P, q) & ri[q]);
            best = max(best, (sc << 13) | (8191u - i));
        }
    }
    best = wave_max(best);
    uint32_t piv = 8191u - (best & 8191u);
    B = lane < W ? (P & ~rows[(uint64_t)piv * ws + lane]) : 0ull;
}
    while (true) {
        uint64_t bm = __ballot(B != 0);
        if (bm == 0) {
            if (depth == 0) return;
            --depth;
            uint64_t* lvl = w.gstack + (uint64_t)depth * 3 * gws;
            if (lane < W) {
                P = lvl[lane];
                XP = lvl[gws + lane];
                B = lvl[2 * gws + lane];
            }
            uint64_t meta = w.gmeta[2 * depth];
            ks = w.gmeta[2 * depth + 1];
            L = (uint32_t)meta;
            anc = (meta >> 32) != 0;
            --rs;
            continue;
        }
        if ((++w.poll & 1023u) == 0 && check_deadline(p, w)) return;
        uint32_t w0 = (uint32_t)__builtin_ctzll(bm);
        uint64_t word = rl64(B, w0);
        uint32_t bit = (uint32_t)__builtin_ctzll(word);
        uint32_t bb = w0 * 64 + bit;
        uint64_t rowb = lane < W ? rows[(uint64_t)bb * ws + lane] : 0ull;
        uint64_t Pc = P & rowb;
        uint64_t XPc = XP & rowb;
        if (lane == w0) {
            B &= ~(1ull << bit);
            P &= ~(1ull << bit);
            XP |= 1ull << bit;
        }
        uint32_t vb = U[bb];
        uint64_t ksc = ks + w.ukey[bb];
        uint32_t npc = wave_sum((uint32_t)__popcll(Pc));
        uint32_t nxc = wave_sum((uint32_t)__popcll(XPc));
        bool more_here = __ballot(B != 0) != 0;
        if (npc == 0) {
            w.nodes += 1;
            if (nxc == 0 && !xx_any(p, w, L, vb)) {
                if (p.flags & MCE_F_STREAM) {
                    if (lane == 0) w.R[rs] = vb;
                    wave_mem_sync();
                }
                report(p, w, rs + 1, ksc);
            }
            continue;
        }
        uint32_t Lc = xx_partition(p, w, L, vb);
        if (donation_wanted(p, w, npc, more_here, anc || depth > 0, depth)) {
            // stage ids of P' and X_P' (ascending) in the own mailbox arrays
            uint32_t bp = 0, bx = 0;
            for (uint32_t t = 0; t < W; ++t) {
                uint64_t pw_ = rl64(Pc, t), xw_ = rl64(XPc, t);
                uint32_t u = t * 64 + lane;
                if ((pw_ >> lane) & 1ull) w.mP[bp + prefix_popc(pw_)] = U[u];
                if ((xw_ >> lane) & 1ull) w.mXP[bx + prefix_popc(xw_)] = U[u];
                bp += (uint32_t)__popcll(pw_);
                bx += (uint32_t)__popcll(xw_);
            }
            wave_mem_sync();
            if (try_donate(p, w, root, rs + 1, ksc, npc, nxc, Lc, vb)) continue;
        }
        if (lane == 0) w.R[rs] = vb;
        if (npc + nxc <= 64) {
            wave_mem_sync();
            compact_and_run_small(p, w, root, U, rows, ws, W, Pc, XPc, Lc, ksc, rs + 1, anc || more_here);
            if (w.abort) return;
            continue;
        }
        // push current level, descend
        uint64_t* lvl = w.gstack + (uint64_t)depth * 3 * gws;
        if (lane < W) {
            lvl[lane] = P;
            lvl[gws + lane] = XP;
            lvl[2 * gws + lane] = B;
        }
        // every lane stores the same meta words, so each later reads its own store
        w.gmeta[2 * depth] = ((uint64_t)(anc ? 1u : 0u) << 32) | L;
        w.gmeta[2 * depth + 1] = ks;
        anc = anc || more_here;
        ++depth;
        ++rs;
        P = Pc;
        XP = XPc;
        L = Lc;
        ks = ksc;
        goto enter;
    }
}

// ---------------------------------------------------------------- tasks
// Run a task whose universe U (ascending ranks) is in w.uarr[0, nu), with P / X_P
// as bitmasks staged in w.pw / w.xw (word per entry), X_X in w.xx[0, L).
__device__ void run_universe(const Params& p, Wg& w, uint32_t root, uint32_t nu, uint32_t L, uint64_t ks,
                             uint32_t rs)
{
    const uint32_t lane = lane_id();
    if (nu <= 64) {
        uint64_t row = build_small_rows(p, w, w.uarr, nu);
        uint64_t P = w.pw[0], XP = w.xw[0];
        uint32_t su = lane < nu ? w.uarr[lane] : 0u;
        uint64_t skey = lane < nu ? p.vkey[su] : 0ull;
        run_small(p, w, root, nu, su, skey, row, P, XP, L, ks, rs, false);
        return;
    }
    for (uint32_t i = lane; i < nu; i += 64) w.ukey[i] = p.vkey[w.uarr[i]];
    const uint32_t W = (nu + 63) >> 6;
    uint64_t* rows;
    uint32_t ws;
    if (nu <= p.lds_cap) {
        rows = w.lrows;
        ws = ((p.lds_cap + 63) >> 6) | 1u;
    } else {
        rows = w.grows;
        ws = W | 1u;
        w.hbm_tasks += 1;
    }
    build_rows(p, w, w.uarr, nu, ws, rows);
    uint64_t P = lane < W ? w.pw[lane] : 0ull;
    uint64_t XP = lane < W ? w.xw[lane] : 0ull;
    run_mid(p, w, root, w.uarr, nu, rows, ws, P, XP, L, ks, rs);
}

__device__ void finish_task(const Params& p, Wg& w, uint32_t root, uint64_t c0, uint64_t h0, uint64_t n0)
{
    flush_hist(p, w);
    w.tasks += 1;
    uint64_t dt = uni64(now_ticks()) - w.task_t0;
    w.busy_ticks += dt;
    w.max_task_ticks = max(w.max_task_ticks, dt);
    if ((p.flags & MCE_F_ROOT_STATS) && lane_id() == 0) {
        uint32_t id = p.perm[root];
        atomicAdd(&p.root_count[id], (unsigned long long)(w.count - c0));
        atomicAdd(&p.root_hash[id], (unsigned long long)(w.hash - h0));
        atomicAdd(&p.root_nodes[id], (unsigned long long)(w.nodes - n0));
    }
}

// First-level subtree of root v (Algorithm 3): P = later neighbours, X = earlier.
__device__ void run_root(const Params& p, Wg& w, uint32_t v)
{
    const uint32_t lane = lane_id();
    uint64_t c0 = w.count, h0 = w.hash, n0 = w.nodes;
    w.task_t0 = uni64(now_ticks());
    uint32_t beg = p.op[v], nu = p.op[v + 1] - beg;
    uint32_t ib = p.ip[v], L = p.ip[v + 1] - ib;
    for (uint32_t i = lane; i < nu; i += 64) w.uarr[i] = p.oc[beg + i];
    for (uint32_t i = lane; i < L; i += 64) w.xx[i] = p.ic[ib + i];
    w.root_list_words += nu + L;
    if (lane == 0) w.R[0] = v;
    const uint32_t W = (nu + 63) >> 6;
    for (uint32_t q = lane; q < W; q += 64) {
        uint32_t rem = nu - q * 64;
        w.pw[q] = rem >= 64 ? ~0ull : ((1ull << rem) - 1);
        w.xw[q] = 0;
    }
    wave_mem_sync();
    run_universe(p, w, v, nu, L, p.vkey[v], 1);
    finish_task(p, w, v, c0, h0, n0);
}

// A task received through the worker list; its lists are in this workgroup's mailbox.
__device__ void run_received(const Params& p, Wg& w)
{
    const uint32_t lane = lane_id();
    uint64_t c0 = w.count, h0 = w.hash, n0 = w.nodes;
    w.task_t0 = uni64(now_ticks());
    MboxHdr h = *w.mbox;
    uint32_t np = uni(h.np), nxp = uni(h.nxp), L = uni(h.nxx), rs = uni(h.rsize), root = uni(h.root);
    uint64_t ks = uni64(h.keysum);
    uint32_t nu = np + nxp;
    uint32_t W = (nu + 63) >> 6;
    for (uint32_t q = lane; q < W; q += 64) {
        w.pw[q] = 0;
        w.xw[q] = 0;
    }
    __syncthreads();
    // merge the two ascending lists into U; mark P / X_P membership
    for (uint32_t i = lane; i < np; i += 64) {
        uint32_t x = w.mP[i];
        uint32_t lo = 0, hi = nxp;
        while (lo < hi) {
            uint32_t mid = (lo + hi) >> 1;
            if (w.mXP[mid] < x) lo = mid + 1;
            else hi = mid;
        }
        uint32_t pos = i + lo;
        w.uarr[pos] = x;
        atomicOr((unsigned long long*)&w.pw[pos >> 6], 1ull << (pos & 63));
    }
    for (uint32_t i = lane; i < nxp; i += 64) {
        uint32_t x = w.mXP[i];
        uint32_t lo = 0, hi = np;
        while (lo < hi) {
            uint32_t mid = (lo + hi) >> 1;
            if (w.mP[mid] < x) lo = mid + 1;
            else hi = mid;
        }
        uint32_t pos = i + lo;
        w.uarr[pos] = x;
        atomicOr((unsigned long long*)&w.xw[pos >> 6], 1ull << (pos & 63));
    }
    wave_mem_sync();
    run_universe(p, w, root, nu, L, ks, rs);
    finish_task(p, w, root, c0, h0, n0);
}

__global__ void __launch_bounds__(64) k_enumerate(Params p)
{
    extern __shared__ __align__(16) unsigned char lds[];
    const uint32_t lane = lane_id();
    const uint32_t me = blockIdx.x;
    Wg w = wg_view(p, me);
    uint8_t* base = p.scratch + (uint64_t)me * p.stride;
    w.xflag = reinterpret_cast<uint64_t*>(base + p.off_flag);
    w.hpos = reinterpret_cast<uint32_t*>(base + p.off_hpos);
    w.spos = reinterpret_cast<uint32_t*>(base + p.off_spos);
    w.grows = reinterpret_cast<uint64_t*>(base + p.off_rows);
    w.gstack = reinterpret_cast<uint64_t*>(base + p.off_stack);
    w.gmeta = reinterpret_cast<uint64_t*>(base + p.off_meta);
    // LDS carve-up
    unsigned char* l = lds;
    w.pw = reinterpret_cast<uint64_t*>(l); l += 64 * 8;
    w.xw = reinterpret_cast<uint64_t*>(l); l += 64 * 8;
    w.sP = reinterpret_cast<uint64_t*>(l); l += kSmallDepth * 8;
    w.sXP = reinterpret_cast<uint64_t*>(l); l += kSmallDepth * 8;
    w.sB = reinterpret_cast<uint64_t*>(l); l += kSmallDepth * 8;
    w.sK = reinterpret_cast<uint64_t*>(l); l += kSmallDepth * 8;
    w.sL = reinterpret_cast<uint32_t*>(l); l += kSmallDepth * 4;
    w.sA = reinterpret_cast<uint32_t*>(l); l += kSmallDepth * 4;
    w.hist = reinterpret_cast<uint32_t*>(l); l += kHistLds * 4;
    w.sidx = reinterpret_cast<uint32_t*>(l); l += 64 * 4;
    w.uarr = reinterpret_cast<uint32_t*>(l); l += ((p.ucap + 1) & ~1u) * 4;
    w.ukey = reinterpret_cast<uint64_t*>(l); l += (size_t)p.ucap * 8;
    w.lrows = reinterpret_cast<uint64_t*>(l);
    for (uint32_t k = lane; k < (uint32_t)kHistLds; k += 64) w.hist[k] = 0;
    __syncthreads();
    w.count = w.hash = w.nodes = w.donations = w.tasks = w.xtests = w.edges = w.hbm_tasks = w.idle_ticks = 0;
    w.root_list_words = 0;
    w.probes = 0;
    w.busy_ticks = w.max_task_ticks = w.task_t0 = 0;
    w.hmax = 0;
    w.wl_tick = 0;
    w.wl_seen = 0;
    w.poll = 0;
    w.me = me;
    w.abort = false;
    w.deadline = uni64(now_ticks()) + p.timeout_ticks;

    const bool use_wl = (p.flags & MCE_F_WORKER_LIST) != 0;
    if (use_wl && lane == 0)
        __hip_atomic_fetch_add(&p.ctrl->packed, 1ull << 32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

    // phase 1: first-level subtrees from the shared counter
    while (!w.abort) {
        uint32_t idx = 0;
        if (lane == 0) idx = atomicAdd(&p.ctrl->root_cursor, 1u);
        idx = uni(idx);
        if (idx >= p.nroots) break;
        run_root(p, w, p.roots[idx]);
        if (w.abort) break;
    }
    // phase 2: worker list
    while (use_wl && !w.abort) {
        uint32_t terminate = 0;
        if (lane == 0) {
            __hip_atomic_store(&p.wflags[me], kFlagIdle, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            unsigned long long old =
                __hip_atomic_fetch_add(&p.ctrl->packed, 1ull, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            uint32_t idle = (uint32_t)old + 1, started = (uint32_t)(old >> 32);
            terminate = idle == started;
            if (!terminate) {
                unsigned long long t =
                    __hip_atomic_fetch_add(&p.ctrl->ring_tail, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                uint32_t* slot = &p.ring[t & p.ring_mask];
                while (__hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != kEmptySlot) {
                    if (now_ticks() > w.deadline) break;
                    __builtin_amdgcn_s_sleep(1);
                }
                __hip_atomic_fetch_add(&p.ctrl->waiting, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(slot, me, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        terminate = uni(terminate);
        if (terminate) {
            for (uint32_t g = lane; g < p.nwg; g += 64)
                __hip_atomic_store(&p.wflags[g], kFlagTerm, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        uint32_t f = kFlagIdle;
        uint64_t t0 = now_ticks();
        if (lane == 0) {
            uint32_t sleep = 1;
            // poll with relaxed loads (an acquire load would invalidate caches on
            // every iteration); acquire once below when a task has arrived
            while ((f = __hip_atomic_load(&p.wflags[me], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == kFlagIdle) {
                if (now_ticks() > w.deadline) break;
                if (sleep < 32) sleep <<= 1;
                for (uint32_t s = 0; s < sleep; ++s) __builtin_amdgcn_s_sleep(2);
            }
        }
        f = uni(f);
        w.idle_ticks += now_ticks() - t0;
        if (f == kFlagIdle) {
            if (lane == 0) atomicOr(&p.ctrl->err, 1u);
            w.abort = true;
            break;
        }
        if (f == kFlagTerm) break;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        run_received(p, w);
    }
    flush_hist(p, w);
    uint64_t probes = 0;
    {
        uint32_t pl = w.probes;
        for (int off = 32; off > 0; off >>= 1) pl += (uint32_t)__shfl_xor((int)pl, off, 64);
        probes = pl;
    }
    if (lane == 0) {
        atomicAdd(&p.acc[2 + MCE_STAT_PROBES], (unsigned long long)probes);
        atomicAdd(&p.acc[2 + MCE_STAT_BUSY_NS], (unsigned long long)w.busy_ticks);
        atomicMax(&p.acc[2 + MCE_STAT_MAX_TASK_NS], (unsigned long long)w.max_task_ticks);
        atomicAdd(&p.acc[2 + MCE_STAT_ROOT_WORDS], (unsigned long long)w.root_list_words);
        atomicAdd(&p.acc[0], (unsigned long long)w.count);
        atomicAdd(&p.acc[1], (unsigned long long)w.hash);
        atomicAdd(&p.acc[2 + MCE_STAT_NODES], (unsigned long long)w.nodes);
        atomicAdd(&p.acc[2 + MCE_STAT_DONATIONS], (unsigned long long)w.donations);
        atomicAdd(&p.acc[2 + MCE_STAT_TASKS], (unsigned long long)w.tasks);
        atomicAdd(&p.acc[2 + MCE_STAT_XTESTS], (unsigned long long)w.xtests);
        atomicAdd(&p.acc[2 + MCE_STAT_BUILD_EDGES], (unsigned long long)w.edges);
        atomicAdd(&p.acc[2 + MCE_STAT_HBM_ROWS], (unsigned long long)w.hbm_tasks);
        atomicAdd(&p.acc[2 + MCE_STAT_IDLE_NS], (unsigned long long)w.idle_ticks);
    }
}

// ---------------------------------------------------------------- root queue
// flags[i] = 1 if the i-th root in processing order is in the window and has P != {}.
__global__ void k_root_flags(const uint32_t* __restrict__ op, const uint32_t* __restrict__ core_r, uint32_t n,
                             uint32_t c, uint32_t mode, const uint32_t* __restrict__ custom,
                             const uint32_t* __restrict__ rank, uint32_t* __restrict__ cand,
                             uint32_t* __restrict__ flag)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        uint32_t r;
        if (mode == 1) r = n - 1 - (uint32_t)i;
        else if (mode == 2) r = rank[custom[i]];
        else r = (uint32_t)i;
        cand[i] = r;
        flag[i] = (core_r[r] <= c && op[r + 1] > op[r]) ? 1u : 0u;
    }
}

__global__ void k_root_compact(const uint32_t* __restrict__ cand, const uint32_t* __restrict__ flag,
                               const uint32_t* __restrict__ pos, uint32_t n, uint32_t* __restrict__ roots)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        if (flag[i]) roots[pos[i]] = cand[i];
}

// Isolated vertices are maximal cliques of size 1 (Algorithm 3 with P = X = {}).
__global__ void k_isolated(const uint32_t* __restrict__ op, const uint32_t* __restrict__ ip,
                           const uint64_t* __restrict__ vkey, uint32_t n, unsigned long long* acc,
                           unsigned long long* hist)
{
    uint64_t cnt = 0, h = 0;
    for (size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (size_t)gridDim.x * blockDim.x) {
        if (op[r + 1] == op[r] && ip[r + 1] == ip[r]) {
            cnt += 1;
            h += fmix64(vkey[r] + kGamma);
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        cnt += shfl64(cnt, lane_id() ^ off);
        h += shfl64(h, lane_id() ^ off);
    }
    if (lane_id() == 0 && cnt) {
        atomicAdd(&acc[0], (unsigned long long)cnt);
        atomicAdd(&acc[1], (unsigned long long)h);
        atomicAdd(&hist[1], (unsigned long long)cnt);
    }
}

unsigned blocks_for(size_t items, unsigned per_block, unsigned cap = 65536)
{
    size_t b = (items + per_block - 1) / per_block;
    if (b == 0) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

}  // namespace

mce_status enumerate_graph(const Oriented& g, const EnumConfig& cfg, EnumState& st, hipStream_t s,
                           EnumOutput& out)
{
    mce_status rc;
    const uint32_t n = g.n;
    const size_t nn = n ? n : 1;
    const uint32_t ucap = std::max(g.max_out, 1u);
    if (ucap > kMaxUniverse) {
        set_error("first-level P larger than " + std::to_string(kMaxUniverse) + " vertices is not supported");
        return MCE_ERR_UNSUPPORTED;
    }
    const uint32_t hist_len = g.degeneracy + 3;
    const uint32_t xcap = std::max(g.max_in, 1u);
    const uint32_t rcap = g.degeneracy + 3;
    const uint32_t wg_words = (ucap + 63) / 64;  // words per set at the largest universe
    const uint32_t ws_g = wg_words | 1u;

    // LDS budget for bitmap rows
    uint32_t lds_cap = cfg.bitmap_max_p ? cfg.bitmap_max_p : 256u;
    lds_cap = std::min(lds_cap, ucap);
    if (lds_cap < 64) lds_cap = 64;
    const uint32_t ws_l = ((lds_cap + 63) / 64) | 1u;
    size_t lds_bytes = 64 * 8 * 2 + kSmallDepth * (8 * 4 + 4 * 2) + kHistLds * 4 + 64 * 4 +
                       (size_t)((ucap + 1) & ~1u) * 4 + (size_t)ucap * 8 + (size_t)lds_cap * ws_l * 8;
    lds_bytes = align_up(lds_bytes, 16);
    if (lds_bytes > 160 * 1024) {
        set_error("LDS budget exceeded; lower bitmap_max_p");
        return MCE_ERR_INVALID_ARG;
    }

    int dev = 0;
    MCE_HIP_TRY(hipGetDevice(&dev));
    int cus = 0;
    MCE_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    int per_cu = 0;
    MCE_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k_enumerate), 64,
                                                             lds_bytes));
    if (per_cu <= 0) per_cu = 1;
    if (cfg.wg_per_cu) per_cu = std::min<int>(per_cu, (int)cfg.wg_per_cu);
    uint32_t G = (uint32_t)(per_cu * cus);
    if (G == 0) G = 1;

    // per-workgroup scratch layout
    uint64_t off = align_up(sizeof(MboxHdr), 256);
    const uint64_t off_P = off; off = align_up(off + (uint64_t)ucap * 4, 256);
    const uint64_t off_XP = off; off = align_up(off + (uint64_t)ucap * 4, 256);
    const uint64_t off_R = off; off = align_up(off + (uint64_t)rcap * 4, 256);
    const uint64_t off_xx = off; off = align_up(off + (uint64_t)xcap * 4, 256);
    const uint64_t off_flag = off; off = align_up(off + ((uint64_t)xcap / 64 + 2) * 8, 256);
    const uint64_t off_hpos = off; off = align_up(off + ((uint64_t)xcap / 2 + 2) * 4, 256);
    const uint64_t off_spos = off; off = align_up(off + ((uint64_t)xcap / 2 + 2) * 4, 256);
    const uint64_t off_rows = off; off = align_up(off + (uint64_t)ucap * ws_g * 8, 256);
    const uint64_t off_stack = off; off = align_up(off + (uint64_t)(ucap + 2) * 3 * wg_words * 8, 256);
    const uint64_t off_meta = off; off = align_up(off + (uint64_t)(ucap + 2) * 16, 256);
    const uint64_t stride = off;

    // a budget of 16 GiB of scratch at most; shrink the grid if needed
    const uint64_t budget = 16ull << 30;
    if ((uint64_t)G * stride > budget) G = std::max<uint64_t>(1, budget / stride);

    if ((rc = st.scratch.alloc((size_t)G * stride)) != MCE_OK) return rc;
    if ((rc = st.ctrl.alloc(sizeof(Ctrl))) != MCE_OK) return rc;
    if ((rc = st.acc.alloc(32 * 8)) != MCE_OK) return rc;
    if ((rc = st.hist.alloc((size_t)hist_len * 8)) != MCE_OK) return rc;
    uint32_t ring_cap = 1;
    while (ring_cap < 2 * G) ring_cap <<= 1;
    if ((rc = st.ring.alloc((size_t)ring_cap * 4)) != MCE_OK) return rc;
    if ((rc = st.flags.alloc((size_t)G * 4)) != MCE_OK) return rc;
    if ((rc = st.roots.alloc(nn * 4)) != MCE_OK) return rc;
    if ((rc = st.tmp_a.alloc(nn * 4)) != MCE_OK) return rc;
    if ((rc = st.tmp_b.alloc((nn + 1) * 4)) != MCE_OK) return rc;
    if ((rc = st.tmp_c.alloc(nn * 4)) != MCE_OK) return rc;
    if ((rc = st.scan_tmp.alloc(scan_tmp_words(nn + 1) * 8 + 64)) != MCE_OK) return rc;

    hipEvent_t e0, e1, e2;
    MCE_HIP_TRY(hipEventCreate(&e0));
    MCE_HIP_TRY(hipEventCreate(&e1));
    MCE_HIP_TRY(hipEventCreate(&e2));
    MCE_HIP_TRY(hipEventRecord(e0, s));

    // reset control state (fill kernels, no memset nodes)
    fill_u64(reinterpret_cast<uint64_t*>(st.ctrl.p), 0, sizeof(Ctrl) / 8, s);
    fill_u64(st.acc.as<uint64_t>(), 0, 32, s);
    fill_u64(st.hist.as<uint64_t>(), 0, hist_len, s);
    fill_u32(st.ring.as<uint32_t>(), kEmptySlot, ring_cap, s);
    fill_u32(st.flags.as<uint32_t>(), kFlagIdle, G, s);

    // root queue: window filter + order-preserving compaction
    uint32_t mode = 0;
    if (cfg.flags & MCE_F_CUSTOM_ORDER) mode = 2;
    else if (cfg.flags & MCE_F_REVERSE_ORDER) mode = 1;
    if (mode == 2 && !cfg.root_order) {
        set_error("MCE_F_CUSTOM_ORDER without root_order");
        return MCE_ERR_INVALID_ARG;
    }
    uint32_t* dpos = st.tmp_b.as<uint32_t>();
    uint32_t* dtotal = reinterpret_cast<uint32_t*>(st.acc.as<uint64_t>() + 30);
    if (n) {
        k_root_flags<<<blocks_for(n, 256, 8192), 256, 0, s>>>(g.op.as<uint32_t>(), g.core_r.as<uint32_t>(), n,
                                                              cfg.max_root_core, mode, cfg.root_order,
                                                              g.rank.as<uint32_t>(), st.tmp_a.as<uint32_t>(),
                                                              st.tmp_c.as<uint32_t>());
        MCE_HIP_TRY(hipGetLastError());
        if ((rc = exclusive_scan_u32(st.tmp_c.as<uint32_t>(), dpos, n, dtotal, st.scan_tmp.as<uint64_t>(), s)) !=
            MCE_OK)
            return rc;
        k_root_compact<<<blocks_for(n, 256, 8192), 256, 0, s>>>(st.tmp_a.as<uint32_t>(), st.tmp_c.as<uint32_t>(), dpos,
                                                                n, st.roots.as<uint32_t>());
        MCE_HIP_TRY(hipGetLastError());
        k_isolated<<<blocks_for(n, 256, 4096), 256, 0, s>>>(g.op.as<uint32_t>(), g.ip.as<uint32_t>(),
                                                            g.vkey.as<uint64_t>(), n,
                                                            reinterpret_cast<unsigned long long*>(st.acc.p),
                                                            reinterpret_cast<unsigned long long*>(st.hist.p));
        MCE_HIP_TRY(hipGetLastError());
        MCE_HIP_TRY(hipStreamSynchronize(s));
    }
    uint32_t nroots = 0;
    if (n) {
        MCE_HIP_TRY(hipMemcpyAsync(&nroots, dtotal, 4, hipMemcpyDeviceToHost, s));
        MCE_HIP_TRY(hipStreamSynchronize(s));
    }
    // (acc[30] doubles as the scan total; clear it before the kernel accumulates)
    fill_u64(st.acc.as<uint64_t>() + 30, 0, 1, s);
    MCE_HIP_TRY(hipEventRecord(e1, s));

    Params p{};
    p.op = g.op.as<uint32_t>();
    p.oc = g.oc.as<uint32_t>();
    p.ip = g.ip.as<uint32_t>();
    p.ic = g.ic.as<uint32_t>();
    p.vkey = g.vkey.as<uint64_t>();
    p.perm = g.perm.as<uint32_t>();
    p.roots = st.roots.as<uint32_t>();
    p.nroots = nroots;
    p.ctrl = reinterpret_cast<Ctrl*>(st.ctrl.p);
    p.acc = reinterpret_cast<unsigned long long*>(st.acc.p);
    p.hist = reinterpret_cast<unsigned long long*>(st.hist.p);
    p.hist_len = hist_len;
    p.scratch = st.scratch.as<uint8_t>();
    p.stride = stride;
    p.off_P = off_P;
    p.off_XP = off_XP;
    p.off_R = off_R;
    p.off_xx = off_xx;
    p.off_flag = off_flag;
    p.off_hpos = off_hpos;
    p.off_spos = off_spos;
    p.off_rows = off_rows;
    p.off_stack = off_stack;
    p.off_meta = off_meta;
    p.ring = st.ring.as<uint32_t>();
    p.ring_mask = ring_cap - 1;
    p.wflags = st.flags.as<uint32_t>();
    p.ucap = ucap;
    p.lds_cap = lds_cap;
    p.wg = wg_words;
    p.xcap = xcap;
    p.rcap = rcap;
    p.flags = cfg.flags;
    p.donate_min_p = cfg.donate_min_p ? cfg.donate_min_p : 10u;
    p.donate_max_depth = cfg.donate_max_depth;
    p.nwg = G;
    p.timeout_ticks = (cfg.timeout_ms ? cfg.timeout_ms : 600000ull) * 100000ull;  // 100 MHz clock
    p.root_count = reinterpret_cast<unsigned long long*>(cfg.root_count);
    p.root_hash = reinterpret_cast<unsigned long long*>(cfg.root_hash);
    p.root_nodes = reinterpret_cast<unsigned long long*>(cfg.root_nodes);
    p.s_verts = cfg.stream_vertices;
    p.s_vcap = cfg.stream_vcap;
    p.s_offs = reinterpret_cast<unsigned long long*>(cfg.stream_offsets);
    p.s_ocap = cfg.stream_ocap;
    if ((cfg.flags & MCE_F_ROOT_STATS) && (!cfg.root_count || !cfg.root_hash || !cfg.root_nodes)) {
        set_error("MCE_F_ROOT_STATS needs root_count, root_hash and root_nodes");
        return MCE_ERR_INVALID_ARG;
    }
    if ((cfg.flags & MCE_F_STREAM) && (!cfg.stream_vertices || !cfg.stream_offsets)) {
        set_error("MCE_F_STREAM needs stream buffers");
        return MCE_ERR_INVALID_ARG;
    }

    if (nroots) {
        k_enumerate<<<G, 64, lds_bytes, s>>>(p);
        MCE_HIP_TRY(hipGetLastError());
    }
    MCE_HIP_TRY(hipEventRecord(e2, s));
    uint64_t acc[32];
    Ctrl ctrl;
    out.hist.assign(hist_len, 0);
    MCE_HIP_TRY(hipMemcpyAsync(acc, st.acc.p, sizeof(acc), hipMemcpyDeviceToHost, s));
    MCE_HIP_TRY(hipMemcpyAsync(&ctrl, st.ctrl.p, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    MCE_HIP_TRY(hipMemcpyAsync(out.hist.data(), st.hist.p, (size_t)hist_len * 8, hipMemcpyDeviceToHost, s));
    MCE_HIP_TRY(hipStreamSynchronize(s));
    float ms_setup = 0, ms_kernel = 0;
    (void)hipEventElapsedTime(&ms_setup, e0, e1);
    (void)hipEventElapsedTime(&ms_kernel, e1, e2);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipEventDestroy(e2);

    out.count = acc[0];
    out.hash = acc[1];
    for (int i = 0; i < 16; ++i) out.stats[i] = acc[2 + i];
    out.stats[MCE_STAT_ROOTS] = nroots;
    out.stats[MCE_STAT_WORKGROUPS] = G;
    out.stats[MCE_STAT_KERNEL_NS] = (uint64_t)(ms_kernel * 1e6);
    out.stats[MCE_STAT_SETUP_NS] = (uint64_t)(ms_setup * 1e6);
    out.stats[MCE_STAT_IDLE_NS] = acc[2 + MCE_STAT_IDLE_NS] * 10;  // 100 MHz ticks -> ns
    out.stats[MCE_STAT_BUSY_NS] = acc[2 + MCE_STAT_BUSY_NS] * 10;
    out.stats[MCE_STAT_MAX_TASK_NS] = acc[2 + MCE_STAT_MAX_TASK_NS] * 10;
    out.stats[MCE_STAT_LDS_BYTES] = lds_bytes;
    out.max_size = 0;
    for (uint32_t k = 0; k < hist_len; ++k)
        if (out.hist[k]) out.max_size = k;
    out.stream_c = ctrl.stream_c;
    out.stream_v = ctrl.stream_v;
    out.stream_truncated = ctrl.stream_trunc != 0;
    out.timed_out = (ctrl.err & 1u) != 0;
    st.grid = G;
    st.lds_cap = lds_cap;
    if (out.timed_out) {
        set_error("enumeration exceeded its timeout; results are invalid");
        return MCE_ERR_TIMEOUT;
    }
    return MCE_OK;
}

}  // namespace mce
