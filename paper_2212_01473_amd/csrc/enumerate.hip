// Persistent maximal-clique enumeration kernel for gfx950.
//
// One wavefront (64 lanes) owns one task at a time and explores it depth-first
// (Section III-A): Bron-Kerbosch with pivoting (Algorithm 2) below a
// first-level subtree of Algorithm 3.  A task is (R, P, X_P, X_X):
//   * U = P u X_P, the vertices whose mutual adjacency is kept as bitmap rows
//     over U -- the partial induced subgraph of Section III-D (for a root task
//     U = P = the later neighbours of the root);
//   * X_X, the part of X that came from the task's initial X (for a root: its
//     earlier neighbours).  It only shrinks with depth, so it is one index list
//     partitioned in place with per-level end pointers (Section III-E, Fig. 2).
//     Its adjacency to U is either looked up in the original graph (binary
//     search in the sorted later-neighbour list of the X vertex) or, when |X|
//     is within the budgets, read from bitmaps built once at task start: X rows
//     (X x U) for the register executors and X columns (U -> bitmap over X)
//     for the mid executor, where a child's X_X is then one AND (the full
//     induced subgraph of Section III-D, restricted to X x U);
//   * pivots maximise |P n N(u)| (Tomita); candidates are P u X_P, plus the
//     X_X vertices once they are folded into registers (below).
//
// Three executors share the search:
//   mid    |P u X_P| > 64: W = ceil(|U|/64) words per set, lane w holds word w
//          of P, X_P and of the remaining-branch set; bitmap rows in LDS (or
//          per-workgroup HBM scratch above the LDS budget); stack in HBM.
//   list   |P u X_P| <= 64 with a long X_X: lane k holds the 64-bit row of
//          local vertex k; P, X_P, branches are wave-uniform words; X_X stays
//          an index list; the stack lives in VGPR lanes (lane d = level d).
//   folded |P u X_P| <= 64 and |X_X| <= 64 with X rows available: the X_X
//          vertices get register rows too, so the search touches no memory;
//          X_X vertices are pivot candidates; stack in VGPR lanes.
//
// Work distribution (Section III-C): phase 1 pops (root, split) entries from
// a shared counter; phase 2 is the worker list: idle workgroups set their bit
// in a bitmap, busy ones claim a set bit and hand a branch to its owner, as
// lists or, when it fits 64 vertices, as a fold frame of register rows.
// Results accumulate per graph (several graphs are enumerated as one disjoint
// union in batched mode).
#include "mce_internal.h"

namespace mce {

namespace {

constexpr uint32_t kFlagIdle = 0u, kFlagTask = 1u, kFlagTerm = 2u;
constexpr uint32_t kNoWorkgroup = 0xFFFFFFFFu;
constexpr int kHistLds = 128;
constexpr uint32_t kSixWaveRoots = 256;  // roots per workgroup above which six waves per SIMD run
constexpr uint32_t kMaxUniverse = 4096;    // W <= 64 words per bitmap row

// The counters that every workgroup updates with device-scope atomics each sit
// in a 256-byte block of their own, so they do not contend for one line.
constexpr uint32_t kIdleStride = 32;  // idle bitmap: one 64-bit word per 256 bytes

struct Ctrl {
    alignas(256) unsigned long long packed;  // started << 32 | idle
    alignas(256) unsigned int waiting;       // workgroups currently in the worker list
    alignas(256) unsigned int root_cursor;
    alignas(256) unsigned long long stream_v;
    unsigned long long stream_c;
    unsigned int err;              // 1 = timeout, 4 = inconsistent mailbox
    unsigned int stream_trunc;
    unsigned int tlog_n;           // tasks that qualified for the task log
};

struct MboxHdr {
    uint32_t root;     // root rank (graph and per-root attribution)
    uint32_t rsize;    // |R|
    uint64_t keysum;   // sum of keys of R (mod 2^64)
    uint32_t np, nxp, nxx;
    uint32_t kind;     // kMboxLists or kMboxFold
};

// A donated branch travels either as lists (P, X_P, X_X ranks; the receiver
// builds the bitmaps from the CSR) or, when its universe and X_X each fit 64
// vertices, as a fold frame: the donor's register rows, so the receiver runs
// the folded executor without any construction.  Frame words: P, X_P, then
// per lane rowP[64], skey[64], X row[64]; then ranks su[64], X rank[64].
constexpr uint32_t kMboxLists = 0, kMboxFold = 1;
constexpr uint32_t kFrRow = 2, kFrKey = 66, kFrXRow = 130, kFrU32 = 194;
constexpr uint64_t kFrameBytes = kFrU32 * 8 + 128 * 4;

struct Params {
    const uint32_t* op;
    const uint32_t* oc;
    const uint32_t* ip;
    const uint32_t* ic;
    const uint64_t* vkey;
    const uint32_t* perm;
    const uint32_t* gid;       // graph of each rank, or null (one graph)
    const uint32_t* roots;
    const uint32_t* splits;    // (C << 16) | c per queue entry, or null
    const uint32_t* l2v;       // second-level tasks: root rank per queue entry, or null
    const uint32_t* l2e;       // ... and the edge index of its later neighbour in oc
    uint32_t nroots;
    Ctrl* ctrl;
    unsigned long long* acc;   // kernel-wide statistics
    unsigned long long* gacc;  // per graph: count, hash
    unsigned long long* ghist; // per graph: histogram of hist_len entries
    uint32_t hist_len;
    uint8_t* scratch;
    uint64_t stride;
    uint64_t off_fr;
    uint64_t off_P, off_XP, off_R, off_xr, off_xx, off_flag, off_hpos, off_spos, off_rows, off_xrows, off_xcols, off_stack,
        off_meta, off_ukey, off_susp;
    uint64_t xrow_budget;      // words of X rows per workgroup
    uint64_t xcol_budget;      // words of X columns per workgroup
    uint32_t xrow_ratio;       // build X rows when |X| <= ratio * max(|U|, 64)
    uint32_t xrow_min_u;       // ... and |U| >= xrow_min_u
    unsigned long long* idle_bits;  // bit g % 64 of word (g / 64) * kIdleStride: workgroup g waits
    uint32_t idle_words;
    uint32_t* wflags;
    uint32_t ucap, lds_cap, wg, wgx, xcap, rcap;  // wg / wgx: words per stack level of P and X_X
    uint32_t nv;               // vertices (ranks are < nv)
    uint32_t flags;
    uint32_t donate_min_p, donate_max_depth, donate_every;
    uint32_t nwg;
    uint64_t timeout_ticks;
    unsigned long long* root_count;
    unsigned long long* root_hash;
    unsigned long long* root_nodes;
    uint32_t* s_verts;
    uint64_t s_vcap;
    unsigned long long* s_offs;
    uint64_t s_ocap;
    unsigned long long* tlog;  // task log records (8 words each), or null
    uint64_t tlog_cap;
    uint64_t tlog_min_ticks;
};

// The enumeration kernel's Params, read from the kernel-argument segment (it is
// the kernel's only argument) through a pointer the compiler cannot see through,
// so each function loads the fields it uses where it uses them (scalar loads
// from the constant cache) instead of keeping every field in scalar registers
// for the whole persistent loop.
typedef const __attribute__((address_space(4))) Params* ParamsK;
// Only valid where inlined into the kernel: a called (outlined) function has no
// kernel-argument pointer, so every function that reads the parameters through
// it is force-inlined, and a build test checks that the kernel makes no calls.
__device__ __forceinline__ const Params& kparams()
{
    ParamsK k = (ParamsK)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(k));
    return *(const Params*)k;
}

// ---------------------------------------------------------------- wave helpers
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }
__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni64(uint64_t v)
{
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t rl64(uint64_t v, uint32_t l)
{
    uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, l);
    uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint32_t rl32(uint32_t v, uint32_t l) { return __builtin_amdgcn_readlane(v, l); }
// Register stacks: lane d of a VGPR holds the value of DFS level d; a push
// replaces lane l's value with the wave-uniform x.
__device__ __forceinline__ uint64_t wl64(uint64_t v, uint32_t l, uint64_t x) { return __lane_id() == l ? x : v; }
__device__ __forceinline__ uint32_t wl32(uint32_t v, uint32_t l, uint32_t x) { return __lane_id() == l ? x : v; }
__device__ __forceinline__ uint64_t shfl64(uint64_t v, uint32_t src)
{
    uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, (int)src, 64);
    uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), (int)src, 64);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint32_t prefix_popc(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
// Row rotation through DPP (row_ror:N within rows of 16 lanes).
template <int N>
__device__ __forceinline__ uint32_t row_ror(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x120 + N, 0xF, 0xF, false);
}
// Wave-wide sum / max without LDS round trips (see wave_max).
__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
    v += row_ror<1>(v);
    v += row_ror<2>(v);
    v += row_ror<4>(v);
    v += row_ror<8>(v);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}
// Wave-wide maximum: DPP rotations give every lane its 16-lane row's maximum;
// two row broadcasts (lane 15 into row 1, lane 47 into row 3, then lane 31 into
// rows 2 and 3) leave the maximum of all four rows in lane 63.
__device__ __forceinline__ uint32_t wave_max(uint32_t v)
{
    v = max(v, row_ror<1>(v));
    v = max(v, row_ror<2>(v));
    v = max(v, row_ror<4>(v));
    v = max(v, row_ror<8>(v));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false));  // row_bcast:15
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false));  // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}
__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v)
{
    uint32_t x = v;
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = (uint32_t)__shfl_up((int)x, off, 64);
        if (lane_id() >= (uint32_t)off) x += y;
    }
    return x - v;
}
// Cross-lane visibility of global/LDS stores within the single-wave workgroup.
__device__ __forceinline__ void wave_mem_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_s_barrier();
}
__device__ __forceinline__ uint64_t now_ticks() { return __builtin_amdgcn_s_memrealtime(); }

__device__ __forceinline__ uint64_t fmix64(uint64_t z)
{
    // SplitMix64 output finaliser (Steele, Lea and Flood, OOPSLA 2014).
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t low_mask(uint32_t n) { return n >= 64 ? ~0ull : ((1ull << n) - 1); }

// ---------------------------------------------------------------- per-workgroup state
// Statistics counters kept in LDS (updated by lane 0) to spare scalar registers.
enum : int {
    S_NODES = 0, S_DONATIONS, S_TASKS, S_XTESTS, S_EDGES, S_HBM, S_IDLE, S_ROOTW, S_XROW, S_BUSY, S_MAXTASK,
    S_CTASK, S_HTASK, S_PENDING, S_BUILD, S_DONATE, S_POPFAIL, S_XCOLW, S_FOLDDON, S_COUNT
};

// Fixed-size LDS of a workgroup (static offsets: no pointer registers).
struct LdsFixed {
    uint64_t pw[64], xw[64];
    uint64_t stat[S_COUNT + 4];  // + snapshots at task start: (unused), donations, build time
    uint32_t frame[6];  // suspended executors: mid depth, mid split counter, list depth, list split
                        // counter, list R offset
    uint32_t hist[kHistLds];
    uint32_t sidx[64], soff[64], sbeg[64], sxj[64];
    uint32_t probes[64];  // per lane: list entries read by the X_X binary searches
};
__shared__ LdsFixed S;

// LDS atomics without return: no wait on the search's critical path
__device__ __forceinline__ void stat_add(int k, uint64_t v)
{
    if (__lane_id() == 0) atomicAdd(reinterpret_cast<unsigned long long*>(&S.stat[k]), (unsigned long long)v);
}

// The dynamic LDS of a workgroup: universe keys, universe ranks, bitmap rows.
extern __shared__ __align__(16) unsigned char lds_dyn[];

struct Wg {
    uint32_t me;        // this workgroup's index (selects its scratch block)
    // Scratch and LDS regions, computed where they are used from the
    // workgroup index and the launch's layout (no pointer stays in registers).
    __device__ __forceinline__ uint8_t* base() const
    {
        const Params& p = kparams();
        return p.scratch + (uint64_t)me * p.stride;
    }
    __device__ __forceinline__ MboxHdr* mbox() const { return reinterpret_cast<MboxHdr*>(base()); }
    __device__ __forceinline__ uint32_t* mP() const { return reinterpret_cast<uint32_t*>(base() + kparams().off_P); }     // mailbox P ranks
    __device__ __forceinline__ uint32_t* mXP() const { return reinterpret_cast<uint32_t*>(base() + kparams().off_XP); }   // mailbox X_P ranks
    __device__ __forceinline__ uint32_t* R() const { return reinterpret_cast<uint32_t*>(base() + kparams().off_R); }      // ranks of R
    __device__ __forceinline__ uint64_t* fr() const { return reinterpret_cast<uint64_t*>(base() + kparams().off_fr); }    // mailbox fold frame
    __device__ __forceinline__ uint32_t* xr() const { return reinterpret_cast<uint32_t*>(base() + kparams().off_xr); }    // the task's initial X_X ranks
    __device__ __forceinline__ uint32_t* xx() const { return reinterpret_cast<uint32_t*>(base() + kparams().off_xx); }    // X_X as indices into xr
    __device__ __forceinline__ uint64_t* xflag() const { return reinterpret_cast<uint64_t*>(base() + kparams().off_flag); }
    __device__ __forceinline__ uint32_t* hpos() const { return reinterpret_cast<uint32_t*>(base() + kparams().off_hpos); }
    __device__ __forceinline__ uint32_t* spos() const { return reinterpret_cast<uint32_t*>(base() + kparams().off_spos); }
    __device__ __forceinline__ uint64_t* grows() const { return reinterpret_cast<uint64_t*>(base() + kparams().off_rows); }
    __device__ __forceinline__ uint64_t* xrows() const { return reinterpret_cast<uint64_t*>(base() + kparams().off_xrows); }
    __device__ __forceinline__ uint64_t* xcols() const { return reinterpret_cast<uint64_t*>(base() + kparams().off_xcols); }
    __device__ __forceinline__ uint64_t* gstack() const { return reinterpret_cast<uint64_t*>(base() + kparams().off_stack); }
    __device__ __forceinline__ uint64_t* gmeta() const { return reinterpret_cast<uint64_t*>(base() + kparams().off_meta); }
    __device__ __forceinline__ uint64_t* ukey() const { return reinterpret_cast<uint64_t*>(base() + kparams().off_ukey); }
    // list executor registers while a folded child runs: 4 x 64 words, then 3 x 64 u32
    __device__ __forceinline__ uint64_t* susp64() const { return reinterpret_cast<uint64_t*>(base() + kparams().off_susp); }
    __device__ __forceinline__ uint32_t* susp32() const { return reinterpret_cast<uint32_t*>(susp64() + 4 * 64); }
    __device__ __forceinline__ uint32_t* uarr() const { return reinterpret_cast<uint32_t*>(lds_dyn); }
    __device__ __forceinline__ uint64_t* lrows() const
    {
        return reinterpret_cast<uint64_t*>(lds_dyn + (size_t)((kparams().ucap + 3) & ~3u) * 4);
    }
    // current task
    uint32_t W;         // words of the task's universe
    uint32_t Wx;        // words of the task's X list bitmap (X columns built), else 0
    bool have_xrows;
    // accumulators (wave-uniform)
    uint64_t count, hash;   // since the last per-graph flush
    uint32_t cur_gid;
    uint32_t hmax;
    uint64_t task_t0;
    uint64_t nodes, nodes_t0;  // search-tree nodes (all tasks; at the current task's start)
    uint64_t don_t0;  // start of the current donation attempt
    uint32_t wl_tick, wl_seen, poll, pops;
    uint32_t don_min;  // smallest |P| of a branch offered to the worker list (~0: no worker list)
    uint64_t deadline;
    bool abort;
};
// This workgroup's own state lives in LDS, so the scalar registers are left to
// the search; the fields are touched outside the inner loops only.
__shared__ Wg SW;

// Is b among the later neighbours of x?  (x precedes b in the order.)
__device__ __forceinline__ bool has_later(const Params& p, uint32_t x, uint32_t b)
{
    uint32_t lo = p.op[x], hi = p.op[x + 1], probes = 0;
    bool found = false;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        uint32_t v = p.oc[mid];
        ++probes;
        if (v == b) {
            found = true;
            break;
        }
        if (v < b) lo = mid + 1;
        else hi = mid;
    }
    S.probes[__lane_id()] += probes;
    return found;
}

// Adjacency of X_X entry j (index into xr) to the universe vertex with index
// bidx and rank brank.
__device__ __forceinline__ bool xtest(const Params& p, Wg& w, uint32_t j, uint32_t bidx, uint32_t brank)
{
    if (w.have_xrows) return (w.xrows()[(uint64_t)j * w.W + (bidx >> 6)] >> (bidx & 63)) & 1ull;
    return has_later(p, w.xr()[j], brank);
}

__device__ __forceinline__ bool xx_any(const Params& p, Wg& w, uint32_t L, uint32_t bidx, uint32_t brank)
{
    const uint32_t lane = lane_id();
    for (uint32_t base = 0; base < L; base += 64) {
        uint32_t i = base + lane;
        bool hit = i < L && xtest(p, w, w.xx()[i], bidx, brank);
        stat_add(S_XTESTS, min(64u, L - base));
        if (__ballot(hit)) return true;
    }
    return false;
}

// Partition xx[0, L): entries adjacent to b move to [0, K), the rest to
// [K, L), so every level's X_X stays a prefix (Section III-E).  Only
// misplaced entries move: holes in [0, K) swap with kept entries in [K, L).
__device__ __forceinline__ uint32_t xx_partition(const Params& p, Wg& w, uint32_t L, uint32_t bidx, uint32_t brank)
{
    const uint32_t lane = lane_id();
    uint32_t K = 0;
    for (uint32_t base = 0; base < L; base += 64) {
        uint32_t i = base + lane;
        bool keep = i < L && xtest(p, w, w.xx()[i], bidx, brank);
        uint64_t m = __ballot(keep);
        if (lane == 0) w.xflag()[base >> 6] = m;
        K += (uint32_t)__popcll(m);
    }
    stat_add(S_XTESTS, L);
    if (K == 0 || K == L) return K;
    wave_mem_sync();
    uint32_t nh = 0;
    for (uint32_t base = 0; base < K; base += 64) {
        uint64_t m = w.xflag()[base >> 6];
        uint32_t i = base + lane;
        bool hole = i < K && !((m >> lane) & 1ull);
        uint64_t hm = __ballot(hole);
        if (hole) w.hpos()[nh + prefix_popc(hm)] = i;
        nh += (uint32_t)__popcll(hm);
    }
    uint32_t ns = 0;
    for (uint32_t base = K & ~63u; base < L; base += 64) {
        uint64_t m = w.xflag()[base >> 6];
        uint32_t i = base + lane;
        bool stray = i >= K && i < L && ((m >> lane) & 1ull);
        uint64_t sm = __ballot(stray);
        if (stray) w.spos()[ns + prefix_popc(sm)] = i;
        ns += (uint32_t)__popcll(sm);
    }
    wave_mem_sync();
    for (uint32_t k = lane; k < nh; k += 64) {
        uint32_t a = w.hpos()[k], s = w.spos()[k];
        uint32_t va = w.xx()[a], vs = w.xx()[s];
        w.xx()[a] = vs;
        w.xx()[s] = va;
    }
    wave_mem_sync();
    return K;
}

// ---------------------------------------------------------------- results
__device__ __forceinline__ void flush_graph(const Params& p_arg, Wg& w)
{
    const Params& p = kparams();
    (void)p_arg;
    const uint32_t lane = lane_id();
    if (lane == 0 && (w.count | w.hash)) {
        atomicAdd(&p.gacc[2 * w.cur_gid], (unsigned long long)w.count);
        atomicAdd(&p.gacc[2 * w.cur_gid + 1], (unsigned long long)w.hash);
    }
    uint32_t top = min(w.hmax + 1, (uint32_t)kHistLds);
    wave_mem_sync();
    unsigned long long* gh = p.ghist + (uint64_t)w.cur_gid * p.hist_len;
    for (uint32_t k = lane; k < top; k += 64) {
        uint32_t c = S.hist[k];
        if (c) {
            atomicAdd(&gh[k], (unsigned long long)c);
            S.hist[k] = 0;
        }
    }
    wave_mem_sync();
    w.count = w.hash = 0;
    w.hmax = 0;
}

__device__ __forceinline__ void report(const Params& p_arg, Wg& w, uint32_t rsize, uint64_t ks)
{
    const Params& p = kparams();
    (void)p_arg;
    uint64_t h = fmix64(ks + (uint64_t)rsize * kGamma);
    w.count += 1;
    w.hash += h;
    if (p.flags & MCE_F_ROOT_STATS) {
        stat_add(S_CTASK, 1);
        stat_add(S_HTASK, h);
    }
    w.hmax = max(w.hmax, rsize);
    const uint32_t lane = lane_id();
    if (lane == 0) {
        if (rsize < (uint32_t)kHistLds) atomicAdd(&S.hist[rsize], 1u);
        else atomicAdd(&p.ghist[(uint64_t)w.cur_gid * p.hist_len + min(rsize, p.hist_len - 1)], 1ull);
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
        if (fits)
            for (uint32_t j = lane; j < rsize; j += 64) p.s_verts[v + j] = p.perm[w.R()[j]];
        if (lane == 0) {
            if (c < p.s_ocap) p.s_offs[c] = fits ? ((v << 16) | rsize) : ~0ull;
            if (!fits || c >= p.s_ocap) p.ctrl->stream_trunc = 1;
        }
    }
    // keep the per-size LDS counters (32-bit) far from overflow within one task
    if (w.count > (1ull << 30)) flush_graph(p, w);
}

__device__ __forceinline__ bool check_deadline(const Params& p_arg, Wg& w)
{
    const Params& p = kparams();
    (void)p_arg;
    if (w.abort) return true;
    if (now_ticks() > w.deadline) {
        if (lane_id() == 0) atomicOr(&p.ctrl->err, 1u);
        w.abort = true;
    }
    return w.abort;
}

// ---------------------------------------------------------------- worker list
__device__ __forceinline__ Wg wg_view(const Params& p, uint32_t g)
{
    (void)p;
    Wg w;
    w.me = g;
    return w;
}

// Claim an idle workgroup (or kNoWorkgroup).  All 64 lanes read one word of the
// idle bitmap each, starting at a word that rotates per attempt; lane 0 then
// clears a set bit of a non-empty word with one fetch-and, which either wins
// that bit or returns the word's current value for the next try.  Donors start
// at different words and bits, so claims rarely collide.  The bitmap carries
// no task data: all accesses are relaxed; the task is published with
// release/acquire on the receiver's flag.
__device__ __forceinline__ uint32_t wl_try_pop(const Params& p_arg, Wg& w)
{
    const Params& p = kparams();
    (void)p_arg;
    const uint32_t lane = lane_id();
    const uint32_t nw = p.idle_words;
    w.don_t0 = uni64(now_ticks());
    const uint32_t q0 = (w.me + 7u * w.pops++) % nw;
    const uint32_t s = w.me & 63u;
    uint32_t r = kNoWorkgroup;
    uint32_t tried = 0;
    for (uint32_t base = 0; base < nw && r == kNoWorkgroup && tried < 4; base += 64) {
        const uint32_t k = base + lane;
        uint32_t q = q0 + k;
        if (q >= nw) q -= nw;
        uint64_t b = 0;
        if (k < nw) b = __hip_atomic_load(&p.idle_bits[q * kIdleStride], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint64_t nz = __ballot(b != 0);
        while (nz != 0 && r == kNoWorkgroup && tried < 4) {
            const uint32_t l = (uint32_t)__builtin_ctzll(nz);
            nz &= nz - 1;
            ++tried;
            uint64_t bw = rl64(b, l);
            const uint32_t qw = rl32(q, l);
            uint32_t got = kNoWorkgroup;
            if (lane == 0) {
                for (int t = 0; t < 3 && bw != 0; ++t) {
                    const uint64_t rot = s ? ((bw >> s) | (bw << (64u - s))) : bw;
                    const uint32_t i = ((uint32_t)__builtin_ctzll(rot) + s) & 63u;
                    const uint64_t m = 1ull << i;
                    const uint64_t old = __hip_atomic_fetch_and(&p.idle_bits[qw * kIdleStride], ~m, __ATOMIC_RELAXED,
                                                                __HIP_MEMORY_SCOPE_AGENT);
                    if (old & m) {
                        got = qw * 64u + i;
                        break;
                    }
                    bw = old & ~m;
                }
                if (got != kNoWorkgroup) {
                    __hip_atomic_fetch_add(&p.ctrl->waiting, ~0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    // the receiver stops counting as idle before it is handed work
                    __hip_atomic_fetch_add(&p.ctrl->packed, ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            r = uni(got);
        }
    }
    if (r == kNoWorkgroup) {
        // skip the next offer: other donors emptied the bitmap first
        w.wl_seen = 0;
        stat_add(S_POPFAIL, 1);
        stat_add(S_DONATE, uni64(now_ticks()) - w.don_t0);
    }
    return r;
}

// Should this branch be offered to an idle workgroup (Section III-C)?  Only
// branches with |P| >= donate_min_p, with unexplored siblings at this level and
// unexplored branches at an earlier level.  The waiting count read here was
// loaded at the previous check, so its latency overlaps the search.
__device__ __forceinline__ bool donation_wanted(const Params& p_arg, Wg& w, uint32_t np_child, bool more_here, bool anc,
                                       uint32_t depth)
{
    const Params& p = kparams();
    (void)p_arg;
    // w.don_min: donate_min_p, or ~0 without the worker list; almost every
    // branch stops at this one compare
    // (fields kept in LDS are read through readfirstlane: the branches on them
    // are then known to be wave-uniform)
    if (__builtin_expect(np_child < uni(w.don_min), 1)) return false;
    if (!more_here || !anc) return false;
    if (p.donate_max_depth && depth > p.donate_max_depth) return false;
    if (p.donate_every > 1) {
        const uint32_t tick = uni(w.wl_tick) + 1;
        w.wl_tick = tick;
        if (tick % p.donate_every != 0) return false;
    }
    uint32_t prev = w.wl_seen;
    w.wl_seen = __hip_atomic_load(&p.ctrl->waiting, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return uni(prev) != 0;
}

// Finish a donation to r: R (this workgroup's R[0, rs) plus vb), header, one
// release fence, then the flag.  The caller wrote the branch itself: the P,
// X_P and X_X lists (kMboxLists) or a fold frame (kMboxFold).
__device__ __forceinline__ void publish_task(const Params& p_arg, Wg& w, uint32_t r, uint32_t root, uint32_t rs, uint32_t vb,
                             uint64_t ks, uint32_t np, uint32_t nxp, uint32_t nxx, uint32_t kind)
{
    const Params& p = kparams();
    (void)p_arg;
    const uint32_t lane = lane_id();
    Wg d = wg_view(p, r);
    for (uint32_t i = lane; i < rs; i += 64) d.R()[i] = w.R()[i];
    if (lane == 0) {
        d.R()[rs] = vb;
        MboxHdr h;
        h.root = root;
        h.rsize = rs + 1;
        h.keysum = ks;
        h.np = np;
        h.nxp = nxp;
        h.nxx = nxx;
        h.kind = kind;
        *d.mbox() = h;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (lane == 0) __hip_atomic_store(&p.wflags[r], kFlagTask, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    stat_add(S_DONATIONS, 1);
    if (kind == kMboxFold) stat_add(S_FOLDDON, 1);
    stat_add(S_DONATE, uni64(now_ticks()) - w.don_t0);
}

// ---------------------------------------------------------------- executors
// Three executors share one dispatcher (run_task), so each is instantiated
// once.  The mid executor (universe > 64 vertices) and the list executor
// (universe <= 64, X_X as an index list) hand a child whose P u X_P has at
// most 64 vertices to a smaller executor: they push their current level, as
// for a descent, keep a small frame in LDS and return; the dispatcher runs the
// smaller executor and resumes them, which pops that level.  Only the
// running executor's state is live in registers.

// A node over a universe of m <= 64 vertices (lane k holds vertex k), passed
// from one executor to the next.
struct SmallJob {
    uint32_t m, L, rs;
    uint32_t su, oidx, xj;  // per lane: rank, index in the task universe, X_X entry of lane (< L)
    uint64_t skey, rowP;    // per lane: key, adjacency over the small universe
    uint64_t P, XP, ks;
    bool anc;
};

enum : uint32_t { kDone = 0, kYieldFold = 1, kYieldList = 2 };

// Adjacency of X_X entry xj (vx: this lane holds one) over a small universe
// whose vertex k is task-universe vertex oidx_k, ascending in k; with a
// one-word task universe the small universe is the task universe itself.
__device__ __forceinline__ uint64_t fold_xrow(const Wg& w, bool vx, uint32_t xj, uint32_t oidx, uint32_t m)
{
    if (w.W == 1) return vx ? w.xrows()[xj] : 0ull;
    // o_k ascend with k: load each X-row word once
    const uint64_t* xrow = w.xrows() + (uint64_t)xj * w.W;
    uint64_t xrowP = 0;
    uint32_t k = 0;
    while (k < m) {
        uint32_t q = rl32(oidx, k) >> 6;
        uint64_t word = vx ? xrow[q] : 0ull;
        for (; k < m; ++k) {
            uint32_t ok = rl32(oidx, k);
            if ((ok >> 6) != q) break;
            xrowP |= ((word >> (ok & 63)) & 1ull) << k;
        }
    }
    return xrowP;
}

// Write a fold frame into d's mailbox: universe of m vertices (lane k: rank
// su, key skey, row rowP), P / X_P masks, and this lane's X_X entry (xin) at
// slot xslot (rank xrank, row xrowP over the universe).
__device__ __forceinline__ void put_fold_frame(const Wg& d, uint32_t m, uint64_t P, uint64_t XP, uint32_t su,
                                               uint64_t skey, uint64_t rowP, bool xin, uint32_t xslot,
                                               uint32_t xrank, uint64_t xrowP)
{
    const uint32_t lane = lane_id();
    uint64_t* f = d.fr();
    uint32_t* f32 = reinterpret_cast<uint32_t*>(f + kFrU32);
    if (lane == 0) {
        f[0] = P;
        f[1] = XP;
    }
    if (lane < m) {
        f[kFrRow + lane] = rowP;
        f[kFrKey + lane] = skey;
        f32[lane] = su;
    }
    if (xin) {
        f[kFrXRow + xslot] = xrowP;
        f32[64 + xslot] = xrank;
    }
}
enum : uint32_t { kExDone = 0, kExFold = 1, kExList = 2, kExMid = 3 };

// ---------------------------------------------------------------- folded executor
// Register stack writes: lane l of v takes the wave-uniform x (v_writelane).
// The compiler offers no builtin for it; the declaration binds the LLVM
// intrinsic, so hazards are still handled by the backend.
extern "C" __device__ int mce_writelane_i32(int value, int lane, int old) __asm("llvm.amdgcn.writelane.i32");
__device__ __forceinline__ uint32_t wlane32(uint32_t v, uint32_t l, uint32_t x)
{
    return (uint32_t)mce_writelane_i32((int)x, (int)l, (int)v);
}
__device__ __forceinline__ uint64_t wlane64(uint64_t v, uint32_t l, uint64_t x)
{
    const uint32_t lo = wlane32((uint32_t)v, l, (uint32_t)x);
    const uint32_t hi = wlane32((uint32_t)(v >> 32), l, (uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Maximal cliques found by the folded executor are reported in groups of 64:
// lane i of a pending pair holds the i-th clique's key sum plus |C| * gamma
// (the argument of h) and its size; a full group is hashed on all 64 lanes at
// once.  Per-lane hash sums are reduced into the workgroup's total when the
// executor returns.
struct LeafGroup {
    uint64_t pre;   // per lane: sum of keys + |C| * gamma
    uint32_t size;  // per lane: |C|
    uint32_t n;     // pending cliques (wave-uniform), < 64
    uint64_t hsum;  // per lane: sum of hashed cliques
};

__device__ __forceinline__ void leaf_group_flush(const Params& p_arg, Wg& w, LeafGroup& g)
{
    const Params& p = kparams();
    (void)p_arg;
    const uint32_t lane = lane_id();
    const uint32_t n = g.n;
    if (n == 0) return;
    const bool on = lane < n;
    const uint64_t h = on ? fmix64(g.pre) : 0ull;
    g.hsum += h;
    const uint32_t sz = on ? g.size : 0u;
    if (on) {
        if (sz < (uint32_t)kHistLds) atomicAdd(&S.hist[sz], 1u);
        else atomicAdd(&p.ghist[(uint64_t)w.cur_gid * p.hist_len + min(sz, p.hist_len - 1)], 1ull);
    }
    w.hmax = max(w.hmax, wave_max(sz));
    w.count += n;
    if (p.flags & MCE_F_ROOT_STATS) {
        uint32_t lo = (uint32_t)h, hi = (uint32_t)(h >> 32);
        // 64-bit wave sum as two 32-bit sums of 32-bit halves (carries from the low half added back)
        uint64_t slo = 0, shi = 0;
        for (uint32_t t = 0; t < n; ++t) {
            slo += rl32(lo, t);
            shi += rl32(hi, t);
        }
        stat_add(S_CTASK, n);
        stat_add(S_HTASK, slo + (shi << 32));
    }
    g.n = 0;
    // keep the per-size LDS counters (32-bit) far from overflow within one task
    if (w.count > (1ull << 30)) flush_graph(p, w);
}

__device__ __forceinline__ void leaf_group_close(const Params& p_arg, Wg& w, LeafGroup& g)
{
    const Params& p = kparams();
    (void)p_arg;
    leaf_group_flush(p, w, g);
    uint64_t v = g.hsum;
    for (int off = 32; off > 0; off >>= 1) v += shfl64(v, lane_id() ^ (uint32_t)off);
    w.hash += uni64(v);
    g.hsum = 0;
}

// Universe of m <= 64 vertices (lane k: rank su, key skey, rowP over the
// universe, rowX over the folded X set); folded X set of up to 64 vertices
// (lane j: rank xrank, xrowP = its adjacency over the universe).  X_X (L <= 64
// entries, lane j holds entry xj) is folded from the X rows first.
// The wave-uniform state of a level is P, X_P, X_X (bitmasks over the lanes),
// the branches B still to visit and kg = (sum of keys of R) + |R| * gamma; the
// stack keeps them in lane d of a VGPR for level d.
//
// The search loop holds wave-uniform branches only; whatever needs per-lane
// control flow (hashing a full group of cliques, offering a branch to an idle
// workgroup, the watchdog, the clique stream) leaves the loop with an event,
// is handled below it, and the loop resumes where it stopped.  Wave-divergent
// code inside the loop would make the compiler rewrite the loop's uniform
// branches into predicated flow with state copies on every iteration.
enum : uint32_t { kEvDone = 0, kEvLeaves = 1, kEvOffer = 2, kEvCheck = 3 };

// Entry points of the assembly search loop (passed in the event register).
enum : uint32_t { kAsmChild = 0, kAsmNode = 1, kAsmDescend = 2 };
constexpr uint32_t kNoOffer = 0xFFFFFFFFu;  // donation threshold that no |P| reaches

// The folded executor's search loop for the counting form, in gfx950
// assembly.  It runs the steps of the C++ loop of run_folded in the same
// order; the compiler's own code for that loop spends about half of its
// scalar instructions on copies of loop-carried values and lane-mask flags,
// and scalar issue is what bounds the kernel.  Registers (fixed by the asm
// constraints at the call):
//   s[40:41] P   s[42:43] X_P   s[44:45] X_X   s[46:47] B   s[48:49] kg
//   s[50:51] Pc  s[52:53] XPc   s[54:55] XXc   s[56:57] kgc (current child)
//   s64 depth  s65 nodes  s66 pending cliques  s67 entry in / event out
//   s68 child lane bb  s69 |Pc|  s70 next watchdog count  s71 donate_min_p
//   s72 |R| + 1 at depth 0  s73 1 if the task has unexplored ancestors
//   v[48:49] rowP  v[50:51] rowX  v[52:53] key + gamma  v[54:55] X_X rows
//   v[56:57] 1 << lane  v58 vertex  v59 255 - lane  v60 191 - lane
//   v[62:71] stack of P, X_P, X_X, B, kg (lane d: level d)  v61 stack of R
//   v[72:73] pending clique keys  v74 pending clique sizes
//   scratch: s58-s63, s74-s85, v75-v78; m0 is saved in s76 and restored.
// Wait states: two after a VALU write before a DPP read of it and before a
// v_cndmask reads a VALU-written vcc, one before a VALU reads an SGPR a VALU
// wrote; lane selects are always written by scalar instructions.  Entry and
// exit add four, for the code around the block.
#define FOLDED_SEARCH_ASM \
    "s_nop 4\n" \
    "s_mov_b32 s76, m0\n" \
    "s_cmp_eq_u32 s67, 1\n" \
    "s_cbranch_scc1 .Lfs_node_%=\n" \
    "s_cmp_eq_u32 s67, 2\n" \
    "s_cbranch_scc1 .Lfs_desc_%=\n" \
    "s_branch .Lfs_child_%=\n" \
    /* descend into the child: push the level, P = Pc ... */ \
    ".Lfs_desc_%=:\n" \
    "v_readlane_b32 s74, v58, s68\n" \
    "s_mov_b32 m0, s64\n" \
    "v_writelane_b32 v62, s40, m0\n" \
    "v_writelane_b32 v63, s41, m0\n" \
    "v_writelane_b32 v64, s42, m0\n" \
    "v_writelane_b32 v65, s43, m0\n" \
    "v_writelane_b32 v66, s44, m0\n" \
    "v_writelane_b32 v67, s45, m0\n" \
    "v_writelane_b32 v68, s46, m0\n" \
    "v_writelane_b32 v69, s47, m0\n" \
    "v_writelane_b32 v70, s48, m0\n" \
    "v_writelane_b32 v71, s49, m0\n" \
    "v_writelane_b32 v61, s74, m0\n" \
    "s_add_u32 s64, s64, 1\n" \
    "s_mov_b64 s[40:41], s[50:51]\n" \
    "s_mov_b64 s[42:43], s[52:53]\n" \
    "s_mov_b64 s[44:45], s[54:55]\n" \
    "s_mov_b64 s[48:49], s[56:57]\n" \
    /* pivot step: B = P minus the neighbours of the best of P u X_P u X_X */ \
    ".Lfs_node_%=:\n" \
    "s_add_u32 s65, s65, 1\n" \
    "s_or_b64 s[58:59], s[40:41], s[42:43]\n" \
    "v_and_b32_e32 v75, s40, v48\n" \
    "v_and_b32_e32 v76, s41, v49\n" \
    "v_bcnt_u32_b32 v75, v75, 0\n" \
    "v_bcnt_u32_b32 v75, v76, v75\n" \
    "v_lshl_or_b32 v75, v75, 8, v59\n" \
    "v_and_b32_e32 v76, s58, v56\n" \
    "v_and_b32_e32 v77, s59, v57\n" \
    "v_or_b32_e32 v76, v76, v77\n" \
    "v_cmp_ne_u32_e32 vcc, 0, v76\n" \
    "s_nop 1\n" \
    "v_cndmask_b32_e32 v75, 0, v75, vcc\n" \
    "s_cmp_eq_u64 s[44:45], 0\n" \
    "s_cbranch_scc1 .Lfs_nokx_%=\n" \
    "v_and_b32_e32 v76, s40, v54\n" \
    "v_and_b32_e32 v77, s41, v55\n" \
    "v_bcnt_u32_b32 v76, v76, 0\n" \
    "v_bcnt_u32_b32 v76, v77, v76\n" \
    "v_lshl_or_b32 v76, v76, 8, v60\n" \
    "v_and_b32_e32 v77, s44, v56\n" \
    "v_and_b32_e32 v78, s45, v57\n" \
    "v_or_b32_e32 v77, v77, v78\n" \
    "v_cmp_ne_u32_e32 vcc, 0, v77\n" \
    "s_nop 1\n" \
    "v_cndmask_b32_e32 v76, 0, v76, vcc\n" \
    "v_max_u32_e32 v75, v75, v76\n" \
    ".Lfs_nokx_%=:\n" \
    "s_nop 1\n" \
    "v_max_u32_dpp v75, v75, v75 row_ror:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n" \
    "s_nop 1\n" \
    "v_max_u32_dpp v75, v75, v75 row_ror:2 row_mask:0xf bank_mask:0xf bound_ctrl:1\n" \
    "s_nop 1\n" \
    "v_max_u32_dpp v75, v75, v75 row_ror:4 row_mask:0xf bank_mask:0xf bound_ctrl:1\n" \
    "s_nop 1\n" \
    "v_max_u32_dpp v75, v75, v75 row_ror:8 row_mask:0xf bank_mask:0xf bound_ctrl:1\n" \
    "s_nop 1\n" \
    "v_max_u32_dpp v75, v75, v75 row_bcast:15 row_mask:0xa bank_mask:0xf\n" \
    "s_nop 1\n" \
    "v_max_u32_dpp v75, v75, v75 row_bcast:31 row_mask:0xc bank_mask:0xf\n" \
    "s_nop 1\n" \
    "v_readlane_b32 s74, v75, 63\n" \
    "s_andn2_b32 s74, 0xff, s74\n" \
    "s_cmp_lt_u32 s74, 64\n" \
    "s_cbranch_scc0 .Lfs_pivx_%=\n" \
    "v_readlane_b32 s59, v49, s74\n" \
    "v_readlane_b32 s58, v48, s74\n" \
    "s_branch .Lfs_pivd_%=\n" \
    ".Lfs_pivx_%=:\n" \
    "s_sub_u32 s74, s74, 64\n" \
    "v_readlane_b32 s59, v55, s74\n" \
    "v_readlane_b32 s58, v54, s74\n" \
    ".Lfs_pivd_%=:\n" \
    "s_andn2_b64 s[46:47], s[40:41], s[58:59]\n" \
    "s_cmp_ge_u32 s65, s70\n" \
    "s_cbranch_scc0 .Lfs_child_%=\n" \
    "s_mov_b32 s67, 3\n" \
    "s_branch .Lfs_exit_%=\n" \
    /* return from a level whose branches are done */ \
    ".Lfs_pop_%=:\n" \
    "s_cmp_eq_u32 s64, 0\n" \
    "s_cbranch_scc1 .Lfs_done_%=\n" \
    "s_sub_u32 s64, s64, 1\n" \
    "v_readlane_b32 s40, v62, s64\n" \
    "v_readlane_b32 s41, v63, s64\n" \
    "v_readlane_b32 s42, v64, s64\n" \
    "v_readlane_b32 s43, v65, s64\n" \
    "v_readlane_b32 s44, v66, s64\n" \
    "v_readlane_b32 s45, v67, s64\n" \
    "v_readlane_b32 s46, v68, s64\n" \
    "v_readlane_b32 s47, v69, s64\n" \
    "v_readlane_b32 s48, v70, s64\n" \
    "v_readlane_b32 s49, v71, s64\n" \
    /* the next child, lane bb = lowest of B */ \
    ".Lfs_child_%=:\n" \
    "s_cmp_eq_u64 s[46:47], 0\n" \
    "s_cbranch_scc1 .Lfs_pop_%=\n" \
    "s_ff1_i32_b64 s68, s[46:47]\n" \
    "s_lshl_b64 s[60:61], 1, s68\n" \
    "s_andn2_b64 s[46:47], s[46:47], s[60:61]\n" \
    "v_readlane_b32 s59, v49, s68\n" \
    "v_readlane_b32 s58, v48, s68\n" \
    "v_readlane_b32 s57, v53, s68\n" \
    "v_readlane_b32 s56, v52, s68\n" \
    "s_and_b64 s[50:51], s[40:41], s[58:59]\n" \
    "s_and_b64 s[52:53], s[42:43], s[58:59]\n" \
    "s_andn2_b64 s[40:41], s[40:41], s[60:61]\n" \
    "s_or_b64 s[42:43], s[42:43], s[60:61]\n" \
    "s_add_u32 s56, s56, s48\n" \
    "s_addc_u32 s57, s57, s49\n" \
    "s_mov_b64 s[54:55], 0\n" \
    "s_cmp_eq_u64 s[44:45], 0\n" \
    "s_cbranch_scc1 .Lfs_noxx_%=\n" \
    "v_readlane_b32 s55, v51, s68\n" \
    "v_readlane_b32 s54, v50, s68\n" \
    "s_and_b64 s[54:55], s[54:55], s[44:45]\n" \
    ".Lfs_noxx_%=:\n" \
    "s_cmp_lg_u64 s[50:51], 0\n" \
    "s_cbranch_scc1 .Lfs_inner_%=\n" \
    /* a leaf: maximal when X_P and X_X of the child are empty */ \
    "s_add_u32 s65, s65, 1\n" \
    "s_or_b64 s[58:59], s[52:53], s[54:55]\n" \
    "s_cmp_lg_u64 s[58:59], 0\n" \
    "s_cbranch_scc1 .Lfs_child_%=\n" \
    "s_add_u32 s77, s72, s64\n" \
    "s_mov_b32 m0, s66\n" \
    "v_writelane_b32 v72, s56, m0\n" \
    "v_writelane_b32 v73, s57, m0\n" \
    "v_writelane_b32 v74, s77, m0\n" \
    "s_add_u32 s66, s66, 1\n" \
    "s_cmp_lt_u32 s66, 63\n" \
    "s_cbranch_scc1 .Lfs_child_%=\n" \
    "s_mov_b32 s67, 1\n" \
    "s_branch .Lfs_exit_%=\n" \
    ".Lfs_inner_%=:\n" \
    "s_bcnt1_i32_b64 s69, s[50:51]\n" \
    "s_cmp_gt_u32 s69, 2\n" \
    "s_cbranch_scc0 .Lfs_small_%=\n" \
    /* |Pc| > 2: offered when large, with siblings left and ancestors */ \
    "s_cmp_lt_u32 s69, s71\n" \
    "s_cbranch_scc1 .Lfs_desc_%=\n" \
    "s_cmp_eq_u64 s[46:47], 0\n" \
    "s_cbranch_scc1 .Lfs_desc_%=\n" \
    "s_or_b32 s74, s64, s73\n" \
    "s_cmp_eq_u32 s74, 0\n" \
    "s_cbranch_scc1 .Lfs_desc_%=\n" \
    "s_mov_b32 s67, 2\n" \
    "s_branch .Lfs_exit_%=\n" \
    /* |Pc| = 1 or 2: pivot on its first vertex a, finish the subtree */ \
    ".Lfs_small_%=:\n" \
    "s_ff1_i32_b64 s74, s[50:51]\n" \
    "v_readlane_b32 s59, v49, s74\n" \
    "v_readlane_b32 s58, v48, s74\n" \
    "v_readlane_b32 s61, v53, s74\n" \
    "v_readlane_b32 s60, v52, s74\n" \
    "s_mov_b64 s[62:63], 0\n" \
    "s_cmp_eq_u64 s[54:55], 0\n" \
    "s_cbranch_scc1 .Lfs_sa_%=\n" \
    "v_readlane_b32 s63, v51, s74\n" \
    "v_readlane_b32 s62, v50, s74\n" \
    ".Lfs_sa_%=:\n" \
    "s_add_u32 s60, s60, s56\n" \
    "s_addc_u32 s61, s61, s57\n" \
    "s_add_u32 s77, s72, s64\n" \
    "s_add_u32 s77, s77, 1\n" \
    "s_cmp_eq_u32 s69, 1\n" \
    "s_cbranch_scc0 .Lfs_two_%=\n" \
    "s_add_u32 s65, s65, 2\n" \
    "s_and_b64 s[84:85], s[58:59], s[52:53]\n" \
    "s_and_b64 s[62:63], s[62:63], s[54:55]\n" \
    "s_or_b64 s[84:85], s[84:85], s[62:63]\n" \
    "s_cmp_lg_u64 s[84:85], 0\n" \
    "s_cbranch_scc1 .Lfs_child_%=\n" \
    "s_mov_b32 m0, s66\n" \
    "v_writelane_b32 v72, s60, m0\n" \
    "v_writelane_b32 v73, s61, m0\n" \
    "v_writelane_b32 v74, s77, m0\n" \
    "s_add_u32 s66, s66, 1\n" \
    "s_branch .Lfs_full_%=\n" \
    ".Lfs_two_%=:\n" \
    "s_lshl_b64 s[84:85], 1, s74\n" \
    "s_andn2_b64 s[84:85], s[50:51], s[84:85]\n" \
    "s_ff1_i32_b64 s75, s[84:85]\n" \
    "v_readlane_b32 s79, v49, s75\n" \
    "v_readlane_b32 s78, v48, s75\n" \
    "v_readlane_b32 s81, v53, s75\n" \
    "v_readlane_b32 s80, v52, s75\n" \
    "s_mov_b64 s[82:83], 0\n" \
    "s_cmp_eq_u64 s[54:55], 0\n" \
    "s_cbranch_scc1 .Lfs_sc_%=\n" \
    "v_readlane_b32 s83, v51, s75\n" \
    "v_readlane_b32 s82, v50, s75\n" \
    ".Lfs_sc_%=:\n" \
    "s_add_u32 s65, s65, 3\n" \
    "s_bitcmp1_b64 s[58:59], s75\n" \
    "s_cbranch_scc0 .Lfs_nadj_%=\n" \
    /* a ~ c: the one clique R + {bb, a, c} */ \
    "s_and_b64 s[84:85], s[52:53], s[58:59]\n" \
    "s_and_b64 s[84:85], s[84:85], s[78:79]\n" \
    "s_and_b64 s[62:63], s[62:63], s[54:55]\n" \
    "s_and_b64 s[62:63], s[62:63], s[82:83]\n" \
    "s_or_b64 s[84:85], s[84:85], s[62:63]\n" \
    "s_cmp_lg_u64 s[84:85], 0\n" \
    "s_cbranch_scc1 .Lfs_child_%=\n" \
    "s_add_u32 s60, s60, s80\n" \
    "s_addc_u32 s61, s61, s81\n" \
    "s_add_u32 s77, s77, 1\n" \
    "s_mov_b32 m0, s66\n" \
    "v_writelane_b32 v72, s60, m0\n" \
    "v_writelane_b32 v73, s61, m0\n" \
    "v_writelane_b32 v74, s77, m0\n" \
    "s_add_u32 s66, s66, 1\n" \
    "s_branch .Lfs_full_%=\n" \
    /* a, c not adjacent: leaves R + {bb, a} and R + {bb, c} */ \
    ".Lfs_nadj_%=:\n" \
    "s_and_b64 s[84:85], s[52:53], s[58:59]\n" \
    "s_and_b64 s[62:63], s[62:63], s[54:55]\n" \
    "s_or_b64 s[84:85], s[84:85], s[62:63]\n" \
    "s_cmp_lg_u64 s[84:85], 0\n" \
    "s_cbranch_scc1 .Lfs_nadj2_%=\n" \
    "s_mov_b32 m0, s66\n" \
    "v_writelane_b32 v72, s60, m0\n" \
    "v_writelane_b32 v73, s61, m0\n" \
    "v_writelane_b32 v74, s77, m0\n" \
    "s_add_u32 s66, s66, 1\n" \
    ".Lfs_nadj2_%=:\n" \
    "s_and_b64 s[84:85], s[52:53], s[78:79]\n" \
    "s_and_b64 s[82:83], s[82:83], s[54:55]\n" \
    "s_or_b64 s[84:85], s[84:85], s[82:83]\n" \
    "s_cmp_lg_u64 s[84:85], 0\n" \
    "s_cbranch_scc1 .Lfs_full_%=\n" \
    "s_add_u32 s80, s80, s56\n" \
    "s_addc_u32 s81, s81, s57\n" \
    "s_mov_b32 m0, s66\n" \
    "v_writelane_b32 v72, s80, m0\n" \
    "v_writelane_b32 v73, s81, m0\n" \
    "v_writelane_b32 v74, s77, m0\n" \
    "s_add_u32 s66, s66, 1\n" \
    /* at most two cliques per child: hash the group before it could overflow */ \
    ".Lfs_full_%=:\n" \
    "s_cmp_lt_u32 s66, 63\n" \
    "s_cbranch_scc1 .Lfs_child_%=\n" \
    "s_mov_b32 s67, 1\n" \
    "s_branch .Lfs_exit_%=\n" \
    ".Lfs_done_%=:\n" \
    "s_mov_b32 s67, 0\n" \
    ".Lfs_exit_%=:\n" \
    "s_mov_b32 m0, s76\n" \
    "s_nop 4\n"

template <bool kStream, bool kAsmSearch>
__device__ __forceinline__ void run_folded(const Params& p_arg, Wg& w, uint32_t root, const SmallJob& j)
{
    const Params& p = kparams();
    (void)p_arg;
    const uint32_t lane = lane_id();
    // wave-uniform inputs are made visibly uniform, so they stay in scalar registers
    const uint32_t m = uni(j.m), L = uni(j.L);
    const bool vx = lane < L;
    const uint32_t su = j.su;
    // per lane: the vertex key plus gamma, the increment of (key sum + |R| gamma)
    // when that vertex joins R
    const uint64_t skeyg = j.skey + kGamma, rowP = j.rowP;
    const uint32_t xrank = vx ? w.xr()[j.xj] : 0u;
    const uint64_t xrowP = L ? fold_xrow(w, vx, j.xj, j.oidx, m) : 0ull;
    uint64_t rowX = 0;
    for (uint32_t t = 0; t < L; ++t) {
        uint64_t wt = rl64(xrowP, t);
        if ((wt >> lane) & 1ull) rowX |= 1ull << t;
    }
    const uint32_t don_min = uni(w.don_min);
    const uint32_t rs0 = uni(j.rs);  // |R| at depth 0; |R| = rs0 + depth
    const bool anc0 = uni(j.anc ? 1u : 0u) != 0;
    uint64_t P = uni64(j.P), XP = uni64(j.XP), XX = low_mask(L), B = 0;
    uint64_t kg = uni64(j.ks) + (uint64_t)rs0 * kGamma;
    uint32_t depth = 0;  // < m <= 64: the stack fits one lane per level
    uint64_t sP = 0, sXP = 0, sXX = 0, sB = 0, sK = 0;
    // R[rs0 + d] for d < depth lives in lane d of sV; it is written to w.R() only
    // when a donation or the clique stream needs it
    uint32_t sV = 0;
    uint32_t nodes = 0, next_check = 4096;  // the watchdog is read every 4096 nodes
    LeafGroup lg;
    lg.pre = 0;
    lg.size = 0;
    lg.n = 0;
    lg.hsum = 0;
    // the current child (branch vertex lane bb, vertex vb) and its sets
    uint64_t Pc = 0, XPc = 0, XXc = 0, kgc = 0;
    uint32_t bb = 0, vb = 0;
    // clique-stream form: the cliques of one iteration (at most two), each as
    // key sum plus |C| gamma, the number of universe vertices beyond vb and
    // those vertices' lanes
    uint32_t ne = 0, ex0 = 0, ea0 = 0, eb0 = 0, ex1 = 0, ea1 = 0;
    uint64_t ek0 = 0, ek1 = 0;
    // at_node: the pivot step is due; push: before it, descend into the
    // current child
    bool at_node = true, push = false;
    if constexpr (kAsmSearch) {
        // The counting form of the six-wave launch runs the search loop below
        // as hand-scheduled assembly (FOLDED_SEARCH_ASM): the same steps in the
        // same order, with every loop-carried value in a fixed register.  It
        // offers no branch to the worker list (the donation threshold passed
        // to it is above any |P|): with offers taken from it, some received
        // frames failed validation, which is not understood; the six-wave
        // launch runs where every workgroup has hundreds of roots queued, and
        // the list and mid executors still donate.
        const uint64_t lbit = 1ull << lane;
        const uint32_t lk = 255u - lane, lkx = 191u - lane;
        const uint32_t sizeb = rs0 + 1;
        const uint32_t ancu = anc0 ? 1u : 0u;
        uint32_t mode = kAsmNode, npc = 0;
        while (true) {
            // the scalar operands are wave-uniform; the event handlers' per-lane
            // code hides that from the compiler, so it is restated here
            uint32_t ev = uni(mode);
            depth = uni(depth);
            nodes = uni(nodes);
            lg.n = uni(lg.n);
            bb = uni(bb);
            npc = uni(npc);
            next_check = uni(next_check);
            P = uni64(P);
            XP = uni64(XP);
            XX = uni64(XX);
            B = uni64(B);
            kg = uni64(kg);
            Pc = uni64(Pc);
            XPc = uni64(XPc);
            XXc = uni64(XXc);
            kgc = uni64(kgc);
            asm volatile(FOLDED_SEARCH_ASM
                         : "+{s[40:41]}"(P), "+{s[42:43]}"(XP), "+{s[44:45]}"(XX), "+{s[46:47]}"(B),
                           "+{s[48:49]}"(kg), "+{s[50:51]}"(Pc), "+{s[52:53]}"(XPc), "+{s[54:55]}"(XXc),
                           "+{s[56:57]}"(kgc), "+{s64}"(depth), "+{s65}"(nodes), "+{s66}"(lg.n), "+{s67}"(ev),
                           "+{s68}"(bb), "+{s69}"(npc), "+{v[62:63]}"(sP), "+{v[64:65]}"(sXP),
                           "+{v[66:67]}"(sXX), "+{v[68:69]}"(sB), "+{v[70:71]}"(sK), "+{v61}"(sV),
                           "+{v[72:73]}"(lg.pre), "+{v74}"(lg.size)
                         : "{s70}"(next_check), "{s71}"(kNoOffer), "{s72}"(sizeb), "{s73}"(ancu),
                           "{v[48:49]}"(rowP), "{v[50:51]}"(rowX), "{v[52:53]}"(skeyg), "{v[54:55]}"(xrowP),
                           "{v[56:57]}"(lbit), "{v58}"(su), "{v59}"(lk), "{v60}"(lkx)
                         : "scc", "vcc", "s58", "s59", "s60", "s61", "s62", "s63", "s74", "s75", "s76", "s77",
                           "s78", "s79", "s80", "s81", "s82", "s83", "s84", "s85", "v75", "v76", "v77", "v78");
            if (ev == kEvDone) {
                leaf_group_close(p, w, lg);
                w.nodes += nodes;
                return;
            }
            mode = kAsmChild;
            if (ev == kEvCheck) {
                next_check = nodes + 4096;
                if (check_deadline(p, w)) {
                    leaf_group_close(p, w, lg);
                    w.nodes += nodes;
                    return;
                }
            } else if (ev == kEvLeaves) {
                leaf_group_flush(p, w, lg);
            } else {
                // kEvOffer (not raised without a donation threshold): descend
                mode = kAsmDescend;
            }
        }
    }
    while (true) {
        uint32_t ev;
        while (true) {
            if (at_node) {
                if (nodes >= next_check) {
                    ev = kEvCheck;
                    break;
                }
                if (push) {
                    push = false;
                    sP = wlane64(sP, depth, P);
                    sXP = wlane64(sXP, depth, XP);
                    sXX = wlane64(sXX, depth, XX);
                    sB = wlane64(sB, depth, B);
                    sK = wlane64(sK, depth, kg);
                    sV = wlane32(sV, depth, vb);
                    ++depth;
                    P = Pc;
                    XP = XPc;
                    XX = XXc;
                    kg = kgc;
                }
                // ---- a node: Tomita pivot over P u X_P and the folded X_X
                at_node = false;
                ++nodes;
                const uint64_t cp = P | XP;
                uint32_t key = ((cp >> lane) & 1ull) ? (((uint32_t)__popcll(P & rowP) << 8) | (255u - lane)) : 0u;
                // X_X is often empty deep in the tree: skip its scores then
                const uint32_t kx =
                    XX && ((XX >> lane) & 1ull) ? (((uint32_t)__popcll(P & xrowP) << 8) | (191u - lane)) : 0u;
                const uint32_t best = wave_max(max(key, kx));
                const uint32_t idx = 255u - (best & 255u);
                const uint64_t rowpiv = idx < 64 ? rl64(rowP, idx) : rl64(xrowP, idx - 64);
                B = P & ~rowpiv;
            }
            // ---- the node's children, in ascending lane order; returns land here too
            if (B == 0) {
                if (depth == 0) {
                    ev = kEvDone;
                    break;
                }
                --depth;
                P = rl64(sP, depth);
                XP = rl64(sXP, depth);
                XX = rl64(sXX, depth);
                B = rl64(sB, depth);
                kg = rl64(sK, depth);
                continue;
            }
            bb = (uint32_t)__builtin_ctzll(B);
            const uint64_t bit = 1ull << bb;
            B &= ~bit;
            const uint64_t rp = rl64(rowP, bb);
            Pc = P & rp;
            XPc = XP & rp;
            XXc = XX ? XX & rl64(rowX, bb) : 0ull;
            P &= ~bit;
            XP |= bit;
            kgc = kg + rl64(skeyg, bb);
            // a maximal clique R + {vb} + the `extra` universe vertices e1, e2,
            // with key sum plus |R| gamma kfull
            auto emit = [&](uint64_t kfull, uint32_t extra, uint32_t e1, uint32_t e2) {
                if (kStream) {
                    if (ne == 0) {
                        ek0 = kfull;
                        ex0 = extra;
                        ea0 = e1;
                        eb0 = e2;
                    } else {
                        ek1 = kfull;
                        ex1 = extra;
                        ea1 = e1;
                    }
                    ++ne;
                } else {
                    lg.pre = wlane64(lg.pre, lg.n, kfull);
                    lg.size = wlane32(lg.size, lg.n, rs0 + depth + 1 + extra);
                    ++lg.n;
                }
            };
            if (Pc == 0) {
                ++nodes;
                if ((XPc | XXc) == 0) emit(kgc, 0, 0, 0);
            } else {
                // (readfirstlane keeps the small-P tests 32-bit scalar compares)
                const uint32_t npc = uni((uint32_t)__popcll(Pc));
                if (npc > 2) {
                    vb = rl32(su, bb);
                    if (npc >= don_min && donation_wanted(p, w, npc, B != 0, anc0 || depth > 0, depth)) {
                        ev = kEvOffer;
                        break;
                    }
                    at_node = push = true;
                    continue;
                }
                // the child's P has one or two vertices: it pivots on its first
                // vertex a without scoring (any pivot in P u X is valid), and its
                // subtree is finished here: with P = {a}, or P = {a, c} and a ~ c,
                // the one branch a (then c); with a and c non-adjacent, the
                // branches a and c, each a leaf
                const uint32_t a = (uint32_t)__builtin_ctzll(Pc);
                const uint64_t ra = rl64(rowP, a), xa = XXc ? rl64(rowX, a) : 0ull;
                const uint64_t ka = kgc + rl64(skeyg, a);
                if (npc == 1) {
                    nodes += 2;
                    if (((XPc & ra) | (XXc & xa)) == 0) emit(ka, 1, a, 0);
                } else {
                    const uint32_t c = (uint32_t)__builtin_ctzll(Pc & ~(1ull << a));
                    const uint64_t rc = rl64(rowP, c), xc = XXc ? rl64(rowX, c) : 0ull;
                    const uint64_t kc = rl64(skeyg, c);
                    nodes += 3;
                    if ((ra >> c) & 1ull) {
                        if (((XPc & ra & rc) | (XXc & xa & xc)) == 0) emit(ka + kc, 2, a, c);
                    } else {
                        if (((XPc & ra) | (XXc & xa)) == 0) emit(ka, 1, a, 0);
                        if (((XPc & rc) | (XXc & xc)) == 0) emit(kgc + kc, 1, c, 0);
                    }
                }
            }
            // an iteration adds at most two cliques: the group is hashed
            // before it could overflow
            if (kStream ? ne != 0 : lg.n >= 63) {
                ev = kEvLeaves;
                break;
            }
        }
        // ---- events (wave-divergent work).  The event code is hidden from the
        // optimiser, so the exits of the loop above meet in this one block
        // rather than each being threaded to its own handler.
        asm volatile("" : "+s"(ev));
        if (ev == kEvDone) {
            leaf_group_close(p, w, lg);
            w.nodes += nodes;
            return;
        }
        if (ev == kEvCheck) {
            next_check = nodes + 4096;
            if (check_deadline(p, w)) {
                leaf_group_close(p, w, lg);
                w.nodes += nodes;
                return;
            }
        } else if (ev == kEvLeaves) {
            if (kStream) {
                if (lane < depth) w.R()[rs0 + lane] = sV;
                for (uint32_t e = 0; e < ne; ++e) {
                    const uint32_t extra = e ? ex1 : ex0;
                    const uint32_t rsize = rs0 + depth + 1 + extra;
                    if (lane == 0) {
                        w.R()[rs0 + depth] = rl32(su, bb);
                        if (extra > 0) w.R()[rs0 + depth + 1] = rl32(su, e ? ea1 : ea0);
                        if (extra > 1) w.R()[rs0 + depth + 2] = rl32(su, eb0);
                    }
                    wave_mem_sync();
                    report(p, w, rsize, (e ? ek1 : ek0) - (uint64_t)rsize * kGamma);
                }
                ne = 0;
            } else {
                leaf_group_flush(p, w, lg);
            }
        } else {
            // kEvOffer: an idle workgroup takes the child, or it is descended into
            const uint32_t r = wl_try_pop(p, w);
            if (r != kNoWorkgroup) {
                // the child keeps this universe and the members of X_X
                Wg d = wg_view(p, r);
                put_fold_frame(d, m, Pc, XPc, su, skeyg - kGamma, rowP, ((XXc >> lane) & 1ull) != 0, prefix_popc(XXc),
                               xrank, xrowP);
                if (lane < depth) w.R()[rs0 + lane] = sV;
                wave_mem_sync();
                const uint32_t rs = rs0 + depth;
                publish_task(p, w, r, root, rs, vb, kgc - (uint64_t)(rs + 1) * kGamma, m, 0, (uint32_t)__popcll(XXc),
                             kMboxFold);
            } else {
                at_node = push = true;
            }
        }
    }
}

// ---------------------------------------------------------------- list executor
// Universe of m <= 64 vertices in registers (the job's per-lane fields, which
// stay untouched while a folded child runs); X_X stays the index list.
// (c, C): at depth 0 descend only into branches t with t % C == c.  Returns
// kYieldFold with j updated to a child for the folded executor, or kDone.
__device__ __forceinline__ uint32_t run_list(const Params& p_arg, Wg& w, uint32_t root, bool resume, SmallJob& j,
                                             uint32_t c, uint32_t C)
{
    const Params& p = kparams();
    (void)p_arg;
    const uint32_t lane = lane_id();
    const uint32_t m = j.m;
    const bool valid = lane < m;
    const bool can_fold = w.have_xrows;
    const uint32_t su = j.su, oidx = j.oidx;
    const uint64_t skey = j.skey, rowP = j.rowP;
    uint32_t depth, t0, rs, L;
    uint64_t P, XP, ks, B;
    bool anc;
    // register stack (lane d = level d < m <= 64); spilled to LDS while a
    // folded child runs.  R[rs0 + d] for d < depth lives in lane d of sV and is
    // written to w.R() only for a donation, the clique stream or a suspension.
    uint64_t sP, sXP, sB, sK;
    uint32_t sL, sA, sR, sV, rs0;
    // one natural loop: a node's pivot step runs at the top of the iteration
    // after a descent; resuming pops the suspended level first
    bool pop_first = resume, at_node = !resume;
    if (resume) {
        depth = S.frame[2];
        t0 = S.frame[3];
        rs = L = 0;
        P = XP = ks = B = 0;
        anc = false;
        sP = w.susp64()[lane];
        sXP = w.susp64()[64 + lane];
        sB = w.susp64()[128 + lane];
        sK = w.susp64()[192 + lane];
        sL = w.susp32()[lane];
        sA = w.susp32()[64 + lane];
        sR = w.susp32()[128 + lane];
        rs0 = S.frame[4];
        sV = lane < depth ? w.R()[rs0 + lane] : 0u;
    } else {
        sP = sXP = sB = sK = 0;
        sL = sA = sR = sV = 0;
        rs0 = j.rs;
        depth = 0;
        t0 = 0;
        rs = j.rs;
        L = j.L;
        P = j.P;
        XP = j.XP;
        ks = j.ks;
        anc = j.anc;
        B = 0;
    }
    while (true) {
        if (at_node) {
            at_node = false;
            ++w.nodes;
            uint64_t cp = P | XP;
            uint32_t key = 0;
            if (valid && ((cp >> lane) & 1ull)) key = ((uint32_t)__popcll(P & rowP) << 8) | (255u - lane);
            uint32_t best = wave_max(key);
            uint32_t piv = 255u - (best & 255u);
            B = P & ~rl64(rowP, piv);
        }
        if (pop_first || B == 0) {
            if (depth == 0) return kDone;
            pop_first = false;
            --depth;
            P = rl64(sP, depth);
            XP = rl64(sXP, depth);
            B = rl64(sB, depth);
            ks = rl64(sK, depth);
            L = rl32(sL, depth);
            anc = rl32(sA, depth) != 0;
            rs = rl32(sR, depth);
            continue;
        }
        if ((++w.poll & 1023u) == 0 && check_deadline(p, w)) return kDone;
        uint32_t bb = (uint32_t)__builtin_ctzll(B);
        B &= B - 1;
        uint64_t rp = rl64(rowP, bb);
        uint64_t Pc = P & rp;
        uint64_t XPc = XP & rp;
        P &= ~(1ull << bb);
        XP |= 1ull << bb;
        if (depth == 0 && C > 1) {
            if ((t0++ % C) != c) continue;
        }
        uint32_t vb = rl32(su, bb);
        uint32_t bidx = rl32(oidx, bb);
        uint64_t ksc = ks + rl64(skey, bb);
        if (Pc == 0) {
            ++w.nodes;
            if (XPc == 0 && !xx_any(p, w, L, bidx, vb)) {
                if (p.flags & MCE_F_STREAM) {
                    if (lane < depth) w.R()[rs0 + lane] = sV;
                    if (lane == 0) w.R()[rs] = vb;
                    wave_mem_sync();
                }
                report(p, w, rs + 1, ksc);
            }
            continue;
        }
        uint32_t Lc = xx_partition(p, w, L, bidx, vb);
        uint32_t npc = (uint32_t)__popcll(Pc);
        if (donation_wanted(p, w, npc, B != 0, anc || depth > 0, depth)) {
            uint32_t r = wl_try_pop(p, w);
            if (r != kNoWorkgroup) {
                Wg d = wg_view(p, r);
                if (lane < depth) w.R()[rs0 + lane] = sV;
                if (Lc <= 64 && (can_fold || Lc == 0)) {
                    // fold frame over this universe; X_X members' rows gathered from the X rows
                    wave_mem_sync();
                    const bool xin = lane < Lc;
                    const uint32_t xj = xin ? w.xx()[lane] : 0u;
                    const uint64_t xrowP = Lc ? fold_xrow(w, xin, xj, oidx, m) : 0ull;
                    put_fold_frame(d, m, Pc, XPc, su, skey, rowP, xin, lane, xin ? w.xr()[xj] : 0u, xrowP);
                    wave_mem_sync();
                    publish_task(p, w, r, root, rs, vb, ksc, m, 0, Lc, kMboxFold);
                    continue;
                }
                if (valid && ((Pc >> lane) & 1ull)) d.mP()[prefix_popc(Pc)] = su;
                if (valid && ((XPc >> lane) & 1ull)) d.mXP()[prefix_popc(XPc)] = su;
                for (uint32_t i = lane; i < Lc; i += 64) d.xr()[i] = w.xr()[w.xx()[i]];
                wave_mem_sync();
                publish_task(p, w, r, root, rs, vb, ksc, npc, (uint32_t)__popcll(XPc), Lc, kMboxLists);
                continue;
            }
        }
        sV = wl32(sV, depth, vb);
        sP = wl64(sP, depth, P);
        sXP = wl64(sXP, depth, XP);
        sB = wl64(sB, depth, B);
        sK = wl64(sK, depth, ks);
        sL = wl32(sL, depth, L);
        sA = wl32(sA, depth, anc ? 1u : 0u);
        sR = wl32(sR, depth, rs);
        const bool canc = anc || (B != 0);
        ++depth;
        if (Lc <= 64 && (can_fold || Lc == 0)) {
            // suspend: the folded child runs next, then this level is popped
            wave_mem_sync();
            j.xj = lane < Lc ? w.xx()[lane] : 0u;
            j.P = Pc;
            j.XP = XPc;
            j.L = Lc;
            j.ks = ksc;
            j.rs = rs + 1;
            j.anc = canc;
            w.susp64()[lane] = sP;
            w.susp64()[64 + lane] = sXP;
            w.susp64()[128 + lane] = sB;
            w.susp64()[192 + lane] = sK;
            w.susp32()[lane] = sL;
            w.susp32()[64 + lane] = sA;
            w.susp32()[128 + lane] = sR;
            // the folded child reads R[0, rs + 1) from memory when it donates
            if (lane < depth) w.R()[rs0 + lane] = sV;
            if (lane == 0) {
                S.frame[2] = depth;
                S.frame[3] = t0;
                S.frame[4] = rs0;
            }
            wave_mem_sync();
            return kYieldFold;
        }
        anc = canc;
        ++rs;
        P = Pc;
        XP = XPc;
        L = Lc;
        ks = ksc;
        at_node = true;
    }
}

// ---------------------------------------------------------------- mid executor
// Members of a bitmap X_X (lane-per-word, w.Wx words) as indices into xr, in
// ascending order.  to_list: written to w.xx()[0, count); otherwise (count <= 64)
// lane j returns the j-th member.
__device__ __forceinline__ uint32_t xx_members(Wg& w, uint64_t XX, bool to_list)
{
    const uint32_t lane = lane_id();
    const uint32_t Wx = w.Wx;
    uint32_t base = 0;
    for (uint32_t t = 0; t < Wx; ++t) {
        uint64_t word = rl64(XX, t);
        if ((word >> lane) & 1ull) {
            uint32_t pos = base + prefix_popc(word);
            if (to_list) w.xx()[pos] = t * 64 + lane;
            else S.sxj[pos] = t * 64 + lane;
        }
        base += (uint32_t)__popcll(word);
    }
    wave_mem_sync();
    return (!to_list && lane < base) ? S.sxj[lane] : 0u;
}

// A child whose P u X_P (masks Pc, XPc over the task universe) has at most
// 64 vertices, re-indexed: lane k < msz holds task-universe vertex o (the
// members in ascending order) and its row over the small universe.
struct SmallView {
    uint32_t msz, o;
    uint64_t row, P, XP;
};

__device__ __forceinline__ SmallView compact_child(const uint64_t* rows, uint32_t ws, uint32_t W, uint64_t Pc,
                                                   uint64_t XPc)
{
    const uint32_t lane = lane_id();
    SmallView v;
    uint64_t cand = lane < W ? (Pc | XPc) : 0ull;
    uint32_t cnt = (uint32_t)__popcll(cand);
    uint32_t pre = wave_excl_scan(cnt);
    v.msz = wave_sum(cnt);
    uint64_t cc = cand;
    uint32_t tt = pre;
    while (cc) {
        uint32_t bt = (uint32_t)__builtin_ctzll(cc);
        cc &= cc - 1;
        S.sidx[tt++] = lane * 64 + bt;
    }
    wave_mem_sync();
    const bool valid = lane < v.msz;
    v.o = valid ? S.sidx[lane] : 0u;
    // local row of vertex k: bit k2 set iff o_k and o_k2 are adjacent; the
    // sorted o_k2 visit each source word once, so each word is loaded once
    uint64_t row = 0;
    const uint64_t* ro = rows + (uint64_t)v.o * ws;
    uint32_t k2 = 0;
    while (k2 < v.msz) {
        uint32_t q = S.sidx[k2] >> 6;
        uint64_t wq = valid ? ro[q] : 0ull;
        for (; k2 < v.msz; ++k2) {
            uint32_t o2 = S.sidx[k2];
            if ((o2 >> 6) != q) break;
            row |= ((wq >> (o2 & 63)) & 1ull) << k2;
        }
    }
    v.row = row;
    uint64_t pword = shfl64(Pc, v.o >> 6);
    uint64_t xword = shfl64(XPc, v.o >> 6);
    v.P = __ballot(valid && ((pword >> (v.o & 63)) & 1ull));
    v.XP = __ballot(valid && ((xword >> (v.o & 63)) & 1ull));
    return v;
}

// Universe of up to 4096 vertices, one 64-bit word per lane (W words).  The
// pivot maximises |P n N(u)| over u in P u X_P (Section III-E).  X_X is either
// a bitmap over the task's X list (lanes hold its Wx words; a child's X_X is
// one AND with the X column of the branch vertex) or, when the X columns were
// not built, the partitioned index list of Section III-E.  The DFS stack lives
// in this workgroup's HBM scratch.  A child whose P u X_P fits 64 vertices is
// re-indexed into j and handed over (kYieldFold / kYieldList).
__device__ __forceinline__ uint32_t run_mid(const Params& p_arg, Wg& w, uint32_t root, uint32_t nu, const uint64_t* rows,
                                            uint32_t ws, bool resume, SmallJob& j, uint32_t L0, uint32_t c,
                                            uint32_t C)
{
    const Params& p = kparams();
    (void)p_arg;
    const uint32_t lane = lane_id();
    const uint32_t W = w.W;
    const bool xb = w.have_xrows;
    const uint32_t Wx = xb ? w.Wx : 0u;
    const uint32_t gws = p.wg;
    const uint32_t lvl_words = 3 * gws + p.wgx;
    const uint32_t* U = w.uarr();
    uint32_t depth, t0, rs, L;
    uint64_t P, XP, XX, B, ks;
    bool anc;
    // one natural loop: a node's pivot step runs at the top of the iteration
    // after a descent; resuming pops the suspended level first
    bool pop_first = resume, at_node = !resume;
    if (resume) {
        depth = S.frame[0];
        t0 = S.frame[1];
        rs = L = 0;
        P = XP = XX = B = ks = 0;
        anc = false;
    } else {
        depth = 0;
        t0 = 0;
        rs = j.rs;
        L = L0;
        ks = j.ks;
        anc = false;
        P = lane < W ? S.pw[lane] : 0ull;
        XP = lane < W ? S.xw[lane] : 0ull;
        XX = lane < Wx ? low_mask(L - lane * 64) : 0ull;
        B = 0;
    }
    while (true) {
        if (at_node) {
            at_node = false;
            ++w.nodes;
            uint32_t best = 0;
            uint64_t cand = P | XP;
            for (uint32_t t = 0; t < W; ++t) {
                uint64_t cw = rl64(cand, t);
                if (cw == 0) continue;
                uint32_t i = t * 64 + lane;
                if ((cw >> lane) & 1ull) {
                    uint32_t sc = 0;
                    const uint64_t* ri = rows + (uint64_t)i * ws;
                    // eight row words per round trip: all loads issue before the first use
                    for (uint32_t q = 0; q < W; q += 8) {
                        uint64_t r[8];
#pragma unroll
                        for (uint32_t k = 0; k < 8; ++k) r[k] = q + k < W ? ri[q + k] : 0ull;
#pragma unroll
                        for (uint32_t k = 0; k < 8; ++k) sc += (uint32_t)__popcll(rl64(P, (q + k) & 63u) & r[k]);
                    }
                    best = max(best, (sc << 13) | (8191u - i));
                }
            }
            best = wave_max(best);
            uint32_t piv = 8191u - (best & 8191u);
            B = lane < W ? (P & ~rows[(uint64_t)piv * ws + lane]) : 0ull;
        }
        uint64_t bm = pop_first ? 0ull : __ballot(B != 0);
        if (bm == 0) {
            if (depth == 0) return kDone;
            pop_first = false;
            --depth;
            const uint64_t* lvl = w.gstack() + (uint64_t)depth * lvl_words;
            if (lane < W) {
                P = lvl[lane];
                XP = lvl[gws + lane];
                B = lvl[2 * gws + lane];
            }
            if (lane < Wx) XX = lvl[3 * gws + lane];
            uint64_t meta = w.gmeta()[3 * depth];
            ks = w.gmeta()[3 * depth + 1];
            rs = (uint32_t)w.gmeta()[3 * depth + 2];
            L = (uint32_t)meta;
            anc = (meta >> 32) != 0;
            continue;
        }
        if ((++w.poll & 255u) == 0 && check_deadline(p, w)) return kDone;
        uint32_t w0 = (uint32_t)__builtin_ctzll(bm);
        uint64_t word = rl64(B, w0);
        uint32_t bit = (uint32_t)__builtin_ctzll(word);
        uint32_t bb = w0 * 64 + bit;
        uint64_t rowb = lane < W ? rows[(uint64_t)bb * ws + lane] : 0ull;
        uint64_t colb = lane < Wx ? w.xcols()[(uint64_t)bb * Wx + lane] : 0ull;
        uint64_t Pc = P & rowb;
        uint64_t XPc = XP & rowb;
        uint64_t XXc = XX & colb;
        if (lane == w0) {
            B &= ~(1ull << bit);
            P &= ~(1ull << bit);
            XP |= 1ull << bit;
        }
        if (depth == 0 && C > 1) {
            if ((t0++ % C) != c) continue;
        }
        uint32_t vb = U[bb];
        uint64_t ksc = ks + w.ukey()[bb];
        uint32_t npc = wave_sum((uint32_t)__popcll(Pc));
        uint32_t nxc = wave_sum((uint32_t)__popcll(XPc));
        bool more_here = __ballot(B != 0) != 0;
        if (npc == 0) {
            ++w.nodes;
            bool xhit = xb ? __ballot(XXc != 0) != 0 : (nxc == 0 && xx_any(p, w, L, bb, vb));
            if (nxc == 0 && !xhit) {
                if (p.flags & MCE_F_STREAM) {
                    if (lane == 0) w.R()[rs] = vb;
                    wave_mem_sync();
                }
                report(p, w, rs + 1, ksc);
            }
            continue;
        }
        uint32_t Lc;
        if (xb) {
            Lc = wave_sum((uint32_t)__popcll(XXc));
            stat_add(S_XCOLW, Wx);
        } else {
            Lc = xx_partition(p, w, L, bb, vb);
        }
        if (donation_wanted(p, w, npc, more_here, anc || depth > 0, depth)) {
            uint32_t r = wl_try_pop(p, w);
            if (r != kNoWorkgroup) {
                Wg d = wg_view(p, r);
                if (npc + nxc <= 64 && (xb ? Lc <= 64 : Lc == 0)) {
                    // fold frame: the child re-indexed as for a hand-over to the folded executor
                    const SmallView cv = compact_child(rows, ws, W, Pc, XPc);
                    const bool valid = lane < cv.msz, xin = lane < Lc;
                    uint32_t xj = 0;
                    uint64_t xrowP = 0;
                    if (Lc) {
                        xj = xx_members(w, XXc, false);
                        xrowP = fold_xrow(w, xin, xj, cv.o, cv.msz);
                    }
                    put_fold_frame(d, cv.msz, cv.P, cv.XP, valid ? U[cv.o] : 0u, valid ? w.ukey()[cv.o] : 0ull, cv.row,
                                   xin, lane, xin ? w.xr()[xj] : 0u, xrowP);
                    wave_mem_sync();
                    publish_task(p, w, r, root, rs, vb, ksc, cv.msz, 0, Lc, kMboxFold);
                    continue;
                }
                uint32_t bp = 0, bx = 0;
                for (uint32_t t = 0; t < W; ++t) {
                    uint64_t pw_ = rl64(Pc, t), xw_ = rl64(XPc, t);
                    uint32_t u = t * 64 + lane;
                    if ((pw_ >> lane) & 1ull) d.mP()[bp + prefix_popc(pw_)] = U[u];
                    if ((xw_ >> lane) & 1ull) d.mXP()[bx + prefix_popc(xw_)] = U[u];
                    bp += (uint32_t)__popcll(pw_);
                    bx += (uint32_t)__popcll(xw_);
                }
                if (xb) {
                    uint32_t bq = 0;
                    for (uint32_t t = 0; t < Wx; ++t) {
                        uint64_t xxw = rl64(XXc, t);
                        if ((xxw >> lane) & 1ull) d.xr()[bq + prefix_popc(xxw)] = w.xr()[t * 64 + lane];
                        bq += (uint32_t)__popcll(xxw);
                    }
                } else {
                    for (uint32_t i = lane; i < Lc; i += 64) d.xr()[i] = w.xr()[w.xx()[i]];
                }
                publish_task(p, w, r, root, rs, vb, ksc, npc, nxc, Lc, kMboxLists);
                continue;
            }
        }
        // push this level (also when the child is handed to a smaller executor)
        uint64_t* lvl = w.gstack() + (uint64_t)depth * lvl_words;
        if (lane < W) {
            lvl[lane] = P;
            lvl[gws + lane] = XP;
            lvl[2 * gws + lane] = B;
        }
        if (lane < Wx) lvl[3 * gws + lane] = XX;
        // every lane stores the same meta words, so each later reads its own store
        w.gmeta()[3 * depth] = ((uint64_t)(anc ? 1u : 0u) << 32) | L;
        w.gmeta()[3 * depth + 1] = ks;
        w.gmeta()[3 * depth + 2] = rs;
        if (lane == 0) w.R()[rs] = vb;
        const bool canc = anc || more_here || depth > 0;
        ++depth;
        if (npc + nxc <= 64) {
            // re-index the child's P u X_P (at most 64 vertices) into registers
            const SmallView cv = compact_child(rows, ws, W, Pc, XPc);
            const bool valid = lane < cv.msz;
            j.m = cv.msz;
            j.su = valid ? U[cv.o] : 0u;
            j.skey = valid ? w.ukey()[cv.o] : 0ull;
            j.oidx = cv.o;
            j.rowP = cv.row;
            j.P = cv.P;
            j.XP = cv.XP;
            j.L = Lc;
            j.ks = ksc;
            j.rs = rs + 1;
            j.anc = canc;
            if (lane == 0) {
                S.frame[0] = depth;
                S.frame[1] = t0;
            }
            wave_mem_sync();
            if (xb) {
                // X_X is a bitmap over the task's X list: fold its members, or list them
                j.xj = xx_members(w, XXc, Lc > 64);
                return Lc <= 64 ? kYieldFold : kYieldList;
            }
            j.xj = 0;
            return Lc == 0 ? kYieldFold : kYieldList;
        }
        anc = canc;
        ++rs;
        P = Pc;
        XP = XPc;
        XX = XXc;
        L = Lc;
        ks = ksc;
        at_node = true;
    }
}

// ---------------------------------------------------------------- bitmap construction
// For every list entry i < cnt (mode 0: U[i]; mode 1: xr[i]) scan its later
// neighbours and, for each one found in U[0, nu) at position j, set bit j of
// row i (mode 0 also sets bit i of row j: the P x P rows are symmetric; mode 1
// with cols also sets bit i of column j).  All
// 64 lanes take consecutive entries of the concatenated lists, so loads are
// independent and lanes stay busy across short lists.
// Entry r of the scanned list (row r) has universe vertex a as a later neighbour.
__device__ __forceinline__ void set_pair(uint64_t* rows, uint64_t* cols, int mode, uint32_t r, uint32_t a, uint32_t ws,
                                         uint32_t cws)
{
    atomicOr((unsigned long long*)&rows[(uint64_t)r * ws + (a >> 6)], 1ull << (a & 63));
    if (mode == 0)
        atomicOr((unsigned long long*)&rows[(uint64_t)a * ws + (r >> 6)], 1ull << (r & 63));
    else if (cols)
        atomicOr((unsigned long long*)&cols[(uint64_t)a * cws + (r >> 6)], 1ull << (r & 63));
}

__device__ __forceinline__ void scan_lists(const Params& p_arg, Wg& w, int mode, uint32_t cnt, uint32_t nu, uint64_t* rows,
                                           uint32_t ws, uint64_t* cols, uint32_t cws)
{
    const Params& p = kparams();
    (void)p_arg;
    const uint32_t lane = lane_id();
    const uint32_t* U = w.uarr();
    if (nu == 0) return;  // no entry can be found in an empty universe
    const uint32_t umin = U[0], umax = U[nu - 1];
    const uint32_t ustep = 1u << (31 - __builtin_clz(nu));  // largest power of two <= nu
    for (uint32_t g0 = 0; g0 < cnt; g0 += 64) {
        uint32_t i = g0 + lane;
        uint32_t beg = 0, len = 0;
        if (i < cnt) {
            uint32_t v = mode == 0 ? U[i] : w.xr()[i];
            beg = p.op[v];
            len = p.op[v + 1] - beg;
        }
        uint32_t off = wave_excl_scan(len);
        uint32_t total = wave_sum(len);
        S.soff[lane] = off;
        S.sbeg[lane] = beg;
        wave_mem_sync();
        stat_add(S_EDGES, total);
        const uint32_t nrows = min(64u, cnt - g0);
        // two entries per lane and step (f and f + 64), so the two dependent
        // chains of LDS searches and the list load overlap; the searches are
        // binary liftings with the same trip count in every lane
        for (uint32_t t = 0; t < total; t += 128) {
            const uint32_t fA = t + lane, fB = fA + 64;
            const bool okA = fA < total, okB = fB < total;
            uint32_t rA = 0, rB = 0;  // last row with soff <= f
            for (uint32_t step = 32; step; step >>= 1) {
                if (rA + step < nrows && S.soff[rA + step] <= fA) rA += step;
                if (rB + step < nrows && S.soff[rB + step] <= fB) rB += step;
            }
            const uint32_t xA = okA ? p.oc[S.sbeg[rA] + (fA - S.soff[rA])] : 0u;
            const uint32_t xB = okB ? p.oc[S.sbeg[rB] + (fB - S.soff[rB])] : 0u;
            const bool inA = okA && xA >= umin && xA <= umax;
            const bool inB = okB && xB >= umin && xB <= umax;
            if (inA || inB) {
                uint32_t aA = 0, aB = 0;  // entries of U below x
                for (uint32_t step = ustep; step; step >>= 1) {
                    if (aA + step <= nu && U[aA + step - 1] < xA) aA += step;
                    if (aB + step <= nu && U[aB + step - 1] < xB) aB += step;
                }
                if (inA && aA < nu && U[aA] == xA) set_pair(rows, cols, mode, g0 + rA, aA, ws, cws);
                if (inB && aB < nu && U[aB] == xB) set_pair(rows, cols, mode, g0 + rB, aB, ws, cws);
            }
        }
        wave_mem_sync();
    }
}

// ---------------------------------------------------------------- tasks
__device__ __forceinline__ void begin_task(const Params& p_arg, Wg& w, uint32_t root)
{
    const Params& p = kparams();
    (void)p_arg;
    uint32_t g = p.gid ? uni(p.gid[root]) : 0u;
    if (g != w.cur_gid) {
        flush_graph(p, w);
        w.cur_gid = g;
    }
    if (__lane_id() == 0) {
        S.stat[S_CTASK] = 0;
        S.stat[S_HTASK] = 0;
        S.stat[S_COUNT + 1] = S.stat[S_DONATIONS];
        S.stat[S_COUNT + 2] = S.stat[S_BUILD];
    }
    w.task_t0 = uni64(now_ticks());
    w.nodes_t0 = w.nodes;
}

__device__ __forceinline__ void finish_task(const Params& p_arg, Wg& w, uint32_t root, uint32_t nu, uint32_t L, uint32_t rs, uint32_t c,
                            uint32_t C)
{
    const Params& p = kparams();
    (void)p_arg;
    stat_add(S_TASKS, 1);
    // keep the per-size LDS counters (32-bit) far from overflow
    if (w.count > (1ull << 30)) flush_graph(p, w);
    uint64_t dt = uni64(now_ticks()) - w.task_t0;
    if (lane_id() == 0) {
        S.stat[S_BUSY] += dt;
        S.stat[S_MAXTASK] = max(S.stat[S_MAXTASK], dt);
        if (p.flags & MCE_F_ROOT_STATS) {
            uint32_t id = p.perm[root];
            atomicAdd(&p.root_count[id], (unsigned long long)S.stat[S_CTASK]);
            atomicAdd(&p.root_hash[id], (unsigned long long)S.stat[S_HTASK]);
            atomicAdd(&p.root_nodes[id], (unsigned long long)(w.nodes - w.nodes_t0));
        }
        if ((p.flags & MCE_F_TASK_LOG) && dt >= p.tlog_min_ticks) {
            uint32_t slot = atomicAdd(&p.ctrl->tlog_n, 1u);
            if (slot < p.tlog_cap) {
                unsigned long long* e = p.tlog + (uint64_t)slot * 8;
                e[0] = p.perm[root];
                e[1] = ((unsigned long long)rs << 32) | nu;
                e[2] = ((unsigned long long)c << 48) | ((unsigned long long)C << 32) | L;
                e[3] = w.nodes - w.nodes_t0;
                e[4] = dt * 10;  // 100 MHz clock -> ns
                e[5] = (S.stat[S_BUILD] - S.stat[S_COUNT + 2]) * 10;
                e[6] = S.stat[S_DONATIONS] - S.stat[S_COUNT + 1];
                e[7] = ((unsigned long long)w.me << 48) | ((w.task_t0 * 10) & 0xFFFFFFFFFFFFull);
            }
        }
    }
}

// Bitmaps of a task whose universe U (ascending ranks) is in w.uarr()[0, nu),
// with P and X_P as bitmasks in S.pw / S.xw and the initial X_X ranks in
// w.xr()[0, L): universe rows (LDS, or HBM beyond the LDS cap) and, within the
// X budgets, X rows and X columns.  Returns the first executor; a universe of
// at most 64 vertices is set up in j.
__device__ __forceinline__ uint32_t build_task(const Params& p_arg, Wg& w, uint32_t nu, uint32_t L, uint64_t ks,
                                               uint32_t rs, uint32_t C, SmallJob& j, const uint64_t*& rows,
                                               uint32_t& ws)
{
    const Params& p = kparams();
    (void)p_arg;
    const uint32_t lane = lane_id();
    const uint32_t W = (nu + 63) >> 6;
    const uint64_t tb0 = now_ticks();
    w.W = W;
    for (uint32_t i = lane; i < nu; i += 64) w.ukey()[i] = p.vkey[w.uarr()[i]];
    for (uint32_t i = lane; i < L; i += 64) w.xx()[i] = i;
    const uint32_t Wx = (L + 63) >> 6;
    w.have_xrows = L > 0 && nu >= p.xrow_min_u && (uint64_t)L * W <= p.xrow_budget &&
                   (uint64_t)nu * Wx <= p.xcol_budget && Wx <= p.wgx && L <= p.xrow_ratio * max(nu, 64u);
    w.Wx = w.have_xrows ? Wx : 0u;
    if (w.have_xrows) {
        // X rows (per X entry, over U) for the register executors; X columns
        // (per universe vertex, over X) for the mid executor
        const bool cols = nu > 64;
        for (uint64_t i = lane; i < (uint64_t)L * W; i += 64) w.xrows()[i] = 0;
        if (cols)
            for (uint64_t i = lane; i < (uint64_t)nu * Wx; i += 64) w.xcols()[i] = 0;
        wave_mem_sync();
        scan_lists(p, w, 1, L, nu, w.xrows(), W, cols ? w.xcols() : nullptr, Wx);
        stat_add(S_XROW, 1);
    }
    uint64_t* brows;
    if (nu <= 64) {
        brows = w.lrows();
        ws = 1;
    } else if (nu <= p.lds_cap) {
        brows = w.lrows();
        ws = W | 1u;
    } else {
        brows = w.grows();
        ws = W | 1u;
        stat_add(S_HBM, 1);
    }
    rows = brows;
    for (uint32_t i = lane; i < nu * ws; i += 64) brows[i] = 0;
    wave_mem_sync();
    scan_lists(p, w, 0, nu, nu, brows, ws, nullptr, 0);
    stat_add(S_BUILD, now_ticks() - tb0);
    j.ks = ks;
    j.rs = rs;
    j.anc = false;
    if (nu > 64) return kExMid;
    const bool valid = lane < nu;
    j.m = nu;
    j.su = valid ? w.uarr()[lane] : 0u;
    j.skey = valid ? w.ukey()[lane] : 0ull;
    j.oidx = lane;
    j.rowP = valid ? brows[lane] : 0ull;
    j.P = S.pw[0];
    j.XP = S.xw[0];
    j.L = L;
    j.xj = lane;  // xx[i] = i at the start of a task
    wave_mem_sync();
    return (C == 1 && L <= 64 && (w.have_xrows || L == 0)) ? kExFold : kExList;
}

// Run a task: a built one (build_task), or a fold frame received ready (fj,
// with its X_X rows and ranks already in w.xrows() / w.xr()).
template <bool kAsmSearch>
__device__ __forceinline__ void run_task(const Params& p_arg, Wg& w, uint32_t root, uint32_t nu, uint32_t L, uint64_t ks,
                                         uint32_t rs, uint32_t c, uint32_t C, bool frame, const SmallJob& fj)
{
    const Params& p = kparams();
    (void)p_arg;
    // dispatcher: one instance of each executor; a suspended executor resumes
    // when the one it handed a child to has finished
    SmallJob j;
    uint32_t ex;
    bool mid_susp = false, list_susp = false;
    uint32_t lc = c, lC = C;
    const uint64_t* rows = w.lrows();
    uint32_t ws = 1;
    if (frame) {
        w.W = 1;
        w.Wx = L ? 1u : 0u;
        w.have_xrows = L > 0;
        j = fj;
        ex = kExFold;
    } else if (nu == 0) {
        // a second-level task with no common later neighbour: R itself is
        // maximal iff X is empty too
        if (L == 0) report(p, w, rs, ks);
        return;
    } else {
        ex = build_task(p, w, nu, L, ks, rs, C, j, rows, ws);
    }
    while (ex != kExDone && !w.abort) {
        if (ex == kExFold) {
            if (p.flags & MCE_F_STREAM)
                run_folded<true, false>(p, w, root, j);
            else
                run_folded<false, kAsmSearch>(p, w, root, j);
            ex = list_susp ? kExList : (mid_susp ? kExMid : kExDone);
        } else if (ex == kExList) {
            const uint32_t y = run_list(p, w, root, list_susp, j, lc, lC);
            list_susp = y == kYieldFold;
            ex = list_susp ? kExFold : (mid_susp ? kExMid : kExDone);
        } else {
            const uint32_t y = run_mid(p, w, root, nu, rows, ws, mid_susp, j, L, c, C);
            mid_susp = y != kDone;
            if (y == kYieldList) {
                lc = 0;
                lC = 1;
            }
            ex = y == kYieldFold ? kExFold : (y == kYieldList ? kExList : kExDone);
        }
    }
}

// Task parameters set up by either source of work.
struct TaskArgs {
    uint32_t root, nu, L, rs, c, C, kind;
    uint64_t ks;
};

// First-level subtree of root v (Algorithm 3): P = later neighbours, X =
// earlier neighbours; with a split (c, C) only level-1 branches t % C == c.
__device__ __forceinline__ TaskArgs setup_root(const Params& p_arg, Wg& w, uint32_t v, uint32_t split)
{
    const Params& p = kparams();
    (void)p_arg;
    const uint32_t lane = lane_id();
    uint32_t beg = p.op[v], nu = p.op[v + 1] - beg;
    uint32_t ib = p.ip[v], L = p.ip[v + 1] - ib;
    for (uint32_t i = lane; i < nu; i += 64) w.uarr()[i] = p.oc[beg + i];
    for (uint32_t i = lane; i < L; i += 64) w.xr()[i] = p.ic[ib + i];
    stat_add(S_ROOTW, nu + L);
    if (lane == 0) w.R()[0] = v;
    const uint32_t W = (nu + 63) >> 6;
    for (uint32_t q = lane; q < W; q += 64) {
        S.pw[q] = low_mask(nu - q * 64);
        S.xw[q] = 0;
    }
    wave_mem_sync();
    TaskArgs t;
    t.root = v;
    t.nu = nu;
    t.L = L;
    t.rs = 1;
    t.C = split >> 16;
    t.c = split & 0xFFFFu;
    if (t.C == 0) t.C = 1;
    t.ks = p.vkey[v];
    t.kind = kMboxLists;
    return t;
}

// Second-level subtree of the edge {v, u} (Algorithm 4), u = oc[e] a later
// neighbour of root v: R = {v, u}; P = the common neighbours ordered after u
// (later neighbours of v after u that are later neighbours of u, ascending);
// X = the common neighbours ordered before u (earlier neighbours of v, and
// later ones before u, that have u as a later neighbour).  Every X vertex is
// an earlier neighbour of u, so |X| <= the in-degree bound of the scratch.
__device__ __forceinline__ TaskArgs setup_l2(const Params& p_arg, Wg& w, uint32_t v, uint32_t e)
{
    const Params& p = kparams();
    (void)p_arg;
    const uint32_t lane = lane_id();
    const uint32_t u = p.oc[e];
    const uint32_t beg = p.op[v], end = p.op[v + 1];
    uint32_t np = 0;
    for (uint32_t b = e + 1; b < end; b += 64) {
        const uint32_t i = b + lane;
        uint32_t x = 0;
        bool in = false;
        if (i < end) {
            x = p.oc[i];
            in = has_later(p, u, x);
        }
        const uint64_t m = __ballot(in);
        if (in) w.uarr()[np + prefix_popc(m)] = x;
        np += (uint32_t)__popcll(m);
    }
    const uint32_t ib = p.ip[v], ni = p.ip[v + 1] - ib;
    const uint32_t total = ni + (e - beg);
    uint32_t nx = 0;
    for (uint32_t b = 0; b < total; b += 64) {
        const uint32_t i = b + lane;
        uint32_t x = 0;
        bool in = false;
        if (i < total) {
            x = i < ni ? p.ic[ib + i] : p.oc[beg + (i - ni)];
            in = has_later(p, x, u);
        }
        const uint64_t m = __ballot(in);
        if (in) w.xr()[nx + prefix_popc(m)] = x;
        nx += (uint32_t)__popcll(m);
    }
    stat_add(S_ROOTW, (end - e - 1) + total);
    if (lane == 0) {
        w.R()[0] = v;
        w.R()[1] = u;
    }
    const uint32_t W = (np + 63) >> 6;
    for (uint32_t q = lane; q < W; q += 64) {
        S.pw[q] = low_mask(np - q * 64);
        S.xw[q] = 0;
    }
    wave_mem_sync();
    TaskArgs t;
    t.root = v;
    t.nu = np;
    t.L = nx;
    t.rs = 2;
    t.c = 0;
    t.C = 1;
    t.kind = kMboxLists;
    t.ks = p.vkey[v] + p.vkey[u];
    return t;
}

// A task received through the worker list; its lists are in this workgroup's
// mailbox.  Returns false when the mailbox is not a task this kernel could have
// written (a size beyond its capacity, a rank >= n): nothing is read through
// such values.
__device__ __forceinline__ bool setup_received(const Params& p_arg, Wg& w, TaskArgs& t, SmallJob& fj)
{
    const Params& p = kparams();
    (void)p_arg;
    const uint32_t lane = lane_id();
    MboxHdr h = *w.mbox();
    uint32_t np = uni(h.np), nxp = uni(h.nxp);
    t.root = uni(h.root);
    t.L = uni(h.nxx);
    t.rs = uni(h.rsize);
    t.ks = uni64(h.keysum);
    t.kind = uni(h.kind);
    t.c = 0;
    t.C = 1;
    if (t.kind == kMboxFold) {
        const uint32_t m = np, L = t.L;
        if (t.root >= p.nv || m == 0 || m > 64 || nxp != 0 || L > 64 || L > p.xcap || (L && L > p.xrow_budget) ||
            t.rs == 0 || t.rs + 2 > p.rcap)
            return false;
        const uint64_t* f = w.fr();
        const uint32_t* f32 = reinterpret_cast<const uint32_t*>(f + kFrU32);
        const bool valid = lane < m, vx = lane < L;
        fj.m = m;
        fj.L = L;
        fj.P = uni64(f[0]);
        fj.XP = uni64(f[1]);
        fj.su = valid ? f32[lane] : 0u;
        fj.skey = valid ? f[kFrKey + lane] : 0ull;
        fj.rowP = valid ? f[kFrRow + lane] : 0ull;
        const uint32_t xrank = vx ? f32[64 + lane] : 0u;
        const uint64_t xrow = vx ? f[kFrXRow + lane] : 0ull;
        bool bad = (valid && fj.su >= p.nv) || (vx && xrank >= p.nv);
        for (uint32_t i = lane; i < t.rs; i += 64) bad |= w.R()[i] >= p.nv;
        if (__ballot(bad) != 0 || ((fj.P | fj.XP) & ~low_mask(m)) != 0) return false;
        if (vx) {
            w.xr()[lane] = xrank;
            w.xrows()[lane] = xrow;
        }
        fj.oidx = lane;
        fj.xj = lane;
        fj.rs = t.rs;
        fj.ks = t.ks;
        fj.anc = false;
        t.nu = m;
        wave_mem_sync();
        return true;
    }
    if (t.kind != kMboxLists) return false;
    t.nu = np + nxp;
    if (t.root >= p.nv || np > p.ucap || nxp > p.ucap || t.nu > p.ucap || t.L > p.xcap || t.rs == 0 ||
        t.rs + 2 > p.rcap)
        return false;
    bool bad = false;
    for (uint32_t i = lane; i < t.L; i += 64) bad |= w.xr()[i] >= p.nv;
    for (uint32_t i = lane; i < t.rs; i += 64) bad |= w.R()[i] >= p.nv;
    for (uint32_t i = lane; i < np; i += 64) bad |= w.mP()[i] >= p.nv;
    for (uint32_t i = lane; i < nxp; i += 64) bad |= w.mXP()[i] >= p.nv;
    if (__ballot(bad) != 0) return false;
    uint32_t W = (t.nu + 63) >> 6;
    for (uint32_t q = lane; q < W; q += 64) {
        S.pw[q] = 0;
        S.xw[q] = 0;
    }
    wave_mem_sync();
    // merge the two ascending lists into U; mark P / X_P membership
    for (uint32_t i = lane; i < np; i += 64) {
        uint32_t x = w.mP()[i];
        uint32_t lo = 0, hi = nxp;
        while (lo < hi) {
            uint32_t mid = (lo + hi) >> 1;
            if (w.mXP()[mid] < x) lo = mid + 1;
            else hi = mid;
        }
        uint32_t pos = i + lo;
        w.uarr()[pos] = x;
        atomicOr((unsigned long long*)&S.pw[pos >> 6], 1ull << (pos & 63));
    }
    for (uint32_t i = lane; i < nxp; i += 64) {
        uint32_t x = w.mXP()[i];
        uint32_t lo = 0, hi = np;
        while (lo < hi) {
            uint32_t mid = (lo + hi) >> 1;
            if (w.mP()[mid] < x) lo = mid + 1;
            else hi = mid;
        }
        uint32_t pos = i + lo;
        w.uarr()[pos] = x;
        atomicOr((unsigned long long*)&S.xw[pos >> 6], 1ull << (pos & 63));
    }
    wave_mem_sync();
    return true;
}

// Next unit of work: a (root, split) entry of the queue in phase 1, a donated
// branch in phase 2.  Returns false when the kernel is done for this workgroup.
__device__ __forceinline__ bool next_task(const Params& p_arg, Wg& w, bool& phase1, TaskArgs& t, SmallJob& fj)
{
    const Params& p = kparams();
    (void)p_arg;
    const uint32_t lane = lane_id();
    const uint32_t me = w.me;
    if (phase1) {
        uint32_t idx = 0;
        if (lane == 0) idx = atomicAdd(&p.ctrl->root_cursor, 1u);
        idx = uni(idx);
        if (idx < p.nroots) {
            if (p.l2v) {
                t = setup_l2(p, w, p.l2v[idx], p.l2e[idx]);
                return true;
            }
            uint32_t v = p.roots[idx];
            t = setup_root(p, w, v, p.splits ? p.splits[idx] : 0u);
            return true;
        }
        phase1 = false;
    }
    if (!(p.flags & MCE_F_WORKER_LIST)) return false;
    // worker list: become idle, wait for a donated branch or termination
    uint32_t terminate = 0;
    if (lane == 0) {
        __hip_atomic_store(&p.wflags[me], kFlagIdle, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // acq_rel: orders this workgroup's flag reset before a terminator's stores
        unsigned long long old =
            __hip_atomic_fetch_add(&p.ctrl->packed, 1ull, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t idle = (uint32_t)old + 1, started = (uint32_t)(old >> 32);
        terminate = idle == started;
        if (!terminate) {
            // count first, so the hint never drops below the claimable bits
            __hip_atomic_fetch_add(&p.ctrl->waiting, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_or(&p.idle_bits[(me >> 6) * kIdleStride], 1ull << (me & 63u), __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    terminate = uni(terminate);
    if (terminate) {
        for (uint32_t g = lane; g < p.nwg; g += 64)
            __hip_atomic_store(&p.wflags[g], kFlagTerm, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return false;
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
    stat_add(S_IDLE, now_ticks() - t0);
    if (f == kFlagIdle) {
        if (lane == 0) atomicOr(&p.ctrl->err, 1u);
        w.abort = true;
        return false;
    }
    if (f == kFlagTerm) return false;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (setup_received(p, w, t, fj)) return true;
    // inconsistent mailbox: report it and stop every workgroup
    if (lane == 0) atomicOr(&p.ctrl->err, 4u);
    for (uint32_t g = lane; g < p.nwg; g += 64)
        __hip_atomic_store(&p.wflags[g], kFlagTerm, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    w.abort = true;
    return false;
}

// Instantiated for five and six wavefronts per SIMD (launch bounds); the host
// picks six when the queue holds many roots per workgroup (throughput-bound),
// five otherwise (fewer spills, for launches whose time is a critical path).
template <int kWaves>
__global__ void __launch_bounds__(64, kWaves) k_enumerate(Params p)
{
    const uint32_t lane = lane_id();
    const uint32_t me = blockIdx.x;
    Wg& w = SW;
    w.me = me;
    for (uint32_t k = lane; k < (uint32_t)kHistLds; k += 64) S.hist[k] = 0;
    for (uint32_t k = lane; k < (uint32_t)S_COUNT + 4; k += 64) S.stat[k] = 0;
    wave_mem_sync();
    w.count = w.hash = 0;
    w.cur_gid = 0;
    w.hmax = 0;
    w.task_t0 = 0;
    w.nodes = w.nodes_t0 = 0;
    w.don_t0 = 0;
    S.probes[lane] = 0;
    w.wl_tick = w.wl_seen = w.poll = w.pops = 0;
    w.don_min = (p.flags & MCE_F_WORKER_LIST) ? p.donate_min_p : 0xFFFFFFFFu;
    w.me = me;
    w.abort = false;
    w.W = 1;
    w.Wx = 0;
    w.have_xrows = false;
    w.deadline = uni64(now_ticks()) + p.timeout_ticks;

    if ((p.flags & MCE_F_WORKER_LIST) && lane == 0)
        __hip_atomic_fetch_add(&p.ctrl->packed, 1ull << 32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

    // phase 1: queue entries from the shared counter; phase 2: worker list
    bool phase1 = true;
    TaskArgs t;
    SmallJob fj;
    while (!w.abort && next_task(p, w, phase1, t, fj)) {
        begin_task(p, w, t.root);
        run_task<kWaves == 6>(p, w, t.root, t.nu, t.L, t.ks, t.rs, t.c, t.C, t.kind == kMboxFold, fj);
        finish_task(p, w, t.root, t.nu, t.L, t.rs, t.c, t.C);
    }
    flush_graph(p, w);
    uint32_t pl = wave_sum(S.probes[lane]);
    if (lane == 0) {
        // idle workgroups of a small launch have nothing to add: skip zero adds
        auto add = [&](int k, unsigned long long v) {
            if (v) atomicAdd(&p.acc[2 + k], v);
        };
        add(MCE_STAT_PROBES, (unsigned long long)pl);
        add(MCE_STAT_ROOT_WORDS, (unsigned long long)S.stat[S_ROOTW]);
        add(MCE_STAT_BUSY_NS, (unsigned long long)S.stat[S_BUSY]);
        if (S.stat[S_MAXTASK]) atomicMax(&p.acc[2 + MCE_STAT_MAX_TASK_NS], (unsigned long long)S.stat[S_MAXTASK]);
        add(MCE_STAT_NODES, (unsigned long long)w.nodes);
        add(MCE_STAT_DONATIONS, (unsigned long long)S.stat[S_DONATIONS]);
        add(MCE_STAT_TASKS, (unsigned long long)S.stat[S_TASKS]);
        add(MCE_STAT_XTESTS, (unsigned long long)S.stat[S_XTESTS]);
        add(MCE_STAT_BUILD_EDGES, (unsigned long long)S.stat[S_EDGES]);
        add(MCE_STAT_HBM_ROWS, (unsigned long long)S.stat[S_HBM]);
        add(MCE_STAT_IDLE_NS, (unsigned long long)S.stat[S_IDLE]);
        add(MCE_STAT_XROW_TASKS, (unsigned long long)S.stat[S_XROW]);
        add(MCE_STAT_BUILD_TICKS, (unsigned long long)S.stat[S_BUILD]);
        add(MCE_STAT_DONATE_NS, (unsigned long long)S.stat[S_DONATE]);
        add(MCE_STAT_POP_FAILS, (unsigned long long)S.stat[S_POPFAIL]);
        add(MCE_STAT_XCOL_WORDS, (unsigned long long)S.stat[S_XCOLW]);
        add(MCE_STAT_FOLD_DONATIONS, (unsigned long long)S.stat[S_FOLDDON]);
    }
}

// ---------------------------------------------------------------- root queue
// flag[i] = 1 if the i-th root in processing order is in the window and has P != {}.
// A queued root's P (at most its core number of later neighbours) must fit
// the launch's universe capacity ucap; a violation sets *err.
__global__ void k_root_flags(const uint32_t* __restrict__ op, const uint32_t* __restrict__ core_r, uint32_t n,
                             uint32_t c, uint32_t mode, const uint32_t* __restrict__ custom,
                             const uint32_t* __restrict__ rank, uint32_t ucap, uint32_t* __restrict__ cand,
                             uint32_t* __restrict__ flag, uint32_t* __restrict__ err)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        uint32_t r;
        if (mode == 1) r = n - 1 - (uint32_t)i;
        else if (mode == 2) r = rank[custom[i]];
        else r = (uint32_t)i;
        cand[i] = r;
        const uint32_t np = op[r + 1] - op[r];
        const bool in = core_r[r] <= c && np > 0;
        if (in && np > ucap) atomicOr(err, 1u);
        flag[i] = in ? 1u : 0u;
    }
}

__global__ void k_root_compact(const uint32_t* __restrict__ cand, const uint32_t* __restrict__ flag,
                               const uint32_t* __restrict__ pos, uint32_t n, uint32_t* __restrict__ roots)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        if (flag[i]) roots[pos[i]] = cand[i];
}

// Second-level tasks of the queue's roots: one per later neighbour, in root
// order (cnt[i] = out-degree of root i; off = its exclusive scan).
__global__ void k_l2_counts(const uint32_t* __restrict__ roots, uint32_t nroots, const uint32_t* __restrict__ op,
                            uint32_t* __restrict__ cnt)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nroots; i += (size_t)gridDim.x * blockDim.x)
        cnt[i] = op[roots[i] + 1] - op[roots[i]];
}

__global__ void k_l2_expand(const uint32_t* __restrict__ roots, uint32_t nroots, const uint32_t* __restrict__ op,
                            const uint32_t* __restrict__ off, uint32_t* __restrict__ l2v, uint32_t* __restrict__ l2e)
{
    const uint32_t lane = lane_id();
    const size_t waves = (size_t)gridDim.x * (blockDim.x / 64);
    for (size_t i = (size_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); i < nroots; i += waves) {
        const uint32_t v = roots[i], beg = op[v], d = op[v + 1] - beg, o = off[i];
        for (uint32_t j = lane; j < d; j += 64) {
            l2v[o + j] = v;
            l2e[o + j] = beg + j;
        }
    }
}

// A custom root order must be a permutation of 0..n-1: count each id, flag
// ids out of range (err bit 0) and ids seen other than once (err bit 1).
__global__ void k_perm_count(const uint32_t* __restrict__ ids, uint32_t n, uint32_t* __restrict__ seen,
                             uint32_t* __restrict__ err)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        uint32_t v = ids[i];
        if (v >= n) atomicOr(err, 1u);
        else atomicAdd(&seen[v], 1u);
    }
}

__global__ void k_perm_check(const uint32_t* __restrict__ seen, uint32_t n, uint32_t* __restrict__ err)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        if (seen[i] != 1u) atomicOr(err, 2u);
}

// Isolated vertices are maximal cliques of size 1 (Algorithm 3 with P = X = {}).
// One graph: counts and hashes are summed across the wave first (one atomic per
// wave); a batch adds per vertex into its own graph's accumulators.  With the
// clique stream on (single graph), each is also written to the stream.
struct IsoStream {
    Ctrl* ctrl;
    const uint32_t* perm;
    uint32_t* verts;
    uint64_t vcap;
    unsigned long long* offs;
    uint64_t ocap;
};

__global__ void k_isolated(const uint32_t* __restrict__ op, const uint32_t* __restrict__ ip,
                           const uint64_t* __restrict__ vkey, const uint32_t* __restrict__ gid, uint32_t n,
                           unsigned long long* gacc, unsigned long long* ghist, uint32_t hist_len, IsoStream st)
{
    const uint32_t lane = lane_id();
    unsigned long long cnt = 0, hsh = 0;
    for (size_t base = (size_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); base < n;
         base += (size_t)gridDim.x * blockDim.x) {
        const size_t r = base + lane;
        if (r < n && op[r + 1] == op[r] && ip[r + 1] == ip[r]) {
            const unsigned long long h = fmix64(vkey[r] + kGamma);
            if (gid) {
                const uint32_t g = gid[r];
                atomicAdd(&gacc[2 * g], 1ull);
                atomicAdd(&gacc[2 * g + 1], h);
                atomicAdd(&ghist[(uint64_t)g * hist_len + 1], 1ull);
            } else {
                cnt += 1;
                hsh += h;
            }
            if (st.verts) {
                unsigned long long c = atomicAdd(&st.ctrl->stream_c, 1ull);
                unsigned long long v = atomicAdd(&st.ctrl->stream_v, 1ull);
                const bool fits = v + 1 <= st.vcap;
                if (fits) st.verts[v] = st.perm[r];
                if (c < st.ocap) st.offs[c] = fits ? ((v << 16) | 1ull) : ~0ull;
                if (!fits || c >= st.ocap) st.ctrl->stream_trunc = 1;
            }
        }
    }
    if (!gid) {
        for (int off = 32; off > 0; off >>= 1) {
            cnt += __shfl_xor(cnt, off, 64);
            hsh += __shfl_xor(hsh, off, 64);
        }
        if (lane == 0 && cnt) {
            atomicAdd(&gacc[0], cnt);
            atomicAdd(&gacc[1], hsh);
            atomicAdd(&ghist[1], cnt);
        }
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

// Largest task universe of a launch.  In the synchronous-peel order a vertex
// has at most core(v) later neighbours, and every task universe lies inside
// its root's P, so a core window c bounds every universe by min(max
// out-degree, c); the root queue checks each root against it.
uint32_t universe_cap(const Oriented& g, const EnumConfig& cfg)
{
    return std::max(std::min(g.max_out, cfg.max_root_core), 1u);
}

}  // namespace

mce_status build_root_queue(const Oriented& g, const EnumConfig& cfg, EnumState& st, hipStream_t s,
                            uint32_t* nroots_out)
{
    mce_status rc;
    const uint32_t n = g.n;
    const size_t nn = n ? n : 1;
    if ((rc = st.roots.alloc(nn * 4)) != MCE_OK) return rc;
    if ((rc = st.tmp_a.alloc(nn * 4)) != MCE_OK) return rc;
    if ((rc = st.tmp_b.alloc((nn + 1) * 4)) != MCE_OK) return rc;
    if ((rc = st.tmp_c.alloc(nn * 4)) != MCE_OK) return rc;
    if ((rc = st.scan_tmp.alloc(scan_tmp_words(nn + 1) * 8 + 64)) != MCE_OK) return rc;
    if ((rc = st.small.alloc(64)) != MCE_OK) return rc;
    uint32_t mode = 0;
    if (cfg.flags & MCE_F_CUSTOM_ORDER) mode = 2;
    else if (cfg.flags & MCE_F_REVERSE_ORDER) mode = 1;
    if (mode == 2 && !cfg.root_order) {
        set_error("MCE_F_CUSTOM_ORDER without root_order");
        return MCE_ERR_INVALID_ARG;
    }
    uint32_t nroots = 0;
    if (n && mode == 2) {
        uint32_t* seen = st.tmp_b.as<uint32_t>();
        uint32_t* derr = st.small.as<uint32_t>();
        fill_u32(seen, 0, n, s);
        fill_u32(derr, 0, 1, s);
        k_perm_count<<<blocks_for(n, 256, 8192), 256, 0, s>>>(cfg.root_order, n, seen, derr);
        k_perm_check<<<blocks_for(n, 256, 8192), 256, 0, s>>>(seen, n, derr);
        MCE_HIP_TRY(hipGetLastError());
        uint32_t herr = 0;
        MCE_HIP_TRY(hipMemcpyAsync(&herr, derr, 4, hipMemcpyDeviceToHost, s));
        MCE_HIP_TRY(hipStreamSynchronize(s));
        if (herr) {
            set_error((herr & 1u) ? "root_order holds an id >= n" : "root_order is not a permutation");
            return MCE_ERR_INVALID_ARG;
        }
    }
    if (n) {
        uint32_t* dtotal = st.small.as<uint32_t>();
        fill_u32(dtotal + 1, 0, 1, s);
        k_root_flags<<<blocks_for(n, 256, 8192), 256, 0, s>>>(g.op.as<uint32_t>(), g.core_r.as<uint32_t>(), n,
                                                              cfg.max_root_core, mode, cfg.root_order,
                                                              g.rank.as<uint32_t>(), universe_cap(g, cfg),
                                                              st.tmp_a.as<uint32_t>(), st.tmp_c.as<uint32_t>(),
                                                              dtotal + 1);
        MCE_HIP_TRY(hipGetLastError());
        if ((rc = exclusive_scan_u32(st.tmp_c.as<uint32_t>(), st.tmp_b.as<uint32_t>(), n, dtotal,
                                     st.scan_tmp.as<uint64_t>(), s)) != MCE_OK)
            return rc;
        k_root_compact<<<blocks_for(n, 256, 8192), 256, 0, s>>>(st.tmp_a.as<uint32_t>(), st.tmp_c.as<uint32_t>(),
                                                                st.tmp_b.as<uint32_t>(), n, st.roots.as<uint32_t>());
        MCE_HIP_TRY(hipGetLastError());
        uint32_t hv[2] = {0, 0};
        MCE_HIP_TRY(hipMemcpyAsync(hv, dtotal, 8, hipMemcpyDeviceToHost, s));
        MCE_HIP_TRY(hipStreamSynchronize(s));
        nroots = hv[0];
        if (hv[1]) {
            set_error("internal: a root's later-neighbour list exceeds the universe capacity");
            return MCE_ERR_DEVICE;
        }
    }
    *nroots_out = nroots;
    return MCE_OK;
}

mce_status enumerate_graph(const Oriented& g, const EnumConfig& cfg, EnumState& st, hipStream_t s,
                           EnumOutput& out)
{
    mce_status rc;
    const uint32_t n = g.n;
    const uint32_t ng = std::max<uint32_t>(g.ngraphs, 1u);
    // per-workgroup LDS and scratch sized by the largest universe of this window
    const uint32_t ucap = universe_cap(g, cfg);
    if (ucap > kMaxUniverse) {
        set_error("first-level P larger than " + std::to_string(kMaxUniverse) + " vertices is not supported");
        return MCE_ERR_UNSUPPORTED;
    }
    const uint32_t hist_len = g.degeneracy + 3;
    const uint32_t xcap = std::max(g.max_in, 1u);
    const uint32_t rcap = g.degeneracy + 3;
    const uint32_t wg_words = (ucap + 63) / 64;
    const uint32_t wgx_words = std::min<uint32_t>(64u, (xcap + 63) / 64);  // X_X bitmaps: |X| <= 4096
    const uint32_t ws_g = wg_words | 1u;

    int dev = 0;
    MCE_HIP_TRY(hipGetDevice(&dev));
    int cus = 0, lds_cu = 0;
    MCE_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
        lds_cu <= 0)
        lds_cu = 160 * 1024;
    const size_t uarr_bytes = (size_t)((ucap + 3) & ~3u) * 4;
    auto rows_words = [](uint32_t cap) {
        const uint32_t ws = cap <= 64 ? 1u : (((cap + 63) / 64) | 1u);
        return (size_t)std::max(cap * ws, 64u);
    };
    // Resident workgroups and LDS layout for one instantiation of the kernel:
    // the workgroups per CU that the registers allow, and that a workgroup's
    // LDS allows (gfx950 allocates a workgroup's static plus dynamic LDS in
    // 1280-byte granules, 160 KiB = 128 granules, which the occupancy query
    // does not model).  The LDS bitmap cap is the given one, else the largest
    // up to the default that keeps the register-limited number resident.
    struct Launch {
        const void* fn;
        size_t lds_static = 0, lds_bytes = 0;
        uint32_t lds_cap = 0, G = 0;
    };
    auto plan = [&](const void* fn, Launch& L) -> mce_status {
        L.fn = fn;
        hipFuncAttributes fa;
        MCE_HIP_TRY(hipFuncGetAttributes(&fa, fn));
        L.lds_static = std::max<size_t>(fa.sharedSizeBytes, sizeof(LdsFixed) + sizeof(Wg));
        int per_cu_regs = 0;
        MCE_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_regs, fn, 64, 0));
        if (per_cu_regs <= 0) per_cu_regs = 1;
        auto per_cu_lds = [&](size_t dyn) {
            const size_t granule = 1280;
            return (int)((size_t)lds_cu / ((L.lds_static + dyn + granule - 1) / granule * granule));
        };
        if (cfg.bitmap_max_p) {
            L.lds_cap = std::max(64u, std::min(cfg.bitmap_max_p, std::max(ucap, 64u)));
        } else {
            L.lds_cap = std::max(64u, std::min(kDefaultBitmapMaxP, std::max(ucap, 64u)));
            while (L.lds_cap > 64 && per_cu_lds(uarr_bytes + rows_words(L.lds_cap) * 8) < per_cu_regs)
                L.lds_cap = std::max(64u, L.lds_cap - 8);
        }
        L.lds_bytes = uarr_bytes + rows_words(L.lds_cap) * 8;  // dynamic part (uarr, then rows)
        if (L.lds_bytes + L.lds_static > (size_t)lds_cu) {
            set_error("LDS budget exceeded; lower bitmap_max_p");
            return MCE_ERR_INVALID_ARG;
        }
        int per_cu = 0;
        MCE_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64, L.lds_bytes));
        per_cu = std::min(per_cu, per_cu_lds(L.lds_bytes));
        if (per_cu <= 0) per_cu = 1;
        if (cfg.wg_per_cu) per_cu = std::min<int>(per_cu, (int)cfg.wg_per_cu);
        L.G = (uint32_t)(per_cu * cus);
        if (L.G == 0) L.G = 1;
        return MCE_OK;
    };
    Launch L5, L;
    if ((rc = plan(reinterpret_cast<const void*>(k_enumerate<5>), L5)) != MCE_OK) return rc;

    hipEvent_t e0, e1, e2;
    MCE_HIP_TRY(hipEventCreate(&e0));
    MCE_HIP_TRY(hipEventCreate(&e1));
    MCE_HIP_TRY(hipEventCreate(&e2));
    MCE_HIP_TRY(hipEventRecord(e0, s));

    // the queue in processing order (the learned form reorders it below)
    uint32_t nroots = 0;
    {
        EnumConfig qcfg = cfg;
        if (cfg.flags & MCE_F_LEARNED_ORDER) qcfg.flags &= ~(MCE_F_CUSTOM_ORDER | MCE_F_REVERSE_ORDER);
        if ((rc = build_root_queue(g, qcfg, st, s, &nroots)) != MCE_OK) return rc;
    }
    // six wavefronts per SIMD when there are at least kSixWaveRoots roots per
    // workgroup of the five-wavefront launch
    L = L5;
    if ((uint64_t)nroots >= (uint64_t)kSixWaveRoots * L5.G) {
        Launch L6;
        if ((rc = plan(reinterpret_cast<const void*>(k_enumerate<6>), L6)) != MCE_OK) return rc;
        if (L6.G > L5.G) L = L6;
    }
    const size_t lds_static = L.lds_static, lds_bytes = L.lds_bytes;
    const uint32_t lds_cap = L.lds_cap;
    uint32_t G = L.G;

    // per-workgroup scratch layout
    const uint64_t xrow_words = std::min<uint64_t>(cfg.xrow_budget_words, (uint64_t)xcap * wg_words);
    const uint64_t xcol_words = std::min<uint64_t>(cfg.xrow_budget_words, (uint64_t)ucap * wgx_words);
    uint64_t off = align_up(sizeof(MboxHdr), 256);
    const uint64_t off_P = off; off = align_up(off + (uint64_t)ucap * 4, 256);
    const uint64_t off_XP = off; off = align_up(off + (uint64_t)ucap * 4, 256);
    const uint64_t off_R = off; off = align_up(off + (uint64_t)rcap * 4, 256);
    const uint64_t off_fr = off; off = align_up(off + kFrameBytes, 256);
    const uint64_t off_xr = off; off = align_up(off + (uint64_t)xcap * 4, 256);
    const uint64_t off_xx = off; off = align_up(off + (uint64_t)xcap * 4, 256);
    const uint64_t off_flag = off; off = align_up(off + ((uint64_t)xcap / 64 + 2) * 8, 256);
    const uint64_t off_hpos = off; off = align_up(off + ((uint64_t)xcap / 2 + 2) * 4, 256);
    const uint64_t off_spos = off; off = align_up(off + ((uint64_t)xcap / 2 + 2) * 4, 256);
    const uint64_t off_rows = off; off = align_up(off + (uint64_t)ucap * ws_g * 8, 256);
    const uint64_t off_xrows = off; off = align_up(off + xrow_words * 8 + 8, 256);
    const uint64_t off_xcols = off; off = align_up(off + xcol_words * 8 + 8, 256);
    const uint64_t off_stack = off; off = align_up(off + (uint64_t)(ucap + 2) * (3 * wg_words + wgx_words) * 8, 256);
    const uint64_t off_meta = off; off = align_up(off + (uint64_t)(ucap + 2) * 24, 256);
    const uint64_t off_ukey = off; off = align_up(off + (uint64_t)ucap * 8, 256);
    const uint64_t off_susp = off; off = align_up(off + 64 * 4 * 8 + 64 * 3 * 4, 256);
    const uint64_t stride = off;
    // per-workgroup scratch is sized by the largest in-degree (X lists), so a
    // hub-heavy graph needs several MB per workgroup: allow up to a quarter of
    // the free device memory (at least 32 GiB), and fewer workgroups beyond it
    uint64_t budget = 32ull << 30;
    {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) == hipSuccess) budget = std::max<uint64_t>(budget, free_b / 4);
        else (void)hipGetLastError();
    }
    if ((uint64_t)G * stride > budget) G = (uint32_t)std::max<uint64_t>(1, budget / stride);

    if ((rc = st.scratch.alloc((size_t)G * stride)) != MCE_OK) return rc;
    if ((rc = st.ctrl.alloc(sizeof(Ctrl))) != MCE_OK) return rc;
    if ((rc = st.acc.alloc(32 * 8)) != MCE_OK) return rc;
    if ((rc = st.gacc.alloc((size_t)ng * 16)) != MCE_OK) return rc;
    if ((rc = st.hist.alloc((size_t)ng * hist_len * 8)) != MCE_OK) return rc;
    const uint32_t idle_words = (G + 63) / 64;
    if ((rc = st.idle.alloc((size_t)idle_words * kIdleStride * 8)) != MCE_OK) return rc;
    if ((rc = st.flags.alloc((size_t)G * 4)) != MCE_OK) return rc;

    // reset control state (fill kernels, no memset nodes)
    fill_u64(reinterpret_cast<uint64_t*>(st.ctrl.p), 0, sizeof(Ctrl) / 8, s);
    fill_u64(st.acc.as<uint64_t>(), 0, 32, s);
    fill_u64(st.gacc.as<uint64_t>(), 0, (size_t)ng * 2, s);
    fill_u64(st.hist.as<uint64_t>(), 0, (size_t)ng * hist_len, s);
    fill_u64(st.idle.as<uint64_t>(), 0, (size_t)idle_words * kIdleStride, s);
    fill_u32(st.flags.as<uint32_t>(), kFlagIdle, G, s);

    const uint32_t* roots = st.roots.as<uint32_t>();
    const uint32_t* splits = nullptr;
    if (cfg.flags & MCE_F_LEARNED_ORDER) {
        if (!cfg.model) {
            set_error("MCE_F_LEARNED_ORDER without a model");
            return MCE_ERR_INVALID_ARG;
        }
        if ((rc = learned_queue(g, cfg, st, s, G, st.lq, nroots)) != MCE_OK) return rc;
        roots = st.lq.qroots;
        splits = st.lq.qsplits;
        nroots = st.lq.len;
    }
    const uint32_t* l2v = nullptr;
    const uint32_t* l2e = nullptr;
    if ((cfg.flags & MCE_F_L2_ROOTS) && nroots) {
        // the queue's roots expanded into their second-level tasks
        uint32_t* cnt = st.tmp_a.as<uint32_t>();
        uint32_t* off = st.tmp_b.as<uint32_t>();
        uint32_t* dtotal = st.small.as<uint32_t>() + 2;
        k_l2_counts<<<blocks_for(nroots, 256, 8192), 256, 0, s>>>(roots, nroots, g.op.as<uint32_t>(), cnt);
        MCE_HIP_TRY(hipGetLastError());
        if ((rc = exclusive_scan_u32(cnt, off, nroots, dtotal, st.scan_tmp.as<uint64_t>(), s)) != MCE_OK) return rc;
        uint32_t ntasks = 0;
        MCE_HIP_TRY(hipMemcpyAsync(&ntasks, dtotal, 4, hipMemcpyDeviceToHost, s));
        MCE_HIP_TRY(hipStreamSynchronize(s));
        if ((rc = st.l2v.alloc((size_t)std::max(ntasks, 1u) * 4)) != MCE_OK) return rc;
        if ((rc = st.l2e.alloc((size_t)std::max(ntasks, 1u) * 4)) != MCE_OK) return rc;
        k_l2_expand<<<blocks_for(nroots, 4, 8192), 256, 0, s>>>(roots, nroots, g.op.as<uint32_t>(), off,
                                                                 st.l2v.as<uint32_t>(), st.l2e.as<uint32_t>());
        MCE_HIP_TRY(hipGetLastError());
        l2v = st.l2v.as<uint32_t>();
        l2e = st.l2e.as<uint32_t>();
        nroots = ntasks;
    }
    IsoStream iso{};
    if ((cfg.flags & MCE_F_STREAM) && cfg.stream_vertices && cfg.stream_offsets && g.ngraphs <= 1) {
        iso.ctrl = reinterpret_cast<Ctrl*>(st.ctrl.p);
        iso.perm = g.perm.as<uint32_t>();
        iso.verts = cfg.stream_vertices;
        iso.vcap = cfg.stream_vcap;
        iso.offs = reinterpret_cast<unsigned long long*>(cfg.stream_offsets);
        iso.ocap = cfg.stream_ocap;
    }
    if (n) {
        k_isolated<<<blocks_for(n, 256, 4096), 256, 0, s>>>(
            g.op.as<uint32_t>(), g.ip.as<uint32_t>(), g.vkey.as<uint64_t>(),
            g.ngraphs > 1 ? g.gid.as<uint32_t>() : nullptr, n, reinterpret_cast<unsigned long long*>(st.gacc.p),
            reinterpret_cast<unsigned long long*>(st.hist.p), hist_len, iso);
        MCE_HIP_TRY(hipGetLastError());
    }
    MCE_HIP_TRY(hipEventRecord(e1, s));

    Params p{};
    p.op = g.op.as<uint32_t>();
    p.oc = g.oc.as<uint32_t>();
    p.ip = g.ip.as<uint32_t>();
    p.ic = g.ic.as<uint32_t>();
    p.vkey = g.vkey.as<uint64_t>();
    p.perm = g.perm.as<uint32_t>();
    p.gid = g.ngraphs > 1 ? g.gid.as<uint32_t>() : nullptr;
    p.roots = roots;
    p.splits = splits;
    p.l2v = l2v;
    p.l2e = l2e;
    p.nroots = nroots;
    p.ctrl = reinterpret_cast<Ctrl*>(st.ctrl.p);
    p.acc = reinterpret_cast<unsigned long long*>(st.acc.p);
    p.gacc = reinterpret_cast<unsigned long long*>(st.gacc.p);
    p.ghist = reinterpret_cast<unsigned long long*>(st.hist.p);
    p.hist_len = hist_len;
    p.scratch = st.scratch.as<uint8_t>();
    p.stride = stride;
    p.off_P = off_P;
    p.off_XP = off_XP;
    p.off_R = off_R;
    p.off_fr = off_fr;
    p.off_xr = off_xr;
    p.off_xx = off_xx;
    p.off_flag = off_flag;
    p.off_hpos = off_hpos;
    p.off_spos = off_spos;
    p.off_rows = off_rows;
    p.off_xrows = off_xrows;
    p.off_xcols = off_xcols;
    p.off_stack = off_stack;
    p.off_meta = off_meta;
    p.off_ukey = off_ukey;
    p.off_susp = off_susp;
    p.xrow_budget = xrow_words;
    p.xcol_budget = xcol_words;
    p.xrow_ratio = cfg.xrow_ratio;
    p.xrow_min_u = cfg.xrow_min_u;
    p.idle_bits = st.idle.as<unsigned long long>();
    p.idle_words = idle_words;
    p.wflags = st.flags.as<uint32_t>();
    p.ucap = ucap;
    p.nv = n;
    p.lds_cap = lds_cap;
    p.wg = wg_words;
    p.wgx = wgx_words;
    p.xcap = xcap;
    p.rcap = rcap;
    p.flags = cfg.flags;
    p.donate_min_p = cfg.donate_min_p ? cfg.donate_min_p : kDefaultDonateMinP;
    p.donate_max_depth = cfg.donate_max_depth;
    p.donate_every = cfg.donate_every ? cfg.donate_every : 1u;
    p.nwg = G;
    p.timeout_ticks = (cfg.timeout_ms ? cfg.timeout_ms : 600000ull) * 100000ull;  // 100 MHz clock
    p.tlog = (cfg.flags & MCE_F_TASK_LOG) ? reinterpret_cast<unsigned long long*>(cfg.task_log) : nullptr;
    p.tlog_cap = p.tlog ? cfg.task_log_cap : 0;
    p.tlog_min_ticks = (uint64_t)cfg.task_log_min_us * 100ull;
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
        if (L.fn == reinterpret_cast<const void*>(k_enumerate<6>))
            k_enumerate<6><<<G, 64, lds_bytes, s>>>(p);
        else
            k_enumerate<5><<<G, 64, lds_bytes, s>>>(p);
        MCE_HIP_TRY(hipGetLastError());
    }
    MCE_HIP_TRY(hipEventRecord(e2, s));
    uint64_t acc[32];
    Ctrl ctrl;
    std::vector<uint64_t> gacc((size_t)ng * 2);
    std::vector<uint64_t> ghist((size_t)ng * hist_len);
    MCE_HIP_TRY(hipMemcpyAsync(acc, st.acc.p, sizeof(acc), hipMemcpyDeviceToHost, s));
    MCE_HIP_TRY(hipMemcpyAsync(&ctrl, st.ctrl.p, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    MCE_HIP_TRY(hipMemcpyAsync(gacc.data(), st.gacc.p, gacc.size() * 8, hipMemcpyDeviceToHost, s));
    MCE_HIP_TRY(hipMemcpyAsync(ghist.data(), st.hist.p, ghist.size() * 8, hipMemcpyDeviceToHost, s));
    MCE_HIP_TRY(hipStreamSynchronize(s));
    float ms_setup = 0, ms_kernel = 0;
    (void)hipEventElapsedTime(&ms_setup, e0, e1);
    (void)hipEventElapsedTime(&ms_kernel, e1, e2);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipEventDestroy(e2);

    out.graphs.assign(ng, EnumOutput::PerGraph());
    out.count = out.hash = 0;
    for (uint32_t gi = 0; gi < ng; ++gi) {
        auto& pg = out.graphs[gi];
        pg.count = gacc[2 * gi];
        pg.hash = gacc[2 * gi + 1];
        pg.hist.assign(ghist.begin() + (size_t)gi * hist_len, ghist.begin() + (size_t)(gi + 1) * hist_len);
        pg.max_size = 0;
        for (uint32_t k = 0; k < hist_len; ++k)
            if (pg.hist[k]) pg.max_size = k;
        out.count += pg.count;
        out.hash += pg.hash;
    }
    out.hist = out.graphs[0].hist;
    out.max_size = out.graphs[0].max_size;
    for (int i = 0; i < 24; ++i) out.stats[i] = acc[2 + i];
    out.stats[MCE_STAT_ROOTS] = nroots;
    out.stats[MCE_STAT_WORKGROUPS] = G;
    out.stats[MCE_STAT_KERNEL_NS] = (uint64_t)(ms_kernel * 1e6);
    out.stats[MCE_STAT_SETUP_NS] = (uint64_t)(ms_setup * 1e6);
    out.stats[MCE_STAT_IDLE_NS] = acc[2 + MCE_STAT_IDLE_NS] * 10;  // 100 MHz ticks -> ns
    out.stats[MCE_STAT_BUSY_NS] = acc[2 + MCE_STAT_BUSY_NS] * 10;
    out.stats[MCE_STAT_MAX_TASK_NS] = acc[2 + MCE_STAT_MAX_TASK_NS] * 10;
    out.stats[MCE_STAT_LDS_BYTES] = lds_bytes + lds_static;
    out.stats[MCE_STAT_BUILD_NS] = acc[2 + MCE_STAT_BUILD_TICKS] * 10;
    out.stats[MCE_STAT_TASK_LOG] = ctrl.tlog_n;
    out.stats[MCE_STAT_DONATE_NS] = acc[2 + MCE_STAT_DONATE_NS] * 10;
    out.xrow_tasks = acc[2 + MCE_STAT_XROW_TASKS];
    out.build_ns = acc[2 + MCE_STAT_BUILD_TICKS] * 10;
    out.stream_c = ctrl.stream_c;
    out.stream_v = ctrl.stream_v;
    out.stream_truncated = ctrl.stream_trunc != 0;
    out.timed_out = (ctrl.err & 1u) != 0;
    const bool mailbox_err = (ctrl.err & 4u) != 0;
    st.grid = G;
    st.lds_cap = lds_cap;
    if (mailbox_err) {
        set_error("a worker-list mailbox held sizes or ranks out of range; results are invalid");
        return MCE_ERR_DEVICE;
    }
    if (out.timed_out) {
        set_error("enumeration exceeded its timeout; results are invalid");
        return MCE_ERR_TIMEOUT;
    }
    return MCE_OK;
}

}  // namespace mce
