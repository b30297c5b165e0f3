// Graph preprocessing on the device: CSR validation, the synchronous-round
// k-core peel that yields core numbers and a degeneracy order (Section II-D,
// "Degeneracy Ordering"; included in the timed region as in Section IV-A), and
// orientation of every row into the later neighbours (the first-level P of
// Algorithm 3) and earlier neighbours (the first-level X), relabelled by rank.
#include "mce_internal.h"

#include <algorithm>
#include <cstring>

namespace mce {

namespace {

constexpr uint32_t kUnset = 0xFFFFFFFFu;
constexpr int kPeelSteps = 16;  // peel steps per graph launch

unsigned blocks_for(size_t items, unsigned per_block, unsigned cap = 65536)
{
    size_t b = (items + per_block - 1) / per_block;
    if (b == 0) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

__device__ inline uint64_t fmix64(uint64_t z)
{
    // SplitMix64 output finaliser (Steele, Lea and Flood, OOPSLA 2014).
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__device__ inline uint32_t lane_id() { return __lane_id(); }

__device__ inline uint32_t prefix_popc(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// ---- validation ---------------------------------------------------------------
// error code: (row << 32) | (pos << 3) | kind; min over the grid wins.
enum : uint32_t { kErrRowPtr = 1, kErrColRange = 2, kErrOrder = 3, kErrSelfLoop = 4, kErrAsym = 5 };

__global__ void k_validate_rowptr(const uint32_t* __restrict__ rp, uint32_t n, uint64_t nnz,
                                  unsigned long long* err)
{
    for (size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x; v <= n;
         v += (size_t)gridDim.x * blockDim.x) {
        bool bad = false;
        if (v == 0 && rp[0] != 0) bad = true;
        if (v == n && (uint64_t)rp[n] != nnz) bad = true;
        if (v < n && rp[v] > rp[v + 1]) bad = true;
        if (bad) atomicMin(err, ((unsigned long long)v << 32) | kErrRowPtr);
    }
}

__device__ bool row_contains(const uint32_t* __restrict__ rp, const uint32_t* __restrict__ ci,
                             uint32_t u, uint32_t w)
{
    uint32_t lo = rp[u], hi = rp[u + 1];
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        uint32_t x = ci[mid];
        if (x == w) return true;
        if (x < w) lo = mid + 1;
        else hi = mid;
    }
    return false;
}

// Symmetry is decided exactly, without hashing.  With strictly increasing rows
// and no self-loops the arcs of each direction form a set of ordered pairs.
// The first pass (kCheckShape) checks ranges, self-loops and order, and counts
// the arcs v -> u with v < u ("up") and with v > u ("down").  The second pass
// (kCheckUp, only when the counts agree) looks up the reverse of every up arc.
// If every up arc has its reverse, reversal maps the up arcs one-to-one into
// the down arcs; equal counts make that map onto, so every down arc has its
// reverse too and the graph is symmetric.  Whenever either pass fails, a
// third pass (kCheckAll) looks up the reverse of every arc and names the first
// offending (row, position).
enum CheckMode : int { kCheckShape = 0, kCheckUp = 1, kCheckAll = 2 };

constexpr uint32_t kLongRow = 2048;  // longer rows are deferred to a workgroup each
constexpr uint32_t kLongBlocks = 2048;  // workgroups of the deferred-row pass (eight per CU)

// Sum two 64-bit counters over the block, one atomic per counter.
__device__ inline void block_add2(unsigned long long (&a)[2], unsigned long long* counts)
{
    const uint32_t lane = lane_id();
    for (int k = 0; k < 2; ++k)
        for (int off = 32; off > 0; off >>= 1) a[k] += __shfl_xor(a[k], off, 64);
    __shared__ unsigned long long part[2][16];
    if (lane == 0)
        for (int k = 0; k < 2; ++k) part[k][threadIdx.x >> 6] = a[k];
    __syncthreads();
    if (threadIdx.x < 2) {
        unsigned long long t = 0;
        for (uint32_t k = 0; k < blockDim.x / 64; ++k) t += part[threadIdx.x][k];
        if (t) atomicAdd(&counts[threadIdx.x], t);
    }
}

// Checks of entry e of row v (row starts at beg) in the given mode; a[] gathers
// the up and down counts of the first pass.
__device__ __forceinline__ void check_arc(const uint32_t* __restrict__ rp, const uint32_t* __restrict__ ci, uint32_t n,
                                          uint32_t v, uint32_t beg, uint32_t e, int mode, unsigned long long* err,
                                          unsigned long long (&a)[2])
{
    uint32_t u = ci[e];
    uint32_t kind = 0;
    if (mode == kCheckUp) {
        if (u > v && !row_contains(rp, ci, u, v)) kind = kErrAsym;
    } else {
        if (u >= n) kind = kErrColRange;
        else if (u == v) kind = kErrSelfLoop;
        else if (e > beg && ci[e - 1] >= u) kind = kErrOrder;
        else if (mode == kCheckAll && !row_contains(rp, ci, u, v)) kind = kErrAsym;
        if (mode == kCheckShape && u < n) a[u > v ? 0 : 1] += 1;
    }
    if (kind) atomicMin(err, ((unsigned long long)v << 32) | ((unsigned long long)(e - beg) << 3) | kind);
}

// One wave per row.  In the first two modes rows longer than kLongRow are left
// to k_validate_long (the first pass lists them in defer, count *ndefer), so no
// wave walks a hub row alone; kCheckAll takes every row.
__global__ void k_validate_cols(const uint32_t* __restrict__ rp, const uint32_t* __restrict__ ci,
                                uint32_t n, unsigned long long* err, unsigned long long* counts, int mode,
                                uint32_t* __restrict__ defer, uint32_t* __restrict__ ndefer)
{
    const uint32_t lane = lane_id();
    const size_t waves = (size_t)gridDim.x * (blockDim.x / 64);
    unsigned long long a[2] = {0, 0};
    for (size_t v = (size_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); v < n; v += waves) {
        uint32_t beg = rp[v], end = rp[v + 1];
        if (mode != kCheckAll && end - beg > kLongRow) {
            if (mode == kCheckShape && lane == 0) defer[atomicAdd(ndefer, 1u)] = (uint32_t)v;
            continue;
        }
        for (uint32_t e = beg + lane; e < end; e += 64) check_arc(rp, ci, n, (uint32_t)v, beg, e, mode, err, a);
    }
    if (mode == kCheckShape) block_add2(a, counts);
}

// The deferred long rows of the first two modes, one workgroup per row.
__global__ void k_validate_long(const uint32_t* __restrict__ rp, const uint32_t* __restrict__ ci, uint32_t n,
                                unsigned long long* err, unsigned long long* counts, int mode,
                                const uint32_t* __restrict__ defer, const uint32_t* __restrict__ ndefer)
{
    unsigned long long a[2] = {0, 0};
    const uint32_t cnt = *ndefer;
    for (uint32_t i = blockIdx.x; i < cnt; i += gridDim.x) {
        const uint32_t v = defer[i];
        const uint32_t beg = rp[v], end = rp[v + 1];
        for (uint32_t e = beg + threadIdx.x; e < end; e += blockDim.x) check_arc(rp, ci, n, v, beg, e, mode, err, a);
    }
    if (mode == kCheckShape) block_add2(a, counts);
}

// ---- peel ----------------------------------------------------------------------
// Synchronous-round peel for the degeneracy order (Section II-D), driven from device memory: every step
// reads its counts from PeelState, so a fixed sequence of launches (captured
// once in a hipGraph) runs any number of rounds; a step after the last round
// does nothing.  One step: a new level when the frontier ran empty (minimum
// remaining degree k, then every remaining vertex of degree <= k), then one
// round of removals, then the bookkeeping.
struct PeelState {
    uint32_t k;            // current level
    uint32_t r;            // round number of the current frontier
    uint32_t n_alive;      // unselected vertices listed in alive[pa] (some may be removed since)
    uint32_t n_alive_next; // entries written to alive[pa ^ 1] by the level selection
    uint32_t n_cur;        // frontier size, in front[pf]
    uint32_t n_next;       // next frontier being written to front[pf ^ 1]
    uint32_t min_deg;      // minimum remaining degree (level selection)
    uint32_t need_level;   // the frontier ran empty: select a new level first
    uint32_t pa, pf;       // buffer parities
    uint32_t done, err;
    unsigned long long removed;
};

__global__ void k_peel_init(const uint32_t* __restrict__ rp, uint32_t n, uint32_t* __restrict__ deg,
                            uint32_t* __restrict__ round, uint32_t* __restrict__ alive,
                            unsigned long long* __restrict__ stats)
{
    uint32_t local_max = 0, local_iso = 0;
    for (size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (size_t)gridDim.x * blockDim.x) {
        uint32_t d = rp[v + 1] - rp[v];
        deg[v] = d;
        round[v] = kUnset;
        alive[v] = (uint32_t)v;
        local_max = max(local_max, d);
        local_iso += (d == 0);
    }
    for (int off = 32; off > 0; off >>= 1) {
        local_max = max(local_max, (uint32_t)__shfl_xor((int)local_max, off));
        local_iso += (uint32_t)__shfl_xor((int)local_iso, off);
    }
    if (lane_id() == 0) {
        atomicMax(&stats[0], (unsigned long long)local_max);
        atomicAdd(&stats[1], (unsigned long long)local_iso);
    }
}

struct PeelBufs {
    uint32_t* alive[2];
    uint32_t* front[2];
    uint32_t* big[2];  // single-launch peel: the frontier's vertices of degree > kPeelBigDeg
};

// A frontier vertex with more arcs than this has its arcs removed by every
// wave of the launch together rather than by one wave, so one hub does not
// leave its round waiting on a single wave's chain of atomics.
constexpr uint32_t kPeelBigDeg = 512;

__global__ void k_pd_level_min(PeelBufs b, const uint32_t* __restrict__ deg, const uint32_t* __restrict__ round,
                               PeelState* ps)
{
    if (ps->done || !ps->need_level) return;
    const uint32_t n_alive = ps->n_alive;
    const uint32_t* A = b.alive[ps->pa];
    uint32_t m = kUnset;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_alive;
         i += (size_t)gridDim.x * blockDim.x) {
        uint32_t v = A[i];
        if (round[v] == kUnset) m = min(m, deg[v]);
    }
    for (int off = 32; off > 0; off >>= 1) m = min(m, (uint32_t)__shfl_xor((int)m, off));
    if (lane_id() == 0 && m != kUnset) atomicMin(&ps->min_deg, m);
}

// The level's first frontier: every remaining vertex of degree <= k (round r,
// core k); the others are compacted into the other alive buffer.
__global__ void k_pd_level_select(PeelBufs b, const uint32_t* __restrict__ deg, uint32_t* __restrict__ round,
                                  uint32_t* __restrict__ core, PeelState* ps)
{
    if (ps->done || !ps->need_level) return;
    const uint32_t n_alive = ps->n_alive, k = max(ps->k, ps->min_deg), r = ps->r;
    const uint32_t* A = b.alive[ps->pa];
    uint32_t* A2 = b.alive[ps->pa ^ 1u];
    uint32_t* F = b.front[ps->pf];
    const uint32_t lane = lane_id();
    for (size_t base = (size_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); base < n_alive;
         base += (size_t)gridDim.x * blockDim.x) {
        size_t i = base + lane;
        uint32_t v = 0;
        bool sel = false, keep = false;
        if (i < n_alive) {
            v = A[i];
            if (round[v] == kUnset) {
                if (deg[v] <= k) sel = true;
                else keep = true;
            }
        }
        uint64_t ms = __ballot(sel), mk = __ballot(keep);
        uint32_t bs = 0, bk = 0;
        if (lane == 0) {
            if (ms) bs = atomicAdd(&ps->n_cur, (uint32_t)__popcll(ms));
            if (mk) bk = atomicAdd(&ps->n_alive_next, (uint32_t)__popcll(mk));
        }
        bs = __shfl(bs, 0);
        bk = __shfl(bk, 0);
        if (sel) {
            round[v] = r;
            core[v] = k;
            F[bs + prefix_popc(ms)] = v;
        }
        if (keep) A2[bk + prefix_popc(mk)] = v;
    }
}

// Remove the frontier: decrement remaining neighbours; a neighbour whose degree
// falls from k+1 to k joins the next round.  One wave per frontier vertex.
__global__ void k_pd_decrement(const uint32_t* __restrict__ rp, const uint32_t* __restrict__ ci, PeelBufs b,
                               uint32_t* __restrict__ deg, uint32_t* __restrict__ round, uint32_t* __restrict__ core,
                               PeelState* ps)
{
    if (ps->done) return;
    const uint32_t n_front = ps->n_cur;
    if (n_front == 0) return;
    const uint32_t k = ps->need_level ? max(ps->k, ps->min_deg) : ps->k;
    const uint32_t r_next = ps->r + 1;
    const uint32_t* F = b.front[ps->pf];
    uint32_t* F2 = b.front[ps->pf ^ 1u];
    const uint32_t lane = lane_id();
    const size_t waves = (size_t)gridDim.x * (blockDim.x / 64);
    for (size_t f = (size_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); f < n_front; f += waves) {
        uint32_t v = F[f];
        uint32_t beg = rp[v], end = rp[v + 1];
        for (uint32_t e0 = beg; e0 < end; e0 += 64) {
            uint32_t e = e0 + lane;
            bool joined = false;
            uint32_t u = 0;
            if (e < end) {
                u = ci[e];
                if (__hip_atomic_load(&round[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == kUnset) {
                    uint32_t old = atomicSub(&deg[u], 1u);
                    if (old == k + 1) {
                        joined = true;
                        __hip_atomic_store(&round[u], r_next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        core[u] = k;
                    }
                }
            }
            uint64_t m = __ballot(joined);
            uint32_t bo = 0;
            if (lane == 0 && m) bo = atomicAdd(&ps->n_next, (uint32_t)__popcll(m));
            bo = __shfl(bo, 0);
            if (joined) F2[bo + prefix_popc(m)] = u;
        }
    }
}

// Bookkeeping after a step (one thread): adopt the level, count the removed
// frontier, advance the round, swap frontiers, and decide what comes next.
__global__ void k_pd_advance(PeelState* ps, uint32_t n)
{
    if (threadIdx.x != 0 || ps->done) return;
    if (ps->need_level) {
        if (ps->min_deg == kUnset || ps->n_cur == 0) {
            ps->err = 1;
            ps->done = 1;
            return;
        }
        ps->k = max(ps->k, ps->min_deg);
        ps->pa ^= 1u;
        ps->n_alive = ps->n_alive_next;
        ps->n_alive_next = 0;
        ps->need_level = 0;
        ps->min_deg = kUnset;
    }
    ps->removed += ps->n_cur;
    ps->r += 1;
    ps->pf ^= 1u;
    ps->n_cur = ps->n_next;
    ps->n_next = 0;
    if (ps->n_cur == 0) {
        if (ps->removed >= n) ps->done = 1;
        else ps->need_level = 1;
    }
}

// ---- single-launch peel ----------------------------------------------------------
// The same rounds as the step kernels above in one launch: every workgroup is
// resident at once (cooperative launch) and the workgroups meet at a grid
// barrier after each phase.  Each workgroup keeps its own copy of the peel's
// bookkeeping (level, round, buffer parities, sizes) and updates it the same way
// from the shared counters after each barrier, so an ordinary round needs one
// barrier and a round that opens a new level three.  The counters of round r
// live in slot r % 3; workgroup 0 clears the slot of round r + 1 when round r
// starts (that slot was last read at the start of round r - 1, before every
// workgroup reached the barriers of round r - 1).
struct alignas(256) PeelSlot {
    uint32_t min_deg, n_front, n_alive, n_next, n_bfront, n_bnext;
};
// Grid barrier arrivals are counted in two levels (workgroups in groups of
// kBarrierGroup, then groups), each counter on its own 256-byte line, so the
// device-scope atomics of one barrier do not queue on a single address.
constexpr uint32_t kBarrierGroup = 16;
constexpr uint32_t kMaxBarrierGroups = 64;
struct alignas(256) BarrierCounter {
    uint32_t c;
};
struct PeelSync {
    BarrierCounter grp[kMaxBarrierGroups];  // arrivals per group of workgroups
    alignas(256) uint32_t count;  // groups arrived at the current barrier
    alignas(256) uint32_t gen;    // barrier generation
    alignas(256) uint32_t err;    // 1: a barrier wait timed out, 2: no remaining vertex, 4: round limit
    PeelSlot slot[3];
    alignas(256) uint32_t out_r, out_k, out_done;
};

// Grid barrier with a bounded wait: false when a wait ran past the deadline or
// another workgroup reported an error (then every workgroup leaves the kernel).
__device__ bool grid_barrier(PeelSync* ps, uint32_t nb, uint64_t deadline)
{
    __shared__ uint32_t ok_s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t ok = 1;
        const uint32_t g = __hip_atomic_load(&ps->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const uint32_t gi = blockIdx.x / kBarrierGroup;
        const uint32_t ngroups = (nb + kBarrierGroup - 1) / kBarrierGroup;
        const uint32_t gsize = min(kBarrierGroup, nb - gi * kBarrierGroup);
        bool last = false;
        const uint32_t in_group =
            __hip_atomic_fetch_add(&ps->grp[gi].c, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (in_group == gsize - 1) {
            // the group's last arrival resets its counter (no workgroup adds to
            // it again before the generation moves on) and arrives for it
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __hip_atomic_store(&ps->grp[gi].c, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const uint32_t arrived = __hip_atomic_fetch_add(&ps->count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            last = arrived == ngroups - 1;
        }
        if (last) {
            __hip_atomic_store(&ps->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ps->gen, g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            while (__hip_atomic_load(&ps->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                if (__hip_atomic_load(&ps->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                    ok = 0;
                    break;
                }
                if (__builtin_amdgcn_s_memrealtime() > deadline) {
                    __hip_atomic_fetch_or(&ps->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        ok_s = ok;
    }
    __syncthreads();
    return ok_s != 0u;
}

__global__ void __launch_bounds__(256) k_peel_persistent(const uint32_t* __restrict__ rp,
                                                         const uint32_t* __restrict__ ci, uint32_t n, PeelBufs b,
                                                         uint32_t* __restrict__ deg, uint32_t* __restrict__ round,
                                                         uint32_t* __restrict__ core, PeelSync* ps,
                                                         uint64_t timeout_ticks)
{
    const uint32_t nb = gridDim.x;
    const uint64_t deadline = __builtin_amdgcn_s_memrealtime() + timeout_ticks;
    const uint32_t lane = lane_id();
    const bool leader = blockIdx.x == 0 && threadIdx.x == 0;
    const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t nthreads = (size_t)nb * blockDim.x;
    const size_t wid = (size_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const size_t nwaves = (size_t)nb * (blockDim.x / 64);
    // bookkeeping, identical in every workgroup
    uint32_t k = 0, r = 0, pa = 0, pf = 0, n_alive = n, n_cur = 0, n_big = 0;
    uint64_t removed = 0;
    bool need_level = n > 0;
    const uint64_t max_rounds = 2 * (uint64_t)n + 4;  // every round removes at least one vertex
    while (removed < n) {
        if (r >= max_rounds) {
            if (leader) __hip_atomic_fetch_or(&ps->err, 4u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        PeelSlot* sl = &ps->slot[r % 3];
        if (leader) {
            PeelSlot* nx = &ps->slot[(r + 1) % 3];
            __hip_atomic_store(&nx->min_deg, kUnset, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&nx->n_front, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&nx->n_alive, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&nx->n_next, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&nx->n_bfront, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&nx->n_bnext, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (need_level) {
            // the minimum remaining degree opens the level
            const uint32_t* A = b.alive[pa];
            uint32_t m = kUnset;
            for (size_t i = tid; i < n_alive; i += nthreads) {
                const uint32_t v = A[i];
                if (round[v] == kUnset) m = min(m, deg[v]);
            }
            for (int off = 32; off > 0; off >>= 1) m = min(m, (uint32_t)__shfl_xor((int)m, off));
            if (lane == 0 && m != kUnset) atomicMin(&sl->min_deg, m);
            if (!grid_barrier(ps, nb, deadline)) return;
            const uint32_t md = __hip_atomic_load(&sl->min_deg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (md == kUnset) {
                if (leader) __hip_atomic_fetch_or(&ps->err, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return;
            }
            k = max(k, md);
            // the level's first frontier: every remaining vertex of degree <= k
            uint32_t* A2 = b.alive[pa ^ 1u];
            uint32_t* F = b.front[pf];
            uint32_t* Bg = b.big[pf];
            // each wave takes chunks of cq x 64 entries (cq up to 16, fewer when
            // the list is short, so every wave has some): it counts its
            // selected, kept and big vertices first, reserves their places with
            // one atomic per counter, then decides again and writes (nothing
            // the decisions read changes in between)
            const uint32_t cq = (uint32_t)min<size_t>(16, max<size_t>(1, n_alive / (nwaves * 64)));
            auto decide = [&](size_t i, uint32_t& v, bool& sel, bool& keep, bool& big) {
                v = 0;
                sel = keep = big = false;
                if (i < n_alive) {
                    v = A[i];
                    if (round[v] == kUnset) {
                        if (deg[v] <= k) {
                            sel = true;
                            big = rp[v + 1] - rp[v] > kPeelBigDeg;
                        } else {
                            keep = true;
                        }
                    }
                }
            };
            for (size_t base = wid * (64 * cq); base < n_alive; base += nwaves * (64 * cq)) {
                uint32_t cs = 0, ck = 0, cb = 0;
                for (uint32_t q = 0; q < cq; ++q) {
                    uint32_t v;
                    bool sel, keep, big;
                    decide(base + q * 64 + lane, v, sel, keep, big);
                    cs += (uint32_t)__popcll(__ballot(sel));
                    ck += (uint32_t)__popcll(__ballot(keep));
                    cb += (uint32_t)__popcll(__ballot(big));
                }
                uint32_t bs = 0, bk = 0, bb = 0;
                if (lane == 0) {
                    if (cs) bs = atomicAdd(&sl->n_front, cs);
                    if (ck) bk = atomicAdd(&sl->n_alive, ck);
                    if (cb) bb = atomicAdd(&sl->n_bfront, cb);
                }
                bs = __shfl(bs, 0);
                bk = __shfl(bk, 0);
                bb = __shfl(bb, 0);
                for (uint32_t q = 0; q < cq; ++q) {
                    uint32_t v;
                    bool sel, keep, big;
                    decide(base + q * 64 + lane, v, sel, keep, big);
                    const uint64_t ms = __ballot(sel), mk = __ballot(keep), mb = __ballot(big);
                    if (sel) {
                        round[v] = r;
                        core[v] = k;
                        F[bs + prefix_popc(ms)] = v;
                    }
                    if (big) Bg[bb + prefix_popc(mb)] = v;
                    if (keep) A2[bk + prefix_popc(mk)] = v;
                    bs += (uint32_t)__popcll(ms);
                    bk += (uint32_t)__popcll(mk);
                    bb += (uint32_t)__popcll(mb);
                }
            }
            if (!grid_barrier(ps, nb, deadline)) return;
            n_cur = __hip_atomic_load(&sl->n_front, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            n_big = __hip_atomic_load(&sl->n_bfront, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            n_alive = __hip_atomic_load(&sl->n_alive, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            pa ^= 1u;
            need_level = false;
        }
        // remove the frontier: a neighbour whose degree falls from k + 1 to k
        // joins the next round.  One wave per frontier vertex of degree at
        // most kPeelBigDeg; the larger ones (listed apart) share the launch's
        // waves evenly, each splitting its arcs over its share.
        {
            const uint32_t* F = b.front[pf];
            const uint32_t* Bg = b.big[pf];
            uint32_t* F2 = b.front[pf ^ 1u];
            uint32_t* B2 = b.big[pf ^ 1u];
            const uint32_t r_next = r + 1;
            // arcs first + q * stride + lane (q < 4) at a time: the four
            // chains of loads and atomics overlap
            auto remove_arcs = [&](uint32_t end, uint64_t first, uint64_t stride) {
                for (uint64_t e0 = first; e0 < end; e0 += 4 * stride) {
                    uint32_t u[4], rd[4], old[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const uint64_t e = e0 + q * stride + lane;
                        u[q] = e < end ? ci[e] : kUnset;
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        rd[q] = u[q] != kUnset
                                    ? __hip_atomic_load(&round[u[q]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                    : 0u;
#pragma unroll
                    for (int q = 0; q < 4; ++q) old[q] = rd[q] == kUnset ? atomicSub(&deg[u[q]], 1u) : 0u;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const bool joined = rd[q] == kUnset && old[q] == k + 1;
                        bool big = false;
                        if (joined) {
                            big = rp[u[q] + 1] - rp[u[q]] > kPeelBigDeg;
                            __hip_atomic_store(&round[u[q]], r_next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            core[u[q]] = k;
                        }
                        const uint64_t m = __ballot(joined), mb = __ballot(big);
                        if (m) {
                            uint32_t bo = 0, bb = 0;
                            if (lane == 0) bo = atomicAdd(&sl->n_next, (uint32_t)__popcll(m));
                            if (lane == 0 && mb) bb = atomicAdd(&sl->n_bnext, (uint32_t)__popcll(mb));
                            bo = __shfl(bo, 0);
                            bb = __shfl(bb, 0);
                            if (joined) F2[bo + prefix_popc(m)] = u[q];
                            if (big) B2[bb + prefix_popc(mb)] = u[q];
                        }
                    }
                }
            };
            for (size_t f = wid; f < n_cur; f += nwaves) {
                const uint32_t v = F[f];
                const uint32_t beg = rp[v], end = rp[v + 1];
                if (end - beg > kPeelBigDeg) continue;
                remove_arcs(end, beg, 64);
            }
            if (n_big >= nwaves) {
                for (size_t i = wid; i < n_big; i += nwaves) {
                    const uint32_t v = Bg[i];
                    remove_arcs(rp[v + 1], rp[v], 64);
                }
            } else if (n_big > 0) {
                // waves wid = i, i + n_big, i + 2 n_big, ... share big vertex i
                const size_t i = wid % n_big, j = wid / n_big;
                const size_t c = (nwaves - 1 - i) / n_big + 1;
                const uint32_t v = Bg[i];
                remove_arcs(rp[v + 1], (uint64_t)rp[v] + j * 64, (uint64_t)c * 64);
            }
        }
        if (!grid_barrier(ps, nb, deadline)) return;
        removed += n_cur;
        r += 1;
        pf ^= 1u;
        n_cur = __hip_atomic_load(&sl->n_next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        n_big = __hip_atomic_load(&sl->n_bnext, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (n_cur == 0 && removed < n) need_level = true;
    }
    if (leader) {
        ps->out_r = r;
        ps->out_k = k;
        ps->out_done = 1u;
    }
}

// ---- per-member peel of a batch -------------------------------------------------------
// A batch loaded as one disjoint union peels every member graph on its own, one
// workgroup per member, with the member's remaining degrees, marks and frontier
// lists in LDS: the same synchronous rounds as above, but with each member's
// own levels, so a member takes its own number of rounds (the union's shared
// levels would make thousands of nearly empty rounds, each a grid-wide step).
// Round numbers restart at 0 in every member; core numbers are the member's.
// out[0] = largest number of rounds, out[1] = largest level.
constexpr uint32_t kMemberPeelCap = 8192;  // vertices per member (degrees then fit below 2^13)

__global__ void __launch_bounds__(512) k_peel_members(const uint32_t* __restrict__ rp,
                                                      const uint32_t* __restrict__ ci,
                                                      const uint32_t* __restrict__ voff, uint32_t ng,
                                                      uint32_t* __restrict__ round, uint32_t* __restrict__ core,
                                                      unsigned int* __restrict__ out)
{
    __shared__ uint32_t deg[kMemberPeelCap];
    __shared__ uint8_t mark[kMemberPeelCap];
    __shared__ uint16_t lst[2][kMemberPeelCap];
    __shared__ uint32_t cnt[2];
    __shared__ uint32_t red[16];
    const uint32_t tid = threadIdx.x, lane = lane_id(), wv = tid >> 6, nw = blockDim.x >> 6;
    for (uint32_t gi = blockIdx.x; gi < ng; gi += gridDim.x) {
        const uint32_t base = voff[gi], n = voff[gi + 1] - base;
        if (n == 0) continue;
        for (uint32_t i = tid; i < n; i += blockDim.x) {
            deg[i] = rp[base + i + 1] - rp[base + i];
            mark[i] = 0;
        }
        __syncthreads();
        uint32_t k = 0, r = 0, removed = 0, ncur = 0, pc = 0;
        while (removed < n) {
            if (ncur == 0) {
                // a new level: the smallest remaining degree, then every remaining
                // vertex of degree <= k
                uint32_t m = kUnset;
                for (uint32_t i = tid; i < n; i += blockDim.x)
                    if (!mark[i]) m = min(m, deg[i]);
                for (int off = 32; off > 0; off >>= 1) m = min(m, (uint32_t)__shfl_xor((int)m, off));
                if (lane == 0) red[wv] = m;
                if (tid == 0) cnt[pc] = 0;
                __syncthreads();
                m = kUnset;
                for (uint32_t w = 0; w < nw; ++w) m = min(m, red[w]);
                k = max(k, m);
                for (uint32_t i = tid; i < n; i += blockDim.x)
                    if (!mark[i] && deg[i] <= k) {
                        mark[i] = 1;
                        lst[pc][atomicAdd(&cnt[pc], 1u)] = (uint16_t)i;
                        round[base + i] = r;
                        core[base + i] = k;
                    }
                __syncthreads();
                ncur = cnt[pc];
            }
            // remove the frontier: a neighbour whose degree falls from k + 1 to k
            // joins the next round (one wave per frontier vertex)
            if (tid == 0) cnt[pc ^ 1u] = 0;
            __syncthreads();
            for (uint32_t f = wv; f < ncur; f += nw) {
                const uint32_t v = lst[pc][f];
                const uint32_t beg = rp[base + v], end = rp[base + v + 1];
                for (uint32_t e = beg + lane; e < end; e += 64) {
                    const uint32_t u = ci[e] - base;
                    if (u < n && !mark[u]) {  // u >= n only in an unvalidated, invalid batch
                        const uint32_t old = atomicSub(&deg[u], 1u);
                        if (old == k + 1) {
                            mark[u] = 1;
                            lst[pc ^ 1u][atomicAdd(&cnt[pc ^ 1u], 1u)] = (uint16_t)u;
                            round[base + u] = r + 1;
                            core[base + u] = k;
                        }
                    }
                }
            }
            __syncthreads();
            removed += ncur;
            r += 1;
            pc ^= 1u;
            ncur = cnt[pc];
            __syncthreads();  // every thread has read cnt[pc] before it is reset
        }
        if (tid == 0) {
            atomicMax(&out[0], r);
            atomicMax(&out[1], k);
        }
        __syncthreads();  // the LDS arrays are reused by the next member
    }
}

// ---- orientation -------------------------------------------------------------------
// rank[], core by rank, key by rank (key of the id local to the vertex's graph),
// and the graph of each rank when a batch is loaded as one disjoint union.
__global__ void k_rank_from_order(const uint32_t* __restrict__ order, uint32_t n, uint32_t* __restrict__ rank,
                                  const uint32_t* __restrict__ core, uint32_t* __restrict__ core_r,
                                  uint64_t* __restrict__ vkey, const uint32_t* __restrict__ gid_in,
                                  const uint32_t* __restrict__ voff, uint32_t* __restrict__ gid_r)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        uint32_t v = order[i];
        rank[v] = (uint32_t)i;
        core_r[i] = core[v];
        uint32_t local = v;
        if (gid_in) {
            uint32_t g = gid_in[v];
            local = v - voff[g];
            gid_r[i] = g;
        }
        vkey[i] = fmix64((uint64_t)local * kGamma + kGamma);
    }
}

// Per-graph maxima and isolated counts (u32 slots: max degree, degeneracy,
// max out-degree, max in-degree, isolated vertices).
__global__ void k_graph_meta(const uint32_t* __restrict__ op, const uint32_t* __restrict__ ip,
                             const uint32_t* __restrict__ core_r, const uint32_t* __restrict__ gid_r, uint32_t n,
                             unsigned int* __restrict__ meta)
{
    for (size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (size_t)gridDim.x * blockDim.x) {
        uint32_t g = gid_r[r];
        uint32_t out = op[r + 1] - op[r], in = ip[r + 1] - ip[r];
        unsigned int* m = meta + (size_t)g * 8;
        atomicMax(&m[0], out + in);
        atomicMax(&m[1], core_r[r]);
        atomicMax(&m[2], out);
        atomicMax(&m[3], in);
        if (out + in == 0) atomicAdd(&m[4], 1u);
    }
}

// Batch graph i must have row_ptr[0] == 0 and row_ptr[n_i] == nnz_i; the
// smallest offending graph index goes to *err (initially all ones).
__global__ void k_batch_ends(const uint32_t* __restrict__ rp_cat, const uint64_t* __restrict__ row_off,
                             const uint64_t* __restrict__ col_off, uint32_t ng, unsigned long long* err)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < ng; i += (size_t)gridDim.x * blockDim.x) {
        uint64_t first = row_off[i], last = row_off[i + 1] - 1;
        if (rp_cat[first] != 0u || (uint64_t)rp_cat[last] != col_off[i + 1] - col_off[i])
            atomicMin(err, (unsigned long long)i);
    }
}

// Union CSR of a batch: row pointers shifted by each graph's first arc, column
// ids by each graph's first vertex; a column outside its own graph is an error.
__global__ void k_union_rows(const uint32_t* __restrict__ rp_cat, const uint64_t* __restrict__ row_off,
                             const uint64_t* __restrict__ col_off, const uint32_t* __restrict__ voff,
                             const uint32_t* __restrict__ gid_in, uint32_t n, uint32_t* __restrict__ urp)
{
    for (size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (size_t)gridDim.x * blockDim.x) {
        uint32_t g = gid_in[v];
        urp[v] = rp_cat[row_off[g] + (v - voff[g])] + (uint32_t)col_off[g];
    }
}

__global__ void k_union_cols(const uint32_t* __restrict__ ci_cat, const uint32_t* __restrict__ urp,
                             const uint32_t* __restrict__ gid_in, const uint32_t* __restrict__ voff,
                             const uint32_t* __restrict__ nloc, uint32_t n, uint32_t* __restrict__ uci,
                             unsigned long long* err)
{
    const uint32_t lane = lane_id();
    const size_t waves = (size_t)gridDim.x * (blockDim.x / 64);
    for (size_t v = (size_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); v < n; v += waves) {
        uint32_t g = gid_in[v];
        uint32_t beg = urp[v], end = urp[v + 1];
        for (uint32_t e = beg + lane; e < end; e += 64) {
            uint32_t c = ci_cat[e];
            if (c >= nloc[g]) {
                atomicMin(err, ((unsigned long long)v << 32) | ((unsigned long long)(e - beg) << 3) | kErrColRange);
                c = 0;
            }
            uci[e] = c + voff[g];
        }
    }
}

// one wave per input vertex: out/in degree in rank space
// Out- and in-degree in the order of every vertex (one wave per row; rows
// longer than kLongRow are listed in defer for k_orient_count_long) and their
// maxima (maxes[0], maxes[1]).
__device__ inline void block_max2(uint32_t m0, uint32_t m1, unsigned int* maxes)
{
    __shared__ uint32_t part[2][16];
    if (lane_id() == 0) {
        part[0][threadIdx.x >> 6] = m0;
        part[1][threadIdx.x >> 6] = m1;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        uint32_t t = 0;
        for (uint32_t k = 0; k < blockDim.x / 64; ++k) t = max(t, part[threadIdx.x][k]);
        if (t) atomicMax(&maxes[threadIdx.x], t);
    }
}

__global__ void k_orient_count(const uint32_t* __restrict__ rp, const uint32_t* __restrict__ ci, uint32_t n,
                               const uint32_t* __restrict__ rank, uint32_t* __restrict__ outdeg,
                               uint32_t* __restrict__ indeg, unsigned int* __restrict__ maxes,
                               uint32_t* __restrict__ defer, uint32_t* __restrict__ ndefer)
{
    const uint32_t lane = lane_id();
    const size_t waves = (size_t)gridDim.x * (blockDim.x / 64);
    uint32_t max_out = 0, max_in = 0;
    for (size_t v = (size_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); v < n; v += waves) {
        uint32_t beg = rp[v], end = rp[v + 1];
        if (end - beg > kLongRow) {
            if (lane == 0) defer[atomicAdd(ndefer, 1u)] = (uint32_t)v;
            continue;
        }
        uint32_t rv = rank[v];
        uint32_t cnt = 0;
        for (uint32_t e = beg + lane; e < end; e += 64) cnt += rank[ci[e]] > rv;
        for (int off = 32; off > 0; off >>= 1) cnt += (uint32_t)__shfl_xor((int)cnt, off);
        uint32_t in = (end - beg) - cnt;
        if (lane == 0) {
            outdeg[rv] = cnt;
            indeg[rv] = in;
        }
        max_out = max(max_out, cnt);
        max_in = max(max_in, in);
    }
    block_max2(max_out, max_in, maxes);
}

// The deferred long rows, one workgroup per row.
__global__ void k_orient_count_long(const uint32_t* __restrict__ rp, const uint32_t* __restrict__ ci,
                                    const uint32_t* __restrict__ rank, uint32_t* __restrict__ outdeg,
                                    uint32_t* __restrict__ indeg, unsigned int* __restrict__ maxes,
                                    const uint32_t* __restrict__ defer, const uint32_t* __restrict__ ndefer)
{
    __shared__ uint32_t part[16];
    uint32_t max_out = 0, max_in = 0;
    const uint32_t total = *ndefer;
    for (uint32_t i = blockIdx.x; i < total; i += gridDim.x) {
        const uint32_t v = defer[i];
        const uint32_t beg = rp[v], end = rp[v + 1], rv = rank[v];
        uint32_t cnt = 0;
        for (uint32_t e = beg + threadIdx.x; e < end; e += blockDim.x) cnt += rank[ci[e]] > rv;
        for (int off = 32; off > 0; off >>= 1) cnt += (uint32_t)__shfl_xor((int)cnt, off);
        if (lane_id() == 0) part[threadIdx.x >> 6] = cnt;
        __syncthreads();
        uint32_t out = 0;
        for (uint32_t k = 0; k < blockDim.x / 64; ++k) out += part[k];
        __syncthreads();
        if (threadIdx.x == 0) {
            outdeg[rv] = out;
            indeg[rv] = (end - beg) - out;
        }
        max_out = max(max_out, out);
        max_in = max(max_in, (end - beg) - out);
    }
    block_max2(max_out, max_in, maxes);
}

__global__ void k_orient_fill(const uint32_t* __restrict__ rp, const uint32_t* __restrict__ ci, uint32_t n,
                              const uint32_t* __restrict__ rank, const uint32_t* __restrict__ op,
                              const uint32_t* __restrict__ ip, uint32_t* __restrict__ oc,
                              uint32_t* __restrict__ ic)
{
    const uint32_t lane = lane_id();
    const size_t waves = (size_t)gridDim.x * (blockDim.x / 64);
    for (size_t v = (size_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); v < n; v += waves) {
        uint32_t beg = rp[v], end = rp[v + 1];
        if (end - beg > kLongRow) continue;  // k_orient_fill_long
        uint32_t rv = rank[v];
        uint32_t po = op[rv], pi = ip[rv];
        for (uint32_t e0 = beg; e0 < end; e0 += 64) {
            uint32_t e = e0 + lane;
            bool valid = e < end;
            uint32_t ru = valid ? rank[ci[e]] : 0u;
            bool later = valid && ru > rv;
            bool earlier = valid && ru < rv;
            uint64_t ml = __ballot(later), me = __ballot(earlier);
            if (later) oc[po + prefix_popc(ml)] = ru;
            if (earlier) ic[pi + prefix_popc(me)] = ru;
            po += (uint32_t)__popcll(ml);
            pi += (uint32_t)__popcll(me);
        }
    }
}

// The rows longer than kLongRow (listed by k_orient_count), one workgroup per
// row, 256 arcs at a time; entries keep the input order, as in k_orient_fill.
__global__ void __launch_bounds__(256) k_orient_fill_long(const uint32_t* __restrict__ rp,
                                                          const uint32_t* __restrict__ ci,
                                                          const uint32_t* __restrict__ rank,
                                                          const uint32_t* __restrict__ op,
                                                          const uint32_t* __restrict__ ip,
                                                          uint32_t* __restrict__ oc, uint32_t* __restrict__ ic,
                                                          const uint32_t* __restrict__ defer,
                                                          const uint32_t* __restrict__ ndefer)
{
    __shared__ uint32_t cnt[2][4];
    const uint32_t lane = lane_id(), wv = threadIdx.x >> 6;
    const uint32_t total = *ndefer;
    for (uint32_t i = blockIdx.x; i < total; i += gridDim.x) {
        const uint32_t v = defer[i];
        const uint32_t beg = rp[v], end = rp[v + 1], rv = rank[v];
        uint32_t po = op[rv], pi = ip[rv];
        for (uint64_t e0 = beg; e0 < end; e0 += 256) {
            const uint64_t e = e0 + threadIdx.x;
            const bool valid = e < end;
            const uint32_t ru = valid ? rank[ci[e]] : 0u;
            const bool later = valid && ru > rv, earlier = valid && ru < rv;
            const uint64_t ml = __ballot(later), me = __ballot(earlier);
            if (lane == 0) {
                cnt[0][wv] = (uint32_t)__popcll(ml);
                cnt[1][wv] = (uint32_t)__popcll(me);
            }
            __syncthreads();
            uint32_t bl = po, be = pi;
            for (uint32_t w = 0; w < wv; ++w) {
                bl += cnt[0][w];
                be += cnt[1][w];
            }
            if (later) oc[bl + prefix_popc(ml)] = ru;
            if (earlier) ic[be + prefix_popc(me)] = ru;
            for (uint32_t w = 0; w < 4; ++w) {
                po += cnt[0][w];
                pi += cnt[1][w];
            }
            __syncthreads();
        }
    }
}

// Sort every out-row ascending (rows are at most kRowSortCap long).  One wave
// per row, bitonic network in LDS.
constexpr int kRowSortCap = 4096;

__global__ void __launch_bounds__(64) k_sort_rows(const uint32_t* __restrict__ op, uint32_t n,
                                                  uint32_t* __restrict__ oc)
{
    __shared__ uint32_t buf[kRowSortCap];
    const uint32_t lane = lane_id();
    for (size_t r = blockIdx.x; r < n; r += gridDim.x) {
        uint32_t beg = op[r], end = op[r + 1];
        uint32_t len = end - beg;
        if (len <= 1) continue;
        uint32_t m = 2;
        while (m < len) m <<= 1;
        for (uint32_t i = lane; i < m; i += 64) buf[i] = i < len ? oc[beg + i] : 0xFFFFFFFFu;
        __syncthreads();
        for (uint32_t k = 2; k <= m; k <<= 1) {
            for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                for (uint32_t i = lane; i < m; i += 64) {
                    uint32_t l = i ^ j;
                    if (l > i) {
                        uint32_t a = buf[i], b = buf[l];
                        bool up = (i & k) == 0;
                        if ((a > b) == up) {
                            buf[i] = b;
                            buf[l] = a;
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (uint32_t i = lane; i < len; i += 64) oc[beg + i] = buf[i];
        __syncthreads();
    }
}

}  // namespace

namespace {

const void* hmisc_zero()
{
    static const uint64_t z[4] = {0, 0, 0, 0};
    return z;
}

// The peel as one cooperative launch (k_peel_persistent).  peeled = false
// leaves the caller to run the step kernels: the device does not support
// cooperative launches, the launch was refused, or a barrier wait timed out.
mce_status peel_single_launch(const uint32_t* rp, const uint32_t* ci, uint32_t n, PeelBufs pb, uint32_t* deg,
                              uint32_t* round, uint32_t* core, hipStream_t s, PeelState& hs, bool& peeled)
{
    peeled = false;
    int dev = 0, coop = 0, cus = 0, per_cu = 0;
    MCE_HIP_TRY(hipGetDevice(&dev));
    MCE_HIP_TRY(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    MCE_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (!coop || cus <= 0) return MCE_OK;
    MCE_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k_peel_persistent),
                                                             256, 0));
    per_cu = std::min(per_cu, 2);
    if (per_cu < 1) return MCE_OK;
    const uint32_t nb = std::min((uint32_t)(per_cu * cus), kBarrierGroup * kMaxBarrierGroups);
    DevBuf sync;
    mce_status st;
    if ((st = sync.alloc(sizeof(PeelSync))) != MCE_OK) return st;
    PeelSync h0;
    std::memset(&h0, 0, sizeof(h0));
    for (auto& sl : h0.slot) sl.min_deg = kUnset;
    MCE_HIP_TRY(hipMemcpyAsync(sync.p, &h0, sizeof(h0), hipMemcpyHostToDevice, s));
    PeelSync* dsync = sync.as<PeelSync>();
    uint64_t ticks = 30ull * 100000000ull;  // 30 s of the 100 MHz device clock per barrier wait
    void* args[] = {(void*)&rp, (void*)&ci, (void*)&n, (void*)&pb, (void*)&deg, (void*)&round, (void*)&core,
                    (void*)&dsync, (void*)&ticks};
    hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_peel_persistent), dim3(nb), dim3(256),
                                              args, 0, s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return MCE_OK;
    }
    PeelSync out;
    MCE_HIP_TRY(hipMemcpyAsync(&out, dsync, sizeof(out), hipMemcpyDeviceToHost, s));
    MCE_HIP_TRY(hipStreamSynchronize(s));
    if (out.err & 1u) return MCE_OK;
    if (out.err & 2u) {
        set_error("internal: peel found no remaining vertex");
        return MCE_ERR_DEVICE;
    }
    if ((out.err & 4u) || !out.out_done) {
        set_error("internal: peel did not finish within 2n + 4 rounds");
        return MCE_ERR_DEVICE;
    }
    hs.r = out.out_r;
    hs.k = out.out_k;
    peeled = true;
    return MCE_OK;
}

}  // namespace

mce_status preprocess_graph(const uint32_t* rp, const uint32_t* ci, uint32_t n, uint64_t nnz,
                            bool validate, hipStream_t s, Oriented& g, const uint32_t* gid_in,
                            const uint32_t* voff, uint32_t ngraphs, uint32_t max_member_n)
{
    mce_status st;
    g.n = n;
    g.nnz = nnz;
    if (nnz >= (1ull << 32)) {
        set_error("nnz must be below 2^32 (uint32 CSR)");
        return MCE_ERR_UNSUPPORTED;
    }
    DevBuf misc;
    if ((st = misc.alloc(256)) != MCE_OK) return st;
    unsigned long long* dmisc = misc.as<unsigned long long>();
    uint64_t hmisc[32];

    if (validate) {
        uint64_t init = ~0ull;
        MCE_HIP_TRY(hipMemcpyAsync(dmisc, &init, 8, hipMemcpyHostToDevice, s));
        k_validate_rowptr<<<blocks_for((size_t)n + 1, 256), 256, 0, s>>>(rp, n, nnz, dmisc);
        MCE_HIP_TRY(hipGetLastError());
        MCE_HIP_TRY(hipMemcpyAsync(hmisc, dmisc, 8, hipMemcpyDeviceToHost, s));
        MCE_HIP_TRY(hipStreamSynchronize(s));
        if (hmisc[0] != ~0ull) {
            set_error("invalid graph: row_ptr not monotone / row_ptr[0] != 0 / row_ptr[n] != nnz at row " +
                      std::to_string(hmisc[0] >> 32));
            return MCE_ERR_INVALID_GRAPH;
        }
        {
            uint64_t z[3] = {0, 0, 0};
            MCE_HIP_TRY(hipMemcpyAsync(dmisc + 1, z, 24, hipMemcpyHostToDevice, s));
        }
        DevBuf defer;
        if ((st = defer.alloc(((size_t)nnz / kLongRow + 1) * 4)) != MCE_OK) return st;
        uint32_t* ndefer = reinterpret_cast<uint32_t*>(dmisc + 3);
        k_validate_cols<<<blocks_for(n, 4, 16384), 256, 0, s>>>(rp, ci, n, dmisc, dmisc + 1, kCheckShape,
                                                                  defer.as<uint32_t>(), ndefer);
        MCE_HIP_TRY(hipGetLastError());
        k_validate_long<<<kLongBlocks, 256, 0, s>>>(rp, ci, n, dmisc, dmisc + 1, kCheckShape, defer.as<uint32_t>(),
                                                    ndefer);
        MCE_HIP_TRY(hipGetLastError());
        MCE_HIP_TRY(hipMemcpyAsync(hmisc, dmisc, 24, hipMemcpyDeviceToHost, s));
        MCE_HIP_TRY(hipStreamSynchronize(s));
        bool name_arc = hmisc[0] == ~0ull && hmisc[1] != hmisc[2];
        if (hmisc[0] == ~0ull && !name_arc) {
            // equal counts: the reverse of every up arc decides symmetry
            k_validate_cols<<<blocks_for(n, 4, 16384), 256, 0, s>>>(rp, ci, n, dmisc, nullptr, kCheckUp,
                                                                     nullptr, nullptr);
            MCE_HIP_TRY(hipGetLastError());
            k_validate_long<<<kLongBlocks, 256, 0, s>>>(rp, ci, n, dmisc, nullptr, kCheckUp, defer.as<uint32_t>(),
                                                        ndefer);
            MCE_HIP_TRY(hipGetLastError());
            MCE_HIP_TRY(hipMemcpyAsync(hmisc, dmisc, 8, hipMemcpyDeviceToHost, s));
            MCE_HIP_TRY(hipStreamSynchronize(s));
            name_arc = hmisc[0] != ~0ull;
        }
        if (name_arc) {
            // asymmetric: name the first arc (in row, position order) without a reverse
            uint64_t init2 = ~0ull;
            MCE_HIP_TRY(hipMemcpyAsync(dmisc, &init2, 8, hipMemcpyHostToDevice, s));
            k_validate_cols<<<blocks_for(n, 4, 16384), 256, 0, s>>>(rp, ci, n, dmisc, nullptr, kCheckAll,
                                                                     nullptr, nullptr);
            MCE_HIP_TRY(hipGetLastError());
            MCE_HIP_TRY(hipMemcpyAsync(hmisc, dmisc, 8, hipMemcpyDeviceToHost, s));
            MCE_HIP_TRY(hipStreamSynchronize(s));
            if (hmisc[0] == ~0ull) {
                set_error("invalid graph: asymmetric (the numbers of arcs in the two directions differ)");
                return MCE_ERR_INVALID_GRAPH;
            }
        }
        if (hmisc[0] != ~0ull) {
            static const char* kinds[] = {"", "row_ptr", "column out of range", "row not strictly increasing",
                                          "self-loop", "asymmetric (missing reverse arc)"};
            uint32_t kind = (uint32_t)(hmisc[0] & 7u);
            set_error(std::string("invalid graph: ") + kinds[kind < 6 ? kind : 0] + " at row " +
                      std::to_string(hmisc[0] >> 32) + " position " +
                      std::to_string((hmisc[0] & 0xFFFFFFFFull) >> 3));
            return MCE_ERR_INVALID_GRAPH;
        }
    }

    // ---- peel
    DevBuf deg, alive_a, alive_b, front_a, front_b, big_a, big_b, psb;
    size_t nn = n ? n : 1;
    if ((st = deg.alloc(nn * 4)) != MCE_OK) return st;
    if ((st = alive_a.alloc(nn * 4)) != MCE_OK) return st;
    if ((st = alive_b.alloc(nn * 4)) != MCE_OK) return st;
    if ((st = front_a.alloc(nn * 4)) != MCE_OK) return st;
    if ((st = front_b.alloc(nn * 4)) != MCE_OK) return st;
    // at most nnz / (kPeelBigDeg + 1) vertices have more arcs than kPeelBigDeg
    const size_t nbig = std::min<size_t>(nn, nnz / (kPeelBigDeg + 1) + 1);
    if ((st = big_a.alloc(nbig * 4)) != MCE_OK) return st;
    if ((st = big_b.alloc(nbig * 4)) != MCE_OK) return st;
    if ((st = g.core.alloc(nn * 4)) != MCE_OK) return st;
    if ((st = g.round.alloc(nn * 4)) != MCE_OK) return st;
    if ((st = psb.alloc(sizeof(PeelState))) != MCE_OK) return st;
    PeelState* ps = psb.as<PeelState>();
    uint32_t* dcore = g.core.as<uint32_t>();
    uint32_t* dround = g.round.as<uint32_t>();

    {
        uint64_t z[4] = {0, 0, 0, 0};
        MCE_HIP_TRY(hipMemcpyAsync(dmisc, z, 32, hipMemcpyHostToDevice, s));
        PeelState p0{};
        p0.n_alive = n;
        p0.min_deg = kUnset;
        p0.need_level = n ? 1u : 0u;
        p0.done = n ? 0u : 1u;
        MCE_HIP_TRY(hipMemcpyAsync(ps, &p0, sizeof(p0), hipMemcpyHostToDevice, s));
    }
    if (n) {
        k_peel_init<<<blocks_for(n, 256, 4096), 256, 0, s>>>(rp, n, deg.as<uint32_t>(), dround,
                                                              alive_a.as<uint32_t>(), dmisc);
        MCE_HIP_TRY(hipGetLastError());
    }
    MCE_HIP_TRY(hipMemcpyAsync(hmisc, dmisc, 16, hipMemcpyDeviceToHost, s));
    MCE_HIP_TRY(hipStreamSynchronize(s));
    g.max_degree = (uint32_t)hmisc[0];
    g.n_isolated = hmisc[1];

    PeelState hs{};
    PeelBufs pb;
    pb.alive[0] = alive_a.as<uint32_t>();
    pb.alive[1] = alive_b.as<uint32_t>();
    pb.front[0] = front_a.as<uint32_t>();
    pb.front[1] = front_b.as<uint32_t>();
    pb.big[0] = big_a.as<uint32_t>();
    pb.big[1] = big_b.as<uint32_t>();
    bool peeled = n == 0;
    g.peel_mode = 0;
    if (n && !g.peel_steps && voff && ngraphs > 1 && max_member_n <= kMemberPeelCap) {
        // a batch of small graphs: every member peels on its own, one workgroup each
        int dev = 0, cus = 0;
        MCE_HIP_TRY(hipGetDevice(&dev));
        MCE_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        MCE_HIP_TRY(hipMemcpyAsync(dmisc + 16, hmisc_zero(), 8, hipMemcpyHostToDevice, s));
        unsigned int* mout = reinterpret_cast<unsigned int*>(dmisc + 16);
        k_peel_members<<<std::max(1u, std::min(ngraphs, 2u * (uint32_t)std::max(cus, 1))), 512, 0, s>>>(
            rp, ci, voff, ngraphs, dround, dcore, mout);
        MCE_HIP_TRY(hipGetLastError());
        unsigned int hout[2] = {0, 0};
        MCE_HIP_TRY(hipMemcpyAsync(hout, mout, 8, hipMemcpyDeviceToHost, s));
        MCE_HIP_TRY(hipStreamSynchronize(s));
        hs.r = hout[0];
        hs.k = hout[1];
        peeled = true;
        g.peel_mode = 3;
    }
    if (!peeled && !g.peel_steps) {
        // one launch with grid barriers; falls back to the step kernels when the
        // device cannot run it (no cooperative launch, or a barrier timed out)
        if ((st = peel_single_launch(rp, ci, n, pb, deg.as<uint32_t>(), dround, dcore, s, hs, peeled)) != MCE_OK)
            return st;
        if (peeled) g.peel_mode = 1;
        else {
            // start over: the attempt may have removed vertices
            MCE_HIP_TRY(hipMemcpyAsync(dmisc, hmisc_zero(), 32, hipMemcpyHostToDevice, s));
            PeelState p0{};
            p0.n_alive = n;
            p0.min_deg = kUnset;
            p0.need_level = 1u;
            MCE_HIP_TRY(hipMemcpyAsync(ps, &p0, sizeof(p0), hipMemcpyHostToDevice, s));
            k_peel_init<<<blocks_for(n, 256, 4096), 256, 0, s>>>(rp, n, deg.as<uint32_t>(), dround,
                                                                  alive_a.as<uint32_t>(), dmisc);
            MCE_HIP_TRY(hipGetLastError());
            MCE_HIP_TRY(hipStreamSynchronize(s));
        }
    }
    if (!peeled) {
        g.peel_mode = 2;
        // kPeelSteps steps captured once, replayed until the peel is done
        const unsigned gsel = blocks_for(n, 256, 1024), gdec = blocks_for(n, 4, 2048);
        hipStream_t cs = nullptr;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        auto cleanup = [&]() {
            if (exec) (void)hipGraphExecDestroy(exec);
            if (graph) (void)hipGraphDestroy(graph);
            if (cs) (void)hipStreamDestroy(cs);
        };
        hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            for (int i = 0; i < kPeelSteps; ++i) {
                k_pd_level_min<<<gsel, 256, 0, cs>>>(pb, deg.as<uint32_t>(), dround, ps);
                k_pd_level_select<<<gsel, 256, 0, cs>>>(pb, deg.as<uint32_t>(), dround, dcore, ps);
                k_pd_decrement<<<gdec, 256, 0, cs>>>(rp, ci, pb, deg.as<uint32_t>(), dround, dcore, ps);
                k_pd_advance<<<1, 64, 0, cs>>>(ps, n);
            }
            hipError_t e2 = hipStreamEndCapture(cs, &graph);
            e = e2 != hipSuccess ? e2 : hipGetLastError();
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            cleanup();
            set_error(std::string("peel graph capture: ") + hipGetErrorString(e));
            return MCE_ERR_DEVICE;
        }
        // two replays in flight: the state after replay i is read while
        // replay i + 1 runs (pinned copies, one event each), so the device
        // does not wait for the host between replays; a replay after the
        // last round does nothing
        PeelState* hst = nullptr;
        hipEvent_t ev[2] = {nullptr, nullptr};
        if (e == hipSuccess) e = hipHostMalloc((void**)&hst, 2 * sizeof(PeelState), hipHostMallocDefault);
        for (int b = 0; b < 2 && e == hipSuccess; ++b) e = hipEventCreateWithFlags(&ev[b], hipEventDisableTiming);
        auto replay = [&](int b) {
            hipError_t r = hipGraphLaunch(exec, s);
            if (r == hipSuccess) r = hipMemcpyAsync(&hst[b], ps, sizeof(PeelState), hipMemcpyDeviceToHost, s);
            if (r == hipSuccess) r = hipEventRecord(ev[b], s);
            return r;
        };
        // every step removes a frontier or selects one, so 2n steps suffice
        const size_t max_replays = 2 * (size_t)n / kPeelSteps + 4;
        bool finished = false;
        if (e == hipSuccess) e = replay(0);
        for (size_t i = 0, b = 0; e == hipSuccess && i < max_replays; ++i, b ^= 1) {
            e = replay((int)(b ^ 1));
            if (e == hipSuccess) e = hipEventSynchronize(ev[b]);
            if (e == hipSuccess && hst[b].done) {
                finished = true;
                break;
            }
        }
        if (e == hipSuccess && !finished) e = hipErrorUnknown;
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e == hipSuccess) hs = *(const PeelState*)(hst[0].done ? &hst[0] : &hst[1]);
        for (int b = 0; b < 2; ++b)
            if (ev[b]) (void)hipEventDestroy(ev[b]);
        if (hst) (void)hipHostFree(hst);
        cleanup();
        if (e != hipSuccess) {
            set_error(std::string("peel: ") + hipGetErrorString(e));
            return MCE_ERR_DEVICE;
        }
        if (hs.err) {
            set_error("internal: peel found no remaining vertex");
            return MCE_ERR_DEVICE;
        }
    }
    const uint32_t r = hs.r;
    const uint32_t degen = hs.k;
    g.rounds = r;
    g.degeneracy = degen;
    alive_a.release();
    alive_b.release();
    front_b.release();
    big_a.release();
    big_b.release();

    // ---- order by (round, id): stable radix sort of ids keyed by round
    DevBuf order, keys;
    if ((st = order.alloc(nn * 4)) != MCE_OK) return st;
    if ((st = keys.alloc(nn * 4)) != MCE_OK) return st;
    MCE_HIP_TRY(hipMemcpyAsync(keys.p, dround, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
    iota_u32(order.as<uint32_t>(), n, s);
    int bits = 0;
    while (bits < 32 && (r >> bits) != 0) ++bits;
    {
        RadixTmp rt;
        if ((st = stable_sort_pairs_u32(keys.as<uint32_t>(), order.as<uint32_t>(), n, bits, rt, s)) != MCE_OK)
            return st;
        MCE_HIP_TRY(hipStreamSynchronize(s));
    }
    keys.release();

    // ---- rank, keys, core by rank
    DevBuf& rank = g.rank;
    if ((st = rank.alloc(nn * 4)) != MCE_OK) return st;
    if ((st = g.core_r.alloc(nn * 4)) != MCE_OK) return st;
    if ((st = g.vkey.alloc(nn * 8)) != MCE_OK) return st;
    g.ngraphs = std::max(ngraphs, 1u);
    if (gid_in) {
        if ((st = g.gid.alloc(nn * 4)) != MCE_OK) return st;
    }
    if (n) {
        k_rank_from_order<<<blocks_for(n, 256, 4096), 256, 0, s>>>(order.as<uint32_t>(), n, rank.as<uint32_t>(),
                                                                    dcore, g.core_r.as<uint32_t>(),
                                                                    g.vkey.as<uint64_t>(), gid_in, voff,
                                                                    gid_in ? g.gid.as<uint32_t>() : nullptr);
        MCE_HIP_TRY(hipGetLastError());
    }

    // ---- orient
    DevBuf outdeg, indeg;
    if ((st = outdeg.alloc((nn + 1) * 4)) != MCE_OK) return st;
    if ((st = indeg.alloc((nn + 1) * 4)) != MCE_OK) return st;
    if ((st = g.op.alloc((nn + 1) * 4)) != MCE_OK) return st;
    if ((st = g.ip.alloc((nn + 1) * 4)) != MCE_OK) return st;
    {
        uint64_t z[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        MCE_HIP_TRY(hipMemcpyAsync(dmisc, z, 64, hipMemcpyHostToDevice, s));
    }
    DevBuf odefer;
    if ((st = odefer.alloc(((size_t)g.nnz / kLongRow + 1) * 4)) != MCE_OK) return st;
    if (n) {
        uint32_t* ndefer = reinterpret_cast<uint32_t*>(dmisc) + 12;
        k_orient_count<<<blocks_for(n, 4, 16384), 256, 0, s>>>(rp, ci, n, rank.as<uint32_t>(),
                                                                outdeg.as<uint32_t>(), indeg.as<uint32_t>(),
                                                                reinterpret_cast<unsigned int*>(dmisc),
                                                                odefer.as<uint32_t>(), ndefer);
        MCE_HIP_TRY(hipGetLastError());
        k_orient_count_long<<<kLongBlocks, 256, 0, s>>>(rp, ci, rank.as<uint32_t>(), outdeg.as<uint32_t>(),
                                                  indeg.as<uint32_t>(), reinterpret_cast<unsigned int*>(dmisc),
                                                  odefer.as<uint32_t>(), ndefer);
        MCE_HIP_TRY(hipGetLastError());
    }
    DevBuf stmp;
    if ((st = stmp.alloc(scan_tmp_words(nn + 1) * 8)) != MCE_OK) return st;
    uint32_t* dtot = reinterpret_cast<uint32_t*>(dmisc) + 8;
    if ((st = exclusive_scan_u32(outdeg.as<uint32_t>(), g.op.as<uint32_t>(), n, dtot, stmp.as<uint64_t>(), s)) !=
        MCE_OK)
        return st;
    if ((st = exclusive_scan_u32(indeg.as<uint32_t>(), g.ip.as<uint32_t>(), n, dtot + 1, stmp.as<uint64_t>(), s)) !=
        MCE_OK)
        return st;
    // row_ptr[n] = totals
    MCE_HIP_TRY(hipMemcpyAsync(g.op.as<uint32_t>() + n, dtot, 4, hipMemcpyDeviceToDevice, s));
    MCE_HIP_TRY(hipMemcpyAsync(g.ip.as<uint32_t>() + n, dtot + 1, 4, hipMemcpyDeviceToDevice, s));
    uint32_t hm[10];
    MCE_HIP_TRY(hipMemcpyAsync(hm, dmisc, 40, hipMemcpyDeviceToHost, s));
    MCE_HIP_TRY(hipStreamSynchronize(s));
    g.max_out = hm[0];
    g.max_in = hm[1];
    uint64_t half_out = hm[8], half_in = hm[9];
    if (half_out + half_in != nnz) {
        set_error("internal: orientation lost arcs");
        return MCE_ERR_DEVICE;
    }
    if (g.max_out >= (uint32_t)kRowSortCap) {
        set_error("degeneracy order gives a first-level P of " + std::to_string(g.max_out) +
                  " vertices; at most " + std::to_string(kRowSortCap - 1) + " are supported");
        return MCE_ERR_UNSUPPORTED;
    }
    if ((st = g.oc.alloc((half_out + 1) * 4)) != MCE_OK) return st;
    if ((st = g.ic.alloc((half_in + 1) * 4)) != MCE_OK) return st;
    if (n) {
        k_orient_fill<<<blocks_for(n, 4, 16384), 256, 0, s>>>(rp, ci, n, rank.as<uint32_t>(), g.op.as<uint32_t>(),
                                                               g.ip.as<uint32_t>(), g.oc.as<uint32_t>(),
                                                               g.ic.as<uint32_t>());
        MCE_HIP_TRY(hipGetLastError());
        k_orient_fill_long<<<kLongBlocks, 256, 0, s>>>(rp, ci, rank.as<uint32_t>(), g.op.as<uint32_t>(),
                                                       g.ip.as<uint32_t>(), g.oc.as<uint32_t>(), g.ic.as<uint32_t>(),
                                                       odefer.as<uint32_t>(),
                                                       reinterpret_cast<uint32_t*>(dmisc) + 12);
        MCE_HIP_TRY(hipGetLastError());
        k_sort_rows<<<blocks_for(n, 1, 65536), 64, 0, s>>>(g.op.as<uint32_t>(), n, g.oc.as<uint32_t>());
        MCE_HIP_TRY(hipGetLastError());
    }
    // perm = order
    g.perm.release();
    g.perm.p = order.p;
    g.perm.bytes = order.bytes;
    order.p = nullptr;
    order.bytes = 0;
    if (!gid_in) {
        g.meta.assign(1, GraphMeta());
        GraphMeta& m = g.meta[0];
        m.n = n;
        m.nnz = nnz;
        m.max_degree = g.max_degree;
        m.degeneracy = g.degeneracy;
        m.max_out = g.max_out;
        m.max_in = g.max_in;
        m.n_isolated = g.n_isolated;
        m.voff = 0;
    } else if (n) {
        DevBuf dmeta;
        if ((st = dmeta.alloc((size_t)g.ngraphs * 32)) != MCE_OK) return st;
        fill_u32(dmeta.as<uint32_t>(), 0, (size_t)g.ngraphs * 8, s);
        k_graph_meta<<<blocks_for(n, 256, 4096), 256, 0, s>>>(g.op.as<uint32_t>(), g.ip.as<uint32_t>(),
                                                               g.core_r.as<uint32_t>(), g.gid.as<uint32_t>(), n,
                                                               dmeta.as<unsigned int>());
        MCE_HIP_TRY(hipGetLastError());
        std::vector<uint32_t> hm((size_t)g.ngraphs * 8);
        MCE_HIP_TRY(hipMemcpyAsync(hm.data(), dmeta.p, hm.size() * 4, hipMemcpyDeviceToHost, s));
        MCE_HIP_TRY(hipStreamSynchronize(s));
        g.meta.resize(g.ngraphs);
        for (uint32_t i = 0; i < g.ngraphs; ++i) {
            GraphMeta& m = g.meta[i];
            m.max_degree = hm[i * 8 + 0];
            m.degeneracy = hm[i * 8 + 1];
            m.max_out = hm[i * 8 + 2];
            m.max_in = hm[i * 8 + 3];
            m.n_isolated = hm[i * 8 + 4];
        }
    }
    MCE_HIP_TRY(hipStreamSynchronize(s));
    return MCE_OK;
}

mce_status preprocess_batch(const uint32_t* rp_cat, const uint32_t* ci_cat, const uint64_t* row_off,
                            const uint64_t* col_off, uint32_t ng, bool validate, bool on_dev, hipStream_t s,
                            Oriented& g)
{
    mce_status st;
    std::vector<uint32_t> voff(ng + 1), nloc(ng);
    uint64_t N = 0, NNZ = col_off[ng] - col_off[0];
    for (uint32_t i = 0; i < ng; ++i) {
        uint64_t ni = row_off[i + 1] - row_off[i] - 1;
        voff[i] = (uint32_t)N;
        nloc[i] = (uint32_t)ni;
        if (validate && !on_dev) {
            uint64_t nnzi = col_off[i + 1] - col_off[i];
            if (rp_cat[row_off[i]] != 0 || (uint64_t)rp_cat[row_off[i] + ni] != nnzi) {
                set_error("invalid graph " + std::to_string(i) + ": row_ptr[0] != 0 or row_ptr[n] != nnz");
                return MCE_ERR_INVALID_GRAPH;
            }
        }
        N += ni;
    }
    voff[ng] = (uint32_t)N;
    if (N >= 0xFFFFFFFFull || NNZ >= (1ull << 32)) {
        set_error("batch too large for uint32 ids");
        return MCE_ERR_UNSUPPORTED;
    }
    std::vector<uint32_t> gid_in(N ? N : 1);
    for (uint32_t i = 0; i < ng; ++i)
        std::fill(gid_in.begin() + voff[i], gid_in.begin() + voff[i + 1], i);
    DevBuf d_rp, d_ci, d_roff, d_coff, d_voff, d_nloc, d_gid, urp, uci, err;
    size_t rp_words = row_off[ng] - row_off[0];
    if (!on_dev) {
        if ((st = d_rp.alloc(rp_words * 4)) != MCE_OK) return st;
        if ((st = d_ci.alloc((NNZ ? NNZ : 1) * 4)) != MCE_OK) return st;
    }
    if ((st = d_roff.alloc((size_t)(ng + 1) * 8)) != MCE_OK) return st;
    if ((st = d_coff.alloc((size_t)(ng + 1) * 8)) != MCE_OK) return st;
    if ((st = d_voff.alloc((size_t)(ng + 1) * 4)) != MCE_OK) return st;
    if ((st = d_nloc.alloc((size_t)ng * 4)) != MCE_OK) return st;
    if ((st = d_gid.alloc(gid_in.size() * 4)) != MCE_OK) return st;
    if ((st = urp.alloc((N + 1) * 4)) != MCE_OK) return st;
    if ((st = uci.alloc((NNZ ? NNZ : 1) * 4)) != MCE_OK) return st;
    if ((st = err.alloc(8)) != MCE_OK) return st;
    std::vector<uint64_t> roff(ng + 1), coff(ng + 1);
    for (uint32_t i = 0; i <= ng; ++i) {
        roff[i] = row_off[i] - row_off[0];
        coff[i] = col_off[i] - col_off[0];
    }
    const uint32_t* src_rp = on_dev ? rp_cat + row_off[0] : d_rp.as<uint32_t>();
    const uint32_t* src_ci = on_dev ? (NNZ ? ci_cat + col_off[0] : nullptr) : d_ci.as<uint32_t>();
    if (!on_dev) {
        MCE_HIP_TRY(hipMemcpyAsync(d_rp.p, rp_cat + row_off[0], rp_words * 4, hipMemcpyHostToDevice, s));
        if (NNZ) MCE_HIP_TRY(hipMemcpyAsync(d_ci.p, ci_cat + col_off[0], NNZ * 4, hipMemcpyHostToDevice, s));
    }
    MCE_HIP_TRY(hipMemcpyAsync(d_roff.p, roff.data(), (ng + 1) * 8, hipMemcpyHostToDevice, s));
    MCE_HIP_TRY(hipMemcpyAsync(d_coff.p, coff.data(), (ng + 1) * 8, hipMemcpyHostToDevice, s));
    MCE_HIP_TRY(hipMemcpyAsync(d_voff.p, voff.data(), (ng + 1) * 4, hipMemcpyHostToDevice, s));
    MCE_HIP_TRY(hipMemcpyAsync(d_nloc.p, nloc.data(), ng * 4, hipMemcpyHostToDevice, s));
    MCE_HIP_TRY(hipMemcpyAsync(d_gid.p, gid_in.data(), gid_in.size() * 4, hipMemcpyHostToDevice, s));
    uint64_t einit = ~0ull;
    MCE_HIP_TRY(hipMemcpyAsync(err.p, &einit, 8, hipMemcpyHostToDevice, s));
    uint32_t nnz32 = (uint32_t)NNZ;
    MCE_HIP_TRY(hipMemcpyAsync(urp.as<uint32_t>() + N, &nnz32, 4, hipMemcpyHostToDevice, s));
    if (validate && on_dev) {
        // per graph: row_ptr[0] == 0 and row_ptr[n] == nnz, checked where the arrays live
        k_batch_ends<<<blocks_for(ng, 256, 4096), 256, 0, s>>>(src_rp, d_roff.as<uint64_t>(), d_coff.as<uint64_t>(),
                                                               ng, err.as<unsigned long long>());
        MCE_HIP_TRY(hipGetLastError());
        uint64_t berr = 0;
        MCE_HIP_TRY(hipMemcpyAsync(&berr, err.p, 8, hipMemcpyDeviceToHost, s));
        MCE_HIP_TRY(hipStreamSynchronize(s));
        if (berr != ~0ull) {
            set_error("invalid graph " + std::to_string((uint32_t)berr) + ": row_ptr[0] != 0 or row_ptr[n] != nnz");
            return MCE_ERR_INVALID_GRAPH;
        }
    }
    if (N) {
        k_union_rows<<<blocks_for(N, 256, 8192), 256, 0, s>>>(src_rp, d_roff.as<uint64_t>(),
                                                              d_coff.as<uint64_t>(), d_voff.as<uint32_t>(),
                                                              d_gid.as<uint32_t>(), (uint32_t)N, urp.as<uint32_t>());
        MCE_HIP_TRY(hipGetLastError());
        if (validate) {
            // row pointers must be monotone before any column range is read
            k_validate_rowptr<<<blocks_for(N + 1, 256), 256, 0, s>>>(urp.as<uint32_t>(), (uint32_t)N, NNZ,
                                                                     err.as<unsigned long long>());
            MCE_HIP_TRY(hipGetLastError());
            uint64_t rerr = 0;
            MCE_HIP_TRY(hipMemcpyAsync(&rerr, err.p, 8, hipMemcpyDeviceToHost, s));
            MCE_HIP_TRY(hipStreamSynchronize(s));
            if (rerr != ~0ull) {
                uint32_t v = (uint32_t)(rerr >> 32);
                uint32_t gi = v < N ? gid_in[v] : ng - 1;
                set_error("invalid graph " + std::to_string(gi) + ": row_ptr not monotone at row " +
                          std::to_string(v - voff[gi]));
                return MCE_ERR_INVALID_GRAPH;
            }
        }
        k_union_cols<<<blocks_for(N, 4, 16384), 256, 0, s>>>(src_ci, urp.as<uint32_t>(),
                                                             d_gid.as<uint32_t>(), d_voff.as<uint32_t>(),
                                                             d_nloc.as<uint32_t>(), (uint32_t)N, uci.as<uint32_t>(),
                                                             err.as<unsigned long long>());
        MCE_HIP_TRY(hipGetLastError());
    }
    uint64_t herr = 0;
    MCE_HIP_TRY(hipMemcpyAsync(&herr, err.p, 8, hipMemcpyDeviceToHost, s));
    MCE_HIP_TRY(hipStreamSynchronize(s));
    d_rp.release();
    d_ci.release();
    if (validate && herr != ~0ull) {
        uint32_t v = (uint32_t)(herr >> 32);
        uint32_t gi = gid_in[v];
        set_error("invalid graph " + std::to_string(gi) + ": column out of range at row " +
                  std::to_string(v - voff[gi]));
        return MCE_ERR_INVALID_GRAPH;
    }
    st = preprocess_graph(urp.as<uint32_t>(), uci.as<uint32_t>(), (uint32_t)N, NNZ, validate, s, g,
                          d_gid.as<uint32_t>(), d_voff.as<uint32_t>(), ng,
                          ng ? *std::max_element(nloc.begin(), nloc.end()) : 0u);
    if (st != MCE_OK) return st;
    for (uint32_t i = 0; i < ng; ++i) {
        g.meta[i].n = nloc[i];
        g.meta[i].nnz = col_off[i + 1] - col_off[i];
        g.meta[i].voff = voff[i];
    }
    return MCE_OK;
}

}  // namespace mce
