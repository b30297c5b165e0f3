/*
 * CPU oracle for exact maximal clique enumeration -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  The product path never calls it.  It shares no code
 * with the GPU library: no headers, no helpers, no tables.
 *
 * What it computes (the plain definition, Section II-A of the paper): the set
 * of all maximal cliques of a simple undirected graph, i.e. vertex sets that
 * are pairwise adjacent and contained in no larger such set; exact, no
 * approximation.  Reported as count, histogram by clique size, and an
 * order-independent 64-bit hash H = sum over cliques C of h(C) mod 2^64.
 *
 * How (in the paper's order): degeneracy ordering (Section II-D, "Degeneracy
 * Ordering"), independent first-level subtrees (Algorithm 3), each explored
 * by Bron-Kerbosch with pivoting (Algorithm 2) where the pivot maximises
 * |P intersect N(u)| over u in P union X (Tomita's rule, Section II-C).  Sets
 * are sorted vertex-id arrays; nothing is blocked, fused or reordered.
 *
 * Core window: only roots v with core(v) <= max_root_core are explored.  The
 * degeneracy order is non-decreasing in core number, and Algorithm 3 reports
 * each maximal clique from its earliest vertex, which therefore has the
 * smallest core number in the clique; the window thus yields exactly the
 * maximal cliques whose minimum core number is <= max_root_core, for any
 * core-sorted order.
 *
 * Hash (not in the paper; a fixed definition both sides implement on their
 * own): fmix is the SplitMix64 output finaliser (Steele, Lea and Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014);
 * key(v) = fmix((v+1)*gamma) is the v-th output of SplitMix64 seeded 0,
 * v the input vertex id; h(C) = fmix(sum_{v in C} key(v) + |C|*gamma).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GAMMA 0x9E3779B97F4A7C15ULL

static uint64_t fmix(uint64_t z)
{
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ULL;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return z;
}

uint64_t oracle_key(uint64_t v) { return fmix(v * GAMMA + GAMMA); }

uint64_t oracle_clique_hash(const uint32_t* ids, uint32_t k)
{
    uint64_t s = 0;
    for (uint32_t i = 0; i < k; ++i) s += oracle_key(ids[i]);
    return fmix(s + (uint64_t)k * GAMMA);
}

/* ------------------------------------------------------------------ ordering */

/*
 * Degeneracy order and core numbers by the bucket algorithm of Batagelj and
 * Zaversnik ("An O(m) algorithm for cores decomposition of networks", 2003):
 * repeatedly take a vertex of minimum current degree.  order[i] is the i-th
 * vertex taken; core[v] its core number.  Each vertex has at most core[v]
 * neighbours later in the order, and core numbers never decrease along it.
 */
int oracle_degeneracy(uint32_t n, const uint32_t* rp, const uint32_t* ci,
                      uint32_t* order, uint32_t* core)
{
    if (n == 0) return 0;
    uint32_t* deg = malloc(sizeof(uint32_t) * n);
    uint32_t* pos = malloc(sizeof(uint32_t) * n);
    uint32_t md = 0;
    for (uint32_t v = 0; v < n; ++v) {
        deg[v] = rp[v + 1] - rp[v];
        if (deg[v] > md) md = deg[v];
    }
    uint32_t* bin = calloc((size_t)md + 1, sizeof(uint32_t));
    for (uint32_t v = 0; v < n; ++v) bin[deg[v]]++;
    uint32_t start = 0;
    for (uint32_t d = 0; d <= md; ++d) {
        uint32_t num = bin[d];
        bin[d] = start;
        start += num;
    }
    for (uint32_t v = 0; v < n; ++v) {
        pos[v] = bin[deg[v]];
        order[pos[v]] = v;
        bin[deg[v]]++;
    }
    for (uint32_t d = md; d >= 1; --d) bin[d] = bin[d - 1];
    bin[0] = 0;
    for (uint32_t i = 0; i < n; ++i) {
        uint32_t v = order[i];
        for (uint32_t e = rp[v]; e < rp[v + 1]; ++e) {
            uint32_t u = ci[e];
            if (deg[u] > deg[v]) {
                uint32_t du = deg[u], pu = pos[u];
                uint32_t pw = bin[du], w = order[pw];
                if (u != w) {
                    pos[u] = pw; order[pu] = w;
                    pos[w] = pu; order[pw] = u;
                }
                bin[du]++;
                deg[u]--;
            }
        }
    }
    for (uint32_t v = 0; v < n; ++v) core[v] = deg[v];
    free(deg); free(pos); free(bin);
    return 0;
}

/*
 * Synchronous-round peel, simulated sequentially.  k starts at 0; each round
 * removes, all at once, every remaining vertex whose remaining degree is at
 * most k, recording core = k and the round index; a round that would remove
 * nothing instead raises k to the minimum remaining degree (and is not
 * counted).  Returns the number of rounds.
 */
int64_t oracle_sync_peel(uint32_t n, const uint32_t* rp, const uint32_t* ci,
                         uint32_t* core, uint32_t* round_out)
{
    uint32_t* deg = malloc(sizeof(uint32_t) * (n ? n : 1));
    uint8_t* alive = malloc(n ? n : 1);
    uint32_t* live = malloc(sizeof(uint32_t) * (n ? n : 1));
    uint32_t* zset = malloc(sizeof(uint32_t) * (n ? n : 1));
    uint32_t nlive = n, k = 0, r = 0;
    for (uint32_t v = 0; v < n; ++v) {
        deg[v] = rp[v + 1] - rp[v];
        alive[v] = 1;
        live[v] = v;
    }
    while (nlive > 0) {
        uint32_t nz = 0, keep = 0;
        for (uint32_t i = 0; i < nlive; ++i) {
            uint32_t v = live[i];
            if (deg[v] <= k) zset[nz++] = v;
            else live[keep++] = v;
        }
        if (nz == 0) {
            uint32_t mn = UINT32_MAX;
            for (uint32_t i = 0; i < nlive; ++i)
                if (deg[live[i]] < mn) mn = deg[live[i]];
            k = mn;
            continue;
        }
        nlive = keep;
        for (uint32_t i = 0; i < nz; ++i) {
            uint32_t v = zset[i];
            core[v] = k;
            round_out[v] = r;
            alive[v] = 0;
        }
        for (uint32_t i = 0; i < nz; ++i) {
            uint32_t v = zset[i];
            for (uint32_t e = rp[v]; e < rp[v + 1]; ++e)
                if (alive[ci[e]]) deg[ci[e]]--;
        }
        r++;
    }
    free(deg); free(alive); free(live); free(zset);
    return (int64_t)r;
}

/* ------------------------------------------------------------ Bron-Kerbosch */

typedef struct {
    /* graph */
    const uint32_t* rp;
    const uint32_t* ci;
    /* per-thread bump arena for set storage */
    uint32_t* arena;
    size_t arena_cap, arena_top;
    int oom;
    /* current clique R */
    uint32_t* R;
    uint32_t rsize;
    /* accumulators */
    uint64_t count, hash, nodes;
    uint64_t* hist;
    uint32_t hist_len;
    uint32_t max_size;
    /* optional clique output */
    uint32_t* out_v;
    uint64_t out_vcap, out_vn;
    uint64_t* out_off;
    uint64_t out_ocap, out_on;
    int out_overflow;
} bk_state;

static uint32_t* arena_get(bk_state* s, size_t k)
{
    if (s->arena_top + k > s->arena_cap) {
        size_t nc = s->arena_cap * 2 + k + 1024;
        uint32_t* na = realloc(s->arena, nc * sizeof(uint32_t));
        if (!na) { s->oom = 1; return NULL; }
        s->arena = na;
        s->arena_cap = nc;
    }
    uint32_t* p = s->arena + s->arena_top;
    s->arena_top += k;
    return p;
}

/* is w in the sorted adjacency row of u? */
static int adjacent(const bk_state* s, uint32_t u, uint32_t w)
{
    uint32_t lo = s->rp[u], hi = s->rp[u + 1];
    while (lo < hi) {
        uint32_t mid = lo + (hi - lo) / 2;
        uint32_t x = s->ci[mid];
        if (x == w) return 1;
        if (x < w) lo = mid + 1; else hi = mid;
    }
    return 0;
}

static void report(bk_state* s)
{
    s->count += 1;
    s->hash += oracle_clique_hash(s->R, s->rsize);
    if (s->rsize < s->hist_len) s->hist[s->rsize] += 1;
    if (s->rsize > s->max_size) s->max_size = s->rsize;
    if (s->out_off) {
        if (s->out_on + 1 <= s->out_ocap && s->out_vn + s->rsize <= s->out_vcap) {
            memcpy(s->out_v + s->out_vn, s->R, sizeof(uint32_t) * s->rsize);
            s->out_vn += s->rsize;
            s->out_off[s->out_on++] = s->out_vn;
        } else {
            s->out_overflow = 1;
        }
    }
}

/*
 * Algorithm 2 (Bron-Kerbosch with pivoting).  P and X are sorted arrays held
 * in the arena at offsets po and xo (offsets, because the arena may grow and
 * move); the callee may overwrite them.
 */
#define AR(off) (s->arena + (off))
static void bk_pivot(bk_state* s, size_t po, uint32_t np, size_t xo, uint32_t nx)
{
    s->nodes += 1;
    if (np == 0 && nx == 0) {
        report(s);
        return;
    }
    if (np == 0) return;
    /* pivot: u in P union X maximising |P intersect N(u)|, ties -> smallest id */
    uint32_t pivot = UINT32_MAX;
    int64_t best = -1;
    for (int pass = 0; pass < 2; ++pass) {
        size_t so = pass == 0 ? po : xo;
        uint32_t ns = pass == 0 ? np : nx;
        for (uint32_t i = 0; i < ns; ++i) {
            uint32_t u = AR(so)[i];
            int64_t c = 0;
            for (uint32_t j = 0; j < np; ++j) c += adjacent(s, u, AR(po)[j]);
            if (c > best || (c == best && u < pivot)) { best = c; pivot = u; }
        }
    }
    /* frame: B (branch set), Pc/Xc (P and X as they change across the loop),
     * Pn/Xn (the child's P and X) */
    size_t mark = s->arena_top;
    if (!arena_get(s, (size_t)np * 3 + ((size_t)nx + np) * 2)) return;
    size_t bo = mark, pco = bo + np, xco = pco + np, pno = xco + nx + np, xno = pno + np;

    /* branch set: P - N(pivot), ascending id, fixed before the loop */
    uint32_t nb = 0;
    for (uint32_t i = 0; i < np; ++i)
        if (!adjacent(s, pivot, AR(po)[i])) AR(bo)[nb++] = AR(po)[i];
    memcpy(AR(pco), AR(po), sizeof(uint32_t) * np);
    memcpy(AR(xco), AR(xo), sizeof(uint32_t) * nx);
    uint32_t npc = np, nxc = nx;

    for (uint32_t bi = 0; bi < nb; ++bi) {
        uint32_t v = AR(bo)[bi];
        /* recursive call on R + {v}, P intersect N(v), X intersect N(v) */
        uint32_t npn = 0, nxn = 0;
        for (uint32_t i = 0; i < npc; ++i)
            if (adjacent(s, v, AR(pco)[i])) AR(pno)[npn++] = AR(pco)[i];
        for (uint32_t i = 0; i < nxc; ++i)
            if (adjacent(s, v, AR(xco)[i])) AR(xno)[nxn++] = AR(xco)[i];
        s->R[s->rsize++] = v;
        bk_pivot(s, pno, npn, xno, nxn);
        s->rsize--;
        if (s->oom) return;
        /* P = P - {v} */
        uint32_t w = 0;
        for (uint32_t i = 0; i < npc; ++i)
            if (AR(pco)[i] != v) AR(pco)[w++] = AR(pco)[i];
        npc = w;
        /* X = X union {v}, kept sorted */
        uint32_t* Xc = AR(xco);
        uint32_t j = nxc;
        while (j > 0 && Xc[j - 1] > v) { Xc[j] = Xc[j - 1]; --j; }
        Xc[j] = v;
        nxc++;
    }
    s->arena_top = mark;
}
#undef AR

typedef struct {
    uint64_t count, hash, nodes;
    uint64_t cliques_written, verts_written;
    uint32_t max_size;
    uint32_t degeneracy;
    int32_t status; /* 0 ok, 1 clique buffer overflow, -1 out of memory */
    int32_t threads;
} oracle_result;

/*
 * Algorithm 3 over a degeneracy order (the bucket order above, or given_order
 * when non-NULL), restricted to roots with core <= max_root_core (and, when
 * root_mask is given, to roots with a non-zero mask byte: used to time a
 * bounded sample and to compare per-root results).  hist[k] counts
 * cliques of size k for k < hist_len.  When clique_offsets is non-NULL the
 * cliques are also written out (input vertex ids; offsets are end positions)
 * and the run is single-threaded.
 */
int oracle_mce(uint32_t n, const uint32_t* rp, const uint32_t* ci,
               uint32_t max_root_core, int nthreads,
               uint64_t* hist, uint32_t hist_len,
               uint32_t* clique_verts, uint64_t vert_cap,
               uint64_t* clique_offsets, uint64_t off_cap,
               const uint8_t* root_mask, const uint32_t* given_order, oracle_result* out)
{
    memset(out, 0, sizeof(*out));
    if (hist) memset(hist, 0, sizeof(uint64_t) * hist_len);
    if (n == 0) return 0;
    uint32_t* order = malloc(sizeof(uint32_t) * n);
    uint32_t* core = malloc(sizeof(uint32_t) * n);
    uint32_t* pos = malloc(sizeof(uint32_t) * n);
    oracle_degeneracy(n, rp, ci, order, core);
    /* a caller-given order (any core-sorted order gives the same window) */
    if (given_order) memcpy(order, given_order, sizeof(uint32_t) * n);
    for (uint32_t i = 0; i < n; ++i) pos[order[i]] = i;
    uint32_t dmax = 0;
    for (uint32_t v = 0; v < n; ++v) if (core[v] > dmax) dmax = core[v];
    out->degeneracy = dmax;
    uint32_t hl = dmax + 2;

    if (clique_offsets) nthreads = 1;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#else
    nthreads = 1;
#endif
    uint64_t* th_hist = calloc((size_t)nthreads * hl, sizeof(uint64_t));
    uint64_t* th_cnt = calloc((size_t)nthreads * 3, sizeof(uint64_t));
    uint32_t* th_max = calloc((size_t)nthreads, sizeof(uint32_t));
    int err = 0, overflow = 0;
    uint64_t vn = 0, on = 0;

#ifdef _OPENMP
#pragma omp parallel num_threads(nthreads) reduction(| : err, overflow)
#endif
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        bk_state s;
        memset(&s, 0, sizeof(s));
        s.rp = rp;
        s.ci = ci;
        s.R = malloc(sizeof(uint32_t) * (hl + 1));
        s.hist = th_hist + (size_t)tid * hl;
        s.hist_len = hl;
        s.out_v = clique_verts;
        s.out_vcap = vert_cap;
        s.out_off = clique_offsets;
        s.out_ocap = off_cap;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
        for (int64_t i = 0; i < (int64_t)n; ++i) {
            uint32_t v = order[i];
            if (core[v] > max_root_core) continue;
            if (root_mask && !root_mask[v]) continue;
            uint32_t deg = rp[v + 1] - rp[v];
            s.arena_top = 0;
            if (!arena_get(&s, (size_t)deg * 2 + 1)) { err = 1; continue; }
            uint32_t* P = s.arena;
            uint32_t* X = s.arena + deg;
            uint32_t np = 0, nx = 0;
            for (uint32_t e = rp[v]; e < rp[v + 1]; ++e) {
                uint32_t u = ci[e];
                if (pos[u] > pos[v]) P[np++] = u;   /* N(v_i) after v_i */
                else X[nx++] = u;                   /* N(v_i) before v_i */
            }
            s.R[0] = v;
            s.rsize = 1;
            bk_pivot(&s, 0, np, (size_t)deg, nx);
            if (s.oom) err = 1;
        }
        th_cnt[tid * 3 + 0] = s.count;
        th_cnt[tid * 3 + 1] = s.hash;
        th_cnt[tid * 3 + 2] = s.nodes;
        th_max[tid] = s.max_size;
        if (s.out_overflow) overflow = 1;
        if (clique_offsets) { vn = s.out_vn; on = s.out_on; }
#ifdef _OPENMP
        if (tid == 0) out->threads = omp_get_num_threads();
#else
        out->threads = 1;
#endif
        free(s.arena);
        free(s.R);
    }
    out->cliques_written = on;
    out->verts_written = vn;
    for (int t = 0; t < nthreads; ++t) {
        out->count += th_cnt[t * 3 + 0];
        out->hash += th_cnt[t * 3 + 1];
        out->nodes += th_cnt[t * 3 + 2];
        if (th_max[t] > out->max_size) out->max_size = th_max[t];
        for (uint32_t k = 0; k < hl && k < hist_len; ++k) hist[k] += th_hist[(size_t)t * hl + k];
    }
    out->status = err ? -1 : (overflow ? 1 : 0);
    free(th_hist); free(th_cnt); free(th_max);
    free(order); free(core); free(pos);
    return out->status;
}

/* Number of threads an unconstrained run would use. */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
