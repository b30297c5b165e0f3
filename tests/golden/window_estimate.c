/* Knuth's estimator of the size of a backtracking tree (D. E. Knuth,
 * "Estimating the efficiency of backtrack programs", Math. Comp. 29, 1975),
 * applied to the Bron-Kerbosch search with pivoting below one first-level
 * root (Algorithm 3): a probe walks from the root to a leaf choosing every
 * child uniformly, and the product of the branching factors along the walk,
 * counted when the leaf is a maximal clique (P and X empty), is an unbiased
 * estimate of the number of maximal cliques the root reports; the sum of
 * the products at every node of the walk estimates the number of search-tree
 * nodes.  Any pivot in
 * P u X gives the same set of maximal cliques; the probe takes the one in P
 * with most neighbours in P.  Used only to size core windows of the
 * workloads (how many cliques a window beyond the tested one holds); it
 * shares nothing with the library.
 *
 * P lives as a bitset over the root's later neighbours U (adjacency rows
 * built once per root); X is split into the part inside U (a bitset) and the
 * earlier neighbours of the root still adjacent to every vertex chosen so far
 * (a list, tested by binary search in the sorted rows of the input CSR).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static uint64_t mix(uint64_t z)
{
    /* SplitMix64 finaliser (Steele, Lea and Flood, OOPSLA 2014) */
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static int has_edge(const uint32_t* rp, const uint32_t* ci, uint32_t a, uint32_t b)
{
    uint32_t lo = rp[a], hi = rp[a + 1];
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (ci[mid] == b) return 1;
        if (ci[mid] < b) lo = mid + 1;
        else hi = mid;
    }
    return 0;
}

/* est[i] = mean over `probes` walks of the clique estimate for root roots[i],
 * nodes[i] the same for the tree size (the root counted as one node).
 * pos[v] = position of v in the vertex order (later neighbours = larger pos).
 * Returns 0, or -1 when a root has more than 4096 later neighbours. */
int window_estimate(uint32_t n, const uint32_t* rp, const uint32_t* ci, const uint32_t* pos,
                    const uint32_t* roots, uint32_t nroots, uint32_t probes, uint64_t seed, double* est,
                    double* nodes)
{
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (uint32_t ri = 0; ri < nroots; ++ri) {
        const uint32_t v = roots[ri];
        const uint32_t deg = rp[v + 1] - rp[v];
        uint32_t* U = malloc(sizeof(uint32_t) * (deg + 1));
        uint32_t* X0 = malloc(sizeof(uint32_t) * (deg + 1));
        uint32_t m = 0, nx0 = 0;
        for (uint32_t e = rp[v]; e < rp[v + 1]; ++e) {
            uint32_t u = ci[e];
            if (pos[u] > pos[v]) U[m++] = u;
            else X0[nx0++] = u;
        }
        if (m > 4096) {
#pragma omp atomic write
            bad = 1;
            est[ri] = 0;
            nodes[ri] = 0;
            free(U);
            free(X0);
            continue;
        }
        const uint32_t W = (m + 63) / 64 ? (m + 63) / 64 : 1;
        uint64_t* row = calloc((size_t)m * W + 1, sizeof(uint64_t));
        for (uint32_t a = 0; a < m; ++a)
            for (uint32_t b = a + 1; b < m; ++b)
                if (has_edge(rp, ci, U[a], U[b])) {
                    row[(size_t)a * W + b / 64] |= 1ull << (b % 64);
                    row[(size_t)b * W + a / 64] |= 1ull << (a % 64);
                }
        uint64_t* P = malloc(sizeof(uint64_t) * W);
        uint64_t* XP = malloc(sizeof(uint64_t) * W);
        uint64_t* B = malloc(sizeof(uint64_t) * W);
        uint32_t* XX = malloc(sizeof(uint32_t) * (nx0 + 1));
        uint64_t state = mix(seed ^ ((uint64_t)v * 0x9E3779B97F4A7C15ULL));
        double acc = 0, acc_nodes = 0;
        for (uint32_t t = 0; t < probes; ++t) {
            for (uint32_t w = 0; w < W; ++w) {
                P[w] = 0;
                XP[w] = 0;
            }
            for (uint32_t a = 0; a < m; ++a) P[a / 64] |= 1ull << (a % 64);
            memcpy(XX, X0, sizeof(uint32_t) * nx0);
            uint32_t nxx = nx0;
            double weight = 1;
            for (;;) {
                acc_nodes += weight;
                int pempty = 1;
                for (uint32_t w = 0; w < W; ++w)
                    if (P[w]) pempty = 0;
                if (pempty) {
                    int xempty = nxx == 0;
                    for (uint32_t w = 0; w < W && xempty; ++w)
                        if (XP[w]) xempty = 0;
                    if (xempty) acc += weight;
                    break;
                }
                /* pivot: the vertex of P with most neighbours in P (first on ties) */
                uint32_t piv = 0, best = 0;
                int found = 0;
                for (uint32_t a = 0; a < m; ++a) {
                    if (!((P[a / 64] >> (a % 64)) & 1)) continue;
                    uint32_t sc = 0;
                    for (uint32_t w = 0; w < W; ++w) sc += (uint32_t)__builtin_popcountll(P[w] & row[(size_t)a * W + w]);
                    if (!found || sc > best) {
                        best = sc;
                        piv = a;
                        found = 1;
                    }
                }
                uint32_t nb = 0;
                for (uint32_t w = 0; w < W; ++w) {
                    B[w] = P[w] & ~row[(size_t)piv * W + w];
                    nb += (uint32_t)__builtin_popcountll(B[w]);
                }
                /* child number k (ascending order): earlier branches move from P to X */
                state += 0x9E3779B97F4A7C15ULL;
                const uint32_t k = (uint32_t)(mix(state) % nb);
                uint32_t seen = 0, b = 0;
                for (uint32_t a = 0; a < m; ++a) {
                    if (!((B[a / 64] >> (a % 64)) & 1)) continue;
                    if (seen == k) {
                        b = a;
                        break;
                    }
                    P[a / 64] &= ~(1ull << (a % 64));
                    XP[a / 64] |= 1ull << (a % 64);
                    ++seen;
                }
                weight *= nb;
                for (uint32_t w = 0; w < W; ++w) {
                    P[w] &= row[(size_t)b * W + w];
                    XP[w] &= row[(size_t)b * W + w];
                }
                uint32_t keep = 0;
                for (uint32_t i = 0; i < nxx; ++i)
                    if (has_edge(rp, ci, XX[i], U[b])) XX[keep++] = XX[i];
                nxx = keep;
            }
        }
        est[ri] = probes ? acc / probes : 0;
        nodes[ri] = probes ? acc_nodes / probes : 0;
        free(P);
        free(XP);
        free(B);
        free(XX);
        free(row);
        free(U);
        free(X0);
    }
    return bad ? -1 : 0;
}
