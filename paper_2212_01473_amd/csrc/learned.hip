// Learned root ordering: cheap per-root features, a 4-64-64-64-1 MLP trained on
// the GPU (FP32 forward, backward and Adam) from subtree costs the plain
// enumeration measures, BF16 inference, and the work queue built from the
// predictions (roots in descending predicted cost, the costliest split into
// level-1 branch groups).  None of this changes which cliques are found: the
// queue is a permutation of the window's roots, and a split root's groups
// together cover exactly its level-1 branches.
#include "mce_internal.h"

#include <cmath>
#include <mutex>
#include <vector>

namespace mce {

namespace {

// Model layout (floats): W1[64][4], b1[64], W2[64][64], b2[64], W3[64][64],
// b3[64], W4[64], b4, mean[4], std[4].
constexpr int kIn = 4, kH = 64;
constexpr int oW1 = 0, ob1 = oW1 + kH * kIn, oW2 = ob1 + kH, ob2 = oW2 + kH * kH, oW3 = ob2 + kH,
              ob3 = oW3 + kH * kH, oW4 = ob3 + kH, ob4 = oW4 + kH, oMean = ob4 + 1, oStd = oMean + kIn,
              kModel = oStd + kIn;
static_assert(kModel == MCE_MODEL_FLOATS, "model layout");
constexpr int kTrainable = oMean;  // mean/std are fitted, not trained

unsigned blocks_for(size_t items, unsigned per_block, unsigned cap = 65536)
{
    size_t b = (items + per_block - 1) / per_block;
    if (b == 0) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

__device__ inline uint32_t lane_id() { return __lane_id(); }

// ---------------------------------------------------------------- features
// Per root v (rank): log1p(degree), log1p(core), log1p(2-hop count = sum of
// neighbour degrees), and the edge density of its later-neighbour set P.  The
// density is exact (edges inside P / C(|P|, 2); 0 when |P| < 2) when P has at
// most kDensityPairs pairs, else the fraction of adjacent pairs among
// kDensityPairs pairs of positions drawn from SplitMix64 seeded with the
// root's vertex key: x_t = output t, a = (x_t mod 2^32) mod |P|,
// b = (x_t >> 32) mod (|P| - 1) moved past a; the pair (P[min], P[max]) is
// adjacent iff P[max] is among the later neighbours of P[min].  One wave per
// root; its lanes test pairs (binary searches in the later-neighbour lists).
constexpr int kFeatWaves = 4;
constexpr uint32_t kDensityPairs = 256;
constexpr uint32_t kExactMaxP = 23;  // C(23, 2) = 253 <= kDensityPairs < C(24, 2)
static_assert(kExactMaxP * (kExactMaxP - 1) / 2 <= kDensityPairs &&
                  (kExactMaxP + 1) * kExactMaxP / 2 > kDensityPairs,
              "exact density exactly when C(|P|, 2) <= kDensityPairs");

__device__ inline uint64_t fmix64(uint64_t z)
{
    // SplitMix64 output finaliser (Steele, Lea and Flood, OOPSLA 2014).
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// Is x among the sorted later neighbours oc[beg, end)?
__device__ inline bool sorted_contains(const uint32_t* __restrict__ oc, uint32_t beg, uint32_t end, uint32_t x)
{
    while (beg < end) {
        const uint32_t mid = (beg + end) >> 1;
        const uint32_t y = oc[mid];
        if (y == x) return true;
        if (y < x) beg = mid + 1;
        else end = mid;
    }
    return false;
}

__global__ void __launch_bounds__(64 * kFeatWaves) k_features(const uint32_t* __restrict__ op,
                                                             const uint32_t* __restrict__ oc,
                                                             const uint32_t* __restrict__ ip,
                                                             const uint32_t* __restrict__ ic,
                                                             const uint32_t* __restrict__ core_r,
                                                             const uint32_t* __restrict__ deg,
                                                             const uint64_t* __restrict__ vkey,
                                                             const uint32_t* __restrict__ roots, uint32_t nr,
                                                             float* __restrict__ feat)
{
    const uint32_t lane = lane_id();
    const uint32_t wv = threadIdx.x >> 6;
    for (size_t k = (size_t)blockIdx.x * kFeatWaves + wv; k < nr; k += (size_t)gridDim.x * kFeatWaves) {
        const uint32_t v = roots[k];
        const uint32_t pb = op[v], np = op[v + 1] - pb;
        const uint32_t xb = ip[v], nx = ip[v + 1] - xb;
        // 2-hop count
        uint64_t two = 0;
        for (uint32_t i = lane; i < np + nx; i += 64) {
            const uint32_t u = i < np ? oc[pb + i] : ic[xb + i - np];
            two += deg[u];
        }
        // adjacent pairs inside P: all of them, or the sampled ones; a pair
        // (P[i], P[j]), i < j, is adjacent iff P[j] is a later neighbour of P[i]
        uint32_t hits = 0;
        if (np >= 2 && np <= kExactMaxP) {
            const uint32_t pairs = np * (np - 1) / 2;
            for (uint32_t t = lane; t < pairs; t += 64) {
                uint32_t i = 0, rem = t;  // pair t in row-major order over i
                while (rem >= np - 1 - i) {
                    rem -= np - 1 - i;
                    ++i;
                }
                const uint32_t u = oc[pb + i], w = oc[pb + i + 1 + rem];
                hits += sorted_contains(oc, op[u], op[u + 1], w);
            }
        } else if (np > kExactMaxP) {
            const uint64_t seed = vkey[v];
            for (uint32_t t = lane; t < kDensityPairs; t += 64) {
                const uint64_t x = fmix64(seed + (uint64_t)(t + 1) * kGamma);
                const uint32_t a = (uint32_t)x % np;
                uint32_t b = (uint32_t)(x >> 32) % (np - 1);
                if (b >= a) ++b;
                const uint32_t lo = min(a, b), hi = max(a, b);
                const uint32_t u = oc[pb + lo], w = oc[pb + hi];
                hits += sorted_contains(oc, op[u], op[u + 1], w);
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            two += __shfl_xor(two, off, 64);
            hits += (uint32_t)__shfl_xor((int)hits, off, 64);
        }
        if (lane == 0) {
            float* f = feat + (size_t)k * 4;
            f[0] = log1pf((float)(np + nx));
            f[1] = log1pf((float)core_r[v]);
            f[2] = log1pf((float)two);
            const double pairs = np <= kExactMaxP ? 0.5 * (double)np * (double)(np - 1) : (double)kDensityPairs;
            f[3] = np >= 2 ? (float)((double)hits / pairs) : 0.f;
        }
    }
}

// Degree of every vertex (later + earlier neighbours), by rank.
__global__ void k_degrees(const uint32_t* __restrict__ op, const uint32_t* __restrict__ ip, uint32_t n,
                          uint32_t* __restrict__ deg)
{
    for (size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (size_t)gridDim.x * blockDim.x)
        deg[v] = (op[v + 1] - op[v]) + (ip[v + 1] - ip[v]);
}

// Input ids to ranks; an id >= nv sets *err and maps to rank 0 (the call then
// fails before any feature is used).
__global__ void k_ids_to_ranks(const uint32_t* __restrict__ ids, uint32_t n, uint32_t nv,
                               const uint32_t* __restrict__ rank, uint32_t* __restrict__ out,
                               uint32_t* __restrict__ err)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        uint32_t v = ids[i];
        if (v >= nv) {
            atomicOr(err, 1u);
            v = 0;
        }
        out[i] = rank[v];
    }
}

// ---------------------------------------------------------------- BF16 inference
__device__ inline uint16_t to_bf16(float f)
{
    uint32_t b = __float_as_uint(f);
    b += 0x7FFFu + ((b >> 16) & 1u);  // round to nearest even
    return (uint16_t)(b >> 16);
}
__device__ inline float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline float bf16r(float f) { return from_bf16(to_bf16(f)); }

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline bf16x4 pack_bf16(float a, float b, float c, float d)
{
    bf16x4 v;
    v[0] = (short)to_bf16(a);
    v[1] = (short)to_bf16(b);
    v[2] = (short)to_bf16(c);
    v[3] = (short)to_bf16(d);
    return v;
}

// Weights, biases and activations rounded to BF16, sums accumulated in FP32.
// The 64x64 layers run on the matrix cores (v_mfma_f32_16x16x16_bf16) in
// transposed form, Z^T = W . H^T: lane l = 16q + c holds, for sample c of a
// 16-sample tile, units 16t + 4q + i (i < 4) of each 16-unit block t -- the B
// operand of the next layer as produced by the previous one.  The 4-input
// first layer and the 1-output last layer run on the vector ALUs.
__global__ void __launch_bounds__(256) k_mlp_infer_bf16(const float* __restrict__ model,
                                                        const float* __restrict__ feat, uint32_t n,
                                                        float* __restrict__ out)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t q = lane >> 4, c = lane & 15u;
    // A fragments of W2 and W3 (rows 16t + c, columns 16kk + 4q .. +3), resident
    bf16x4 w2f[4][4], w3f[4][4];
    float b2r[16], b3r[16], w4r[16], w1r[16][kIn], b1r[16];
    for (int t = 0; t < 4; ++t) {
        const int row = 16 * t + (int)c;
        for (int kk = 0; kk < 4; ++kk) {
            const float* r2 = model + oW2 + row * kH + 16 * kk + 4 * (int)q;
            const float* r3 = model + oW3 + row * kH + 16 * kk + 4 * (int)q;
            w2f[t][kk] = pack_bf16(r2[0], r2[1], r2[2], r2[3]);
            w3f[t][kk] = pack_bf16(r3[0], r3[1], r3[2], r3[3]);
        }
        for (int i = 0; i < 4; ++i) {
            const int j = 16 * t + 4 * (int)q + i;  // unit held in slot 4t + i
            b1r[4 * t + i] = bf16r(model[ob1 + j]);
            b2r[4 * t + i] = bf16r(model[ob2 + j]);
            b3r[4 * t + i] = bf16r(model[ob3 + j]);
            w4r[4 * t + i] = bf16r(model[oW4 + j]);
            for (int f = 0; f < kIn; ++f) w1r[4 * t + i][f] = bf16r(model[oW1 + j * kIn + f]);
        }
    }
    float mean[kIn], sd[kIn];
    for (int f = 0; f < kIn; ++f) {
        mean[f] = model[oMean + f];
        sd[f] = model[oStd + f];
    }
    const float b4 = bf16r(model[ob4]);
    const size_t waves = (size_t)gridDim.x * (blockDim.x / 64);
    const size_t ntiles = ((size_t)n + 15) / 16;
    for (size_t tile = (size_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); tile < ntiles; tile += waves) {
        const size_t s = tile * 16 + c;
        const bool valid = s < n;
        float a0[kIn];
        for (int f = 0; f < kIn; ++f) a0[f] = valid ? bf16r((feat[s * kIn + f] - mean[f]) / sd[f]) : 0.f;
        // layer 1 on the VALUs, straight into the B-operand layout
        bf16x4 h[4];
        for (int t = 0; t < 4; ++t) {
            float v[4];
            for (int i = 0; i < 4; ++i) {
                float acc = b1r[4 * t + i];
                for (int f = 0; f < kIn; ++f) acc += w1r[4 * t + i][f] * a0[f];
                v[i] = fmaxf(acc, 0.f);
            }
            h[t] = pack_bf16(v[0], v[1], v[2], v[3]);
        }
        // layers 2 and 3 on the matrix cores
        for (int layer = 0; layer < 2; ++layer) {
            f32x4 z[4];
            for (int t = 0; t < 4; ++t) {
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
                for (int kk = 0; kk < 4; ++kk)
                    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(layer == 0 ? w2f[t][kk] : w3f[t][kk], h[kk],
                                                                    acc, 0, 0, 0);
                z[t] = acc;
            }
            for (int t = 0; t < 4; ++t) {
                const float* bias = layer == 0 ? b2r : b3r;
                h[t] = pack_bf16(fmaxf(z[t][0] + bias[4 * t], 0.f), fmaxf(z[t][1] + bias[4 * t + 1], 0.f),
                                 fmaxf(z[t][2] + bias[4 * t + 2], 0.f), fmaxf(z[t][3] + bias[4 * t + 3], 0.f));
            }
        }
        // layer 4: this lane's 16 units, then the four lanes of the sample
        float y = 0.f;
        for (int t = 0; t < 4; ++t)
            for (int i = 0; i < 4; ++i) y += w4r[4 * t + i] * from_bf16((uint16_t)h[t][i]);
        y += __shfl_xor(y, 16, 64);
        y += __shfl_xor(y, 32, 64);
        if (q == 0 && valid) out[s] = y + b4;
    }
}

// ---------------------------------------------------------------- FP32 training
// Activations are stored feature-major ([64][n]) so a thread per sample reads
// and writes coalesced columns.
struct TrainBufs {
    float *a0, *h1, *h2, *h3, *d1, *d2, *d3, *dy, *part;
};

// Forward, loss term and backward through the activations for one sample per
// thread: stores a0 (normalised input), h1..h3, dy = dL/dy, d3..d1 = dL/dz
// (pre-activation gradients).  Loss = mean over samples of (y - t)^2.
__global__ void __launch_bounds__(256) k_mlp_fwd_bwd(const float* __restrict__ model,
                                                     const float* __restrict__ feat,
                                                     const float* __restrict__ target, uint32_t n, TrainBufs b,
                                                     float* __restrict__ loss_part)
{
    __shared__ float w[kModel];
    __shared__ float red[256];
    for (int i = threadIdx.x; i < kModel; i += blockDim.x) w[i] = model[i];
    __syncthreads();
    float lsum = 0.f;
    for (size_t s = (size_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (size_t)gridDim.x * blockDim.x) {
        float a0[kIn];
        for (int i = 0; i < kIn; ++i) {
            a0[i] = (feat[s * kIn + i] - w[oMean + i]) / w[oStd + i];
            b.a0[(size_t)i * n + s] = a0[i];
        }
        float h[kH];
        for (int j = 0; j < kH; ++j) {
            float acc = w[ob1 + j];
            for (int i = 0; i < kIn; ++i) acc += w[oW1 + j * kIn + i] * a0[i];
            h[j] = fmaxf(acc, 0.f);
            b.h1[(size_t)j * n + s] = h[j];
        }
        float g[kH];
        for (int j = 0; j < kH; ++j) {
            float acc = w[ob2 + j];
            for (int k = 0; k < kH; ++k) acc += w[oW2 + j * kH + k] * h[k];
            g[j] = fmaxf(acc, 0.f);
            b.h2[(size_t)j * n + s] = g[j];
        }
        float y = w[ob4];
        for (int j = 0; j < kH; ++j) {
            float acc = w[ob3 + j];
            for (int k = 0; k < kH; ++k) acc += w[oW3 + j * kH + k] * g[k];
            float h3 = fmaxf(acc, 0.f);
            b.h3[(size_t)j * n + s] = h3;
            y += w[oW4 + j] * h3;
        }
        float r = y - target[s];
        lsum += r * r;
        float dy = 2.f * r / (float)n;
        b.dy[s] = dy;
        // backward through the activations
        float d3[kH];
        for (int j = 0; j < kH; ++j) {
            d3[j] = b.h3[(size_t)j * n + s] > 0.f ? dy * w[oW4 + j] : 0.f;
            b.d3[(size_t)j * n + s] = d3[j];
        }
        float d2[kH];
        for (int k = 0; k < kH; ++k) {
            float acc = 0.f;
            for (int j = 0; j < kH; ++j) acc += d3[j] * w[oW3 + j * kH + k];
            d2[k] = g[k] > 0.f ? acc : 0.f;
            b.d2[(size_t)k * n + s] = d2[k];
        }
        for (int k = 0; k < kH; ++k) {
            float acc = 0.f;
            for (int j = 0; j < kH; ++j) acc += d2[j] * w[oW2 + j * kH + k];
            b.d1[(size_t)k * n + s] = h[k] > 0.f ? acc : 0.f;
        }
    }
    red[threadIdx.x] = lsum;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

// Weight gradients: per block, sums over one chunk of samples for every
// trainable parameter (dW_l[j][k] = sum_s d_l[j][s] * x_{l-1}[k][s]); partial
// sums go to part[block][param] and are reduced in a fixed order afterwards,
// so the result does not depend on scheduling.
constexpr int kGradChunk = 4096;
constexpr int kTile = 64;

__global__ void __launch_bounds__(256) k_mlp_grad_partial(TrainBufs b, uint32_t n)
{
    __shared__ float dt[kH][kTile + 1];
    __shared__ float xt[kH][kTile + 1];
    const uint32_t s0 = blockIdx.x * kGradChunk;
    const uint32_t s1 = min(n, s0 + kGradChunk);
    float* part = b.part + (size_t)blockIdx.x * kTrainable;
    // the four layers: (delta, input, rows, cols, W offset, b offset)
    for (int layer = 0; layer < 4; ++layer) {
        const float* D = layer == 0 ? b.d1 : layer == 1 ? b.d2 : layer == 2 ? b.d3 : b.dy;
        const float* X = layer == 0 ? b.a0 : layer == 1 ? b.h1 : layer == 2 ? b.h2 : b.h3;
        const int rows = layer == 3 ? 1 : kH;
        const int cols = layer == 0 ? kIn : kH;
        const int oW = layer == 0 ? oW1 : layer == 1 ? oW2 : layer == 2 ? oW3 : oW4;
        const int oB = layer == 0 ? ob1 : layer == 1 ? ob2 : layer == 2 ? ob3 : ob4;
        // each thread owns up to 16 (j, k) pairs of this layer plus bias terms
        float accw[16];
        float accb = 0.f;
        for (int q = 0; q < 16; ++q) accw[q] = 0.f;
        for (uint32_t t0 = s0; t0 < s1; t0 += kTile) {
            uint32_t cnt = min((uint32_t)kTile, s1 - t0);
            for (int idx = threadIdx.x; idx < kH * kTile; idx += blockDim.x) {
                int r = idx / kTile, c = idx % kTile;
                dt[r][c] = (r < rows && (uint32_t)c < cnt) ? D[(size_t)r * n + t0 + c] : 0.f;
                xt[r][c] = (r < cols && (uint32_t)c < cnt) ? X[(size_t)r * n + t0 + c] : 0.f;
            }
            __syncthreads();
            for (int q = 0; q < 16; ++q) {
                int pidx = threadIdx.x * 16 + q;  // 0 .. 4095
                int j = pidx / kH, k = pidx % kH;
                if (j < rows && k < cols) {
                    float a = 0.f;
                    for (uint32_t c = 0; c < cnt; ++c) a += dt[j][c] * xt[k][c];
                    accw[q] += a;
                }
            }
            if ((int)threadIdx.x < rows) {
                float a = 0.f;
                for (uint32_t c = 0; c < cnt; ++c) a += dt[threadIdx.x][c];
                accb += a;
            }
            __syncthreads();
        }
        for (int q = 0; q < 16; ++q) {
            int pidx = threadIdx.x * 16 + q;
            int j = pidx / kH, k = pidx % kH;
            if (j < rows && k < cols) part[oW + (layer == 3 ? k : j * cols + k)] = accw[q];
        }
        if ((int)threadIdx.x < rows) part[oB + threadIdx.x] = accb;
        __syncthreads();
    }
}

__global__ void k_grad_reduce(const float* __restrict__ part, uint32_t nparts, float* __restrict__ grad)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kModel; i += gridDim.x * blockDim.x) {
        float a = 0.f;
        if (i < kTrainable)
            for (uint32_t p = 0; p < nparts; ++p) a += part[(size_t)p * kTrainable + i];
        grad[i] = a;
    }
}

// Adam (Kingma and Ba, 2015), bias-corrected, on the trainable parameters.
__global__ void k_adam(float* __restrict__ model, const float* __restrict__ grad, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kTrainable; i += gridDim.x * blockDim.x) {
        float g = grad[i];
        float mi = b1 * m[i] + (1.f - b1) * g;
        float vi = b2 * v[i] + (1.f - b2) * g * g;
        m[i] = mi;
        v[i] = vi;
        float mh = mi / c1, vh = vi / c2;
        model[i] -= lr * mh / (sqrtf(vh) + eps);
    }
}

// mean / std of each feature column (two passes, double accumulation) into the model.
__global__ void k_fit_norm(const float* __restrict__ feat, uint32_t n, float* __restrict__ model)
{
    __shared__ double red[256];
    int f = blockIdx.x;  // one block per feature
    double s = 0;
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) s += feat[(size_t)i * kIn + f];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    double mean = red[0] / (n ? n : 1);
    __syncthreads();
    double q = 0;
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        double d = feat[(size_t)i * kIn + f] - mean;
        q += d * d;
    }
    red[threadIdx.x] = q;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double sd = sqrt(red[0] / (n ? n : 1));
        model[oMean + f] = (float)mean;
        model[oStd + f] = (float)(sd > 1e-6 ? sd : 1.0);
    }
}

// ---------------------------------------------------------------- learned queue
// Sort key: descending predicted cost (quantised log-cost), stable in rank order.
__global__ void k_score_keys(const float* __restrict__ score, uint32_t n, uint32_t* __restrict__ key)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        float s = fminf(fmaxf(score[i], 0.f), 63.f);
        uint32_t q = (uint32_t)(s * 65536.f);  // < 2^22
        key[i] = (1u << 22) - 1u - q;
    }
}

// Total predicted tree nodes, sum of expm1(score): per-block partial sums over
// a fixed grid, then one block adds them in order (deterministic).
constexpr int kSumBlocks = 256;

__global__ void __launch_bounds__(256) k_pred_partial(const float* __restrict__ score, uint32_t n,
                                                      double* __restrict__ part)
{
    __shared__ double red[256];
    double acc = 0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        acc += (double)expm1f(fminf(fmaxf(score[i], 0.f), 40.f));
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_pred_total(const double* __restrict__ part, int nparts, double* __restrict__ total)
{
    if (threadIdx.x == 0) {
        double s = 0;
        for (int i = 0; i < nparts; ++i) s += part[i];
        *total = s;
    }
}

// Number of groups each scored root (in descending predicted cost) is split
// into: predicted nodes / target, capped, where target is the projected
// makespan (total predicted nodes over the workgroups), so only a root that
// alone would outlast the launch is split; the first `top` roots (a caller's
// request) get kMaxSplit groups when predicted at least `floor_nodes`.
constexpr uint32_t kMaxSplit = 64;

// Roots with at least kScoreMinP later neighbours are scored by the model, at
// most about kScoreBudget per workgroup of the launch (the roots with the most
// later neighbours; the features cost grows with the number scored).
constexpr uint32_t kScoreMinP = 16;
constexpr uint32_t kScoreBudget = 8;
constexpr uint32_t kPHistCap = 4097;  // |P| <= 4096 for any root the enumeration accepts

// Histogram of |P| (later neighbours) over the queued roots with |P| >= minp,
// |P| capped at kPHistCap - 1: per workgroup in LDS, then merged.
__global__ void __launch_bounds__(256) k_p_hist(const uint32_t* __restrict__ roots, uint32_t n,
                                                const uint32_t* __restrict__ op, uint32_t minp,
                                                uint32_t* __restrict__ hist)
{
    __shared__ uint32_t h[kPHistCap];
    for (uint32_t b = threadIdx.x; b < kPHistCap; b += blockDim.x) h[b] = 0;
    __syncthreads();
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const uint32_t r = roots[i];
        const uint32_t np = op[r + 1] - op[r];
        if (np >= minp) atomicAdd(&h[min(np, kPHistCap - 1)], 1u);
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < kPHistCap; b += blockDim.x)
        if (h[b]) atomicAdd(&hist[b], h[b]);
}

__global__ void k_score_flags(const uint32_t* __restrict__ roots, uint32_t n, const uint32_t* __restrict__ op,
                              uint32_t minp, uint32_t* __restrict__ flag)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const uint32_t r = roots[i];
        flag[i] = (op[r + 1] - op[r]) >= minp ? 1u : 0u;
    }
}

// Stable partition of the queue: flagged roots to heavy[pos], the others to
// light[i - pos] (pos = exclusive prefix sum of the flags).
__global__ void k_partition_roots(const uint32_t* __restrict__ roots, const uint32_t* __restrict__ flag,
                                  const uint32_t* __restrict__ pos, uint32_t n, uint32_t* __restrict__ heavy,
                                  uint32_t* __restrict__ light)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        if (flag[i]) heavy[pos[i]] = roots[i];
        else light[i - pos[i]] = roots[i];
    }
}

__global__ void k_split_counts(const float* __restrict__ score_sorted, uint32_t n, uint32_t top,
                               float floor_nodes, float target, uint32_t* __restrict__ groups)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        float nodes = expm1f(fminf(fmaxf(score_sorted[i], 0.f), 40.f));
        float g = fminf(fmaxf(ceilf(nodes / target), 1.f), (float)kMaxSplit);
        uint32_t c = (uint32_t)g;
        if (i < top && nodes >= floor_nodes) c = kMaxSplit;
        groups[i] = c;
    }
}

__global__ void k_split_expand(const uint32_t* __restrict__ roots_sorted, const uint32_t* __restrict__ groups,
                               const uint32_t* __restrict__ pos, uint32_t n, uint32_t* __restrict__ qroots,
                               uint32_t* __restrict__ qsplits)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        uint32_t C = groups[i], base = pos[i], r = roots_sorted[i];
        for (uint32_t c = 0; c < C; ++c) {
            qroots[base + c] = r;
            qsplits[base + c] = C > 1 ? ((C << 16) | c) : 0u;
        }
    }
}

template <class T>
__global__ void k_gather(const T* __restrict__ src, const uint32_t* __restrict__ idx, uint32_t n,
                         T* __restrict__ dst)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[idx[i]];
}

}  // namespace

mce_status root_features(const Oriented& g, const uint32_t* roots_rank, uint32_t nr, float* feat, hipStream_t s)
{
    if (nr == 0) return MCE_OK;
    DevBuf deg;
    mce_status st;
    if ((st = deg.alloc((size_t)(g.n ? g.n : 1) * 4)) != MCE_OK) return st;
    k_degrees<<<blocks_for(g.n, 256, 8192), 256, 0, s>>>(g.op.as<uint32_t>(), g.ip.as<uint32_t>(), g.n,
                                                         deg.as<uint32_t>());
    MCE_HIP_TRY(hipGetLastError());
    k_features<<<blocks_for(nr, kFeatWaves, 65536), 64 * kFeatWaves, 0, s>>>(
        g.op.as<uint32_t>(), g.oc.as<uint32_t>(), g.ip.as<uint32_t>(), g.ic.as<uint32_t>(), g.core_r.as<uint32_t>(),
        deg.as<uint32_t>(), g.vkey.as<uint64_t>(), roots_rank, nr, feat);
    MCE_HIP_TRY(hipGetLastError());
    MCE_HIP_TRY(hipStreamSynchronize(s));  // before the degree array is released
    return MCE_OK;
}

mce_status ids_to_ranks(const Oriented& g, const uint32_t* ids, uint32_t n, uint32_t* out, hipStream_t s)
{
    if (!n) return MCE_OK;
    if (g.n == 0) {
        set_error("root id out of range (graph has no vertices)");
        return MCE_ERR_INVALID_ARG;
    }
    DevBuf err;
    mce_status st;
    if ((st = err.alloc(4)) != MCE_OK) return st;
    fill_u32(err.as<uint32_t>(), 0, 1, s);
    k_ids_to_ranks<<<blocks_for(n, 256, 8192), 256, 0, s>>>(ids, n, g.n, g.rank.as<uint32_t>(), out,
                                                            err.as<uint32_t>());
    MCE_HIP_TRY(hipGetLastError());
    uint32_t herr = 0;
    MCE_HIP_TRY(hipMemcpyAsync(&herr, err.p, 4, hipMemcpyDeviceToHost, s));
    MCE_HIP_TRY(hipStreamSynchronize(s));
    if (herr) {
        set_error("root id out of range");
        return MCE_ERR_INVALID_ARG;
    }
    return MCE_OK;
}

mce_status model_predict(const float* model, const float* feat, uint32_t n, float* out, hipStream_t s)
{
    if (!n) return MCE_OK;
    k_mlp_infer_bf16<<<blocks_for((n + 15) / 16, 4, 4096), 256, 0, s>>>(model, feat, n, out);
    MCE_HIP_TRY(hipGetLastError());
    return MCE_OK;
}

namespace {
// Sizes and layout of the training buffers for n samples: activations
// (feature-major a0, h1..h3, d1..d3, dy), per-chunk gradient partials and
// per-block loss partials.
size_t act_floats(uint32_t n) { return ((size_t)kIn + 6 * kH + 1) * n; }
uint32_t grad_parts(uint32_t n) { return (n + kGradChunk - 1) / kGradChunk; }
uint32_t loss_parts(uint32_t n) { return blocks_for(n, 256, 2048); }

TrainBufs bind_bufs(float* act, float* part, uint32_t n)
{
    TrainBufs b;
    b.a0 = act;
    b.h1 = b.a0 + (size_t)kIn * n;
    b.h2 = b.h1 + (size_t)kH * n;
    b.h3 = b.h2 + (size_t)kH * n;
    b.d1 = b.h3 + (size_t)kH * n;
    b.d2 = b.d1 + (size_t)kH * n;
    b.d3 = b.d2 + (size_t)kH * n;
    b.dy = b.d3 + (size_t)kH * n;
    b.part = part;
    return b;
}

// Forward/backward, gradient partials and their fixed-order reduction into
// grad; the loss (mean over samples, summed in double on the host in block
// order) when loss_host is given.
mce_status run_loss_grad(const float* model, const float* feat, const float* target, uint32_t n, const TrainBufs& b,
                         uint32_t nparts, float* lpart, uint32_t nloss, float* grad, hipStream_t s, float* loss_host)
{
    k_mlp_fwd_bwd<<<nloss, 256, 0, s>>>(model, feat, target, n, b, lpart);
    MCE_HIP_TRY(hipGetLastError());
    k_mlp_grad_partial<<<nparts, 256, 0, s>>>(b, n);
    MCE_HIP_TRY(hipGetLastError());
    k_grad_reduce<<<blocks_for(kModel, 256), 256, 0, s>>>(b.part, nparts, grad);
    MCE_HIP_TRY(hipGetLastError());
    if (loss_host) {
        constexpr uint32_t kChunk = 64;  // partials copied per round trip (host stack, no heap)
        float lp[kChunk];
        double t = 0;
        for (uint32_t i0 = 0; i0 < nloss; i0 += kChunk) {
            const uint32_t k = nloss - i0 < kChunk ? nloss - i0 : kChunk;
            MCE_HIP_TRY(hipMemcpyAsync(lp, lpart + i0, k * 4, hipMemcpyDeviceToHost, s));
            MCE_HIP_TRY(hipStreamSynchronize(s));
            for (uint32_t i = 0; i < k; ++i) t += lp[i];
        }
        *loss_host = (float)(t / (n ? n : 1));
    }
    return MCE_OK;
}

struct TrainState {
    DevBuf act, part, grad, m, v, lpart;
    TrainBufs b;
    uint32_t nparts = 0, nloss = 0;
    mce_status setup(uint32_t n)
    {
        mce_status st;
        if ((st = act.alloc(act_floats(n) * 4 + 64)) != MCE_OK) return st;
        nparts = grad_parts(n);
        if ((st = part.alloc((size_t)nparts * kTrainable * 4 + 64)) != MCE_OK) return st;
        if ((st = grad.alloc(kModel * 4)) != MCE_OK) return st;
        if ((st = m.alloc(kModel * 4)) != MCE_OK) return st;
        if ((st = v.alloc(kModel * 4)) != MCE_OK) return st;
        nloss = loss_parts(n);
        if ((st = lpart.alloc((size_t)nloss * 4)) != MCE_OK) return st;
        b = bind_bufs(act.as<float>(), part.as<float>(), n);
        return MCE_OK;
    }
    mce_status loss_grad(const float* model, const float* feat, const float* target, uint32_t n, hipStream_t s,
                         float* loss_host)
    {
        return run_loss_grad(model, feat, target, n, b, nparts, lpart.as<float>(), nloss, grad.as<float>(), s,
                             loss_host);
    }
};
}  // namespace

mce_status model_loss_grad(const float* model, const float* feat, const float* target, uint32_t n, float* grad,
                           float* loss, hipStream_t s)
{
    if (n == 0) {
        set_error("no samples");
        return MCE_ERR_INVALID_ARG;
    }
    TrainState ts;
    mce_status st = ts.setup(n);
    if (st != MCE_OK) return st;
    if ((st = ts.loss_grad(model, feat, target, n, s, loss)) != MCE_OK) return st;
    MCE_HIP_TRY(hipMemcpyAsync(grad, ts.grad.p, kModel * 4, hipMemcpyDeviceToDevice, s));
    MCE_HIP_TRY(hipStreamSynchronize(s));
    return MCE_OK;
}

// ---------------------------------------------------------------- loss and gradient without allocation
// For callers that cannot allocate device memory: the activations and partial
// sums of mce_model_loss_grad live in one file-scope device array of fixed
// size instead of buffers allocated per call.  Each device that runs the
// library holds its own copy until the process ends; its address on a device
// is looked up once, with that device current, and kept.  Calls on one device
// share the array, so overlapping calls there race; nothing in it has to start
// at zero (every word a call reads was written earlier in the same call).
constexpr uint32_t kNaMax = MCE_NOALLOC_MAX_SAMPLES;
constexpr size_t kNaActBytes = (((size_t)kIn + 6 * kH + 1) * kNaMax * 4 + 255) & ~(size_t)255;
constexpr size_t kNaPartBytes = ((size_t)((kNaMax + kGradChunk - 1) / kGradChunk) * kTrainable * 4 + 255) & ~(size_t)255;
constexpr size_t kNaLossBytes = ((size_t)((kNaMax + 255) / 256) * 4 + 255) & ~(size_t)255;
constexpr size_t kNaBytes = kNaActBytes + kNaPartBytes + kNaLossBytes;
static_assert((kNaMax + 255) / 256 <= 2048, "loss partials: one per block of 256 samples");

static __device__ __align__(256) unsigned char scratch[kNaBytes];

namespace {
constexpr int kNaDevices = 64;
std::mutex g_na_mu;
unsigned char* g_na_ptr[kNaDevices] = {};

// The device address of this device's scratch array; the stream (if given)
// must belong to the current device.
mce_status noalloc_scratch(hipStream_t s, unsigned char** out)
{
    int dev = 0;
    MCE_HIP_TRY(hipGetDevice(&dev));
    if (s) {
        hipDevice_t sd = 0;
        MCE_HIP_TRY(hipStreamGetDevice(s, &sd));
        if ((int)sd != dev) {
            set_error("the stream belongs to another device than the current one");
            return MCE_ERR_INVALID_ARG;
        }
    }
    if (dev < 0 || dev >= kNaDevices) {
        set_error("device index beyond the library's table of scratch addresses");
        return MCE_ERR_DEVICE;
    }
    std::lock_guard<std::mutex> lock(g_na_mu);
    if (!g_na_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            return MCE_ERR_DEVICE;
        }
        g_na_ptr[dev] = static_cast<unsigned char*>(p);
    }
    *out = g_na_ptr[dev];
    return MCE_OK;
}
}  // namespace

mce_status model_loss_grad_noalloc(const float* model, const float* feat, const float* target, uint32_t n,
                                   float* grad, float* loss, hipStream_t s)
{
    if (n == 0) {
        set_error("no samples");
        return MCE_ERR_INVALID_ARG;
    }
    if (n > kNaMax) {
        set_error("n = " + std::to_string(n) + " exceeds MCE_NOALLOC_MAX_SAMPLES = " + std::to_string(kNaMax) +
                  " (use mce_model_loss_grad)");
        return MCE_ERR_INVALID_ARG;
    }
    unsigned char* base = nullptr;
    mce_status st = noalloc_scratch(s, &base);
    if (st != MCE_OK) return st;
    const TrainBufs b = bind_bufs(reinterpret_cast<float*>(base), reinterpret_cast<float*>(base + kNaActBytes), n);
    float* lpart = reinterpret_cast<float*>(base + kNaActBytes + kNaPartBytes);
    if ((st = run_loss_grad(model, feat, target, n, b, grad_parts(n), lpart, loss_parts(n), grad, s, loss)) != MCE_OK)
        return st;
    MCE_HIP_TRY(hipStreamSynchronize(s));
    return MCE_OK;
}

mce_status model_fit_norm(float* model, const float* feat, uint32_t n, hipStream_t s)
{
    k_fit_norm<<<kIn, 256, 0, s>>>(feat, n, model);
    MCE_HIP_TRY(hipGetLastError());
    return MCE_OK;
}

mce_status model_train(float* model, const float* feat, const float* target, uint32_t n, uint32_t epochs, float lr,
                       float b1, float b2, float eps, bool fit_norm, float* loss_hist, hipStream_t s)
{
    if (n == 0) {
        set_error("no samples");
        return MCE_ERR_INVALID_ARG;
    }
    TrainState ts;
    mce_status st = ts.setup(n);
    if (st != MCE_OK) return st;
    if (fit_norm && (st = model_fit_norm(model, feat, n, s)) != MCE_OK) return st;
    fill_u32(reinterpret_cast<uint32_t*>(ts.m.p), 0, kModel, s);
    fill_u32(reinterpret_cast<uint32_t*>(ts.v.p), 0, kModel, s);
    double c1 = 1.0, c2 = 1.0;
    for (uint32_t e = 0; e < epochs; ++e) {
        float l = 0;
        if ((st = ts.loss_grad(model, feat, target, n, s, loss_hist ? &l : nullptr)) != MCE_OK) return st;
        if (loss_hist) loss_hist[e] = l;
        c1 *= b1;
        c2 *= b2;
        k_adam<<<blocks_for(kTrainable, 256), 256, 0, s>>>(model, ts.grad.as<float>(), ts.m.as<float>(),
                                                            ts.v.as<float>(), lr, b1, b2, eps, (float)(1.0 - c1),
                                                            (float)(1.0 - c2));
        MCE_HIP_TRY(hipGetLastError());
    }
    MCE_HIP_TRY(hipStreamSynchronize(s));
    return MCE_OK;
}

// Work queue from a model: window roots (rank order) -> features -> scores ->
// stable descending sort -> optional split of the costliest roots.
mce_status learned_queue(const Oriented& g, const EnumConfig& cfg, EnumState& st, hipStream_t s, uint32_t grid,
                         LearnedQueue& q, uint32_t built_n)
{
    mce_status rc;
    uint32_t nroots = built_n;
    if (built_n == kQueueNotBuilt) {
        EnumConfig plain = cfg;
        plain.flags &= ~(MCE_F_CUSTOM_ORDER | MCE_F_REVERSE_ORDER);
        if ((rc = build_root_queue(g, plain, st, s, &nroots)) != MCE_OK) return rc;
    }
    q.n = nroots;
    if (!nroots) return MCE_OK;
    size_t nn = nroots;
    uint32_t* roots = st.roots.as<uint32_t>();
    // the roots with the most later neighbours (at least kScoreMinP; subtrees
    // with fewer have at most 3^(kScoreMinP/3) leaves) are scored; the others
    // follow in degeneracy order
    if ((rc = q.flag.alloc(nn * 4)) != MCE_OK) return rc;
    if ((rc = q.pos.alloc((nn + 1) * 4)) != MCE_OK) return rc;
    if ((rc = q.scan_tmp.alloc(scan_tmp_words(nn + 1) * 8 + 64)) != MCE_OK) return rc;
    if ((rc = q.total.alloc(8)) != MCE_OK) return rc;
    if ((rc = q.heavy.alloc(nn * 4)) != MCE_OK) return rc;
    if ((rc = q.light.alloc(nn * 4)) != MCE_OK) return rc;
    // the |P| threshold: the smallest t >= kScoreMinP with at most the budget of
    // roots at or above it (ties at t all go in)
    uint32_t minp = kScoreMinP;
    {
        const uint32_t cap = kPHistCap;  // bins 0 .. cap - 1
        std::vector<uint32_t> hh(cap, 0u);
        if ((rc = q.phist.alloc((size_t)cap * 4)) != MCE_OK) return rc;
        fill_u32(q.phist.as<uint32_t>(), 0u, cap, s);
        k_p_hist<<<blocks_for(nn, 256, 512), 256, 0, s>>>(roots, nroots, g.op.as<uint32_t>(), kScoreMinP,
                                                          q.phist.as<uint32_t>());
        MCE_HIP_TRY(hipGetLastError());
        MCE_HIP_TRY(hipMemcpyAsync(hh.data(), q.phist.p, (size_t)cap * 4, hipMemcpyDeviceToHost, s));
        MCE_HIP_TRY(hipStreamSynchronize(s));
        const uint64_t budget = (uint64_t)kScoreBudget * std::max(grid, 1u);
        uint64_t above = 0;
        uint32_t t = cap;  // count of bins t .. cap - 1 is `above`
        while (t > kScoreMinP && above + hh[t - 1] <= budget) above += hh[--t];
        minp = std::max(kScoreMinP, t == cap ? cap - 1 : t);
    }
    q.min_p = minp;
    k_score_flags<<<blocks_for(nn, 256, 8192), 256, 0, s>>>(roots, nroots, g.op.as<uint32_t>(), minp,
                                                            q.flag.as<uint32_t>());
    MCE_HIP_TRY(hipGetLastError());
    if ((rc = exclusive_scan_u32(q.flag.as<uint32_t>(), q.pos.as<uint32_t>(), nn, q.total.as<uint32_t>(),
                                 q.scan_tmp.as<uint64_t>(), s)) != MCE_OK)
        return rc;
    k_partition_roots<<<blocks_for(nn, 256, 8192), 256, 0, s>>>(roots, q.flag.as<uint32_t>(), q.pos.as<uint32_t>(),
                                                                nroots, q.heavy.as<uint32_t>(),
                                                                q.light.as<uint32_t>());
    MCE_HIP_TRY(hipGetLastError());
    uint32_t nh = 0;
    MCE_HIP_TRY(hipMemcpyAsync(&nh, q.total.p, 4, hipMemcpyDeviceToHost, s));
    MCE_HIP_TRY(hipStreamSynchronize(s));
    const uint32_t nl = nroots - nh;
    q.scored = nh;
    // order the scored roots by descending predicted cost (stable)
    const size_t nhs = nh ? nh : 1;
    if ((rc = q.feat.alloc(nhs * 16)) != MCE_OK) return rc;
    if ((rc = q.score.alloc(nhs * 4)) != MCE_OK) return rc;
    if ((rc = q.keys.alloc(nhs * 4)) != MCE_OK) return rc;
    if ((rc = q.sorted.alloc(nhs * 4)) != MCE_OK) return rc;
    if ((rc = q.roots.alloc(nhs * 4)) != MCE_OK) return rc;
    if ((rc = q.score_sorted.alloc(nhs * 4)) != MCE_OK) return rc;
    if (nh) {
        const uint32_t* heavy = q.heavy.as<uint32_t>();
        if ((rc = root_features(g, heavy, nh, q.feat.as<float>(), s)) != MCE_OK) return rc;
        if ((rc = model_predict(reinterpret_cast<const float*>(cfg.model), q.feat.as<float>(), nh,
                                q.score.as<float>(), s)) != MCE_OK)
            return rc;
        k_score_keys<<<blocks_for(nh, 256, 8192), 256, 0, s>>>(q.score.as<float>(), nh, q.keys.as<uint32_t>());
        MCE_HIP_TRY(hipGetLastError());
        iota_u32(q.sorted.as<uint32_t>(), nh, s);
        {
            RadixTmp rt;
            if ((rc = stable_sort_pairs_u32(q.keys.as<uint32_t>(), q.sorted.as<uint32_t>(), nh, 22, rt, s)) != MCE_OK)
                return rc;
            MCE_HIP_TRY(hipStreamSynchronize(s));
        }
        k_gather<uint32_t><<<blocks_for(nh, 256, 8192), 256, 0, s>>>(heavy, q.sorted.as<uint32_t>(), nh,
                                                                     q.roots.as<uint32_t>());
        k_gather<float><<<blocks_for(nh, 256, 8192), 256, 0, s>>>(q.score.as<float>(), q.sorted.as<uint32_t>(), nh,
                                                                  q.score_sorted.as<float>());
        MCE_HIP_TRY(hipGetLastError());
    }
    // groups per scored root: split only roots predicted above the projected
    // makespan (total predicted nodes over the workgroups), in proportion, and
    // the split_top costliest when asked
    if ((rc = q.groups.alloc(nhs * 4 + 4)) != MCE_OK) return rc;
    if ((rc = q.gpos.alloc(nhs * 4 + 4)) != MCE_OK) return rc;
    uint32_t len_h = nh;
    const bool split = (cfg.flags & MCE_F_SPLIT) != 0 && nh > 0;
    if (split) {
        if ((rc = q.psum.alloc((kSumBlocks + 1) * 8)) != MCE_OK) return rc;
        k_pred_partial<<<kSumBlocks, 256, 0, s>>>(q.score_sorted.as<float>(), nh, q.psum.as<double>());
        k_pred_total<<<1, 64, 0, s>>>(q.psum.as<double>(), kSumBlocks, q.psum.as<double>() + kSumBlocks);
        MCE_HIP_TRY(hipGetLastError());
        double total = 0;
        MCE_HIP_TRY(hipMemcpyAsync(&total, q.psum.as<double>() + kSumBlocks, 8, hipMemcpyDeviceToHost, s));
        MCE_HIP_TRY(hipStreamSynchronize(s));
        const float target = (float)std::max(64.0, total / (double)std::max(grid, 1u));
        const uint32_t top = std::min(cfg.split_top, nh);
        const float floor_nodes = (float)std::max(64.0, 4.0 * total / (double)nh);
        k_split_counts<<<blocks_for(nh, 256, 8192), 256, 0, s>>>(q.score_sorted.as<float>(), nh, top, floor_nodes,
                                                                 target, q.groups.as<uint32_t>());
        MCE_HIP_TRY(hipGetLastError());
        if ((rc = exclusive_scan_u32(q.groups.as<uint32_t>(), q.gpos.as<uint32_t>(), nh, q.total.as<uint32_t>(),
                                     q.scan_tmp.as<uint64_t>(), s)) != MCE_OK)
            return rc;
        MCE_HIP_TRY(hipMemcpyAsync(&len_h, q.total.p, 4, hipMemcpyDeviceToHost, s));
        MCE_HIP_TRY(hipStreamSynchronize(s));
    }
    // the queue: scored roots (expanded into their groups), then the others
    const uint32_t len = len_h + nl;
    if ((rc = q.sroots.alloc((size_t)len * 4 + 4)) != MCE_OK) return rc;
    if ((rc = q.ssplits.alloc((size_t)len * 4 + 4)) != MCE_OK) return rc;
    if (split) {
        k_split_expand<<<blocks_for(nh, 256, 8192), 256, 0, s>>>(q.roots.as<uint32_t>(), q.groups.as<uint32_t>(),
                                                                 q.gpos.as<uint32_t>(), nh, q.sroots.as<uint32_t>(),
                                                                 q.ssplits.as<uint32_t>());
        MCE_HIP_TRY(hipGetLastError());
    } else if (nh) {
        MCE_HIP_TRY(hipMemcpyAsync(q.sroots.p, q.roots.p, (size_t)nh * 4, hipMemcpyDeviceToDevice, s));
    }
    if (nl) MCE_HIP_TRY(hipMemcpyAsync(q.sroots.as<uint32_t>() + len_h, q.light.p, (size_t)nl * 4,
                                       hipMemcpyDeviceToDevice, s));
    if (split) fill_u32(q.ssplits.as<uint32_t>() + len_h, 0u, nl, s);  // one group each
    MCE_HIP_TRY(hipStreamSynchronize(s));
    q.qroots = q.sroots.as<uint32_t>();
    q.qsplits = split ? q.ssplits.as<uint32_t>() : nullptr;
    q.len = len;
    return MCE_OK;
}

}  // namespace mce
