// Device-wide primitives: exclusive scan, fills, and a stable LSD radix sort of
// (key, value) pairs.  Written for wave64 / gfx950.
#include "mce_internal.h"

namespace mce {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

template <class T>
__device__ T block_exclusive_scan(T v, T* lds, T& total)
{
    // Hillis-Steele over the wave, then over wave totals.
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    T x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        T y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) lds[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        T acc = 0;
        for (int w = 0; w < kScanThreads / 64; ++w) {
            T t = lds[w];
            lds[w] = acc;
            acc += t;
        }
        lds[kScanThreads / 64] = acc;
    }
    __syncthreads();
    T res = x - v + lds[wave];
    total = lds[kScanThreads / 64];
    __syncthreads();
    return res;
}

template <class T>
__global__ void __launch_bounds__(kScanThreads) k_block_reduce(const T* __restrict__ in, size_t n,
                                                                T* __restrict__ sums)
{
    __shared__ T lds[kScanThreads / 64 + 1];
    size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
    T s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) s += in[base + i];
    T total;
    (void)block_exclusive_scan<T>(s, lds, total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

template <class T>
__global__ void __launch_bounds__(kScanThreads) k_block_scan(const T* in, T* out, size_t n,
                                                              const T* __restrict__ offsets,
                                                              T* total_dev)
{
    __shared__ T lds[kScanThreads / 64 + 1];
    size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
    T v[kScanItems];
    T s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = (base + i < n) ? in[base + i] : T(0);
        s += v[i];
    }
    T total;
    T pre = block_exclusive_scan<T>(s, lds, total);
    T off = offsets ? offsets[blockIdx.x] : T(0);
    T run = off + pre;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
    if (total_dev && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total_dev = off + total;
}

template <class T>
mce_status scan_impl(const T* in, T* out, size_t n, T* total_dev, uint64_t* tmp, hipStream_t s)
{
    if (n == 0) {
        if (total_dev) {
            T z = 0;
            MCE_HIP_TRY(hipMemcpyAsync(total_dev, &z, sizeof(T), hipMemcpyHostToDevice, s));
            MCE_HIP_TRY(hipStreamSynchronize(s));
        }
        return MCE_OK;
    }
    size_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 1) {
        k_block_scan<T><<<1, kScanThreads, 0, s>>>(in, out, n, nullptr, total_dev);
        MCE_HIP_TRY(hipGetLastError());
        return MCE_OK;
    }
    T* sums = reinterpret_cast<T*>(tmp);
    k_block_reduce<T><<<(unsigned)nb, kScanThreads, 0, s>>>(in, n, sums);
    MCE_HIP_TRY(hipGetLastError());
    // scan the block sums in place (recursively), using the rest of tmp
    mce_status st = scan_impl<T>(sums, sums, nb, nullptr, tmp + nb, s);
    if (st != MCE_OK) return st;
    k_block_scan<T><<<(unsigned)nb, kScanThreads, 0, s>>>(in, out, n, sums, total_dev);
    MCE_HIP_TRY(hipGetLastError());
    return MCE_OK;
}

template <class T>
__global__ void k_fill(T* p, T v, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_iota(uint32_t* p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = (uint32_t)i;
}

unsigned grid_for(size_t n, unsigned threads)
{
    size_t b = (n + threads - 1) / threads;
    if (b > 65536) b = 65536;
    if (b == 0) b = 1;
    return (unsigned)b;
}

// ---- stable radix sort (8-bit digits) --------------------------------------------
constexpr int kRadixThreads = 256;
constexpr int kRadixWaves = kRadixThreads / 64;
constexpr int kRadixChunks = 16;                       // chunks of 64 keys per wave
constexpr int kRadixSeg = 64 * kRadixChunks;           // keys per wave
constexpr int kRadixTile = kRadixSeg * kRadixWaves;    // keys per block

__global__ void __launch_bounds__(kRadixThreads) k_radix_count(const uint32_t* __restrict__ keys,
                                                               size_t n, int shift, uint32_t nblocks,
                                                               uint32_t* __restrict__ hist)
{
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    size_t base = (size_t)blockIdx.x * kRadixTile;
    for (int i = threadIdx.x; i < kRadixTile; i += kRadixThreads) {
        size_t idx = base + i;
        if (idx < n) atomicAdd(&cnt[(keys[idx] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(size_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

__device__ inline uint32_t lanemask_lt_popc(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__global__ void __launch_bounds__(kRadixThreads) k_radix_scatter(
    const uint32_t* __restrict__ keys, const uint32_t* __restrict__ vals, size_t n, int shift,
    uint32_t nblocks, const uint32_t* __restrict__ hist_scanned, uint32_t* __restrict__ okeys,
    uint32_t* __restrict__ ovals)
{
    __shared__ uint32_t cnt[kRadixWaves][256];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < kRadixWaves * 256; i += kRadixThreads) (&cnt[0][0])[i] = 0;
    __syncthreads();
    const size_t seg = (size_t)blockIdx.x * kRadixTile + (size_t)wave * kRadixSeg;
    for (int c = 0; c < kRadixChunks; ++c) {
        size_t idx = seg + (size_t)c * 64 + lane;
        if (idx < n) atomicAdd(&cnt[wave][(keys[idx] >> shift) & 255u], 1u);
    }
    __syncthreads();
    {
        int d = threadIdx.x;  // one digit per thread
        uint32_t run = hist_scanned[(size_t)d * nblocks + blockIdx.x];
        for (int w = 0; w < kRadixWaves; ++w) {
            uint32_t t = cnt[w][d];
            cnt[w][d] = run;
            run += t;
        }
    }
    __syncthreads();
    for (int c = 0; c < kRadixChunks; ++c) {
        size_t idx = seg + (size_t)c * 64 + lane;
        bool valid = idx < n;
        uint32_t k = valid ? keys[idx] : 0u;
        uint32_t v = valid ? vals[idx] : 0u;
        uint32_t dg = (k >> shift) & 255u;
        uint64_t match = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t bal = __ballot((dg >> b) & 1u);
            match &= ((dg >> b) & 1u) ? bal : ~bal;
        }
        uint32_t rank = lanemask_lt_popc(match);
        uint32_t basev = valid ? cnt[wave][dg] : 0u;
        if (valid) {
            okeys[basev + rank] = k;
            ovals[basev + rank] = v;
        }
        __builtin_amdgcn_wave_barrier();
        if (valid && rank == 0) cnt[wave][dg] = basev + (uint32_t)__popcll(match);
        __builtin_amdgcn_wave_barrier();
    }
}

}  // namespace

size_t scan_tmp_words(size_t n)
{
    size_t w = 0;
    size_t m = n;
    while (m > (size_t)kScanTile) {
        m = (m + kScanTile - 1) / kScanTile;
        w += m;
    }
    return w + 64;
}

mce_status exclusive_scan_u32(const uint32_t* in, uint32_t* out, size_t n, uint32_t* total_dev,
                              uint64_t* tmp, hipStream_t s)
{
    // block sums of u32 tiles fit in the u64 tmp area (we only use the low half)
    return scan_impl<uint32_t>(in, out, n, total_dev, tmp, s);
}

mce_status exclusive_scan_u64(const uint64_t* in, uint64_t* out, size_t n, uint64_t* total_dev,
                              uint64_t* tmp, hipStream_t s)
{
    return scan_impl<uint64_t>(in, out, n, total_dev, tmp, s);
}

void fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s)
{
    if (n) k_fill<uint32_t><<<grid_for(n, 256), 256, 0, s>>>(p, v, n);
}

void fill_u64(uint64_t* p, uint64_t v, size_t n, hipStream_t s)
{
    if (n) k_fill<uint64_t><<<grid_for(n, 256), 256, 0, s>>>(p, v, n);
}

void iota_u32(uint32_t* p, size_t n, hipStream_t s)
{
    if (n) k_iota<<<grid_for(n, 256), 256, 0, s>>>(p, n);
}

mce_status stable_sort_pairs_u32(uint32_t* keys, uint32_t* vals, size_t n, int key_bits,
                                 RadixTmp& tmp, hipStream_t s)
{
    if (n <= 1 || key_bits <= 0) return MCE_OK;
    size_t nblocks = (n + kRadixTile - 1) / kRadixTile;
    size_t hn = nblocks * 256;
    mce_status st;
    if ((st = tmp.keys_alt.alloc(n * 4)) != MCE_OK) return st;
    if ((st = tmp.vals_alt.alloc(n * 4)) != MCE_OK) return st;
    if ((st = tmp.hist.alloc(hn * 4)) != MCE_OK) return st;
    if ((st = tmp.scan_tmp.alloc(scan_tmp_words(hn) * 8)) != MCE_OK) return st;
    uint32_t* k0 = keys;
    uint32_t* v0 = vals;
    uint32_t* k1 = tmp.keys_alt.as<uint32_t>();
    uint32_t* v1 = tmp.vals_alt.as<uint32_t>();
    int passes = (key_bits + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        int shift = 8 * p;
        k_radix_count<<<(unsigned)nblocks, kRadixThreads, 0, s>>>(k0, n, shift, (uint32_t)nblocks,
                                                                  tmp.hist.as<uint32_t>());
        MCE_HIP_TRY(hipGetLastError());
        st = exclusive_scan_u32(tmp.hist.as<uint32_t>(), tmp.hist.as<uint32_t>(), hn, nullptr,
                                tmp.scan_tmp.as<uint64_t>(), s);
        if (st != MCE_OK) return st;
        k_radix_scatter<<<(unsigned)nblocks, kRadixThreads, 0, s>>>(
            k0, v0, n, shift, (uint32_t)nblocks, tmp.hist.as<uint32_t>(), k1, v1);
        MCE_HIP_TRY(hipGetLastError());
        std::swap(k0, k1);
        std::swap(v0, v1);
    }
    if (k0 != keys) {
        MCE_HIP_TRY(hipMemcpyAsync(keys, k0, n * 4, hipMemcpyDeviceToDevice, s));
        MCE_HIP_TRY(hipMemcpyAsync(vals, v0, n * 4, hipMemcpyDeviceToDevice, s));
    }
    return MCE_OK;
}

}  // namespace mce
