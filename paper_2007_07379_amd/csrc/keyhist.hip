// Deferred binning of samples (Fig. 2 step 3): the sweep kernel stores each
// sample's bin index alpha * 2^K + phi as a 32-bit key, and these kernels count
// the keys into the circuit's histogram through LDS.  The histogram is cut
// into buckets of 2^15 bins (128 KiB of LDS).  The keys are first
// partitioned by bucket with a counting sort (per-tile bucket counts, a scan
// per bucket, a scatter of each key's low 15 bits as a 16-bit word into its
// bucket's region); then the workgroups that own a bucket count its keys in
// LDS and write the counts to partial rows (no atomics in HBM); a last kernel
// adds the partial rows into the histogram with coalesced accesses.  Every
// key is read twice as 32 bits, written once and read once as 16 bits.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "keyhist.h"

namespace pbit {

namespace {

constexpr uint32_t LDS_BITS = 15;
constexpr uint32_t TILE = 8192;  // keys per tile of the partition
constexpr uint32_t TILE_THREADS = 256;
constexpr uint32_t HIST_THREADS = 1024;
constexpr uint32_t ALIGN = 8;  // bucket regions start at multiples of 8 keys (16 bytes)

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Scratch layout: tile counts (bucket-major), aligned and raw bucket sizes,
// bucket bases, the partitioned 16-bit keys, the partial rows.
struct Layout {
    uint32_t bits, lb, NB, T, C;
    uint64_t cnt_off, size_off, base_off, out_off, part_off, bytes;
};

Layout layout(uint64_t M, uint32_t bits) {
    Layout L;
    L.bits = bits;
    L.lb = std::min(bits, LDS_BITS);
    L.NB = 1u << (bits - L.lb);
    L.T = (uint32_t)((M + TILE - 1) / TILE);
    // about 512 counting workgroups, partial rows of at most KEYHIST_PART_BYTES
    const uint64_t cap = KEYHIST_PART_BYTES / ((uint64_t)4 << bits);
    L.C = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(512 / L.NB, cap));
    uint64_t o = 0;
    auto take = [&](uint64_t b) {
        const uint64_t at = o;
        o += (b + 255) & ~255ull;
        return at;
    };
    L.cnt_off = take((uint64_t)L.NB * L.T * 4);
    L.size_off = take((uint64_t)L.NB * 8);
    L.base_off = take((uint64_t)L.NB * 4);
    L.out_off = take((M + (uint64_t)ALIGN * L.NB) * 2);
    L.part_off = take((uint64_t)L.C << bits << 2);
    L.bytes = o;
    return L;
}

// The keys of tile t, four at a time where whole, each passed to f.
template <typename F>
__device__ __forceinline__ void tile_keys(const uint32_t *__restrict__ keys, uint64_t M, uint32_t t, F f) {
    const uint64_t k0 = (uint64_t)t * TILE;
    const uint64_t k1 = k0 + TILE < M ? k0 + TILE : M;
    const uint64_t v1 = k1 >> 2;  // whole vectors below k1 (k0 is a multiple of 4)
    const u32x4 *kv = (const u32x4 *)keys;
    for (uint64_t v = (k0 >> 2) + threadIdx.x; v < v1; v += TILE_THREADS) {
        const u32x4 q = kv[v];
        f(q.x);
        f(q.y);
        f(q.z);
        f(q.w);
    }
    for (uint64_t k = (v1 << 2) + threadIdx.x; k < k1; k += TILE_THREADS) f(keys[k]);
}

// cnt[b * T + t] = keys of tile t in bucket b.  Keys of bucket NB or above
// (never produced by the sweep kernels) are skipped here and in the scatter.
__global__ void __launch_bounds__(TILE_THREADS) count_kernel(const uint32_t *__restrict__ keys, uint64_t M,
                                                            Layout L, unsigned char *__restrict__ ws) {
    __shared__ uint32_t c[KEYHIST_MAX_BUCKETS];
    for (uint32_t b = threadIdx.x; b < L.NB; b += TILE_THREADS) c[b] = 0u;
    __syncthreads();
    tile_keys(keys, M, blockIdx.x, [&](uint32_t k) {
        const uint32_t b = k >> L.lb;
        if (b < L.NB) atomicAdd(&c[b], 1u);
    });
    __syncthreads();
    uint32_t *cnt = (uint32_t *)(ws + L.cnt_off);
    for (uint32_t b = threadIdx.x; b < L.NB; b += TILE_THREADS) cnt[(uint64_t)b * L.T + blockIdx.x] = c[b];
}

// Workgroup b: exclusive prefix of bucket b's tile counts, in place; the
// bucket's size rounded up to ALIGN goes to size[b], the size itself to
// size[NB + b].
__global__ void __launch_bounds__(256) scan_kernel(Layout L, unsigned char *__restrict__ ws) {
    __shared__ uint32_t part[256];
    uint32_t *col = (uint32_t *)(ws + L.cnt_off) + (uint64_t)blockIdx.x * L.T;
    const uint32_t per = (L.T + 255) / 256;
    const uint32_t i0 = std::min(threadIdx.x * per, L.T);
    const uint32_t i1 = std::min(i0 + per, L.T);
    uint32_t s = 0;
    for (uint32_t i = i0; i < i1; ++i) s += col[i];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (uint32_t k = 0; k < 256; ++k) {
            const uint32_t v = part[k];
            part[k] = run;
            run += v;
        }
        uint32_t *size = (uint32_t *)(ws + L.size_off);
        size[blockIdx.x] = (run + ALIGN - 1) & ~(ALIGN - 1);
        size[L.NB + blockIdx.x] = run;
    }
    __syncthreads();
    uint32_t run = part[threadIdx.x];
    for (uint32_t i = i0; i < i1; ++i) {
        const uint32_t v = col[i];
        col[i] = run;
        run += v;
    }
}

// base[b] = sum of the aligned sizes of the buckets below b.
__global__ void __launch_bounds__(64) base_kernel(Layout L, unsigned char *__restrict__ ws) {
    if (threadIdx.x != 0) return;
    const uint32_t *size = (const uint32_t *)(ws + L.size_off);
    uint32_t *base = (uint32_t *)(ws + L.base_off);
    uint32_t run = 0;
    for (uint32_t b = 0; b < L.NB; ++b) {
        base[b] = run;
        run += size[b];
    }
}

// Each key's low bits go to its bucket's region, at the tile's offset there
// plus its rank within the tile (the order inside a bucket is immaterial).
// The tile is first sorted by bucket in LDS (rank by LDS atomic, bucket
// starts by a scan), so consecutive threads then write consecutive 16-bit
// words of each bucket's run.
__global__ void __launch_bounds__(TILE_THREADS) scatter_kernel(const uint32_t *__restrict__ keys, uint64_t M,
                                                              Layout L, unsigned char *__restrict__ ws) {
    constexpr uint32_t PER = TILE / TILE_THREADS;  // keys per thread
    __shared__ uint32_t rank[KEYHIST_MAX_BUCKETS];
    __shared__ uint32_t start[KEYHIST_MAX_BUCKETS];
    __shared__ uint32_t goff[KEYHIST_MAX_BUCKETS];
    __shared__ uint32_t sorted[TILE];
    const uint32_t *cnt = (const uint32_t *)(ws + L.cnt_off);
    const uint32_t *base = (const uint32_t *)(ws + L.base_off);
    for (uint32_t b = threadIdx.x; b < L.NB; b += TILE_THREADS) {
        rank[b] = 0u;
        goff[b] = base[b] + cnt[(uint64_t)b * L.T + blockIdx.x];
    }
    __syncthreads();
    const uint64_t k0 = (uint64_t)blockIdx.x * TILE;
    const uint64_t k1 = k0 + TILE < M ? k0 + TILE : M;
    uint32_t key[PER], r[PER];
#pragma unroll
    for (uint32_t j = 0; j < PER / 4; ++j) {
        const uint64_t k = k0 + 4ull * (threadIdx.x + j * TILE_THREADS);
        if (k + 4 <= k1) {
            const u32x4 q = *(const u32x4 *)(keys + k);
            key[4 * j] = q.x;
            key[4 * j + 1] = q.y;
            key[4 * j + 2] = q.z;
            key[4 * j + 3] = q.w;
        } else {
#pragma unroll
            for (uint32_t e = 0; e < 4; ++e) key[4 * j + e] = k + e < k1 ? keys[k + e] : 0xFFFFFFFFu;
        }
    }
#pragma unroll
    for (uint32_t e = 0; e < PER; ++e) {
        const uint32_t b = key[e] >> L.lb;
        r[e] = b < L.NB ? atomicAdd(&rank[b], 1u) : 0u;
    }
    __syncthreads();
    // exclusive prefix of the tile's bucket counts
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (uint32_t b = 0; b < L.NB; ++b) {
            start[b] = run;
            run += rank[b];
        }
    }
    __syncthreads();
#pragma unroll
    for (uint32_t e = 0; e < PER; ++e) {
        const uint32_t b = key[e] >> L.lb;
        if (b < L.NB) sorted[start[b] + r[e]] = key[e];
    }
    __syncthreads();
    const uint32_t n = start[L.NB - 1] + rank[L.NB - 1];  // keys of this tile below 2^bits
    uint16_t *out = (uint16_t *)(ws + L.out_off);
    const uint32_t mask = (1u << L.lb) - 1u;
    for (uint32_t i = threadIdx.x; i < n; i += TILE_THREADS) {
        const uint32_t k = sorted[i];
        const uint32_t b = k >> L.lb;
        out[goff[b] + (i - start[b])] = (uint16_t)(k & mask);
    }
}

// Workgroup w = c * NB + b: chunk c of bucket b's keys counted in LDS and
// written to partial row c.
__global__ void __launch_bounds__(HIST_THREADS) bucket_kernel(Layout L, unsigned char *__restrict__ ws) {
    __shared__ uint32_t h[1u << LDS_BITS];
    const uint32_t b = blockIdx.x % L.NB, c = blockIdx.x / L.NB;
    const uint32_t nbin = 1u << L.lb;
    for (uint32_t i = threadIdx.x; i < nbin; i += HIST_THREADS) h[i] = 0u;
    __syncthreads();
    const uint32_t n = ((const uint32_t *)(ws + L.size_off))[L.NB + b];
    const uint32_t base = ((const uint32_t *)(ws + L.base_off))[b];
    const uint32_t per = ((n + L.C - 1) / L.C + ALIGN - 1) & ~(ALIGN - 1);
    const uint32_t e0 = std::min(c * per, n);
    const uint32_t e1 = std::min(e0 + per, n);
    const uint16_t *keys = (const uint16_t *)(ws + L.out_off) + base;
    // the region and e0 start at multiples of 8 keys: 16-byte vectors, then the tail
    const u32x4 *kv = (const u32x4 *)(keys + e0);
    const uint32_t nv = (e1 - e0) / 8;
    for (uint32_t v = threadIdx.x; v < nv; v += HIST_THREADS) {
        const u32x4 q = kv[v];
        atomicAdd(&h[q.x & 0xFFFFu], 1u);
        atomicAdd(&h[q.x >> 16], 1u);
        atomicAdd(&h[q.y & 0xFFFFu], 1u);
        atomicAdd(&h[q.y >> 16], 1u);
        atomicAdd(&h[q.z & 0xFFFFu], 1u);
        atomicAdd(&h[q.z >> 16], 1u);
        atomicAdd(&h[q.w & 0xFFFFu], 1u);
        atomicAdd(&h[q.w >> 16], 1u);
    }
    for (uint32_t e = e0 + nv * 8 + threadIdx.x; e < e1; e += HIST_THREADS) atomicAdd(&h[keys[e]], 1u);
    __syncthreads();
    uint32_t *row = (uint32_t *)(ws + L.part_off) + ((uint64_t)c << L.bits) + ((uint64_t)b << L.lb);
    for (uint32_t i = threadIdx.x; i < nbin; i += HIST_THREADS) row[i] = h[i];
}

__global__ void __launch_bounds__(256) reduce_kernel(Layout L, const unsigned char *__restrict__ ws,
                                                    uint32_t *__restrict__ hist) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i >= (1u << L.bits)) return;
    const uint32_t *part = (const uint32_t *)(ws + L.part_off);
    uint32_t acc[4] = {0u, 0u, 0u, 0u};
    uint32_t c = 0;
    for (; c + 4 <= L.C; c += 4) {
#pragma unroll
        for (uint32_t r = 0; r < 4; ++r) acc[r] += part[((uint64_t)(c + r) << L.bits) + i];
    }
    for (; c < L.C; ++c) acc[0] += part[((uint64_t)c << L.bits) + i];
    const uint32_t v = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    if (v) hist[i] += v;
}

}  // namespace

size_t keyhist_scratch_bytes(uint64_t M, uint32_t bits) { return (size_t)layout(M, bits).bytes; }

hipError_t launch_keyhist(const uint32_t *keys, uint64_t M, uint32_t bits, void *scratch, uint32_t *hist,
                          hipStream_t s) {
    if (!M) return hipSuccess;
    if (bits > KEYHIST_MAX_BITS || M > KEYHIST_MAX_KEYS) return hipErrorInvalidValue;
    const Layout L = layout(M, bits);
    unsigned char *ws = (unsigned char *)scratch;
    hipLaunchKernelGGL(count_kernel, dim3(L.T), dim3(TILE_THREADS), 0, s, keys, M, L, ws);
    hipLaunchKernelGGL(scan_kernel, dim3(L.NB), dim3(256), 0, s, L, ws);
    hipLaunchKernelGGL(base_kernel, dim3(1), dim3(64), 0, s, L, ws);
    hipLaunchKernelGGL(scatter_kernel, dim3(L.T), dim3(TILE_THREADS), 0, s, keys, M, L, ws);
    hipLaunchKernelGGL(bucket_kernel, dim3(L.NB * L.C), dim3(HIST_THREADS), 0, s, L, ws);
    hipLaunchKernelGGL(reduce_kernel, dim3(((1u << bits) + 255) / 256), dim3(256), 0, s, L, ws, hist);
    return hipGetLastError();
}

}  // namespace pbit
