// Stable LSD radix sort of 32-bit keys (below 2^bits) carrying 32-bit
// values, 7 bits per pass.  A pass counts the digits of every tile of T
// consecutive elements, takes the exclusive prefix of the counts in
// digit-major order (digit d of tile t after every tile of smaller digits and
// every earlier tile of digit d), and scatters: one wavefront walks its tile
// in index order, 64 elements per step, and ranks the lanes that share a
// digit by a match mask built from seven ballots.  Equal keys keep their
// input order, so the output is the same on every run.
#pragma once

#include <algorithm>

#include "bucket.hpp"
#include "common.hpp"

namespace hermes {

constexpr int kSortBits = 7;
constexpr int kSortDigits = 1 << kSortBits;
constexpr int kSortWaves = kThreads / 64;   // tiles per workgroup (one per wavefront)
constexpr int kSortBatch = 8;               // 64-element steps whose loads are issued together

// Elements per tile: a multiple of 64, large enough that the digit-count
// matrix stays within the scan's reach (kScanBlock^2 entries).
inline int64_t sort_tile(int64_t n) {
    const int64_t max_tiles = int64_t(kScanBlock) * kScanBlock / kSortDigits;
    int64_t steps = 16;
    while ((n + 64 * steps - 1) / (64 * steps) > max_tiles) steps *= 2;
    return 64 * steps;
}
inline int64_t sort_tiles(int64_t n) {
    const int64_t t = sort_tile(n);
    return n > 0 ? (n + t - 1) / t : 1;
}
inline int sort_passes(uint32_t max_key) {
    int bits = 1;
    while (bits < 32 && (max_key >> bits) != 0) ++bits;
    return (bits + kSortBits - 1) / kSortBits;
}

// Workspace (bytes, each part 256-aligned): the second key and value
// buffers, the digit counts, their prefix and the scan's block sums.
struct SortLayout {
    size_t key2, val2, hist, hoff, blocksum, total;
};

inline SortLayout sort_layout(int64_t n) {
    const int64_t m = int64_t(kSortDigits) * sort_tiles(n);
    SortLayout l{};
    size_t at = 0;
    l.key2 = at;
    at += align256(size_t(n) * 4);
    l.val2 = at;
    at += align256(size_t(n) * 4);
    l.hist = at;
    at += align256(size_t(m) * 4);
    l.hoff = at;
    at += align256(size_t(m + 1) * 4);
    l.blocksum = at;
    at += align256(size_t((m + kScanBlock - 1) / kScanBlock) * 4);
    l.total = at;
    return l;
}

// hist[d * ntiles + t] = the number of elements of tile t with digit d.
static __global__ __launch_bounds__(kThreads) void k_sort_hist(const uint32_t* __restrict__ key, int64_t n,
                                                               int64_t tile, int64_t ntiles, int shift,
                                                               uint32_t* __restrict__ hist) {
    __shared__ uint32_t cnt[kSortWaves][kSortDigits];
    const int wv = threadIdx.x / 64, lane = threadIdx.x % 64;
    for (int d = lane; d < kSortDigits; d += 64) cnt[wv][d] = 0u;
    __syncthreads();
    const int64_t t = int64_t(blockIdx.x) * kSortWaves + wv;
    if (t < ntiles) {
        const int64_t end = std::min(n, (t + 1) * tile);
        for (int64_t i = t * tile + lane; i < end; i += 64) atomicAdd(&cnt[wv][(key[i] >> shift) & (kSortDigits - 1)], 1u);
    }
    __syncthreads();
    if (t < ntiles)
        for (int d = lane; d < kSortDigits; d += 64) hist[int64_t(d) * ntiles + t] = cnt[wv][d];
}

// Stable scatter of one pass; val_in NULL means value = index.  key_out may
// be NULL (last pass: only the values are needed).
static __global__ __launch_bounds__(kThreads) void k_sort_scatter(const uint32_t* __restrict__ key_in,
                                                                  const uint32_t* __restrict__ val_in, int64_t n,
                                                                  int64_t tile, int64_t ntiles, int shift,
                                                                  const uint32_t* __restrict__ hoff,
                                                                  uint32_t* __restrict__ key_out,
                                                                  uint32_t* __restrict__ val_out) {
    __shared__ uint32_t cnt[kSortWaves][kSortDigits];
    const int wv = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int64_t t = int64_t(blockIdx.x) * kSortWaves + wv;
    if (t >= ntiles) return;   // whole wavefront; no workgroup barrier follows
    for (int d = lane; d < kSortDigits; d += 64) cnt[wv][d] = hoff[int64_t(d) * ntiles + t];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const uint64_t below = (uint64_t(1) << lane) - 1;
    const int64_t end = std::min(n, (t + 1) * tile);
    // kSortBatch steps' keys and values are loaded together (their latencies
    // overlap), then ranked step by step in index order
    for (int64_t base0 = t * tile; base0 < end; base0 += 64 * kSortBatch) {   // uniform over the wavefront
        uint32_t kb[kSortBatch], vb[kSortBatch];
#pragma unroll
        for (int u = 0; u < kSortBatch; ++u) {
            const int64_t i = base0 + 64 * u + lane;
            kb[u] = i < end ? key_in[i] : 0u;
            vb[u] = i < end ? (val_in ? val_in[i] : uint32_t(i)) : 0u;
        }
#pragma unroll
        for (int u = 0; u < kSortBatch; ++u) {
            const int64_t base = base0 + 64 * u;
            if (base >= end) break;   // uniform
            const bool valid = base + lane < end;
            const uint32_t k = kb[u], v = vb[u];
            const int d = int((k >> shift) & (kSortDigits - 1));
            uint64_t m = __ballot(valid);
#pragma unroll
            for (int b = 0; b < kSortBits; ++b) {
                const bool bit = (d >> b) & 1;
                const uint64_t bb = __ballot(valid && bit);
                m &= bit ? bb : ~bb;
            }
            // every lane of digit d reads the same running offset, then the
            // lowest of them advances it by the group's size
            const uint32_t start = cnt[wv][d];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (valid && (m & below) == 0) cnt[wv][d] = start + uint32_t(__popcll(m));
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (valid) {
                const uint32_t dst = start + uint32_t(__popcll(m & below));
                if (key_out) key_out[dst] = k;
                val_out[dst] = v;
            }
        }
    }
}

// off[t] = the first slot of key t in the sorted keys skey[0 .. n), for
// t = 0 .. n_keys (off[n_keys] = n): every slot whose key differs from the
// previous slot's opens the keys in between.
static __global__ __launch_bounds__(kThreads) void k_sorted_offsets(const uint32_t* __restrict__ skey, int64_t n,
                                                                    int64_t n_keys, uint32_t* __restrict__ off) {
    const int64_t stride = int64_t(gridDim.x) * kThreads;
    for (int64_t j = int64_t(blockIdx.x) * kThreads + threadIdx.x; j < n; j += stride) {
        const int64_t k = skey[j];
        const int64_t prev = j > 0 ? int64_t(skey[j - 1]) : -1;
        for (int64_t t = prev + 1; t <= k; ++t) off[t] = uint32_t(j);
        if (j == n - 1)
            for (int64_t t = k + 1; t <= n_keys; ++t) off[t] = uint32_t(n);
    }
}

// Sort key[0 .. n) (keys <= max_key) with values 0 .. n-1; the values in key
// order end in val_out, and the sorted keys in key_sorted when it is given.
// key is overwritten.  n < 2^32.
inline void radix_sort_indices(uint32_t* key, int64_t n, uint32_t max_key, uint32_t* val_out, char* work,
                               hipStream_t stream, uint32_t* key_sorted = nullptr) {
    if (n <= 0) return;
    const SortLayout l = sort_layout(n);
    uint32_t* key2 = reinterpret_cast<uint32_t*>(work + l.key2);
    uint32_t* val2 = reinterpret_cast<uint32_t*>(work + l.val2);
    uint32_t* hist = reinterpret_cast<uint32_t*>(work + l.hist);
    uint32_t* hoff = reinterpret_cast<uint32_t*>(work + l.hoff);
    uint32_t* bsum = reinterpret_cast<uint32_t*>(work + l.blocksum);
    const int64_t tile = sort_tile(n), ntiles = sort_tiles(n);
    const int blocks = int((ntiles + kSortWaves - 1) / kSortWaves);
    const int passes = sort_passes(max_key);
    // ping-pong so that the last pass writes val_out
    uint32_t* kin = key;
    const uint32_t* vin = nullptr;
    for (int p = 0; p < passes; ++p) {
        const bool last = p == passes - 1;
        uint32_t* kout = last ? key_sorted : (kin == key ? key2 : key);
        uint32_t* vout = last ? val_out : ((passes - 1 - p) % 2 == 1 ? val2 : val_out);
        const int shift = p * kSortBits;
        hipLaunchKernelGGL(k_sort_hist, dim3(blocks), dim3(kThreads), 0, stream, kin, n, tile, ntiles, shift, hist);
        launch_tile_scan(hist, int64_t(kSortDigits) * ntiles, hoff, bsum, stream);
        hipLaunchKernelGGL(k_sort_scatter, dim3(blocks), dim3(kThreads), 0, stream, kin, vin, n, tile, ntiles, shift,
                           hoff, kout, vout);
        kin = kout;
        vin = vout;
    }
}

}  // namespace hermes
