// Stable LSD radix sort of 32-bit keys (below 2^bits) carrying 32-bit
// values, 7 bits per pass.  A pass counts the digits of every tile of
// kSortTile consecutive elements, takes the exclusive prefix of the counts in
// digit-major order (digit d of tile t after every tile of smaller digits and
// every earlier tile of digit d), and scatters a tile per workgroup: each
// wavefront ranks its quarter of the tile in index order, 64 elements per
// step, by a match mask built from seven ballots; the ranks, prefixed over
// the earlier wavefronts and digits, place the tile in LDS sorted by digit,
// and the workgroup writes each digit's run to its contiguous destination.
// Equal keys keep their input order, so the output is the same on every run.
#pragma once

#include <algorithm>

#include "bucket.hpp"
#include "common.hpp"

namespace hermes {

constexpr int kSortBits = 7;
constexpr int kSortDigits = 1 << kSortBits;
constexpr int kSortWaves = kThreads / 64;
constexpr int kSortPer = 16;                              // elements per thread of a tile
constexpr int kSortTile = kThreads * kSortPer;            // 4096 elements per tile (workgroup)
constexpr int kSortWaveElems = kSortTile / kSortWaves;    // a wavefront's contiguous quarter

inline int64_t sort_tiles(int64_t n) { return n > 0 ? (n + kSortTile - 1) / kSortTile : 1; }
inline int sort_passes(uint32_t max_key) {
    int bits = 1;
    while (bits < 32 && (max_key >> bits) != 0) ++bits;
    return (bits + kSortBits - 1) / kSortBits;
}

// Workspace (bytes, each part 256-aligned): the second key and value
// buffers, the digit counts, their prefix and the scan's scratch.
struct SortLayout {
    size_t key2, val2, hist, hoff, tmp, total;
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
    l.tmp = at;
    at += align256(size_t(scan_tmp_entries(m)) * 4);
    l.total = at;
    return l;
}

// hist[d * ntiles + t] = the number of elements of tile t with digit d.
static __global__ __launch_bounds__(kThreads) void k_sort_hist(const uint32_t* __restrict__ key, int64_t n,
                                                               int64_t ntiles, int shift,
                                                               uint32_t* __restrict__ hist) {
    __shared__ uint32_t cnt[kSortDigits];
    const int64_t t = blockIdx.x;
    for (int d = threadIdx.x; d < kSortDigits; d += kThreads) cnt[d] = 0u;
    __syncthreads();
    const int64_t b0 = t * kSortTile, end = std::min(n, b0 + kSortTile);
    for (int64_t i = b0 + threadIdx.x; i < end; i += kThreads) atomicAdd(&cnt[(key[i] >> shift) & (kSortDigits - 1)], 1u);
    __syncthreads();
    for (int d = threadIdx.x; d < kSortDigits; d += kThreads) hist[int64_t(d) * ntiles + t] = cnt[d];
}

// Stable scatter of one pass, one tile per workgroup; val_in NULL means
// value = index, key_out NULL skips the keys (the last pass may need only
// the values).
static __global__ __launch_bounds__(kThreads) void k_sort_scatter(const uint32_t* __restrict__ key_in,
                                                                  const uint32_t* __restrict__ val_in, int64_t n,
                                                                  int64_t ntiles, int shift,
                                                                  const uint32_t* __restrict__ hoff,
                                                                  uint32_t* __restrict__ key_out,
                                                                  uint32_t* __restrict__ val_out) {
    __shared__ uint32_t wcnt[kSortWaves][kSortDigits];   // per wavefront: counts, then exclusive prefix over waves
    __shared__ uint32_t dstart[kSortDigits];             // the tile's first slot of each digit
    __shared__ uint32_t gbase[kSortDigits];              // the destination of that slot
    __shared__ uint32_t lkey[kSortTile], lval[kSortTile];
    const int wv = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int64_t t = blockIdx.x;
    const int64_t b0 = t * kSortTile;
    const int cnt_tile = int(std::min<int64_t>(kSortTile, n - b0));
    for (int e = threadIdx.x; e < kSortWaves * kSortDigits; e += kThreads) wcnt[e / kSortDigits][e % kSortDigits] = 0u;
    for (int d = threadIdx.x; d < kSortDigits; d += kThreads) gbase[d] = hoff[int64_t(d) * ntiles + t];
    // this wavefront's elements, loaded together
    uint32_t kb[kSortPer], vb[kSortPer];
    const int64_t w0 = b0 + int64_t(wv) * kSortWaveElems;
#pragma unroll
    for (int u = 0; u < kSortPer; ++u) {
        const int64_t i = w0 + 64 * u + lane;
        kb[u] = i < b0 + cnt_tile ? key_in[i] : 0u;
        vb[u] = i < b0 + cnt_tile ? (val_in ? val_in[i] : uint32_t(i)) : 0u;
    }
    __syncthreads();   // wcnt zeroed
    // rank within the wavefront's quarter, in index order
    const uint64_t below = (uint64_t(1) << lane) - 1;
    uint32_t rank[kSortPer];
#pragma unroll
    for (int u = 0; u < kSortPer; ++u) {
        const bool valid = w0 + 64 * u + lane < b0 + cnt_tile;
        const int d = int((kb[u] >> shift) & (kSortDigits - 1));
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < kSortBits; ++b) {
            const bool bit = (d >> b) & 1;
            const uint64_t bb = __ballot(valid && bit);
            m &= bit ? bb : ~bb;
        }
        const uint32_t start = valid ? wcnt[wv][d] : 0u;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (valid && (m & below) == 0) wcnt[wv][d] = start + uint32_t(__popcll(m));
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        rank[u] = start + uint32_t(__popcll(m & below));
    }
    __syncthreads();
    // per digit (thread d < 128, two wavefronts): exclusive prefix over the
    // wavefronts, then an exclusive scan over the digits by lane shuffles,
    // the second wavefront adding the first one's total
    __shared__ uint32_t half_total;
    uint32_t tot = 0, incl = 0;
    if (threadIdx.x < kSortDigits) {
        const int d = threadIdx.x;
        for (int w = 0; w < kSortWaves; ++w) {
            const uint32_t c = wcnt[w][d];
            wcnt[w][d] = tot;
            tot += c;
        }
        incl = tot;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(incl, o);
            if (lane >= o) incl += y;
        }
        if (threadIdx.x == 63) half_total = incl;
    }
    __syncthreads();
    if (threadIdx.x < kSortDigits) dstart[threadIdx.x] = incl - tot + (threadIdx.x >= 64 ? half_total : 0u);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kSortPer; ++u) {
        if (w0 + 64 * u + lane < b0 + cnt_tile) {
            const int d = int((kb[u] >> shift) & (kSortDigits - 1));
            const uint32_t pos = dstart[d] + wcnt[wv][d] + rank[u];
            lkey[pos] = kb[u];
            lval[pos] = vb[u];
        }
    }
    __syncthreads();
    // slot i of the sorted tile goes to gbase[d] + (i - dstart[d]): runs of
    // one digit land contiguously
    for (int i = threadIdx.x; i < cnt_tile; i += kThreads) {
        const uint32_t k = lkey[i];
        const int d = int((k >> shift) & (kSortDigits - 1));
        const uint32_t dst = gbase[d] + (uint32_t(i) - dstart[d]);
        if (key_out) key_out[dst] = k;
        val_out[dst] = lval[i];
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
    uint32_t* tmp = reinterpret_cast<uint32_t*>(work + l.tmp);
    const int64_t ntiles = sort_tiles(n);
    const int passes = sort_passes(max_key);
    // ping-pong so that the last pass writes val_out
    uint32_t* kin = key;
    const uint32_t* vin = nullptr;
    for (int p = 0; p < passes; ++p) {
        const bool last = p == passes - 1;
        uint32_t* kout = last ? key_sorted : (kin == key ? key2 : key);
        uint32_t* vout = last ? val_out : ((passes - 1 - p) % 2 == 1 ? val2 : val_out);
        const int shift = p * kSortBits;
        hipLaunchKernelGGL(k_sort_hist, dim3(unsigned(ntiles)), dim3(kThreads), 0, stream, kin, n, ntiles, shift,
                           hist);
        launch_scan(hist, int64_t(kSortDigits) * ntiles, hoff, tmp, stream);
        hipLaunchKernelGGL(k_sort_scatter, dim3(unsigned(ntiles)), dim3(kThreads), 0, stream, kin, vin, n, ntiles,
                           shift, hoff, kout, vout);
        kin = kout;
        vin = vout;
    }
}

}  // namespace hermes
