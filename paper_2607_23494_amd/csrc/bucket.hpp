// Bucketing of points by tiles of E^3 cells (E = 16 unless given): the tile
// of a point and the exclusive prefix sum of per-tile counts, used by the
// assignment and the readout (which sort their points by tile) and by the
// radix sort and the triangle sums (prefix sums).
#pragma once

#include "common.hpp"

namespace hermes {

constexpr int kBucketTile = 16;    // cells per tile edge (N >= 16; the whole grid below)
constexpr int kScanBlock = 1024;   // entries per block of the tile-offset scan

template <int N, int E = kBucketTile> struct tile_grid {
    static constexpr int TS = N < E ? N : E;
    static constexpr int NT = N / TS;                // tiles per axis
    static constexpr int TILES = NT * NT * NT;
};

// Cell of a position along one axis (periodic wrap into [0, N)) and the
// fractional offset within it, in float64.
template <int N>
__device__ __forceinline__ int cell_of(float x, double scale, double& frac) {
    double u = double(x) * scale;
    u -= double(N) * floor(u / double(N));
    const double f = floor(u);
    int c = int(f);
    frac = u - f;
    if (c >= N) {   // u rounded up to N: the next image's node 0
        c = 0;
        frac = 0.0;
    }
    return c;
}

template <int N, int E = kBucketTile>
__device__ __forceinline__ int tile_of_point(const float* __restrict__ pos, int64_t i, double scale) {
    using G = tile_grid<N, E>;
    double f;
    const int cx = cell_of<N>(pos[3 * i], scale, f);
    const int cy = cell_of<N>(pos[3 * i + 1], scale, f);
    const int cz = cell_of<N>(pos[3 * i + 2], scale, f);
    return ((cx / G::TS) * G::NT + cy / G::TS) * G::NT + cz / G::TS;
}

// Exclusive prefix sum of cnt[0 .. n) in blocks of kScanBlock: the block's
// prefix to out, its total to blocksum.
static __global__ __launch_bounds__(kScanBlock) void k_scan_block(const uint32_t* __restrict__ cnt, int64_t n,
                                                                  uint32_t* __restrict__ out,
                                                                  uint32_t* __restrict__ blocksum) {
    __shared__ uint32_t s[kScanBlock];
    const int64_t i = int64_t(blockIdx.x) * kScanBlock + threadIdx.x;
    const uint32_t v = i < n ? cnt[i] : 0u;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int d = 1; d < kScanBlock; d <<= 1) {   // inclusive Hillis-Steele scan
        const uint32_t t = threadIdx.x >= d ? s[threadIdx.x - d] : 0u;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    if (i < n) out[i] = s[threadIdx.x] - v;
    if (threadIdx.x == kScanBlock - 1) blocksum[blockIdx.x] = s[threadIdx.x];
}

// Exclusive prefix of the block totals (one block; nblk <= kScanBlock), and
// the grand total at out[n].
static __global__ __launch_bounds__(kScanBlock) void k_scan_totals(uint32_t* __restrict__ blocksum, int nblk,
                                                                   uint32_t* __restrict__ out, int64_t n) {
    __shared__ uint32_t s[kScanBlock];
    const uint32_t v = int(threadIdx.x) < nblk ? blocksum[threadIdx.x] : 0u;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int d = 1; d < kScanBlock; d <<= 1) {
        const uint32_t t = threadIdx.x >= d ? s[threadIdx.x - d] : 0u;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    if (int(threadIdx.x) < nblk) blocksum[threadIdx.x] = s[threadIdx.x] - v;
    if (threadIdx.x == kScanBlock - 1) out[n] = s[threadIdx.x];
}

static __global__ __launch_bounds__(kScanBlock) void k_scan_add(uint32_t* __restrict__ out, int64_t n,
                                                                const uint32_t* __restrict__ blocksum) {
    const int64_t i = int64_t(blockIdx.x) * kScanBlock + threadIdx.x;
    if (i < n) out[i] += blocksum[blockIdx.x];
}

// off[0 .. tiles] = exclusive prefix of count (off[tiles] = total).
inline void launch_tile_scan(const uint32_t* count, int64_t tiles, uint32_t* off, uint32_t* blocksum,
                             hipStream_t stream) {
    const int nblk = int((tiles + kScanBlock - 1) / kScanBlock);
    hipLaunchKernelGGL(k_scan_block, dim3(nblk), dim3(kScanBlock), 0, stream, count, tiles, off, blocksum);
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kScanBlock), 0, stream, blocksum, nblk, off, tiles);
    hipLaunchKernelGGL(k_scan_add, dim3(nblk), dim3(kScanBlock), 0, stream, off, tiles, blocksum);
}

static __global__ void k_scan_set_total(uint32_t* __restrict__ dst, const uint32_t* __restrict__ src) {
    if (threadIdx.x == 0) dst[0] = src[0];
}

// uint32 entries of scratch that launch_scan needs for n counts.
inline int64_t scan_tmp_entries(int64_t n) {
    const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
    return nb <= kScanBlock ? nb : 2 * nb + 1 + scan_tmp_entries(nb);
}

// off[0 .. n] = exclusive prefix of cnt (off[n] = total) for any n < 2^32
// whose total fits 32 bits: blocks of kScanBlock, then the block totals
// scanned the same way (recursively) and added back.
inline void launch_scan(const uint32_t* cnt, int64_t n, uint32_t* off, uint32_t* tmp, hipStream_t stream) {
    const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
    if (nb <= kScanBlock) {
        launch_tile_scan(cnt, n, off, tmp, stream);
        return;
    }
    uint32_t* bs = tmp;            // nb block totals
    uint32_t* boff = tmp + nb;     // their exclusive prefix, nb + 1 entries
    hipLaunchKernelGGL(k_scan_block, dim3(unsigned(nb)), dim3(kScanBlock), 0, stream, cnt, n, off, bs);
    launch_scan(bs, nb, boff, tmp + 2 * nb + 1, stream);
    hipLaunchKernelGGL(k_scan_add, dim3(unsigned(nb)), dim3(kScanBlock), 0, stream, off, n, boff);
    hipLaunchKernelGGL(k_scan_set_total, dim3(1), dim3(64), 0, stream, off + n, boff + nb);
}

}  // namespace hermes
