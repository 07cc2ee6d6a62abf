// MRA projection of a weighted catalogue onto scaling-function
// coefficients (Sec. 3.1, Eq. phi_projection), with B3 (64 taps per point)
// or the D4 function (27 taps).
//
// The taps of every point are accumulated per tile of TS^3 cells in LDS and
// in 64-bit fixed point:
//   1. prep     the tile of every point (by the cell of the point), and the
//               per-block sums of w and |w|
//   2. scale    sum_w (the output) and the fixed-point scale 2^k, chosen from
//               sum |w| so that no cell's sum can overflow: every cell is a
//               sum of contributions of magnitude <= |w_i| M (M = 1 for B3,
//               max |phi|^3 < 4 for D4, whose phi reaches (1 + sqrt3)/2), so
//               |cell| <= sum |w| M 2^k <= 2^61
//   3. sort     a stable radix sort of the points by tile (a tile's points
//               in index order), and each tile's list offset from the sorted
//               keys
//   5. tiles    one workgroup per tile: a wavefront loads 64 points, then
//               for each of them lane t adds tap t (64 distinct cells; D4:
//               27 taps per half-wavefront, two points at a time) to an LDS
//               region of (TS + 3)^3 cells (the tile and the stencil's
//               reach: one cell below and two above for B3, two below for
//               D4); the region is then added to the global accumulator
//               with 64-bit atomics
//   6. convert  eps = acc 2^-k
// Each contribution is rounded once to a multiple of 2^-k; integer addition
// commutes, so the grid is the same bit for bit whatever the order in which
// points, tiles and workgroups are processed.
#include <cmath>

#include "bucket.hpp"
#include "common.hpp"
#include "interp.hpp"
#include "kernels.hpp"
#include "sort.hpp"

namespace hermes {

constexpr int kAsgPrepBlocks = 2048;
constexpr int kTileThreads = 512;  // threads of the per-tile workgroups

template <int N> struct asg_cfg : tile_grid<N> {
    static constexpr int RG = tile_grid<N>::TS + 3;   // LDS region edge
    static constexpr int RCELLS = RG * RG * RG;
};

// Per-call scalars written by k_asg_scale.
struct AsgScale {
    double scale;       // 2^k
    double inv_scale;   // 2^-k
};

inline int asg_prep_blocks(int64_t n_pts) {
    const int64_t want = (n_pts + kThreads - 1) / kThreads;
    return int(want < kAsgPrepBlocks ? (want > 0 ? want : 1) : kAsgPrepBlocks);
}

// Workspace layout (bytes, each part 256-aligned): the accumulator, the
// points' tile keys and the keys in sorted order, the tile offsets, the point
// list in tile order, the prep partials, the scale, the sort's buffers.
struct AsgLayout {
    size_t acc, key, skey, off, list, partial, scale, sort, total;
};

inline AsgLayout asg_layout(int n, int64_t n_pts) {
    const int ts = n < kBucketTile ? n : kBucketTile;
    const int64_t tiles = int64_t(n / ts) * (n / ts) * (n / ts);
    const int64_t np = n_pts > 0 ? n_pts : 1;
    AsgLayout l{};
    size_t at = 0;
    l.acc = at;
    at += align256(size_t(n) * n * n * sizeof(int64_t));
    l.key = at;
    at += align256(size_t(np) * 4);
    l.skey = at;
    at += align256(size_t(np) * 4);
    l.off = at;
    at += align256(size_t(tiles + 1) * 4);
    l.list = at;
    at += align256(size_t(np) * 4);
    l.partial = at;
    at += align256(size_t(asg_prep_blocks(n_pts)) * 2 * sizeof(double));
    l.scale = at;
    at += align256(sizeof(AsgScale));
    l.sort = at;
    at += sort_layout(np).total;
    l.total = at;
    return l;
}

size_t assign_workspace(int n, int64_t n_pts) { return asg_layout(n, n_pts).total; }

// B3 weight of node i0 - 1 + o (o = 0 .. 3) for the fractional offset t in
// [0, 1): B3 at distance d = |t + 1 - o| < 2, without branches.
template <typename T>
__device__ __forceinline__ T b3_tap(T t, int o) {
    const T d = fabs(t + T(1 - o));
    const T e = T(2) - d;
    constexpr T kSixth = T(1) / T(6);
    return d < T(1) ? (T(4) - T(6) * d * d + T(3) * d * d * d) * kSixth : e * e * e * kSixth;
}

// Broadcast of lane j's value (j uniform across the wavefront).
__device__ __forceinline__ int bcast(int v, int j) { return __builtin_amdgcn_readlane(v, j); }
__device__ __forceinline__ float bcast(float v, int j) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
}
__device__ __forceinline__ double bcast(double v, int j) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane(int(b & 0xffffffffll), j);
    const int hi = __builtin_amdgcn_readlane(int(b >> 32), j);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

template <int N>
__global__ __launch_bounds__(kThreads) void k_asg_prep(const float* __restrict__ pos, const float* __restrict__ weight,
                                                       int64_t n_pts, double scale, uint32_t* __restrict__ key,
                                                       double* __restrict__ partial) {
    __shared__ double red[kThreads];
    double s = 0.0, sa = 0.0;
    const int64_t stride = int64_t(gridDim.x) * kThreads;
    for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < n_pts; i += stride) {
        const double w = weight ? double(weight[i]) : 1.0;
        s += w;
        sa += fabs(w);
        key[i] = uint32_t(tile_of_point<N>(pos, i, scale));
    }
    s = block_sum(s, red);
    sa = block_sum(sa, red);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = s;
        partial[2 * blockIdx.x + 1] = sa;
    }
}

// sum_w and the fixed-point scale 2^k, k = 61 - head - ceil(log2(sum |w|)),
// from the per-block partials (2^head bounds a point's largest tap weight).
// One workgroup: thread t adds the partials t, t + kThreads, ... in order,
// then the fixed tree of block_sum, so the sums repeat bit for bit.
__global__ __launch_bounds__(kThreads) void k_asg_scale(const double* __restrict__ partial, int nblocks, int head,
                                                        double* __restrict__ sum_w, AsgScale* __restrict__ sc) {
    __shared__ double red[kThreads];
    double s = 0.0, sa = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kThreads) {
        s += partial[2 * b];
        sa += partial[2 * b + 1];
    }
    s = block_sum(s, red);
    sa = block_sum(sa, red);
    if (threadIdx.x != 0) return;
    sum_w[0] = s;
    int e = 0;
    if (sa > 0.0) {
        frexp(sa, &e);   // sa < 2^e
    }
    const int k = min(1000, 61 - head - e);   // 2^k stays finite for tiny weights
    sc->scale = ldexp(1.0, k);
    sc->inv_scale = ldexp(1.0, -k);
}

// One workgroup per tile.  A wavefront takes 64 of the tile's points at a
// time, one per lane (index, weight, cell and fractions, computed once), then
// walks through them.  B3: for point j, lane t adds tap t = (ox, oy, oz) =
// (t / 16, t / 4 % 4, t % 4); D4: lanes 0-26 add the 27 taps (t / 9, t / 3 % 3,
// t % 3) of point j and lanes 32-58 those of point j + 1.  The cell
// i0 - LO + o of a tap sits at local index i0 - tile origin + o in
// [0, TS + 2] per axis of the region, whose origin is LO cells below the
// tile; the taps of one point hit distinct cells.  In float32 with B3 each
// lane first evaluates the twelve axis weights of its own point into the
// wavefront's LDS rows (row a 4 + o holds b3_tap(frac_a, o) of the 64
// points, rows 65 apart so that the four rows a tap instruction reads sit
// on different banks), and the tap of point j multiplies three of them: the
// same products in the same order as evaluating them per tap.
template <typename T, int N, int B>
__global__ __launch_bounds__(kTileThreads) void k_asg_tiles(const float* __restrict__ pos, const float* __restrict__ weight,
                                                        double scale, const uint32_t* __restrict__ off,
                                                        const uint32_t* __restrict__ list,
                                                        const AsgScale* __restrict__ sc,
                                                        const double* __restrict__ tab,
                                                        unsigned long long* __restrict__ acc) {
    using G = asg_cfg<N>;
    constexpr int TS = G::TS, NT = G::NT, RG = G::RG, RCELLS = G::RCELLS;
    constexpr int LO = BasisTaps<B>::LO;
    constexpr int NW = kTileThreads / 64;
    __shared__ unsigned long long reg[RCELLS];
    constexpr bool STAGE = B == HERMES_BASIS_B3 && sizeof(T) == 4;   // axis weights staged in LDS
    constexpr int WROW = 65;
    __shared__ float wax[STAGE ? NW * 12 * WROW : 1];
    const int tile = blockIdx.x;
    const uint32_t p0 = off[tile], p1 = off[tile + 1];
    if (p0 == p1) return;   // uniform: an empty tile adds nothing
    const int tx = tile / (NT * NT), ty = (tile / NT) % NT, tz = tile % NT;
    const int ox0 = tx * TS, oy0 = ty * TS, oz0 = tz * TS;
    for (int c = threadIdx.x; c < RCELLS; c += kTileThreads) reg[c] = 0ull;
    __syncthreads();
    const double fxp = sc->scale;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), lane = threadIdx.x % 64;
    // this lane's tap (and, for D4, which of the two points it serves)
    const int half = B == HERMES_BASIS_DB2 ? lane >> 5 : 0;
    const int sub = B == HERMES_BASIS_DB2 ? lane & 31 : lane;
    const bool on = B == HERMES_BASIS_DB2 ? sub < 27 : true;
    const int ox = B == HERMES_BASIS_DB2 ? sub / 9 : lane >> 4;
    const int oy = B == HERMES_BASIS_DB2 ? (sub / 3) % 3 : (lane >> 2) & 3;
    const int oz = B == HERMES_BASIS_DB2 ? sub % 3 : lane & 3;
    const int tap = (ox * RG + oy) * RG + oz;
    for (uint32_t k0 = p0 + 64u * wv; k0 < p1; k0 += 64u * NW) {
        const uint32_t k = k0 + lane;
        int loc = 0;
        T fx = T(0), fy = T(0), fz = T(0);
        double wq = 0.0;
        if (k < p1) {
            const uint32_t i = list[k];
            double frx, fry, frz;
            const int cx = cell_of<N>(pos[3 * size_t(i)], scale, frx);
            const int cy = cell_of<N>(pos[3 * size_t(i) + 1], scale, fry);
            const int cz = cell_of<N>(pos[3 * size_t(i) + 2], scale, frz);
            loc = ((cx - ox0) * RG + (cy - oy0)) * RG + (cz - oz0);
            fx = T(frx);
            fy = T(fry);
            fz = T(frz);
            wq = (weight ? double(weight[i]) : 1.0) * fxp;
        }
        const int cnt = int(min(64u, p1 - k0));
        if constexpr (B == HERMES_BASIS_DB2) {
            for (int j = 0; j < cnt; j += 2) {
                // lanes of the upper half take point j + 1 (if there is one)
                const int jj = j + 1 < cnt ? j + 1 : j;
                const double tx = half ? bcast(double(fx), jj) : bcast(double(fx), j);
                const double ty = half ? bcast(double(fy), jj) : bcast(double(fy), j);
                const double tz = half ? bcast(double(fz), jj) : bcast(double(fz), j);
                const double wj = half ? bcast(wq, jj) : bcast(wq, j);
                const int lj = half ? bcast(loc, jj) : bcast(loc, j);
                if (on && (half == 0 || j + 1 < cnt)) {
                    const double wt = db2_phi(tx + double(LO - ox), tab) * db2_phi(ty + double(LO - oy), tab) *
                                      db2_phi(tz + double(LO - oz), tab);
                    const long long q = llrint(wj * wt);
                    atomicAdd(&reg[lj + tap], (unsigned long long)q);
                }
            }
        } else if constexpr (STAGE) {
            float* wrow = wax + wv * 12 * WROW;
            const T fr[3] = {fx, fy, fz};
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int o = 0; o < 4; ++o) wrow[(4 * a + o) * WROW + lane] = b3_tap<T>(fr[a], o);
            wave_sync();
            const float* rx = wrow + ox * WROW;
            const float* ry = wrow + (4 + oy) * WROW;
            const float* rz = wrow + (8 + oz) * WROW;
            for (int j = 0; j < cnt; ++j) {
                const T wt = rx[j] * ry[j] * rz[j];
                const long long q = llrint(bcast(wq, j) * double(wt));
                atomicAdd(&reg[bcast(loc, j) + tap], (unsigned long long)q);
            }
            wave_sync();   // every lane's reads of this batch precede the next batch's writes
        } else {
            for (int j = 0; j < cnt; ++j) {
                const T wt = b3_tap<T>(bcast(fx, j), ox) * b3_tap<T>(bcast(fy, j), oy) * b3_tap<T>(bcast(fz, j), oz);
                const long long q = llrint(bcast(wq, j) * double(wt));
                atomicAdd(&reg[bcast(loc, j) + tap], (unsigned long long)q);
            }
        }
    }
    __syncthreads();
    for (int c = threadIdx.x; c < RCELLS; c += kTileThreads) {
        const unsigned long long v = reg[c];
        if (v == 0ull) continue;
        const int lx = c / (RG * RG), ly = (c / RG) % RG, lz = c % RG;
        const int gx = (ox0 - LO + lx + N) & (N - 1);
        const int gy = (oy0 - LO + ly + N) & (N - 1);
        const int gz = (oz0 - LO + lz + N) & (N - 1);
        atomicAdd(acc + (size_t(gx) * N + gy) * N + gz, v);
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_asg_convert(const long long* __restrict__ acc, int64_t n,
                                                          const AsgScale* __restrict__ sc, T* __restrict__ eps) {
    const double inv = sc->inv_scale;
    const int64_t stride = int64_t(gridDim.x) * kThreads;
    for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += stride)
        eps[i] = T(double(acc[i]) * inv);
}

template <typename T, int N>
static hermes_status assign_n(hermes_ctx ctx, const float* pos, const float* weight, int64_t n_pts, double box_L,
                              void* eps, double* sum_w, void* work, hipStream_t stream) {
    using G = asg_cfg<N>;
    const int64_t cells = int64_t(N) * N * N;
    const AsgLayout l = asg_layout(N, n_pts);
    char* w = static_cast<char*>(work);
    long long* acc = reinterpret_cast<long long*>(w + l.acc);
    uint32_t* key = reinterpret_cast<uint32_t*>(w + l.key);
    uint32_t* skey = reinterpret_cast<uint32_t*>(w + l.skey);
    uint32_t* off = reinterpret_cast<uint32_t*>(w + l.off);
    uint32_t* list = reinterpret_cast<uint32_t*>(w + l.list);
    double* partial = reinterpret_cast<double*>(w + l.partial);
    AsgScale* sc = reinterpret_cast<AsgScale*>(w + l.scale);
    const double scale = double(N) / box_L;
    const int pblocks = asg_prep_blocks(n_pts);
    {
        LaunchScope ls(ctx, stream, "fill");
        launch_fill<long long>(acc, cells, 0ll, stream);
        launch_fill<double>(partial, 2 * int64_t(pblocks), 0.0, stream);
    }
    {
        LaunchScope ls(ctx, stream, "assign");
        if (n_pts > 0)
            hipLaunchKernelGGL((k_asg_prep<N>), dim3(pblocks), dim3(kThreads), 0, stream, pos, weight, n_pts, scale,
                               key, partial);
        const int head = ctx->basis == HERMES_BASIS_DB2 ? 2 : 0;
        hipLaunchKernelGGL(k_asg_scale, dim3(1), dim3(kThreads), 0, stream, partial, pblocks, head, sum_w, sc);
        if (n_pts > 0) {
            radix_sort_indices(key, n_pts, uint32_t(G::TILES - 1), list, w + l.sort, stream, skey);
            hipLaunchKernelGGL(k_sorted_offsets, dim3(pblocks), dim3(kThreads), 0, stream, skey, n_pts,
                               int64_t(G::TILES), off);
            if (ctx->basis == HERMES_BASIS_DB2)
                hipLaunchKernelGGL((k_asg_tiles<T, N, HERMES_BASIS_DB2>), dim3(G::TILES), dim3(kTileThreads), 0, stream,
                                   pos, weight, scale, off, list, sc, ctx->t.db2tab,
                                   reinterpret_cast<unsigned long long*>(acc));
            else
                hipLaunchKernelGGL((k_asg_tiles<T, N, HERMES_BASIS_B3>), dim3(G::TILES), dim3(kTileThreads), 0, stream,
                                   pos, weight, scale, off, list, sc, ctx->t.db2tab,
                                   reinterpret_cast<unsigned long long*>(acc));
        }
        const int64_t want = (cells + kThreads - 1) / kThreads;
        hipLaunchKernelGGL((k_asg_convert<T>), dim3(int(want < 8192 ? want : 8192)), dim3(kThreads), 0, stream, acc,
                           cells, sc, static_cast<T*>(eps));
    }
    return check_launch("hermes_assign");
}

hermes_status assign_impl(hermes_ctx ctx, const float* pos, const float* weight, int64_t n_pts, double box_L,
                          int n, int dtype, void* eps, double* sum_w, void* work, hipStream_t stream) {
#define HERMES_ASSIGN_CASE(NN)                                                                                  \
    case NN:                                                                                                    \
        return dtype == HERMES_F32                                                                              \
                   ? assign_n<float, NN>(ctx, pos, weight, n_pts, box_L, eps, sum_w, work, stream)             \
                   : assign_n<double, NN>(ctx, pos, weight, n_pts, box_L, eps, sum_w, work, stream);
    switch (n) {
        HERMES_ASSIGN_CASE(8)
        HERMES_ASSIGN_CASE(16)
        HERMES_ASSIGN_CASE(32)
        HERMES_ASSIGN_CASE(64)
        HERMES_ASSIGN_CASE(128)
        HERMES_ASSIGN_CASE(256)
        HERMES_ASSIGN_CASE(512)
        HERMES_ASSIGN_CASE(1024)
        default:
            return fail(HERMES_ERR_ARG, "hermes_assign: unsupported N");
    }
#undef HERMES_ASSIGN_CASE
}

}  // namespace hermes
