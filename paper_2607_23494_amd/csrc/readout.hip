// Readout of a coefficient field at arbitrary positions (Sec. 3.1: the
// filtered field n_W(x) = sum_l eps~_l phi_l(x) read at any point) and the
// density-derived marks of Sec. 3.3.1 (Eqs. power-law-mark,
// inverse-density-mark).
//
// The value at a point is the node sum v = sum_l f_l prod_a phi(x_a/h - l_a)
// (64 nodes with B3, 27 with the D4 function), the transpose of the
// assignment's scatter: one thread per point gathers its rows of nodes.
// Large calls first bucket the points by tiles of 8^3 cells (16^3 at 1024^3)
// with a stable radix sort of their tile keys (a tile's points stay in index
// order; the positions are copied in list order beside the point indices).  Where
// the tiles hold enough points, a workgroup stages the nodes around a tile
// (up to four fields at once) in LDS and reads the tile's points from there;
// sparser calls read the bucketed points by per-lane gathers.  Either way the
// arithmetic is that of the unbucketed read, bit for bit, and each value is
// written at its point's index.
// Optionally the value becomes a mark and is multiplied by a weight (the
// marked catalogue for hermes_assign), and the moments <v^p>, p = 2..4, over
// the points are accumulated in float64 (counts in cells by sampling
// positions).
#include <algorithm>
#include <cmath>

#include "bucket.hpp"
#include "common.hpp"
#include "interp.hpp"
#include "kernels.hpp"
#include "sort.hpp"

namespace hermes {

struct MarkParams {
    int kind;
    double exponent, offset, self_term;
};

__device__ __forceinline__ double apply_mark(const MarkParams& mk, double v) {
    const double rho = fmax(1.0 + v - mk.self_term, 0.0);
    if (mk.kind == HERMES_MARK_POWER_LAW) return pow(rho + mk.offset, mk.exponent);
    if (mk.kind == HERMES_MARK_INVERSE_DENSITY) return pow((mk.offset + 1.0) / (mk.offset + rho), mk.exponent);
    return v;
}

// Points below this count are read in the given order (no workspace).
constexpr int64_t kReadoutBucketMin = int64_t(1) << 16;

// Bucket edge: 8 cells while the tile count stays within the offset scan's
// reach (kScanBlock^2 tiles), else 16.
constexpr int rd_edge(int n) { return (n / 8) * (n / 8) * (n / 8) <= kScanBlock * kScanBlock ? 8 : 16; }

static bool readout_buckets(int64_t n_pts) { return n_pts >= kReadoutBucketMin && n_pts <= INT32_MAX; }

// The tile-staged read: at least kRdTileDensity points per tile on average,
// at most kRdTileFields fields per pass, kRdTileBlocks workgroups at most.
constexpr int kRdTileDensity = 8;
constexpr int kRdTileFields = 4;
constexpr int kRdTileBlocks = 2048;
constexpr size_t kRdLdsBudget = 65536;   // bytes of staged nodes per workgroup

// Workspace layout (bytes, each part 256-aligned): the points' tile keys,
// the keys in sorted order, the tile offsets, the point list (indices in
// tile order), the positions in list order, the per-workgroup moment sums,
// and the sort's buffers.
struct RdLayout {
    size_t key, skey, off, list, spos, part, sort, total;
};

static RdLayout rd_layout(int n, int64_t n_pts) {
    const int ts = n < rd_edge(n) ? n : rd_edge(n);
    const int64_t tiles = int64_t(n / ts) * (n / ts) * (n / ts);
    RdLayout l{};
    size_t at = 0;
    l.key = at;
    at += align256(size_t(n_pts) * 4);
    l.skey = at;
    at += align256(size_t(n_pts) * 4);
    l.off = at;
    at += align256(size_t(tiles + 1) * 4);
    l.list = at;
    at += align256(size_t(n_pts) * 4);
    l.spos = at;
    at += align256(size_t(n_pts) * 12);
    l.part = at;
    at += align256(size_t(kRdTileBlocks) * kRdTileFields * 3 * sizeof(double));
    l.sort = at;
    at += sort_layout(n_pts).total;
    l.total = at;
    return l;
}

// Tile of every point (the cell of its wrapped position, divided by E).
template <int N, int E>
__global__ __launch_bounds__(kThreads) void k_readout_keys(const float* __restrict__ pos, int64_t n_pts,
                                                           double scale, uint32_t* __restrict__ key) {
    const int64_t stride = int64_t(gridDim.x) * kThreads;
    for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < n_pts; i += stride)
        key[i] = uint32_t(tile_of_point<N, E>(pos, i, scale));
}

// Positions in list order.
__global__ __launch_bounds__(kThreads) void k_readout_gather_pos(const float* __restrict__ pos, int64_t n_pts,
                                                                 const uint32_t* __restrict__ list,
                                                                 float* __restrict__ spos) {
    const int64_t stride = int64_t(gridDim.x) * kThreads;
    for (int64_t j = int64_t(blockIdx.x) * kThreads + threadIdx.x; j < n_pts; j += stride) {
        const int64_t i = list[j];
        spos[3 * j] = pos[3 * i];
        spos[3 * j + 1] = pos[3 * i + 1];
        spos[3 * j + 2] = pos[3 * i + 2];
    }
}

size_t readout_workspace(int n, int64_t n_pts) { return readout_buckets(n_pts) ? rd_layout(n, n_pts).total : 0; }

// Point j of the launch is point list[j] at position pos[j] (bucketed: pos
// holds the positions in list order) or point j.
template <typename T, int N, int B>
__global__ __launch_bounds__(kThreads) void k_readout(const T* __restrict__ field, const float* __restrict__ pos,
                                                      const float* __restrict__ weight, int64_t n_pts,
                                                      double scale, MarkParams mk, const double* __restrict__ tab,
                                                      const uint32_t* __restrict__ list, T* __restrict__ out,
                                                      double* __restrict__ mom) {
    __shared__ double red[kThreads];
    double m2 = 0.0, m3 = 0.0, m4 = 0.0;
    const int64_t stride = int64_t(gridDim.x) * kThreads;
    for (int64_t j = int64_t(blockIdx.x) * kThreads + threadIdx.x; j < n_pts; j += stride) {
        const int64_t i = list ? int64_t(list[j]) : j;
        const double u[3] = {double(pos[3 * j]) * scale, double(pos[3 * j + 1]) * scale,
                             double(pos[3 * j + 2]) * scale};   // position in cell units
        const double v = basis_value<T, N, B>(field, u, tab);
        if (mom) {
            const double v2 = v * v;
            m2 += v2;
            m3 += v2 * v;
            m4 += v2 * v2;
        }
        if (out) {
            double r = mk.kind == HERMES_MARK_NONE ? v : apply_mark(mk, v);
            if (weight) r *= double(weight[i]);
            out[i] = T(r);
        }
    }
    if (mom) {
        const double s2 = block_sum(m2, red);
        const double s3 = block_sum(m3, red);
        const double s4 = block_sum(m4, red);
        if (threadIdx.x == 0) {
            unsafeAtomicAdd(mom + 0, s2);
            unsafeAtomicAdd(mom + 1, s3);
            unsafeAtomicAdd(mom + 2, s4);
        }
    }
}

// Tile-staged read.  A tile of TS^3 cells is read from the RS^3 nodes
// around it (RS = TS + NT - 1): region index i along an axis holds node
// o - LO + i (mod N), so a point in cell c reads indices c - o .. c - o + NT - 1.
template <typename T, int N, int B> struct rd_tile_cfg {
    using G = tile_grid<N, rd_edge(N)>;
    static constexpr int TS = G::TS, NTA = G::NT;
    static constexpr int RS = TS + BasisTaps<B>::NT - 1;
    static constexpr int RV = RS * RS * RS;
    static constexpr int FC_LDS = int(kRdLdsBudget / (size_t(RV) * sizeof(T)));
    static constexpr int FC = FC_LDS < 1 ? 1 : (FC_LDS > kRdTileFields ? kRdTileFields : FC_LDS);
};

// The node sum of basis_value in the same order and precision, on the
// staged region.
template <typename T, int RS, int NT>
__device__ __forceinline__ double region_sum(const T* __restrict__ reg, const int rel[3], const double tap[3][NT]) {
    double val = 0.0;
#pragma unroll
    for (int ox = 0; ox < NT; ++ox) {
        double vx = 0.0;
#pragma unroll
        for (int oy = 0; oy < NT; ++oy) {
            const T* row = reg + ((rel[0] + ox) * RS + rel[1] + oy) * RS + rel[2];
            double vy = 0.0;
#pragma unroll
            for (int oz = 0; oz < NT; ++oz) vy += tap[2][oz] * double(row[oz]);
            vx += tap[1][oy] * vy;
        }
        val += tap[0][ox] * vx;
    }
    return val;
}

// Fields f0 .. f0 + nf - 1 (nf <= FC) at the bucketed points: workgroup g
// takes the contiguous run of tiles holding points g n / G .. (g + 1) n / G;
// per-workgroup moment sums go to part[g][f][3].
template <typename T, int N, int B>
__global__ __launch_bounds__(kThreads) void k_readout_tiles(const T* __restrict__ fields, int nf,
                                                            const float* __restrict__ spos,
                                                            const float* __restrict__ weight, double scale,
                                                            MarkParams mk, const double* __restrict__ tab,
                                                            const uint32_t* __restrict__ off,
                                                            const uint32_t* __restrict__ list, T* __restrict__ out,
                                                            int64_t n_pts, double* __restrict__ part) {
    using Cf = rd_tile_cfg<T, N, B>;
    using P = BasisTaps<B>;
    constexpr int NT = P::NT, LO = P::LO, RS = Cf::RS, RV = Cf::RV, FC = Cf::FC, TS = Cf::TS, NTA = Cf::NTA;
    constexpr int64_t TILES = int64_t(NTA) * NTA * NTA;
    __shared__ T reg[FC][RV];
    __shared__ double red[kThreads];
    const int64_t total = off[TILES];
    auto first_at = [&](int64_t t) {   // smallest tile in [0, TILES] with off >= t
        int64_t a = 0, b = TILES;
        while (a < b) {
            const int64_t mid = (a + b) / 2;
            if (int64_t(off[mid]) < t) a = mid + 1;
            else b = mid;
        }
        return a;
    };
    const int64_t t_begin = first_at(total * blockIdx.x / gridDim.x);
    const int64_t t_end = first_at(total * (int64_t(blockIdx.x) + 1) / gridDim.x);
    double mom[FC][3];
#pragma unroll
    for (int f = 0; f < FC; ++f) mom[f][0] = mom[f][1] = mom[f][2] = 0.0;
    for (int64_t t = t_begin; t < t_end; ++t) {
        const uint32_t lo = off[t], hi = off[t + 1];
        if (lo == hi) continue;   // uniform over the workgroup
        const int o[3] = {int(t / (int64_t(NTA) * NTA)) * TS, int((t / NTA) % NTA) * TS, int(t % NTA) * TS};
        __syncthreads();   // the previous tile's reads are done
        for (int e = threadIdx.x; e < nf * RV; e += kThreads) {
            const int f = e / RV, r = e - f * RV;
            const int i = r / (RS * RS), j = (r / RS) % RS, k = r % RS;
            const int gx = (o[0] - LO + i) & (N - 1), gy = (o[1] - LO + j) & (N - 1), gz = (o[2] - LO + k) & (N - 1);
            reg[f][r] = fields[int64_t(f) * N * N * N + (int64_t(gx) * N + gy) * N + gz];
        }
        __syncthreads();
        for (int64_t j = int64_t(lo) + threadIdx.x; j < int64_t(hi); j += kThreads) {
            const int64_t i = list[j];
            int rel[3];
            double tap[3][NT];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                double v = double(spos[3 * j + a]) * scale;   // as basis_value: wrap, floor, offset
                v -= double(N) * floor(v / double(N));
                const double fl = floor(v);
                int c = int(fl);
                P::weights(v - fl, tab, tap[a]);
                if (c >= N) c = 0;   // v rounded up to N: node 0 of the next image (as the bucketing)
                rel[a] = c - o[a];
            }
            const double w = weight ? double(weight[i]) : 1.0;
#pragma unroll
            for (int f = 0; f < FC; ++f) {
                if (f < nf) {
                    const double v = region_sum<T, RS, NT>(reg[f], rel, tap);
                    const double v2 = v * v;
                    mom[f][0] += v2;
                    mom[f][1] += v2 * v;
                    mom[f][2] += v2 * v2;
                    if (out) {
                        double r = mk.kind == HERMES_MARK_NONE ? v : apply_mark(mk, v);
                        if (weight) r *= w;
                        out[int64_t(f) * n_pts + i] = T(r);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int f = 0; f < FC; ++f) {
        if (f < nf) {
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const double s = block_sum(mom[f][m], red);
                if (threadIdx.x == 0) part[(int64_t(blockIdx.x) * FC + f) * 3 + m] = s;
            }
        }
    }
}

// moments[f][m] = (sum over the workgroups' partials) / n: one workgroup per
// output, thread t summing partials t, t + kThreads, ..., then the block's
// tree sum (a fixed order).
__global__ __launch_bounds__(kThreads) void k_readout_moments(const double* __restrict__ part, int blocks, int fc,
                                                              double inv_n, double* __restrict__ moments) {
    __shared__ double red[kThreads];
    const int f = blockIdx.x / 3, m = blockIdx.x % 3;
    double s = 0.0;
    for (int b = threadIdx.x; b < blocks; b += kThreads) s += part[(int64_t(b) * fc + f) * 3 + m];
    s = block_sum(s, red);
    if (threadIdx.x == 0) moments[blockIdx.x] = s * inv_n;
}

__global__ void k_scale3(double* __restrict__ mom, double s) {
    if (threadIdx.x < 3) mom[threadIdx.x] *= s;
}

// Every field of the call is read at the same points, after one bucketing.
template <typename T, int N>
static hermes_status readout_n(hermes_ctx ctx, const void* fields, int n_fields, double box_L, const float* pos,
                               const float* weight, int64_t n_pts, const MarkParams& mk, void* out,
                               double* moments, void* work, hipStream_t stream) {
    if (moments) {
        LaunchScope ls(ctx, stream, "fill");
        launch_fill<double>(moments, 3 * int64_t(n_fields), 0.0, stream);
    }
    if (n_pts > 0) {
        const double scale = double(N) / box_L;
        const int64_t want = (n_pts + kThreads - 1) / kThreads;
        const int blocks = int(want < 8192 ? want : 8192);
        const uint32_t* list = nullptr;
        const float* rpos = pos;
        if (work && readout_buckets(n_pts)) {
            constexpr int E = rd_edge(N);
            using G = tile_grid<N, E>;
            const RdLayout l = rd_layout(N, n_pts);
            char* w = static_cast<char*>(work);
            uint32_t* key = reinterpret_cast<uint32_t*>(w + l.key);
            uint32_t* skey = reinterpret_cast<uint32_t*>(w + l.skey);
            uint32_t* off = reinterpret_cast<uint32_t*>(w + l.off);
            uint32_t* lst = reinterpret_cast<uint32_t*>(w + l.list);
            float* spos = reinterpret_cast<float*>(w + l.spos);
            LaunchScope ls(ctx, stream, "bucket");
            hipLaunchKernelGGL((k_readout_keys<N, E>), dim3(blocks), dim3(kThreads), 0, stream, pos, n_pts, scale, key);
            radix_sort_indices(key, n_pts, uint32_t(G::TILES - 1), lst, w + l.sort, stream, skey);
            hipLaunchKernelGGL(k_sorted_offsets, dim3(blocks), dim3(kThreads), 0, stream, skey, n_pts,
                               int64_t(G::TILES), off);
            hipLaunchKernelGGL(k_readout_gather_pos, dim3(blocks), dim3(kThreads), 0, stream, pos, n_pts, lst, spos);
            list = lst;
            rpos = spos;
        }
        if (list && n_pts >= int64_t(kRdTileDensity) * tile_grid<N, rd_edge(N)>::TILES) {
            const RdLayout l = rd_layout(N, n_pts);
            char* w = static_cast<char*>(work);
            const uint32_t* off = reinterpret_cast<const uint32_t*>(w + l.off);
            double* part = reinterpret_cast<double*>(w + l.part);
            const bool db2 = ctx->basis == HERMES_BASIS_DB2;
            const int fc = db2 ? rd_tile_cfg<T, N, HERMES_BASIS_DB2>::FC : rd_tile_cfg<T, N, HERMES_BASIS_B3>::FC;
            const int grid = int(std::min<int64_t>({int64_t(tile_grid<N, rd_edge(N)>::TILES), int64_t(4) * ctx->cus,
                                                    int64_t(kRdTileBlocks)}));
            for (int f0 = 0; f0 < n_fields; f0 += fc) {
                const int nf = std::min(fc, n_fields - f0);
                const T* fld = static_cast<const T*>(fields) + int64_t(f0) * N * N * N;
                T* o = out ? static_cast<T*>(out) + int64_t(f0) * n_pts : nullptr;
                {
                    LaunchScope ls(ctx, stream, "readout");
                    if (db2)
                        hipLaunchKernelGGL((k_readout_tiles<T, N, HERMES_BASIS_DB2>), dim3(grid), dim3(kThreads), 0,
                                           stream, fld, nf, rpos, weight, scale, mk, ctx->t.db2tab, off, list, o,
                                           n_pts, part);
                    else
                        hipLaunchKernelGGL((k_readout_tiles<T, N, HERMES_BASIS_B3>), dim3(grid), dim3(kThreads), 0,
                                           stream, fld, nf, rpos, weight, scale, mk, ctx->t.db2tab, off, list, o,
                                           n_pts, part);
                }
                if (moments) {
                    LaunchScope ls(ctx, stream, "reduce");
                    hipLaunchKernelGGL(k_readout_moments, dim3(3 * nf), dim3(kThreads), 0, stream, part, grid, fc,
                                       1.0 / double(n_pts), moments + 3 * f0);
                }
            }
            return check_launch("hermes_readout");
        }
        for (int f = 0; f < n_fields; ++f) {
            LaunchScope ls(ctx, stream, "readout");
            const T* fld = static_cast<const T*>(fields) + int64_t(f) * N * N * N;
            T* o = out ? static_cast<T*>(out) + int64_t(f) * n_pts : nullptr;
            double* m = moments ? moments + 3 * f : nullptr;
            if (ctx->basis == HERMES_BASIS_DB2)
                hipLaunchKernelGGL((k_readout<T, N, HERMES_BASIS_DB2>), dim3(blocks), dim3(kThreads), 0, stream, fld,
                                   rpos, weight, n_pts, scale, mk, ctx->t.db2tab, list, o, m);
            else
                hipLaunchKernelGGL((k_readout<T, N, HERMES_BASIS_B3>), dim3(blocks), dim3(kThreads), 0, stream, fld,
                                   rpos, weight, n_pts, scale, mk, ctx->t.db2tab, list, o, m);
            if (m) hipLaunchKernelGGL(k_scale3, dim3(1), dim3(64), 0, stream, m, 1.0 / double(n_pts));
        }
    }
    return check_launch("hermes_readout");
}

hermes_status readout_impl(hermes_ctx ctx, const void* fields, int n_fields, int n, int dtype, double box_L,
                           const float* pos, const float* weight, int64_t n_pts, const hermes_mark* mark, void* out,
                           double* moments, void* work, hipStream_t stream) {
    MarkParams mk{HERMES_MARK_NONE, 0.0, 0.0, 0.0};
    if (mark) {
        mk.kind = mark->kind;
        mk.exponent = mark->exponent;
        mk.offset = mark->offset;
        mk.self_term = mark->self_term;
    }
#define HERMES_READOUT_CASE(NN)                                                                                \
    case NN:                                                                                                   \
        return dtype == HERMES_F32                                                                             \
                   ? readout_n<float, NN>(ctx, fields, n_fields, box_L, pos, weight, n_pts, mk, out, moments,   \
                                          work, stream)                                                          \
                   : readout_n<double, NN>(ctx, fields, n_fields, box_L, pos, weight, n_pts, mk, out, moments,  \
                                           work, stream);
    switch (n) {
        HERMES_READOUT_CASE(8)
        HERMES_READOUT_CASE(16)
        HERMES_READOUT_CASE(32)
        HERMES_READOUT_CASE(64)
        HERMES_READOUT_CASE(128)
        HERMES_READOUT_CASE(256)
        HERMES_READOUT_CASE(512)
        HERMES_READOUT_CASE(1024)
        default:
            return fail(HERMES_ERR_ARG, "hermes_readout: unsupported N");
    }
#undef HERMES_READOUT_CASE
}

}  // namespace hermes
