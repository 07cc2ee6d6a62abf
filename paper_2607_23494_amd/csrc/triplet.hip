// Monte-Carlo triangle sums (Sec. 3.4, particle-based summation, Eq.
// particle-based-sum; Sec. 4.3.3, the dual-/triplet-sphere 3PCF).
//
// A sample is a primary vertex x (a catalogue point, or a uniform point of
// the box drawn from the generator) and a random rotation (u, v): u uniform
// on the sphere, v uniform on the circle orthogonal to u.  For every opening
// angle theta_j = (j + 1/2) pi / n_theta the triangle has its second vertex at
// x + r12 u and its third at x + r13 (cos theta_j u + sin theta_j v); the
// secondary vertices read the filtered fields f2, f3 through the basis
// expansion.
// The sums over samples of a, a f2, a f3 and a f2 f3 (a = the point's weight,
// or f1 at a box point) are accumulated in float64.
//
// Random numbers are Philox4x64-10 blocks (Salmon, Moraes, Dror and Shaw,
// SC'11) with counter (centre, rotation, 0, 0) for a rotation and
// (centre, 0, 1, 0) for a box point, key (seed, 0): every sample can be drawn
// by any thread, and the oracle draws the same numbers.
//
// Two paths draw the same samples.  The block-local path (float32 fields,
// f2 and f3 one array, the reach within a staged region; see below) buckets
// the centres and reads the fields from the nodes around each bucket staged
// in LDS.  The direct path reads them through tile-packed copies (each tile
// holds, for a pair of x planes, the 4 x 4 (y, z) block of nodes a point in
// its cell reaches, so a read is two or three 128-byte loads) up to 512^3 in
// float32 and 256^3 in float64, larger grids directly, one thread per sample
// (grid-stride).  Either way, per opening angle the wavefront's 64 samples
// are summed in a fixed order (DPP steps) and added to the wavefront's LDS
// accumulators, so every sum is formed in a fixed order and the result does
// not depend on timing.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "bucket.hpp"
#include "common.hpp"
#include "interp.hpp"
#include "kernels.hpp"
#include "sort.hpp"

namespace hermes {

constexpr int kTripletBlocks = 2048;   // workgroups of the sampling kernel (grid-stride)
constexpr int kTripletWaves = kThreads / 64;

constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull, kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull, kPhiloxW1 = 0xBB67AE8584CAA73Bull;

// Ten Philox4x64 rounds on the counter c with key (k0, k1).
__device__ __forceinline__ void philox4x64(uint64_t c[4], uint64_t k0, uint64_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t lo0 = kPhiloxM0 * c[0], hi0 = __umul64hi(kPhiloxM0, c[0]);
        const uint64_t lo1 = kPhiloxM1 * c[2], hi1 = __umul64hi(kPhiloxM1, c[2]);
        const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
}

// The top 53 bits of a word plus one half, scaled to (0, 1).
__device__ __forceinline__ double uniform53(uint64_t w) { return (double(w >> 11) + 0.5) * 0x1p-53; }

// One DPP step on a double: the value of the lane CTRL selects, in the rows
// ROWS enables (0 in the others).
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp_f64(double v) {
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
    const int lo = __builtin_amdgcn_update_dpp(0, int(unsigned(b)), CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, int(unsigned(b >> 32)), CTRL, ROWS, 0xF, false);
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(unsigned(hi)) << 32) |
                                                       unsigned(lo)));
}

// Sum over the wavefront's 64 lanes (all active), the same in every lane, in
// a fixed order: within rows of 16 by quad permutes and mirrors (every lane
// of a row then holds the row's sum), then the row broadcasts 15 and 31
// carry rows 0 and 2 into rows 1 and 3 and rows 0 + 1 into row 3, whose lane
// 63 holds the total.  DPP moves stay in the vector unit: no LDS round trip
// per step.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_f64<0xB1>(v);          // quad_perm(1, 0, 3, 2)
    v += dpp_f64<0x4E>(v);          // quad_perm(2, 3, 0, 1)
    v += dpp_f64<0x141>(v);         // row_half_mirror
    v += dpp_f64<0x140>(v);         // row_mirror
    v += dpp_f64<0x142, 0xA>(v);    // row_bcast:15 into rows 1, 3
    v += dpp_f64<0x143, 0xC>(v);    // row_bcast:31 into rows 2, 3
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
    const unsigned lo = unsigned(__builtin_amdgcn_readlane(int(unsigned(b)), 63));
    const unsigned hi = unsigned(__builtin_amdgcn_readlane(int(unsigned(b >> 32)), 63));
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// Primary vertex c: a uniform point of the box from the generator, or
// catalogue point c, mapped into [0, L) when WRAP (the block-local path
// buckets centres by it).
template <bool BOX, bool WRAP>
__device__ __forceinline__ void centre_of(int64_t c, const float* __restrict__ centres, double box_L, uint64_t seed,
                                          double x[3]) {
    if constexpr (BOX) {
        uint64_t w[4] = {uint64_t(c), 0, 1, 0};
        philox4x64(w, seed, 0);
        x[0] = box_L * uniform53(w[0]);
        x[1] = box_L * uniform53(w[1]);
        x[2] = box_L * uniform53(w[2]);
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            x[a] = double(centres[3 * c + a]);
            if constexpr (WRAP) x[a] -= box_L * floor(x[a] / box_L);
        }
    }
}

// Rotation r of centre c: u uniform on the sphere, v uniform on the circle
// orthogonal to u.
__device__ __forceinline__ void rotation_of(int64_t c, int64_t r, uint64_t seed, double u[3], double v[3]) {
    uint64_t w[4] = {uint64_t(c), uint64_t(r), 0, 0};
    philox4x64(w, seed, 0);
    const double cz = 2.0 * uniform53(w[0]) - 1.0;
    const double phi = 2.0 * M_PI * uniform53(w[1]);
    const double psi = 2.0 * M_PI * uniform53(w[2]);
    const double sz = sqrt(fmax(0.0, 1.0 - cz * cz));
    u[0] = sz * cos(phi);
    u[1] = sz * sin(phi);
    u[2] = cz;
    // orthonormal basis of the plane orthogonal to u (Duff et al., JCGT
    // 2017), then v at angle psi in it
    const double sg = u[2] >= 0.0 ? 1.0 : -1.0;
    const double ia = -1.0 / (sg + u[2]);
    const double b = u[0] * u[1] * ia;
    const double e1[3] = {1.0 + sg * u[0] * u[0] * ia, sg * b, -sg * u[0]};
    const double e2[3] = {b, sg + u[1] * u[1] * ia, -u[1]};
    const double cp = cos(psi), sp = sin(psi);
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = cp * e1[k] + sp * e2[k];
}

// Tile-packed copies: sixteen times the field (8.6 GB per float32 field at
// 512^3); larger grids read the plain array.
template <typename T> constexpr int tile_max_n() { return sizeof(T) == 4 ? 512 : 256; }

// The 2 x 4 x 4 block of a pair of x planes: Tile<T> at (x2, y, z) holds the
// field at (2 x2 + i, y - LO + a, z - LO + b), i < 2, a, b < 4 (indices mod
// N), in that order: one 128-byte line in float32.  A point's nodes along x
// fall in two or three consecutive pairs.
template <typename T> struct alignas(32 * sizeof(T)) Tile {
    T v[32];
};

// Partial sums and tile-packed copies (the direct path).
static size_t triplet_workspace_direct(int n, int dtype, int n_theta) {
    const size_t part = align256(size_t(kTripletBlocks) * n_theta * 4 * sizeof(double));
    const bool f32 = dtype == HERMES_F32;
    if (n > (f32 ? tile_max_n<float>() : tile_max_n<double>())) return part;
    const size_t elem = f32 ? sizeof(Tile<float>) : sizeof(Tile<double>);
    return part + 3 * align256(size_t(n / 2) * n * n * elem);
}

template <typename T, int N, int LO>
__global__ __launch_bounds__(kThreads) void k_pack_tiles(const T* __restrict__ f, Tile<T>* __restrict__ out) {
    const int64_t total = int64_t(N / 2) * N * N;
    const int64_t stride = int64_t(gridDim.x) * kThreads;
    for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < total; i += stride) {
        const int x2 = int(i / (int64_t(N) * N));
        const int y = int((i / N) & (N - 1)), z = int(i & (N - 1));
        Tile<T> t;
#pragma unroll
        for (int xi = 0; xi < 2; ++xi)
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    t.v[(xi * 4 + a) * 4 + b] =
                        f[(int64_t(2 * x2 + xi) * N + ((y - LO + a) & (N - 1))) * N + ((z - LO + b) & (N - 1))];
        out[i] = t;
    }
}

// basis_value on a tile-packed field: the (y, z) taps of each plane of the
// two or three pairs that hold the point's x nodes, then the x taps.
template <typename T, int N, int B>
__device__ __forceinline__ double basis_value_tiles(const Tile<T>* __restrict__ p, const double u[3],
                                                    const double* __restrict__ tab) {
    using P = BasisTaps<B>;
    constexpr int NT = P::NT, LO = P::LO;
    constexpr int NP = NT / 2 + 1;   // pairs that can hold the x nodes
    int cell[3];
    double tap[3][NT];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double v = u[a];
        v -= double(N) * floor(v / double(N));   // periodic wrap into [0, N)
        const double f = floor(v);
        cell[a] = int(f);
        P::weights(v - f, tab, tap[a]);
    }
    const int x0 = (cell[0] - LO) & (N - 1), odd = x0 & 1, last = (odd + NT - 1) >> 1;
    const size_t yz = size_t(cell[1] & (N - 1)) * N + (cell[2] & (N - 1));
    double s[2 * NP];   // s[2 k + i]: plane i of pair k, (y, z) taps applied
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        s[2 * k] = 0.0;
        s[2 * k + 1] = 0.0;
        if (k <= last) {
            const int x2 = ((x0 >> 1) + k) & (N / 2 - 1);
            const Tile<T> t = p[size_t(x2) * N * N + yz];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                double vx = 0.0;
#pragma unroll
                for (int oy = 0; oy < NT; ++oy) {
                    double vy = 0.0;
#pragma unroll
                    for (int oz = 0; oz < NT; ++oz) vy += tap[2][oz] * double(t.v[(i * 4 + oy) * 4 + oz]);
                    vx += tap[1][oy] * vy;
                }
                s[2 * k + i] = vx;
            }
        }
    }
    // node ox is plane ox + odd of the loaded run: a bit select keeps the
    // indices of s static (no private-memory copy of s)
    const unsigned long long pick = 0ull - static_cast<unsigned long long>(odd);
    double val = 0.0;
#pragma unroll
    for (int ox = 0; ox < NT; ++ox) {
        const unsigned long long a = __double_as_longlong(s[ox]), b = __double_as_longlong(s[ox + 1]);
        val += tap[0][ox] * __longlong_as_double(static_cast<long long>((a & ~pick) | (b & pick)));
    }
    return val;
}

// A field read by the sampling kernel: tiles or the plain array.
template <typename T, int N, int B>
struct FieldRef {
    const T* f;
    const Tile<T>* t;
    const double* tab;   // the D4 table (unused by B3)
    __device__ __forceinline__ double at(const double u[3]) const {
        if constexpr (N <= tile_max_n<T>()) return basis_value_tiles<T, N, B>(t, u, tab);
        else return basis_value<T, N, B>(f, u, tab);
    }
};

template <typename T, int N, bool BOX, int B>
__global__ __launch_bounds__(kThreads) void k_triplet(FieldRef<T, N, B> f1, FieldRef<T, N, B> f2, FieldRef<T, N, B> f3,
                                                      bool has_f1, const float* __restrict__ centres,
                                                      const float* __restrict__ weights, int64_t n_centres, int n_rot,
                                                      double box_L, double r12, double r13, int n_theta,
                                                      uint64_t seed, double* __restrict__ part) {
    __shared__ double acc[kTripletWaves][HERMES_MAX_THETA][2];   // per wavefront: sum a f3, sum a f2 f3
    __shared__ double red[kThreads];
    __shared__ double cs[HERMES_MAX_THETA][2];                    // cos, sin of the opening angles
    const int wv = threadIdx.x / 64, lane = threadIdx.x % 64;
    for (int j = threadIdx.x; j < kTripletWaves * HERMES_MAX_THETA; j += kThreads) {
        acc[j / HERMES_MAX_THETA][j % HERMES_MAX_THETA][0] = 0.0;
        acc[j / HERMES_MAX_THETA][j % HERMES_MAX_THETA][1] = 0.0;
    }
    for (int j = threadIdx.x; j < n_theta; j += kThreads) {
        const double th = (double(j) + 0.5) * M_PI / double(n_theta);
        cs[j][0] = cos(th);
        cs[j][1] = sin(th);
    }
    __syncthreads();
    const double scale = double(N) / box_L;
    const int64_t total = n_centres * int64_t(n_rot);
    const int64_t stride = int64_t(gridDim.x) * kThreads;
    double s0 = 0.0, s1 = 0.0;
    // the loop bound is uniform over a wavefront, so all of its lanes take part
    // in every butterfly
    for (int64_t base = int64_t(blockIdx.x) * kThreads + wv * 64; base < total; base += stride) {
        const int64_t s = base + lane;
        const bool live = s < total;
        double a = 0.0, v2 = 0.0, x[3] = {0.0, 0.0, 0.0}, u[3] = {0.0, 0.0, 1.0}, v[3] = {1.0, 0.0, 0.0};
        if (live) {
            const int64_t c = s / n_rot, r = s - (s / n_rot) * n_rot;
            centre_of<BOX, false>(c, centres, box_L, seed, x);
            if constexpr (BOX) {
                if (has_f1) {
                    const double uc[3] = {x[0] * scale, x[1] * scale, x[2] * scale};
                    a = f1.at(uc);
                } else {
                    a = 1.0;
                }
            } else {
                a = weights ? double(weights[c]) : 1.0;
            }
            rotation_of(c, r, seed, u, v);
            const double p2[3] = {(x[0] + r12 * u[0]) * scale, (x[1] + r12 * u[1]) * scale,
                                  (x[2] + r12 * u[2]) * scale};
            v2 = f2.at(p2);
        }
        s0 += a;
        s1 += a * v2;
        for (int j = 0; j < n_theta; ++j) {
            double p3 = 0.0, p23 = 0.0;
            if (live) {
                const double ct = cs[j][0], st = cs[j][1];
                const double q[3] = {(x[0] + r13 * (ct * u[0] + st * v[0])) * scale,
                                     (x[1] + r13 * (ct * u[1] + st * v[1])) * scale,
                                     (x[2] + r13 * (ct * u[2] + st * v[2])) * scale};
                const double v3 = f3.at(q);
                p3 = a * v3;
                p23 = a * v2 * v3;
            }
            p3 = wave_sum(p3);
            p23 = wave_sum(p23);
            if (lane == 0) {
                acc[wv][j][0] += p3;
                acc[wv][j][1] += p23;
            }
        }
    }
    const double b0 = block_sum(s0, red);
    const double b1 = block_sum(s1, red);   // block_sum ends with a barrier: acc is complete
    for (int j = threadIdx.x; j < n_theta; j += kThreads) {
        double t3 = 0.0, t23 = 0.0;
        for (int k = 0; k < kTripletWaves; ++k) {
            t3 += acc[k][j][0];
            t23 += acc[k][j][1];
        }
        double* dst = part + (int64_t(blockIdx.x) * n_theta + j) * 4;
        dst[0] = b0;
        dst[1] = b1;
        dst[2] = t3;
        dst[3] = t23;
    }
}

__global__ void k_triplet_final(const double* __restrict__ part, int n_blocks, int n_theta, double* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_theta * 4) return;
    double s = 0.0;
    for (int b = 0; b < n_blocks; ++b) s += part[int64_t(b) * n_theta * 4 + i];
    out[i] = s;
}

// ---------------------------------------------------------------- block-local path
// For float32 fields with f2 and f3 the same array, the centres are
// bucketed by blocks of E^3 cells and a workgroup stages the nodes around
// its block (a kTriReg^3 region, 133 KB of LDS) once, then draws every
// sample of the block's centres from it: the 1 + n_theta reads of a sample
// become LDS reads instead of gathers of 128-byte lines from L2.  Usable when
// the triangles' reach fits the region: E + 2 M + NT - 1 <= kTriReg with the
// margin M = floor(max(r12, r13) N / L) + 2 cells.  Workgroup g takes the
// contiguous run of buckets that holds centres g n_c / G .. (g + 1) n_c / G
// (about equal sample counts), so the sums keep a fixed order.  Node
// (i, j, k) of the region sits at i kTriPS + j kTriRS + k: with rows of 32
// floats the bank of a read would be its z node alone, and a wavefront's 64
// samples around one centre span only about 2 M + 4 z nodes, so several
// lanes would share each bank; the padded strides spread them as random
// addresses would (about five lanes on the busiest of 32 banks instead of
// seven to nine, by a model of the sample geometry).
constexpr int kTriReg = 32;             // region edge (nodes)
constexpr int kTriRS = kTriReg + 1;     // row stride (floats)
constexpr int kTriPS = kTriReg * kTriRS + 8;   // plane stride (floats)
constexpr int kTriThreads = 1024;       // one workgroup per CU (the region's LDS)
constexpr int kTriWaves = kTriThreads / 64;

// Bucket edge in cells: 4, or 8 or 16 where the bucket count would exceed
// the offset scan's reach (kScanBlock^2).
__host__ __device__ constexpr int tri_blk(int n) {
    return int64_t(n / 4) * (n / 4) * (n / 4) <= int64_t(kScanBlock) * kScanBlock   ? 4
           : int64_t(n / 8) * (n / 8) * (n / 8) <= int64_t(kScanBlock) * kScanBlock ? 8
                                                                                    : 16;
}
inline int64_t tri_buckets(int n) {
    const int nb = n / tri_blk(n);
    return int64_t(nb) * nb * nb;
}

// Bucket arrays of the block-local path (bytes, each part 256-aligned):
// bucket keys, the centre list in bucket order (centres of one bucket in
// index order), per-bucket counts, their offsets and the scan's block sums,
// then the sort's buffers.
struct TriLayout {
    size_t key, list, count, off, blocksum, sort, total;
};

static TriLayout tri_layout(int n, int64_t n_c) {
    const int64_t k = tri_buckets(n);
    const int64_t nblk = (k + kScanBlock - 1) / kScanBlock;
    TriLayout l{};
    size_t at = 0;
    l.key = at;
    at += align256(size_t(n_c) * 4);
    l.list = at;
    at += align256(size_t(n_c) * 4);
    l.count = at;
    at += align256(size_t(k) * 4);
    l.off = at;
    at += align256(size_t(k + 1) * 4);
    l.blocksum = at;
    at += align256(size_t(nblk) * 4);
    l.sort = at;
    at += sort_layout(n_c).total;
    l.total = at;
    return l;
}

// The direct path's workspace, then (float32, 1 <= n_c < 2^31) the bucket
// arrays of the block-local path; a workspace sized without them runs the
// direct path.
size_t triplet_workspace(int n, int dtype, int n_theta, int64_t n_c) {
    const size_t direct = triplet_workspace_direct(n, dtype, n_theta);
    if (dtype != HERMES_F32 || n_c < 1 || n_c > INT32_MAX) return direct;
    return direct + tri_layout(n, n_c).total;
}

// Bucket of every centre (its cell, clamped to the grid, divided by E).
template <int N, bool BOX>
__global__ __launch_bounds__(kThreads) void k_tri_keys(const float* __restrict__ centres, int64_t n_c, double box_L,
                                                       uint64_t seed, uint32_t* __restrict__ key,
                                                       uint32_t* __restrict__ count) {
    constexpr int E = tri_blk(N), NB = N / E;
    const double scale = double(N) / box_L;
    const int64_t stride = int64_t(gridDim.x) * kThreads;
    for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < n_c; i += stride) {
        double x[3];
        centre_of<BOX, true>(i, centres, box_L, seed, x);
        int b[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            int cell = int(floor(x[a] * scale));
            cell = cell < 0 ? 0 : (cell > N - 1 ? N - 1 : cell);
            b[a] = cell / E;
        }
        const uint32_t k = uint32_t((b[0] * NB + b[1]) * NB + b[2]);
        key[i] = k;
        atomicAdd(count + k, 1u);
    }
}

// The basis expansion at u (cell units) from the staged region: region index
// t along an axis holds node o - M - LO + t, so the nodes of a point in cell c
// start at index c - o + M.
template <int B>
__device__ __forceinline__ double region_value(const float* __restrict__ reg, const double u[3], const int o[3],
                                               int marg, const double* __restrict__ tab) {
    using P = BasisTaps<B>;
    constexpr int NT = P::NT;
    int rel[3];
    double tap[3][NT];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double f = floor(u[a]);
        rel[a] = int(f) - o[a] + marg;
        P::weights(u[a] - f, tab, tap[a]);
    }
    const float* p = reg + rel[0] * kTriPS + rel[1] * kTriRS + rel[2];
    double val = 0.0;
#pragma unroll
    for (int ox = 0; ox < NT; ++ox) {
        double vx = 0.0;
#pragma unroll
        for (int oy = 0; oy < NT; ++oy) {
            double vy = 0.0;
#pragma unroll
            for (int oz = 0; oz < NT; ++oz) vy += tap[2][oz] * double(p[ox * kTriPS + oy * kTriRS + oz]);
            vx += tap[1][oy] * vy;
        }
        val += tap[0][ox] * vx;
    }
    return val;
}

__device__ __forceinline__ double block_sum_tri(double v, double* scratch) {
    scratch[threadIdx.x] = v;
    __syncthreads();
    for (int s = kTriThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) scratch[threadIdx.x] += scratch[threadIdx.x + s];
        __syncthreads();
    }
    const double r = scratch[0];
    __syncthreads();
    return r;
}

// 161,792 bytes at n_theta = HERMES_MAX_THETA, within the 160 KiB of a CU.
inline size_t tri_lds_bytes(int n_theta) {
    return size_t(kTriReg) * kTriPS * sizeof(float) + size_t(kTriWaves) * n_theta * 2 * sizeof(double) +
           size_t(n_theta) * 2 * sizeof(double) + size_t(kTriThreads) * sizeof(double);
}

// F1R: f1 is the staged field too (read at the centre, inside the block).
template <int N, bool BOX, int B, bool F1R>
__global__ __launch_bounds__(kTriThreads) void k_triplet_blocks(
    const float* __restrict__ f1, const float* __restrict__ f23, const double* __restrict__ tab, bool has_f1,
    const float* __restrict__ centres, const float* __restrict__ weights, int n_rot, double box_L, double r12,
    double r13, int n_theta, uint64_t seed, int marg, const uint32_t* __restrict__ off,
    const uint32_t* __restrict__ list, double* __restrict__ part) {
    constexpr int E = tri_blk(N), NB = N / E, LO = BasisTaps<B>::LO;
    constexpr int64_t K = int64_t(NB) * NB * NB;
    constexpr int RV = kTriReg * kTriReg * kTriReg;   // region nodes
    static_assert(kTriReg * kTriPS % 2 == 0, "the float64 arrays follow the region");
    extern __shared__ double lds_raw[];
    float* reg = reinterpret_cast<float*>(lds_raw);
    double* acc = lds_raw + kTriReg * kTriPS / 2;   // [wave][j][2]: sum a f3, sum a f2 f3
    double* cs = acc + kTriWaves * n_theta * 2;     // [j][2]: cos, sin of the opening angles
    double* red = cs + n_theta * 2;                 // [kTriThreads]
    const int wv = threadIdx.x / 64, lane = threadIdx.x % 64;
    for (int j = threadIdx.x; j < kTriWaves * n_theta * 2; j += kTriThreads) acc[j] = 0.0;
    for (int j = threadIdx.x; j < n_theta; j += kTriThreads) {
        const double th = (double(j) + 0.5) * M_PI / double(n_theta);
        cs[2 * j] = cos(th);
        cs[2 * j + 1] = sin(th);
    }
    const double scale = double(N) / box_L;
    // this workgroup's buckets: those whose first centre falls in
    // [g n_c / G, (g + 1) n_c / G), a contiguous range of buckets holding
    // about n_c / G centres (off is non-decreasing)
    const int64_t n_c = off[K];
    auto first_at = [&](int64_t t) {   // smallest b in [0, K] with off[b] >= t
        int64_t lo_b = 0, hi_b = K;
        while (lo_b < hi_b) {
            const int64_t mid = (lo_b + hi_b) / 2;
            if (int64_t(off[mid]) < t) lo_b = mid + 1;
            else hi_b = mid;
        }
        return lo_b;
    };
    const int64_t b_begin = first_at(n_c * blockIdx.x / gridDim.x);
    const int64_t b_end = first_at(n_c * (int64_t(blockIdx.x) + 1) / gridDim.x);
    double s0 = 0.0, s1 = 0.0;
    for (int64_t b = b_begin; b < b_end; ++b) {
        const uint32_t lo = off[b], hi = off[b + 1];
        if (lo == hi) continue;   // uniform over the workgroup
        const int o[3] = {int(b / (NB * NB)) * E, int((b / NB) % NB) * E, int(b % NB) * E};
        __syncthreads();   // the previous block's reads (and the set-up above) are done
        for (int e = threadIdx.x; e < RV; e += kTriThreads) {
            const int i = e / (kTriReg * kTriReg), j = (e / kTriReg) % kTriReg, k = e % kTriReg;
            const int gx = (o[0] - marg - LO + i) & (N - 1), gy = (o[1] - marg - LO + j) & (N - 1),
                      gz = (o[2] - marg - LO + k) & (N - 1);
            reg[i * kTriPS + j * kTriRS + k] = f23[(int64_t(gx) * N + gy) * N + gz];
        }
        __syncthreads();
        const int64_t tot = int64_t(hi - lo) * n_rot;
        // the loop bound is uniform over a wavefront: every lane takes part in
        // every butterfly
        for (int64_t base = int64_t(wv) * 64; base < tot; base += kTriThreads) {
            const int64_t s = base + lane;
            const bool live = s < tot;
            double a = 0.0, v2 = 0.0, x[3] = {0.0, 0.0, 0.0}, u[3] = {0.0, 0.0, 1.0}, v[3] = {1.0, 0.0, 0.0};
            if (live) {
                const int64_t k = s / n_rot, r = s - k * n_rot;
                const int64_t c = list[lo + k];
                centre_of<BOX, true>(c, centres, box_L, seed, x);
                if constexpr (BOX) {
                    if (has_f1) {
                        const double uc[3] = {x[0] * scale, x[1] * scale, x[2] * scale};
                        if constexpr (F1R) a = region_value<B>(reg, uc, o, marg, tab);
                        else a = basis_value<float, N, B>(f1, uc, tab);
                    } else {
                        a = 1.0;
                    }
                } else {
                    a = weights ? double(weights[c]) : 1.0;
                }
                rotation_of(c, r, seed, u, v);
                const double p2[3] = {(x[0] + r12 * u[0]) * scale, (x[1] + r12 * u[1]) * scale,
                                      (x[2] + r12 * u[2]) * scale};
                v2 = region_value<B>(reg, p2, o, marg, tab);
            }
            s0 += a;
            s1 += a * v2;
            for (int j = 0; j < n_theta; ++j) {
                double p3 = 0.0, p23 = 0.0;
                if (live) {
                    const double ct = cs[2 * j], st = cs[2 * j + 1];
                    const double q[3] = {(x[0] + r13 * (ct * u[0] + st * v[0])) * scale,
                                         (x[1] + r13 * (ct * u[1] + st * v[1])) * scale,
                                         (x[2] + r13 * (ct * u[2] + st * v[2])) * scale};
                    const double v3 = region_value<B>(reg, q, o, marg, tab);
                    p3 = a * v3;
                    p23 = a * v2 * v3;
                }
                p3 = wave_sum(p3);
                p23 = wave_sum(p23);
                if (lane == 0) {
                    acc[(wv * n_theta + j) * 2] += p3;
                    acc[(wv * n_theta + j) * 2 + 1] += p23;
                }
            }
        }
    }
    const double b0 = block_sum_tri(s0, red);
    const double b1 = block_sum_tri(s1, red);   // ends with a barrier: acc is complete
    for (int j = threadIdx.x; j < n_theta; j += kTriThreads) {
        double t3 = 0.0, t23 = 0.0;
        for (int k = 0; k < kTriWaves; ++k) {
            t3 += acc[(k * n_theta + j) * 2];
            t23 += acc[(k * n_theta + j) * 2 + 1];
        }
        double* dst = part + (int64_t(blockIdx.x) * n_theta + j) * 4;
        dst[0] = b0;
        dst[1] = b1;
        dst[2] = t3;
        dst[3] = t23;
    }
}

template <int N, bool BOX, int B, bool F1R>
static void launch_blocks(int grid, size_t lds, hipStream_t stream, const float* f1, const float* f23,
                          const double* tab, const float* centres, const float* weights, int n_rot, double box_L,
                          double r12, double r13, int n_theta, uint64_t seed, int marg, const uint32_t* off,
                          const uint32_t* list, double* part) {
    auto kern = k_triplet_blocks<N, BOX, B, F1R>;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                              int(lds));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kTriThreads), lds, stream, f1, f23, tab, f1 != nullptr, centres,
                       weights, n_rot, box_L, r12, r13, n_theta, seed, marg, off, list, part);
}

template <int N, int B>
static hermes_status triplet_blocks(hermes_ctx ctx, const float* f1, const float* f23, double box_L,
                                    const float* centres, const float* weights, int64_t n_centres, double r12,
                                    double r13, int n_theta, int n_rot, uint64_t seed, int marg, double* out,
                                    void* work, hipStream_t stream) {
    double* part = static_cast<double*>(work);
    char* base = static_cast<char*>(work) + triplet_workspace_direct(N, HERMES_F32, n_theta);
    const TriLayout l = tri_layout(N, n_centres);
    uint32_t* key = reinterpret_cast<uint32_t*>(base + l.key);
    uint32_t* list = reinterpret_cast<uint32_t*>(base + l.list);
    uint32_t* count = reinterpret_cast<uint32_t*>(base + l.count);
    uint32_t* off = reinterpret_cast<uint32_t*>(base + l.off);
    uint32_t* blocksum = reinterpret_cast<uint32_t*>(base + l.blocksum);
    const int64_t nk = tri_buckets(N);
    const bool box = centres == nullptr;
    {
        LaunchScope ls(ctx, stream, "bucket");
        launch_fill<uint32_t>(count, nk, 0u, stream);
        const int64_t want = (n_centres + kThreads - 1) / kThreads;
        const int g = int(want < 8192 ? want : 8192);
        if (box)
            hipLaunchKernelGGL((k_tri_keys<N, true>), dim3(g), dim3(kThreads), 0, stream, centres, n_centres, box_L,
                               seed, key, count);
        else
            hipLaunchKernelGGL((k_tri_keys<N, false>), dim3(g), dim3(kThreads), 0, stream, centres, n_centres, box_L,
                               seed, key, count);
        launch_tile_scan(count, nk, off, blocksum, stream);
        radix_sort_indices(key, n_centres, uint32_t(nk - 1), list, base + l.sort, stream);
    }
    const int grid = int(std::min<int64_t>({nk, int64_t(ctx->cus), int64_t(kTripletBlocks)}));
    const size_t lds = tri_lds_bytes(n_theta);
    const double* tab = ctx->t.db2tab;
    {
        LaunchScope ls(ctx, stream, "triplet");
        if (!box)
            launch_blocks<N, false, B, false>(grid, lds, stream, nullptr, f23, tab, centres, weights, n_rot, box_L,
                                              r12, r13, n_theta, seed, marg, off, list, part);
        else if (f1 == f23)
            launch_blocks<N, true, B, true>(grid, lds, stream, f1, f23, tab, centres, weights, n_rot, box_L, r12,
                                            r13, n_theta, seed, marg, off, list, part);
        else
            launch_blocks<N, true, B, false>(grid, lds, stream, f1, f23, tab, centres, weights, n_rot, box_L, r12,
                                             r13, n_theta, seed, marg, off, list, part);
    }
    {
        LaunchScope ls(ctx, stream, "reduce");
        hipLaunchKernelGGL(k_triplet_final, dim3((n_theta * 4 + 127) / 128), dim3(128), 0, stream, part, grid,
                           n_theta, out);
    }
    return check_launch("hermes_triplet_mc");
}

template <typename T, int N, int B>
static hermes_status triplet_nb(hermes_ctx ctx, const void* f1, const void* f2, const void* f3, double box_L,
                                const float* centres, const float* weights, int64_t n_centres, double r12,
                                double r13, int n_theta, int n_rot, uint64_t seed, double* out, void* work,
                                size_t work_bytes, hipStream_t stream) {
    double* part = static_cast<double*>(work);
    const double* tab = ctx->t.db2tab;
    if constexpr (std::is_same<T, float>::value) {
        // block-local path: f2 and f3 one array, the reach within the region,
        // the bucket arrays in the workspace
        const double reach = std::max(r12, r13) * double(N) / box_L;
        const int marg = int(std::floor(reach)) + 2;
        if (f2 == f3 && n_centres >= 1 && n_centres <= INT32_MAX &&
            tri_blk(N) + 2 * marg + BasisTaps<B>::NT - 1 <= kTriReg && tri_lds_bytes(n_theta) <= size_t(160) * 1024 &&
            work_bytes >= triplet_workspace(N, HERMES_F32, n_theta, n_centres))
            return triplet_blocks<N, B>(ctx, static_cast<const float*>(f1), static_cast<const float*>(f2), box_L,
                                        centres, weights, n_centres, r12, r13, n_theta, n_rot, seed, marg, out, work,
                                        stream);
    }
    FieldRef<T, N, B> r1{static_cast<const T*>(f1), nullptr, tab}, r2{static_cast<const T*>(f2), nullptr, tab},
        r3{static_cast<const T*>(f3), nullptr, tab};
    if constexpr (N <= tile_max_n<T>()) {
        // pack every distinct field once
        char* base = static_cast<char*>(work) + align256(size_t(kTripletBlocks) * n_theta * 4 * sizeof(double));
        const size_t fb = align256(size_t(N / 2) * N * N * sizeof(Tile<T>));
        const void* src[3] = {f2, f3, f1};
        FieldRef<T, N, B>* dst[3] = {&r2, &r3, &r1};
        LaunchScope ls(ctx, stream, "pack_tiles");
        for (int i = 0; i < 3; ++i) {
            if (!src[i]) continue;
            int same = -1;
            for (int k = 0; k < i; ++k)
                if (src[k] == src[i]) same = k;
            if (same >= 0) {
                dst[i]->t = dst[same]->t;
                continue;
            }
            Tile<T>* t = reinterpret_cast<Tile<T>*>(base + size_t(i) * fb);
            dst[i]->t = t;
            const int64_t want = (int64_t(N / 2) * N * N + kThreads - 1) / kThreads;
            hipLaunchKernelGGL((k_pack_tiles<T, N, BasisTaps<B>::LO>), dim3(int(want < 8192 ? want : 8192)),
                               dim3(kThreads), 0, stream, static_cast<const T*>(src[i]), t);
        }
    }
    const int64_t total = n_centres * int64_t(n_rot);
    const int64_t want = (total + kThreads - 1) / kThreads;
    const int blocks = int(want < 1 ? 1 : (want < kTripletBlocks ? want : kTripletBlocks));
    {
        LaunchScope ls(ctx, stream, "triplet");
        if (centres) {
            hipLaunchKernelGGL((k_triplet<T, N, false, B>), dim3(blocks), dim3(kThreads), 0, stream, r1, r2, r3,
                               f1 != nullptr, centres, weights, n_centres, n_rot, box_L, r12, r13, n_theta, seed, part);
        } else {
            hipLaunchKernelGGL((k_triplet<T, N, true, B>), dim3(blocks), dim3(kThreads), 0, stream, r1, r2, r3,
                               f1 != nullptr, centres, weights, n_centres, n_rot, box_L, r12, r13, n_theta, seed, part);
        }
    }
    {
        LaunchScope ls(ctx, stream, "reduce");
        hipLaunchKernelGGL(k_triplet_final, dim3((n_theta * 4 + 127) / 128), dim3(128), 0, stream, part, blocks,
                           n_theta, out);
    }
    return check_launch("hermes_triplet_mc");
}

template <typename T, int N>
static hermes_status triplet_n(hermes_ctx ctx, const void* f1, const void* f2, const void* f3, double box_L,
                               const float* centres, const float* weights, int64_t n_centres, double r12,
                               double r13, int n_theta, int n_rot, uint64_t seed, double* out, void* work,
                               size_t work_bytes, hipStream_t stream) {
    if (ctx->basis == HERMES_BASIS_DB2)
        return triplet_nb<T, N, HERMES_BASIS_DB2>(ctx, f1, f2, f3, box_L, centres, weights, n_centres, r12, r13,
                                                  n_theta, n_rot, seed, out, work, work_bytes, stream);
    return triplet_nb<T, N, HERMES_BASIS_B3>(ctx, f1, f2, f3, box_L, centres, weights, n_centres, r12, r13, n_theta,
                                             n_rot, seed, out, work, work_bytes, stream);
}

hermes_status triplet_impl(hermes_ctx ctx, const void* f1, const void* f2, const void* f3, int n, int dtype,
                           double box_L, const float* centres, const float* weights, int64_t n_centres, double r12,
                           double r13, int n_theta, int n_rot, uint64_t seed, double* out, void* work,
                           size_t work_bytes, hipStream_t stream) {
#define HERMES_TRIPLET_CASE(NN)                                                                                    \
    case NN:                                                                                                       \
        return dtype == HERMES_F32                                                                                 \
                   ? triplet_n<float, NN>(ctx, f1, f2, f3, box_L, centres, weights, n_centres, r12, r13, n_theta, \
                                          n_rot, seed, out, work, work_bytes, stream)                             \
                   : triplet_n<double, NN>(ctx, f1, f2, f3, box_L, centres, weights, n_centres, r12, r13, n_theta, \
                                           n_rot, seed, out, work, work_bytes, stream);
    switch (n) {
        HERMES_TRIPLET_CASE(8)
        HERMES_TRIPLET_CASE(16)
        HERMES_TRIPLET_CASE(32)
        HERMES_TRIPLET_CASE(64)
        HERMES_TRIPLET_CASE(128)
        HERMES_TRIPLET_CASE(256)
        HERMES_TRIPLET_CASE(512)
        HERMES_TRIPLET_CASE(1024)
        default:
            return fail(HERMES_ERR_ARG, "hermes_triplet_mc: unsupported N");
    }
#undef HERMES_TRIPLET_CASE
}

}  // namespace hermes
