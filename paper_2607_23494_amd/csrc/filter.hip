// Batched window filtering and the 3PCF multipole contraction.
//
// For a batch of nb windows that share one angular factor A(k^) (1 for the
// isotropic windows, 4 pi i^l Y^R_lm(k^) for the multipole windows of
// Sec. 3.3.3 Eq. multipole-window), each filtered field is
//   f_b = iDFT[ delta^ Phi^ A R_b(|k|) ]      (Sec. 4.2, K_W = W^ Phi^)
// and the three inverse passes are:
//   X  (k_win_x):  form B = delta^ Phi^ A s / N^3 for a tile once (float64),
//                  then for every window multiply by the radial factor R_b
//                  (exact values per |n~|^2, read from a per-column table),
//                  inverse FFT along x and write the batch spectrum b;
//   Y  (k_inv_y_pack): inverse FFT along y of all nb spectra in place, fused
//                  with the packing step of the c2r transform along z;
//   Z  (k_c2r_z):  the length-N/2 complex inverse along z for all nb windows
//                  of a row group at once and a fused epilogue: either the
//                  counts-in-cells moments (and optionally the stored
//                  fields), or the contraction sum_x delta(x) f_b1(x) f_b2(x)
//                  of the 3PCF (Sec. 3.4, Eq. particle_nfold with a naked
//                  primary vertex).
// Grid-wide sums are accumulated in float32 over a row group (<= 1024 cells)
// and in float64 across groups and workgroups.
#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "common.hpp"
#include "fft_kernels.hpp"
#include "kernels.hpp"
#include "special.hpp"

namespace hermes {

constexpr int kMaxBatch = 32;        // windows per batch (registers of the epilogues)
constexpr int kFilterChunk = 8;      // windows per workspace batch in hermes_filter_bins
constexpr int kZGroups = 1024;       // persistent workgroups of the z pass

struct WinSet {
    int type[kMaxBatch];
    int ell[kMaxBatch];
    int out[kMaxBatch];              // destination index of each window
    double lo[kMaxBatch];
    double hi[kMaxBatch];
    int n;
};

template <int N> struct zrows {
    static constexpr int M = N / 2;
    static constexpr int R = M >= 256 ? 1 : 256 / M;   // rows per group
};

// Line stride of the element-major z tile: the line count made odd.
__host__ __device__ constexpr int z_lt(int nlines) { return nlines | 1; }

constexpr size_t kZLdsBudget = 81920;   // bytes: two z-pass workgroups per CU

template <typename T, int N>
constexpr size_t z_lds_bytes(int nb) {
    using C = typename cplx_of<T>::type;
    constexpr int R = zrows<N>::R, M = N / 2;
    const size_t lines = size_t(M) * z_lt(nb * R) * sizeof(C) + size_t(R) * N * sizeof(T) + size_t(R) * N * 2 +
                         size_t(M) * sizeof(C);
    const size_t red = size_t(kThreads) * 16 * sizeof(double);
    return lines > red ? lines : red;
}

// Largest batch whose z-pass tile fits the LDS budget.
template <typename T, int N>
constexpr int z_max_batch() {
    int nb = kMaxBatch;
    while (nb > 1 && z_lds_bytes<T, N>(nb) > kZLdsBudget) --nb;
    return nb;
}

inline int z_max_batch_rt(int n, bool dbl) {
#define HERMES_ZMB(NN) \
    case NN:           \
        return dbl ? z_max_batch<double, NN>() : z_max_batch<float, NN>();
    switch (n) {
        HERMES_ZMB(8)
        HERMES_ZMB(16)
        HERMES_ZMB(32)
        HERMES_ZMB(64)
        HERMES_ZMB(128)
        HERMES_ZMB(256)
        HERMES_ZMB(512)
        HERMES_ZMB(1024)
    }
#undef HERMES_ZMB
    return 1;
}

// bytes of one padded half spectrum [N][N][pitch]
// Padded plane stride (complex elements) of the batch spectra: N rows of the
// padded pitch plus kPlanePad, so that consecutive x planes do not start at a
// near power-of-two distance (the x pass writes one row per plane per tile;
// measured about 2 % faster at 512^3 than without the pad).
constexpr int kPlanePad = 64;
template <int N> __host__ __device__ constexpr int64_t plane_stride() { return int64_t(N) * pitch_of<N>() + kPlanePad; }
inline int64_t plane_stride_rt(int n) { return int64_t(n) * pitch_rt(n) + kPlanePad; }

// bytes of one padded batch spectrum [N][plane_stride]
inline size_t spec_bytes(int n, bool dbl) {
    return size_t(n) * plane_stride_rt(n) * (dbl ? 16 : 8);
}

// ---------------------------------------------------------------- radial table
// tab[b * nq + q] = R_b(k_q), k_q = kfac sqrt(q), evaluated in float64; one
// thread per (q, window b = blockIdx.y).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_radial(T* __restrict__ tab, int64_t nq, WinSet ws, double kfac,
                                                     const double* __restrict__ gl) {
    const int64_t q = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    const int b = blockIdx.y;
    if (q >= nq || b >= ws.n) return;
    const double k = kfac * sqrt(double(q));
    double v;
    switch (ws.type[b]) {
        case HERMES_WIN_SHELL: v = w_shell(k, ws.lo[b], ws.hi[b]); break;
        case HERMES_WIN_SPHERE: v = w_sphere(k * ws.hi[b]); break;
        case HERMES_WIN_GAUSS: v = exp(-0.5 * (k * ws.hi[b]) * (k * ws.hi[b])); break;
        default: v = jbar(ws.ell[b], k, ws.lo[b], ws.hi[b], gl); break;
    }
    tab[b * nq + q] = T(v);
}

// ---------------------------------------------------------------- kz order
// Order of the kz columns in the padded spectra of the inverse passes (after
// the x pass): the mirror pair (k, M - k), M = N/2, sits at positions 2k and
// 2k + 1 (k <= M/2), so that the packing step of the c2r transform along z
// combines neighbouring columns.  Positions 0 .. M hold kz = 0 .. M exactly
// once (position 1 holds kz = M); position M + 1 would repeat kz = M/2 and the
// positions above it are row padding.  After the y pass a row holds the packed
// c2r input Z[k], k < M: Z[kz_of_pos(pos)] at every position but 1 (kz = M has
// no Z), so Z[M/2] stays at position M, in the tile that computes it.
template <int N> __host__ __device__ constexpr int kz_of_pos(int pos) { return (pos & 1) ? N / 2 - (pos >> 1) : (pos >> 1); }
template <int N> __host__ __device__ constexpr bool pos_used(int pos) { return pos <= N / 2; }
// The z pass reads Z[k], k < M, from M row positions: position 0 and 2 .. M
// (Z[M/2] at position M).  Slot s in [0, M) of that list: the position it is
// read from and the index k it holds.
template <int N> __host__ __device__ constexpr int zslot_pos(int s) { return s == 1 ? N / 2 : s; }
template <int N> __host__ __device__ constexpr int zk_of_pos(int s) { return s == 1 ? N / 4 : kz_of_pos<N>(s); }

// ---------------------------------------------------------------- column table
// The radial factor unrolled along x for every (|ky|, kz) column:
// U[(row(a, c) nb + b) HP + ax] = tab[b nq + a^2 + c^2 + ax^2] for ax < H =
// N/2 + 1 (zeros up to the pitch HP, a multiple of 16 bytes), with
// row(a, c) = c (c + 1) / 2 + a for a <= c (the factor is symmetric in |ky|
// and kz).  The x pass copies the runs of a tile's columns with 16-byte
// loads instead of scattering into tab.
inline int64_t col_rows(int n) { return int64_t(n / 2 + 1) * (n / 2 + 2) / 2; }
inline int col_pitch_rt(int n, size_t elem) {
    const int v = int(16 / elem);
    return (n / 2 + 1 + v - 1) / v * v;
}
template <typename T, int N> __host__ __device__ constexpr int col_pitch() {
    constexpr int v = 16 / int(sizeof(T));
    return (N / 2 + 1 + v - 1) / v * v;
}
inline size_t col_table_bytes(int n, int nb, size_t elem) {
    return size_t(col_rows(n)) * nb * col_pitch_rt(n, elem) * elem;
}

__device__ __forceinline__ int64_t col_row(int a, int c) {
    if (a > c) { const int t = a; a = c; c = t; }
    return int64_t(c) * (c + 1) / 2 + a;
}

// One workgroup per (row, window); the window is the slow grid axis, so the
// workgroups in flight gather from one window's table, which stays in L2.
template <typename T, int N>
__global__ __launch_bounds__(kThreads) void k_radial_cols(const T* __restrict__ tab, int64_t nq, int nb,
                                                          T* __restrict__ U) {
    constexpr int H = N / 2 + 1, HP = col_pitch<T, N>();
    const int64_t row = blockIdx.x;
    const int b = blockIdx.y;
    // invert row = c (c + 1) / 2 + a, 0 <= a <= c
    int c = int((sqrt(8.0 * double(row) + 1.0) - 1.0) * 0.5);
    while (int64_t(c + 1) * (c + 2) / 2 <= row) ++c;
    while (int64_t(c) * (c + 1) / 2 > row) --c;
    const int a = int(row - int64_t(c) * (c + 1) / 2);
    const int64_t q0 = int64_t(a) * a + int64_t(c) * c;
    const T* tb = tab + b * nq + q0;
    T* dst = U + (row * nb + b) * HP;
    for (int ax = threadIdx.x; ax < HP; ax += kThreads) dst[ax] = ax < H ? tb[int64_t(ax) * ax] : T(0);
}

// ---------------------------------------------------------------- pass X
// Column passes (x and y) use one column per thread; float tiles are 16
// columns x N (128-byte row segments) on 1024 threads, double tiles 8 columns
// on 512 threads (64 KB of LDS either way).
template <typename T> constexpr int win_vec() { return 1; }
template <typename T> constexpr int win_threads() { return sizeof(T) == 4 ? 1024 : 512; }

// Tiles of TC consecutive columns of the padded (ky, kz) plane of B: for every
// window b multiply by the radial factor R_b(q), q = |n~|^2, inverse FFT along
// x and write spectrum b.  Rows are 128-byte aligned, so a tile writes whole
// 128-byte lines of every x plane; the stores are non-temporal (measured about
// 20 % faster for this plane-strided pattern at 512^3).  The table runs of
// window b + 1 are loaded before the FFT of window b so their latency
// overlaps it.
template <typename T> struct vec16 {
    typedef T type __attribute__((ext_vector_type(16 / sizeof(T))));
};

// First column of x-pass tile b.  When tiles tile the rows (TC divides the
// pitch), the tiles (ky, t) and (N - ky, t), which read the same table runs
// (the radial factor depends on |ky|), are dispatched back to back so the
// second read finds the runs in the last-level cache: b = 0 .. 2 TPR - 1 are
// the rows ky = 0 and N/2, then pairs (ky, N - ky), ky = 1 .. N/2 - 1.
template <int N, int PP, int TC>
__device__ __forceinline__ int x_tile_origin(int b) {
    if constexpr (PP % TC == 0) {
        constexpr int TPR = PP / TC;   // tiles per row
        int ky, t;
        if (b < 2 * TPR) {
            ky = b < TPR ? 0 : N / 2;
            t = b % TPR;
        } else {
            const int u = (b - 2 * TPR) / 2, side = (b - 2 * TPR) % 2;
            const int a = 1 + u / TPR;
            t = u % TPR;
            ky = side ? N - a : a;
        }
        return ky * PP + t * TC;
    } else {
        return b * TC;
    }
}

// NM angular factors (1 or 2: two m of one l, which share the radial table)
// per launch: yc[a] and out[a] for a < NM; the table runs and delta^ are read
// once for both.
template <typename T, int N, int VEC, int NT, int NM>
__global__ __launch_bounds__(NT) void k_win_x(const typename cplx_of<T>::type* __restrict__ dk,
                                                    int sh, YlmConst yc0, YlmConst yc1, double sre, double sim,
                                                    const double* __restrict__ phi1d,
                                                    typename cplx_of<T>::type* __restrict__ out0,
                                                    typename cplx_of<T>::type* __restrict__ out1,
                                                    int64_t bin_stride, int nb, const T* __restrict__ U,
                                                    const typename cplx_of<T>::type* __restrict__ tw) {
    using C = typename cplx_of<T>::type;
    using V = typename vec16<T>::type;
    using G = col_cfg<T, N, VEC, NT>;
    constexpr int TC = G::TC, LPR = G::LPR, RPP = G::RPP;
    constexpr int H = N / 2 + 1, PP = pitch_of<N>(), HP = col_pitch<T, N>();
    constexpr int64_t PLANE = int64_t(N) * PP;
    constexpr int VE = 16 / int(sizeof(T));           // table values per 16-byte chunk
    constexpr int CPC = HP / VE;                       // chunks per column run
    constexpr int NCH = TC * CPC;                      // chunks per tile and window
    constexpr int CPT = (NCH + NT - 1) / NT;
    __shared__ C s[N * TC];
    __shared__ C twl[N];
    __shared__ V su[NCH];                              // the tile's table runs, column v at [v CPC, (v+1) CPC)
    __shared__ C raw1[NM > 1 ? 8 * VEC * NT : 1];      // the second factor's tile values, [i][v][thread]
    stage_twiddles<C, N, NT>(twl, tw);
    const int c0 = x_tile_origin<N, PP, TC>(blockIdx.x);
    const int lc = (threadIdx.x % LPR) * VEC, r0 = threadIdx.x / LPR;
    // columns past N/2 in a row are padding: neither read nor written
    // output column c of a row is position c % PP, i.e. kz = kz_of_pos(c % PP)
    auto col_ok = [&](int c, int64_t& row, int& kz) {
        const int ky = c / PP, pos = c - (c / PP) * PP;
        kz = kz_of_pos<N>(pos);
        row = col_row(abs(signed_mode<N>(ky & (N - 1))), kz);
        return c < PLANE && pos_used<N>(pos);
    };
    bool ok[VEC];
    int kyv[VEC], kzv[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
        int64_t row;
        const int c = c0 + lc + v;
        ok[v] = col_ok(c, row, kzv[v]);
        kyv[v] = (c / PP) & (N - 1);
    }
    // 16-byte chunks of the table runs this thread copies into su
    const V* csrc[CPT];
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
        const int i = threadIdx.x + u * NT;
        const int v = i / CPC;
        int64_t row = 0;
        int kz;
        const bool good = i < NCH && col_ok(c0 + v, row, kz);
        // chunks of padding columns (never stored) read the first run instead
        csrc[u] = good ? reinterpret_cast<const V*>(U + row * nb * HP) + (i - v * CPC) : reinterpret_cast<const V*>(U);
    }
    V ureg[CPT];
    auto uload = [&](int b) {
#pragma unroll
        for (int u = 0; u < CPT; ++u) ureg[u] = csrc[u][int64_t(b) * CPC];
    };
    auto ustore = [&]() {
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int i = threadIdx.x + u * NT;
            if (i < NCH) su[i] = ureg[u];
        }
    };
    const T* suf = reinterpret_cast<const T*>(su);
    // raw = delta^ Phi^ A s / N^3 of the tile (A = 1 or the Nyquist-averaged
    // Y^R_lm, s the complex constant), in float64 and rounded once
    // (the first factor's in registers, the second's in LDS)
    C raw[8][VEC];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int kx = r0 + i * RPP;
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            raw[i][v] = C{T(0), T(0)};
            if constexpr (NM > 1) raw1[(i * VEC + v) * NT + threadIdx.x] = C{T(0), T(0)};
            if (ok[v]) {
                const int ky = kyv[v], kz = kzv[v];
                const C d = dk[(int64_t(kx) * N + ky) * (N / 2 + 1) + kz];
                const double f0 = phi1d[N + kx] * phi1d[N + ky] * phi1d[N + kz];
                const double re = double(d.x) * sre - double(d.y) * sim;
                const double im = double(d.x) * sim + double(d.y) * sre;
#pragma unroll
                for (int a = 0; a < NM; ++a) {
                    double f = f0;
                    if (sh)
                        f *= ylm_mode(a ? yc1 : yc0, signed_mode<N>(kx), signed_mode<N>(ky), kz, kx == N / 2,
                                      ky == N / 2, kz == N / 2);
                    if (a == 0)
                        raw[i][v] = C{T(re * f), T(im * f)};
                    else
                        raw1[(i * VEC + v) * NT + threadIdx.x] = C{T(re * f), T(im * f)};
                }
            }
        }
    }
    uload(0);
    ustore();
    __syncthreads();
    for (int b = 0; b < nb; ++b) {
#pragma unroll
        for (int a = 0; a < NM; ++a) {
            C x[8][VEC];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int ax = abs(signed_mode<N>(r0 + i * RPP));
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    const T r = suf[(lc + v) * HP + ax];
                    const C w = a ? raw1[(i * VEC + v) * NT + threadIdx.x] : raw[i][v];
                    x[i][v] = C{w.x * r, w.y * r};
                }
            }
            const bool last = a == NM - 1;   // the last reader of su for window b
            if (a == 0 && b + 1 < nb) uload(b + 1);   // lands during the transform
            C* ob = (a ? out1 : out0) + b * bin_stride + c0;
            // padding positions above N/2 + 1 hold zeros and are stored too,
            // so every row is written in whole 128-byte lines
            auto st = [&](int p, int line, C val) {
                const int c = c0 + line;
                if (c < PLANE) st_stream(ob + int64_t(p) * plane_stride<N>() + line, val);
            };
            if constexpr (N > 8) {
                // the next window's runs go to su before this window's last
                // stores are issued (su was last read before the transform's
                // first barrier): waiting for the loads never waits for them
                col_fft_front<C, N, TC, VEC, true, NT, 0>(s, twl, x, lc, r0);
                if (last && b + 1 < nb) ustore();
                auto fin = [&](int jj, int line, const C* v, int R, int NS) {
#pragma unroll
                    for (int r = 0; r < R; ++r) st(jj + r * NS, line, v[r]);
                };
                col_fft_last<C, N, TC, true, NT, 0>(s, twl, fin);
                __syncthreads();
            } else {
                col_fft<C, N, TC, VEC, true, NT, 0>(s, twl, x, lc, r0, st);
                __syncthreads();
                if (last && b + 1 < nb) {
                    ustore();
                    __syncthreads();
                }
            }
        }
    }
}

// ---------------------------------------------------------------- pass Y
// Inverse FFT along y of every (window, x) plane fused with the packing step
// of the c2r transform along z that follows: with M = N/2, the length-N real
// inverse of X[0..M] equals the length-M complex inverse of
//   Z[k] = (X[k] + X*[M-k]) + i e^{+2 pi i k/N} (X[k] - X*[M-k]),  k < M,
// whose output holds samples 2n and 2n+1 in its real and imaginary parts.
// Columns k and M - k are neighbours in the pair order (kz_of_pos), so a tile
// of TC consecutive positions holds whole pairs; the pair is combined right
// after the transform and Z[kz] overwrites X[kz] at its own position (kz = M
// at position 1 has no Z and is left as it is), so no tile writes a position
// that another tile reads.  With TC <= 64 the last Stockham stage leaves the two
// columns of a pair in neighbouring lanes of one wavefront; wider tiles pair
// through LDS.  Position M + 1 is loaded as a copy of kz = M/2, the partner of
// position M.  One 8-byte column per thread and load round.
template <typename T, int N> struct ypack_cfg {
    static constexpr int NT = win_threads<T>();
    static constexpr int TC = col_cfg<T, N, 1, NT>::TC;   // positions per tile
    static constexpr int TILES = (N / 2 + 2 + TC - 1) / TC;
};

template <typename T, int N>
__global__ __launch_bounds__((ypack_cfg<T, N>::NT)) void k_inv_y_pack(typename cplx_of<T>::type* __restrict__ data,
                                                         int64_t plane_stride,
                                                         const typename cplx_of<T>::type* __restrict__ tw) {
    using C = typename cplx_of<T>::type;
    constexpr int TC = ypack_cfg<T, N>::TC, NT = ypack_cfg<T, N>::NT;
    constexpr int M = N / 2, PP = pitch_of<N>(), PER = N / 8;
    static_assert(TC % 2 == 0, "pairs per tile");
    __shared__ C s[N * TC];
    __shared__ C twl[N];
    stage_twiddles<C, N, NT>(twl, tw);
    C* base = data + int64_t(blockIdx.y) * plane_stride;
    const int c0 = blockIdx.x * TC;
    const int c = threadIdx.x % TC, j = threadIdx.x / TC;
    const int pos = c0 + c;
    const int lpos = pos == M + 1 ? M : pos;
    C x[8][1];
    // streaming (non-temporal) accesses where a tile row fills whole 128-byte
    // lines (measured faster at 512^3); with 64-byte row segments (float at
    // 1024^3) they were much slower than plain ones
    constexpr bool STREAM = TC * int(sizeof(C)) >= 128;
    auto ld = [&](const C* q) { return STREAM ? ld_stream(q) : *q; };
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i][0] = pos <= M + 1 ? ld(base + int64_t(j + i * PER) * PP + lpos) : C{T(0), T(0)};
    // Z[kz] from own X[kz] and partner X[M-kz]: (X + X'*) + i e^{+2 pi i kz/N} (X - X'*),
    // e^{+2 pi i kz/N} = conj(tw[N + kz])
    auto pack = [&](C own, C oth, C w) {
        const C sum{own.x + oth.x, own.y - oth.y};
        const C dif{own.x - oth.x, own.y + oth.y};
        const C t = c_mul(C{w.x, -w.y}, dif);
        return C{sum.x - t.y, sum.y + t.x};
    };
    if constexpr (TC <= 64 && N > 8) {
        auto fin = [&](int jj, int line, const C* v, int R, int NS) {
            const int p = c0 + line;
            // every position of the row is stored, also position 1 and the
            // padding above M (values nobody reads), so rows are written in
            // whole 128-byte lines
            const bool store = p < PP;
            const C w = twl[kz_of_pos<N>(p) & (N - 1)];
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                if (r < R) {
                    const C oth{__shfl_xor(v[r].x, 1), __shfl_xor(v[r].y, 1)};
                    const C z = pack(v[r], oth, w);
                    if (store) {
                        if constexpr (STREAM)
                            st_stream(base + int64_t(jj + r * NS) * PP + p, z);
                        else
                            base[int64_t(jj + r * NS) * PP + p] = z;
                    }
                }
            }
        };
        col_fft_fin<C, N, TC, 1, true, NT, 0>(s, twl, x, c, j, fin);
    } else {
        col_fft_lds<C, N, TC, 1, true, NT, 0>(s, twl, x, c, j);
        for (int e = threadIdx.x; e < N * TC; e += NT) {
            const int y = e / TC, q = e - (e / TC) * TC;
            const int p = c0 + q;
            if (p >= PP) continue;
            base[int64_t(y) * PP + p] = pack(s[y * TC + q], s[y * TC + (q ^ 1)], twl[kz_of_pos<N>(p) & (N - 1)]);
        }
    }
}

// ---------------------------------------------------------------- pass Z
enum { EPI_MOMENTS = 0, EPI_CONTRACT = 1 };

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));

// Contraction of one row group on the matrix cores.  With y_b(c) =
// sqrt|delta(c)| x_b(c) and s(c) the sign of delta(c), the group's share is
//   C[i][j] = sum_c s(c) y_i(c) y_j(c),   i, j < 32,
// and the split y = y_hi + y_lo in bf16 (PREC 1) or fp16 (PREC 2) gives
//   C = H + L + L^T + O(y_lo^2),  H = sum_c s y_hi y_hi^T,  L = sum_c s y_lo y_hi^T,
// i.e. the three hi/lo products of the split with the two mixed ones equal up
// to a transpose.  Both terms are 32x32x16 MFMAs over 16 cells with the
// operand B = s y_hi (the sign flips the packed halves with one xor per two
// cells).  Wave w takes a quarter of the group's cells; lane l supplies bin
// l % 32 at cells 8 (l / 32) .. +7 of each step; lanes past the last window
// repeat it (rows and columns >= nb of C are never read).  H is added to the
// float64 accumulators once per group; L, about 2^-8 of H, stays in float32
// across groups and is transposed in the final reduction.
// sr[c] = sqrt|delta(c)|, sgn[c / 2] = the sign bits of cells c, c + 1 at bits
// 15 and 31.
template <typename T, int N, int PREC, int LT>
__device__ __forceinline__ void mfma_contract(const typename cplx_of<T>::type* s, const float* sr,
                                              const uint32_t* sgn, int nb, double* acc64, f32x16_t& accl) {
    using C = typename cplx_of<T>::type;
    using V = typename std::conditional<PREC == HERMES_PREC_BF16X3, bf16x8_t, f16x8_t>::type;
    using E = typename std::conditional<PREC == HERMES_PREC_BF16X3, __bf16, _Float16>::type;
    constexpr int R = zrows<N>::R;
    constexpr int CELLS = R * N;
    constexpr int PER_WAVE = CELLS / (kThreads / 64);
    static_assert(PER_WAVE % 16 == 0, "16-cell MFMA steps");
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    const int bin = min(l % 32, nb - 1), half = l / 32;
    f32x16_t acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    for (int step = 0; step < PER_WAVE / 16; ++step) {
        const int c0 = w * PER_WAVE + step * 16 + 8 * half;   // 8 consecutive cells of one row
        const int r = c0 / N, z = c0 - r * N;
        const C* src = s + (z >> 1) * LT + bin * R + r;   // complex element z/2 of the line
        const float4 r0 = *reinterpret_cast<const float4*>(sr + c0);
        const float4 r1 = *reinterpret_cast<const float4*>(sr + c0 + 4);
        const u32x4_t sm = *reinterpret_cast<const u32x4_t*>(sgn + c0 / 2);
        const float rr[8] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
        float y[8];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const C v = src[u * LT];
            y[2 * u] = float(v.x) * rr[2 * u];
            y[2 * u + 1] = float(v.y) * rr[2 * u + 1];
        }
        V hi, lo;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            hi[t] = (E)y[t];
            lo[t] = (E)(y[t] - float(hi[t]));
        }
        const V hs = __builtin_bit_cast(V, __builtin_bit_cast(u32x4_t, hi) ^ sm);
        if constexpr (PREC == HERMES_PREC_BF16X3) {
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hi, hs, acc, 0, 0, 0);
            accl = __builtin_amdgcn_mfma_f32_32x32x16_bf16(lo, hs, accl, 0, 0, 0);
        } else {
            acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(hi, hs, acc, 0, 0, 0);
            accl = __builtin_amdgcn_mfma_f32_32x32x16_f16(lo, hs, accl, 0, 0, 0);
        }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) acc64[r] += double(acc[r]);
}

// Non-temporal load of the complex value at byte offset off from base through
// a raw buffer resource: a wavefront-uniform base costs scalar instructions
// only and the per-lane part is one 32-bit offset.
template <typename C>
__device__ __forceinline__ C ld_stream_buf(const C* base, unsigned off) {
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<C*>(base), 0, 0x7fffffff, 0x00020000);
    if constexpr (sizeof(C) == 8) {
        return __builtin_bit_cast(C, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 2));
    } else {
        static_assert(sizeof(C) == 16, "complex float or double");
        return __builtin_bit_cast(C, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 2));
    }
}

// Inverse along z of nb windows x R rows per group (the input rows hold the
// packed Z[0..M-1], M = N/2, in the pair order, written by the y pass), then
// the epilogue.  Persistent workgroups.  The nb R lines of a group are split
// into four contiguous runs, one per wavefront: a wavefront loads its lines,
// stores them to LDS and transforms them on its own (no workgroup barrier),
// then issues the loads of its lines of the next group, whose latency the
// epilogue hides; the workgroup synchronises only around the epilogue, which
// reads every line.  For M >= 64 a lane loads elements lane + 64 i of a
// line: one wavefront-contiguous run from a uniform base address.
// Dynamic LDS: the nb R lines of M complex stored element-major with line
// stride LT = z_lt(NBCAP R) (a compile-time stride keeps every LDS offset of
// the FFT stages an immediate), the delta rows [R][N] (sqrt|delta| for the
// matrix-core contraction), their packed sign bits [R N / 2], then the
// per-stage twiddles of the length-M transform (em_stage_twiddles).  Real
// sample z of line c sits at float index 2 ((z / 2) LT + c) + z % 2.
// NBCAP bounds nb (registers).
template <typename T, int N, int EPI, int NBCAP, int PREC>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_c2r_z(const typename cplx_of<T>::type* __restrict__ spec,
                                                    int64_t bin_stride, int nb, const T* __restrict__ delta,
                                                    T* __restrict__ out, WinSet map,
                                                    double* __restrict__ part,
                                                    const typename cplx_of<T>::type* __restrict__ tw) {
    using C = typename cplx_of<T>::type;
    constexpr int M = N / 2, PP = pitch_of<N>();
    constexpr int R = zrows<N>::R;
    constexpr int CELLS = R * N;
    constexpr int GROUPS = N * N / R;
    constexpr int MAXLINES = NBCAP * R;
    constexpr int NW = kThreads / 64;                       // wavefronts
    constexpr int MAXLW = (MAXLINES + NW - 1) / NW;         // lines per wavefront
    constexpr int MAXE = (MAXLW * M + 63) / 64;             // elements per lane
    constexpr int DPT = CELLS / kThreads;   // delta cells per thread (consecutive)
    static_assert(CELLS % kThreads == 0 && DPT % 2 == 0, "delta cells in pairs");
    constexpr bool MF = EPI == EPI_CONTRACT && PREC != HERMES_PREC_FP32;
    extern __shared__ double lds_raw[];
    C* s = reinterpret_cast<C*>(lds_raw);
    T* sf = reinterpret_cast<T*>(lds_raw);
    const int nlines = nb * R;
    constexpr int LT = z_lt(MAXLINES);
    T* sd = reinterpret_cast<T*>(s + M * LT);
    uint32_t* sgn = reinterpret_cast<uint32_t*>(sd + R * N);
    C* twl = reinterpret_cast<C*>(sgn + R * N / 2);
    auto at = [&](int line, int z) { return 2 * ((z >> 1) * LT + line) + (z & 1); };
    em_stage_twiddles<C, M>(twl, tw + M, threadIdx.x, kThreads);

    // this wavefront's lines [c_lo, c_lo + nlw)
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), lane = threadIdx.x % 64;
    const int c_lo = wv * nlines / NW, nlw = (wv + 1) * nlines / NW - c_lo;
    const EmMap em = em_map(nlw > 0 ? nlw : 1, lane);
    C* sw = s + c_lo;
    // element i of the lane: local line and position
    auto elem = [&](int i, int& ll, int& pos) {
        const int e = lane + 64 * i;
        ll = e / M;
        pos = e - ll * M;
    };

    // contraction roles: 4x4 bin tiles (I <= J) x cell groups
    const int nt4 = (nb + 3) / 4;
    const int ntp = nt4 * (nt4 + 1) / 2;
    const int cg_n = kThreads / ntp;
    const int tp = threadIdx.x % ntp, cg = threadIdx.x / ntp;
    int ti = 0, tj = 0;
    {
        int idx = tp;
        for (int I = 0; I < nt4; ++I) {
            if (idx < nt4 - I) {
                ti = I;
                tj = I + idx;
                break;
            }
            idx -= nt4 - I;
        }
    }
    // moments roles: one window per thread, subs cell groups
    const int subs = kThreads / nb;
    const int mb = threadIdx.x % nb, msub = threadIdx.x / nb;

    double acc64[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) acc64[i] = 0.0;
    f32x16_t accl;   // the L term of the matrix-core contraction
#pragma unroll
    for (int i = 0; i < 16; ++i) accl[i] = 0.f;

    typedef T dvec_t __attribute__((ext_vector_type(DPT)));
    C pre[MAXE];
    dvec_t dpre;
    auto fetch = [&](int g) {
        const int64_t row0 = int64_t(g) * R;
#pragma unroll
        for (int i = 0; i < MAXE; ++i) {
            int ll, pos;
            elem(i, ll, pos);
            if (ll < nlw) {
                const int line = c_lo + ll, b = line / R;
                const int64_t row = row0 + (line - b * R);   // (x, y) = (row / N, row % N)
                const C* base = spec + b * bin_stride + (row / N) * plane_stride<N>() + (row % N) * PP;
                if constexpr (M >= 64) {
                    pre[i] = ld_stream_buf(base, unsigned(zslot_pos<N>(pos)) * unsigned(sizeof(C)));   // line uniform in i
                } else {
                    pre[i] = ld_stream(base + zslot_pos<N>(pos));
                }
            }
        }
        if (EPI == EPI_CONTRACT) dpre = *reinterpret_cast<const dvec_t*>(delta + row0 * N + DPT * threadIdx.x);
    };
    __syncthreads();   // twiddles
    if (blockIdx.x < GROUPS) fetch(blockIdx.x);
    for (int g = blockIdx.x; g < GROUPS; g += gridDim.x) {
        const int64_t row0 = int64_t(g) * R;
#pragma unroll
        for (int i = 0; i < MAXE; ++i) {
            int ll, pos;
            elem(i, ll, pos);
            if (ll < nlw) sw[zk_of_pos<N>(pos) * LT + ll] = pre[i];
        }
        if constexpr (MF) {
#pragma unroll
            for (int p = 0; p < DPT / 2; ++p) {
                const float d0 = float(dpre[2 * p]), d1 = float(dpre[2 * p + 1]);
                sd[DPT * threadIdx.x + 2 * p] = T(sqrtf(fabsf(d0)));
                sd[DPT * threadIdx.x + 2 * p + 1] = T(sqrtf(fabsf(d1)));
                sgn[DPT / 2 * threadIdx.x + p] = ((__float_as_uint(d0) >> 16) & 0x8000u) | (__float_as_uint(d1) & 0x80000000u);
            }
        } else if constexpr (EPI == EPI_CONTRACT) {
#pragma unroll
            for (int i = 0; i < DPT; ++i) sd[DPT * threadIdx.x + i] = dpre[i];
        }
        if (nlw == MAXLW)
            wave_fft_em<C, M, true, MAXLW, LT, true>(sw, twl, em);
        else if (nlw > 0)
            wave_fft_em<C, M, true, MAXLW, LT>(sw, twl, em);
        // the next group's rows load while the epilogue runs
        if (g + int(gridDim.x) < GROUPS) fetch(g + gridDim.x);
        __syncthreads();
        if constexpr (MF) {
            mfma_contract<T, N, PREC, LT>(s, reinterpret_cast<const float*>(sd), sgn, nb, acc64, accl);
        } else if constexpr (EPI == EPI_CONTRACT) {
            if (cg < cg_n) {
                float acc[4][4];
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc[a][c] = 0.f;
                for (int cell = cg; cell < CELLS; cell += cg_n) {
                    const int r = cell / N, z = cell - r * N;
                    const float d = float(sd[cell]);
                    float xa[4], xb[4];
#pragma unroll
                    for (int a = 0; a < 4; ++a) {
                        const int b1 = 4 * ti + a, b2 = 4 * tj + a;
                        xa[a] = b1 < nb ? float(sf[at(b1 * R + r, z)]) * d : 0.f;
                        xb[a] = b2 < nb ? float(sf[at(b2 * R + r, z)]) : 0.f;
                    }
#pragma unroll
                    for (int a = 0; a < 4; ++a)
#pragma unroll
                        for (int c = 0; c < 4; ++c) acc[a][c] = fmaf(xa[a], xb[c], acc[a][c]);
                }
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc64[a * 4 + c] += double(acc[a][c]);
            }
        } else {
            if (out) {
                for (int e = threadIdx.x; e < nb * CELLS; e += kThreads) {
                    const int b = e / CELLS, rem = e - b * CELLS;
                    const int r = rem / N, z = rem - r * N;
                    out[int64_t(map.out[b]) * N * N * N + (row0 + r) * N + z] = sf[at(b * R + r, z)];
                }
            }
            if (part && msub < subs) {
                T s2 = 0, s3 = 0, s4 = 0;
                for (int cell = msub; cell < CELLS; cell += subs) {
                    const int r = cell / N, z = cell - r * N;
                    const T v = sf[at(mb * R + r, z)];
                    const T v2 = v * v;
                    s2 += v2;
                    s3 += v2 * v;
                    s4 += v2 * v2;
                }
                acc64[0] += double(s2);
                acc64[1] += double(s3);
                acc64[2] += double(s4);
            }
        }
        __syncthreads();
    }

    // workgroup reduction of the float64 partial sums
    double* red = lds_raw;
    if constexpr (MF) {
        // acc64[r] (H) and accl[r] (L) of lane l in wave w hold entry (i, j),
        // j = l % 32, i = 8 (r / 4) + 4 (l / 32) + r % 4 (32x32 MFMA
        // accumulator layout); C = H + L + L^T
        const int w = threadIdx.x / 64, l = threadIdx.x % 64;
        for (int st = 0; st < 4; ++st) {
            if (w == st) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int i = 8 * (r / 4) + 4 * (l / 32) + (r % 4), j = l % 32;
                    red[i * 32 + j] = (st == 0 ? 0.0 : red[i * 32 + j]) + acc64[r] + double(accl[r]);
                }
            }
            __syncthreads();
            if (w == st) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int i = 8 * (r / 4) + 4 * (l / 32) + (r % 4), j = l % 32;
                    red[j * 32 + i] += double(accl[r]);
                }
            }
            __syncthreads();
        }
        double* dst = part + int64_t(blockIdx.x) * nb * nb;
        for (int e = threadIdx.x; e < nb * nb; e += kThreads) dst[e] = red[(e / nb) * 32 + e % nb];
    } else if constexpr (EPI == EPI_CONTRACT) {
#pragma unroll
        for (int i = 0; i < 16; ++i) red[threadIdx.x * 16 + i] = acc64[i];
        __syncthreads();
        if (threadIdx.x < ntp) {
            double sum[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) sum[i] = 0.0;
            for (int c = 0; c < cg_n; ++c)
#pragma unroll
                for (int i = 0; i < 16; ++i) sum[i] += red[(c * ntp + threadIdx.x) * 16 + i];
            double* dst = part + int64_t(blockIdx.x) * nb * nb;
            for (int a = 0; a < 4; ++a)
                for (int c = 0; c < 4; ++c) {
                    const int b1 = 4 * ti + a, b2 = 4 * tj + c;
                    if (b1 < nb && b2 < nb) {
                        dst[b1 * nb + b2] = sum[a * 4 + c];
                        dst[b2 * nb + b1] = sum[a * 4 + c];
                    }
                }
        }
    } else if (part) {
        for (int i = 0; i < 3; ++i) red[threadIdx.x * 3 + i] = acc64[i];
        __syncthreads();
        if (threadIdx.x < nb) {
            double sum[3] = {0.0, 0.0, 0.0};
            for (int c = 0; c < subs; ++c)
                for (int i = 0; i < 3; ++i) sum[i] += red[(c * nb + threadIdx.x) * 3 + i];
            double* dst = part + (int64_t(blockIdx.x) * nb + threadIdx.x) * 3;
            for (int i = 0; i < 3; ++i) dst[i] = sum[i];
        }
    }
}

// dst[i] (+)= scale * sum_g part[g * n + i]; one workgroup per output element.
__global__ __launch_bounds__(kThreads) void k_reduce_part(const double* __restrict__ part, int ngroups, int n,
                                                          double scale, double* __restrict__ dst, int accumulate) {
    __shared__ double red[kThreads];
    const int i = blockIdx.x;
    double s = 0.0;
    for (int g = threadIdx.x; g < ngroups; g += kThreads) s += part[int64_t(g) * n + i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) dst[i] = (accumulate ? dst[i] : 0.0) + scale * s;
}

// moments[map.out[b]][p] = scale * sum_g part[g][b][p]; one workgroup per (b, p).
__global__ __launch_bounds__(kThreads) void k_reduce_moments(const double* __restrict__ part, int ngroups,
                                                             WinSet map, double scale,
                                                             double* __restrict__ moments) {
    __shared__ double red[kThreads];
    const int i = blockIdx.x;
    double s = 0.0;
    for (int g = threadIdx.x; g < ngroups; g += kThreads) s += part[int64_t(g) * map.n * 3 + i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) moments[map.out[i / 3] * 3 + i % 3] = scale * s;
}

template <typename KernelT>
inline void allow_lds(KernelT kernel, size_t bytes) {
    if (bytes > 65536)
        (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
}

template <int N>
constexpr int z_grid() {
    return (N * N / zrows<N>::R) < kZGroups ? (N * N / zrows<N>::R) : kZGroups;
}

inline int z_grid_rt(int n) {
    const int groups = n * n / (n / 2 >= 256 ? 1 : 256 / (n / 2));
    return groups < kZGroups ? groups : kZGroups;
}

// Persistent grid of a z-pass kernel: the workgroups that are resident at
// once (occupancy query, once per kernel), capped at kZGroups (the partial-sum
// rows the workspaces hold) and at the group count.
template <typename KernelT>
inline int resident_grid(hermes_ctx ctx, KernelT kernel, int threads, size_t lds, int groups) {
    static std::mutex mu;
    static std::map<const void*, int> per_cu;   // workgroups per CU, by kernel
    int v = 0;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = per_cu.find(reinterpret_cast<const void*>(kernel));
        if (it != per_cu.end()) {
            v = it->second;
        } else {
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, reinterpret_cast<const void*>(kernel), threads, lds) !=
                    hipSuccess ||
                v < 1)
                v = 1;
            per_cu[reinterpret_cast<const void*>(kernel)] = v;
        }
    }
    return std::min({v * ctx->cus, kZGroups, groups});
}

template <typename T, int N, int EPI, int NBCAP, int PREC>
static int launch_z(hermes_ctx ctx, const typename cplx_of<T>::type* sp, int64_t bin_stride, int nb, const T* delta,
                    T* out, const WinSet& ws, double* part, const typename cplx_of<T>::type* tw, hipStream_t stream) {
    constexpr int CAP = NBCAP < z_max_batch<T, N>() ? NBCAP : z_max_batch<T, N>();
    const size_t lds = z_lds_bytes<T, N>(CAP);
    allow_lds(k_c2r_z<T, N, EPI, CAP, PREC>, lds);
    const int grid = resident_grid(ctx, k_c2r_z<T, N, EPI, CAP, PREC>, kThreads, lds, N * N / zrows<N>::R);
    hipLaunchKernelGGL((k_c2r_z<T, N, EPI, CAP, PREC>), dim3(grid), dim3(kThreads), lds, stream, sp, bin_stride,
                       nb, delta, out, ws, part, tw);
    return grid;
}

// Pass X over nb windows for one angular factor (m), or for two (m, m2) of
// the same l sharing the radial table, writing spec_ws and spec_ws2.
template <typename T, int N>
static void run_x(hermes_ctx ctx, const void* delta_k, double box_L, const WinSet& ws, int sh, int ell, int m,
                  int m2, bool pair, bool build_table, void* spec_ws, void* spec_ws2, T* rtab, T* ucol,
                  hipStream_t stream) {
    using C = typename cplx_of<T>::type;
    constexpr int PP = pitch_of<N>();
    constexpr int XVEC = win_vec<T>(), XNT = win_threads<T>();
    constexpr int TC = col_cfg<T, N, XVEC, XNT>::TC;
    const C* tw = tw_ptr<T>(ctx->t);
    const int nb = ws.n;
    const int64_t nq = qmax_of(N) + 1;
    const int64_t plane = int64_t(N) * PP;            // columns of one (ky, kz) plane
    const int64_t bin_stride = int64_t(N) * plane_stride<N>();
    if (build_table) {
        LaunchScope ls(ctx, stream, "radial_table");
        hipLaunchKernelGGL((k_radial<T>), dim3((nq + kThreads - 1) / kThreads, nb), dim3(kThreads), 0, stream, rtab, nq,
                           ws, 2.0 * M_PI / box_L, ctx->t.gl);
        hipLaunchKernelGGL((k_radial_cols<T, N>), dim3(col_rows(N), nb), dim3(kThreads), 0, stream, rtab, nq, nb, ucol);
    }
    // scale: angular constant times 1/N^3 (inverse DFT normalisation)
    const double inv = 1.0 / (double(N) * N * N);
    double sre = inv, sim = 0.0;
    if (sh) {
        const double f = 4.0 * M_PI * inv;
        switch (ell & 3) {
            case 0: sre = f; break;
            case 1: sre = 0.0; sim = f; break;
            case 2: sre = -f; break;
            default: sre = 0.0; sim = -f; break;
        }
    }
    C* sp = static_cast<C*>(spec_ws);
    const YlmConst y0 = ylm_const(ell, m);
    bool paired = false;
    if constexpr (std::is_same<T, float>::value) {   // the 3PCF path (float only)
        if (pair) {
            LaunchScope ls(ctx, stream, "inv_x_window2");
            hipLaunchKernelGGL((k_win_x<T, N, XVEC, XNT, 2>), dim3((plane + TC - 1) / TC), dim3(XNT), 0, stream,
                               static_cast<const C*>(delta_k), sh, y0, ylm_const(ell, m2), sre, sim, basis_phi1d(ctx),
                               sp, static_cast<C*>(spec_ws2), bin_stride, nb, ucol, tw);
            paired = true;
        }
    }
    if (!paired) {
        LaunchScope ls(ctx, stream, "inv_x_window");
        hipLaunchKernelGGL((k_win_x<T, N, XVEC, XNT, 1>), dim3((plane + TC - 1) / TC), dim3(XNT), 0, stream,
                           static_cast<const C*>(delta_k), sh, y0, y0, sre, sim, basis_phi1d(ctx), sp, sp, bin_stride,
                           nb, ucol, tw);
    }
}

// Passes Y and Z over the nb windows of one batch spectrum; returns the
// number of z-pass workgroups (rows of partial sums written to part).
template <typename T, int N, int EPI>
static int run_yz(hermes_ctx ctx, const T* delta, const WinSet& ws, void* spec_ws, double* part, T* out,
                  int precision, hipStream_t stream) {
    using C = typename cplx_of<T>::type;
    const C* tw = tw_ptr<T>(ctx->t);
    const int nb = ws.n;
    const int64_t bin_stride = int64_t(N) * plane_stride<N>();
    C* sp = static_cast<C*>(spec_ws);
    {
        LaunchScope ls(ctx, stream, "inv_y");
        using YC = ypack_cfg<T, N>;
        hipLaunchKernelGGL((k_inv_y_pack<T, N>), dim3(YC::TILES, nb * N), dim3(YC::NT), 0, stream, sp,
                           plane_stride<N>(), tw);
    }
    LaunchScope ls(ctx, stream, EPI == EPI_CONTRACT ? "inv_z_contract" : "inv_z_moments");
    if constexpr (EPI == EPI_CONTRACT) {
        // register capacity: 20 bins (the common case) or the full batch
        const bool small = nb <= 20;
        if (precision == HERMES_PREC_BF16X3) {
            if (small) return launch_z<T, N, EPI, 20, HERMES_PREC_BF16X3>(ctx, sp, bin_stride, nb, delta, out, ws, part, tw, stream);
            return launch_z<T, N, EPI, kMaxBatch, HERMES_PREC_BF16X3>(ctx, sp, bin_stride, nb, delta, out, ws, part, tw, stream);
        } else if (precision == HERMES_PREC_FP16X3) {
            if (small) return launch_z<T, N, EPI, 20, HERMES_PREC_FP16X3>(ctx, sp, bin_stride, nb, delta, out, ws, part, tw, stream);
            return launch_z<T, N, EPI, kMaxBatch, HERMES_PREC_FP16X3>(ctx, sp, bin_stride, nb, delta, out, ws, part, tw, stream);
        } else {
            if (small) return launch_z<T, N, EPI, 20, HERMES_PREC_FP32>(ctx, sp, bin_stride, nb, delta, out, ws, part, tw, stream);
            return launch_z<T, N, EPI, kMaxBatch, HERMES_PREC_FP32>(ctx, sp, bin_stride, nb, delta, out, ws, part, tw, stream);
        }
    } else {
        return launch_z<T, N, EPI, kFilterChunk, HERMES_PREC_FP32>(ctx, sp, bin_stride, nb, delta, out, ws, part, tw, stream);
    }
}

// One batch: pass X, Y, Z over nb windows sharing the angular factor.
template <typename T, int N, int EPI>
static int run_batch(hermes_ctx ctx, const void* delta_k, const T* delta, double box_L, const WinSet& ws, int sh,
                     int ell, int m, bool build_table, void* spec_ws, T* rtab, T* ucol, double* part, T* out,
                     int precision, hipStream_t stream) {
    run_x<T, N>(ctx, delta_k, box_L, ws, sh, ell, m, m, false, build_table, spec_ws, spec_ws, rtab, ucol, stream);
    return run_yz<T, N, EPI>(ctx, delta, ws, spec_ws, part, out, precision, stream);
}

// ---------------------------------------------------------------- filter_bins
size_t filter_workspace(int n, int dtype, int n_win) {
    const bool dbl = dtype == HERMES_F64;
    const int chunk = std::min({n_win, kFilterChunk, z_max_batch_rt(n, dbl)});
    const size_t nq = size_t(qmax_of(n) + 1);
    return align256(spec_bytes(n, dbl) * chunk) + align256(nq * chunk * (dbl ? 8 : 4)) +
           align256(col_table_bytes(n, chunk, dbl ? 8 : 4)) + align256(size_t(z_grid_rt(n)) * chunk * 3 * sizeof(double));
}

template <typename T, int N>
static hermes_status filter_n(hermes_ctx ctx, const void* delta_k, double box_L, const hermes_window* win, int n_win,
                              void* out, double* moments, void* work, hipStream_t stream) {
    const bool dbl = sizeof(T) == 8;
    const int chunk = std::min({n_win, kFilterChunk, z_max_batch<T, N>()});
    const size_t nq = size_t(qmax_of(N) + 1);
    char* w = static_cast<char*>(work);
    void* spec = w;
    char* tail = w + align256(spec_bytes(N, dbl) * chunk);
    T* rtab = reinterpret_cast<T*>(tail);
    tail += align256(nq * chunk * sizeof(T));
    T* ucol = reinterpret_cast<T*>(tail);
    tail += align256(col_table_bytes(N, chunk, sizeof(T)));
    double* part = reinterpret_cast<double*>(tail);
    // group windows by angular factor: isotropic ones together, SH ones by (l, m)
    struct Key {
        int sh, ell, m;
    };
    std::vector<int> order(n_win);
    for (int i = 0; i < n_win; ++i) order[i] = i;
    auto key = [&](int i) {
        const hermes_window& x = win[i];
        return x.type == HERMES_WIN_SH_SHELL ? Key{1, x.ell, x.m} : Key{0, 0, 0};
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const Key ka = key(a), kb = key(b);
        if (ka.sh != kb.sh) return ka.sh < kb.sh;
        if (ka.ell != kb.ell) return ka.ell < kb.ell;
        return ka.m < kb.m;
    });
    const double inv_nc = 1.0 / (double(N) * N * N);
    size_t i = 0;
    while (i < order.size()) {
        const Key k0 = key(order[i]);
        WinSet ws{};
        ws.n = 0;
        while (i < order.size() && ws.n < chunk) {
            const Key k = key(order[i]);
            if (k.sh != k0.sh || k.ell != k0.ell || k.m != k0.m) break;
            const hermes_window& x = win[order[i]];
            ws.type[ws.n] = x.type;
            ws.ell[ws.n] = x.ell;
            ws.lo[ws.n] = x.r_lo;
            ws.hi[ws.n] = x.r_hi;
            ws.out[ws.n] = order[i];
            ++ws.n;
            ++i;
        }
        const int grid = run_batch<T, N, EPI_MOMENTS>(ctx, delta_k, nullptr, box_L, ws, k0.sh, k0.ell, k0.m, true,
                                                      spec, rtab, ucol, moments ? part : nullptr,
                                                      static_cast<T*>(out), HERMES_PREC_FP32, stream);
        if (moments) {
            LaunchScope ls(ctx, stream, "reduce");
            hipLaunchKernelGGL(k_reduce_moments, dim3(ws.n * 3), dim3(kThreads), 0, stream, part, grid, ws, inv_nc,
                               moments);
        }
    }
    return check_launch("hermes_filter_bins");
}

hermes_status filter_impl(hermes_ctx ctx, const void* delta_k, int n, int dtype, double box_L,
                          const hermes_window* win, int n_win, void* out, double* moments, void* work, size_t,
                          hipStream_t stream) {
#define HERMES_FILTER_CASE(NN)                                                                                   \
    case NN:                                                                                                     \
        return dtype == HERMES_F32                                                                               \
                   ? filter_n<float, NN>(ctx, delta_k, box_L, win, n_win, out, moments, work, stream)          \
                   : filter_n<double, NN>(ctx, delta_k, box_L, win, n_win, out, moments, work, stream);
    switch (n) {
        HERMES_FILTER_CASE(8)
        HERMES_FILTER_CASE(16)
        HERMES_FILTER_CASE(32)
        HERMES_FILTER_CASE(64)
        HERMES_FILTER_CASE(128)
        HERMES_FILTER_CASE(256)
        HERMES_FILTER_CASE(512)
        HERMES_FILTER_CASE(1024)
        default:
            return fail(HERMES_ERR_ARG, "hermes_filter_bins: unsupported N");
    }
#undef HERMES_FILTER_CASE
}

// ---------------------------------------------------------------- zeta_l
// Two m of one l share a pass X (and its reads of delta^ and the radial
// table) when a second batch spectrum fits: grids up to 512^3.
inline bool zeta_pairs(int n) { return n <= 512; }

size_t zeta_workspace(int n, int n_bins) {
    const size_t nq = size_t(qmax_of(n) + 1);
    return align256(spec_bytes(n, false) * n_bins) * (zeta_pairs(n) ? 2 : 1) + align256(nq * n_bins * sizeof(float)) +
           align256(col_table_bytes(n, n_bins, sizeof(float))) +
           align256(size_t(z_grid_rt(n)) * n_bins * n_bins * sizeof(double));
}

template <int N>
static hermes_status zeta_n(hermes_ctx ctx, const float* delta, const void* delta_k, double box_L,
                            const Edges& edges, int l_max, int precision, double* zeta, void* work,
                            hipStream_t stream) {
    const int nb = edges.n_bins;
    if (nb > z_max_batch<float, N>())
        return fail(HERMES_ERR_UNSUPPORTED, "hermes_zeta_l: too many radial bins for this grid size");
    if (precision != HERMES_PREC_FP32 && nb > 32)
        return fail(HERMES_ERR_UNSUPPORTED, "hermes_zeta_l: the matrix-core contraction takes at most 32 bins");
    const size_t nq = size_t(qmax_of(N) + 1);
    char* w = static_cast<char*>(work);
    const bool pairs = zeta_pairs(N);
    void* spec = w;
    char* tail = w + align256(spec_bytes(N, false) * nb);
    void* spec2 = tail;
    if (pairs) tail += align256(spec_bytes(N, false) * nb);
    float* rtab = reinterpret_cast<float*>(tail);
    tail += align256(nq * nb * sizeof(float));
    float* ucol = reinterpret_cast<float*>(tail);
    tail += align256(col_table_bytes(N, nb, sizeof(float)));
    double* part = reinterpret_cast<double*>(tail);
    const double scale = 1.0 / (4.0 * M_PI * double(N) * N * N);
    {
        LaunchScope ls(ctx, stream, "fill");
        launch_fill<double>(zeta, int64_t(l_max + 1) * nb * nb, 0.0, stream);
    }
    for (int ell = 0; ell <= l_max; ++ell) {
        WinSet ws{};
        ws.n = nb;
        for (int b = 0; b < nb; ++b) {
            ws.type[b] = HERMES_WIN_SH_SHELL;
            ws.ell[b] = ell;
            ws.lo[b] = edges.e[b];
            ws.hi[b] = edges.e[b + 1];
            ws.out[b] = b;
        }
        for (int m = -ell; m <= ell;) {
            const bool pair = pairs && m < ell;   // (m, m + 1) in one pass X
            run_x<float, N>(ctx, delta_k, box_L, ws, 1, ell, m, m + 1, pair, m == -ell, spec, spec2, rtab, ucol,
                            stream);
            for (int k = 0; k < (pair ? 2 : 1); ++k) {
                const int grid =
                    run_yz<float, N, EPI_CONTRACT>(ctx, delta, ws, k ? spec2 : spec, part, nullptr, precision, stream);
                LaunchScope ls(ctx, stream, "reduce");
                hipLaunchKernelGGL(k_reduce_part, dim3(nb * nb), dim3(kThreads), 0, stream, part, grid, nb * nb,
                                   scale, zeta + int64_t(ell) * nb * nb, 1);
            }
            m += pair ? 2 : 1;
        }
    }
    return check_launch("hermes_zeta_l");
}

hermes_status zeta_impl(hermes_ctx ctx, const float* delta, const void* delta_k, int n, double box_L,
                        const Edges& edges, int l_max, int precision, double* zeta, void* work, size_t,
                        hipStream_t stream) {
#define HERMES_ZETA_CASE(NN) \
    case NN:                 \
        return zeta_n<NN>(ctx, delta, delta_k, box_L, edges, l_max, precision, zeta, work, stream);
    switch (n) {
        HERMES_ZETA_CASE(8)
        HERMES_ZETA_CASE(16)
        HERMES_ZETA_CASE(32)
        HERMES_ZETA_CASE(64)
        HERMES_ZETA_CASE(128)
        HERMES_ZETA_CASE(256)
        HERMES_ZETA_CASE(512)
        HERMES_ZETA_CASE(1024)
        default:
            return fail(HERMES_ERR_ARG, "hermes_zeta_l: unsupported N");
    }
#undef HERMES_ZETA_CASE
}

}  // namespace hermes
