// Anisotropic 2PCF with axisymmetric windows (Sec. 2.2.3, redshift space:
// thin ring, finite-width ring, Gaussian-blurred ring; Table A1 (d), (f)-(i):
// Gaussian shell, cylinder, cylindrical shell, disk, ring):
//
//   xi_W = N^-6 sum_n |delta^_n|^2 Phi^(n) W^(k_par, k_perp)
//
// (Sec. 3.3.1 Parseval form of the field-window product).  Every window is
// even in each component and depends on a mode only through the integers
// n_par = |n~_los| and q = |n~_perp|^2, so the sum is regrouped exactly:
//
//   H(q, n_par) = sum over modes with those integers of |delta^|^2 Phi^,
//   xi_W = N^-6 sum_{n_par} A_W(k_par) sum_q B_W(k_perp(q)) H(q, n_par)
//
// for windows that factor into a line-of-sight part A and a transverse part
// B (rings, disk, cylinder, cylindrical shell), and with W evaluated per
// (q, n_par) for the Gaussian shell, which depends on |k| only.  q runs over
// the sums of two squares (a compact rank), so no row of H is empty by
// construction.
//
// Pass 1 reads the half spectrum once and scatters H with float64 atomics (one
// per four sign-related modes).  Pass 2 is a float64 product of H with the
// transverse factors: a table of B_w(k_perp(q)) (Bessel functions in float64)
// is written for a batch of 64-window tiles, then a workgroup takes one tile
// (lane = window) and a range of q, stages the chunk's factors in LDS, and
// each of its 16 wavefronts accumulates its own rows n_par, reading H rows as
// wavefront-uniform values.  The line-of-sight factor is applied once per row
// at the end and the wavefronts' shares are summed in LDS.  Pass 3 sums the
// workgroups' partial results per window in a fixed order.
#include <cmath>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

namespace hermes {

struct AnisoWin {
    int kind;     // hermes_aniso_kind, or -1 for padding
    int slot;     // index of the window in the caller's list
    double rp, rl, dp, dl;
};

constexpr int kAnisoQC = 64;         // q values per chunk (transverse factors staged in LDS)
constexpr int kAnisoBlocks = 2048;   // workgroups aimed for per launch of pass 2
constexpr int kAnisoThreads = 1024;   // pass-2b workgroup: 16 wavefronts share one staged chunk
constexpr int kAnisoWaves = kAnisoThreads / 64;
constexpr size_t kAnisoTableBytes = size_t(256) << 20;   // transverse factors of one batch of tiles

static_assert(kAnisoQC >= kAnisoWaves, "the chunk tile also holds the wavefronts' partial sums");

template <int N> struct aniso_cfg {
    static constexpr int ROWS = N / 2 + 1;                                           // n_par = 0..N/2
    static constexpr int ZS = ROWS > kAnisoWaves * 17 ? 2 : 1;                       // row splits over blockIdx.z
    static constexpr int RPW = (ROWS + kAnisoWaves * ZS - 1) / (kAnisoWaves * ZS);   // rows per wavefront
};

inline int aniso_zs_rt(int n) { return n / 2 + 1 > kAnisoWaves * 17 ? 2 : 1; }

// H is read up to ZS 16 RPW - (N/2 + 1) < 32 values past its last row.
constexpr int64_t kAnisoHPad = 64;

static int aniso_tiles_max(int n_win) { return (n_win + 63) / 64 + 1; }

// Workspace layout and launch shape of one call, a function of (N, n_win)
// only (no split into separable and Gaussian-shell tiles needs more): H
// [nq][N/2+1] (+ padding), the padded window list, the partial sums
// [slots][padded windows] and the transverse-factor table of a batch of tb
// tiles.  Every launch uses gy q-range slices, so every window has ZS gy
// partial sums (one per workgroup).
struct AnisoPlan {
    int64_t nq;
    int tiles_max, tb, gy;
    size_t h_bytes, w_bytes, p_bytes, t_bytes;
};

static AnisoPlan aniso_plan(hermes_ctx ctx, int n, int n_win) {
    AnisoPlan p{};
    p.nq = ctx->nq2[ilog2(n)];
    p.tiles_max = aniso_tiles_max(n_win);
    const int64_t per_tile = p.nq * 64 * int64_t(sizeof(double));
    int64_t tb = int64_t(kAnisoTableBytes) / per_tile;
    tb = tb < 1 ? 1 : (tb > p.tiles_max ? p.tiles_max : tb);
    p.tb = int(tb);
    const int nchunks = int((p.nq + kAnisoQC - 1) / kAnisoQC);
    int gy = kAnisoBlocks / p.tb;
    gy = gy < 1 ? 1 : (gy > nchunks ? nchunks : gy);
    p.gy = gy;
    const int zs = aniso_zs_rt(n);
    p.h_bytes = align256(size_t(p.nq * (n / 2 + 1) + kAnisoHPad) * sizeof(double));
    p.w_bytes = align256(size_t(p.tiles_max) * 64 * sizeof(AnisoWin));
    p.p_bytes = align256(size_t(zs) * gy * size_t(p.tiles_max) * 64 * sizeof(double));
    p.t_bytes = align256(size_t(p.tb) * size_t(per_tile));
    return p;
}

size_t aniso_workspace(hermes_ctx ctx, int n, int n_win) {
    const AnisoPlan p = aniso_plan(ctx, n, n_win);
    return p.h_bytes + p.w_bytes + p.p_bytes + p.t_bytes;
}

// One thread per representative (|kx|, |ky|, kz), kx, ky in [0, N/2]; the
// modes (+-kx, +-ky, kz) share n_par and q.
template <typename T, int N>
__global__ __launch_bounds__(kThreads) void k_aniso_hist(const typename cplx_of<T>::type* __restrict__ dk, int los,
                                                         const double* __restrict__ phi1d,
                                                         const int* __restrict__ q2rank, double* __restrict__ H) {
    constexpr int M = N / 2, P = M + 1;
    const int64_t total = int64_t(P) * P * P;
    const int64_t t = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (t >= total) return;
    const int kz = int(t % P);
    const int iy = int((t / P) % P);
    const int ix = int(t / (int64_t(P) * P));
    if (ix == 0 && iy == 0 && kz == 0) return;   // delta^(0) = 0
    const int xs[2] = {ix, (N - ix) & (N - 1)};
    const int ys[2] = {iy, (N - iy) & (N - 1)};
    const int nx = (ix == 0 || ix == M) ? 1 : 2;
    const int ny = (iy == 0 || iy == M) ? 1 : 2;
    double p = 0.0;
    for (int a = 0; a < nx; ++a)
        for (int b = 0; b < ny; ++b) {
            const auto v = dk[(int64_t(xs[a]) * N + ys[b]) * P + kz];
            p += double(v.x) * v.x + double(v.y) * v.y;
        }
    const double herm = (kz == 0 || kz == M) ? 1.0 : 2.0;
    p *= herm * phi1d[N + ix] * phi1d[N + iy] * phi1d[N + kz];
    const int npar = los == 0 ? ix : (los == 1 ? iy : kz);
    const int qperp = ix * ix + iy * iy + kz * kz - npar * npar;
    unsafeAtomicAdd(H + int64_t(q2rank[qperp]) * P + npar, p);
}

__device__ __forceinline__ double sinc_d(double x) {
    if (fabs(x) < 1e-4) return 1.0 - x * x / 6.0;
    return sin(x) / x;
}

// 2 J1(x) / x
__device__ __forceinline__ double jinc_d(double x) {
    if (fabs(x) < 1e-4) return 1.0 - x * x / 8.0;
    return 2.0 * j1(x) / x;
}

// Transverse factor B_W(k_perp).
__device__ __forceinline__ double aniso_perp(const AnisoWin& w, double kp) {
    switch (w.kind) {
        case HERMES_ANISO_RING:
        case HERMES_ANISO_CYLSHELL:
            return j0(kp * w.rp);
        case HERMES_ANISO_GAUSS_RING: {
            const double g = kp * w.dp;
            return j0(kp * w.rp) * exp(-0.5 * g * g);
        }
        case HERMES_ANISO_DISK:
        case HERMES_ANISO_CYLINDER:
            return jinc_d(kp * w.rp);
        case HERMES_ANISO_RING_BIN: {
            // (1 / (R dR)) int_{R - dR/2}^{R + dR/2} J0(k rho) rho d rho, with
            // int J0(k rho) rho d rho = rho J1(k rho) / k
            if (kp == 0.0) return 1.0;
            const double a = w.rp - 0.5 * w.dp, b = w.rp + 0.5 * w.dp;
            return (b * j1(kp * b) - a * j1(kp * a)) / (kp * w.rp * w.dp);
        }
        default:
            return 0.0;
    }
}

// Line-of-sight factor A_W(k_par).
__device__ __forceinline__ double aniso_par(const AnisoWin& w, double kl) {
    switch (w.kind) {
        case HERMES_ANISO_RING:
        case HERMES_ANISO_GAUSS_RING:
        case HERMES_ANISO_DISK:
            return cos(kl * w.rl);
        case HERMES_ANISO_RING_BIN:
            return sinc_d(0.5 * kl * w.dl) * cos(kl * w.rl);
        case HERMES_ANISO_CYLINDER:
        case HERMES_ANISO_CYLSHELL:
            return sinc_d(kl * w.rl);
        default:
            return 0.0;
    }
}

// Gaussian shell (Table A1 (d)), Rs = rp, Rg = dp, as a function of |k|.
__device__ __forceinline__ double aniso_gauss_shell(const AnisoWin& w, double k) {
    const double rs = w.rp, rg = w.dp;
    const double x = k * rs;
    return (rg * rg * cos(x) + rs * rs * sinc_d(x)) / (rs * rs + rg * rg) * exp(-0.5 * k * k * rg * rg);
}

// Pass 2a.  Transverse factors of a batch of separable tiles,
// T[tile][q][lane] = B_w(k_perp(q)) for window w = 64 tile + lane, one thread
// per entry (the Bessel functions stay out of the accumulating kernel).
__global__ __launch_bounds__(kThreads) void k_aniso_perp(const AnisoWin* __restrict__ win,
                                                         const int* __restrict__ rank2q, int nq, double kfac,
                                                         double* __restrict__ T) {
    const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (i >= int64_t(nq) * 64) return;
    const int q = int(i / 64), lane = int(i % 64);
    const AnisoWin w = win[blockIdx.y * 64 + lane];
    T[int64_t(blockIdx.y) * nq * 64 + i] = aniso_perp(w, kfac * sqrt(double(rank2q[q])));
}

// Pass 2b.  Grid (tiles of this launch, q-range slices, row splits); the
// wavefront (blockIdx.z, w) holds rows [RPW (16 z + w), + RPW) of every q of
// its slices.  Separable tiles (GEN false) stage the chunk's transverse
// factors from T in LDS; Gaussian-shell tiles (GEN true) evaluate the window
// per (q, n_par).  Padding windows contribute zero.
template <int N, bool GEN>
__global__ __launch_bounds__(kAnisoThreads) void k_aniso_sum(const double* __restrict__ H, const int* __restrict__ rank2q,
                                                        int nq, const AnisoWin* __restrict__ win,
                                                        const double* __restrict__ T, int tile0, int n_pad,
                                                        double kfac, double* __restrict__ part) {
    using G = aniso_cfg<N>;
    constexpr int ROWS = G::ROWS, RPW = G::RPW;
    __shared__ double F[kAnisoQC][64];
    const int wv = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int wslot = __builtin_amdgcn_readfirstlane(int(blockIdx.z) * kAnisoWaves + wv);
    const int row0 = wslot * RPW;
    const int nrows = ROWS - row0 < RPW ? ROWS - row0 : RPW;   // <= 0: no rows (still stages factors)
    const int tile = tile0 + int(blockIdx.x);
    const AnisoWin w = win[tile * 64 + lane];
    double acc[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) acc[r] = 0.0;
    const int nchunks = (nq + kAnisoQC - 1) / kAnisoQC;
    for (int c = blockIdx.y; c < nchunks; c += gridDim.y) {
        const int q0 = c * kAnisoQC;
        const int qn = nq - q0 < kAnisoQC ? nq - q0 : kAnisoQC;
        if constexpr (!GEN) {
            const double* src = T + (int64_t(blockIdx.x) * nq + q0) * 64;
            for (int e = threadIdx.x; e < qn * 64; e += kAnisoThreads) F[e / 64][e % 64] = src[e];
            __syncthreads();
            if (nrows > 0) {
                for (int i = 0; i < qn; ++i) {
                    const double f = F[i][lane];
                    // rows past the last one read the next q's row or the zero
                    // padding; those accumulators are never used
                    const double* h = H + int64_t(q0 + i) * ROWS + row0;
#pragma unroll
                    for (int r = 0; r < RPW; ++r) acc[r] = fma(h[r], f, acc[r]);
                }
            }
            __syncthreads();
        } else if (nrows > 0) {
#pragma unroll 1
            for (int i = 0; i < qn; ++i) {
                const double kp2 = kfac * kfac * double(rank2q[q0 + i]);
                const double* h = H + int64_t(q0 + i) * ROWS + row0;
#pragma unroll
                for (int r = 0; r < RPW; ++r) {
                    if (r < nrows) {
                        const double kl = kfac * double(row0 + r);
                        acc[r] = fma(h[r], w.kind < 0 ? 0.0 : aniso_gauss_shell(w, sqrt(kl * kl + kp2)), acc[r]);
                    }
                }
            }
        }
    }
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < RPW; ++r)
        if (r < nrows) s += (GEN ? 1.0 : aniso_par(w, kfac * double(row0 + r))) * acc[r];
    // the wavefronts' rows, summed in a fixed order: one partial per workgroup
    __syncthreads();
    F[wv][lane] = s;
    __syncthreads();
    if (wv == 0) {
        double t = 0.0;
        for (int k = 0; k < kAnisoWaves; ++k) t += F[k][lane];
        const int64_t slot = int64_t(blockIdx.z) * gridDim.y + blockIdx.y;
        part[slot * n_pad + tile * 64 + lane] = t;
    }
}

__global__ void k_aniso_final(const double* __restrict__ part, int n_slots, int n_pad,
                              const AnisoWin* __restrict__ win, double scale, double* __restrict__ xi) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_pad || win[i].kind < 0) return;
    double s = 0.0;
    for (int k = 0; k < n_slots; ++k) s += part[int64_t(k) * n_pad + i];
    xi[win[i].slot] = s * scale;
}

template <typename T, int N>
static hermes_status aniso_n(hermes_ctx ctx, const void* delta_k, double box_L, const std::vector<AnisoWin>& wins,
                             int sep_tiles, int n_win, int los, double* xi, void* work, hipStream_t stream) {
    using C = typename cplx_of<T>::type;
    using G = aniso_cfg<N>;
    constexpr int P = N / 2 + 1;
    const AnisoPlan pl = aniso_plan(ctx, N, n_win);
    const int nq = int(pl.nq);
    const int tiles = int(wins.size() / 64);
    const int n_pad = tiles * 64;
    const int n_slots = G::ZS * pl.gy;
    char* base = static_cast<char*>(work);
    double* H = reinterpret_cast<double*>(base);
    AnisoWin* dwin = reinterpret_cast<AnisoWin*>(base + pl.h_bytes);
    double* part = reinterpret_cast<double*>(base + pl.h_bytes + pl.w_bytes);
    double* tab = reinterpret_cast<double*>(base + pl.h_bytes + pl.w_bytes + pl.p_bytes);
    const double kfac = 2.0 * M_PI / box_L;
    if (hipMemcpyAsync(dwin, wins.data(), size_t(n_pad) * sizeof(AnisoWin), hipMemcpyHostToDevice, stream) !=
        hipSuccess)
        return check_launch("hermes_xi_aniso: window upload");
    {
        LaunchScope ls(ctx, stream, "fill");
        launch_fill<double>(H, int64_t(nq) * P + kAnisoHPad, 0.0, stream);
    }
    const int64_t reps = int64_t(P) * P * P;
    {
        LaunchScope ls(ctx, stream, "aniso_hist");
        hipLaunchKernelGGL((k_aniso_hist<T, N>), dim3((reps + kThreads - 1) / kThreads), dim3(kThreads), 0, stream,
                           static_cast<const C*>(delta_k), los, basis_phi1d(ctx), ctx->t.q2rank, H);
    }
    for (int t0 = 0; t0 < sep_tiles; t0 += pl.tb) {
        const int nb = sep_tiles - t0 < pl.tb ? sep_tiles - t0 : pl.tb;
        {
            LaunchScope ls(ctx, stream, "aniso_perp");
            hipLaunchKernelGGL(k_aniso_perp, dim3(int((int64_t(nq) * 64 + kThreads - 1) / kThreads), nb),
                               dim3(kThreads), 0, stream, dwin + int64_t(t0) * 64, ctx->t.rank2q, nq, kfac, tab);
        }
        LaunchScope ls(ctx, stream, "aniso_sum");
        hipLaunchKernelGGL((k_aniso_sum<N, false>), dim3(nb, pl.gy, G::ZS), dim3(kAnisoThreads), 0, stream, H,
                           ctx->t.rank2q, nq, dwin, tab, t0, n_pad, kfac, part);
    }
    if (tiles > sep_tiles) {
        LaunchScope ls(ctx, stream, "aniso_sum");
        hipLaunchKernelGGL((k_aniso_sum<N, true>), dim3(tiles - sep_tiles, pl.gy, G::ZS), dim3(kAnisoThreads), 0, stream,
                           H, ctx->t.rank2q, nq, dwin, tab, sep_tiles, n_pad, kfac, part);
    }
    {
        const double nc = double(N) * N * N;
        LaunchScope ls(ctx, stream, "reduce");
        hipLaunchKernelGGL(k_aniso_final, dim3((n_pad + 127) / 128), dim3(128), 0, stream, part, n_slots, n_pad, dwin,
                           1.0 / (nc * nc), xi);
    }
    return check_launch("hermes_xi_aniso");
}

hermes_status xi_aniso_impl(hermes_ctx ctx, const void* delta_k, int n, int dtype, double box_L,
                            const hermes_aniso_window* win, int n_win, int los_axis, double* xi, void* work,
                            hipStream_t stream) {
    // separable windows first (grouped by kind, so that most tiles hold one
    // kind), then Gaussian shells, each group padded to whole tiles of 64
    std::vector<AnisoWin> wins;
    wins.reserve(size_t(aniso_tiles_max(n_win)) * 64);
    int sep_tiles = 0;
    for (int pass = 0; pass < 2; ++pass) {
        const size_t start = wins.size();
        for (int kind = HERMES_ANISO_RING; kind <= HERMES_ANISO_GAUSS_SHELL; ++kind) {
            if ((kind == HERMES_ANISO_GAUSS_SHELL) != (pass == 1)) continue;
            for (int i = 0; i < n_win; ++i)
                if (win[i].kind == kind)
                    wins.push_back(AnisoWin{kind, i, win[i].r_perp, win[i].r_par, win[i].d_perp, win[i].d_par});
        }
        if (wins.size() > start)
            while (wins.size() % 64) wins.push_back(AnisoWin{-1, 0, 0.0, 0.0, 0.0, 0.0});
        if (pass == 0) sep_tiles = int(wins.size() / 64);
    }
#define HERMES_ANISO_CASE(NN)                                                                                   \
    case NN:                                                                                                    \
        return dtype == HERMES_F32                                                                              \
                   ? aniso_n<float, NN>(ctx, delta_k, box_L, wins, sep_tiles, n_win, los_axis, xi, work, stream) \
                   : aniso_n<double, NN>(ctx, delta_k, box_L, wins, sep_tiles, n_win, los_axis, xi, work, stream);
    switch (n) {
        HERMES_ANISO_CASE(8)
        HERMES_ANISO_CASE(16)
        HERMES_ANISO_CASE(32)
        HERMES_ANISO_CASE(64)
        HERMES_ANISO_CASE(128)
        HERMES_ANISO_CASE(256)
        HERMES_ANISO_CASE(512)
        HERMES_ANISO_CASE(1024)
        default:
            return fail(HERMES_ERR_ARG, "hermes_xi_aniso: unsupported N");
    }
#undef HERMES_ANISO_CASE
}

}  // namespace hermes
