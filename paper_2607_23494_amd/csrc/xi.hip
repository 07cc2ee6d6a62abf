// 2PCF and its Legendre multipoles by Parseval (Sec. 3.3.1 Eq.
// pair-counting-kspace; Sec. 3.3.3 DD_l).
//
// The radial window depends on a mode only through the integer
// q = |n~|^2, so the sum over modes is regrouped exactly as
//   xi_l[b] = N^-6 (2l+1) (-1)^{l/2} sum_q R_lb(q) H_l(q),
//   H_l(q)  = sum_{|n~|^2 = q} |delta^_n|^2 Phi^(n) L_l(mu_n).
// Pass 1 reads the half spectrum once and scatters H with float64 atomics
// (one atomic per four sign-related modes); pass 2 evaluates R_lb(q) in
// float64 (thick shell in closed form for l = 0, bin-averaged j_l by
// quadrature for l > 0) and reduces.
//
// Optionally the same passes give the shot-noise factor of each bin,
//   S_lb = N^-3 sum_n K_lb(n) B~(n),  K_lb(n) = (2l+1) (-1)^{l/2} R_lb(q) L_l(mu) Phi^(n),
// B~(n) = prod_a sum_{|d|<=3} B7(d) e^{2 pi i n_a d / N} (the B3 autocorrelation
// at integer lags; 1 for the orthonormal D4 basis), i.e. the kernel summed
// against the self-pair term of the assigned field: for iid points
// E xi_lb = (sum w^2 / W^2) (N^3 S_lb - K_lb(0)).
// Its histogram Hs includes the mode n = 0.
#include "common.hpp"
#include "fft_core.hpp"
#include "kernels.hpp"
#include "special.hpp"

namespace hermes {

struct EllSet {
    int l[HERMES_MAX_ELLS];
    int n;
};

constexpr int kXiSplit = 64;   // q-range chunks per (l, bin) in pass 2

// Scratch of hermes_xi_static: one copy per device, resolved to a device
// address once per context (hermes_create, with the context's device
// current).  Host code uses only that address, never the array's name.
static __device__ __align__(256) unsigned char scratch[kXiStaticBytes];

hermes_status xi_static_init(hermes_ctx ctx) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(HERMES_ERR_HIP, std::string("hermes_create: static scratch: ") + hipGetErrorString(e));
    ctx->xi_scratch = ptr;
    return HERMES_OK;
}

// H and Hs [n_ells][nq], then the pass-2 partials of xi and of S.
size_t xi_workspace(int n, int n_ells, int n_bins) {
    const size_t nq = size_t(qmax_of(n) + 1);
    return 2 * align256(nq * n_ells * sizeof(double)) +
           2 * align256(size_t(n_ells) * n_bins * kXiSplit * sizeof(double));
}

// One thread per representative (|kx|, |ky|, kz), kx, ky in [0, N/2]; the
// modes (+-kx, +-ky, kz) share q and |mu| and are summed before the atomic.
// With swap (line of sight z, or only l = 0), (|ky|, |kx|, kz) shares them
// too (phi^ is the same function per axis): the thread with |kx| <= |ky|
// adds both, the other one does nothing, and half the atomics remain.
template <typename T, int N>
__global__ __launch_bounds__(kThreads) void k_xi_hist(const typename cplx_of<T>::type* __restrict__ dk,
                                                      EllSet ells, int los, const double* __restrict__ phi1d,
                                                      const double* __restrict__ b7dft, double* __restrict__ H,
                                                      double* __restrict__ Hs, int64_t nq, bool swap) {
    constexpr int M = N / 2, P = M + 1;
    const int64_t total = int64_t(P) * P * P;
    const int64_t t = int64_t(blockIdx.x) * kThreads + threadIdx.x;
    if (t >= total) return;
    const int kz = int(t % P);
    const int iy = int((t / P) % P);
    const int ix = int(t / (int64_t(P) * P));
    if (swap && ix > iy) return;   // added by the thread of (iy, ix)
    const int xs[2] = {ix, (N - ix) & (N - 1)};
    const int ys[2] = {iy, (N - iy) & (N - 1)};
    const int nx = (ix == 0 || ix == M) ? 1 : 2;
    const int ny = (iy == 0 || iy == M) ? 1 : 2;
    const int pairs = swap && ix != iy ? 2 : 1;   // (ix, iy) and, swapped, (iy, ix)
    double p = 0.0;
    for (int a = 0; a < nx; ++a)
        for (int b = 0; b < ny; ++b) {
            const auto v = dk[(int64_t(xs[a]) * N + ys[b]) * P + kz];
            p += double(v.x) * v.x + double(v.y) * v.y;
            if (pairs == 2) {
                const auto w = dk[(int64_t(ys[b]) * N + xs[a]) * P + kz];
                p += double(w.x) * w.x + double(w.y) * w.y;
            }
        }
    const int64_t q = int64_t(ix) * ix + int64_t(iy) * iy + int64_t(kz) * kz;
    const double herm = (kz == 0 || kz == M) ? 1.0 : 2.0;
    const double ph = herm * phi1d[N + ix] * phi1d[N + iy] * phi1d[N + kz];
    const int comp = los == 0 ? ix : (los == 1 ? iy : kz);
    const double mu = q == 0 ? 0.0 : double(comp) / sqrt(double(q));
    if (Hs) {
        // B~ is even in every component: the nx ny sign-related modes share it
        const double ps = double(nx * ny * pairs) * ph * b7dft[N + ix] * b7dft[N + iy] * b7dft[N + kz];
        for (int i = 0; i < ells.n; ++i) unsafeAtomicAdd(Hs + int64_t(i) * nq + q, ps * legendre(ells.l[i], mu));
    }
    if (q == 0) return;
    p *= ph;
    for (int i = 0; i < ells.n; ++i) unsafeAtomicAdd(H + int64_t(i) * nq + q, p * legendre(ells.l[i], mu));
}

// sum_q h(q) R_lb(q) over one q chunk for xi (H) and, when Hs is given, S (Hs)
__global__ __launch_bounds__(kThreads) void k_xi_sum(const double* __restrict__ H, const double* __restrict__ Hs,
                                                     int64_t nq, EllSet ells, Edges edges, double kfac,
                                                     const double* __restrict__ gl, double* __restrict__ part,
                                                     double* __restrict__ part_s) {
    __shared__ double red[kThreads];
    const int b = blockIdx.x, il = blockIdx.y, sp = blockIdx.z;
    const int ell = ells.l[il];
    const double lo = edges.e[b], hi = edges.e[b + 1];
    const int64_t chunk = (nq + kXiSplit - 1) / kXiSplit;
    const int64_t q0 = sp * chunk, q1 = min(nq, q0 + chunk);
    double acc = 0.0, acc_s = 0.0;
    for (int64_t q = q0 + threadIdx.x; q < q1; q += kThreads) {
        const double h = H[int64_t(il) * nq + q];
        const double hs = Hs ? Hs[int64_t(il) * nq + q] : 0.0;
        if (h == 0.0 && hs == 0.0) continue;
        const double k = kfac * sqrt(double(q));
        const double r = ell == 0 ? w_shell(k, lo, hi) : jbar(ell, k, lo, hi, gl);
        acc += h * r;
        acc_s += hs * r;
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) part[(int64_t(il) * gridDim.x + b) * kXiSplit + sp] = s;
    if (Hs) {
        const double ss = block_sum(acc_s, red);
        if (threadIdx.x == 0) part_s[(int64_t(il) * gridDim.x + b) * kXiSplit + sp] = ss;
    }
}

__global__ void k_xi_final(const double* __restrict__ part, const double* __restrict__ part_s, EllSet ells,
                           int n_bins, double inv_nc, double* __restrict__ xi, double* __restrict__ shot) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ells.n * n_bins) return;
    const int il = i / n_bins;
    const int ell = ells.l[il];
    const double pref = (2 * ell + 1) * (((ell / 2) & 1) ? -1.0 : 1.0);
    double s = 0.0;
    for (int sp = 0; sp < kXiSplit; ++sp) s += part[int64_t(i) * kXiSplit + sp];
    xi[i] = pref * s * inv_nc * inv_nc;
    if (shot) {
        double ss = 0.0;
        for (int sp = 0; sp < kXiSplit; ++sp) ss += part_s[int64_t(i) * kXiSplit + sp];
        shot[i] = pref * ss * inv_nc;
    }
}

// out[b] = (1 + xi_m[b]) / (1 + xi[b]): the marked correlation function
// normalised by the unmarked pair counts (Sec. 4.3.2).
__global__ void k_mark_ratio(const double* __restrict__ xim, const double* __restrict__ xi, int n,
                             double* __restrict__ out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < n) out[b] = (1.0 + xim[b]) / (1.0 + xi[b]);
}

hermes_status mark_ratio_impl(const double* xim, const double* xi, int n, double* out, hipStream_t stream) {
    if (n > 0) hipLaunchKernelGGL(k_mark_ratio, dim3((n + 255) / 256), dim3(256), 0, stream, xim, xi, n, out);
    return check_launch("hermes_mark_ratio");
}

template <typename T, int N>
static hermes_status xi_n(hermes_ctx ctx, const void* delta_k, double box_L, const Edges& edges, const EllSet& ells,
                          int los, double* xi, double* shot, void* work, hipStream_t stream) {
    using C = typename cplx_of<T>::type;
    constexpr int P = N / 2 + 1;
    const int64_t nq = qmax_of(N) + 1;
    const size_t hbytes = align256(nq * ells.n * sizeof(double));
    const size_t pbytes = align256(size_t(ells.n) * edges.n_bins * kXiSplit * sizeof(double));
    char* w = static_cast<char*>(work);
    double* H = reinterpret_cast<double*>(w);
    double* Hs = shot ? reinterpret_cast<double*>(w + hbytes) : nullptr;
    double* part = reinterpret_cast<double*>(w + 2 * hbytes);
    double* part_s = reinterpret_cast<double*>(w + 2 * hbytes + pbytes);
    {
        LaunchScope ls(ctx, stream, "fill");
        launch_fill<double>(H, nq * ells.n, 0.0, stream);
        if (Hs) launch_fill<double>(Hs, nq * ells.n, 0.0, stream);
    }
    const int64_t reps = int64_t(P) * P * P;
    {
        LaunchScope ls(ctx, stream, "xi_hist");
        bool swap = los == 2;   // mu = kz / |k| does not change under kx <-> ky
        if (!swap) {
            swap = true;        // nor does P_0(mu) = 1
            for (int i = 0; i < ells.n; ++i) swap = swap && ells.l[i] == 0;
        }
        hipLaunchKernelGGL((k_xi_hist<T, N>), dim3((reps + kThreads - 1) / kThreads), dim3(kThreads), 0, stream,
                           static_cast<const C*>(delta_k), ells, los, basis_phi1d(ctx), basis_selfdft(ctx), H, Hs, nq,
                           swap);
    }
    {
        LaunchScope ls(ctx, stream, "xi_sum");
        hipLaunchKernelGGL(k_xi_sum, dim3(edges.n_bins, ells.n, kXiSplit), dim3(kThreads), 0, stream, H, Hs, nq,
                           ells, edges, 2.0 * M_PI / box_L, ctx->t.gl, part, part_s);
    }
    const int n_out = ells.n * edges.n_bins;
    const double nc = double(N) * N * N;
    {
        LaunchScope ls(ctx, stream, "reduce");
        hipLaunchKernelGGL(k_xi_final, dim3((n_out + 127) / 128), dim3(128), 0, stream, part, part_s, ells,
                           edges.n_bins, 1.0 / nc, xi, shot);
    }
    return check_launch("hermes_xi");
}

hermes_status xi_impl(hermes_ctx ctx, const void* delta_k, int n, int dtype, double box_L, const Edges& edges,
                      const int* ell_list, int n_ells, int los_axis, double* xi, double* shot, void* work,
                      size_t, hipStream_t stream) {
    EllSet ells{};
    ells.n = n_ells;
    for (int i = 0; i < n_ells; ++i) ells.l[i] = ell_list[i];
#define HERMES_XI_CASE(NN)                                                                                 \
    case NN:                                                                                               \
        return dtype == HERMES_F32                                                                         \
                   ? xi_n<float, NN>(ctx, delta_k, box_L, edges, ells, los_axis, xi, shot, work, stream)         \
                   : xi_n<double, NN>(ctx, delta_k, box_L, edges, ells, los_axis, xi, shot, work, stream);
    switch (n) {
        HERMES_XI_CASE(8)
        HERMES_XI_CASE(16)
        HERMES_XI_CASE(32)
        HERMES_XI_CASE(64)
        HERMES_XI_CASE(128)
        HERMES_XI_CASE(256)
        HERMES_XI_CASE(512)
        HERMES_XI_CASE(1024)
        default:
            return fail(HERMES_ERR_ARG, "hermes_xi: unsupported N");
    }
#undef HERMES_XI_CASE
}

}  // namespace hermes
