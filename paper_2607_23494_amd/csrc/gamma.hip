// 3PCF monopole through triple connection coefficients (Sec. 3.3.2, Eqs.
// 3PCF-ddd-monopole, con-coeff, DDD-vector-product):
//
//   out[b1][b2] = N^-3 sum_l e_l sum_{a,b} Gamma_{a,b} f_b1[l + a] f_b2[l + b],
//   Gamma_{a,b} = int phi(x) phi(x - a) phi(x - b) d^3x,
//
// with the cubic B-spline as phi.  The stencil sum is the integral over the
// box of the product of the three B3 expansions e(x) f_b1(x) f_b2(x) (cell
// units).  On one unit cell each expansion is a polynomial of degree 3 per
// axis, so the product is integrated exactly by 5-point Gauss-Legendre per
// axis; the expansions are evaluated at the 125 points of a cell by sum
// factorisation (4 nodes -> 5 points, one axis at a time) instead of
// contracting the 7^6 offsets of Gamma.
//
// A workgroup takes bricks of 1 x 1 x CZ cells: per field it stages the
// 4 x 4 x (CZ + 3) coefficients in LDS, evaluates the brick's 125 CZ points
// in three passes, and keeps the point values of e (times the quadrature
// weight) and of every f_b in LDS; then each thread takes bin pairs
// (b1 <= b2) and sums e w f_b1 f_b2 over the brick's points.  Per-brick sums
// are float T, sums across bricks float64; the workgroups' partials are added
// in a fixed order.
#include <cmath>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

namespace hermes {

constexpr int kGammaCZ = 4;                        // cells per brick along z
constexpr int kGammaS = 125 * kGammaCZ;            // quadrature points per brick
constexpr int kGammaZS = 5 * kGammaCZ;             // points along z per brick
constexpr int kGammaRZ = kGammaCZ + 3;             // coefficient nodes along z per brick
constexpr int kGammaMaxFields = 32;               // bins per call
constexpr int kGammaMaxPairs = kGammaMaxFields * (kGammaMaxFields + 1) / 2;
constexpr int kGammaBlocks = 2048;                 // persistent workgroups over the bricks

// B3 at the quadrature points of a unit cell for the four nodes that reach
// it (P[q][o] = B3(t_q + 1 - o), node o = cell - 1 + o) and the weights.
struct GammaQuad {
    double p[5][4];
    double w[5];
};

static GammaQuad gamma_quad() {
    // 5-point Gauss-Legendre on [-1, 1], by Newton iteration on P_5
    double x[5], wq[5];
    for (int i = 0; i < 5; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / 5.5), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= 5; ++k) {
                const double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = 5 * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = z;
        wq[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
    auto b3 = [](double t) {
        const double a = std::fabs(t);
        if (a < 1.0) return (4.0 - 6.0 * a * a + 3.0 * a * a * a) / 6.0;
        if (a < 2.0) return (2.0 - a) * (2.0 - a) * (2.0 - a) / 6.0;
        return 0.0;
    };
    GammaQuad g{};
    for (int q = 0; q < 5; ++q) {
        const double t = 0.5 * (x[q] + 1.0);
        g.w[q] = 0.5 * wq[q];
        for (int o = 0; o < 4; ++o) g.p[q][o] = b3(t + 1.0 - o);
    }
    return g;
}

size_t gamma_workspace() { return align256(size_t(kGammaBlocks) * kGammaMaxPairs * sizeof(double)); }

template <typename KernelT>
static void allow_lds_gamma(KernelT kernel, size_t bytes) {
    if (bytes > 65536)
        (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
}

template <typename T, int N>
__global__ __launch_bounds__(kThreads) void k_ddd_gamma(const T* __restrict__ eps, const T* __restrict__ fields,
                                                        int nf, GammaQuad gq, double* __restrict__ part) {
    constexpr int BRICKS = N * N * (N / kGammaCZ);
    extern __shared__ double lds_raw[];
    T* vals = reinterpret_cast<T*>(lds_raw);                       // [nf + 1][kGammaS]: e w, then f_b
    T* reg = vals + (nf + 1) * kGammaS;                            // [4][4][kGammaRZ] coefficients
    T* sa = reg + 16 * kGammaRZ;                                   // [4][4][kGammaZS] after the z pass
    T* sb = sa + 16 * kGammaZS;                                    // [4][5][kGammaZS] after the y pass
    const int npairs = nf * (nf + 1) / 2;
    double acc[(kGammaMaxPairs + kThreads - 1) / kThreads];
#pragma unroll
    for (int i = 0; i < (kGammaMaxPairs + kThreads - 1) / kThreads; ++i) acc[i] = 0.0;
    for (int brick = blockIdx.x; brick < BRICKS; brick += gridDim.x) {
        const int cz0 = (brick % (N / kGammaCZ)) * kGammaCZ;
        const int cy = (brick / (N / kGammaCZ)) % N;
        const int cx = brick / (N / kGammaCZ) / N;
        for (int f = 0; f <= nf; ++f) {
            const T* src = f == 0 ? eps : fields + int64_t(f - 1) * N * N * N;
            for (int i = threadIdx.x; i < 16 * kGammaRZ; i += kThreads) {
                const int ox = i / (4 * kGammaRZ), oy = (i / kGammaRZ) % 4, oz = i % kGammaRZ;
                const int x = (cx - 1 + ox) & (N - 1), y = (cy - 1 + oy) & (N - 1), z = (cz0 - 1 + oz) & (N - 1);
                reg[i] = src[(int64_t(x) * N + y) * N + z];
            }
            __syncthreads();
            // z: [ox][oy][k q] = sum_o P[q][o] reg[ox][oy][k + o]
            for (int i = threadIdx.x; i < 16 * kGammaZS; i += kThreads) {
                const int oxy = i / kGammaZS, sz = i % kGammaZS, k = sz / 5, q = sz % 5;
                const T* r = reg + oxy * kGammaRZ + k;
                sa[i] = T(gq.p[q][0]) * r[0] + T(gq.p[q][1]) * r[1] + T(gq.p[q][2]) * r[2] + T(gq.p[q][3]) * r[3];
            }
            __syncthreads();
            // y: [ox][qy][sz] = sum_o P[qy][o] sa[ox][o][sz]
            for (int i = threadIdx.x; i < 20 * kGammaZS; i += kThreads) {
                const int ox = i / (5 * kGammaZS), qy = (i / kGammaZS) % 5, sz = i % kGammaZS;
                const T* a = sa + ox * 4 * kGammaZS + sz;
                sb[i] = T(gq.p[qy][0]) * a[0] + T(gq.p[qy][1]) * a[kGammaZS] + T(gq.p[qy][2]) * a[2 * kGammaZS] +
                        T(gq.p[qy][3]) * a[3 * kGammaZS];
            }
            __syncthreads();
            // x: [qx][qy][sz] = sum_o P[qx][o] sb[o][qy][sz]; e carries the weights
            T* dst = vals + f * kGammaS;
            for (int i = threadIdx.x; i < kGammaS; i += kThreads) {
                const int qx = i / (5 * kGammaZS), rest = i % (5 * kGammaZS);
                const T* b = sb + rest;
                T v = T(gq.p[qx][0]) * b[0] + T(gq.p[qx][1]) * b[5 * kGammaZS] + T(gq.p[qx][2]) * b[10 * kGammaZS] +
                      T(gq.p[qx][3]) * b[15 * kGammaZS];
                if (f == 0) {
                    const int qy = rest / kGammaZS, qz = (rest % kGammaZS) % 5;
                    v *= T(gq.w[qx] * gq.w[qy] * gq.w[qz]);
                }
                dst[i] = v;
            }
            __syncthreads();
        }
        // pairs b1 <= b2, thread t takes pairs t, t + 256, ...
#pragma unroll
        for (int i = 0; i < (kGammaMaxPairs + kThreads - 1) / kThreads; ++i) {
            const int pr = threadIdx.x + i * kThreads;
            if (pr < npairs) {
                int b1 = 0, rem = pr;
                while (rem >= nf - b1) {
                    rem -= nf - b1;
                    ++b1;
                }
                const int b2 = b1 + rem;
                const T* e = vals;
                const T* p1 = vals + (b1 + 1) * kGammaS;
                const T* p2 = vals + (b2 + 1) * kGammaS;
                T s = T(0);
                for (int k = 0; k < kGammaS; ++k) s += e[k] * p1[k] * p2[k];
                acc[i] += double(s);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < (kGammaMaxPairs + kThreads - 1) / kThreads; ++i) {
        const int pr = threadIdx.x + i * kThreads;
        if (pr < npairs) part[int64_t(blockIdx.x) * kGammaMaxPairs + pr] = acc[i];
    }
}

__global__ void k_gamma_final(const double* __restrict__ part, int n_blocks, int nf, double scale,
                              double* __restrict__ out) {
    const int pr = blockIdx.x * blockDim.x + threadIdx.x;
    if (pr >= nf * (nf + 1) / 2) return;
    int b1 = 0, rem = pr;
    while (rem >= nf - b1) {
        rem -= nf - b1;
        ++b1;
    }
    const int b2 = b1 + rem;
    double s = 0.0;
    for (int b = 0; b < n_blocks; ++b) s += part[int64_t(b) * kGammaMaxPairs + pr];
    out[b1 * nf + b2] = s * scale;
    out[b2 * nf + b1] = s * scale;
}

template <typename T, int N>
static hermes_status gamma_n(hermes_ctx ctx, const void* eps, const void* fields, int nf, double* out, void* work,
                             hipStream_t stream) {
    static const GammaQuad gq = gamma_quad();
    const size_t lds = (size_t(nf + 1) * kGammaS + 16 * kGammaRZ + 16 * kGammaZS + 20 * kGammaZS) * sizeof(T);
    allow_lds_gamma(k_ddd_gamma<T, N>, lds);
    constexpr int BRICKS = N * N * (N / kGammaCZ);
    const int blocks = BRICKS < kGammaBlocks ? BRICKS : kGammaBlocks;
    double* part = static_cast<double*>(work);
    {
        LaunchScope ls(ctx, stream, "ddd_gamma");
        hipLaunchKernelGGL((k_ddd_gamma<T, N>), dim3(blocks), dim3(kThreads), lds, stream, static_cast<const T*>(eps),
                           static_cast<const T*>(fields), nf, gq, part);
    }
    {
        LaunchScope ls(ctx, stream, "reduce");
        const double nc = double(N) * N * N;
        hipLaunchKernelGGL(k_gamma_final, dim3((nf * (nf + 1) / 2 + 127) / 128), dim3(128), 0, stream, part, blocks,
                           nf, 1.0 / nc, out);
    }
    return check_launch("hermes_ddd_gamma");
}

hermes_status gamma_impl(hermes_ctx ctx, const void* eps, const void* fields, int n_fields, int n, int dtype,
                         double* out, void* work, hipStream_t stream) {
#define HERMES_GAMMA_CASE(NN)                                                                        \
    case NN:                                                                                         \
        return dtype == HERMES_F32 ? gamma_n<float, NN>(ctx, eps, fields, n_fields, out, work, stream) \
                                   : gamma_n<double, NN>(ctx, eps, fields, n_fields, out, work, stream);
    switch (n) {
        HERMES_GAMMA_CASE(8)
        HERMES_GAMMA_CASE(16)
        HERMES_GAMMA_CASE(32)
        HERMES_GAMMA_CASE(64)
        HERMES_GAMMA_CASE(128)
        HERMES_GAMMA_CASE(256)
        HERMES_GAMMA_CASE(512)
        HERMES_GAMMA_CASE(1024)
        default:
            return fail(HERMES_ERR_ARG, "hermes_ddd_gamma: unsupported N");
    }
#undef HERMES_GAMMA_CASE
}

}  // namespace hermes
