// 3PCF monopole through triple connection coefficients (Sec. 3.3.2, Eqs.
// 3PCF-ddd-monopole, con-coeff, DDD-vector-product):
//
//   out[b1][b2] = N^-3 sum_l e_l sum_{a,b} Gamma_{a,b} f_b1[l + a] f_b2[l + b],
//   Gamma_{a,b} = int phi(x) phi(x - a) phi(x - b) d^3x,
//
// Gamma is separable, prod_axes gamma(a_i, b_i), and both bases reduce the
// stencil to sums over 125 "points" per cell of products of per-axis
// operators applied to the node values:
//   out = N^-3 sum_l sum_{q in 5^3} W_q (P_e eps)_{l,q} (P_f f_b1)_{l,q} (P_f f_b2)_{l,q},
// with (P f)_{l,q} = sum_o prod_axes P[q_i][o_i] f[l - LO + o] over NT nodes
// per axis.
//  - B3 (NT = 4, LO = 1): the stencil sum is the integral over the box of
//    the product of the three B3 expansions (cell units).  On one unit cell
//    each expansion is a cubic per axis, so 5-point Gauss-Legendre per axis
//    integrates the product exactly: P_e = P_f = B3 at the Gauss points, W
//    the Gauss weights (instead of contracting the 7^6 offsets of Gamma).
//  - D4 (NT = 5, LO = 2): gamma = V diag(lambda) V^T (a symmetric 5 x 5
//    matrix over the offsets -2..2), so sum_{a,b} Gamma_{a,b} f1[l+a]
//    f2[l+b] = sum_q lambda_q F1_q[l] F2_q[l] with F_q = the separable
//    stencil prod V[o_i][q_i]: P_f[q][o] = V[o][q], P_e picks the node
//    itself (o = 2), W = lambda.
//
// A workgroup takes bricks of 1 x 1 x CZ cells (in float the next brick's
// coefficients load into registers meanwhile): for groups of fields it
// stages the NT x NT x (CZ + NT - 1) coefficients in LDS, evaluates the
// brick's 125 CZ points in three passes, and keeps the point values of e
// (times W) and of every f_b in LDS; then each thread takes a 4 x 4 tile of
// bin pairs over a slice of the points (nine LDS reads per sixteen FMAs).
// Per-brick sums are float T, sums across bricks float64; the slices and
// the workgroups' partials are added in a fixed order.
#include <cmath>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

namespace hermes {

constexpr int kGammaCZ = 4;                        // cells per brick along z
constexpr int kGammaS = 125 * kGammaCZ;            // points per brick
constexpr int kGammaZS = 5 * kGammaCZ;             // points along z per brick
constexpr int kGammaMaxFields = 32;               // bins per call
constexpr int kGammaBlocks = 2048;                 // persistent workgroups over the bricks

// Coefficient nodes along z per brick.
template <int NT> constexpr int gamma_rz() { return kGammaCZ + NT - 1; }

// Per-axis operators: pe (for eps) and pf (for the fields) map the NT nodes
// cell - LO + o to the five points q; w holds the point weights per axis.
struct GammaOps {
    double pe[5][5];
    double pf[5][5];
    double w[5];
};

static GammaOps gamma_ops_b3() {
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
    GammaOps g{};
    for (int q = 0; q < 5; ++q) {
        const double t = 0.5 * (x[q] + 1.0);
        g.w[q] = 0.5 * wq[q];
        for (int o = 0; o < 4; ++o) g.pe[q][o] = g.pf[q][o] = b3(t + 1.0 - o);
    }
    return g;
}

static GammaOps gamma_ops_db2() {
    double lam[5], vec[5][5];
    db2_gamma_factors(lam, vec);
    GammaOps g{};
    for (int q = 0; q < 5; ++q) {
        g.w[q] = lam[q];
        for (int o = 0; o < 5; ++o) {
            g.pf[q][o] = vec[o][q];
            g.pe[q][o] = o == 2 ? 1.0 : 0.0;
        }
    }
    return g;
}

size_t gamma_workspace() {
    return align256(size_t(kGammaBlocks) * kGammaMaxFields * kGammaMaxFields * sizeof(double));
}

template <typename KernelT>
static void allow_lds_gamma(KernelT kernel, size_t bytes) {
    if (bytes > 65536)
        (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
}

// Fields evaluated per barrier group (LDS for the staged coefficients and the
// two intermediate passes of FG fields; 32 fields fit in 160 KB of LDS).
template <typename T, int NT> constexpr int gamma_fg() {
    return sizeof(T) == 4 ? (NT == 4 ? 8 : 4) : (NT == 4 ? 4 : 2);
}

// float: the next brick's coefficients of every field are loaded into
// registers while the current brick is evaluated (and all fields'
// coefficients are staged in LDS at once); float64 stages them per group.
template <typename T> constexpr bool gamma_prefetch() { return sizeof(T) == 4; }
template <int NT> constexpr int gamma_pre() {
    return ((kGammaMaxFields + 1) * NT * NT * gamma_rz<NT>() + kThreads - 1) / kThreads;
}

template <typename T, int NT>
constexpr size_t gamma_lds_bytes(int nf) {
    constexpr int FG = gamma_fg<T, NT>();
    const size_t regs = size_t(gamma_prefetch<T>() ? nf + 1 : FG) * NT * NT * gamma_rz<NT>();
    return (size_t(nf + 1) * kGammaS + regs + size_t(FG) * (NT * NT * kGammaZS + NT * 5 * kGammaZS)) * sizeof(T);
}

template <typename T, int N, int NT>
__global__ __launch_bounds__(kThreads) void k_ddd_gamma(const T* __restrict__ eps, const T* __restrict__ fields,
                                                        int nf, GammaOps gq, double* __restrict__ part) {
    constexpr int BRICKS = N * N * (N / kGammaCZ);
    constexpr int FG = gamma_fg<T, NT>();
    constexpr bool PRE = gamma_prefetch<T>();
    constexpr int RZ = gamma_rz<NT>(), NN = NT * NT, LO = NT == 4 ? 1 : 2;
    constexpr int NPRE = gamma_pre<NT>();
    extern __shared__ double lds_raw[];
    T* vals = reinterpret_cast<T*>(lds_raw);                       // [nf + 1][kGammaS]: e w, then f_b
    T* reg = vals + (nf + 1) * kGammaS;                            // [nf + 1 or FG][NT][NT][RZ] coefficients
    T* sa = reg + (PRE ? nf + 1 : FG) * NN * RZ;                   // [FG][NT][NT][kGammaZS] after the z pass
    T* sb = sa + FG * NN * kGammaZS;                               // [FG][NT][5][kGammaZS] after the y pass
    // pair roles: 4 x 4 bin tiles (I <= J) x sample slices
    const int nt4 = (nf + 3) / 4;
    const int ntp = nt4 * (nt4 + 1) / 2;
    const int slices = kThreads / ntp;
    const int tp = threadIdx.x % ntp, slice = threadIdx.x / ntp;
    int ti = 0, tj = 0;
    for (int I = 0, idx = tp; I < nt4; ++I) {
        if (idx < nt4 - I) {
            ti = I;
            tj = I + idx;
            break;
        }
        idx -= nt4 - I;
    }
    double acc64[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) acc64[i] = 0.0;
    // coefficient i (field-major: field, ox, oy, oz) of a brick
    auto coef = [&](int brick, int i) -> T {
        const int cz0 = (brick % (N / kGammaCZ)) * kGammaCZ;
        const int cy = (brick / (N / kGammaCZ)) % N;
        const int cx = brick / (N / kGammaCZ) / N;
        const int f = i / (NN * RZ), e = i % (NN * RZ);
        const int ox = e / (NT * RZ), oy = (e / RZ) % NT, oz = e % RZ;
        const int x = (cx - LO + ox) & (N - 1), y = (cy - LO + oy) & (N - 1), z = (cz0 - LO + oz) & (N - 1);
        const T* src = f == 0 ? eps : fields + int64_t(f - 1) * N * N * N;
        return src[(int64_t(x) * N + y) * N + z];
    };
    const int ncoef = (nf + 1) * NN * RZ;
    T pre[PRE ? NPRE : 1];
    if constexpr (PRE) {
        if (int(blockIdx.x) < BRICKS) {
#pragma unroll
            for (int k = 0; k < NPRE; ++k) {
                const int i = threadIdx.x + k * kThreads;
                if (i < ncoef) pre[k] = coef(blockIdx.x, i);
            }
        }
    }
    for (int brick = blockIdx.x; brick < BRICKS; brick += gridDim.x) {
        if constexpr (PRE) {
            // stage this brick's coefficients, then load the next brick's
#pragma unroll
            for (int k = 0; k < NPRE; ++k) {
                const int i = threadIdx.x + k * kThreads;
                if (i < ncoef) reg[i] = pre[k];
            }
            const int nxt = brick + int(gridDim.x);
            if (nxt < BRICKS) {
#pragma unroll
                for (int k = 0; k < NPRE; ++k) {
                    const int i = threadIdx.x + k * kThreads;
                    if (i < ncoef) pre[k] = coef(nxt, i);
                }
            }
            __syncthreads();
        }
        for (int f0 = 0; f0 <= nf; f0 += FG) {
            const int fg = nf + 1 - f0 < FG ? nf + 1 - f0 : FG;
            if constexpr (!PRE) {
                for (int i = threadIdx.x; i < fg * NN * RZ; i += kThreads)
                    reg[i] = coef(brick, f0 * NN * RZ + i);
                __syncthreads();
            }
            const T* greg = reg + (PRE ? f0 * NN * RZ : 0);
            // z: [f][ox][oy][k q] = sum_o P[q][o] reg[f][ox][oy][k + o]
            for (int i = threadIdx.x; i < fg * NN * kGammaZS; i += kThreads) {
                const int fo = i / kGammaZS, sz = i % kGammaZS, k = sz / 5, q = sz % 5;
                const double(&P)[5][5] = f0 + fo / NN == 0 ? gq.pe : gq.pf;
                const T* r = greg + fo * RZ + k;
                T v = T(0);
#pragma unroll
                for (int o = 0; o < NT; ++o) v += T(P[q][o]) * r[o];
                sa[i] = v;
            }
            __syncthreads();
            // y: [f][ox][qy][sz] = sum_o P[qy][o] sa[f][ox][o][sz]
            for (int i = threadIdx.x; i < fg * NT * 5 * kGammaZS; i += kThreads) {
                const int fox = i / (5 * kGammaZS), qy = (i / kGammaZS) % 5, sz = i % kGammaZS;
                const double(&P)[5][5] = f0 + fox / NT == 0 ? gq.pe : gq.pf;
                const T* a = sa + fox * NT * kGammaZS + sz;
                T v = T(0);
#pragma unroll
                for (int o = 0; o < NT; ++o) v += T(P[qy][o]) * a[o * kGammaZS];
                sb[i] = v;
            }
            __syncthreads();
            // x: [qx][qy][sz] = sum_o P[qx][o] sb[f][o][qy][sz]; e carries the weights
            for (int i = threadIdx.x; i < fg * kGammaS; i += kThreads) {
                const int f = i / kGammaS, e = i % kGammaS;
                const int qx = e / (5 * kGammaZS), rest = e % (5 * kGammaZS);
                const double(&P)[5][5] = f0 + f == 0 ? gq.pe : gq.pf;
                const T* b = sb + f * NT * 5 * kGammaZS + rest;
                T v = T(0);
#pragma unroll
                for (int o = 0; o < NT; ++o) v += T(P[qx][o]) * b[o * 5 * kGammaZS];
                if (f0 + f == 0) {
                    const int qy = rest / kGammaZS, qz = (rest % kGammaZS) % 5;
                    v *= T(gq.w[qx] * gq.w[qy] * gq.w[qz]);
                }
                vals[(f0 + f) * kGammaS + e] = v;
            }
            __syncthreads();
        }
        // the tile's 4 x 4 block of pair sums over this slice's points
        if (slice < slices) {
            T acc[4][4];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[a][c] = T(0);
            for (int k = slice; k < kGammaS; k += slices) {
                const T e = vals[k];
                T y1[4], y2[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const int b1 = 4 * ti + a, b2 = 4 * tj + a;
                    y1[a] = b1 < nf ? e * vals[(b1 + 1) * kGammaS + k] : T(0);
                    y2[a] = b2 < nf ? vals[(b2 + 1) * kGammaS + k] : T(0);
                }
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc[a][c] += y1[a] * y2[c];
            }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc64[4 * a + c] += double(acc[a][c]);
        }
        __syncthreads();
    }
    // sum the slices of every tile in a fixed order; the workgroup's full
    // matrix goes to part[block][b1 * 32 + b2]
    double* red = lds_raw;
#pragma unroll
    for (int i = 0; i < 16; ++i) red[threadIdx.x * 16 + i] = acc64[i];
    __syncthreads();
    if (threadIdx.x < ntp) {
        double sum[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) sum[i] = 0.0;
        for (int c = 0; c < slices; ++c)
#pragma unroll
            for (int i = 0; i < 16; ++i) sum[i] += red[(c * ntp + threadIdx.x) * 16 + i];
        double* dst = part + int64_t(blockIdx.x) * kGammaMaxFields * kGammaMaxFields;
        for (int a = 0; a < 4; ++a)
            for (int c = 0; c < 4; ++c) {
                const int b1 = 4 * ti + a, b2 = 4 * tj + c;
                if (b1 < nf && b2 < nf) {
                    dst[b1 * kGammaMaxFields + b2] = sum[4 * a + c];
                    dst[b2 * kGammaMaxFields + b1] = sum[4 * a + c];
                }
            }
    }
}

__global__ void k_gamma_final(const double* __restrict__ part, int n_blocks, int nf, double scale,
                              double* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nf * nf) return;
    const int b1 = i / nf, b2 = i % nf;
    double s = 0.0;
    for (int b = 0; b < n_blocks; ++b) s += part[int64_t(b) * kGammaMaxFields * kGammaMaxFields + b1 * kGammaMaxFields + b2];
    out[i] = s * scale;
}

template <typename T, int N, int NT>
static hermes_status gamma_nb(hermes_ctx ctx, const void* eps, const void* fields, int nf, const GammaOps& gq,
                              double* out, void* work, hipStream_t stream) {
    const size_t lds_f = gamma_lds_bytes<T, NT>(nf), lds_r = size_t(kThreads) * 16 * sizeof(double);
    const size_t lds = lds_f > lds_r ? lds_f : lds_r;
    if (lds > size_t(160) * 1024) return fail(HERMES_ERR_UNSUPPORTED, "hermes_ddd_gamma: too many fields for LDS");
    allow_lds_gamma(k_ddd_gamma<T, N, NT>, lds);
    constexpr int BRICKS = N * N * (N / kGammaCZ);
    const int blocks = BRICKS < kGammaBlocks ? BRICKS : kGammaBlocks;
    double* part = static_cast<double*>(work);
    {
        LaunchScope ls(ctx, stream, "ddd_gamma");
        hipLaunchKernelGGL((k_ddd_gamma<T, N, NT>), dim3(blocks), dim3(kThreads), lds, stream,
                           static_cast<const T*>(eps), static_cast<const T*>(fields), nf, gq, part);
    }
    {
        LaunchScope ls(ctx, stream, "reduce");
        const double nc = double(N) * N * N;
        hipLaunchKernelGGL(k_gamma_final, dim3((nf * nf + 127) / 128), dim3(128), 0, stream, part, blocks,
                           nf, 1.0 / nc, out);
    }
    return check_launch("hermes_ddd_gamma");
}

template <typename T, int N>
static hermes_status gamma_n(hermes_ctx ctx, const void* eps, const void* fields, int nf, double* out, void* work,
                             hipStream_t stream) {
    if (ctx->basis == HERMES_BASIS_DB2) {
        static const GammaOps ops = gamma_ops_db2();
        return gamma_nb<T, N, 5>(ctx, eps, fields, nf, ops, out, work, stream);
    }
    static const GammaOps ops = gamma_ops_b3();
    return gamma_nb<T, N, 4>(ctx, eps, fields, nf, ops, out, work, stream);
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
