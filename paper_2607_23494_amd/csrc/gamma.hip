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
// A workgroup takes bricks of 1 x 1 x CZ cells.  Its wavefronts share out
// the fields: a wavefront stages a field's NT x NT x (CZ + NT - 1)
// coefficients in its own LDS scratch (loaded into registers while its
// previous field was evaluated), evaluates the brick's 125 CZ points in
// three passes synchronising only itself, and writes the point values (e
// times W, or f_b) to LDS.  After one barrier each thread takes a 4 x 4 tile
// of bin pairs over a slice of the points (nine LDS reads per sixteen FMAs);
// a second barrier frees the values.  Per-brick sums are float T, sums
// across bricks float64; the slices and the workgroups' partials are added
// in a fixed order.
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
constexpr int kGammaThreads = 512;                 // eight wavefronts per workgroup

// Coefficient nodes along z per brick.
template <int NT> constexpr int gamma_rz() { return kGammaCZ + NT - 1; }

// Per-axis operators: pe (for eps) and pf (for the fields) map the NT nodes
// cell - LO + o to the five points q; w holds the point weights per axis.
struct GammaOps {
    double pe[5][5];
    double pf[5][5];
    double w[5];
};

// The same in the field type, passed to the kernel (uniform operands).
template <typename T> struct GammaOpsT {
    T pe[5][5];
    T pf[5][5];
    T w[5];
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

template <typename T>
static GammaOpsT<T> gamma_ops_cast(const GammaOps& g) {
    GammaOpsT<T> o{};
    for (int q = 0; q < 5; ++q) {
        o.w[q] = T(g.w[q]);
        for (int k = 0; k < 5; ++k) {
            o.pe[q][k] = T(g.pe[q][k]);
            o.pf[q][k] = T(g.pf[q][k]);
        }
    }
    return o;
}

size_t gamma_workspace() {
    return align256(size_t(kGammaBlocks) * kGammaMaxFields * kGammaMaxFields * sizeof(double));
}

template <typename KernelT>
static void allow_lds_gamma(KernelT kernel, size_t bytes) {
    if (bytes > 65536)
        (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
}

// Per-wavefront scratch (elements): the field's staged coefficients, which
// the y-pass output later overwrites, then the z-pass output.
template <int NT> constexpr int gamma_nc() { return NT * NT * gamma_rz<NT>(); }
template <int NT> constexpr int gamma_scr() {
    return (gamma_nc<NT>() > NT * 5 * kGammaZS ? gamma_nc<NT>() : NT * 5 * kGammaZS) + NT * NT * kGammaZS;
}

template <typename T, int NT>
constexpr size_t gamma_lds_bytes(int nf, int ne) {
    return (size_t(nf + 1) * kGammaS + size_t(ne) * gamma_scr<NT>() + 5 * kGammaZS) * sizeof(T);
}

// One workgroup per brick at a time (persistent over the bricks).  Each of
// the first `ne` wavefronts evaluates every ne-th field on its own: it stages
// the field's NT x NT x RZ coefficients (loaded into registers while the
// previous field was evaluated) in its LDS scratch and runs the z, y and x
// passes, synchronising only itself; a work item of a pass reads NT inputs
// and writes the five points q (the operators are uniform).  Then the block
// forms the pair sums.
template <typename T, int N, int NT>
__global__ __launch_bounds__(kGammaThreads) void k_ddd_gamma(const T* __restrict__ eps, const T* __restrict__ fields,
                                                        int nf, int ne, GammaOpsT<T> gq, double* __restrict__ part) {
    constexpr int BRICKS = N * N * (N / kGammaCZ);
    constexpr int RZ = gamma_rz<NT>(), NN = NT * NT, LO = NT == 4 ? 1 : 2;
    constexpr int NC = gamma_nc<NT>(), PL = (NC + 63) / 64;
    constexpr int SB = NT * 5 * kGammaZS;
    constexpr int ZS = kGammaZS;
    extern __shared__ double lds_raw[];
    T* vals = reinterpret_cast<T*>(lds_raw);                        // [nf + 1][kGammaS]: e w, then f_b
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), lane = threadIdx.x % 64;   // wv: uniform
    T* scr = vals + (nf + 1) * kGammaS + wv * gamma_scr<NT>();
    T* rg = scr;                                                    // [NT][NT][RZ] coefficients
    T* sbw = scr;                                                   // [NT][5][ZS] after the y pass
    T* saw = scr + (NC > SB ? NC : SB);                             // [NT][NT][ZS] after the z pass
    T* wyz = vals + (nf + 1) * kGammaS + ne * gamma_scr<NT>();      // [5][ZS]: w[qy] w[qz] of the e points
    for (int i = threadIdx.x; i < 5 * ZS; i += kGammaThreads) wyz[i] = gq.w[i / ZS] * gq.w[(i % ZS) % 5];
    // pair roles: 4 x 4 bin tiles (I <= J) x sample slices
    const int nt4 = (nf + 3) / 4;
    const int ntp = nt4 * (nt4 + 1) / 2;
    const int slices = kGammaThreads / ntp;
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
    // this lane's coefficients of field f for a brick (field-major: ox, oy, oz)
    auto load = [&](int brick, int f, T (&r)[PL]) {
        const int cz0 = (brick % (N / kGammaCZ)) * kGammaCZ;
        const int cy = (brick / (N / kGammaCZ)) % N;
        const int cx = brick / (N / kGammaCZ) / N;
        const T* src = f == 0 ? eps : fields + int64_t(f - 1) * N * N * N;
#pragma unroll
        for (int p = 0; p < PL; ++p) {
            const int i = lane + 64 * p;
            if (i < NC) {
                const int ox = i / (NT * RZ), oy = (i / RZ) % NT, oz = i % RZ;
                const int x = (cx - LO + ox) & (N - 1), y = (cy - LO + oy) & (N - 1), z = (cz0 - LO + oz) & (N - 1);
                r[p] = src[(int64_t(x) * N + y) * N + z];
            }
        }
    };
    const bool evaluates = wv < ne && wv <= nf;   // a wavefront with a field (its first is wv)
    T cur[PL];
    if (evaluates && int(blockIdx.x) < BRICKS) load(blockIdx.x, wv, cur);
    __syncthreads();   // wyz
    for (int brick = blockIdx.x; brick < BRICKS; brick += gridDim.x) {
        if (evaluates) {
            for (int f = wv; f <= nf; f += ne) {
#pragma unroll
                for (int p = 0; p < PL; ++p)
                    if (lane + 64 * p < NC) rg[lane + 64 * p] = cur[p];
                // the next (brick, field) of this wavefront loads meanwhile
                int f2 = f + ne, b2 = brick;
                if (f2 > nf) {
                    f2 = wv;
                    b2 = brick + int(gridDim.x);
                }
                if (b2 < BRICKS) load(b2, f2, cur);
                wave_sync();
                const T(&P)[5][5] = f == 0 ? gq.pe : gq.pf;
                // z: saw[ox][oy][k q] = sum_o P[q][o] rg[ox][oy][k + o]
                for (int it = lane; it < NN * kGammaCZ; it += 64) {
                    const int row = it / kGammaCZ, k = it % kGammaCZ;
                    T in[NT];
#pragma unroll
                    for (int o = 0; o < NT; ++o) in[o] = rg[row * RZ + k + o];
#pragma unroll
                    for (int q = 0; q < 5; ++q) {
                        T v = T(0);
#pragma unroll
                        for (int o = 0; o < NT; ++o) v += P[q][o] * in[o];
                        saw[row * ZS + k * 5 + q] = v;
                    }
                }
                wave_sync();
                // y: sbw[ox][qy][sz] = sum_o P[qy][o] saw[ox][o][sz]
                for (int it = lane; it < NT * ZS; it += 64) {
                    const int ox = it / ZS, sz = it % ZS;
                    T in[NT];
#pragma unroll
                    for (int o = 0; o < NT; ++o) in[o] = saw[(ox * NT + o) * ZS + sz];
#pragma unroll
                    for (int q = 0; q < 5; ++q) {
                        T v = T(0);
#pragma unroll
                        for (int o = 0; o < NT; ++o) v += P[q][o] * in[o];
                        sbw[(ox * 5 + q) * ZS + sz] = v;
                    }
                }
                wave_sync();
                // x: vals[f][qx][qy][sz] = sum_o P[qx][o] sbw[o][qy][sz]; e carries the weights
                T* dst = vals + f * kGammaS;
                for (int it = lane; it < 5 * ZS; it += 64) {
                    T in[NT];
#pragma unroll
                    for (int o = 0; o < NT; ++o) in[o] = sbw[o * 5 * ZS + it];
                    const T wt = f == 0 ? wyz[it] : T(1);
#pragma unroll
                    for (int q = 0; q < 5; ++q) {
                        T v = T(0);
#pragma unroll
                        for (int o = 0; o < NT; ++o) v += P[q][o] * in[o];
                        dst[q * 5 * ZS + it] = f == 0 ? v * (gq.w[q] * wt) : v;
                    }
                }
                wave_sync();
            }
        }
        __syncthreads();
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

// out[b1 nf + b2] = scale sum_b part[b][b1][b2]; one workgroup per entry,
// thread t adds the blocks t, t + kThreads, ... in order, then the fixed tree
// of block_sum, so the result repeats bit for bit.
__global__ __launch_bounds__(kThreads) void k_gamma_final(const double* __restrict__ part, int n_blocks, int nf,
                                                          double scale, double* __restrict__ out) {
    __shared__ double red[kThreads];
    const int i = blockIdx.x;
    const int b1 = i / nf, b2 = i % nf;
    double s = 0.0;
    for (int b = threadIdx.x; b < n_blocks; b += kThreads)
        s += part[int64_t(b) * kGammaMaxFields * kGammaMaxFields + b1 * kGammaMaxFields + b2];
    s = block_sum(s, red);
    if (threadIdx.x == 0) out[i] = s * scale;
}

template <typename T, int N, int NT>
static hermes_status gamma_nb(hermes_ctx ctx, const void* eps, const void* fields, int nf, const GammaOps& g64,
                              double* out, void* work, hipStream_t stream) {
    // as many evaluating wavefronts (8, 4, 2 or 1) as the LDS holds scratch for
    int ne = kGammaThreads / 64;
    while (ne > 1 && gamma_lds_bytes<T, NT>(nf, ne) > size_t(160) * 1024) ne /= 2;
    const size_t lds_f = gamma_lds_bytes<T, NT>(nf, ne), lds_r = size_t(kGammaThreads) * 16 * sizeof(double);
    const size_t lds = lds_f > lds_r ? lds_f : lds_r;
    if (lds > size_t(160) * 1024) return fail(HERMES_ERR_UNSUPPORTED, "hermes_ddd_gamma: too many fields for LDS");
    allow_lds_gamma(k_ddd_gamma<T, N, NT>, lds);
    const GammaOpsT<T> gq = gamma_ops_cast<T>(g64);
    constexpr int BRICKS = N * N * (N / kGammaCZ);
    const int blocks = BRICKS < kGammaBlocks ? BRICKS : kGammaBlocks;
    double* part = static_cast<double*>(work);
    {
        LaunchScope ls(ctx, stream, "ddd_gamma");
        hipLaunchKernelGGL((k_ddd_gamma<T, N, NT>), dim3(blocks), dim3(kGammaThreads), lds, stream,
                           static_cast<const T*>(eps), static_cast<const T*>(fields), nf, ne, gq, part);
    }
    {
        LaunchScope ls(ctx, stream, "reduce");
        const double nc = double(N) * N * N;
        hipLaunchKernelGGL(k_gamma_final, dim3(nf * nf), dim3(kThreads), 0, stream, part, blocks,
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
