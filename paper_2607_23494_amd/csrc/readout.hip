// Readout of a coefficient field at arbitrary positions (Sec. 3.1: the
// filtered field n_W(x) = sum_l eps~_l phi_l(x) read at any point) and the
// density-derived marks of Sec. 3.3.1 (Eqs. power-law-mark,
// inverse-density-mark).
//
// The value at a point is the node sum v = sum_l f_l prod_a phi(x_a/h - l_a)
// (64 nodes with B3, 27 with the D4 function), the transpose of the
// assignment's scatter: one thread per point gathers its rows of nodes.  Optionally the value becomes a mark and is multiplied by a weight
// (the marked catalogue for hermes_assign), and the moments <v^p>, p = 2..4,
// over the points are accumulated in float64 (counts in cells by sampling
// positions).
#include <cmath>

#include "common.hpp"
#include "interp.hpp"
#include "kernels.hpp"

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

template <typename T, int N, int B>
__global__ __launch_bounds__(kThreads) void k_readout(const T* __restrict__ field, const float* __restrict__ pos,
                                                      const float* __restrict__ weight, int64_t n_pts,
                                                      double scale, MarkParams mk, const double* __restrict__ tab,
                                                      T* __restrict__ out, double* __restrict__ mom) {
    __shared__ double red[kThreads];
    double m2 = 0.0, m3 = 0.0, m4 = 0.0;
    const int64_t stride = int64_t(gridDim.x) * kThreads;
    for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < n_pts; i += stride) {
        const double u[3] = {double(pos[3 * i]) * scale, double(pos[3 * i + 1]) * scale,
                             double(pos[3 * i + 2]) * scale};   // position in cell units
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

__global__ void k_scale3(double* __restrict__ mom, double s) {
    if (threadIdx.x < 3) mom[threadIdx.x] *= s;
}

template <typename T, int N>
static hermes_status readout_n(hermes_ctx ctx, const void* field, double box_L, const float* pos,
                               const float* weight, int64_t n_pts, const MarkParams& mk, void* out,
                               double* moments, hipStream_t stream) {
    if (moments) {
        LaunchScope ls(ctx, stream, "fill");
        launch_fill<double>(moments, 3, 0.0, stream);
    }
    if (n_pts > 0) {
        LaunchScope ls(ctx, stream, "readout");
        const int64_t want = (n_pts + kThreads - 1) / kThreads;
        const int blocks = int(want < 8192 ? want : 8192);
        if (ctx->basis == HERMES_BASIS_DB2)
            hipLaunchKernelGGL((k_readout<T, N, HERMES_BASIS_DB2>), dim3(blocks), dim3(kThreads), 0, stream,
                               static_cast<const T*>(field), pos, weight, n_pts, double(N) / box_L, mk,
                               ctx->t.db2tab, static_cast<T*>(out), moments);
        else
            hipLaunchKernelGGL((k_readout<T, N, HERMES_BASIS_B3>), dim3(blocks), dim3(kThreads), 0, stream,
                               static_cast<const T*>(field), pos, weight, n_pts, double(N) / box_L, mk,
                               ctx->t.db2tab, static_cast<T*>(out), moments);
        if (moments)
            hipLaunchKernelGGL(k_scale3, dim3(1), dim3(64), 0, stream, moments, 1.0 / double(n_pts));
    }
    return check_launch("hermes_readout");
}

hermes_status readout_impl(hermes_ctx ctx, const void* field, int n, int dtype, double box_L, const float* pos,
                           const float* weight, int64_t n_pts, const hermes_mark* mark, void* out,
                           double* moments, hipStream_t stream) {
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
                   ? readout_n<float, NN>(ctx, field, box_L, pos, weight, n_pts, mk, out, moments, stream)   \
                   : readout_n<double, NN>(ctx, field, box_L, pos, weight, n_pts, mk, out, moments, stream);
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
