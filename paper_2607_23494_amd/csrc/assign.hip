// MRA projection of a weighted catalogue onto B3 scaling-function
// coefficients (Sec. 3.1, Eq. phi_projection), as a wavefront-parallel
// scatter of 64 taps per point with hardware float atomics.
#include "common.hpp"
#include "kernels.hpp"

namespace hermes {

// B3 weights of the four nodes i0-1 .. i0+2 for fractional offset t in [0, 1).
__device__ __forceinline__ void b3_taps(double t, double w[4]) {
    const double s = 1.0 - t;
    w[0] = s * s * s / 6.0;
    w[1] = (4.0 - 6.0 * t * t + 3.0 * t * t * t) / 6.0;
    w[2] = (4.0 - 6.0 * s * s + 3.0 * s * s * s) / 6.0;
    w[3] = t * t * t / 6.0;
}

template <typename T, int N>
__global__ __launch_bounds__(kThreads) void k_assign(const float* __restrict__ pos,
                                                     const float* __restrict__ weight,
                                                     int64_t n_pts, double scale, T* __restrict__ eps,
                                                     double* __restrict__ sum_w) {
    __shared__ double red[kThreads];
    double wsum = 0.0;
    const int64_t stride = int64_t(gridDim.x) * kThreads;
    for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < n_pts; i += stride) {
        const double w = weight ? double(weight[i]) : 1.0;
        wsum += w;
        int cell[3];
        double tap[3][4];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double u = double(pos[3 * i + a]) * scale;     // position in cell units
            u -= double(N) * floor(u / double(N));         // periodic wrap into [0, N)
            const double f = floor(u);
            cell[a] = int(f);
            b3_taps(u - f, tap[a]);
        }
#pragma unroll
        for (int ox = 0; ox < 4; ++ox) {
            const int cx = (cell[0] - 1 + ox) & (N - 1);
            const double wx = w * tap[0][ox];
#pragma unroll
            for (int oy = 0; oy < 4; ++oy) {
                const int cy = (cell[1] - 1 + oy) & (N - 1);
                const double wxy = wx * tap[1][oy];
                T* row = eps + (size_t(cx) * N + cy) * N;
#pragma unroll
                for (int oz = 0; oz < 4; ++oz) {
                    const int cz = (cell[2] - 1 + oz) & (N - 1);
                    unsafeAtomicAdd(row + cz, T(wxy * tap[2][oz]));
                }
            }
        }
    }
    red[threadIdx.x] = wsum;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) unsafeAtomicAdd(sum_w, red[0]);
}

template <typename T, int N>
static hermes_status assign_n(hermes_ctx ctx, const float* pos, const float* weight, int64_t n_pts, double box_L,
                              void* eps, double* sum_w, hipStream_t stream) {
    const int64_t cells = int64_t(N) * N * N;
    {
        LaunchScope ls(ctx, stream, "fill");
        launch_fill<T>(static_cast<T*>(eps), cells, T(0), stream);
    }
    {
        LaunchScope ls(ctx, stream, "fill");
        launch_fill<double>(sum_w, 1, 0.0, stream);
    }
    if (n_pts > 0) {
        LaunchScope ls(ctx, stream, "assign");
        const int64_t want = (n_pts + kThreads - 1) / kThreads;
        const int blocks = int(want < 8192 ? want : 8192);
        hipLaunchKernelGGL((k_assign<T, N>), dim3(blocks), dim3(kThreads), 0, stream, pos, weight, n_pts,
                           double(N) / box_L, static_cast<T*>(eps), sum_w);
    }
    return check_launch("hermes_assign");
}

hermes_status assign_impl(hermes_ctx ctx, const float* pos, const float* weight, int64_t n_pts, double box_L,
                          int n, int dtype, void* eps, double* sum_w, hipStream_t stream) {
#define HERMES_ASSIGN_CASE(NN)                                                                  \
    case NN:                                                                                    \
        return dtype == HERMES_F32 ? assign_n<float, NN>(ctx, pos, weight, n_pts, box_L, eps, sum_w, stream) \
                                   : assign_n<double, NN>(ctx, pos, weight, n_pts, box_L, eps, sum_w, stream);
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
