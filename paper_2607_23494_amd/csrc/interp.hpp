// B3 interpolation of a coefficient field at an arbitrary point (Sec. 3.1:
// the value of n_W(x) = sum_l f_l phi_l(x) at any position), shared by the
// readout and the Monte-Carlo triangle kernels.
#pragma once

#include "common.hpp"

namespace hermes {

// B3 weights of the nodes i0-1 .. i0+2 for the fractional offset t in [0, 1).
__device__ __forceinline__ void b3_weights(double t, double w[4]) {
    const double s = 1.0 - t;
    w[0] = s * s * s / 6.0;
    w[1] = (4.0 - 6.0 * t * t + 3.0 * t * t * t) / 6.0;
    w[2] = (4.0 - 6.0 * s * s + 3.0 * s * s * s) / 6.0;
    w[3] = t * t * t / 6.0;
}

// sum_l f_l prod_a B3(u_a - l_a) over the 64 nodes around u (cell units, any
// real values; node indices mod N), accumulated in float64.
template <typename T, int N>
__device__ __forceinline__ double b3_value(const T* __restrict__ field, const double u[3]) {
    int cell[3];
    double tap[3][4];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double v = u[a];
        v -= double(N) * floor(v / double(N));   // periodic wrap into [0, N)
        const double f = floor(v);
        cell[a] = int(f);
        b3_weights(v - f, tap[a]);
    }
    int cz[4];
#pragma unroll
    for (int oz = 0; oz < 4; ++oz) cz[oz] = (cell[2] - 1 + oz) & (N - 1);
    double val = 0.0;
#pragma unroll
    for (int ox = 0; ox < 4; ++ox) {
        const int cx = (cell[0] - 1 + ox) & (N - 1);
        double vx = 0.0;
#pragma unroll
        for (int oy = 0; oy < 4; ++oy) {
            const int cy = (cell[1] - 1 + oy) & (N - 1);
            const T* row = field + (size_t(cx) * N + cy) * N;
            const double vy = tap[2][0] * double(row[cz[0]]) + tap[2][1] * double(row[cz[1]]) +
                              tap[2][2] * double(row[cz[2]]) + tap[2][3] * double(row[cz[3]]);
            vx += tap[1][oy] * vy;
        }
        val += tap[0][ox] * vx;
    }
    return val;
}

}  // namespace hermes

namespace hermes {

// A row's four B3 taps in one aligned vector: Quad<T> at node (x, y, z) holds
// the field at z - 1, z, z + 1, z + 2 (mod N) of row (x, y), so a point's 64
// taps are 16 vector loads instead of 64 scalar ones.
template <typename T> struct alignas(4 * sizeof(T)) Quad {
    T v[4];
};

template <typename T, int N>
__global__ __launch_bounds__(kThreads) void k_pack_rows(const T* __restrict__ f, Quad<T>* __restrict__ out) {
    const int64_t total = int64_t(N) * N * N;
    const int64_t stride = int64_t(gridDim.x) * kThreads;
    for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < total; i += stride) {
        const int64_t row = i & ~int64_t(N - 1);
        const int z = int(i & (N - 1));
        Quad<T> q;
#pragma unroll
        for (int o = 0; o < 4; ++o) q.v[o] = f[row + ((z - 1 + o) & (N - 1))];
        out[i] = q;
    }
}

// b3_value on a packed field.
template <typename T, int N>
__device__ __forceinline__ double b3_value_packed(const Quad<T>* __restrict__ p, const double u[3]) {
    int cell[3];
    double tap[3][4];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double v = u[a];
        v -= double(N) * floor(v / double(N));
        const double f = floor(v);
        cell[a] = int(f);
        b3_weights(v - f, tap[a]);
    }
    double val = 0.0;
#pragma unroll
    for (int ox = 0; ox < 4; ++ox) {
        const int cx = (cell[0] - 1 + ox) & (N - 1);
        double vx = 0.0;
#pragma unroll
        for (int oy = 0; oy < 4; ++oy) {
            const int cy = (cell[1] - 1 + oy) & (N - 1);
            const Quad<T> q = p[(size_t(cx) * N + cy) * N + (cell[2] & (N - 1))];
            const double vy = tap[2][0] * double(q.v[0]) + tap[2][1] * double(q.v[1]) + tap[2][2] * double(q.v[2]) +
                              tap[2][3] * double(q.v[3]);
            vx += tap[1][oy] * vy;
        }
        val += tap[0][ox] * vx;
    }
    return val;
}

}  // namespace hermes
