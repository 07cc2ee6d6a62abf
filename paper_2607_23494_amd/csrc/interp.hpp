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
