// Value of a coefficient field's basis expansion at an arbitrary point
// (Sec. 3.1: n_W(x) = sum_l f_l phi_l(x) read at any position), shared by
// the readout, Monte-Carlo triangle and assignment kernels.
#pragma once

#include "common.hpp"

namespace hermes {

// B3 weights of the nodes i0-1 .. i0+2 for the fractional offset t in [0, 1)
// (multiplied by the rounded 1/6 rather than divided: one rounding more, no
// division sequence).
__device__ __forceinline__ void b3_weights(double t, double w[4]) {
    constexpr double kSixth = 1.0 / 6.0;
    const double s = 1.0 - t;
    w[0] = s * s * s * kSixth;
    w[1] = (4.0 - 6.0 * t * t + 3.0 * t * t * t) * kSixth;
    w[2] = (4.0 - 6.0 * s * s + 3.0 * s * s * s) * kSixth;
    w[3] = t * t * t * kSixth;
}

// The D4 function at x in [0, 3]: the dyadic table (spacing 2^-kDb2Level)
// interpolated linearly.  x = 3 (reachable by rounding) reads phi(3) = 0.
__device__ __forceinline__ double db2_phi(double x, const double* __restrict__ tab) {
    const double s = x * double(1 << kDb2Level);
    int i = int(s);
    i = i < kDb2Tab - 2 ? i : kDb2Tab - 2;
    const double f = s - double(i);
    const double a = tab[i], b = tab[i + 1];
    return a + f * (b - a);
}

// Per-axis reach of a point at u = i0 + t (t in [0, 1)): the NT nodes
// i0 - LO + o, o < NT, with weights phi(t + LO - o).
template <int B> struct BasisTaps;
template <> struct BasisTaps<HERMES_BASIS_B3> {
    static constexpr int NT = 4, LO = 1;
    __device__ static __forceinline__ void weights(double t, const double* __restrict__, double w[4]) {
        b3_weights(t, w);
    }
};
template <> struct BasisTaps<HERMES_BASIS_DB2> {
    static constexpr int NT = 3, LO = 2;
    __device__ static __forceinline__ void weights(double t, const double* __restrict__ tab, double w[3]) {
        w[0] = db2_phi(t + 2.0, tab);
        w[1] = db2_phi(t + 1.0, tab);
        w[2] = db2_phi(t, tab);
    }
};

// sum_l f_l prod_a phi(u_a - l_a) over the NT^3 nodes around u (cell units,
// any real values; node indices mod N), accumulated in float64.
template <typename T, int N, int B>
__device__ __forceinline__ double basis_value(const T* __restrict__ field, const double u[3],
                                              const double* __restrict__ tab) {
    using P = BasisTaps<B>;
    constexpr int NT = P::NT, LO = P::LO;
    int cell[3];
    double tap[3][NT];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double v = u[a];
        v -= double(N) * floor(v / double(N));   // periodic wrap into [0, N)
        const double f = floor(v);
        cell[a] = int(f);
        P::weights(v - f, tab, tap[a]);
    }
    int cz[NT];
#pragma unroll
    for (int oz = 0; oz < NT; ++oz) cz[oz] = (cell[2] - LO + oz) & (N - 1);
    double val = 0.0;
#pragma unroll
    for (int ox = 0; ox < NT; ++ox) {
        const int cx = (cell[0] - LO + ox) & (N - 1);
        double vx = 0.0;
#pragma unroll
        for (int oy = 0; oy < NT; ++oy) {
            const int cy = (cell[1] - LO + oy) & (N - 1);
            const T* row = field + (size_t(cx) * N + cy) * N;
            double vy = 0.0;
#pragma unroll
            for (int oz = 0; oz < NT; ++oz) vy += tap[2][oz] * double(row[cz[oz]]);
            vx += tap[1][oy] * vy;
        }
        val += tap[0][ox] * vx;
    }
    return val;
}

}  // namespace hermes
