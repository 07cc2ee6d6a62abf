// Pass kernels of the 3-D real FFT on an N^3 grid.
//
// Forward: (1) r2c along z with the contrast delta = eps/eps_bar - 1 fused
// into the load, (2) c2c along y, (3) c2c along x.  Each pass reads and
// writes HBM once.  The strided passes stage a tile of TC adjacent columns
// (contiguous in memory) times the full line length in LDS, so that every
// global access is a run of TC consecutive complex values.
#pragma once

#include "fft_core.hpp"

namespace hermes {

constexpr int kLdsBudget = 65536;   // bytes of LDS per workgroup used by the pass kernels

template <typename T> struct fft_cfg;
template <> struct fft_cfg<float> { static constexpr int elems = 8192; };   // complex per 64 KB
template <> struct fft_cfg<double> { static constexpr int elems = 4096; };

// columns per tile of a strided pass: TC * (N + 1) complex fit the budget
template <typename T, int N> struct strided_cfg {
    static constexpr int LP = N + 1;
    static constexpr int TC = fft_cfg<T>::elems / LP;
};

template <typename T> inline const typename cplx_of<T>::type* tw_ptr(const Tables& t);
template <> inline const float2* tw_ptr<float>(const Tables& t) { return t.tw32; }
template <> inline const double2* tw_ptr<double>(const Tables& t) { return t.tw64; }

// ---------------------------------------------------------------- forward z (r2c)
// rows of N reals -> rows of N/2+1 complex.  Real pairs are packed into a
// length-N/2 complex FFT and separated afterwards.
template <typename T, int N>
__global__ __launch_bounds__(kThreads) void k_fwd_z(const T* __restrict__ eps, const double* __restrict__ sum_w,
                                                    T* __restrict__ delta_out,
                                                    typename cplx_of<T>::type* __restrict__ dk,
                                                    const typename cplx_of<T>::type* __restrict__ tw) {
    using C = typename cplx_of<T>::type;
    constexpr int M = N / 2, P = M + 1, LP = M;
    constexpr int LINES = fft_cfg<T>::elems / M;
    constexpr int ROWS = N * N;
    __shared__ C s[LINES * LP];
    const int row0 = blockIdx.x * LINES;
    const int nl = min(LINES, ROWS - row0);
    const double inv_mean = double(N) * double(N) * double(N) / sum_w[0];
    // load + contrast
    for (int e = threadIdx.x; e < nl * M; e += kThreads) {
        const int64_t g = int64_t(row0) * N + 2 * e;      // rows are contiguous
        const T a = T(double(eps[g]) * inv_mean - 1.0);
        const T b = T(double(eps[g + 1]) * inv_mean - 1.0);
        if (delta_out) {
            delta_out[g] = a;
            delta_out[g + 1] = b;
        }
        s[e] = C{a, b};   // line e / M, element e % M, LP == M
    }
    lds_fft<C, M, LP, LINES, false>(s, tw, nl);
    // separate the packed transforms: X[k] = (Z[k] + Z*[M-k])/2 - i/2 W^k (Z[k] - Z*[M-k])
    for (int e = threadIdx.x; e < nl * P; e += kThreads) {
        const int line = e / P, k = e - line * P;
        const C zk = s[line * LP + (k & (M - 1))];
        const C zm = s[line * LP + ((M - k) & (M - 1))];
        const C sum{zk.x + zm.x, zk.y - zm.y};
        const C dif{zk.x - zm.x, zk.y + zm.y};
        const C t = c_mul(tw[N + k], dif);
        dk[int64_t(row0) * P + e] = C{T(0.5) * (sum.x + t.y), T(0.5) * (sum.y - t.x)};
    }
}

// ---------------------------------------------------------------- strided c2c
// In-place FFT along an axis of length N with element stride `stride`, for
// `ncols` contiguous columns in each of gridDim.y planes.  zero_dc clears
// element 0 of plane 0 after the transform.
template <typename T, int N, bool INV>
__global__ __launch_bounds__(kThreads) void k_c2c_strided(typename cplx_of<T>::type* __restrict__ data,
                                                          int64_t plane_stride, int ncols, int64_t stride,
                                                          int zero_dc,
                                                          const typename cplx_of<T>::type* __restrict__ tw) {
    using C = typename cplx_of<T>::type;
    constexpr int LP = strided_cfg<T, N>::LP, TC = strided_cfg<T, N>::TC;
    constexpr int EL = TC * N;
    __shared__ C s[TC * LP];
    const int c0 = blockIdx.x * TC;
    const int nc = min(TC, ncols - c0);
    C* base = data + int64_t(blockIdx.y) * plane_stride + c0;
    for (int e = threadIdx.x; e < EL; e += kThreads) {
        const int col = e % TC, pos = e / TC;
        if (col < nc) s[col * LP + pos] = base[int64_t(pos) * stride + col];
    }
    lds_fft<C, N, LP, TC, INV>(s, tw, nc);
    for (int e = threadIdx.x; e < EL; e += kThreads) {
        const int col = e % TC, pos = e / TC;
        if (col < nc) {
            C v = s[col * LP + pos];
            if (zero_dc && blockIdx.y == 0 && c0 + col == 0 && pos == 0) v = C{T(0), T(0)};
            base[int64_t(pos) * stride + col] = v;
        }
    }
}

template <typename T, int N, bool INV>
inline void launch_c2c_strided(typename cplx_of<T>::type* data, int n_planes, int64_t plane_stride, int ncols,
                               int64_t stride, bool zero_dc, const typename cplx_of<T>::type* tw,
                               hipStream_t stream) {
    constexpr int TC = strided_cfg<T, N>::TC;
    const int tiles = (ncols + TC - 1) / TC;
    hipLaunchKernelGGL((k_c2c_strided<T, N, INV>), dim3(tiles, n_planes), dim3(kThreads), 0, stream, data,
                       plane_stride, ncols, stride, zero_dc ? 1 : 0, tw);
}

}  // namespace hermes
