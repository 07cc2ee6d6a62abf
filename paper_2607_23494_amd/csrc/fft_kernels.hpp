// Pass kernels of the 3-D real FFT on an N^3 grid.
//
// Forward: (1) r2c along z with the contrast delta = eps/eps_bar - 1 fused
// into the load, (2) c2c along y, (3) c2c along x.  Each pass reads and
// writes HBM once.  The strided (column) passes stage a tile of TC adjacent
// columns times the full line length in LDS in the interleaved layout, with
// all of a thread's global loads issued before the first is consumed and
// 16-byte accesses where the layout is 16-byte aligned.
#pragma once

#include "fft_core.hpp"

namespace hermes {

template <typename T> struct fft_cfg;
template <> struct fft_cfg<float> { static constexpr int elems = 8192; };   // complex per 64 KB tile
template <> struct fft_cfg<double> { static constexpr int elems = 4096; };

constexpr int kColThreads = 512;   // threads of the column-pass workgroups

// Column tile geometry: TC columns x N positions for NT threads (default
// kColThreads), each owning VEC adjacent columns (one 8- or 16-byte access) at
// 8 positions N/8 apart; LPR lanes per tile row, RPP = N/8 rows per load round.
template <typename T, int N, int VEC_ = 16 / int(sizeof(typename cplx_of<T>::type)), int NT_ = kColThreads>
struct col_cfg {
    using C = typename cplx_of<T>::type;
    static constexpr int VEC = VEC_;
    static constexpr int NT = NT_;
    static constexpr int TC = NT * 8 * VEC / N;
    static constexpr int LPR = TC / VEC;
    static constexpr int RPP = NT / LPR;
    static constexpr int NLD = N / RPP;
    static_assert(TC >= VEC && NLD == 8 && RPP == N / 8, "column tile");
};

// Row pitch (complex elements) of the internal padded half spectra: N/2+1
// rounded up to 16, so every row starts on a 128-byte boundary.
template <int N> constexpr int pitch_of() { return ((N / 2 + 1) + 15) / 16 * 16; }
inline int pitch_rt(int n) { return ((n / 2 + 1) + 15) / 16 * 16; }

template <typename T> inline const typename cplx_of<T>::type* tw_ptr(const Tables& t);
template <> inline const float2* tw_ptr<float>(const Tables& t) { return t.tw32; }
template <> inline const double2* tw_ptr<double>(const Tables& t) { return t.tw64; }

// 16-byte vector of complex values
template <typename C> struct vec_of;
template <> struct vec_of<float2> { using type = float4; };
template <> struct vec_of<double2> { using type = double2; };

template <typename C, int VEC>
__device__ __forceinline__ void vec_split(const typename vec_of<C>::type& v, C* out) {
    if constexpr (VEC == 2) {
        out[0] = C{v.x, v.y};
        out[1] = C{v.z, v.w};
    } else {
        out[0] = v;
    }
}

template <typename C, int VEC>
__device__ __forceinline__ typename vec_of<C>::type vec_join(const C* in) {
    if constexpr (VEC == 2) {
        return typename vec_of<C>::type{in[0].x, in[0].y, in[1].x, in[1].y};
    } else {
        return in[0];
    }
}

// Streaming load of one complex value or one 16-byte vector, marked
// non-temporal: for rows read once and whole (the z pass).  Not for the
// column passes, whose neighbouring tiles share cache lines.
typedef float f32x2_nt __attribute__((ext_vector_type(2)));
typedef float f32x4_nt __attribute__((ext_vector_type(4)));
typedef double f64x2_nt __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 ld_stream(const float2* p) {
    const f32x2_nt v = __builtin_nontemporal_load(reinterpret_cast<const f32x2_nt*>(p));
    return float2{v.x, v.y};
}
__device__ __forceinline__ double2 ld_stream(const double2* p) {
    const f64x2_nt v = __builtin_nontemporal_load(reinterpret_cast<const f64x2_nt*>(p));
    return double2{v.x, v.y};
}
// Non-temporal store of one complex value.
__device__ __forceinline__ void st_stream(float2* p, float2 v) {
    __builtin_nontemporal_store(f32x2_nt{v.x, v.y}, reinterpret_cast<f32x2_nt*>(p));
}
__device__ __forceinline__ void st_stream(double2* p, double2 v) {
    __builtin_nontemporal_store(f64x2_nt{v.x, v.y}, reinterpret_cast<f64x2_nt*>(p));
}
__device__ __forceinline__ float4 ld_stream(const float4* p) {
    const f32x4_nt v = __builtin_nontemporal_load(reinterpret_cast<const f32x4_nt*>(p));
    return float4{v.x, v.y, v.z, v.w};
}

// Load VEC consecutive complex values at src (columns lc.. of a tile with nc
// valid columns); 16-byte access when allowed and fully valid.
template <typename C, int VEC, bool VECLD>
__device__ __forceinline__ void load_cols(const C* src, int lc, int nc, C* out) {
    using V = typename vec_of<C>::type;
    if constexpr (VEC == 1) {
        out[0] = lc < nc ? src[0] : C{0, 0};
    } else if (VECLD && lc + VEC <= nc) {
        vec_split<C, VEC>(*reinterpret_cast<const V*>(src), out);
    } else {
#pragma unroll
        for (int v = 0; v < VEC; ++v) out[v] = lc + v < nc ? src[v] : C{0, 0};
    }
}

template <typename C, int VEC, bool VECLD>
__device__ __forceinline__ void store_cols(C* dst, int lc, int nc, const C* in) {
    using V = typename vec_of<C>::type;
    if constexpr (VEC == 1) {
        if (lc < nc) dst[0] = in[0];
    } else if (VECLD && lc + VEC <= nc) {
        *reinterpret_cast<V*>(dst) = vec_join<C, VEC>(in);
    } else {
#pragma unroll
        for (int v = 0; v < VEC; ++v)
            if (lc + v < nc) dst[v] = in[v];
    }
}

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
    constexpr int EPT = LINES * M / kThreads;
    __shared__ C s[LINES * LP];
    const int row0 = blockIdx.x * LINES;
    const int nl = min(LINES, ROWS - row0);
    const double inv_mean = double(N) * double(N) * double(N) / sum_w[0];
    const C* src = reinterpret_cast<const C*>(eps) + int64_t(row0) * M;   // real pairs
    C pre[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int e = threadIdx.x + i * kThreads;
        pre[i] = e < nl * M ? src[e] : C{0, 0};
    }
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int e = threadIdx.x + i * kThreads;
        if (e < nl * M) {
            const C d{T(double(pre[i].x) * inv_mean - 1.0), T(double(pre[i].y) * inv_mean - 1.0)};
            if (delta_out) reinterpret_cast<C*>(delta_out)[int64_t(row0) * M + e] = d;
            s[e] = d;   // line e / M, element e % M, LP == M
        }
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

// ---------------------------------------------------------------- column c2c
// In-place FFT along an axis of length N with element stride `stride`, for
// `ncols` contiguous columns in each of gridDim.y planes.  zero_dc clears
// element 0 of plane 0 after the transform.  VECLD requires 16-byte aligned
// rows (stride, plane_stride and the base pointer multiples of VEC).
template <typename T, int N, bool INV, bool VECLD, int VEC_>
__global__ __launch_bounds__(kColThreads) void k_c2c_cols(typename cplx_of<T>::type* __restrict__ data,
                                                       int64_t plane_stride, int ncols, int64_t stride,
                                                       int zero_dc,
                                                       const typename cplx_of<T>::type* __restrict__ tw) {
    using C = typename cplx_of<T>::type;
    using G = col_cfg<T, N, VEC_>;
    constexpr int TC = G::TC, VEC = G::VEC, LPR = G::LPR, RPP = G::RPP, NLD = G::NLD;
    __shared__ C s[N * TC];
    __shared__ C twl[N];
    stage_twiddles<C, N, kColThreads>(twl, tw);
    const int c0 = blockIdx.x * TC;
    const int nc = min(TC, ncols - c0);
    C* base = data + int64_t(blockIdx.y) * plane_stride + c0;
    const int lc = (threadIdx.x % LPR) * VEC, r0 = threadIdx.x / LPR;
    C buf[NLD][VEC];
#pragma unroll
    for (int i = 0; i < NLD; ++i) load_cols<C, VEC, VECLD>(base + int64_t(r0 + i * RPP) * stride + lc, lc, nc, buf[i]);
    const bool dc_tile = zero_dc && blockIdx.y == 0 && c0 == 0;
    auto st = [&](int p, int line, C v) {
        if (line < nc) base[int64_t(p) * stride + line] = (dc_tile && p == 0 && line == 0) ? C{0, 0} : v;
    };
    col_fft<C, N, TC, VEC, INV, kColThreads, 0>(s, twl, buf, lc, r0, st);
}

// Tiles of 8-byte columns: more, smaller workgroups per CU keep more loads in
// flight than 16-byte tiles, which these strided column passes need; at
// N = 1024 that tile is only four float columns (32-byte row segments), so
// there a thread takes two.
template <typename T, int N> constexpr int c2c_vec() { return sizeof(T) == 4 && N >= 1024 ? 2 : 1; }

template <typename T, int N, bool INV, bool VECLD>
inline void launch_c2c_cols(typename cplx_of<T>::type* data, int n_planes, int64_t plane_stride, int ncols,
                            int64_t stride, bool zero_dc, const typename cplx_of<T>::type* tw, hipStream_t stream) {
    constexpr int VEC = c2c_vec<T, N>();
    constexpr int TC = col_cfg<T, N, VEC>::TC;
    const int tiles = (ncols + TC - 1) / TC;
    hipLaunchKernelGGL((k_c2c_cols<T, N, INV, VECLD, VEC>), dim3(tiles, n_planes), dim3(kColThreads), 0, stream, data,
                       plane_stride, ncols, stride, zero_dc ? 1 : 0, tw);
}

}  // namespace hermes
