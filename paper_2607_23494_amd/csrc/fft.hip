// Forward transform of the density contrast (Sec. 4.2): delta = eps/eps_bar - 1
// fused into an r2c pass along z, then c2c passes along y and x; the k = 0
// mode is cleared in the last pass.
#include "common.hpp"
#include "fft_kernels.hpp"

namespace hermes {

template <typename T, int N>
static hermes_status fft_n(hermes_ctx ctx, const void* eps, const double* sum_w, void* delta_k, void* delta,
                           hipStream_t stream) {
    using C = typename cplx_of<T>::type;
    constexpr int M = N / 2, P = M + 1;
    constexpr int LINES = fft_cfg<T>::elems / M;
    const C* tw = tw_ptr<T>(ctx->t);
    C* dk = static_cast<C*>(delta_k);
    const int rows = N * N;
    {
        LaunchScope ls(ctx, stream, "fwd_z");
        hipLaunchKernelGGL((k_fwd_z<T, N>), dim3((rows + LINES - 1) / LINES), dim3(kThreads), 0, stream,
                           static_cast<const T*>(eps), sum_w, static_cast<T*>(delta), dk, tw);
    }
    {   // y: N planes (one per x), P columns, stride P
        LaunchScope ls(ctx, stream, "fwd_y");
        launch_c2c_cols<T, N, false, false>(dk, N, int64_t(N) * P, P, P, false, tw, stream);
    }
    {   // x: one plane of N*P columns, stride N*P
        LaunchScope ls(ctx, stream, "fwd_x");
        launch_c2c_cols<T, N, false, true>(dk, 1, 0, N * P, int64_t(N) * P, true, tw, stream);
    }
    return check_launch("hermes_fft");
}

hermes_status fft_impl(hermes_ctx ctx, const void* eps, const double* sum_w, int n, int dtype, void* delta_k,
                       void* delta, hipStream_t stream) {
#define HERMES_FFT_CASE(NN)                                                                      \
    case NN:                                                                                     \
        return dtype == HERMES_F32 ? fft_n<float, NN>(ctx, eps, sum_w, delta_k, delta, stream) \
                                   : fft_n<double, NN>(ctx, eps, sum_w, delta_k, delta, stream);
    switch (n) {
        HERMES_FFT_CASE(8)
        HERMES_FFT_CASE(16)
        HERMES_FFT_CASE(32)
        HERMES_FFT_CASE(64)
        HERMES_FFT_CASE(128)
        HERMES_FFT_CASE(256)
        HERMES_FFT_CASE(512)
        HERMES_FFT_CASE(1024)
        default:
            return fail(HERMES_ERR_ARG, "hermes_fft: unsupported N");
    }
#undef HERMES_FFT_CASE
}

}  // namespace hermes
