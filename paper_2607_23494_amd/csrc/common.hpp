// Internal declarations shared by the HIP translation units of libhermes.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "hermes.h"

namespace hermes {

constexpr int kThreads = 256;      // threads per workgroup for every kernel
constexpr int kMaxN = 1024;        // largest grid per axis
constexpr int kTwTable = 2 * 2048; // twiddle entries: table for length L at [L, 2L)
constexpr int kDb2Level = 12;      // the D4 function is tabulated at x = i / 2^12, x in [0, 3]
constexpr int kDb2Tab = 3 * (1 << kDb2Level) + 1;

// Per-device constant tables owned by a context.
struct Tables {
    float2* tw32 = nullptr;     // exp(-2 pi i m / L) at tw[L + m], L = 1..2048 (powers of 2)
    double2* tw64 = nullptr;
    double* phi1d = nullptr;    // sinc^8(pi n~/N) at phi1d[N + i], i in [0, N)
    double* b7dft = nullptr;    // sum_{|d|<=3} B7(d) cos(2 pi d i / N) at b7dft[N + i]
    double* phi1d_db2 = nullptr;   // |phi^(2 pi n~/N)|^2 of the D4 function, same layout
    double* ones = nullptr;        // 1 at every index: the D4 self-pair kernel (orthonormal basis)
    double* db2tab = nullptr;      // D4 phi at x = i / 2^kDb2Level, i < kDb2Tab
    double* gl = nullptr;       // kGLSub (16) Gauss-Legendre nodes, then their weights, on [-1, 1]
    int* q2rank = nullptr;      // rank of q among the sums of two squares a^2 + b^2 (-1 if none), q <= 2 (kMaxN/2)^2
    int* rank2q = nullptr;      // the sums of two squares in increasing order
};

// Optional per-kernel timing: launches are bracketed with HIP events on the
// launch stream; durations are collected when the records are read.
struct Profiler {
    bool on = false;
    std::mutex mu;
    struct Pending {
        const char* name;
        hipEvent_t a, b;
    };
    std::vector<hipEvent_t> pool;
    std::vector<Pending> pending;
    std::map<std::string, std::pair<int64_t, double>> acc;   // name -> (launches, total ms)
};

}  // namespace hermes

struct hermes_ctx_s {
    int device = 0;
    int cus = 256;                // compute units of the device
    int basis = HERMES_BASIS_B3;  // scaling function of every basis-dependent call
    hermes::Tables t;
    hermes::Profiler prof;
    void* xi_scratch = nullptr;   // device address of the static 2PCF scratch array on this device
    int nq2[11] = {};             // sums of two squares <= 2 (N/2)^2, indexed by log2 N
};

namespace hermes {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
hermes_status fail(hermes_status st, const std::string& msg);
hermes_status check_launch(const char* what);

// Brackets one kernel launch with timing events when profiling is on.
class LaunchScope {
public:
    LaunchScope(hermes_ctx c, hipStream_t s, const char* name);
    ~LaunchScope();
    LaunchScope(const LaunchScope&) = delete;
    LaunchScope& operator=(const LaunchScope&) = delete;

private:
    hermes_ctx c_;
    hipStream_t s_;
    const char* name_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
};

inline bool valid_n(int n) { return n >= 8 && n <= kMaxN && (n & (n - 1)) == 0; }

// ---------------------------------------------------------------- basis
// Per-axis basis kernel Phi^ and self-pair kernel of the context's basis.
inline const double* basis_phi1d(hermes_ctx c) {
    return c->basis == HERMES_BASIS_DB2 ? c->t.phi1d_db2 : c->t.phi1d;
}
inline const double* basis_selfdft(hermes_ctx c) {
    return c->basis == HERMES_BASIS_DB2 ? c->t.ones : c->t.b7dft;
}
// Host tables of the D4 function (basis.hip).
std::vector<double> db2_phi_table();
double db2_phi_hat_sq(double w);
void db2_gamma_factors(double lam[5], double vec[5][5]);

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// ---------------------------------------------------------------- types
template <typename T> struct cplx_of;
template <> struct cplx_of<float> { using type = float2; };
template <> struct cplx_of<double> { using type = double2; };

template <typename T> struct tw_of;

// Bin edges passed by value to kernels.
struct Edges {
    double e[HERMES_MAX_BINS + 1];
    int n_bins;
};

// Workspace layout helpers (bytes, 256-aligned).
inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

inline int64_t qmax_of(int n) { return 3LL * (n / 2) * (n / 2); }

// ---------------------------------------------------------------- entry points
// (implemented per translation unit, dispatched by dtype / N)
hermes_status assign_impl(hermes_ctx ctx, const float* pos, const float* weight, int64_t n_pts,
                          double box_L, int n, int dtype, void* eps, double* sum_w, void* work,
                          hipStream_t stream);
size_t assign_workspace(int n, int64_t n_pts);
hermes_status fft_impl(hermes_ctx ctx, const void* eps, const double* sum_w, int n, int dtype,
                       void* delta_k, void* delta, hipStream_t stream);
hermes_status xi_impl(hermes_ctx ctx, const void* delta_k, int n, int dtype, double box_L,
                      const Edges& edges, const int* ells, int n_ells, int los_axis, double* xi,
                      double* shot, void* work, size_t work_bytes, hipStream_t stream);
size_t xi_workspace(int n, int n_ells, int n_bins);
// The static scratch array of the allocation-free 2PCF entry point.
constexpr size_t kXiStaticBytes = size_t(16) << 20;
hermes_status xi_static_init(hermes_ctx ctx);
hermes_status filter_impl(hermes_ctx ctx, const void* delta_k, int n, int dtype, double box_L,
                          const hermes_window* win, int n_win, void* out, double* moments,
                          void* work, size_t work_bytes, hipStream_t stream);
size_t filter_workspace(int n, int dtype, int n_win);
hermes_status zeta_impl(hermes_ctx ctx, const float* delta, const void* delta_k, int n,
                        double box_L, const Edges& edges, int l_max, int precision, double* zeta,
                        void* work, size_t work_bytes, hipStream_t stream);
size_t zeta_workspace(int n, int n_bins);
hermes_status xi_aniso_impl(hermes_ctx ctx, const void* delta_k, int n, int dtype, double box_L,
                            const hermes_aniso_window* win, int n_win, int los_axis, double* xi, void* work,
                            hipStream_t stream);
size_t aniso_workspace(hermes_ctx ctx, int n, int n_win);
hermes_status triplet_impl(hermes_ctx ctx, const void* f1, const void* f2, const void* f3, int n, int dtype,
                           double box_L, const float* centres, const float* weights, int64_t n_centres, double r12,
                           double r13, int n_theta, int n_rot, uint64_t seed, double* out, void* work,
                           size_t work_bytes, hipStream_t stream);
size_t triplet_workspace(int n, int dtype, int n_theta, int64_t n_centres);
hermes_status mark_ratio_impl(const double* xim, const double* xi, int n, double* out, hipStream_t stream);
hermes_status gamma_impl(hermes_ctx ctx, const void* eps, const void* fields, int n_fields, int n, int dtype,
                         double* out, void* work, hipStream_t stream);
size_t gamma_workspace();
hermes_status readout_impl(hermes_ctx ctx, const void* fields, int n_fields, int n, int dtype, double box_L,
                           const float* pos, const float* weight, int64_t n_pts, const hermes_mark* mark, void* out,
                           double* moments, void* work, hipStream_t stream);
size_t readout_workspace(int n, int64_t n_pts);

}  // namespace hermes
