// C ABI entry points: argument validation, context tables, dispatch.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <iterator>
#include <string>
#include <vector>

#include "common.hpp"

namespace hermes {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

hermes_status fail(hermes_status st, const std::string& msg) {
    set_error(msg);
    return st;
}

hermes_status check_launch(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(HERMES_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
    return HERMES_OK;
}

LaunchScope::LaunchScope(hermes_ctx c, hipStream_t s, const char* name) : c_(c), s_(s), name_(name) {
    if (!c_ || !c_->prof.on) return;
    std::lock_guard<std::mutex> lk(c_->prof.mu);
    auto take = [&]() {
        hipEvent_t e = nullptr;
        if (!c_->prof.pool.empty()) {
            e = c_->prof.pool.back();
            c_->prof.pool.pop_back();
        } else if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
        }
        return e;
    };
    a_ = take();
    b_ = take();
    if (a_ && b_) {
        (void)hipEventRecord(a_, s_);
    } else {
        if (a_) c_->prof.pool.push_back(a_);
        if (b_) c_->prof.pool.push_back(b_);
        a_ = b_ = nullptr;
    }
}

LaunchScope::~LaunchScope() {
    if (!a_) return;
    (void)hipEventRecord(b_, s_);
    std::lock_guard<std::mutex> lk(c_->prof.mu);
    c_->prof.pending.push_back({name_, a_, b_});
}

// Gauss-Legendre nodes and weights on [-1, 1] by Newton iteration on P_n.
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.resize(n);
    w.resize(n);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

static hermes_status build_tables(hermes_ctx c) {
    std::vector<float2> tw32(kTwTable);
    std::vector<double2> tw64(kTwTable);
    for (int L = 1; L <= kTwTable / 2; L *= 2) {
        for (int m = 0; m < L; ++m) {
            const double a = -2.0 * M_PI * double(m) / double(L);
            tw64[L + m] = double2{std::cos(a), std::sin(a)};
            tw32[L + m] = float2{float(std::cos(a)), float(std::sin(a))};
        }
    }
    std::vector<double> phi(2 * kMaxN, 0.0);
    for (int n = 1; n <= kMaxN; n *= 2) {
        for (int i = 0; i < n; ++i) {
            const int s = i <= n / 2 ? i : i - n;
            const double a = M_PI * double(s) / double(n);
            const double sn = s == 0 ? 1.0 : std::sin(a) / a;
            phi[n + i] = std::pow(sn, 8);
        }
    }
    // DFT of the B3 autocorrelation at integer lags, the centred B-spline of
    // degree 7: B7(0) = 2416/5040, B7(+-1) = 1191/5040, B7(+-2) = 120/5040,
    // B7(+-3) = 1/5040 (the self-pair kernel of the shot-noise factor)
    std::vector<double> b7(2 * kMaxN, 0.0);
    {
        const double c[4] = {2416.0 / 5040.0, 1191.0 / 5040.0, 120.0 / 5040.0, 1.0 / 5040.0};
        for (int n = 1; n <= kMaxN; n *= 2)
            for (int i = 0; i < n; ++i) {
                double v = c[0];
                for (int d = 1; d <= 3; ++d) v += 2.0 * c[d] * std::cos(2.0 * M_PI * double(d) * double(i) / double(n));
                b7[n + i] = v;
            }
    }
    // the D4 basis: |phi^|^2 per axis, the self-pair kernel (1: orthonormal)
    // and the dyadic table of phi
    std::vector<double> phi_db2(2 * kMaxN, 0.0), ones(2 * kMaxN, 1.0);
    for (int n = 1; n <= kMaxN; n *= 2)
        for (int i = 0; i < n; ++i) {
            const int s = i <= n / 2 ? i : i - n;
            phi_db2[n + i] = db2_phi_hat_sq(2.0 * M_PI * double(s) / double(n));
        }
    const std::vector<double> db2tab = db2_phi_table();
    if (db2tab.size() != size_t(kDb2Tab)) return fail(HERMES_ERR_HIP, "hermes_create: D4 table size");
    std::vector<double> gx, gw;
    gauss_legendre(16, gx, gw);
    std::vector<double> gl(32);
    for (int i = 0; i < 16; ++i) {
        gl[i] = gx[i];
        gl[16 + i] = gw[i];
    }
    // sums of two squares a^2 + b^2 up to 2 (kMaxN/2)^2 (the transverse |n_perp|^2
    // of the anisotropic 2PCF), their ranks, and how many lie below 2 (N/2)^2
    const int qmax2 = 2 * (kMaxN / 2) * (kMaxN / 2);
    std::vector<int> q2rank(size_t(qmax2) + 1, -1), rank2q;
    for (int a = 0; a * a <= qmax2; ++a)
        for (int b = a; a * a + b * b <= qmax2; ++b) q2rank[size_t(a) * a + size_t(b) * b] = 0;
    for (int q = 0; q <= qmax2; ++q)
        if (q2rank[q] == 0) {
            q2rank[q] = int(rank2q.size());
            rank2q.push_back(q);
        }
    for (int n = 1, lg = 0; n <= kMaxN; n *= 2, ++lg) {
        const int lim = 2 * (n / 2) * (n / 2);
        int cnt = 0;
        while (cnt < int(rank2q.size()) && rank2q[cnt] <= lim) ++cnt;
        c->nq2[lg] = cnt;
    }
    auto up = [](void** dst, const void* src, size_t bytes) -> hipError_t {
        hipError_t e = hipMalloc(dst, bytes);
        if (e != hipSuccess) return e;
        return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
    };
    hipError_t e;
    if ((e = up((void**)&c->t.tw32, tw32.data(), tw32.size() * sizeof(float2))) != hipSuccess ||
        (e = up((void**)&c->t.tw64, tw64.data(), tw64.size() * sizeof(double2))) != hipSuccess ||
        (e = up((void**)&c->t.phi1d, phi.data(), phi.size() * sizeof(double))) != hipSuccess ||
        (e = up((void**)&c->t.b7dft, b7.data(), b7.size() * sizeof(double))) != hipSuccess ||
        (e = up((void**)&c->t.phi1d_db2, phi_db2.data(), phi_db2.size() * sizeof(double))) != hipSuccess ||
        (e = up((void**)&c->t.ones, ones.data(), ones.size() * sizeof(double))) != hipSuccess ||
        (e = up((void**)&c->t.db2tab, db2tab.data(), db2tab.size() * sizeof(double))) != hipSuccess ||
        (e = up((void**)&c->t.gl, gl.data(), gl.size() * sizeof(double))) != hipSuccess ||
        (e = up((void**)&c->t.q2rank, q2rank.data(), q2rank.size() * sizeof(int))) != hipSuccess ||
        (e = up((void**)&c->t.rank2q, rank2q.data(), rank2q.size() * sizeof(int))) != hipSuccess)
        return fail(HERMES_ERR_HIP, std::string("hermes_create: ") + hipGetErrorString(e));
    return HERMES_OK;
}

// Bin edges: strictly increasing, edges[0] >= 0 and every edge below L/2 (a
// separation of L/2 or more reaches the periodic image of the box).
static hermes_status get_edges(const double* edges, int n_bins, double box_L, Edges& out, const char* who) {
    if (!edges) return fail(HERMES_ERR_ARG, std::string(who) + ": edges is NULL");
    if (n_bins < 1 || n_bins > HERMES_MAX_BINS)
        return fail(HERMES_ERR_ARG, std::string(who) + ": n_bins must be in [1, 64]");
    if (!(edges[0] >= 0.0)) return fail(HERMES_ERR_ARG, std::string(who) + ": edges[0] must be >= 0");
    for (int i = 0; i < n_bins; ++i)
        if (!(edges[i + 1] > edges[i]))
            return fail(HERMES_ERR_ARG, std::string(who) + ": edges must be strictly increasing");
    if (!(edges[n_bins] < 0.5 * box_L))
        return fail(HERMES_ERR_ARG, std::string(who) + ": edges must be below L/2");
    for (int i = 0; i <= n_bins; ++i) out.e[i] = edges[i];
    out.n_bins = n_bins;
    return HERMES_OK;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

}  // namespace hermes

using namespace hermes;

extern "C" {

const char* hermes_last_error(void) { return g_last_error.c_str(); }

hermes_status hermes_create(hermes_ctx* out, int device) {
    if (!out) return fail(HERMES_ERR_ARG, "hermes_create: out is NULL");
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return fail(HERMES_ERR_ARG, "hermes_create: no such HIP device");
    DeviceGuard g(device);
    hermes_ctx c = new hermes_ctx_s();
    c->device = device;
    {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
            c->cus = cus;
    }
    hermes_status st = build_tables(c);
    if (st == HERMES_OK) st = xi_static_init(c);
    if (st != HERMES_OK) {
        hermes_destroy(c);
        return st;
    }
    *out = c;
    return HERMES_OK;
}

hermes_status hermes_set_basis(hermes_ctx ctx, int basis) {
    if (!ctx) return fail(HERMES_ERR_ARG, "hermes_set_basis: ctx is NULL");
    if (basis != HERMES_BASIS_B3 && basis != HERMES_BASIS_DB2)
        return fail(HERMES_ERR_ARG, "hermes_set_basis: unknown basis");
    ctx->basis = basis;
    return HERMES_OK;
}

int hermes_get_basis(hermes_ctx ctx) { return ctx ? ctx->basis : -1; }

void hermes_destroy(hermes_ctx ctx) {
    if (!ctx) return;
    DeviceGuard g(ctx->device);
    {
        std::lock_guard<std::mutex> lk(ctx->prof.mu);
        for (auto& p : ctx->prof.pending) {
            (void)hipEventSynchronize(p.b);
            (void)hipEventDestroy(p.a);
            (void)hipEventDestroy(p.b);
        }
        for (hipEvent_t e : ctx->prof.pool) (void)hipEventDestroy(e);
        ctx->prof.pending.clear();
        ctx->prof.pool.clear();
    }
    (void)hipFree(ctx->t.q2rank);
    (void)hipFree(ctx->t.rank2q);
    (void)hipFree(ctx->t.tw32);
    (void)hipFree(ctx->t.tw64);
    (void)hipFree(ctx->t.phi1d);
    (void)hipFree(ctx->t.b7dft);
    (void)hipFree(ctx->t.phi1d_db2);
    (void)hipFree(ctx->t.ones);
    (void)hipFree(ctx->t.db2tab);
    (void)hipFree(ctx->t.gl);
    delete ctx;
}

hermes_status hermes_profile_enable(hermes_ctx ctx, int enable) {
    if (!ctx) return fail(HERMES_ERR_ARG, "hermes_profile_enable: NULL context");
    std::lock_guard<std::mutex> lk(ctx->prof.mu);
    ctx->prof.on = enable != 0;
    return HERMES_OK;
}

static void drain(hermes_ctx ctx) {
    for (auto& p : ctx->prof.pending) {
        float ms = 0.f;
        (void)hipEventSynchronize(p.b);
        if (hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess) ms = 0.f;
        auto& acc = ctx->prof.acc[p.name];
        acc.first += 1;
        acc.second += ms;
        ctx->prof.pool.push_back(p.a);
        ctx->prof.pool.push_back(p.b);
    }
    ctx->prof.pending.clear();
}

hermes_status hermes_profile_reset(hermes_ctx ctx) {
    if (!ctx) return fail(HERMES_ERR_ARG, "hermes_profile_reset: NULL context");
    DeviceGuard g(ctx->device);
    std::lock_guard<std::mutex> lk(ctx->prof.mu);
    drain(ctx);
    ctx->prof.acc.clear();
    return HERMES_OK;
}

hermes_status hermes_profile_read(hermes_ctx ctx, int index, char* name, size_t name_len, int64_t* launches,
                                  double* total_ms) {
    if (!ctx || !name || name_len == 0 || !launches || !total_ms)
        return fail(HERMES_ERR_ARG, "hermes_profile_read: NULL argument");
    DeviceGuard g(ctx->device);
    std::lock_guard<std::mutex> lk(ctx->prof.mu);
    drain(ctx);
    if (index < 0 || index >= int(ctx->prof.acc.size()))
        return fail(HERMES_ERR_ARG, "hermes_profile_read: index past the last record");
    auto it = ctx->prof.acc.begin();
    std::advance(it, index);
    std::snprintf(name, name_len, "%s", it->first.c_str());
    *launches = it->second.first;
    *total_ms = it->second.second;
    return HERMES_OK;
}

hermes_status hermes_workspace_size(hermes_ctx ctx, int op, int n_grid, int dtype, int n_batch,
                                    int n_ells, size_t* bytes) {
    if (!ctx || !bytes) return fail(HERMES_ERR_ARG, "hermes_workspace_size: NULL argument");
    if (!valid_n(n_grid)) return fail(HERMES_ERR_ARG, "hermes_workspace_size: N must be a power of two in [8, 1024]");
    if (dtype != HERMES_F32 && dtype != HERMES_F64) return fail(HERMES_ERR_ARG, "hermes_workspace_size: bad dtype");
    switch (op) {
        case HERMES_OP_ASSIGN:
            if (n_batch < 0) return fail(HERMES_ERR_ARG, "hermes_workspace_size: ASSIGN needs n_batch = points >= 0");
            *bytes = assign_workspace(n_grid, n_batch);
            return HERMES_OK;
        case HERMES_OP_FFT:
            *bytes = 0;
            return HERMES_OK;
        case HERMES_OP_XI:
            if (n_ells < 1 || n_ells > HERMES_MAX_ELLS || n_batch < 1 || n_batch > HERMES_MAX_BINS)
                return fail(HERMES_ERR_ARG, "hermes_workspace_size: XI needs 1..8 multipoles and 1..64 bins");
            *bytes = xi_workspace(n_grid, n_ells, n_batch);
            return HERMES_OK;
        case HERMES_OP_FILTER:
            if (n_batch < 1) return fail(HERMES_ERR_ARG, "hermes_workspace_size: FILTER needs n_batch >= 1");
            *bytes = filter_workspace(n_grid, dtype, n_batch);
            return HERMES_OK;
        case HERMES_OP_XI_ANISO:
            if (n_batch < 1 || n_batch > HERMES_MAX_ANISO)
                return fail(HERMES_ERR_ARG, "hermes_workspace_size: XI_ANISO needs 1..2^20 windows");
            *bytes = aniso_workspace(ctx, n_grid, n_batch);
            return HERMES_OK;
        case HERMES_OP_TRIPLET:
            if (n_batch < 1 || n_batch > HERMES_MAX_THETA)
                return fail(HERMES_ERR_ARG, "hermes_workspace_size: TRIPLET needs 1..64 opening angles");
            if (n_ells < 0) return fail(HERMES_ERR_ARG, "hermes_workspace_size: TRIPLET needs n_ells (centres) >= 0");
            *bytes = triplet_workspace(n_grid, dtype, n_batch, n_ells);
            return HERMES_OK;
        case HERMES_OP_DDD_GAMMA:
            *bytes = gamma_workspace();
            return HERMES_OK;
        case HERMES_OP_READOUT:
            if (n_batch < 0) return fail(HERMES_ERR_ARG, "hermes_workspace_size: READOUT needs n_batch >= 0");
            *bytes = readout_workspace(n_grid, n_batch);
            return HERMES_OK;
        case HERMES_OP_ZETA:
            if (dtype != HERMES_F32) return fail(HERMES_ERR_UNSUPPORTED, "hermes_workspace_size: ZETA runs in float32");
            if (n_batch < 1 || n_batch > HERMES_MAX_BINS)
                return fail(HERMES_ERR_ARG, "hermes_workspace_size: ZETA needs 1..64 bins");
            *bytes = zeta_workspace(n_grid, n_batch);
            return HERMES_OK;
        default:
            return fail(HERMES_ERR_ARG, "hermes_workspace_size: unknown op");
    }
}

hermes_status hermes_assign(hermes_ctx ctx, const float* pos, const float* weight, int64_t n_pts,
                            double box_L, int n_grid, int dtype, void* eps, double* sum_w, void* work,
                            size_t work_bytes, hipStream_t stream) {
    if (!ctx || !eps || !sum_w || !work || (n_pts > 0 && !pos))
        return fail(HERMES_ERR_ARG, "hermes_assign: NULL argument");
    if (n_pts < 0) return fail(HERMES_ERR_ARG, "hermes_assign: n_pts < 0");
    if (n_pts > int64_t(UINT32_MAX)) return fail(HERMES_ERR_ARG, "hermes_assign: more than 2^32 - 1 points");
    if (!(box_L > 0.0)) return fail(HERMES_ERR_ARG, "hermes_assign: box_L must be > 0");
    if (!valid_n(n_grid)) return fail(HERMES_ERR_ARG, "hermes_assign: N must be a power of two in [8, 1024]");
    if (dtype != HERMES_F32 && dtype != HERMES_F64) return fail(HERMES_ERR_ARG, "hermes_assign: bad dtype");
    if (work_bytes < assign_workspace(n_grid, n_pts)) return fail(HERMES_ERR_OOM, "hermes_assign: workspace too small");
    DeviceGuard g(ctx->device);
    return assign_impl(ctx, pos, weight, n_pts, box_L, n_grid, dtype, eps, sum_w, work, stream);
}

hermes_status hermes_fft(hermes_ctx ctx, const void* eps, const double* sum_w, int n_grid, int dtype,
                         void* delta_k, void* delta, hipStream_t stream) {
    if (!ctx || !eps || !sum_w || !delta_k) return fail(HERMES_ERR_ARG, "hermes_fft: NULL argument");
    if (!valid_n(n_grid)) return fail(HERMES_ERR_ARG, "hermes_fft: N must be a power of two in [8, 1024]");
    if (dtype != HERMES_F32 && dtype != HERMES_F64) return fail(HERMES_ERR_ARG, "hermes_fft: bad dtype");
    DeviceGuard g(ctx->device);
    return fft_impl(ctx, eps, sum_w, n_grid, dtype, delta_k, delta, stream);
}

hermes_status hermes_xi(hermes_ctx ctx, const void* delta_k, int n_grid, int dtype, double box_L,
                        const double* edges, int n_bins, const int* ells, int n_ells, int los_axis,
                        double* xi, double* shot, void* work, size_t work_bytes, hipStream_t stream) {
    if (!ctx || !delta_k || !xi || !ells || !work) return fail(HERMES_ERR_ARG, "hermes_xi: NULL argument");
    if (!valid_n(n_grid)) return fail(HERMES_ERR_ARG, "hermes_xi: N must be a power of two in [8, 1024]");
    if (dtype != HERMES_F32 && dtype != HERMES_F64) return fail(HERMES_ERR_ARG, "hermes_xi: bad dtype");
    if (!(box_L > 0.0)) return fail(HERMES_ERR_ARG, "hermes_xi: box_L must be > 0");
    if (los_axis < 0 || los_axis > 2) return fail(HERMES_ERR_ARG, "hermes_xi: los_axis must be 0, 1 or 2");
    if (n_ells < 1 || n_ells > HERMES_MAX_ELLS) return fail(HERMES_ERR_ARG, "hermes_xi: n_ells must be in [1, 8]");
    for (int i = 0; i < n_ells; ++i)
        if (ells[i] < 0 || ells[i] > HERMES_MAX_LMAX || (ells[i] & 1))
            return fail(HERMES_ERR_ARG, "hermes_xi: multipoles must be even and in [0, 16]");
    Edges e;
    hermes_status st = get_edges(edges, n_bins, box_L, e, "hermes_xi");
    if (st != HERMES_OK) return st;
    if (work_bytes < xi_workspace(n_grid, n_ells, n_bins))
        return fail(HERMES_ERR_OOM, "hermes_xi: workspace too small");
    DeviceGuard g(ctx->device);
    return xi_impl(ctx, delta_k, n_grid, dtype, box_L, e, ells, n_ells, los_axis, xi, shot, work, work_bytes,
                   stream);
}

hermes_status hermes_xi_static(hermes_ctx ctx, const void* delta_k, int n_grid, int dtype, double box_L,
                               const double* edges, int n_bins, const int* ells, int n_ells, int los_axis,
                               double* xi, double* shot, hipStream_t stream) {
    if (!ctx || !delta_k || !xi || !ells) return fail(HERMES_ERR_ARG, "hermes_xi_static: NULL argument");
    if (!valid_n(n_grid)) return fail(HERMES_ERR_ARG, "hermes_xi_static: N must be a power of two in [8, 1024]");
    if (dtype != HERMES_F32 && dtype != HERMES_F64) return fail(HERMES_ERR_ARG, "hermes_xi_static: bad dtype");
    if (!(box_L > 0.0)) return fail(HERMES_ERR_ARG, "hermes_xi_static: box_L must be > 0");
    if (los_axis < 0 || los_axis > 2) return fail(HERMES_ERR_ARG, "hermes_xi_static: los_axis must be 0, 1 or 2");
    if (n_ells < 1 || n_ells > HERMES_MAX_ELLS)
        return fail(HERMES_ERR_ARG, "hermes_xi_static: n_ells must be in [1, 8]");
    for (int i = 0; i < n_ells; ++i)
        if (ells[i] < 0 || ells[i] > HERMES_MAX_LMAX || (ells[i] & 1))
            return fail(HERMES_ERR_ARG, "hermes_xi_static: multipoles must be even and in [0, 16]");
    Edges e;
    hermes_status st = get_edges(edges, n_bins, box_L, e, "hermes_xi_static");
    if (st != HERMES_OK) return st;
    const size_t need = xi_workspace(n_grid, n_ells, n_bins);
    if (need > kXiStaticBytes)
        return fail(HERMES_ERR_UNSUPPORTED, "hermes_xi_static: needs " + std::to_string(need) +
                                                " bytes of scratch; the static array holds " +
                                                std::to_string(kXiStaticBytes));
    if (!ctx->xi_scratch) return fail(HERMES_ERR_HIP, "hermes_xi_static: static scratch not resolved");
    DeviceGuard g(ctx->device);
    return xi_impl(ctx, delta_k, n_grid, dtype, box_L, e, ells, n_ells, los_axis, xi, shot, ctx->xi_scratch,
                   kXiStaticBytes, stream);
}

hermes_status hermes_xi_aniso(hermes_ctx ctx, const void* delta_k, int n_grid, int dtype, double box_L,
                              const hermes_aniso_window* win, int n_win, int los_axis, double* xi, void* work,
                              size_t work_bytes, hipStream_t stream) {
    if (!ctx || !delta_k || !win || !xi || !work) return fail(HERMES_ERR_ARG, "hermes_xi_aniso: NULL argument");
    if (!valid_n(n_grid)) return fail(HERMES_ERR_ARG, "hermes_xi_aniso: N must be a power of two in [8, 1024]");
    if (dtype != HERMES_F32 && dtype != HERMES_F64) return fail(HERMES_ERR_ARG, "hermes_xi_aniso: bad dtype");
    if (!(box_L > 0.0) || !std::isfinite(box_L)) return fail(HERMES_ERR_ARG, "hermes_xi_aniso: box_L must be > 0");
    if (los_axis < 0 || los_axis > 2) return fail(HERMES_ERR_ARG, "hermes_xi_aniso: los_axis must be 0, 1 or 2");
    if (n_win < 1 || n_win > HERMES_MAX_ANISO)
        return fail(HERMES_ERR_ARG, "hermes_xi_aniso: n_win must be in [1, 2^20]");
    for (int i = 0; i < n_win; ++i) {
        const hermes_aniso_window& w = win[i];
        const std::string at = "hermes_xi_aniso: window " + std::to_string(i) + ": ";
        if (w.reserved != 0) return fail(HERMES_ERR_ARG, at + "reserved must be 0");
        if (w.kind < HERMES_ANISO_RING || w.kind > HERMES_ANISO_GAUSS_SHELL)
            return fail(HERMES_ERR_ARG, at + "unknown kind");
        const double p[4] = {w.r_perp, w.r_par, w.d_perp, w.d_par};
        for (double v : p)
            if (!std::isfinite(v) || v < 0.0) return fail(HERMES_ERR_ARG, at + "parameters must be finite and >= 0");
        if (!(w.r_perp < 0.5 * box_L) || !(w.r_par < 0.5 * box_L))
            return fail(HERMES_ERR_ARG, at + "r_perp and r_par must be below L/2");
        if (w.kind == HERMES_ANISO_RING_BIN && (!(w.d_perp > 0.0) || !(w.r_perp >= 0.5 * w.d_perp)))
            return fail(HERMES_ERR_ARG, at + "RING_BIN needs d_perp > 0 and r_perp >= d_perp / 2");
        if (w.kind == HERMES_ANISO_GAUSS_SHELL && !(w.r_perp > 0.0 || w.d_perp > 0.0))
            return fail(HERMES_ERR_ARG, at + "GAUSS_SHELL needs r_perp > 0 or d_perp > 0");
    }
    if (work_bytes < aniso_workspace(ctx, n_grid, n_win))
        return fail(HERMES_ERR_OOM, "hermes_xi_aniso: workspace too small");
    DeviceGuard g(ctx->device);
    return xi_aniso_impl(ctx, delta_k, n_grid, dtype, box_L, win, n_win, los_axis, xi, work, stream);
}

hermes_status hermes_mark_ratio(const double* xi_marked, const double* xi, int n, double* out,
                                hipStream_t stream) {
    if (!xi_marked || !xi || !out) return fail(HERMES_ERR_ARG, "hermes_mark_ratio: NULL argument");
    if (n < 0) return fail(HERMES_ERR_ARG, "hermes_mark_ratio: n < 0");
    return mark_ratio_impl(xi_marked, xi, n, out, stream);
}

hermes_status hermes_triplet_mc(hermes_ctx ctx, const void* f1, const void* f2, const void* f3, int n_grid,
                                int dtype, double box_L, const float* centres, const float* weights,
                                int64_t n_centres, double r12, double r13, int n_theta, int n_rot, uint64_t seed,
                                double* out, void* work, size_t work_bytes, hipStream_t stream) {
    if (!ctx || !f2 || !f3 || !out || !work) return fail(HERMES_ERR_ARG, "hermes_triplet_mc: NULL argument");
    if (!valid_n(n_grid)) return fail(HERMES_ERR_ARG, "hermes_triplet_mc: N must be a power of two in [8, 1024]");
    if (dtype != HERMES_F32 && dtype != HERMES_F64) return fail(HERMES_ERR_ARG, "hermes_triplet_mc: bad dtype");
    if (!(box_L > 0.0) || !std::isfinite(box_L)) return fail(HERMES_ERR_ARG, "hermes_triplet_mc: box_L must be > 0");
    if (centres && f1) return fail(HERMES_ERR_ARG, "hermes_triplet_mc: f1 is read at box points only (centres NULL)");
    if (!centres && weights) return fail(HERMES_ERR_ARG, "hermes_triplet_mc: weights need centres");
    if (n_centres < 0) return fail(HERMES_ERR_ARG, "hermes_triplet_mc: n_centres < 0");
    if (n_rot < 1) return fail(HERMES_ERR_ARG, "hermes_triplet_mc: n_rot must be >= 1");
    if (n_centres > (int64_t(1) << 62) / n_rot)
        return fail(HERMES_ERR_ARG, "hermes_triplet_mc: n_centres n_rot must be below 2^62");
    if (n_theta < 1 || n_theta > HERMES_MAX_THETA)
        return fail(HERMES_ERR_ARG, "hermes_triplet_mc: n_theta must be in [1, 64]");
    if (!std::isfinite(r12) || !std::isfinite(r13) || r12 < 0.0 || r13 < 0.0 || !(r12 < 0.5 * box_L) ||
        !(r13 < 0.5 * box_L))
        return fail(HERMES_ERR_ARG, "hermes_triplet_mc: r12 and r13 must be in [0, L/2)");
    if (work_bytes < triplet_workspace(n_grid, dtype, n_theta, 0))
        return fail(HERMES_ERR_OOM, "hermes_triplet_mc: workspace too small");
    DeviceGuard g(ctx->device);
    return triplet_impl(ctx, f1, f2, f3, n_grid, dtype, box_L, centres, weights, n_centres, r12, r13, n_theta, n_rot,
                        seed, out, work, work_bytes, stream);
}

hermes_status hermes_ddd_gamma(hermes_ctx ctx, const void* eps, const void* fields, int n_fields, int n_grid,
                               int dtype, double* out, void* work, size_t work_bytes, hipStream_t stream) {
    if (!ctx || !eps || !fields || !out || !work) return fail(HERMES_ERR_ARG, "hermes_ddd_gamma: NULL argument");
    if (!valid_n(n_grid)) return fail(HERMES_ERR_ARG, "hermes_ddd_gamma: N must be a power of two in [8, 1024]");
    if (dtype != HERMES_F32 && dtype != HERMES_F64) return fail(HERMES_ERR_ARG, "hermes_ddd_gamma: bad dtype");
    if (n_fields < 1 || n_fields > HERMES_MAX_GAMMA_FIELDS)
        return fail(HERMES_ERR_ARG, "hermes_ddd_gamma: n_fields must be in [1, 32]");
    if (work_bytes < gamma_workspace()) return fail(HERMES_ERR_OOM, "hermes_ddd_gamma: workspace too small");
    DeviceGuard g(ctx->device);
    return gamma_impl(ctx, eps, fields, n_fields, n_grid, dtype, out, work, stream);
}

hermes_status hermes_filter_bins(hermes_ctx ctx, const void* delta_k, int n_grid, int dtype,
                                 double box_L, const hermes_window* win, int n_win, void* out,
                                 double* moments, void* work, size_t work_bytes, hipStream_t stream) {
    if (!ctx || !delta_k || !win || !work) return fail(HERMES_ERR_ARG, "hermes_filter_bins: NULL argument");
    if (!out && !moments) return fail(HERMES_ERR_ARG, "hermes_filter_bins: out and moments both NULL");
    if (!valid_n(n_grid)) return fail(HERMES_ERR_ARG, "hermes_filter_bins: N must be a power of two in [8, 1024]");
    if (dtype != HERMES_F32 && dtype != HERMES_F64) return fail(HERMES_ERR_ARG, "hermes_filter_bins: bad dtype");
    if (!(box_L > 0.0)) return fail(HERMES_ERR_ARG, "hermes_filter_bins: box_L must be > 0");
    if (n_win < 1) return fail(HERMES_ERR_ARG, "hermes_filter_bins: n_win must be >= 1");
    for (int i = 0; i < n_win; ++i) {
        const hermes_window& w = win[i];
        if (w.reserved != 0) return fail(HERMES_ERR_ARG, "hermes_filter_bins: reserved field must be 0");
        switch (w.type) {
            case HERMES_WIN_SPHERE:
            case HERMES_WIN_GAUSS:
                if (!(w.r_hi > 0.0)) return fail(HERMES_ERR_ARG, "hermes_filter_bins: radius must be > 0");
                break;
            case HERMES_WIN_SHELL:
                if (!(w.r_lo >= 0.0 && w.r_hi > w.r_lo))
                    return fail(HERMES_ERR_ARG, "hermes_filter_bins: shell needs 0 <= r_lo < r_hi");
                break;
            case HERMES_WIN_SH_SHELL:
                if (!(w.r_lo >= 0.0 && w.r_hi > w.r_lo))
                    return fail(HERMES_ERR_ARG, "hermes_filter_bins: shell needs 0 <= r_lo < r_hi");
                if (w.ell < 0 || w.ell > HERMES_MAX_LMAX || w.m < -w.ell || w.m > w.ell)
                    return fail(HERMES_ERR_ARG, "hermes_filter_bins: need 0 <= ell <= 16 and |m| <= ell");
                break;
            default:
                return fail(HERMES_ERR_ARG, "hermes_filter_bins: unknown window type");
        }
    }
    if (work_bytes < filter_workspace(n_grid, dtype, n_win))
        return fail(HERMES_ERR_OOM, "hermes_filter_bins: workspace too small");
    DeviceGuard g(ctx->device);
    return filter_impl(ctx, delta_k, n_grid, dtype, box_L, win, n_win, out, moments, work, work_bytes, stream);
}

hermes_status hermes_zeta_l(hermes_ctx ctx, const float* delta, const void* delta_k, int n_grid,
                            double box_L, const double* edges, int n_bins, int l_max, int precision,
                            double* zeta, void* work, size_t work_bytes, hipStream_t stream) {
    if (!ctx || !delta || !delta_k || !zeta || !work) return fail(HERMES_ERR_ARG, "hermes_zeta_l: NULL argument");
    if (!valid_n(n_grid)) return fail(HERMES_ERR_ARG, "hermes_zeta_l: N must be a power of two in [8, 1024]");
    if (!(box_L > 0.0)) return fail(HERMES_ERR_ARG, "hermes_zeta_l: box_L must be > 0");
    if (l_max < 0 || l_max > HERMES_MAX_LMAX) return fail(HERMES_ERR_ARG, "hermes_zeta_l: l_max must be in [0, 16]");
    if (precision != HERMES_PREC_FP32 && precision != HERMES_PREC_BF16X3 && precision != HERMES_PREC_FP16X3)
        return fail(HERMES_ERR_ARG, "hermes_zeta_l: unknown precision");
    Edges e;
    hermes_status st = get_edges(edges, n_bins, box_L, e, "hermes_zeta_l");
    if (st != HERMES_OK) return st;
    if (work_bytes < zeta_workspace(n_grid, n_bins)) return fail(HERMES_ERR_OOM, "hermes_zeta_l: workspace too small");
    DeviceGuard g(ctx->device);
    return zeta_impl(ctx, delta, delta_k, n_grid, box_L, e, l_max, precision, zeta, work, work_bytes, stream);
}

static hermes_status readout_checked(const char* who, hermes_ctx ctx, const void* fields, int n_fields, int n_grid,
                                     int dtype, double box_L, const float* pos, const float* weight, int64_t n_pts,
                                     const hermes_mark* mark, void* out, double* moments, void* work,
                                     size_t work_bytes, hipStream_t stream) {
    const std::string w(who);
    if (!ctx || !fields || (n_pts > 0 && !pos)) return fail(HERMES_ERR_ARG, w + ": NULL argument");
    if (n_fields < 1 || n_fields > HERMES_MAX_READOUT_FIELDS)
        return fail(HERMES_ERR_ARG, w + ": n_fields must be in [1, 64]");
    if (!out && !moments) return fail(HERMES_ERR_ARG, w + ": out and moments both NULL");
    if (n_pts < 0) return fail(HERMES_ERR_ARG, w + ": n_pts < 0");
    if (!valid_n(n_grid)) return fail(HERMES_ERR_ARG, w + ": N must be a power of two in [8, 1024]");
    if (dtype != HERMES_F32 && dtype != HERMES_F64) return fail(HERMES_ERR_ARG, w + ": bad dtype");
    if (!(box_L > 0.0)) return fail(HERMES_ERR_ARG, w + ": box_L must be > 0");
    if (mark) {
        if (mark->reserved != 0) return fail(HERMES_ERR_ARG, w + ": reserved field must be 0");
        if (mark->kind != HERMES_MARK_NONE && mark->kind != HERMES_MARK_POWER_LAW &&
            mark->kind != HERMES_MARK_INVERSE_DENSITY)
            return fail(HERMES_ERR_ARG, w + ": unknown mark kind");
        if (!std::isfinite(mark->exponent) || !std::isfinite(mark->offset) || !std::isfinite(mark->self_term))
            return fail(HERMES_ERR_ARG, w + ": mark parameters must be finite");
        if (mark->offset < 0.0) return fail(HERMES_ERR_ARG, w + ": mark offset must be >= 0");
        const bool divides = mark->kind == HERMES_MARK_INVERSE_DENSITY ||
                             (mark->kind == HERMES_MARK_POWER_LAW && mark->exponent < 0.0);
        if (divides && !(mark->offset > 0.0)) return fail(HERMES_ERR_ARG, w + ": this mark needs offset > 0");
    }
    if (work && work_bytes < readout_workspace(n_grid, n_pts)) return fail(HERMES_ERR_OOM, w + ": workspace too small");
    DeviceGuard g(ctx->device);
    return readout_impl(ctx, fields, n_fields, n_grid, dtype, box_L, pos, weight, n_pts, mark, out, moments, work,
                        stream);
}

hermes_status hermes_readout(hermes_ctx ctx, const void* field, int n_grid, int dtype, double box_L,
                             const float* pos, const float* weight, int64_t n_pts, const hermes_mark* mark,
                             void* out, double* moments, void* work, size_t work_bytes, hipStream_t stream) {
    return readout_checked("hermes_readout", ctx, field, 1, n_grid, dtype, box_L, pos, weight, n_pts, mark, out,
                           moments, work, work_bytes, stream);
}

hermes_status hermes_readout_fields(hermes_ctx ctx, const void* fields, int n_fields, int n_grid, int dtype,
                                    double box_L, const float* pos, const float* weight, int64_t n_pts,
                                    const hermes_mark* mark, void* out, double* moments, void* work,
                                    size_t work_bytes, hipStream_t stream) {
    return readout_checked("hermes_readout_fields", ctx, fields, n_fields, n_grid, dtype, box_L, pos, weight, n_pts,
                           mark, out, moments, work, work_bytes, stream);
}

}  // extern "C"
