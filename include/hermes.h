/*
 * hermes.h -- C ABI of the MI355X (gfx950) field-window estimator library.
 *
 * The library computes, on one GPU, the hot path of the in-situ field-window
 * estimator of clustering statistics:
 *   catalogue -> scaling-function coefficients     (hermes_assign)
 *   -> density contrast and its 3-D real FFT        (hermes_fft)
 *   -> 2PCF and its Legendre multipoles by Parseval  (hermes_xi)
 *   -> window-filtered fields, counts-in-cells moments (hermes_filter_bins)
 *   -> 3PCF multipoles zeta_l(r1, r2)                 (hermes_zeta_l)
 *   -> anisotropic 2PCF with axisymmetric windows     (hermes_xi_aniso)
 *   -> field values and density marks at positions    (hermes_readout)
 *   -> Monte-Carlo triangle sums (dual-/triplet-sphere 3PCF) (hermes_triplet_mc)
 *   -> 3PCF monopole through connection coefficients  (hermes_ddd_gamma)
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Grid: N^3 nodes, N a power of two in [8, 1024]; node l = (lx, ly, lz)
 *    sits at position l*h, h = L/N, in a periodic box of side L.  Real
 *    fields are row-major [N][N][N] with lz fastest.
 *  - Half spectrum: complex [N][N][N/2+1] (interleaved re, im), index
 *    (kx, ky, kz) with kz in [0, N/2]; forward DFT unnormalised,
 *    f^(n) = sum_l f_l exp(-2 pi i n.l / N).  Signed mode n~ in (-N/2, N/2],
 *    k = 2 pi n~ / L.
 *  - dtype: HERMES_F32 (float fields, complex64 spectra) or HERMES_F64
 *    (double fields, complex128 spectra).  Positions and weights are always
 *    float32.  Grid-wide reductions are always accumulated in float64.
 *  - Basis: the scaling function phi of the MRA expansion is a property of
 *    the context (hermes_set_basis): the centred cubic B-spline B3 (default;
 *    not orthonormal, 4 nodes per axis) or the orthonormal Daubechies D4
 *    function (support [0, 3], 3 nodes per axis).  It fixes the
 *    projection and readout taps, the kernel Phi^ = |phi^|^2 of every
 *    window, the self-pair kernel of the shot-noise factor and the
 *    connection coefficients.  Coefficient fields of one basis are only
 *    meaningful to calls made with the same basis.
 *  - Every device buffer is owned by the caller, including workspace, whose
 *    size hermes_workspace_size() reports.  The library owns only the opaque
 *    context (twiddle, basis-kernel and quadrature tables).  No entry point
 *    allocates device memory.
 *  - All calls are asynchronous on the given stream; outputs (device
 *    pointers, including the double-precision statistics) are valid after the
 *    stream has been synchronised.  Host arrays passed in (bin edges, window
 *    lists, multipole lists) are read before the call returns.
 *  - Errors: every entry point returns a hermes_status; on anything but
 *    HERMES_OK, hermes_last_error() returns a thread-local message.  Argument
 *    errors (ERR_ARG, ERR_OOM, ERR_UNSUPPORTED) are detected before any
 *    kernel is launched; HERMES_ERR_HIP reports a HIP runtime error raised by
 *    a launch.
 */
#ifndef HERMES_H
#define HERMES_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum hermes_status {
    HERMES_OK = 0,
    HERMES_ERR_ARG = 1,         /* bad pointer, size, bin edges, multipole, ... */
    HERMES_ERR_OOM = 2,         /* workspace smaller than hermes_workspace_size() */
    HERMES_ERR_HIP = 3,         /* HIP runtime error */
    HERMES_ERR_UNSUPPORTED = 4  /* valid request outside what the library supports */
} hermes_status;

typedef enum hermes_dtype { HERMES_F32 = 0, HERMES_F64 = 1 } hermes_dtype;

/* Precision of the 3PCF contraction (the FFTs always run in float32). */
typedef enum hermes_precision {
    HERMES_PREC_FP32 = 0,   /* float32 vector FMA contraction */
    HERMES_PREC_BF16X3 = 1, /* y = sqrt|delta| f split hi+lo in bf16; hi.hi and lo.hi MFMA products
                               (the hi.lo one by symmetry), fp32 accumulate */
    HERMES_PREC_FP16X3 = 2  /* the same split in fp16 */
} hermes_precision;

/* Window kinds (Table A1 (a)-(c) and the multipole windows of Sec. 3.3.3). */
typedef enum hermes_window_type {
    HERMES_WIN_SHELL = 0,    /* volume-normalised thick shell [r_lo, r_hi] (Eq. Wshell_k) */
    HERMES_WIN_SPHERE = 1,   /* spherical top-hat of radius r_hi (Table A1 (b)) */
    HERMES_WIN_GAUSS = 2,    /* Gaussian exp(-k^2 r_hi^2 / 2) (Table A1 (c)) */
    HERMES_WIN_SH_SHELL = 3  /* 4 pi i^l jbar_l(k; r_lo, r_hi) Y^R_lm(k^) (Eq. multipole-window) */
} hermes_window_type;

/* One window.  r_lo is ignored for SPHERE and GAUSS; ell and m (real
 * spherical-harmonic index, -ell..ell) are used by SH_SHELL only. */
typedef struct hermes_window {
    int32_t type;
    int32_t ell;
    int32_t m;
    int32_t reserved;   /* must be 0 */
    double r_lo;
    double r_hi;
} hermes_window;

/* Operation ids for hermes_workspace_size(). */
typedef enum hermes_op {
    HERMES_OP_ASSIGN = 0,
    HERMES_OP_FFT = 1,
    HERMES_OP_XI = 2,
    HERMES_OP_FILTER = 3,
    HERMES_OP_ZETA = 4,
    HERMES_OP_XI_ANISO = 5,
    HERMES_OP_TRIPLET = 6,
    HERMES_OP_DDD_GAMMA = 7,
    HERMES_OP_READOUT = 8
} hermes_op;

typedef struct hermes_ctx_s* hermes_ctx;

#define HERMES_MAX_BINS 64   /* bins per hermes_xi / hermes_zeta_l call */
#define HERMES_MAX_ELLS 8    /* multipoles per hermes_xi call */
#define HERMES_MAX_LMAX 16   /* highest 3PCF multipole */
#define HERMES_MAX_ANISO (1 << 20)   /* windows per hermes_xi_aniso call */
#define HERMES_MAX_THETA 64          /* opening angles per hermes_triplet_mc call */
#define HERMES_MAX_GAMMA_FIELDS 32   /* filtered fields per hermes_ddd_gamma call */
#define HERMES_MAX_READOUT_FIELDS 64 /* fields per hermes_readout_fields call */

/* Create a context on HIP device `device`; fills *out.  Allocates the
 * context's constant tables (about 2.7 MB, both bases) on that device.  The
 * basis starts as HERMES_BASIS_B3. */
hermes_status hermes_create(hermes_ctx* out, int device);

/* Scaling function of the MRA basis (Sec. 3.1: a compactly supported
 * scaling function phi, the basis phi_l(x) = prod_a phi(x_a/h - l_a)).
 *   B3   centred cubic B-spline, support [-2, 2]: a point reaches the nodes
 *        i0 - 1 .. i0 + 2 per axis (i0 = floor(x/h)); Phi^ per axis
 *        sinc^8(pi n~/N); not orthonormal (its autocorrelation at integer
 *        lags is the degree-7 B-spline)
 *   DB2  Daubechies D4 (the paper's default), orthonormal, support [0, 3]:
 *        a point reaches the nodes i0 - 2 .. i0 per axis with weights
 *        phi(x/h - l), phi tabulated at x = i / 2^12 from the refinement
 *        relation with the D4 filter and interpolated linearly between;
 *        Phi^ per axis |phi^(2 pi n~/N)|^2 = prod_{j>=1} |m0(w/2^j)|^2; the
 *        self-pair kernel is the Kronecker delta */
typedef enum hermes_basis { HERMES_BASIS_B3 = 0, HERMES_BASIS_DB2 = 1 } hermes_basis;

/* Select the basis of every later call on this context (the tables of both
 * are resident, so calls already queued are unaffected).  ERR_ARG for an
 * unknown basis.  hermes_get_basis returns the current one (-1 for NULL). */
hermes_status hermes_set_basis(hermes_ctx ctx, int basis);
int hermes_get_basis(hermes_ctx ctx);

/* Release a context (NULL is ignored).  Not to be called while work that
 * uses it is still in flight. */
void hermes_destroy(hermes_ctx ctx);

/* Thread-local text of the last error raised on this thread ("" if none). */
const char* hermes_last_error(void);

/* Device workspace, in bytes, that `op` needs for an N^3 grid.  n_batch is
 * the number of points (ASSIGN, READOUT), windows (FILTER, XI_ANISO), radial
 * bins (ZETA), opening angles (TRIPLET) or fields (DDD_GAMMA);
 * n_ells the number of multipoles (XI), or the number of primary vertices
 * (TRIPLET: 0 gives the minimum, which runs the direct path; see
 * hermes_triplet_mc).  Zero for FFT, which needs none. */
hermes_status hermes_workspace_size(hermes_ctx ctx, int op, int n_grid, int dtype,
                                    int n_batch, int n_ells, size_t* bytes);

/* MRA projection of a weighted catalogue (Sec. 3.1, Eq. phi_projection):
 *   eps_l = sum_i w_i prod_a phi(x_{i,a}/h - l_a),  l_a taken mod N,
 * with the context's scaling function phi (B3: 64 nodes per point; D4: 27).
 * Position fractions and tap weights are formed in float64.  The taps are
 * summed in 64-bit fixed point with the power-of-two step 2^-k, k = 61 -
 * ceil(log2 sum_i |w_i|) (59 - ... for D4, whose taps reach |phi|^3 < 4),
 * each tap rounded once to a multiple of it: the grid is the same bit for bit
 * on every run, and for float64 it carries an absolute error of at most
 * 2^-(k+1) per tap.
 *   pos    device float32 [n_pts][3], any real values (wrapped into the box)
 *   weight device float32 [n_pts], or NULL for unit weights (Eq. dendis;
 *          marks or physical values as in Eq. weighted_field); finite
 *   eps    device [N^3] of dtype; overwritten
 *   sum_w  device double[1]; overwritten with sum_i w_i (float64, summed in
 *          a fixed order)
 *   work   device workspace of >= hermes_workspace_size(ASSIGN, n_batch =
 *          n_pts) bytes: the 64-bit grid (8 N^3 bytes), per-tile counts and
 *          point lists (4 n_pts bytes)
 * n_pts may be 0 (eps is zeroed, sum_w = 0).  ERR_ARG for NULL buffers,
 * n_pts < 0 or >= 2^32, box_L <= 0 or N not a power of two in [8, 1024];
 * ERR_OOM if work_bytes is too small. */
hermes_status hermes_assign(hermes_ctx ctx, const float* pos, const float* weight,
                            int64_t n_pts, double box_L, int n_grid, int dtype,
                            void* eps, double* sum_w, void* work, size_t work_bytes,
                            hipStream_t stream);

/* Density contrast and forward transform (Sec. 4.2; analytic uniform random
 * of Sec. 4.3.1):  delta_l = eps_l / eps_bar - 1, eps_bar = sum_w / N^3,
 * then delta^ = r2c DFT of delta with delta^(0) := 0.
 *   eps     device [N^3] of dtype (read only)
 *   sum_w   device double[1] from hermes_assign
 *   delta_k device complex [N][N][N/2+1] of dtype; overwritten
 *   delta   device [N^3] of dtype receiving delta_l, or NULL
 * ERR_ARG if sum_w holds zero is NOT detected (the result is then inf/nan). */
hermes_status hermes_fft(hermes_ctx ctx, const void* eps, const double* sum_w,
                         int n_grid, int dtype, void* delta_k, void* delta,
                         hipStream_t stream);

/* 2PCF and its Legendre multipoles by Parseval (Sec. 3.3.1 Eq.
 * pair-counting-kspace; Sec. 3.3.3 DD_l with the bin-averaged radial factor):
 *   xi_l[b] = N^-6 sum_n |delta^_n|^2 Phi^(n) (2l+1) i^l jbar_l(k_n; b) L_l(mu_n),
 * Phi^(n) = prod_a Phi^_1(n~_a) the basis kernel (B3: sinc^8(pi n~_a / N),
 * the Fourier transform of the B3 autocorrelation; D4: |phi^|^2), mu = k_los/|k|,
 * jbar_0 = volume-normalised thick shell (Eq. Wshell_k).  Raw estimator:
 * no shot-noise subtraction (the self-pair term of Sec. 2.2 Eq. CFpow is left
 * to the caller, who can take it from `shot`).
 *   delta_k  device half spectrum from hermes_fft
 *   edges    host double [n_bins+1], strictly increasing, edges[0] >= 0,
 *            every edge < box_L / 2 (ERR_ARG otherwise)
 *   ells     host int [n_ells], even values in [0, HERMES_MAX_LMAX]
 *   los_axis 0, 1 or 2 (plane-parallel line of sight)
 *   xi       device double [n_ells][n_bins]; overwritten
 *   shot     device double [n_ells][n_bins] or NULL: the shot-noise factor
 *            S_lb = sum_D K_lb(D) B7(D1) B7(D2) B7(D3) over lags |D_a| <= 3,
 *            K_lb(D) the real-space window kernel above and B7 the degree-7
 *            centred B-spline (the B3 autocorrelation at integer lags; with
 *            D4 the Kronecker delta, S_lb = K_lb(0)); for
 *            iid points of weights w_i, E xi_lb = (sum w^2 / W^2)
 *            (N^3 S_lb - K_lb(n = 0)), K_0b(0) = 1, K_lb(0) = 0 for l > 0
 *   work     device workspace of >= hermes_workspace_size(XI) bytes */
hermes_status hermes_xi(hermes_ctx ctx, const void* delta_k, int n_grid, int dtype,
                        double box_L, const double* edges, int n_bins,
                        const int* ells, int n_ells, int los_axis, double* xi,
                        double* shot, void* work, size_t work_bytes, hipStream_t stream);

/* hermes_xi for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same statistic, arguments and errors as hermes_xi, without a workspace.  The
 * histogram and partial sums live in a 16 MiB scratch array that the library
 * holds statically on every device it runs on, until the process ends;
 * nothing is allocated.  ERR_UNSUPPORTED when the call needs more scratch than
 * that (hermes_workspace_size(XI) > 16 MiB, e.g. two or more multipoles at
 * 1024^3).  Each call clears what it accumulates before use, but every call on
 * a device shares the one array: calls that overlap on a device (two streams,
 * threads or contexts) race and must be serialised by the caller. */
hermes_status hermes_xi_static(hermes_ctx ctx, const void* delta_k, int n_grid, int dtype,
                               double box_L, const double* edges, int n_bins,
                               const int* ells, int n_ells, int los_axis, double* xi,
                               double* shot, hipStream_t stream);

/* Window-filtered fields (Sec. 4.2: eps_W = iFT[FT(eps) W^ Phi^]) and their
 * counts-in-cells moments (Sec. 3.1 filtered field, Sec. 2.2.2 Eq. varw):
 *   out_w(l) = N^-3 sum_n delta^_n Phi^(n) W^_w(k_n) exp(2 pi i n.l/N)   (real)
 *   moments[w] = ( <out_w^2>, <out_w^3>, <out_w^4> ), mean over all nodes.
 * Windows of kind SH_SHELL use the Nyquist-averaged real spherical harmonic.
 *   win      host array of n_win windows
 *   out      device [n_win][N^3] of dtype, or NULL to skip storing fields
 *   moments  device double [n_win][3], or NULL
 *   work     device workspace of >= hermes_workspace_size(FILTER, n_win) */
hermes_status hermes_filter_bins(hermes_ctx ctx, const void* delta_k, int n_grid,
                                 int dtype, double box_L, const hermes_window* win,
                                 int n_win, void* out, double* moments, void* work,
                                 size_t work_bytes, hipStream_t stream);

/* 3PCF multipoles with a naked primary vertex (Sec. 3.3.3 Eqs.
 * multipole-window, iFFT-multipoleSFC, 2-fold-translation; Sec. 3.4):
 *   a_lmb(x) = iDFT[delta^ Phi^ 4 pi i^l jbar_l(k; b) Y^R_lm(k^)](x)  (real),
 *   zeta_l[b1][b2] = (4 pi N^3)^-1 sum_{m=-l..l} sum_x delta(x) a_lmb1(x) a_lmb2(x),
 * i.e. the Legendre coefficients of the rotation-averaged triple product.
 * Float32 FFTs; the contraction per `precision`; float64 across tiles.
 *   delta    device float [N^3]: the contrast written by hermes_fft
 *   delta_k  device complex64 half spectrum from hermes_fft
 *   edges    host double [n_bins+1], strictly increasing, edges[0] >= 0,
 *            every edge < box_L / 2 (ERR_ARG otherwise)
 *   l_max    0..HERMES_MAX_LMAX
 *   zeta     device double [l_max+1][n_bins][n_bins]; overwritten
 *   work     device workspace of >= hermes_workspace_size(ZETA, n_bins) */
hermes_status hermes_zeta_l(hermes_ctx ctx, const float* delta, const void* delta_k,
                            int n_grid, double box_L, const double* edges, int n_bins,
                            int l_max, int precision, double* zeta, void* work,
                            size_t work_bytes, hipStream_t stream);

/* Axisymmetric windows about the line of sight (Sec. 2.2.3 redshift space:
 * circular ring; Table A1 (d), (f)-(i)).  With k_par the line-of-sight
 * component of k, k_perp = |k - k_par e_los|, R = r_perp, H = r_par:
 *   RING         cos(k_par H) J0(k_perp R)                  (thin double ring; A1 (i))
 *   RING_BIN     sinc(k_par dH / 2) cos(k_par H) <J0(k_perp rho)>, the average
 *                over the annulus rho in [R - dR/2, R + dR/2] with weight
 *                rho / (R dR)                               (finite bins, dR = d_perp,
 *                                                           dH = d_par)
 *   GAUSS_RING   cos(k_par H) J0(k_perp R) exp(-k_perp^2 s^2 / 2), s = d_perp
 *                                                           (Gaussian-blurred ring)
 *   DISK         2 J1(k_perp R) / (k_perp R) cos(k_par H)   (pair of disks; A1 (h))
 *   CYLINDER     2 J1(k_perp R) / (k_perp R) sinc(k_par H)  (filled, half-height H; A1 (f))
 *   CYLSHELL     J0(k_perp R) sinc(k_par H)                 (side wall; A1 (g))
 *   GAUSS_SHELL  (Rg^2 cos(k Rs) + Rs^2 sinc(k Rs)) / (Rs^2 + Rg^2) exp(-k^2 Rg^2 / 2),
 *                Rs = r_perp, Rg = d_perp, k = |k|        (isotropic; A1 (d))
 * with sinc x = sin x / x.  Unused parameters are ignored (must still be
 * finite and >= 0). */
typedef enum hermes_aniso_kind {
    HERMES_ANISO_RING = 0,
    HERMES_ANISO_RING_BIN = 1,
    HERMES_ANISO_GAUSS_RING = 2,
    HERMES_ANISO_DISK = 3,
    HERMES_ANISO_CYLINDER = 4,
    HERMES_ANISO_CYLSHELL = 5,
    HERMES_ANISO_GAUSS_SHELL = 6
} hermes_aniso_kind;

typedef struct hermes_aniso_window {
    int32_t kind;
    int32_t reserved;   /* must be 0 */
    double r_perp;
    double r_par;
    double d_perp;
    double d_par;
} hermes_aniso_window;

/* Anisotropic 2PCF with axisymmetric windows, by Parseval (Sec. 2.2.3
 * xi(r_par, r_perp) as the field-window product; Sec. 3.3.1):
 *   xi[w] = N^-6 sum_n |delta^_n|^2 Phi^(n) W^_w(k_par, k_perp),
 * Phi^ as in hermes_xi, plane-parallel line of sight along los_axis.  Raw
 * estimator (no shot-noise subtraction).  The sum is regrouped exactly over
 * (|n_los|, |n_perp|^2); the grouping's float64 atomics make the last bits
 * depend on the order of additions.
 *   delta_k  device half spectrum from hermes_fft
 *   win      host array of n_win windows, read before the call returns
 *   xi       device double [n_win]; overwritten
 *   work     device workspace of >= hermes_workspace_size(XI_ANISO, n_batch =
 *            n_win) bytes
 * ERR_ARG for NULL buffers, a bad N, dtype, box_L or los_axis, n_win outside
 * [1, HERMES_MAX_ANISO], a non-zero reserved field, an unknown kind, a
 * non-finite or negative parameter, r_perp or r_par >= L/2, RING_BIN with
 * d_perp <= 0 or r_perp < d_perp / 2, GAUSS_SHELL with r_perp = d_perp = 0;
 * ERR_OOM if work_bytes is too small. */
hermes_status hermes_xi_aniso(hermes_ctx ctx, const void* delta_k, int n_grid, int dtype,
                              double box_L, const hermes_aniso_window* win, int n_win,
                              int los_axis, double* xi, void* work, size_t work_bytes,
                              hipStream_t stream);

/* Mark ratio of the density-marked 2PCF (Sec. 3.3.1 Eqs. power-law-mark,
 * inverse-density-mark; Sec. 4.3.2): the marked correlation function is the
 * 2PCF of the mark-weighted catalogue normalised by the unmarked pair counts,
 *   out[b] = (1 + xi_marked[b]) / (1 + xi[b]),  b < n,
 * with xi_marked and xi from hermes_xi on the mark-weighted and the plain
 * catalogue over the same bins.  xi_marked, xi and out are device double
 * [n] (out may alias either input); computed in float64 on the stream.
 * ERR_ARG for NULL pointers or n < 0. */
hermes_status hermes_mark_ratio(const double* xi_marked, const double* xi, int n, double* out,
                                hipStream_t stream);

/* Monte-Carlo triangle sums (Sec. 3.4 particle-based summation, Eq.
 * particle-based-sum; Sec. 4.3.3 dual-/triplet-sphere 3PCF).  Primary
 * vertices: the n_centres catalogue points `centres` (dual sphere; primary
 * factor a = weight, or 1 when weights is NULL), or, when centres is NULL,
 * n_centres uniform points of the box (triplet sphere; a = f1 read at the
 * point, or 1 when f1 is NULL).  Each primary vertex x gets n_rot random
 * rotations (u, v), u uniform on the sphere and v uniform on the circle
 * orthogonal to u; for theta_j = (j + 1/2) pi / n_theta the triangle's other
 * vertices are x + r12 u and x + r13 (cos theta_j u + sin theta_j v), where
 * f2 and f3 are read through the basis expansion (as hermes_readout;
 * positions in float64).
 *   out[j] = ( sum a, sum a f2(x2), sum a f3(x3_j), sum a f2(x2) f3(x3_j) )
 * over all (centre, rotation), accumulated in float64 in a fixed order (the
 * result is the same on every run).  The ratio of the last to the first is
 * the Monte-Carlo mean triple product: with filtered contrasts
 * f = delta_W it estimates the smoothed 3PCF at (r12, r13, theta_j) (box
 * points with a = 1 + f1), or the particle-weighted pair product of the
 * dual-sphere scheme.
 * Random numbers: Philox4x64-10 (Salmon et al., SC'11), key (seed, 0),
 * counter (centre, rotation, 0, 0) for a rotation's words w0..w2 (cos of the
 * polar angle 2 u0 - 1, azimuth 2 pi u1, angle of v 2 pi u2) and
 * (centre, 0, 1, 0) for a box point (L u0, L u1, L u2), u = (w >> 11 + 1/2) 2^-53;
 * the frame orthogonal to u is built as in Duff et al. (JCGT 2017).
 *   f1, f2, f3  device [N^3] fields of dtype (f1 NULL unless box points)
 *   centres     device float32 [n_centres][3] or NULL; weights device float32
 *               [n_centres] or NULL (only with centres)
 *   out         device double [n_theta][4]; overwritten
 *   work        device workspace of >= hermes_workspace_size(TRIPLET, n_batch
 *               = n_theta, n_ells = 0) bytes: the partial sums and three
 *               tile-packed copies of the fields, for N <= 512 in float32
 *               (64 N^3 bytes each) and N <= 256 in float64 (128 N^3 bytes
 *               each); a tile holds, for a pair of x planes, the 4 x 4 (y, z)
 *               block of nodes that points in a cell reach (D4 uses 3 x 3 of
 *               it).  Sized with n_ells = n_centres (< 2^31), it also holds
 *               the bucket lists of the block-local path (about 16 bytes per
 *               centre plus 8 bytes per bucket), which is taken when the
 *               fields are float32, f2 == f3 (one array) and the reach fits
 *               the staged region: E + 2 (floor(max(r12, r13) N / L) + 2) +
 *               NT - 1 <= 32, with E = 4 cells per bucket edge for N <= 256
 *               (8 at 512, 16 at 1024) and NT = 4 (B3) or 3 (D4).  There the
 *               centres are sorted by bucket (stable, so a bucket's centres
 *               stay in index order) and a workgroup stages the 32^3 nodes
 *               around its bucket in LDS; both paths draw the same samples and
 *               agree to rounding
 * ERR_ARG for NULL f2, f3, out or work, f1 given with centres, weights
 * without centres, n_centres < 0, n_rot < 1, n_centres n_rot >= 2^62,
 * n_theta outside [1, HERMES_MAX_THETA], r12 or r13 negative, not finite or
 * >= L/2, a bad N, dtype or box_L; ERR_OOM if work_bytes is too small. */
hermes_status hermes_triplet_mc(hermes_ctx ctx, const void* f1, const void* f2, const void* f3,
                                int n_grid, int dtype, double box_L, const float* centres,
                                const float* weights, int64_t n_centres, double r12, double r13,
                                int n_theta, int n_rot, uint64_t seed, double* out, void* work,
                                size_t work_bytes, hipStream_t stream);

/* 3PCF monopole through triple connection coefficients (Sec. 3.3.2, Eqs.
 * 3pcfddd, 3PCF-ddd-monopole, con-coeff, DDD-vector-product), with the
 * context's scaling function phi:
 *   out[b1][b2] = N^-3 sum_l eps_l sum_{a,b} Gamma_{a,b} f_b1[l + a] f_b2[l + b],
 *   Gamma_{a,b} = int phi(x) phi(x - a) phi(x - b) d^3x = prod_axes gamma(a_i, b_i),
 * i.e. the box mean of the product of the three basis expansions.  B3
 * (offsets in [-3, 3]^3): computed as that exact integral (5-point
 * Gauss-Legendre per cell and axis).  D4 (orthonormal; offsets in [-2, 2]^3,
 * gamma from the refinement relation): computed through gamma = V diag(lambda)
 * V^T per axis, out = N^-3 sum_l sum_r lambda_r eps_l F_b1,r[l] F_b2,r[l] with
 * F_b,r = f_b filtered by the separable five-tap stencil V_r, the exact
 * stencil sum (Eq. DDD-vector-product: the paper's exact 3PCF monopole of
 * the smoothed fields).  With eps = delta from hermes_fft and f_b the
 * thick-shell filtered contrasts of hermes_filter_bins it is the 3PCF
 * monopole of the paper's MRA route; the node-sum form of zeta_0
 * (hermes_zeta_l) replaces the integral by the node values.
 *   eps     device [N^3] of dtype
 *   fields  device [n_fields][N^3] of dtype
 *   out     device double [n_fields][n_fields] (symmetric); overwritten
 *   work    device workspace of >= hermes_workspace_size(DDD_GAMMA) bytes
 * Per cell brick the sums are formed in dtype, across bricks in float64 in
 * a fixed order.  ERR_ARG for NULL buffers, n_fields outside [1, 32], a bad
 * N or dtype; ERR_OOM if work_bytes is too small. */
hermes_status hermes_ddd_gamma(hermes_ctx ctx, const void* eps, const void* fields, int n_fields,
                               int n_grid, int dtype, double* out, void* work, size_t work_bytes,
                               hipStream_t stream);

/* Density-derived marks (Sec. 3.3.1).  With v the value read at a point
 * (hermes_readout) and rho = max(1 + v - self_term, 0) the local density in
 * units of the mean (self_term removes a point's own contribution; the clip
 * keeps the density non-negative):
 *   POWER_LAW        m = (rho + offset)^exponent           (Eq. power-law-mark,
 *                                                          offset = epsilon)
 *   INVERSE_DENSITY  m = ((offset + 1) / (offset + rho))^exponent
 *                                                          (Eq. inverse-density-mark,
 *                                                          offset = rho_* / rho_bar) */
typedef enum hermes_mark_kind {
    HERMES_MARK_NONE = 0,
    HERMES_MARK_POWER_LAW = 1,
    HERMES_MARK_INVERSE_DENSITY = 2
} hermes_mark_kind;

typedef struct hermes_mark {
    int32_t kind;
    int32_t reserved;    /* must be 0 */
    double exponent;     /* alpha (power law) or p (inverse density) */
    double offset;       /* epsilon or rho_* / rho_bar; > 0 where rho = 0 would divide by zero */
    double self_term;    /* subtracted from 1 + v before the clip (contrast units) */
} hermes_mark;

/* Readout of a coefficient field at arbitrary positions (Sec. 3.1: the
 * filtered field n_W(x) = sum_l eps~_l phi_l(x) is read at any point, e.g. at
 * random positions for counts in cells or at the catalogue's points for
 * density-derived marks):
 *   v_i = sum_l f_l prod_a phi(x_{i,a}/h - l_a),  l_a mod N  (B3: 64 nodes,
 * D4: 27), the transpose of hermes_assign.  Position fractions are formed in float64.
 *   field   device [N^3] of dtype (a filtered field from hermes_filter_bins,
 *           the contrast from hermes_fft, ...)
 *   pos     device float32 [n_pts][3], any real values (wrapped into the box)
 *   weight  device float32 [n_pts] or NULL: multiplies each output
 *   mark    host hermes_mark or NULL (NULL or kind NONE: out_i = w_i v_i)
 *   out     device [n_pts] of dtype, or NULL: out_i = w_i m(v_i)
 *   moments device double[3], or NULL: the means over the points of v^2, v^3,
 *           v^4 (unweighted, unmarked), accumulated in float64; with the
 *           tile-staged read (below) in a fixed order, the same on every run,
 *           otherwise by float64 atomics across workgroups (order not fixed);
 *           zeros for n_pts = 0
 *   work    device workspace of >= hermes_workspace_size(READOUT, n_batch =
 *           n_pts) bytes, or NULL.  With it, calls of 2^16 to 2^31 - 1 points
 *           first bucket the points by tiles of 8^3 cells (16^3 at N = 1024)
 *           with a stable radix sort of their tile keys (keys, sorted keys,
 *           a 4-byte index and a copy of the position per point, and the
 *           sort's buffers: about 32 bytes per point) and read them tile by
 *           tile; when the tiles hold at least 8 points on average, a
 *           workgroup stages the nodes around a tile in LDS and reads the
 *           tile's points from there.  The size is 0 outside that range.
 *           NULL reads the points in the given order.  Values are the same
 *           bit for bit either way and land at their points' indices.
 * ERR_ARG for NULL buffers, out and moments both NULL, n_pts < 0, box_L <= 0,
 * a bad N or dtype, a non-zero reserved field, an unknown mark kind, a
 * non-finite exponent, offset < 0, or offset = 0 where rho = 0 would divide by
 * zero (inverse density, or a power law with a negative exponent); ERR_OOM if
 * work is given and work_bytes is too small. */
hermes_status hermes_readout(hermes_ctx ctx, const void* field, int n_grid, int dtype,
                             double box_L, const float* pos, const float* weight,
                             int64_t n_pts, const hermes_mark* mark, void* out,
                             double* moments, void* work, size_t work_bytes,
                             hipStream_t stream);

/* hermes_readout of n_fields fields at the same points (e.g. one field
 * smoothed at several radii, the counts in random spheres of Sec. 3.1): the
 * points are bucketed once.  fields is device [n_fields][N^3] of dtype; out,
 * if not NULL, is [n_fields][n_pts]; moments, if not NULL, is double
 * [n_fields][3].  The workspace is the same as hermes_readout's for n_pts
 * points.  ERR_ARG as hermes_readout, and for n_fields outside
 * [1, HERMES_MAX_READOUT_FIELDS]. */
hermes_status hermes_readout_fields(hermes_ctx ctx, const void* fields, int n_fields, int n_grid,
                                    int dtype, double box_L, const float* pos, const float* weight,
                                    int64_t n_pts, const hermes_mark* mark, void* out, double* moments,
                                    void* work, size_t work_bytes, hipStream_t stream);

/* Per-kernel timing for measurement.  While enabled, every kernel launch of
 * this context is bracketed with HIP events recorded on its launch stream;
 * hermes_profile_read synchronises the outstanding events and returns, for
 * the index-th kernel class (alphabetical; ERR_ARG past the last one), its
 * name, launch count and summed duration in milliseconds.  Reset clears the
 * totals.  Timing adds two event records per launch. */
hermes_status hermes_profile_enable(hermes_ctx ctx, int enable);
hermes_status hermes_profile_reset(hermes_ctx ctx);
hermes_status hermes_profile_read(hermes_ctx ctx, int index, char* name, size_t name_len,
                                  int64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif

#endif /* HERMES_H */
