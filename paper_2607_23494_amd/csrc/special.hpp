// Device special functions for the window kernels, all in float64:
// spherical Bessel j_l, the spherical top-hat and thick-shell windows, the
// r^2-weighted bin average of j_l, real spherical harmonics and Legendre
// polynomials.
#pragma once

#include "common.hpp"

namespace hermes {

constexpr int kGLSub = 16;  // Gauss-Legendre nodes per sub-interval of a bin

// Spherical Bessel function j_l(x), x >= 0.  Power series below x = l + 1
// (where upward recurrence loses accuracy), upward recurrence from j_0, j_1
// above.
__device__ __forceinline__ double sph_jl(int l, double x) {
    if (l == 0) {
        if (x < 1e-3) {
            const double x2 = x * x;
            return 1.0 - x2 / 6.0 + x2 * x2 / 120.0;
        }
        return sin(x) / x;
    }
    if (x < l + 1.0) {
        double pref = 1.0;
        for (int i = 1; i <= l; ++i) pref *= x / (2 * i + 1);
        const double x2h = 0.5 * x * x;
        double term = 1.0, sum = 1.0;
        for (int k = 1; k < 80; ++k) {
            term *= -x2h / (double(k) * (2 * l + 2 * k + 1));
            sum += term;
            if (fabs(term) < 1e-18 * fabs(sum)) break;
        }
        return pref * sum;
    }
    double s, c;
    sincos(x, &s, &c);
    double j0 = s / x;
    double j1 = s / (x * x) - c / x;
    for (int n = 1; n < l; ++n) {
        const double j2 = (2 * n + 1) / x * j1 - j0;
        j0 = j1;
        j1 = j2;
    }
    return j1;
}

// Spherical top-hat 3 (sin x - x cos x) / x^3 (Table A1 (b)).
__device__ __forceinline__ double w_sphere(double x) {
    if (x < 0.05) {
        const double x2 = x * x;
        return 1.0 - x2 / 10.0 + x2 * x2 / 280.0 - x2 * x2 * x2 / 15120.0;
    }
    double s, c;
    sincos(x, &s, &c);
    return 3.0 * (s - x * c) / (x * x * x);
}

// Volume-normalised thick shell, the difference of two spheres (Eq. Wshell_k).
__device__ __forceinline__ double w_shell(double k, double lo, double hi) {
    const double h3 = hi * hi * hi, l3 = lo * lo * lo;
    return (h3 * w_sphere(k * hi) - l3 * w_sphere(k * lo)) / (h3 - l3);
}

// r^2-weighted average of j_l(k r) over [lo, hi] (finite-bin radial factor of
// the multipole windows).  l = 0 is the thick shell in closed form; l > 0 uses
// kGLSub-point Gauss-Legendre on sub-intervals of at most 8 radians of k r.
__device__ __forceinline__ double jbar(int l, double k, double lo, double hi, const double* gl) {
    if (l == 0) return w_shell(k, lo, hi);
    if (k == 0.0) return 0.0;
    const int nsub = max(1, int(ceil(k * (hi - lo) / 8.0)));
    const double width = (hi - lo) / nsub;
    double acc = 0.0;
    for (int s = 0; s < nsub; ++s) {
        const double a = lo + s * width;
        const double mid = a + 0.5 * width, half = 0.5 * width;
        for (int g = 0; g < kGLSub; ++g) {
            const double r = mid + half * gl[g];
            acc += gl[kGLSub + g] * half * r * r * sph_jl(l, k * r);
        }
    }
    return acc * 3.0 / (hi * hi * hi - lo * lo * lo);
}

// Legendre polynomial L_l(mu).
__device__ __forceinline__ double legendre(int l, double mu) {
    if (l == 0) return 1.0;
    double p0 = 1.0, p1 = mu;
    for (int n = 1; n < l; ++n) {
        const double p2 = ((2 * n + 1) * mu * p1 - n * p0) / (n + 1);
        p0 = p1;
        p1 = p2;
    }
    return p1;
}

// Real orthonormal spherical harmonic of the unit vector (x, y, z):
//   m > 0: sqrt2 N_lm P~_l^m(z) Re (x + i y)^m / sin^m theta ...
// computed through Q_l^m(z) = P_l^m(z) / (1 - z^2)^{m/2} so that
// sin^m(theta) e^{i m phi} = (x + i y)^m needs no division; P~ carries no
// Condon-Shortley phase.  m < 0 takes the imaginary part with |m|.  Every
// factor that depends on (l, m) only is prepared once on the host (YlmConst):
// the normalisation sqrt2^{[m != 0]} N_lm (2|m| - 1)!! and the coefficients of
//   Q_ll = a_ll z Q_{ll-1} - b_ll Q_{ll-2},  a = (2 ll - 1)/(ll - |m|),
//   b = (ll + |m| - 1)/(ll - |m|),  Q_{|m|} = 1,  Q_{|m|+1} = (2|m| + 1) z,
// so a mode costs multiplies and adds only.
struct YlmConst {
    int l, m, am;
    double nrm;
    double a[HERMES_MAX_LMAX + 1], b[HERMES_MAX_LMAX + 1];
};

inline YlmConst ylm_const(int l, int m) {
    YlmConst c{};
    c.l = l;
    c.m = m;
    c.am = m < 0 ? -m : m;
    double qmm = 1.0;
    for (int i = 1; i <= c.am; ++i) qmm *= (2 * i - 1);
    double ratio = 1.0;   // (l - |m|)! / (l + |m|)!
    for (int i = l - c.am + 1; i <= l + c.am; ++i) ratio /= i;
    c.nrm = sqrt((2 * l + 1) * ratio / (4.0 * 3.14159265358979323846)) * qmm;
    if (m != 0) c.nrm *= 1.41421356237309504880;
    for (int ll = c.am + 2; ll <= l; ++ll) {
        c.a[ll] = double(2 * ll - 1) / (ll - c.am);
        c.b[ll] = double(ll + c.am - 1) / (ll - c.am);
    }
    return c;
}

__device__ __forceinline__ double ylm_real(const YlmConst& c, double x, double y, double z) {
    double q = 1.0;
    if (c.l > c.am) {
        double q0 = 1.0;
        double q1 = z * (2 * c.am + 1);
        for (int ll = c.am + 2; ll <= c.l; ++ll) {
            const double q2 = c.a[ll] * z * q1 - c.b[ll] * q0;
            q0 = q1;
            q1 = q2;
        }
        q = q1;
    }
    if (c.m == 0) return c.nrm * q;
    double cr = 1.0, ci = 0.0;
    for (int i = 0; i < c.am; ++i) {
        const double t = cr * x - ci * y;
        ci = cr * y + ci * x;
        cr = t;
    }
    return c.nrm * q * (c.m > 0 ? cr : ci);
}

// Y^R_lm at signed mode (sx, sy, sz), averaged over the signed
// representatives +-N/2 of every Nyquist component (nyq_* true).  At k = 0
// the value is 1/sqrt(4 pi) for l = 0 and 0 otherwise.
__device__ __forceinline__ double ylm_mode(const YlmConst& c, int sx, int sy, int sz, bool nyq_x, bool nyq_y,
                                           bool nyq_z) {
    const double q = double(sx) * sx + double(sy) * sy + double(sz) * sz;
    if (q == 0.0) return c.l == 0 ? 0.28209479177387814347 : 0.0;
    const double inv = 1.0 / sqrt(q);
    if (!(nyq_x || nyq_y || nyq_z)) return ylm_real(c, sx * inv, sy * inv, sz * inv);
    double acc = 0.0;
    int cnt = 0;
    for (int fx = 0; fx <= (nyq_x ? 1 : 0); ++fx)
        for (int fy = 0; fy <= (nyq_y ? 1 : 0); ++fy)
            for (int fz = 0; fz <= (nyq_z ? 1 : 0); ++fz) {
                const double x = (fx ? -sx : sx) * inv;
                const double y = (fy ? -sy : sy) * inv;
                const double z = (fz ? -sz : sz) * inv;
                acc += ylm_real(c, x, y, z);
                ++cnt;
            }
    return acc / cnt;
}

}  // namespace hermes
