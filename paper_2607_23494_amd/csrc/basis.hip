// Host-side tables of the Daubechies D4 ("db2") scaling function, the
// orthonormal, compactly supported basis of Sec. 3.1 (the paper's default;
// B3 is the library's other basis).
//
// phi satisfies phi(x) = sqrt2 sum_k h_k phi(2x - k) with the four-tap D4
// filter h = (1 + sqrt3, 3 + sqrt3, 3 - sqrt3, 1 - sqrt3) / (4 sqrt2) and has
// support [0, 3].  Three tables are derived from it:
//  - phi at the dyadic points x = i / 2^12 (linear interpolation between them
//    is the phi used to project and to read fields), built from the integer
//    values phi(1) = (1 + sqrt3)/2, phi(2) = (1 - sqrt3)/2 one level at a time;
//  - |phi^(w)|^2 per axis at the grid modes, by the infinite product
//    prod_j |m0(w / 2^j)|^2 with |m0(w)|^2 = cos^4(w/2) (1 + 2 sin^2(w/2));
//  - the triple connection coefficients gamma(a, b) = int phi(x) phi(x - a)
//    phi(x - b) dx (Eq. con-coeff per axis), the fixed point of the
//    refinement map gamma(a, b) = sqrt2 sum_{i,j,k} h_i h_j h_k
//    gamma(2a + j - i, 2b + k - i) found by power iteration (its other
//    eigenvalues are at most 1/2 in modulus), normalised by sum gamma = 1,
//    and its eigen-decomposition gamma = V diag(lambda) V^T by Jacobi sweeps.
#include <cmath>
#include <vector>

#include "common.hpp"

namespace hermes {

static void db2_filter(double h[4]) {
    const double s = std::sqrt(3.0), d = 4.0 * std::sqrt(2.0);
    h[0] = (1.0 + s) / d;
    h[1] = (3.0 + s) / d;
    h[2] = (3.0 - s) / d;
    h[3] = (1.0 - s) / d;
}

std::vector<double> db2_phi_table() {
    double h[4];
    db2_filter(h);
    const double s3 = std::sqrt(3.0);
    // level 0: x = 0, 1, 2, 3
    std::vector<double> cur = {0.0, 0.5 * (1.0 + s3), 0.5 * (1.0 - s3), 0.0};
    for (int lev = 1; lev <= kDb2Level; ++lev) {
        const int half = 1 << (lev - 1);      // index distance of one unit of x on the previous level
        std::vector<double> nxt(size_t(3) * (size_t(1) << lev) + 1, 0.0);
        for (size_t i = 0; i < cur.size(); ++i) nxt[2 * i] = cur[i];
        for (size_t i = 1; i < nxt.size(); i += 2) {
            // x = i / 2^lev: phi(x) = sqrt2 sum_k h_k phi(2x - k), 2x - k = (i - k 2^(lev-1)) / 2^(lev-1)
            double acc = 0.0;
            for (int k = 0; k < 4; ++k) {
                const long j = long(i) - long(k) * half;
                if (j >= 0 && j < long(cur.size())) acc += h[k] * cur[size_t(j)];
            }
            nxt[i] = std::sqrt(2.0) * acc;
        }
        cur.swap(nxt);
    }
    return cur;
}

double db2_phi_hat_sq(double w) {
    double p = 1.0;
    for (int j = 1; j <= 60; ++j) {
        const double a = 0.5 * std::ldexp(w, -j);
        const double c = std::cos(a), s = std::sin(a);
        p *= c * c * c * c * (1.0 + 2.0 * s * s);
    }
    return p;
}

// gamma[a + 2][b + 2] for a, b in [-2, 2].
static void db2_gamma(double g[5][5]) {
    double h[4];
    db2_filter(h);
    double t[25][25] = {};
    for (int a = -2; a <= 2; ++a)
        for (int b = -2; b <= 2; ++b)
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j)
                    for (int k = 0; k < 4; ++k) {
                        const int a2 = 2 * a + j - i, b2 = 2 * b + k - i;
                        if (a2 < -2 || a2 > 2 || b2 < -2 || b2 > 2) continue;
                        t[(a + 2) * 5 + b + 2][(a2 + 2) * 5 + b2 + 2] += std::sqrt(2.0) * h[i] * h[j] * h[k];
                    }
    double v[25] = {};
    v[2 * 5 + 2] = 1.0;   // gamma(0, 0) carries most of the weight
    for (int it = 0; it < 200; ++it) {
        double w[25] = {}, sum = 0.0;
        for (int r = 0; r < 25; ++r) {
            for (int c = 0; c < 25; ++c) w[r] += t[r][c] * v[c];
            sum += w[r];
        }
        for (int r = 0; r < 25; ++r) v[r] = w[r] / sum;
    }
    for (int a = 0; a < 5; ++a)
        for (int b = 0; b < 5; ++b) g[a][b] = 0.5 * (v[a * 5 + b] + v[b * 5 + a]);   // symmetric up to rounding
}

// Symmetric 5 x 5 eigen-decomposition a = v diag(lam) v^T (cyclic Jacobi).
static void jacobi5(const double in[5][5], double lam[5], double v[5][5]) {
    double a[5][5];
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j) {
            a[i][j] = in[i][j];
            v[i][j] = i == j ? 1.0 : 0.0;
        }
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < 5; ++p)
            for (int q = p + 1; q < 5; ++q) off += a[p][q] * a[p][q];
        if (off < 1e-40) break;
        for (int p = 0; p < 5; ++p)
            for (int q = p + 1; q < 5; ++q) {
                if (a[p][q] == 0.0) continue;
                const double theta = 0.5 * (a[q][q] - a[p][p]) / a[p][q];
                const double tt = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(tt * tt + 1.0), s = tt * c;
                for (int k = 0; k < 5; ++k) {   // columns p, q
                    const double akp = a[k][p], akq = a[k][q];
                    a[k][p] = c * akp - s * akq;
                    a[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < 5; ++k) {   // rows p, q
                    const double apk = a[p][k], aqk = a[q][k];
                    a[p][k] = c * apk - s * aqk;
                    a[q][k] = s * apk + c * aqk;
                }
                for (int k = 0; k < 5; ++k) {
                    const double vkp = v[k][p], vkq = v[k][q];
                    v[k][p] = c * vkp - s * vkq;
                    v[k][q] = s * vkp + c * vkq;
                }
            }
    }
    for (int i = 0; i < 5; ++i) lam[i] = a[i][i];
}

void db2_gamma_factors(double lam[5], double vec[5][5]) {
    double g[5][5];
    db2_gamma(g);
    jacobi5(g, lam, vec);
}

}  // namespace hermes
