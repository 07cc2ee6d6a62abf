"""Plain FP64 CPU oracle of the field-window estimator.

TEST INFRASTRUCTURE ONLY.  Nothing in the library calls this module: it is
imported by the tests, by the smoke check and by the CPU-baseline leg of the
benchmark, and by nothing else.  It shares no code with the HIP path.

Everything here is written for obviousness, not speed: float64 throughout,
full complex spectra (no Hermitian shortcut), explicit loops over l, m and
bins.  Library primitives used as single steps: scipy.fft (a DFT), numpy's
bincount (a histogram), scipy.special (spherical Bessel, cylindrical Bessel
J0 and J1, Legendre, spherical harmonics) and numpy's Gauss-Legendre nodes.

Parts: the two scaling functions (the cubic B-spline, and the orthonormal
Daubechies D4 function with its spectrum and connection coefficients);
assignment, contrast and DFT; the basis kernel and radial windows;
the 2PCF and its multipoles by Parseval with the shot-noise factor;
filtered fields and counts-in-cells moments; 3PCF multipoles; readout at
arbitrary positions and density marks; axisymmetric windows and the
anisotropic 2PCF; Monte-Carlo triangle sums with the Philox4x64-10
generator; the connection-coefficient 3PCF monopole.  Every function is
pinned by tests/test_oracle_pins.py against an independent route (closed
forms, brute force on small grids, library routines, invariants); parity is
unpinned only for the conventions named there (the absolute normalisation
of zeta_l against the paper's other convention, and the choice between B3,
the library's default, and the paper's D4 basis).  Every function that
depends on the scaling function takes ``basis`` = "b3" (default) or "db2".

Conventions (the paper's notation; section / equation named per function):
  grid node l = (lx, ly, lz), l_a in {0..N-1}, sits at position l*h, h = L/N;
  array index [lx, ly, lz], lz fastest;
  forward DFT  f^(n) = sum_l f_l exp(-2 pi i n.l/N)  (unnormalised),
  inverse      f_l   = N^-3 sum_n f^(n) exp(+2 pi i n.l/N);
  signed mode index n~_a in (-N/2, N/2], k = 2 pi n~ / L.
"""
from __future__ import annotations

import functools
import os

import numpy as np
import scipy.fft as sfft
from scipy.special import eval_legendre, j0, j1, spherical_jn, sph_harm_y

_WORKERS = max(1, os.cpu_count() or 1)
_GL_POINTS = 64


# ----------------------------------------------------------------------------
# Assignment (Sec. 3.1, Eq. phi_projection): eps_l = sum_i w_i phi(x_i/h - l)
# ----------------------------------------------------------------------------

def bspline3(t):
    """Centred cubic B-spline: the scaling function phi used for projection.

    B3(t) = (4 - 6 t^2 + 3|t|^3)/6 for |t| < 1, (2-|t|)^3/6 for 1 <= |t| < 2,
    0 otherwise.  (Sec. 3.1: compactly supported MRA scaling function.)
    """
    a = np.abs(np.asarray(t, dtype=np.float64))
    out = np.zeros_like(a)
    m1 = a < 1.0
    out[m1] = (4.0 - 6.0 * a[m1] ** 2 + 3.0 * a[m1] ** 3) / 6.0
    m2 = (a >= 1.0) & (a < 2.0)
    out[m2] = (2.0 - a[m2]) ** 3 / 6.0
    return out


# ----------------------------------------------------------------------------
# The Daubechies D4 ("db2") scaling function (Sec. 3.1: an orthonormal,
# compactly supported MRA scaling function; the paper's default basis).
# Refinement relation phi(x) = sqrt2 sum_k h_k phi(2x - k), support [0, 3].
# ----------------------------------------------------------------------------

DB2_LEVEL = 12   # phi is tabulated at x = i / 2^12 and interpolated linearly between


def db2_filter():
    """Low-pass filter h_0..h_3 of the orthonormal Daubechies scaling function
    with two vanishing moments (Daubechies 1988, the D4 filter):
    h = (1 + sqrt3, 3 + sqrt3, 3 - sqrt3, 1 - sqrt3) / (4 sqrt2)."""
    s = np.sqrt(3.0)
    return np.array([1.0 + s, 3.0 + s, 3.0 - s, 1.0 - s]) / (4.0 * np.sqrt(2.0))


def db2_phi_integers():
    """phi(0), phi(1), phi(2), phi(3): the refinement relation at the integers,
    phi(i) = sqrt2 sum_j h_{2i-j} phi(j), makes them an eigenvector of
    eigenvalue 1, normalised so that sum_i phi(i) = 1 (partition of unity)."""
    h = db2_filter()
    m = np.zeros((4, 4))
    for i in range(4):
        for j in range(4):
            if 0 <= 2 * i - j < 4:
                m[i, j] = np.sqrt(2.0) * h[2 * i - j]
    w, v = np.linalg.eig(m)
    e = np.real(v[:, np.argmin(np.abs(w - 1.0))])
    return e / e.sum()


@functools.lru_cache(maxsize=4)
def _db2_table(level):
    h = db2_filter()
    cur = db2_phi_integers()
    for lev in range(1, level + 1):
        step = 2 ** (lev - 1)            # one unit of x in the previous level's index
        new = np.zeros(3 * 2 ** lev + 1)
        new[0::2] = cur                  # the previous level's points
        for i in range(1, new.size, 2):  # the new points x = i / 2^lev
            s = 0.0
            for k in range(4):
                j = i - k * step         # 2x - k on the previous level
                if 0 <= j < cur.size:
                    s += h[k] * cur[j]
            new[i] = np.sqrt(2.0) * s
        cur = new
    cur.setflags(write=False)
    return cur


def db2_phi_table(level=DB2_LEVEL):
    """phi at x = i / 2^level, i = 0 .. 3 * 2^level, from the integer values by
    the refinement relation, one dyadic level at a time."""
    return _db2_table(int(level)).copy()


def db2_phi(x, level=DB2_LEVEL):
    """The D4 scaling function as used to project and read fields: the level
    table interpolated linearly, zero outside [0, 3]."""
    t = _db2_table(int(level))
    grid = np.arange(t.size) / 2.0 ** level
    return np.interp(np.asarray(x, dtype=np.float64), grid, t, left=0.0, right=0.0)


def db2_m0_sq(w):
    """|m0(w)|^2 with m0(w) = 2^-1/2 sum_k h_k e^{-i k w}: the squared
    frequency response of the refinement filter."""
    h = db2_filter()
    w = np.asarray(w, dtype=np.float64)
    m = sum(h[k] * np.exp(-1j * k * w) for k in range(4)) / np.sqrt(2.0)
    return np.abs(m) ** 2


def db2_phi_hat_sq(w):
    """|phi^(w)|^2, the Fourier transform of the D4 autocorrelation, by the
    infinite product phi^(w) = prod_{j >= 1} m0(w / 2^j) (phi^(0) = 1),
    truncated after 60 factors (the rest are 1 in float64 for |w| <= pi)."""
    w = np.asarray(w, dtype=np.float64)
    p = np.ones_like(w)
    for j in range(1, 61):
        p = p * db2_m0_sq(w / 2.0 ** j)
    return p


def db2_connection_1d():
    """gamma[a + 2, b + 2] = int phi(x) phi(x - a) phi(x - b) dx, a, b in
    [-2, 2] (Eq. con-coeff per axis; zero where the supports do not meet).

    Inserting the refinement relation into the three factors gives
    gamma(a, b) = sqrt2 sum_{i,j,k} h_i h_j h_k gamma(2a + j - i, 2b + k - i),
    with gamma = 0 outside [-2, 2]^2: the eigenvector of eigenvalue 1, scaled
    so that sum_{a,b} gamma(a, b) = int phi (sum_a phi(. - a))^2 = 1."""
    h = db2_filter()
    pairs = [(a, b) for a in range(-2, 3) for b in range(-2, 3)]
    index = {p: i for i, p in enumerate(pairs)}
    t = np.zeros((25, 25))
    for (a, b), row in index.items():
        for i in range(4):
            for j in range(4):
                for k in range(4):
                    tgt = (2 * a + j - i, 2 * b + k - i)
                    if tgt in index:
                        t[row, index[tgt]] += np.sqrt(2.0) * h[i] * h[j] * h[k]
    w, v = np.linalg.eig(t)
    e = np.real(v[:, np.argmin(np.abs(w - 1.0))])
    e = e / e.sum()
    g = np.zeros((5, 5))
    for (a, b), row in index.items():
        g[a + 2, b + 2] = e[row]
    return g


def db2_derivative_coefficients():
    """r[m + 2] = int phi(x - m) phi'(x) dx, m in [-2, 2] (App. B, the
    derivative connection coefficients of the D4 basis).  Inserting the
    refinement relation gives r_m = 2 sum_{i,k} h_i h_k r_{2m+i-k}: the
    eigenvector of eigenvalue 1, scaled so that sum_m m r_m = -1 (from
    sum_m m phi(x - m) = x - const and integration by parts).  Used only to
    pin the filter and the refinement method against the paper's values."""
    h = db2_filter()
    a = np.zeros((5, 5))
    for m in range(-2, 3):
        for i in range(4):
            for k in range(4):
                tgt = 2 * m + i - k
                if -2 <= tgt <= 2:
                    a[m + 2, tgt + 2] += 2.0 * h[i] * h[k]
    w, v = np.linalg.eig(a)
    e = np.real(v[:, np.argmin(np.abs(w - 1.0))])
    return e / -np.dot(np.arange(-2, 3), e)


BASES = ("b3", "db2")


def basis_nodes(basis):
    """Per axis, the nodes a point at u (cell units, i0 = floor(u)) reaches:
    (first offset, count, phi), nodes i0 + off .. i0 + off + count - 1 with
    weight phi(u - l).  B3 (support [-2, 2]): i0-1 .. i0+2; D4 (support
    [0, 3]): i0-2 .. i0."""
    if basis == "b3":
        return -1, 4, bspline3
    if basis == "db2":
        return -2, 3, db2_phi
    raise ValueError(basis)


def assign(pos, weight, box_L, n, basis="b3"):
    """Project a weighted catalogue onto the N^3 grid of scaling-function
    coefficients.

    Sec. 3.1, Eq. phi_projection: eps_l = sum_i w_i prod_a phi(x_{i,a}/h - l_a),
    node index taken mod N (periodic box); phi = B3 or the D4 function.
    ``weight`` None means unit weights (Eq. dendis with w_i = 1; Eq.
    weighted_field for marks).  Returns (eps [N,N,N] float64, sum of weights).
    """
    off, nn, phi = basis_nodes(basis)
    pos = np.asarray(pos, dtype=np.float32)
    h = float(box_L) / n
    u = pos.astype(np.float64) / h
    npts = u.shape[0]
    w = np.ones(npts) if weight is None else np.asarray(weight, dtype=np.float64)
    i0 = np.floor(u).astype(np.int64)
    eps = np.zeros(n ** 3)
    # per axis: node index (mod N) and weight of the nodes i0+off .. i0+off+nn-1
    offs = range(off, off + nn)
    cells = [[np.mod(i0[:, a] + o, n) for o in offs] for a in range(3)]
    taps = [[phi(u[:, a] - (i0[:, a] + o)) for o in offs] for a in range(3)]
    for ox in range(nn):
        # the (oy, oz) taps of one ox in a single histogram call
        flat = np.concatenate([(cells[0][ox] * n + cells[1][oy]) * n + cells[2][oz]
                               for oy in range(nn) for oz in range(nn)])
        vals = np.concatenate([w * taps[0][ox] * taps[1][oy] * taps[2][oz]
                               for oy in range(nn) for oz in range(nn)])
        eps += np.bincount(flat, weights=vals, minlength=n ** 3)
    return eps.reshape(n, n, n), float(w.sum())


def contrast(eps, sum_w):
    """delta_l = eps_l / eps_bar - 1 with eps_bar = sum_w / N^3 (Sec. 2 notation;
    Sec. 4.2 field_mean_density; uniform analytic random, Sec. 4.3.1)."""
    n3 = eps.size
    return eps / (sum_w / n3) - 1.0


def dft3(field):
    """Full complex forward DFT of a real field; the k=0 mode is set to zero."""
    fh = sfft.fftn(np.asarray(field, dtype=np.complex128), workers=_WORKERS)
    fh[0, 0, 0] = 0.0
    return fh


def idft3(spec):
    """Inverse DFT including the N^-3 factor (complex result)."""
    return sfft.ifftn(spec, workers=_WORKERS)


# ----------------------------------------------------------------------------
# Mode geometry and the basis kernel (Sec. 3.3.1 Eq. shift-scaling_coeff-kspace;
# Sec. 4.2 discrete kernel K_W = W^ Phi^)
# ----------------------------------------------------------------------------

def signed_index(n, nyquist_sign=+1):
    """Signed mode index per axis; the Nyquist index N/2 (even N) maps to
    +N/2 or -N/2 according to ``nyquist_sign``."""
    i = np.arange(n)
    s = np.where(i <= n // 2, i, i - n).astype(np.float64)
    if n % 2 == 0 and nyquist_sign < 0:
        s[n // 2] = -n / 2
    return s


def phi_hat_1d(n, basis="b3"):
    """Per-axis Fourier transform of the basis autocorrelation at the grid
    modes, alias images dropped (Eq. shift-scaling_coeff-kspace keeps only the
    principal mode): |B3^|^2 = sinc^8(pi n~/N), or |phi^|^2 of the D4 function
    at w = 2 pi n~/N."""
    s = signed_index(n)
    if basis == "db2":
        return db2_phi_hat_sq(2.0 * np.pi * s / n)
    if basis != "b3":
        raise ValueError(basis)
    return np.sinc(s / n) ** 8          # np.sinc(x) = sin(pi x)/(pi x)


def phi_hat(n, basis="b3"):
    p = phi_hat_1d(n, basis)
    return p[:, None, None] * p[None, :, None] * p[None, None, :]


def mode_vectors(n, box_L, signs=(1, 1, 1)):
    """k-vector components (broadcastable [N,1,1], [1,N,1], [1,1,N])."""
    f = 2.0 * np.pi / box_L
    kx = f * signed_index(n, signs[0])[:, None, None]
    ky = f * signed_index(n, signs[1])[None, :, None]
    kz = f * signed_index(n, signs[2])[None, None, :]
    return kx, ky, kz


def mode_q(n):
    """Integer |n~|^2 for every mode (Nyquist sign irrelevant)."""
    s = signed_index(n).astype(np.int64)
    return s[:, None, None] ** 2 + s[None, :, None] ** 2 + s[None, None, :] ** 2


# ----------------------------------------------------------------------------
# Window functions (Sec. 2.2.1 Eqs. Wshell, Wshell_k; Table A1 (a)-(c);
# Sec. 3.3.3 multipole windows)
# ----------------------------------------------------------------------------

def w_sphere(x):
    """Spherical top-hat 3(sin x - x cos x)/x^3 (Table A1 (b)); Taylor series
    1 - x^2/10 + x^4/280 - x^6/15120 below x = 0.05."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    small = np.abs(x) < 0.05
    xs = x[small]
    x2 = xs * xs
    out[small] = 1.0 - x2 / 10.0 + x2 * x2 / 280.0 - x2 * x2 * x2 / 15120.0
    xl = x[~small]
    out[~small] = 3.0 * (np.sin(xl) - xl * np.cos(xl)) / xl ** 3
    return out


def w_shell(k, r_lo, r_hi):
    """Volume-normalised thick shell: difference of two spheres (Eq. Wshell_k)."""
    return (r_hi ** 3 * w_sphere(k * r_hi) - r_lo ** 3 * w_sphere(k * r_lo)) / (r_hi ** 3 - r_lo ** 3)


def w_gauss(k, R):
    """Gaussian low-pass exp(-k^2 R^2 / 2) (Table A1 (c))."""
    return np.exp(-0.5 * (k * R) ** 2)


def jbar(ell, k, r_lo, r_hi):
    """Finite-bin radial factor: the r^2-weighted bin average of j_l(k r)
    (Sec. 3.3.3: replace j_l(kr) by its average over the radial window),
    by 64-point Gauss-Legendre quadrature on [r_lo, r_hi]."""
    k = np.asarray(k, dtype=np.float64)
    x, wq = np.polynomial.legendre.leggauss(_GL_POINTS)
    r = 0.5 * (r_hi - r_lo) * x + 0.5 * (r_hi + r_lo)
    wr = 0.5 * (r_hi - r_lo) * wq * r * r
    vol = (r_hi ** 3 - r_lo ** 3) / 3.0
    flat = k.reshape(-1)
    out = np.zeros(flat.shape)
    for rj, wj in zip(r, wr):
        out += wj * spherical_jn(ell, flat * rj)
    return (out / vol).reshape(k.shape)


def ylm_real(ell, m, kx, ky, kz):
    """Real orthonormal spherical harmonic of the direction of k.

    m > 0: sqrt2 (-1)^m Re Y_l^m; m < 0: sqrt2 (-1)^m Im Y_l^|m|; m = 0: Y_l^0.
    At k = 0 the value is 1/sqrt(4 pi) for l = 0 and 0 otherwise.
    """
    kx, ky, kz = np.broadcast_arrays(kx, ky, kz)
    kk = np.sqrt(kx * kx + ky * ky + kz * kz)
    zero = kk == 0.0
    safe = np.where(zero, 1.0, kk)
    theta = np.arccos(np.clip(kz / safe, -1.0, 1.0))
    phi = np.arctan2(ky, kx)
    y = sph_harm_y(ell, abs(m), theta, phi)
    if m > 0:
        out = np.sqrt(2.0) * (-1) ** m * y.real
    elif m < 0:
        out = np.sqrt(2.0) * (-1) ** m * y.imag
    else:
        out = y.real.copy()
    out = np.where(zero, (1.0 / np.sqrt(4.0 * np.pi)) if ell == 0 else 0.0, out)
    return out


def radial_by_q(n, box_L, fn):
    """Evaluate a radial function of |k| once per integer q = |n~|^2 in
    [0, max q] and spread it over the grid (same value at every mode of
    equal |k|)."""
    q = mode_q(n)
    kq = 2.0 * np.pi / box_L * np.sqrt(np.arange(int(q.max()) + 1, dtype=np.float64))
    return fn(kq)[q]


def nyquist_average(n, box_L, fn):
    """Average a k-space kernel over the two signed representatives of every
    Nyquist index (even N): K(n) = mean over s in {+,-}^3 of fn(k_s), where
    only components at the Nyquist index change sign.  Off the Nyquist planes
    all eight evaluations coincide, so K equals fn there and only the modes
    on a Nyquist plane are re-evaluated."""
    kx, ky, kz = mode_vectors(n, box_L)
    out = np.array(np.broadcast_to(fn(kx, ky, kz), (n, n, n)), dtype=np.float64)
    if n % 2:
        return out
    h = n // 2
    ix, iy, iz = np.nonzero((np.arange(n)[:, None, None] == h) | (np.arange(n)[None, :, None] == h)
                            | (np.arange(n)[None, None, :] == h))
    f = 2.0 * np.pi / box_L
    acc = np.zeros(ix.size)
    for sx in (1, -1):
        for sy in (1, -1):
            for sz in (1, -1):
                acc += fn(f * signed_index(n, sx)[ix], f * signed_index(n, sy)[iy], f * signed_index(n, sz)[iz])
    out[ix, iy, iz] = acc / 8.0
    return out


# ----------------------------------------------------------------------------
# Two-point statistics by Parseval (Sec. 3.3.1 Eqs. pair-counting-kspace,
# xi-deltaDD-over-RR; Sec. 3.3.3 Legendre multipoles DD_l)
# ----------------------------------------------------------------------------

def xi_multipoles(delta_hat, box_L, edges, ells=(0,), los_axis=2, basis="b3"):
    """xi_l[b] = N^-6 sum_n |delta^_n|^2 Phi^(n) (2l+1) i^l jbar_l(k;b) L_l(mu_k).

    Full spectrum, every mode.  l = 0 uses the thick-shell window (identical
    to jbar_0).  Only even l carry a real value; odd l are rejected.
    Returns float64 [len(ells), n_bins].
    """
    n = delta_hat.shape[0]
    nc = float(n) ** 3
    edges = np.asarray(edges, dtype=np.float64)
    p = (np.abs(delta_hat) ** 2) * phi_hat(n, basis)
    kx, ky, kz = mode_vectors(n, box_L)
    kk = np.sqrt(kx * kx + ky * ky + kz * kz)
    klos = (kx, ky, kz)[los_axis]
    mu = np.where(kk > 0, klos / np.where(kk > 0, kk, 1.0), 0.0)
    out = np.zeros((len(ells), len(edges) - 1))
    for il, ell in enumerate(ells):
        if ell % 2:
            raise ValueError("odd multipoles of the auto-correlation vanish; use even l")
        leg = eval_legendre(ell, mu) if ell > 0 else 1.0
        pref = (2 * ell + 1) * (-1) ** (ell // 2)
        pl = p * leg
        for b in range(len(edges) - 1):
            lo, hi = edges[b], edges[b + 1]
            if ell == 0:
                rad = radial_by_q(n, box_L, lambda kq: w_shell(kq, lo, hi))
            else:
                rad = radial_by_q(n, box_L, lambda kq: jbar(ell, kq, lo, hi))
            out[il, b] = pref * np.sum(pl * rad) / nc ** 2
    return out


# B3 autocorrelation at integer lags: the centred B-spline of degree 7.
B7_LAGS = {0: 2416.0 / 5040.0, 1: 1191.0 / 5040.0, 2: 120.0 / 5040.0, 3: 1.0 / 5040.0}


def self_pair_lags(basis="b3"):
    """Autocorrelation int phi(x) phi(x - d) dx of the basis at integer lags
    d >= 0 (the cell average of the self-pair kernel): the degree-7 B-spline
    for B3; the Kronecker delta for the orthonormal D4 function."""
    if basis == "b3":
        return B7_LAGS
    if basis == "db2":
        return {0: 1.0}
    raise ValueError(basis)


def shot_factor(n, box_L, edges, ells=(0,), los_axis=2, basis="b3"):
    """Shot-noise factor of the Parseval 2PCF estimator (reading of the
    self-pair term of Sec. 2.2 Eq. CFpow for the field estimator):
        S_lb = sum_D K_lb(D) B7(D_1) B7(D_2) B7(D_3),  |D_a| <= 3,
    with K_lb(D) = N^-3 sum_n K_lb(n) e^{+2 pi i n.D/N} the real-space window
    kernel of xi_multipoles, K_lb(n) = (2l+1) (-1)^{l/2} R_lb(|k|) L_l(mu) Phi^(n)
    (every mode, n = 0 included), and B7 the B3 autocorrelation at integer
    lags (for the D4 basis the Kronecker delta: S_lb = K_lb(0)).  For iid
    points E xi_lb = (sum w^2 / W^2) (N^3 S_lb - K_lb(0)).
    Returns float64 [len(ells), n_bins].
    """
    edges = np.asarray(edges, dtype=np.float64)
    kx, ky, kz = mode_vectors(n, box_L)
    kk = np.sqrt(kx * kx + ky * ky + kz * kz)
    klos = (kx, ky, kz)[los_axis]
    mu = np.where(kk > 0, klos / np.where(kk > 0, kk, 1.0), 0.0)
    ph = phi_hat(n, basis)
    ac = self_pair_lags(basis)
    lags = range(-max(ac), max(ac) + 1)
    out = np.zeros((len(ells), len(edges) - 1))
    for il, ell in enumerate(ells):
        if ell % 2:
            raise ValueError("odd multipoles of the auto-correlation vanish; use even l")
        leg = eval_legendre(ell, mu) if ell > 0 else 1.0
        pref = (2 * ell + 1) * (-1) ** (ell // 2)
        for b in range(len(edges) - 1):
            lo, hi = edges[b], edges[b + 1]
            if ell == 0:
                rad = radial_by_q(n, box_L, lambda kq: w_shell(kq, lo, hi))
            else:
                rad = radial_by_q(n, box_L, lambda kq: jbar(ell, kq, lo, hi))
            kd = idft3(pref * rad * leg * ph).real
            s = 0.0
            for dx in lags:
                for dy in lags:
                    for dz in lags:
                        s += kd[dx % n, dy % n, dz % n] * ac[abs(dx)] * ac[abs(dy)] * ac[abs(dz)]
            out[il, b] = s
    return out


# ----------------------------------------------------------------------------
# Counts-in-cells moments (Sec. 3.1 filtered field n_W; Sec. 2.2.2 Eq. varw)
# ----------------------------------------------------------------------------

def filtered_field(delta_hat, box_L, kernel_of_k, basis="b3"):
    """delta_W = Re iDFT[delta^ Phi^ W^(|k|)] for a radial window."""
    n = delta_hat.shape[0]
    rad = radial_by_q(n, box_L, kernel_of_k)
    return idft3(delta_hat * phi_hat(n, basis) * rad).real


def cic_window(kind, R):
    """The radial window W^(|k|) of a counts-in-cells cell: "sphere" (Table A1
    (b)) or "gauss" (Table A1 (c)) of radius R."""
    if kind == "sphere":
        return lambda kq: w_sphere(kq * R)
    if kind == "gauss":
        return lambda kq: w_gauss(kq, R)
    raise ValueError(kind)


def field_moments(field):
    """<f^2>, <f^3>, <f^4>: means over all grid nodes (Sec. 2.2.2 Eq. varw and
    its higher-order analogues)."""
    return np.array([np.mean(field ** 2), np.mean(field ** 3), np.mean(field ** 4)])


def cic_moments(delta_hat, box_L, windows, basis="b3"):
    """<delta_W^p> for p = 2, 3, 4 (mean over all grid nodes) per window.

    ``windows``: list of ("sphere"|"gauss", R).  Returns float64 [n_win, 3].
    """
    out = np.zeros((len(windows), 3))
    for i, (kind, R) in enumerate(windows):
        out[i] = field_moments(filtered_field(delta_hat, box_L, cic_window(kind, R), basis))
    return out


# ----------------------------------------------------------------------------
# 3PCF multipoles (Sec. 3.3.3 Eqs. multipole-window, iFFT-multipoleSFC,
# 2-fold-translation; Sec. 3.4 particle_nfold with a naked primary vertex)
# ----------------------------------------------------------------------------

def sh_window(n, box_L, ell, m):
    """Nyquist-averaged real spherical harmonic Y^R_lm(k^) on the grid."""
    return nyquist_average(n, box_L, lambda kx, ky, kz: ylm_real(ell, m, kx, ky, kz))


def multipole_field(delta_hat, box_L, ell, m, r_lo, r_hi, ylm=None, basis="b3"):
    """a_lmb(x) = iDFT[delta^ Phi^ 4 pi i^l jbar_l(k;b) Y^R_lm(k^)] (real).

    Returns (real part, max |imag part|).
    """
    n = delta_hat.shape[0]
    if ylm is None:
        ylm = sh_window(n, box_L, ell, m)
    rad = radial_by_q(n, box_L, lambda kq: jbar(ell, kq, r_lo, r_hi))
    kern = 4.0 * np.pi * (1j ** ell) * rad * ylm * phi_hat(n, basis)
    f = idft3(delta_hat * kern)
    return f.real, float(np.max(np.abs(f.imag)))


def zeta_multipoles(delta, delta_hat, box_L, edges, ells, bins=None, basis="b3"):
    """zeta_l[b1,b2] = (4 pi N^3)^-1 sum_m sum_x delta(x) a_lmb1(x) a_lmb2(x).

    Explicit loops over l in ``ells``, m = -l..l and the bins in ``bins``
    (default all).  Returns float64 [len(ells), len(bins), len(bins)].
    """
    n = delta_hat.shape[0]
    nc = float(n) ** 3
    edges = np.asarray(edges, dtype=np.float64)
    if bins is None:
        bins = list(range(len(edges) - 1))
    out = np.zeros((len(ells), len(bins), len(bins)))
    for il, ell in enumerate(ells):
        for m in range(-ell, ell + 1):
            ylm = sh_window(n, box_L, ell, m)
            fields = []
            for b in bins:
                a, _ = multipole_field(delta_hat, box_L, ell, m, edges[b], edges[b + 1], ylm, basis)
                fields.append(a)
            for i in range(len(bins)):
                da = delta * fields[i]
                for j in range(len(bins)):
                    out[il, i, j] += np.sum(da * fields[j])
        out[il] /= 4.0 * np.pi * nc
    return out


# ----------------------------------------------------------------------------
# Readout at arbitrary positions and density-derived marks (Sec. 3.1: the
# filtered field n_W(x) = sum_l eps~_l phi_l(x) read at any point; Sec. 3.3.1
# Eqs. power-law-mark, inverse-density-mark)
# ----------------------------------------------------------------------------

def readout(field, pos, box_L, basis="b3"):
    """Value of the scaling-function expansion of a coefficient field at
    arbitrary points: v_i = sum_l f_l prod_a phi(x_{i,a}/h - l_a), l mod N.

    Sec. 3.1 reads the filtered field n_W(x) = sum_l eps~_l phi_l(x) at any
    position; the value at a point is this 64-node (B3) or 27-node (D4) sum,
    the transpose of the assignment's scatter (no Gram inverse for B3).
    Returns float64 [n_pts].
    """
    return interpolate(field, np.asarray(pos, dtype=np.float32).astype(np.float64), box_L, basis)


def interpolate(field, x, box_L, basis="b3"):
    """The same node sum at float64 positions x [n, 3] (any real values;
    node indices are taken mod N)."""
    off, nn, phi = basis_nodes(basis)
    f = np.asarray(field, dtype=np.float64)
    n = f.shape[0]
    u = np.asarray(x, dtype=np.float64).reshape(-1, 3) / (float(box_L) / n)
    i0 = np.floor(u).astype(np.int64)
    out = np.zeros(u.shape[0])
    offs = range(off, off + nn)
    for ox in offs:
        ix = np.mod(i0[:, 0] + ox, n)
        wx = phi(u[:, 0] - (i0[:, 0] + ox))
        for oy in offs:
            iy = np.mod(i0[:, 1] + oy, n)
            wy = phi(u[:, 1] - (i0[:, 1] + oy))
            for oz in offs:
                iz = np.mod(i0[:, 2] + oz, n)
                wz = phi(u[:, 2] - (i0[:, 2] + oz))
                out += wx * wy * wz * f[ix, iy, iz]
    return out


def readout_moments(field, pos, box_L, basis="b3"):
    """<v^p>, p = 2, 3, 4, the mean over the points of the read-out values
    (counts in cells by sampling positions, Sec. 3.1)."""
    v = readout(field, pos, box_L, basis)
    return np.array([np.mean(v ** 2), np.mean(v ** 3), np.mean(v ** 4)])


def density_mark(dens, kind, exponent, offset, self_term=0.0):
    """Marks from the smoothed density read at the points.

    ``dens`` = 1 + delta_R(x_i); the local density in units of the mean is
    rho = max(dens - self_term, 0) (``self_term`` removes the point's own
    contribution, as the paper's marked-2PCF example does, and the clip keeps
    the density non-negative).
      power_law:       m = (rho + offset)^exponent,  offset = epsilon
                       (Eq. power-law-mark)
      inverse_density: m = ((offset + 1) / (offset + rho))^exponent,
                       offset = rho_* / rho_bar (Eq. inverse-density-mark)
    """
    rho = np.maximum(np.asarray(dens, dtype=np.float64) - self_term, 0.0)
    if kind == "power_law":
        return (rho + offset) ** exponent
    if kind == "inverse_density":
        return ((offset + 1.0) / (offset + rho)) ** exponent
    raise ValueError(kind)


def marked_xi(pos, weight, box_L, n, edges, R, kind, exponent, offset, self_term=0.0, basis="b3"):
    """The density-marked 2PCF of Sec. 3.3.1 (and its example in Sec. 4.3.2):
    smooth the number field with a spherical window of radius R, read 1 +
    delta_R at every point, form the marks, project the mark-weighted
    catalogue and measure its 2PCF; M(r) = (1 + xi_m) / (1 + xi).

    Returns (xi_marked [n_bins], xi [n_bins], M [n_bins]).
    """
    eps, sw = assign(pos, None, box_L, n, basis)
    dh = dft3(contrast(eps, sw))
    xi = xi_multipoles(dh, box_L, edges, basis=basis)[0]
    dR = filtered_field(dh, box_L, lambda kq: w_sphere(kq * R), basis)
    m = density_mark(1.0 + readout(dR, pos, box_L, basis), kind, exponent, offset, self_term)
    w = m if weight is None else np.asarray(weight, dtype=np.float64) * m
    eps_m, sw_m = assign(pos, w, box_L, n, basis)
    xi_m = xi_multipoles(dft3(contrast(eps_m, sw_m)), box_L, edges, basis=basis)[0]
    return xi_m, xi, (1.0 + xi_m) / (1.0 + xi)


# ----------------------------------------------------------------------------
# Axisymmetric windows and the anisotropic 2PCF (Sec. 2.2.3, redshift space:
# circular ring; Table A1 (d)-(i)).  k_par is the line-of-sight component of
# k, k_perp = |k - k_par e_los|.
# ----------------------------------------------------------------------------

ANISO_KINDS = ("ring", "ring_bin", "gauss_ring", "disk", "cylinder", "cylshell", "gauss_shell")


def ring_bin_j0(kperp, r_perp, d_perp):
    """<J0(k_perp rho)> over the annulus rho in [r_perp - d/2, r_perp + d/2]
    with weight rho / (r_perp d) (the finite-width ring of Sec. 2.2.3), by
    64-point Gauss-Legendre quadrature."""
    kperp = np.asarray(kperp, dtype=np.float64)
    x, wq = np.polynomial.legendre.leggauss(_GL_POINTS)
    a, b = r_perp - 0.5 * d_perp, r_perp + 0.5 * d_perp
    rho = 0.5 * (b - a) * x + 0.5 * (b + a)
    wr = 0.5 * (b - a) * wq * rho / (r_perp * d_perp)
    flat = kperp.reshape(-1)
    out = np.zeros(flat.shape)
    for rj, wj in zip(rho, wr):
        out += wj * j0(flat * rj)
    return out.reshape(kperp.shape)


def _sinc(x):
    """sin(x) / x with the limit 1 at 0."""
    x = np.asarray(x, dtype=np.float64)
    return np.sinc(x / np.pi)


def _jinc(x):
    """2 J1(x) / x with the limit 1 at 0."""
    x = np.asarray(x, dtype=np.float64)
    safe = np.where(x == 0.0, 1.0, x)
    return np.where(x == 0.0, 1.0, 2.0 * j1(safe) / safe)


def w_aniso(kind, kpar, kperp, r_perp, r_par, d_perp=0.0, d_par=0.0):
    """Fourier-space axisymmetric window (Table A1 and Sec. 2.2.3):

      ring        cos(k_par H) J0(k_perp R)                          (i)
      ring_bin    sinc(k_par dH/2) cos(k_par H) <J0(k_perp rho)>_dR   (finite bins)
      gauss_ring  cos(k_par H) J0(k_perp R) exp(-k_perp^2 s^2 / 2)    (s = d_perp)
      disk        2 J1(k_perp R)/(k_perp R) cos(k_par H)              (h)
      cylinder    2 J1(k_perp R)/(k_perp R) sin(k_par H)/(k_par H)    (f)
      cylshell    J0(k_perp R) sin(k_par H)/(k_par H)                 (g)
      gauss_shell (Rg^2 cos(k Rs) + Rs^2 sin(k Rs)/(k Rs)) / (Rs^2 + Rg^2)
                  exp(-k^2 Rg^2 / 2), k^2 = k_par^2 + k_perp^2,       (d)
                  Rs = r_perp, Rg = d_perp
    with R = r_perp, H = r_par.
    """
    kpar = np.asarray(kpar, dtype=np.float64)
    kperp = np.asarray(kperp, dtype=np.float64)
    if kind == "ring":
        return np.cos(kpar * r_par) * j0(kperp * r_perp)
    if kind == "ring_bin":
        return _sinc(0.5 * kpar * d_par) * np.cos(kpar * r_par) * ring_bin_j0(kperp, r_perp, d_perp)
    if kind == "gauss_ring":
        return np.cos(kpar * r_par) * j0(kperp * r_perp) * np.exp(-0.5 * (kperp * d_perp) ** 2)
    if kind == "disk":
        return _jinc(kperp * r_perp) * np.cos(kpar * r_par)
    if kind == "cylinder":
        return _jinc(kperp * r_perp) * _sinc(kpar * r_par)
    if kind == "cylshell":
        return j0(kperp * r_perp) * _sinc(kpar * r_par)
    if kind == "gauss_shell":
        k = np.sqrt(kpar * kpar + kperp * kperp)
        rs, rg = r_perp, d_perp
        return ((rg * rg * np.cos(k * rs) + rs * rs * _sinc(k * rs)) / (rs * rs + rg * rg)
                * np.exp(-0.5 * (k * rg) ** 2))
    raise ValueError(kind)


def xi_aniso(delta_hat, box_L, windows, los_axis=2, basis="b3"):
    """xi_W = N^-6 sum_n |delta^_n|^2 Phi^(n) W^(k_par, k_perp) for every
    window (Sec. 2.2.3 Eq. for xi(r_par, r_perp) as the field-window product;
    Sec. 3.3.1 Parseval form).  Full spectrum, every mode.
    ``windows``: tuples (kind, r_perp, r_par[, d_perp[, d_par]]).
    Returns float64 [len(windows)]."""
    n = delta_hat.shape[0]
    nc = float(n) ** 3
    p = (np.abs(delta_hat) ** 2) * phi_hat(n, basis)
    k = mode_vectors(n, box_L)
    kpar = k[los_axis]
    others = [k[a] for a in range(3) if a != los_axis]
    kperp = np.sqrt(others[0] ** 2 + others[1] ** 2)
    out = np.zeros(len(windows))
    for i, w in enumerate(windows):
        kind, rp, rl = w[0], float(w[1]), float(w[2])
        dp = float(w[3]) if len(w) > 3 else 0.0
        dl = float(w[4]) if len(w) > 4 else 0.0
        out[i] = np.sum(p * w_aniso(kind, kpar, kperp, rp, rl, dp, dl)) / nc ** 2
    return out


# ----------------------------------------------------------------------------
# Monte-Carlo triangle sampling (Sec. 3.4, particle-based summation, Eq.
# particle-based-sum; Sec. 4.3.3, the dual-/triplet-sphere 3PCF): triangles
# with sides r12, r13 and opening angle theta, randomly rotated about a
# primary vertex that is a catalogue point (dual sphere) or a uniform random
# point of the box (triplet sphere); the secondary vertices read filtered
# fields.  Random numbers come from the counter-based Philox4x64-10 generator,
# so every sample is addressed by its (centre, rotation) indices.
# ----------------------------------------------------------------------------

_PHILOX_M = (0xD2E7470EE14C6C93, 0xCA5A826395121157)
_PHILOX_W = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)
_U64 = (1 << 64) - 1


def philox4x64(counter, key, rounds=10):
    """One block of Philox4x64 (Salmon, Moraes, Dror and Shaw, SC'11): four
    64-bit words from a four-word counter and a two-word key.  Each round
    multiplies words 0 and 2 by the two constants (128-bit products), mixes
    the high halves with words 1, 3 and the key, and bumps the key by the
    Weyl constants."""
    c0, c1, c2, c3 = (int(v) & _U64 for v in counter)
    k0, k1 = (int(v) & _U64 for v in key)
    for _ in range(rounds):
        p0 = _PHILOX_M[0] * c0
        p1 = _PHILOX_M[1] * c2
        c0, c1, c2, c3 = ((p1 >> 64) ^ c1 ^ k0) & _U64, p1 & _U64, ((p0 >> 64) ^ c3 ^ k1) & _U64, p0 & _U64
        k0 = (k0 + _PHILOX_W[0]) & _U64
        k1 = (k1 + _PHILOX_W[1]) & _U64
    return c0, c1, c2, c3


def uniform53(word):
    """A 64-bit word to a double in (0, 1): its top 53 bits plus one half."""
    return ((int(word) >> 11) + 0.5) * 2.0 ** -53


def triangle_frame(c, r, seed):
    """Unit vectors (u, v) of rotation r about centre c: u uniform on the
    sphere (cos alpha and phi from two words), v uniform on the circle
    orthogonal to u (angle psi from the third word), through the orthonormal
    basis of u built as in Duff et al. (JCGT 2017)."""
    w = philox4x64((c, r, 0, 0), (seed, 0))
    cz = 2.0 * uniform53(w[0]) - 1.0
    phi = 2.0 * np.pi * uniform53(w[1])
    psi = 2.0 * np.pi * uniform53(w[2])
    sz = np.sqrt(max(0.0, 1.0 - cz * cz))
    u = np.array([sz * np.cos(phi), sz * np.sin(phi), cz])
    s = 1.0 if u[2] >= 0.0 else -1.0
    a = -1.0 / (s + u[2])
    b = u[0] * u[1] * a
    e1 = np.array([1.0 + s * u[0] * u[0] * a, s * b, -s * u[0]])
    e2 = np.array([b, s + u[1] * u[1] * a, -u[1]])
    v = np.cos(psi) * e1 + np.sin(psi) * e2
    return u, v


def box_centre(c, seed, box_L):
    """Primary vertex c of the triplet-sphere scheme: uniform in the box."""
    w = philox4x64((c, 0, 1, 0), (seed, 0))
    return np.array([box_L * uniform53(w[0]), box_L * uniform53(w[1]), box_L * uniform53(w[2])])


def triplet_thetas(n_theta):
    """Opening angles at the centres of n_theta equal bins of [0, pi]."""
    return (np.arange(n_theta) + 0.5) * np.pi / n_theta


def triplet_mc(f2, f3, box_L, r12, r13, n_theta, n_rot, seed, centres=None, weights=None, n_box=0, f1=None,
               basis="b3"):
    """Monte-Carlo triple sums over random triangles (Sec. 3.4 Eq.
    particle-based-sum; Sec. 4.3.3).

    Primary vertices: the catalogue points ``centres`` (float32 [n, 3]) with
    ``weights`` (or 1) as the primary factor a (the naked primary vertex of
    the dual-sphere scheme), or, when ``centres`` is None, ``n_box`` uniform
    points of the box with a = f1(x) (or 1 without f1; triplet sphere).  For
    each centre, n_rot rotations (u, v); for each opening angle theta_j the
    vertices x2 = x + r12 u and x3 = x + r13 (cos theta_j u + sin theta_j v)
    read f2 and f3 (the basis expansion, interpolate).  Returns float64 [n_theta, 4]: the sums
    of a, a f2(x2), a f3(x3) and a f2(x2) f3(x3) over all (centre, rotation).
    """
    thetas = triplet_thetas(n_theta)
    if centres is not None:
        xc = np.asarray(centres, dtype=np.float32).astype(np.float64)
        a = np.ones(xc.shape[0]) if weights is None else np.asarray(weights, dtype=np.float32).astype(np.float64)
    else:
        xc = np.array([box_centre(c, seed, box_L) for c in range(n_box)]).reshape(-1, 3)
        a = np.ones(xc.shape[0]) if f1 is None else interpolate(f1, xc, box_L, basis)
    n_c = xc.shape[0]
    frames = [triangle_frame(c, r, seed) for c in range(n_c) for r in range(n_rot)]
    u = np.array([f[0] for f in frames]).reshape(n_c * n_rot, 3)
    v = np.array([f[1] for f in frames]).reshape(n_c * n_rot, 3)
    x = np.repeat(xc, n_rot, axis=0)
    aa = np.repeat(a, n_rot)
    v2 = interpolate(f2, x + r12 * u, box_L, basis)
    out = np.zeros((n_theta, 4))
    for j, th in enumerate(thetas):
        v3 = interpolate(f3, x + r13 * (np.cos(th) * u + np.sin(th) * v), box_L, basis)
        out[j] = [np.sum(aa), np.sum(aa * v2), np.sum(aa * v3), np.sum(aa * v2 * v3)]
    return out


# ----------------------------------------------------------------------------
# 3PCF monopole through triple connection coefficients (Sec. 3.3.2, Eqs.
# 3pcfddd, 2-fold-density, 3PCF-ddd-monopole, con-coeff, DDD-vector-product),
# Gamma_{a,b} is the overlap of three translated scaling functions: nonzero
# for offsets a, b in [-3, 3]^3 with B3, in [-2, 2]^3 with the D4 function.
# ----------------------------------------------------------------------------

def connection_1d():
    """gamma[a + 3, b + 3] = int B3(x) B3(x - a) B3(x - b) dx, a, b in [-3, 3]:
    the one-dimensional factor of Gamma_{a,b} (Eq. con-coeff is a product of
    three such factors).  The integrand is a polynomial of degree 9 on each
    unit interval of the support [-2, 2] of B3(x), so 5-point Gauss-Legendre
    per interval is exact."""
    xg, wg = np.polynomial.legendre.leggauss(5)
    g = np.zeros((7, 7))
    for lo in range(-2, 2):
        x = lo + 0.5 * (xg + 1.0)
        w = 0.5 * wg
        for a in range(-3, 4):
            for b in range(-3, 4):
                g[a + 3, b + 3] += np.sum(w * bspline3(x) * bspline3(x - a) * bspline3(x - b))
    return g


def connection_coefficients(basis="b3"):
    """(gamma, reach): the one-dimensional factor of Gamma_{a,b} for offsets
    a, b in [-reach, reach] (B3: connection_1d, reach 3; D4:
    db2_connection_1d, reach 2)."""
    if basis == "b3":
        return connection_1d(), 3
    if basis == "db2":
        return db2_connection_1d(), 2
    raise ValueError(basis)


def two_fold_coefficients(f1, f2, basis="b3"):
    """Coefficients of the two-fold field (Eq. 3PCF-ddd-monopole):
    e_l = sum_a f1[l + a] sum_b Gamma_{a,b} f2[l + b], offsets a, b over
    [-reach, reach]^3, node indices mod N, Gamma_{a,b} = prod_d gamma(a_d, b_d)."""
    f1 = np.asarray(f1, dtype=np.float64)
    f2 = np.asarray(f2, dtype=np.float64)
    g, c = connection_coefficients(basis)
    rng = range(-c, c + 1)
    offs = [(x, y, z) for x in rng for y in rng for z in rng]
    shift = lambda f, o: np.roll(f, shift=(-o[0], -o[1], -o[2]), axis=(0, 1, 2))   # f[l + o]
    s2 = {b: shift(f2, b) for b in offs}
    out = np.zeros_like(f1)
    for a in offs:
        inner = np.zeros_like(f1)
        for b in offs:
            inner += g[a[0] + c, b[0] + c] * g[a[1] + c, b[1] + c] * g[a[2] + c, b[2] + c] * s2[b]
        out += shift(f1, a) * inner
    return out


def ddd_gamma(eps, f1, f2, basis="b3"):
    """Triplet count of Eq. DDD-vector-product, per node: N^-3 sum_l eps_l
    e_l(f1, f2), the box mean of the product of the three basis expansions
    (with eps = delta and f_i shell-filtered contrasts, the 3PCF monopole of
    the smoothed fields; a node sum replaced by the exact integral)."""
    e = two_fold_coefficients(f1, f2, basis)
    return float(np.sum(np.asarray(eps, dtype=np.float64) * e)) / np.asarray(eps).size
