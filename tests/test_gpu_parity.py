"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances are normwise per statistic, e = max|x - x_ref| / max|x_ref| over
the bins of one statistic (each xi_l, each zeta_l matrix, each moment):
float32 path <= 1e-5, float64 path <= 1e-10; integer-free, so no bit-exact
cases apart from the empty catalogue.
"""
import functools

import numpy as np
import pytest
import torch

import oracle as O
from paper_2607_23494_amd import synth

pytestmark = pytest.mark.gpu

TOL = {torch.float32: 1e-5, torch.float64: 1e-10}


def normwise(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.max(np.abs(ref))
    assert scale > 0
    return float(np.max(np.abs(got - ref)) / scale)


def _cat(n_par, n_ch, sigma, L, seed, marks=False):
    pos = synth.neyman_scott(n_par, n_ch, sigma, L, seed)
    w = synth.lognormal_marks(pos.shape[0], seed) if marks else None
    return pos, w


def _gpu_field(hermes, pos, w, L, n, dtype):
    tp = torch.from_numpy(pos).cuda()
    tw = torch.from_numpy(w).cuda() if w is not None else None
    eps, sw = hermes.assign(tp, tw, L, n, dtype=dtype)
    dk, delta = hermes.fft(eps, sw)
    return eps, sw, dk, delta


def _oracle_field(pos, w, L, n):
    eps, sw = O.assign(pos, w, L, n)
    delta = O.contrast(eps, sw)
    return eps, sw, delta, O.dft3(delta)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("n", [8, 32, 64])
def test_assign(hermes, dtype, n):
    L = 100.0
    pos, w = _cat(60, 30, 1.5, L, 1000 + n, marks=True)
    eps, sw = hermes.assign(torch.from_numpy(pos).cuda(), torch.from_numpy(w).cuda(), L, n, dtype=dtype)
    oe, osw = O.assign(pos, w, L, n)
    assert normwise(eps.cpu().numpy(), oe) < TOL[dtype]
    assert abs(sw.item() - osw) < 1e-12 * osw


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_assign_bitwise_reproducible_and_order_free(hermes, dtype):
    """The taps are summed in 64-bit fixed point: repeated calls give the same
    grid bit for bit, and so does any permutation of the catalogue (sum_w is
    summed in a fixed order: equal across calls, equal to rounding under a
    permutation)."""
    for n, (pos, w, L) in [(64, (*_cat(200, 40, 2.0, 150.0, 1500, marks=True), 150.0)),
                           (512, (*synth.WORKLOADS["ns512_3pcf"].catalogue(), 1000.0))]:
        tp, tw = torch.from_numpy(pos).cuda(), torch.from_numpy(w).cuda()
        e1, s1 = hermes.assign(tp, tw, L, n, dtype=dtype)
        e2, s2 = hermes.assign(tp, tw, L, n, dtype=dtype)
        assert torch.equal(e1, e2) and torch.equal(s1, s2), n
        perm = torch.from_numpy(np.random.default_rng(n).permutation(pos.shape[0])).cuda()
        e3, s3 = hermes.assign(tp[perm].contiguous(), tw[perm].contiguous(), L, n, dtype=dtype)
        assert torch.equal(e1, e3), n
        assert abs(s3.item() - s1.item()) <= 1e-14 * s1.item()
        del e1, e2, e3
        torch.cuda.empty_cache()


def test_assign_heavy_point_batches(hermes):
    """Two points carrying 2 % of sum |w| each: their taps reach 2^54
    fixed-point units (the scale leaves 2^61 for sum |w|).  Compared with the
    oracle over the whole grid and over the cells the heavy points do not reach
    (normalised by their own largest value, so the heavy taps do not hide the
    light ones)."""
    L, n = 100.0, 64
    pos, _ = _cat(400, 50, 2.0, L, 1700)
    w = np.random.default_rng(17).uniform(0.5, 1.5, pos.shape[0]).astype(np.float32)
    heavy = [123, 9000]
    w[heavy] = np.float32(0.02 * w.sum())
    eps, _ = hermes.assign(torch.from_numpy(pos).cuda(), torch.from_numpy(w).cuda(), L, n, dtype=torch.float32)
    got = eps.cpu().numpy()
    oe, _ = O.assign(pos, w, L, n)
    assert normwise(got, oe) < TOL[torch.float32]
    far = np.ones((n, n, n), dtype=bool)
    for h in heavy:
        c = np.floor(pos[h].astype(np.float64) * n / L).astype(int)
        idx = [np.arange(c[a] - 2, c[a] + 3) % n for a in range(3)]
        far[np.ix_(*idx)] = False
    assert normwise(got[far], oe[far]) < TOL[torch.float32]


def test_assign_wraps_and_empty(hermes):
    L, n = 50.0, 16
    rng = np.random.default_rng(4)
    pos = rng.uniform(-3 * L, 4 * L, (500, 3)).astype(np.float32)   # far outside the box
    eps, _ = hermes.assign(torch.from_numpy(pos).cuda(), None, L, n, dtype=torch.float64)
    oe, _ = O.assign(pos, None, L, n)
    assert normwise(eps.cpu().numpy(), oe) < 1e-10
    empty = torch.zeros((0, 3), dtype=torch.float32, device="cuda")
    eps0, sw0 = hermes.assign(empty, None, L, n)
    assert sw0.item() == 0.0 and torch.count_nonzero(eps0).item() == 0


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("n", [8, 16, 64, 128])
def test_fft_on_oracle_field(hermes, dtype, n):
    """The forward transform alone, fed with the oracle's coefficients."""
    L = 200.0
    pos, w = _cat(80, 20, 3.0, L, 2000 + n)
    oe, osw, od, odh = _oracle_field(pos, w, L, n)
    eps = torch.from_numpy(oe).to(dtype).cuda()
    sw = torch.tensor([osw], dtype=torch.float64, device="cuda")
    dk, delta = hermes.fft(eps, sw)
    half = odh[:, :, : n // 2 + 1]
    assert normwise(delta.cpu().numpy(), od) < TOL[dtype]
    got = dk.cpu().numpy()
    assert normwise(got.real, half.real) < TOL[dtype] * 5
    assert normwise(got.imag, half.imag) < TOL[dtype] * 5
    assert got[0, 0, 0] == 0


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_xi_multipoles(hermes, dtype):
    L, n = 300.0, 64
    pos, _ = _cat(300, 30, 3.0, L, 3001)
    pos[:, 2] = np.mod(pos[:, 2] + np.random.default_rng(5).normal(0, 6.0, pos.shape[0]), L).astype(np.float32)
    _, _, dk, _ = _gpu_field(hermes, pos, None, L, n, dtype)
    _, _, _, odh = _oracle_field(pos, None, L, n)
    edges = np.linspace(8.0, 80.0, 11)
    ells = (0, 2, 4)
    got = hermes.xi(dk, L, edges, ells=ells, los_axis=2).cpu().numpy()
    ref = O.xi_multipoles(odh, L, edges, ells=ells, los_axis=2)
    for i in range(3):
        assert normwise(got[i], ref[i]) < TOL[dtype], ells[i]
    gx = hermes.xi(dk, L, edges, ells=(2,), los_axis=0).cpu().numpy()
    rx = O.xi_multipoles(odh, L, edges, ells=(2,), los_axis=0)
    assert normwise(gx[0], rx[0]) < TOL[dtype]
    # shot-noise factors, float64 on the device whatever the field precision;
    # the self-pair kernel shares the grid's cubic symmetry, so S_2b vanishes
    # up to rounding and every multipole is compared on the monopole's scale
    _, shot = hermes.xi(dk, L, edges, ells=ells, los_axis=2, shot=True)
    shot = shot.cpu().numpy()
    sref = O.shot_factor(n, L, edges, ells=ells, los_axis=2)
    scale = np.max(np.abs(sref[0]))
    for i in range(3):
        assert np.max(np.abs(shot[i] - sref[i])) < 1e-10 * scale, ells[i]
    assert np.max(np.abs(sref[1])) < 1e-12 * scale


def test_xi_fp64_workload_small(hermes):
    """The 64^3 FP64 workload: 2e4 clustered points, 20 bins over [5, 50]."""
    wl = synth.WORKLOADS["ns64_fp64"]
    pos, w = wl.catalogue()
    _, _, dk, _ = _gpu_field(hermes, pos, w, wl.box_L, wl.n_grid, torch.float64)
    _, _, _, odh = _oracle_field(pos, w, wl.box_L, wl.n_grid)
    edges = synth.EDGES["ns64_fp64"]
    got = hermes.xi(dk, wl.box_L, edges).cpu().numpy()
    ref = O.xi_multipoles(odh, wl.box_L, edges)
    assert normwise(got, ref) < 1e-10


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_filter_moments_and_fields(hermes, dtype):
    L, n = 128.0, 32
    pos, _ = _cat(100, 20, 2.0, L, 4001)
    _, _, dk, _ = _gpu_field(hermes, pos, None, L, n, dtype)
    _, _, _, odh = _oracle_field(pos, None, L, n)
    wins = [("sphere", 0.0, 6.0), ("gauss", 0.0, 4.0), ("shell", 5.0, 9.0), ("sphere", 0.0, 11.0)]
    fields, mom = hermes.filter_bins(dk, L, wins, store_fields=True)
    fields = fields.cpu().numpy()
    mom = mom.cpu().numpy()
    for i, (kind, lo, hi) in enumerate(wins):
        if kind == "sphere":
            fn = lambda kq, R=hi: O.w_sphere(kq * R)
        elif kind == "gauss":
            fn = lambda kq, R=hi: O.w_gauss(kq, R)
        else:
            fn = lambda kq, a=lo, b=hi: O.w_shell(kq, a, b)
        ref = O.filtered_field(odh, L, fn)
        assert normwise(fields[i], ref) < TOL[dtype], kind
        for p in range(3):
            want = np.mean(ref ** (p + 2))
            assert abs(mom[i, p] - want) < TOL[dtype] * np.mean(np.abs(ref) ** (p + 2)), (kind, p)


def test_filter_sh_window_field(hermes):
    L, n = 96.0, 32
    pos, _ = _cat(60, 25, 2.0, L, 4002)
    _, _, dk, _ = _gpu_field(hermes, pos, None, L, n, torch.float64)
    _, _, _, odh = _oracle_field(pos, None, L, n)
    wins = [("sh_shell", 6.0, 11.0, 3, -2), ("sh_shell", 6.0, 11.0, 1, 1), ("sh_shell", 4.0, 8.0, 0, 0)]
    fields, _ = hermes.filter_bins(dk, L, wins, store_fields=True, moments=False)
    fields = fields.cpu().numpy()
    for i, (_, lo, hi, ell, m) in enumerate(wins):
        ref, im = O.multipole_field(odh, L, ell, m, lo, hi)
        assert im < 1e-12 * np.max(np.abs(ref))
        assert normwise(fields[i], ref) < 1e-10, (ell, m)


ZETA_TOL = {"fp32": 1e-5, "bf16x3": 1e-3, "fp16x3": 1e-3}


@pytest.fixture(scope="module")
def small_zeta_case():
    L, n = 120.0, 32
    pos, _ = _cat(40, 40, 2.0, L, 5001)
    _, _, od, odh = _oracle_field(pos, None, L, n)
    edges = np.array([6.0, 10.0, 15.0, 21.0, 28.0])
    lmax = 4
    ref = O.zeta_multipoles(od, odh, L, edges, ells=tuple(range(lmax + 1)))
    return pos, L, n, edges, lmax, ref


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp16x3"])
def test_zeta_small(hermes, small_zeta_case, precision):
    pos, L, n, edges, lmax, ref = small_zeta_case
    _, _, dk, delta = _gpu_field(hermes, pos, None, L, n, torch.float32)
    got = hermes.zeta_l(delta, dk, L, edges, lmax, precision=precision).cpu().numpy()
    for ell in range(lmax + 1):
        assert normwise(got[ell], ref[ell]) < ZETA_TOL[precision], (precision, ell)
    if precision == "fp32":
        assert np.max(np.abs(got - got.transpose(0, 2, 1))) == 0


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_zeta_ragged_bins_and_tiny_grid(hermes, precision):
    """Odd bin counts (ragged 4x4 tiles and MFMA padding), l_max = 0 and the
    smallest grid."""
    for n, L, edges, lmax in [(8, 40.0, [3.0, 7.0, 11.0], 2), (32, 100.0, np.linspace(5, 40, 8), 0),
                              (16, 64.0, [4.0, 9.0], 3)]:
        pos, _ = _cat(20, 30, 2.0, L, 5100 + n)
        _, _, dk, delta = _gpu_field(hermes, pos, None, L, n, torch.float32)
        _, _, od, odh = _oracle_field(pos, None, L, n)
        got = hermes.zeta_l(delta, dk, L, edges, lmax, precision=precision).cpu().numpy()
        ref = O.zeta_multipoles(od, odh, L, np.asarray(edges), ells=tuple(range(lmax + 1)))
        for ell in range(lmax + 1):
            assert normwise(got[ell], ref[ell]) < ZETA_TOL[precision], (n, ell)


@pytest.fixture(scope="module")
def high_ell_case():
    """A clustered 32^3 field and every multipole l <= 10 over four bins: the
    real harmonics up to l = 10 on and off the Nyquist planes."""
    L, n = 110.0, 32
    pos, w = _cat(50, 30, 2.0, L, 5301, marks=True)
    _, _, od, odh = _oracle_field(pos, w, L, n)
    edges = np.array([5.0, 9.0, 14.0, 20.0, 27.0])
    lmax = 10
    ref = O.zeta_multipoles(od, odh, L, edges, ells=tuple(range(lmax + 1)))
    return pos, w, L, n, edges, lmax, ref


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp16x3"])
def test_zeta_high_ell_clustered(hermes, high_ell_case, precision):
    pos, w, L, n, edges, lmax, ref = high_ell_case
    _, _, dk, delta = _gpu_field(hermes, pos, w, L, n, torch.float32)
    got = hermes.zeta_l(delta, dk, L, edges, lmax, precision=precision).cpu().numpy()
    for ell in range(lmax + 1):
        assert normwise(got[ell], ref[ell]) < ZETA_TOL[precision], (precision, ell)


@functools.lru_cache(maxsize=None)
def _wide_case(n_bins):
    L, n = 160.0, 64
    pos, _ = _cat(50, 40, 2.5, L, 5200 + n_bins)
    _, _, od, odh = _oracle_field(pos, None, L, n)
    edges = np.linspace(4.0, 52.0, n_bins + 1)
    ref = O.zeta_multipoles(od, odh, L, edges, ells=(0, 1, 2))
    return pos, L, n, edges, ref


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("n_bins", [20, 21, 24, 32])
def test_zeta_wide_batches(hermes, precision, n_bins):
    """20 radial bins (every z-pass wavefront owns its full line count) and
    more: the batch-cap-32 kernels of the z pass, with partial (21, 24) and
    full (32) wavefront line counts, on a 64^3 grid (8 rows per group)."""
    pos, L, n, edges, ref = _wide_case(n_bins)
    _, _, dk, delta = _gpu_field(hermes, pos, None, L, n, torch.float32)
    lmax = 2
    got = hermes.zeta_l(delta, dk, L, edges, lmax, precision=precision).cpu().numpy()
    for ell in range(lmax + 1):
        assert normwise(got[ell], ref[ell]) < ZETA_TOL[precision], (n_bins, ell)


def test_errors_are_reported(hermes):
    from paper_2607_23494_amd.hermes import HermesError
    dk = torch.zeros((16, 16, 9), dtype=torch.complex64, device="cuda")
    with pytest.raises(HermesError, match="strictly increasing"):
        hermes.xi(dk, 10.0, [1.0, 3.0, 2.0])
    with pytest.raises(HermesError, match="even"):
        hermes.xi(dk, 10.0, [1.0, 2.0], ells=(1,))
    with pytest.raises(HermesError, match="power of two"):
        hermes.assign(torch.zeros((4, 3), device="cuda"), None, 10.0, 12)
    # separations of half the box or more reach the periodic image
    with pytest.raises(HermesError, match="below L/2"):
        hermes.xi(dk, 10.0, [1.0, 5.0])
    delta = torch.zeros((16, 16, 16), dtype=torch.float32, device="cuda")
    with pytest.raises(HermesError, match="below L/2"):
        hermes.zeta_l(delta, dk, 10.0, [1.0, 2.0, 6.0], 1)
    hermes.xi(dk, 10.0, [1.0, 4.99])


# --------------------------------------------------------------------------
# grids whose y pass spans several tiles per plane (128^3, 256^3): the column
# pairs of the c2r packing meet only inside one tile, and nothing a tile
# reads is written by another
# --------------------------------------------------------------------------

@functools.lru_cache(maxsize=None)
def _mid_case(n):
    L = {128: 400.0, 256: 800.0}[n]
    pos, _ = _cat(400, 40, 3.0, L, 5400 + n)
    _, _, od, odh = _oracle_field(pos, None, L, n)
    edges = np.linspace(10.0, 70.0, 5)
    lmax = 3 if n == 128 else 2
    ref = O.zeta_multipoles(od, odh, L, edges, ells=tuple(range(lmax + 1)))
    return pos, L, edges, lmax, ref, odh


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp16x3"])
@pytest.mark.parametrize("n", [128, 256])
def test_zeta_multi_tile_grids(hermes, n, precision):
    pos, L, edges, lmax, ref, _ = _mid_case(n)
    _, _, dk, delta = _gpu_field(hermes, pos, None, L, n, torch.float32)
    got = hermes.zeta_l(delta, dk, L, edges, lmax, precision=precision).cpu().numpy()
    for ell in range(lmax + 1):
        assert normwise(got[ell], ref[ell]) < ZETA_TOL[precision], (n, precision, ell)


@pytest.mark.parametrize("n", [128, 256])
def test_filter_fields_multi_tile_grids(hermes, n):
    pos, L, _, _, _, odh = _mid_case(n)
    _, _, dk, _ = _gpu_field(hermes, pos, None, L, n, torch.float32)
    wins = [("sphere", 0.0, 12.0), ("shell", 20.0, 28.0), ("sh_shell", 15.0, 25.0, 2, -1)]
    fields, mom = hermes.filter_bins(dk, L, wins, store_fields=True)
    fields = fields.cpu().numpy()
    refs = [O.filtered_field(odh, L, lambda kq: O.w_sphere(kq * 12.0)),
            O.filtered_field(odh, L, lambda kq: O.w_shell(kq, 20.0, 28.0)),
            O.multipole_field(odh, L, 2, -1, 15.0, 25.0)[0]]
    for i, ref in enumerate(refs):
        assert normwise(fields[i], ref) < 1e-5, (n, wins[i][0])


@pytest.mark.parametrize("n", [128, 256])
def test_zeta_is_deterministic_across_calls_and_streams(hermes, n):
    """The contraction has no atomics: the same inputs give bitwise the same
    result, also when four calls run at once on four streams."""
    pos, L, edges, lmax, _, _ = _mid_case(n)
    _, _, dk, delta = _gpu_field(hermes, pos, None, L, n, torch.float32)
    for precision in ("fp32", "bf16x3"):
        a = hermes.zeta_l(delta, dk, L, edges, lmax, precision=precision).cpu().numpy()
        b = hermes.zeta_l(delta, dk, L, edges, lmax, precision=precision).cpu().numpy()
        assert np.array_equal(a, b), precision
        streams = [torch.cuda.Stream() for _ in range(4)]
        torch.cuda.synchronize()
        outs = [hermes.zeta_l(delta, dk, L, edges, lmax, precision=precision, stream=s) for s in streams]
        torch.cuda.synchronize()
        for o in outs:
            assert np.array_equal(o.cpu().numpy(), a), precision
