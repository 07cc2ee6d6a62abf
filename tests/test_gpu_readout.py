"""Parity of hermes_readout (values at arbitrary positions, density marks,
moments over sampled positions) with the FP64 oracle, through the C ABI.

Tolerances as elsewhere: normwise, float32 path <= 1e-5, float64 <= 1e-10.
"""
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
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def _field(n, seed, dtype):
    """A seeded smooth-ish random field: white noise (host, the given dtype)."""
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((n, n, n)).astype(np.float32 if dtype == torch.float32 else np.float64)
    return f


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("n", [8, 32, 64])
def test_readout_values(hermes, dtype, n):
    L = 90.0
    f = _field(n, 100 + n, dtype)
    rng = np.random.default_rng(n)
    pos = rng.uniform(-2 * L, 3 * L, (5000, 3)).astype(np.float32)     # far outside the box too
    got, _ = hermes.readout(torch.from_numpy(f).cuda(), L, torch.from_numpy(pos).cuda())
    ref = O.readout(f, pos, L)
    assert normwise(got.cpu().numpy(), ref) < TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("mark", [("power_law", 0.3, 0.1, 0.05), ("power_law", -0.7, 0.2, 0.0),
                                  ("inverse_density", 1.0, 1.0, 0.02), ("inverse_density", -1.0, 0.5, 0.0)])
def test_readout_marks_with_weights(hermes, dtype, mark):
    L, n = 120.0, 32
    pos = synth.neyman_scott(50, 30, 2.0, L, 6001)
    w = synth.lognormal_marks(pos.shape[0], 6001)
    eps, sw = O.assign(pos, None, L, n)
    dh = O.dft3(O.contrast(eps, sw))
    dR = O.filtered_field(dh, L, lambda kq: O.w_sphere(kq * 8.0))
    field = dR.astype(np.float32) if dtype == torch.float32 else dR
    got, _ = hermes.readout(torch.from_numpy(field).cuda(), L, torch.from_numpy(pos).cuda(),
                            weight=torch.from_numpy(w).cuda(), mark=mark)
    kind, ex, off, st = mark
    ref = w.astype(np.float64) * O.density_mark(1.0 + O.readout(field, pos, L), kind, ex, off, st)
    assert normwise(got.cpu().numpy(), ref) < TOL[dtype], mark


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_readout_moments_and_empty(hermes, dtype):
    L, n = 64.0, 16
    f = _field(n, 7, dtype)
    pos = np.random.default_rng(8).uniform(0, L, (20000, 3)).astype(np.float32)
    vals, mom = hermes.readout(torch.from_numpy(f).cuda(), L, torch.from_numpy(pos).cuda(), moments=True)
    ref = O.readout_moments(f, pos, L)
    # the values are formed in float64 from the same field values on both sides
    assert np.max(np.abs(mom.cpu().numpy() - ref) / np.abs(ref)) < 1e-12
    empty = torch.zeros((0, 3), dtype=torch.float32, device="cuda")
    none, mom0 = hermes.readout(torch.from_numpy(f).cuda(), L, empty, want_values=False, moments=True)
    assert none is None and torch.count_nonzero(mom0).item() == 0


def test_mark_ratio_values_and_errors(hermes):
    """hermes_mark_ratio: (1 + a) / (1 + b) per bin, in place too; errors."""
    from paper_2607_23494_amd.hermes import HermesError
    a = torch.tensor([0.5, -0.25, 3.0, 0.0], dtype=torch.float64, device="cuda")
    b = torch.tensor([1.0, 0.5, -0.5, 0.0], dtype=torch.float64, device="cuda")
    got = hermes.mark_ratio(a, b).cpu().numpy()
    assert np.array_equal(got, np.array([0.75, 0.5, 8.0, 1.0]))
    hermes.mark_ratio(a, b, out=a)
    assert np.array_equal(a.cpu().numpy(), np.array([0.75, 0.5, 8.0, 1.0]))
    with pytest.raises(ValueError):
        hermes.mark_ratio(a, b.float())
    from paper_2607_23494_amd.hermes import _lib, _stream
    import ctypes
    assert _lib.hermes_mark_ratio(None, ctypes.c_void_p(b.data_ptr()), 4, ctypes.c_void_p(b.data_ptr()),
                                  _stream(0)) != 0


def test_readout_errors(hermes):
    from paper_2607_23494_amd.hermes import HermesError
    f = torch.zeros((16, 16, 16), dtype=torch.float32, device="cuda")
    p = torch.zeros((4, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(HermesError, match="offset > 0"):
        hermes.readout(f, 10.0, p, mark=("inverse_density", 1.0, 0.0))
    with pytest.raises(HermesError, match="offset > 0"):
        hermes.readout(f, 10.0, p, mark=("power_law", -0.5, 0.0))
    with pytest.raises(HermesError, match="both NULL"):
        hermes.readout(f, 10.0, p, want_values=False, moments=False)


def test_marked_2pcf_workflow(hermes):
    """The density-marked 2PCF end to end on the GPU (assign, FFT, sphere
    filter, readout at the points, marks, marked assignment, FFT, 2PCF)
    against the oracle's workflow."""
    L, n, R = 120.0, 64, 8.0
    pos = synth.neyman_scott(80, 30, 2.0, L, seed=6101)
    edges = np.linspace(3.0, 45.0, 15)
    tp = torch.from_numpy(pos).cuda()
    for kind, ex, off, st in [("power_law", 0.3, 0.1, 0.02), ("inverse_density", 1.0, 1.0, 0.02)]:
        eps, sw = hermes.assign(tp, None, L, n)
        dk, _ = hermes.fft(eps, sw, want_delta=False)
        xi = hermes.xi(dk, L, edges).cpu().numpy()[0]
        fields, _ = hermes.filter_bins(dk, L, [("sphere", 0.0, R)], store_fields=True, moments=False)
        marks, _ = hermes.readout(fields[0], L, tp, mark=(kind, ex, off, st))
        eps_m, sw_m = hermes.assign(tp, marks, L, n)
        dk_m, _ = hermes.fft(eps_m, sw_m, want_delta=False)
        xm_t = hermes.xi(dk_m, L, edges)
        xm = xm_t.cpu().numpy()[0]
        M = hermes.mark_ratio(xm_t, hermes.xi(dk, L, edges)).cpu().numpy()[0]
        rxm, rxi, rM = O.marked_xi(pos, None, L, n, edges, R, kind, ex, off, st)
        assert normwise(xi, rxi) < 1e-5
        assert normwise(xm, rxm) < 1e-5, kind
        assert normwise(M, rM) < 1e-5, kind


# --------------------------------------------------------------------------
# full size, in the benchmark's launch configuration
# --------------------------------------------------------------------------

def test_readout_ns512_catalogue_sampled(hermes):
    """A seeded 512^3 float32 field read at all 10^7 points of the 512^3
    workload's catalogue; 20 000 sampled points against the oracle, and the
    transpose identity sum_i w_i v_i = sum_l f_l eps_l over all points."""
    wl = synth.WORKLOADS["ns512_3pcf"]
    pos, w = wl.catalogue()
    n, L = wl.n_grid, wl.box_L
    f = _field(n, 512, torch.float32)
    tf, tp, tw = torch.from_numpy(f).cuda(), torch.from_numpy(pos).cuda(), torch.from_numpy(w).cuda()
    vals, _ = hermes.readout(tf, L, tp)
    vals = vals.cpu().numpy()
    idx = np.random.default_rng(9).choice(pos.shape[0], 20000, replace=False)
    ref = O.readout(f, pos[idx], L)
    assert normwise(vals[idx], ref) < 1e-5
    eps, _ = hermes.assign(tp, tw, L, n)
    rhs = float(np.sum(f.astype(np.float64) * eps.cpu().numpy()))
    lhs = float(np.sum(w.astype(np.float64) * vals))
    scale = float(np.sum(np.abs(w.astype(np.float64) * vals)))
    assert abs(lhs - rhs) < 1e-5 * scale


def test_readout_moments_1024_random_positions(hermes):
    """Counts in cells by sampling: moments of a seeded 1024^3 field over
    10^6 uniform random positions against the oracle."""
    n, L = 1024, 2000.0
    f = _field(n, 1024, torch.float32)
    pos = np.random.default_rng(10).uniform(0, L, (1_000_000, 3)).astype(np.float32)
    _, mom = hermes.readout(torch.from_numpy(f).cuda(), L, torch.from_numpy(pos).cuda(), want_values=False,
                            moments=True)
    torch.cuda.empty_cache()
    ref = O.readout_moments(f, pos, L)
    got = mom.cpu().numpy()
    # <v^3> of white noise is near zero: judged on the scale of <v^2>^(3/2)
    assert abs(got[0] - ref[0]) < 1e-12 * ref[0]
    assert abs(got[1] - ref[1]) < 1e-12 * ref[0] ** 1.5
    assert abs(got[2] - ref[2]) < 1e-12 * ref[2]


@pytest.mark.parametrize("basis", ["b3", "db2"])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_readout_bucketed_matches_direct_and_oracle(hermes, dtype, basis):
    """3e5 points (above the bucketing threshold) at 64^3: the tile-bucketed
    read agrees with the oracle, and bit for bit with the same call without a
    workspace (points read in the given order); the moments agree to
    rounding."""
    import ctypes
    from paper_2607_23494_amd.hermes import _lib, _Mark, context
    n, L = 64, 80.0
    f = _field(n, 700, dtype)
    rng = np.random.default_rng(7)
    pos = rng.uniform(-L, 2 * L, (300_000, 3)).astype(np.float32)
    tf, tp = torch.from_numpy(f).cuda(), torch.from_numpy(pos).cuda()
    with hermes.basis(basis):
        got, mom = hermes.readout(tf, L, tp, moments=True)
        ref = O.readout(f, pos, L, basis=basis)
        assert normwise(got.cpu().numpy(), ref) < TOL[dtype]
        direct = torch.empty_like(got)
        dmom = torch.empty(3, dtype=torch.float64, device="cuda")
        code = 0 if dtype == torch.float32 else 1
        st = _lib.hermes_readout(context(0), ctypes.c_void_p(tf.data_ptr()), n, code, L,
                                 ctypes.c_void_p(tp.data_ptr()), None, pos.shape[0], None,
                                 ctypes.c_void_p(direct.data_ptr()), ctypes.c_void_p(dmom.data_ptr()), None, 0,
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st == 0
        torch.cuda.synchronize()
        assert torch.equal(got, direct)
        assert torch.allclose(mom, dmom, rtol=1e-12, atol=0)


def test_readout_ns512_random_spheres_bench_configuration(hermes):
    """The random-sphere counts-in-cells launch of the benchmark: 10^8
    uniform random positions read from a 512^3 float32 field through the
    bucketed path; 20 000 sampled positions against the oracle, and the
    moments against those of the values read back."""
    n, L = 512, 1000.0
    f = _field(n, 513, torch.float32)
    tf = torch.from_numpy(f).cuda()
    g = torch.Generator(device="cuda").manual_seed(2607)
    rpos = (torch.rand((100_000_000, 3), device="cuda", generator=g) * L).contiguous()
    vals, mom = hermes.readout(tf, L, rpos, moments=True)
    idx = torch.from_numpy(np.random.default_rng(10).choice(100_000_000, 20000, replace=False)).cuda()
    sub = rpos[idx].cpu().numpy()
    ref = O.readout(f, sub, L)
    assert normwise(vals[idx].cpu().numpy(), ref) < 1e-5
    v = vals.double()
    want = torch.stack([(v ** 2).mean(), (v ** 3).mean(), (v ** 4).mean()]).cpu().numpy()
    scale = torch.stack([(v.abs() ** 2).mean(), (v.abs() ** 3).mean(), (v.abs() ** 4).mean()]).cpu().numpy()
    got = mom.cpu().numpy()
    assert np.max(np.abs(got - want) / scale) < 1e-6   # the kernel's values before their float32 rounding


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_readout_bucketed_marks_and_weights(hermes, dtype):
    """Density marks times weights through the bucketed path (2e5 points):
    each output lands at its own point's index."""
    L, n = 120.0, 32
    rng = np.random.default_rng(66)
    pos = rng.uniform(0, L, (200_000, 3)).astype(np.float32)
    w = rng.lognormal(0.0, 0.5, 200_000).astype(np.float32)
    f = (0.3 * _field(n, 77, dtype)).astype(np.float32 if dtype == torch.float32 else np.float64)
    mark = ("power_law", 0.7, 0.1, 0.02)
    got, _ = hermes.readout(torch.from_numpy(f).cuda(), L, torch.from_numpy(pos).cuda(),
                            weight=torch.from_numpy(w).cuda(), mark=mark)
    ref = w.astype(np.float64) * O.density_mark(1.0 + O.readout(f, pos, L), *mark)
    assert normwise(got.cpu().numpy(), ref) < TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_readout_fields_equals_single_reads(hermes, dtype):
    """Three fields at the same 2e5 points in one call (one bucketing): each
    row bit for bit the single-field read, moments to rounding; errors."""
    from paper_2607_23494_amd.hermes import HermesError
    n, L = 32, 50.0
    f = np.stack([_field(n, 900 + k, dtype) for k in range(3)])
    rng = np.random.default_rng(8)
    pos = torch.from_numpy(rng.uniform(-L, 2 * L, (200_000, 3)).astype(np.float32)).cuda()
    tf = torch.from_numpy(f).cuda()
    vals, mom = hermes.readout_fields(tf, L, pos, moments=True)
    for k in range(3):
        v1, m1 = hermes.readout(tf[k], L, pos, moments=True)
        assert torch.equal(vals[k], v1)
        assert torch.allclose(mom[k], m1, rtol=1e-12, atol=0)
    ref = O.readout(f[1], pos.cpu().numpy(), L)
    assert normwise(vals[1].cpu().numpy(), ref) < TOL[dtype]
    with pytest.raises(HermesError):
        hermes.readout_fields(torch.zeros((65, 8, 8, 8), device="cuda"), L, pos[:10].contiguous())


@pytest.mark.parametrize("basis", ["b3", "db2"])
def test_readout_fields_1024_tile_passes(hermes, basis):
    """1024^3: tiles of 16^3 cells, and the staged nodes of only two float32
    fields fit the LDS budget, so three fields take two passes; 3e6 points
    (above 8 per tile): every row equals the unbucketed single-field read
    (no workspace) bit for bit, and the moments agree to rounding."""
    import ctypes
    from paper_2607_23494_amd.hermes import _lib, context
    n, L = 1024, 500.0
    g = torch.Generator(device="cuda").manual_seed(1024)
    f = torch.randn((3, n, n, n), device="cuda", generator=g)
    pos = (torch.rand((3_000_000, 3), device="cuda", generator=g) * 1.5 * L - 0.25 * L).contiguous()
    with hermes.basis(basis):
        vals, mom = hermes.readout_fields(f, L, pos, moments=True)
        for k in range(3):
            direct = torch.empty(pos.shape[0], dtype=torch.float32, device="cuda")
            dmom = torch.empty(3, dtype=torch.float64, device="cuda")
            st = _lib.hermes_readout(context(0), ctypes.c_void_p(f[k].data_ptr()), n, 0, L,
                                     ctypes.c_void_p(pos.data_ptr()), None, pos.shape[0], None,
                                     ctypes.c_void_p(direct.data_ptr()), ctypes.c_void_p(dmom.data_ptr()), None, 0,
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
            assert st == 0
            torch.cuda.synchronize()
            assert torch.equal(vals[k], direct), k
            assert torch.allclose(mom[k], dmom, rtol=1e-12, atol=0), k
    del f
    torch.cuda.empty_cache()
