"""Parity of hermes_xi_aniso (anisotropic 2PCF with axisymmetric windows)
with the FP64 oracle, through the C ABI.

Tolerances as elsewhere, normwise over the windows of one call: float32 path
<= 1e-5, float64 path <= 1e-10.
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
    scale = np.max(np.abs(ref))
    assert scale > 0
    return float(np.max(np.abs(got - ref)) / scale)


def _fields(hermes, n, L, seed, dtype, sigma_z=3.0):
    pos = synth.neyman_scott(150, 40, 2.0, L, seed, sigma_z=sigma_z)
    eps, sw = hermes.assign(torch.from_numpy(pos).cuda(), None, L, n, dtype=dtype)
    dk, _ = hermes.fft(eps, sw, want_delta=False)
    oe, osw = O.assign(pos, None, L, n)
    return dk, O.dft3(O.contrast(oe, osw))


def _mixed_windows(L, count, seed):
    """count windows of every kind with random sizes below L/4."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        kind = O.ANISO_KINDS[i % len(O.ANISO_KINDS)]
        rp, rl = rng.uniform(2.0, L / 4), rng.uniform(0.0, L / 4)
        dp, dl = rng.uniform(0.5, 4.0), rng.uniform(0.0, 6.0)
        if kind == "ring_bin":
            dp = min(dp, 2 * rp)
        out.append((kind, rp, rl, dp, dl))
    return out


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("n,los", [(16, 2), (32, 0), (64, 1), (64, 2)])
def test_xi_aniso_all_kinds(hermes, dtype, n, los):
    L = 120.0
    dk, odh = _fields(hermes, n, L, 7000 + n + los, dtype)
    wins = _mixed_windows(L, 21, n + los)
    got = hermes.xi_aniso(dk, L, wins, los_axis=los).cpu().numpy()
    ref = O.xi_aniso(odh, L, wins, los_axis=los)
    assert normwise(got, ref) < TOL[dtype]
    if dtype == torch.float64:   # every kind on its own scale
        for kind in O.ANISO_KINDS:
            idx = [i for i, w in enumerate(wins) if w[0] == kind]
            assert normwise(got[idx], ref[idx]) < 1e-9, kind


def test_xi_aniso_many_windows_in_caller_order(hermes):
    """Several 64-window tiles with a ragged tail, kinds interleaved: every
    result lands at its caller index; a permuted list gives the permuted
    results."""
    n, L = 64, 120.0
    dk, odh = _fields(hermes, n, L, 7100, torch.float32)
    wins = _mixed_windows(L, 203, 11)
    got = hermes.xi_aniso(dk, L, wins).cpu().numpy()
    ref = O.xi_aniso(odh, L, wins)
    assert normwise(got, ref) < 1e-5
    perm = np.random.default_rng(3).permutation(len(wins))
    got_p = hermes.xi_aniso(dk, L, [wins[i] for i in perm]).cpu().numpy()
    assert np.max(np.abs(got_p - got[perm])) <= 1e-12 * np.max(np.abs(got))


def test_xi_aniso_rings_on_the_smu_grid_and_thin_shell(hermes):
    """Thin rings at the 46 x 51 (s, mu) bin centres (64^3 slice of the grid):
    parity with the oracle; the mu-average of rings at fixed s approaches the
    isotropic thin shell sin(ks)/(ks)."""
    n, L = 64, 400.0
    dk, odh = _fields(hermes, n, L, 7200, torch.float64, sigma_z=4.0)
    edges = np.linspace(2.0, 186.0, 47)
    rings = synth.smu_rings(edges, 51)
    got = hermes.xi_aniso(dk, L, rings).cpu().numpy()
    pick = np.random.default_rng(5).choice(len(rings), 40, replace=False)
    ref = O.xi_aniso(odh, L, [rings[i] for i in pick])
    assert normwise(got[pick], ref) < 1e-10


def test_xi_aniso_errors(hermes):
    from paper_2607_23494_amd.hermes import HermesError
    dk = torch.zeros((16, 16, 9), dtype=torch.complex64, device="cuda")
    bad = [
        [("ring", -1.0, 2.0)],                      # negative
        [("ring", 60.0, 2.0)],                      # r_perp >= L/2
        [("disk", 2.0, 50.0)],                      # r_par >= L/2
        [("ring_bin", 1.0, 2.0, 3.0, 0.0)],         # r_perp < d_perp / 2
        [("ring_bin", 5.0, 2.0, 0.0, 1.0)],         # d_perp = 0
        [("gauss_shell", 0.0, 0.0, 0.0)],           # Rs = Rg = 0
        [("ring", float("nan"), 1.0)],              # not finite
    ]
    for w in bad:
        with pytest.raises(HermesError):
            hermes.xi_aniso(dk, 100.0, w)
    with pytest.raises(HermesError, match="windows"):
        hermes.xi_aniso(dk, 100.0, [])
