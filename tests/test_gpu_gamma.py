"""Parity of hermes_ddd_gamma (3PCF monopole through triple connection
coefficients) with the FP64 oracle's stencil contraction, through the C ABI.

Tolerances: float64 <= 1e-10, float32 <= 1e-5, normwise over the bin-pair
matrix.
"""
import itertools

import numpy as np
import pytest
import torch

import oracle as O
from paper_2607_23494_amd import synth

pytestmark = pytest.mark.gpu


def normwise(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.max(np.abs(ref))
    assert scale > 0
    return float(np.max(np.abs(got - ref)) / scale)


def _oracle_matrix(e, fields):
    nb = len(fields)
    ref = np.zeros((nb, nb))
    for b1, b2 in itertools.combinations_with_replacement(range(nb), 2):
        ref[b1, b2] = ref[b2, b1] = O.ddd_gamma(e, fields[b1], fields[b2])
    return ref


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n", [8, 16])
def test_ddd_gamma_random_fields(hermes, dtype, n):
    rng = np.random.default_rng(900 + n)
    npdt = np.float64 if dtype == torch.float64 else np.float32
    e = rng.standard_normal((n, n, n)).astype(npdt)
    f = rng.standard_normal((3, n, n, n)).astype(npdt)
    got = hermes.ddd_gamma(torch.from_numpy(e).cuda(), torch.from_numpy(f).cuda()).cpu().numpy()
    ref = _oracle_matrix(e, list(f))
    assert normwise(got, ref) < (1e-10 if dtype == torch.float64 else 1e-5)
    assert np.array_equal(got, got.T)


def test_ddd_gamma_end_to_end_shells(hermes):
    """Contrast of a clustered catalogue and two thick-shell filtered fields
    at 32^3: each side builds its own fields (assign, FFT, filter)."""
    n, L = 32, 100.0
    pos = synth.neyman_scott(80, 40, 2.0, L, 9100)
    edges = [(6.0, 12.0), (12.0, 20.0)]
    tp = torch.from_numpy(pos).cuda()
    eps, sw = hermes.assign(tp, None, L, n)
    dk, delta = hermes.fft(eps, sw)
    fields, _ = hermes.filter_bins(dk, L, [("shell", lo, hi) for lo, hi in edges], store_fields=True,
                                   moments=False)
    got = hermes.ddd_gamma(delta, fields).cpu().numpy()
    oe, osw = O.assign(pos, None, L, n)
    od = O.contrast(oe, osw)
    odh = O.dft3(od)
    of = [O.filtered_field(odh, L, lambda kq, lo=lo, hi=hi: O.w_shell(kq, lo, hi)) for lo, hi in edges]
    ref = _oracle_matrix(od, of)
    assert normwise(got, ref) < 1e-5


def test_ddd_gamma_full_size_properties(hermes):
    """20 fields at 512^3 (the 3PCF bin count): constant fields give the
    product of the constants; a periodic shift of every field by (1, 2, 3)
    cells leaves the matrix unchanged; the result is the same on a second
    call."""
    n, nb = 512, 20
    g = torch.Generator(device="cuda").manual_seed(5)
    e = torch.randn((n, n, n), device="cuda", generator=g)
    f = torch.randn((nb, n, n, n), device="cuda", generator=g)
    a = hermes.ddd_gamma(e, f)
    b = hermes.ddd_gamma(e, f)
    assert torch.equal(a, b)
    es = torch.roll(e, shifts=(1, 2, 3), dims=(0, 1, 2)).contiguous()
    fs = torch.roll(f, shifts=(1, 2, 3), dims=(1, 2, 3)).contiguous()
    c = hermes.ddd_gamma(es, fs)
    assert normwise(c.cpu().numpy(), a.cpu().numpy()) < 1e-5
    del es, fs, f
    torch.cuda.empty_cache()
    k = torch.full((n, n, n), 2.0, device="cuda")
    fc = torch.stack([torch.full((n, n, n), float(i + 1), device="cuda") for i in range(3)])
    got = hermes.ddd_gamma(k, fc).cpu().numpy()
    want = 2.0 * np.outer(np.arange(1, 4), np.arange(1, 4))
    assert np.max(np.abs(got - want) / want) < 1e-5


def test_ddd_gamma_errors(hermes):
    from paper_2607_23494_amd.hermes import HermesError
    e = torch.zeros((8, 8, 8), device="cuda")
    with pytest.raises(HermesError):
        hermes.ddd_gamma(e, torch.zeros((33, 8, 8, 8), device="cuda"))
    with pytest.raises(ValueError):
        hermes.ddd_gamma(e, torch.zeros((2, 8, 8, 4), device="cuda"))


@pytest.mark.parametrize("basis", ["b3", "db2"])
def test_ddd_gamma_fewer_fields_than_wavefronts(hermes, basis):
    """One, two and three fields (fewer than the workgroup's wavefronts) at
    256^3: constant fields give the product of the constants; a random
    8^3 case with one field against the oracle."""
    n = 256
    with hermes.basis(basis):
        k = torch.full((n, n, n), 2.0, device="cuda")
        for nf in (1, 2, 3):
            fc = torch.stack([torch.full((n, n, n), float(i + 1), device="cuda") for i in range(nf)])
            got = hermes.ddd_gamma(k, fc).cpu().numpy()
            want = 2.0 * np.outer(np.arange(1, nf + 1), np.arange(1, nf + 1))
            assert np.max(np.abs(got - want) / want) < 1e-5, nf
        rng = np.random.default_rng(31)
        e = rng.standard_normal((8, 8, 8))
        f = rng.standard_normal((1, 8, 8, 8))
        got = hermes.ddd_gamma(torch.from_numpy(e).cuda(), torch.from_numpy(f).cuda()).cpu().numpy()
        ref = O.ddd_gamma(e, f[0], f[0], basis=basis)
        assert abs(got[0, 0] - ref) < 1e-10 * max(1.0, abs(ref))


@pytest.mark.parametrize("basis", ["b3", "db2"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_ddd_gamma_thirty_two_fields(hermes, basis, dtype):
    """The largest call, 32 fields (float64 D4 then evaluates with fewer
    wavefronts to fit its LDS): the leading 20 x 20 block equals the 20-field
    call, the matrix is symmetric, and three pairs match the oracle."""
    n = 8
    rng = np.random.default_rng(320)
    npdt = np.float64 if dtype == torch.float64 else np.float32
    e = rng.standard_normal((n, n, n)).astype(npdt)
    f = rng.standard_normal((32, n, n, n)).astype(npdt)
    te, tf = torch.from_numpy(e).cuda(), torch.from_numpy(f).cuda()
    tol = 1e-10 if dtype == torch.float64 else 1e-5
    with hermes.basis(basis):
        full = hermes.ddd_gamma(te, tf).cpu().numpy()
        part = hermes.ddd_gamma(te, tf[:20].contiguous()).cpu().numpy()
    assert np.array_equal(full, full.T)
    assert normwise(full[:20, :20], part) < tol
    for b1, b2 in ((0, 31), (17, 25), (31, 31)):
        ref = O.ddd_gamma(e, f[b1], f[b2], basis=basis)
        assert abs(full[b1, b2] - ref) < tol * max(1.0, np.max(np.abs(full))), (b1, b2)
