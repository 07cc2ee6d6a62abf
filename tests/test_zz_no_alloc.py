"""The allocation-free 2PCF entry point (hermes_xi_static) against hermes_xi:
two calls in a row, the second on a smaller grid with fewer bins, then a
request larger than the static scratch, which is refused before any launch."""
import numpy as np
import pytest
import torch

from paper_2607_23494_amd import synth

pytestmark = pytest.mark.gpu


def _spectrum(hermes, n, L, seed, dtype):
    pos = synth.neyman_scott(60, 30, 2.0, L, seed)
    eps, sw = hermes.assign(torch.from_numpy(pos).cuda(), None, L, n, dtype=dtype)
    dk, _ = hermes.fft(eps, sw, want_delta=False)
    return dk


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_xi_static_matches_xi(hermes, dtype):
    cases = [(64, 200.0, np.linspace(4.0, 60.0, 29), (0, 2, 4)),     # the larger call first
             (32, 120.0, np.linspace(5.0, 40.0, 8), (0,))]
    for n, L, edges, ells in cases:
        dk = _spectrum(hermes, n, L, 9000 + n, dtype)
        ref, sref = hermes.xi(dk, L, edges, ells=ells, shot=True)
        got, sgot = hermes.xi_static(dk, L, edges, ells=ells, shot=True)
        ref, sref, got, sgot = (t.cpu().numpy() for t in (ref, sref, got, sgot))
        for i in range(len(ells)):
            # same kernels; only the order of the float64 histogram atomics differs
            assert np.max(np.abs(got[i] - ref[i])) <= 1e-12 * np.max(np.abs(ref[i])), (n, ells[i])
            assert np.max(np.abs(sgot[i] - sref[i])) <= 1e-12 * np.max(np.abs(sref[0])), (n, ells[i])


def test_xi_static_refuses_more_than_its_scratch(hermes):
    from paper_2607_23494_amd.hermes import HermesError
    dk = torch.zeros((16, 16, 9), dtype=torch.complex64, device="cuda")
    # a 1024^3 request with two multipoles needs about 25 MB of scratch (a
    # full-size spectrum is passed all the same)
    big = torch.zeros((1024, 1024, 513), dtype=torch.complex64, device="cuda")
    from paper_2607_23494_amd import hermes as H
    e = np.array([2.0, 10.0])
    el = np.array([0, 2], dtype=np.int32)
    out = torch.empty((2, 1), dtype=torch.float64, device="cuda")
    import ctypes
    st = H._lib.hermes_xi_static(H.context(0), H._ptr(big), 1024, 0, 2000.0, e.ctypes.data_as(ctypes.c_void_p), 1,
                                 el.ctypes.data_as(ctypes.c_void_p), 2, 2, H._ptr(out), None,
                                 H._stream(0, None))
    assert st == 4 and "static array" in H._lib.hermes_last_error().decode()
    del big
    torch.cuda.empty_cache()
    hermes.xi_static(dk, 10.0, [1.0, 2.0])   # still usable afterwards
