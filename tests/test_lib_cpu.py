"""Host-side checks that need no GPU: the library loads and exports every
entry point the public header declares; the package import is GPU-free."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hermes.h")
LIB = os.path.join(ROOT, "paper_2607_23494_amd", "libhermes.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hermes_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_five_operations():
    names = declared_functions()
    for op in ("hermes_assign", "hermes_fft", "hermes_filter_bins", "hermes_xi", "hermes_zeta_l"):
        assert op in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        from paper_2607_23494_amd.build import build
        build()
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_package_import_is_gpu_free():
    import paper_2607_23494_amd
    from paper_2607_23494_amd import synth
    pos = synth.neyman_scott(3, 4, 1.0, 10.0, seed=1)
    assert pos.dtype.name == "float32" and pos.shape == (12, 3)
    assert (pos >= 0).all() and (pos < 10.0).all()
    assert paper_2607_23494_amd.__doc__
