"""C-ABI checks that need no GPU: every function declared in include/*.h is
exported by the built library, lattice tables, and parameter validation (which
runs before any device call)."""
import ctypes as C
import glob
import os
import re

import numpy as np
import pytest

import paper_2003_11069_amd as P
from paper_2003_11069_amd import lb as lbmod

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    txt = open(header).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b((?:lb|ws)_[a-z0-9_]+)\s*\(", txt)))


LIBS = {"lbnci.h": os.path.join(ROOT, "paper_2003_11069_amd", "liblbnci.so"),
        "wsnet.h": os.path.join(ROOT, "paper_2003_11069_amd", "liblbnci.so")}


@pytest.mark.parametrize("header", sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))))
def test_header_symbols_exported(header):
    lib_path = LIBS.get(os.path.basename(header))
    if lib_path is None:
        lib_path = os.path.join(ROOT, "paper_2003_11069_amd", "lib" + os.path.basename(header)[:-2] + ".so")
    assert os.path.exists(lib_path), f"library for {header} not built"
    lib = C.CDLL(lib_path)
    names = _declared(header)
    assert names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.parametrize("lat,Q", [(P.LB_D2Q9, 9), (P.LB_D3Q27, 27)])
def test_lattice_tables(lat, Q):
    c, w = P.lattice_tables(lat)
    assert len(w) == Q
    d = 2 if lat == P.LB_D2Q9 else 3
    cc = c[:, :d].astype(float)
    assert abs(w.sum() - 1) < 1e-15
    assert np.abs(w @ cc).max() < 1e-16
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", w, cc, cc), np.eye(d) / 3, atol=1e-16)
    # opposite of direction k is Q-1-k in the library's order
    assert (c[::-1] == -c).all()


BAD = [dict(tau=0.5), dict(tau=0.3), dict(beta=1.5), dict(beta=-0.1), dict(nx=0), dict(nz=2),
       dict(h_min=5.0, h_max=4.0), dict(h_max=4.5), dict(h_min=0.0), dict(A_nci=-1.0),
       dict(storage=7), dict(lattice=5), dict(walls_y=1, ny=2), dict(A_s=-0.1), dict(tau2=0.4),
       dict(tau2=-1.0), dict(nci_mode=2), dict(nci_mode=-1),
       dict(rho_ratio=2.0, alpha1=0.3), dict(rho_ratio=-1.0), dict(rho_ratio=2.0, alpha1=1.0),
       dict(rho_ratio=3.0, alpha1=0.5), dict(mass_tol=-1.0), dict(mass_tol=float("nan")),
       dict(mass_tol=float("inf"))]


@pytest.mark.parametrize("bad", BAD)
def test_create_rejects_invalid(bad):
    with pytest.raises(P.LBError) as ei:
        P.Lattice(P.Params(**bad))
    assert ei.value.code == -1


def test_batch_rejects_continuous_nci():
    """Batches run the integer probe only; the check precedes any device call."""
    ps = [P.Params(nx=64, ny=32), P.Params(nx=64, ny=32, nci_mode=1)]
    with pytest.raises(P.LBError) as ei:
        P.Batch(ps)
    assert ei.value.code == -1 and "nci_mode" in str(ei.value)


def test_stream_calls_reject_null():
    """The argument checks of lb_stream_create / lb_stream_destroy precede
    any runtime call."""
    lib = P.load_library()
    assert lib.lb_stream_create(None) == -1
    assert lib.lb_stream_destroy(None) == -1
    assert lbmod.current_stream_handle() == 0


def test_last_error_message():
    with pytest.raises(P.LBError):
        P.Lattice(P.Params(tau=0.4))
    lib = P.load_library()
    assert b"tau" in lib.lb_last_error()


def test_missing_library_fails_loudly(tmp_path):
    saved = lbmod._lib
    lbmod._lib = None
    try:
        with pytest.raises(RuntimeError):
            lbmod.load_library(str(tmp_path / "nope.so"))
    finally:
        lbmod._lib = saved


WS_BAD = [dict(levels=1), dict(levels=7), dict(base=12), dict(base=0), dict(cin=0), dict(cin=9),
          dict(cout=9), dict(max_batch=0), dict(H=100), dict(H=8, W=8), dict(conv_algo=2), dict(conv_algo=-1)]


@pytest.mark.parametrize("bad", WS_BAD)
def test_ws_create_rejects_invalid(bad):
    """Configuration checks of the warm-start network run before any device call."""
    from paper_2003_11069_amd import ws
    cfg = ws.UNetConfig(**{**dict(levels=4, base=32, cin=3, cout=3, H=128, W=256, max_batch=2), **bad})
    with pytest.raises(ws.WSError) as ei:
        ws.UNet(cfg, stream=0)
    assert ei.value.code == -1
