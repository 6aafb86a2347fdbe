"""CPU checks of the C-ABI library: it loads, exports every entry point that
include/mfs.h declares, its host-side geometry agrees with the oracle's,
and it reports errors without touching a GPU.  No GPU compute here."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import geometry

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mfs.h")


def declared_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mfs_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    import paper_1506_05083_amd as m
    if not os.path.exists(m.LIB_PATH):
        pytest.fail("libmfs.so is not built (python -m paper_1506_05083_amd.build)")
    return m


def test_exports_every_declared_symbol(lib):
    L = ctypes.CDLL(lib.LIB_PATH)
    syms = declared_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(L, s), s


def test_binding_covers_the_header(lib):
    assert set(lib._SIGS) == set(declared_symbols())


@pytest.mark.parametrize("make", [W.sphere_free_space, W.periodic_k10, W.small_periodic])
def test_host_geometry_matches_oracle(lib, make):
    b = make().body
    g = lib.polar_geometry(b.shape.a, b.shape.eps, b.shape.j, b.M, b.N, b.tau, b.colloc)
    o = geometry.build_geometry(b)
    for k in ("rho", "z", "nrho", "nz", "srho", "sz"):
        assert np.max(np.abs(g[k] - getattr(o, k))) < 1e-14, k


def test_invalid_geometry_rejected_on_host(lib):
    with pytest.raises(lib.MfsError) as e:
        lib.polar_geometry(-1.0, 0.0, 0, 10, 8, 0.1)
    assert e.value.status == lib.MFS_EINVAL
    assert "polar" in str(e.value)


def test_missing_library_fails_loudly(lib, monkeypatch, tmp_path):
    monkeypatch.setattr(lib, "_lib", None)
    monkeypatch.setattr(lib, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(RuntimeError):
        lib.lib()


@pytest.mark.parametrize("N,M,tau,colloc", [(450, 540, 0.05, "mid"), (60, 72, 0.05, "gauss"), (120, 144, 0.2, "mid")])
def test_host_cup_geometry_matches_oracle(lib, N, M, tau, colloc):
    """The library's cup (its own complex erf) against the oracle's (scipy's)."""
    sh = W.CupShape()
    b = W.Body(sh, N=N, M=M, P=8, q=16, k=1.0, tau=tau, colloc=colloc)
    g = lib.body_geometry(sh, M, N, tau, colloc)
    o = geometry.build_geometry(b)
    for k in ("rho", "z", "nrho", "nz", "srho", "sz"):
        assert np.max(np.abs(g[k] - getattr(o, k))) < 1e-14, k


@pytest.mark.parametrize("bad", [dict(outer=-1.0), dict(half=1.5), dict(b=4.0), dict(tau=0.5)])
def test_invalid_cup_rejected_on_host(lib, bad):
    kw = dict(outer=0.35, half=0.2, b=0.5, M=12, N=10, tau=0.05)
    kw.update(bad)
    with pytest.raises(lib.MfsError) as e:
        lib.cup_geometry(**kw)
    assert e.value.status == lib.MFS_EINVAL
    assert "cup" in str(e.value)
