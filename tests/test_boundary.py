"""CPU tests of the C ABI boundary: the library loads, exports every entry point
the header declares, its host-side assembly matches the oracle's tables, its
small dense solver is correct, and bad inputs return error codes.  No device
compute is called."""
import os
import re

import numpy as np
import pytest

from paper_2607_27440_amd import workloads as W
from oracle import operator as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def klst():
    from paper_2607_27440_amd import klst as k
    return k


def _declared():
    src = open(os.path.join(ROOT, "include", "klst.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(klst_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol(klst):
    names = _declared()
    assert len(names) >= 15
    for nm in names:
        assert hasattr(klst._lib, nm), nm
    assert set(names) == set(klst.EXPORTS)


@pytest.mark.parametrize("mk", [W.config1, W.config2,
                                lambda: W.make_workload("dv1", mach=2.2, Ny=9, Qx=12, Qy=1, beta=0.4,
                                                        sigma=0, nev=2, base="bimodal", delta=2.0, Dv=1),
                                lambda: W.make_workload("ny56", mach=2.0, Ny=56, Qx=7, Qy=5, beta=0.5,
                                                        sigma=0, nev=4, base="bimodal", delta=2.5, Dv=2),
                                lambda: W.make_workload("ny72", mach=2.0, Ny=72, Qx=7, Qy=5, beta=0.5,
                                                        sigma=0, nev=4, base="bimodal", delta=2.5, Dv=2)])
def test_host_tables_match_oracle(klst, mk):
    wl = mk()
    P = O.Pencil(wl)
    t = klst.host_tables(wl)
    rel = lambda a, b: np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)
    assert rel(t["Dx"], P.Dx) <= 1e-14
    assert rel(t["nu"], P.state["nu"]) <= 1e-14
    assert rel(t["U"], P.U) <= 1e-13
    assert rel(t["M"], P.M) <= 1e-13
    # node by node, relative to the node's largest entry
    for j in range(P.Ny):
        assert rel(t["U"][j], P.U[j]) <= 1e-13, j
        assert rel(t["M"][j], P.M[j]) <= 1e-13, j
    assert (t["bc"] == P.bc).all()


@pytest.mark.parametrize("m", [1, 2, 7, 33, 64])
def test_host_sorted_schur(klst, m):
    rng = np.random.default_rng(m)
    G = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    U, T = klst.host_sorted_schur(G)
    assert np.abs(G @ U - U @ T).max() <= 1e-12 * max(1, np.abs(G).max()) * m
    assert np.abs(U.conj().T @ U - np.eye(m)).max() <= 1e-13 * m
    assert np.abs(np.tril(T, -1)).max() == 0.0
    d = np.abs(np.diag(T))
    assert np.all(np.diff(d) <= 1e-12 * d.max())
    assert np.allclose(np.sort_complex(np.diag(T)), np.sort_complex(np.linalg.eigvals(G)), atol=1e-10 * m)


def test_bad_inputs_are_rejected(klst):
    wl = W.config1()
    bad = []
    w1 = W.config1(); w1.Ny = 2; w1.rho = w1.rho[:2]; w1.u = w1.u[:2]; w1.T = w1.T[:2]; bad.append(w1)
    w2 = W.config1(); w2.w = w2.w.copy(); w2.w[3] = -1.0; bad.append(w2)
    w3 = W.config1(); w3.T = w3.T.copy(); w3.T[5] = np.nan; bad.append(w3)
    w4 = W.config1(); w4.rho = w4.rho.copy(); w4.rho[0] = -1.0; bad.append(w4)
    w5 = W.config1(); w5.Dv = 1; bad.append(w5)                  # Dv = 1 needs xi_y == 0
    for b in bad:
        with pytest.raises(klst.KlstError) as ei:
            klst.host_tables(b)
        assert ei.value.status == klst.EINVAL
    klst.host_tables(wl)


def test_create_without_device_fails_cleanly(klst):
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a device is visible")
    except ImportError:
        pass
    with pytest.raises(klst.KlstError) as ei:
        klst.Context()
    assert ei.value.status == klst.EDEVICE


@pytest.mark.parametrize("kw", [dict(m_max=249), dict(m_min=0), dict(m_min=10, m_max=11), dict(gmres_m=0),
                                dict(gmres_m=257), dict(tol=0.0), dict(inner_rtol=-1.0), dict(precision=2),
                                dict(op_mode=2), dict(pc_kernel=3), dict(precision=1, pc_kernel=0),
                                dict(inner_max_it=-1), dict(reorth=2), dict(method=2), dict(krylov32=2), dict(lines_per_block=0),
                                dict(lines_per_block=17), dict(max_it=0)])
def test_invalid_options_are_rejected_before_any_device_use(klst, kw):
    """Option validation precedes device selection: every out-of-range option
    returns EINVAL (documented ranges in include/klst.h), with or without a GPU."""
    with pytest.raises(klst.KlstError) as ei:
        klst.Context(**kw)
    assert ei.value.status == klst.EINVAL, kw


def test_footprint_model(klst):
    """The admission model grows with the problem and the search space, accounts
    for the shift-invert basis and the mixed-precision mirrors, and is 0 for
    invalid sizes."""
    f = lambda *a, **kw: klst.footprint_bytes(*a, klst.default_options(**kw))
    base = f(64, 96, 8)
    assert base > 0
    assert f(96, 96, 8) > base and f(64, 128, 8) > base and f(64, 96, 16) > base
    assert f(64, 96, 8, m_max=60) > f(64, 96, 8, m_max=30)
    assert f(64, 96, 8, precision=1) > base
    assert f(64, 96, 8, method=1, m_max=60) > f(64, 96, 8, method=1, m_max=30) > 0
    assert f(0, 96, 8) == 0 and f(64, 0, 8) == 0 and f(64, 96, 0) == 0
    # the vectors alone: at least the JD search and test spaces at n = 2 Ny Nxi
    n = 2 * 64 * 96
    assert base >= 16 * n * 2 * 31
