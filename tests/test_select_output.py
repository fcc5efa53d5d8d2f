"""The library's choice of returned eigenpairs (klst_host_select_output, the
step klst_solve ends with), on constructed locked sets: conjugate partners are
recognised from the eigenvectors, not from eigenvalue distance, so two distinct
members of a tight cluster that happen to be near-conjugates are both
completed, while true partners locked separately are not duplicated.  CPU only."""
import numpy as np
import pytest

klst = pytest.importorskip("paper_2607_27440_amd.klst")

PERM = np.array([1, 0, 3, 2, 5, 4, 6, 7])       # a reflection of the entries


def _rc(x):
    """R conj(x) for the reflection PERM."""
    return np.conj(x[PERM])


def _gram(X):
    k = X.shape[1]
    G = np.array([[np.vdot(_rc(X[:, i]), X[:, j]) for j in range(k)] for i in range(k)])
    return G, np.sum(np.abs(X) ** 2, axis=0)


def _rand(seed, n=8):
    r = np.random.default_rng(seed)
    return r.standard_normal(n) + 1j * r.standard_normal(n)


def test_no_reflection_returns_the_locked_pairs_nearest_first():
    lam = np.array([2.0 + 1j, 0.5 - 0.5j, 0.5 + 0.5j, 1.0])
    out, src, mir = klst.host_select_output(lam, 0.0, 3)
    assert list(src) == [2, 1, 3] and not mir.any()
    assert np.array_equal(out, lam[[2, 1, 3]])


def test_near_conjugate_cluster_members_are_both_completed():
    """lambda_a and conj(lambda_b) 1e-8 apart, but distinct eigenpairs (their
    eigenvectors are not reflections of each other): both partners are added."""
    la = 0.9027 + 0.2174j
    lb = la * (1 + 1e-8)
    xa = _rand(1)
    xb = _rc(_rand(2))                 # eigenvector of conj(lb): unrelated to R conj(xa)
    lam = np.array([la, np.conj(lb)])
    G, n2 = _gram(np.stack([xa, xb], axis=1))
    out, src, mir = klst.host_select_output(lam, 0.0, 4, G, n2)
    assert len(out) == 4 and mir.sum() == 2
    for v in lam:
        assert np.min(np.abs(out - np.conj(v))) == 0.0
    # the eigenvalue-distance rule alone would have paired them
    assert abs(lam[1] - np.conj(lam[0])) < 1e-6 * abs(lam[0])


def test_true_partners_locked_separately_are_not_duplicated():
    la = 0.5028 + 0.1691j
    xa = _rand(3)
    xb = np.exp(0.7j) * _rc(xa) + 1e-7 * _rand(4)     # the partner, to the solver's accuracy
    lam = np.array([la, np.conj(la) * (1 + 3e-9)])
    G, n2 = _gram(np.stack([xa, xb], axis=1))
    out, src, mir = klst.host_select_output(lam, 0.0, 4, G, n2)
    assert len(out) == 2 and not mir.any()


def test_real_eigenvalue_is_its_own_partner_and_near_axis_complex_is_not():
    xr = _rand(5)
    xr = xr + _rc(xr)                                  # R conj(x) = x: a real eigenvalue's vector
    lr = 0.7 + 0.0j
    xc = _rand(6)                                      # complex eigenvalue near the real axis
    lc = 0.9 + 1e-8j
    lam = np.array([lr, lc])
    G, n2 = _gram(np.stack([xr, xc], axis=1))
    out, src, mir = klst.host_select_output(lam, 0.0, 5, G, n2)
    assert len(out) == 3
    assert list(mir) == [False, False, True] and src[2] == 1
    assert out[2] == np.conj(lc)


def test_ties_put_positive_imaginary_part_first():
    lam = np.array([1 - 1j, 1 + 1j])
    xa = _rand(7)
    X = np.stack([xa, np.exp(0.3j) * _rc(xa)], axis=1)
    G, n2 = _gram(X)
    out, src, mir = klst.host_select_output(lam, 0.0, 2, G, n2)
    assert out[0].imag > 0 and list(src) == [1, 0]
