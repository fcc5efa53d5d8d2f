"""Pins of the oracle pieces the parity tests rest on, each against something
other than itself:

  * Pencil.apply_structured (the reference at sizes where A is not assembled)
    against the explicitly assembled pencil, at configs 1 and 2 and the edge
    shapes, real and complex shifts;
  * condition numbers: QZ left vectors and the adjoint structured inverse give
    the same kappa, and kappa is the first-order sensitivity of the eigenvalue
    (a perturbation along y x^H moves it by kappa eps, any unit perturbation by
    at most that);
  * residuals(): the definition on a diagonal pencil with known eigenpairs, and
    its structured branch against its explicit branch;
  * order_nearest(): brute-force ordering of constructed values;
  * parity.match(): constructed duplicates, skipped nearer eigenvalues,
    conjugate ties and the conditioning-widened bound;
  * LineBlockILU0Rows (the row-built block-Jacobi ILU(0)) against LineBlockILU0
    (the same preconditioner from the assembled matrix).
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from paper_2607_27440_amd import workloads as W
from oracle import eig as E
from oracle import jd as J
from oracle import operator as O
from oracle import parity as PAR

U = 2.0 ** -53

EDGE = {
    "dv1": lambda: W.make_workload("dv1", mach=2.2, Ny=12, Qx=16, Qy=1, beta=0.4, sigma=0.0, nev=4,
                                   base="bimodal", delta=2.0, Dv=1),
    "collisionless": lambda: W.make_workload("free", mach=1.5, Ny=10, Qx=4, Qy=3, beta=0.8, sigma=0.0,
                                             nev=4, base="bimodal", delta=2.0, vmax=5.0, nu_inf=0.0),
    "ragged": lambda: W.make_workload("ragged", mach=2.5, Ny=17, Qx=5, Qy=3, beta=0.6, sigma=0.02j, nev=4,
                                      base="bimodal", delta=3.0),
    "tiny": lambda: W.make_workload("tiny", mach=1.3, Ny=3, Qx=2, Qy=2, beta=0.5, sigma=0.0, nev=2,
                                    base="maxwellian", delta=2.0),
    "c1": W.config1,
    "c2": W.config2,
}


# ------------------------------------------------------- structured apply --
@pytest.mark.parametrize("tau", [0.0, 0.37, 0.3 - 0.7j])
@pytest.mark.parametrize("case", list(EDGE))
def test_apply_structured_equals_assembled_pencil(case, tau):
    wl = EDGE[case]()
    P = O.Pencil(wl)
    x = W.random_vector(wl.n, 7)
    ref = P.A @ x - tau * (P.B @ x)
    got = P.apply_structured(x, tau)
    # entrywise: both sum the same row products in different orders
    absA = abs(P.A) @ np.abs(x) + abs(tau) * np.abs(P.B @ x)
    L = wl.Ny + 2 * wl.Nxi + 8
    assert np.all(np.abs(got - ref) <= 2 * L * U * absA + 1e-300)
    # inflow rows are identity rows of A and zero rows of B
    bc = P.bc.ravel()
    assert np.array_equal(got[bc], x[bc])


def test_apply_structured_detects_a_dropped_term():
    """The comparison above is sharp: leaving out the moment coupling, or
    shifting the inflow rows, breaks it by far more than rounding."""
    wl = W.config1()
    P = O.Pencil(wl)
    x = W.random_vector(wl.n, 8)
    ref = P.A @ x
    X = x.reshape(P.Ny, 2, P.Nxi)
    m = np.einsum("jafk,jfk->ja", P.M, X)
    coupling = np.einsum("jfak,ja->jfk", P.U, m).ravel()
    coupling[P.bc.ravel()] = 0.0
    assert np.max(np.abs(P.apply_structured(x) + coupling - ref)) > 1e-3 * np.max(np.abs(ref))


# ------------------------------------------------------- condition numbers --
def _c1_qz():
    wl = W.config1()
    P = O.Pencil(wl)
    lam, X, Y, _ = E.qz_all(P)
    idx = E.order_nearest(lam, wl.sigma)[:10]
    return wl, P, lam[idx], X[:, idx], Y[:, idx]


def test_condition_numbers_from_qz_and_from_adjoint_shift_invert_agree():
    wl, P, lam, X, Y = _c1_qz()
    k_qz = E.condition_numbers(P, lam, X, Y)
    Ysi = E.left_vectors_si(P, lam, wl.sigma)
    k_si = E.condition_numbers(P, lam, X, Ysi)
    assert np.allclose(k_si, k_qz, rtol=1e-6), np.max(np.abs(k_si / k_qz - 1))
    # left vectors solve the adjoint problem y^H (A - lambda B) = 0
    for i in range(len(lam)):
        r = (P.A - lam[i] * P.B).conj().T @ Ysi[:, i]
        assert np.linalg.norm(r) <= 1e-10 * abs(P.A).sum(axis=1).max() * np.linalg.norm(Ysi[:, i])


def test_condition_number_is_the_first_order_sensitivity():
    """lambda(A + eps E, B) - lambda = eps y^H E x / (y^H B x) + O(eps^2): with
    E = y x^H / (|y| |x|) the shift is kappa eps; with random unit E it is at
    most kappa eps."""
    wl, P, lam, X, Y = _c1_qz()
    kap = E.condition_numbers(P, lam, X, Y)
    A, B = P.dense()
    eps = 1e-7
    rng = np.random.default_rng(3)
    for i in (0, 2, 5):
        x, y = X[:, i], Y[:, i]
        Emat = np.outer(y, x.conj()) / (np.linalg.norm(y) * np.linalg.norm(x))
        mu = sla.eigvals(A + eps * Emat, B)
        mu = mu[np.isfinite(mu)]
        shift = np.min(np.abs(mu - lam[i]))
        assert abs(shift / (eps * kap[i]) - 1) < 1e-2, (i, shift, eps * kap[i])
        R = rng.standard_normal(A.shape) + 1j * rng.standard_normal(A.shape)
        R /= np.linalg.norm(R, 2)
        mu = sla.eigvals(A + eps * R, B)
        mu = mu[np.isfinite(mu)]
        assert np.min(np.abs(mu - lam[i])) <= 1.01 * eps * kap[i]


# --------------------------------------------------------------- residuals --
class _DiagPencil:
    """Duck-typed pencil A = diag(d), B = I for residual checks."""

    def __init__(self, d):
        self.n = len(d)
        self.A = sp.diags(d).tocsr()
        self.B = sp.identity(self.n, format="csr", dtype=complex)


def test_residuals_definition_on_a_diagonal_pencil():
    d = np.array([2.0, -1.5 + 0.5j, 3.0j, 0.0, 1e-8])
    P = _DiagPencil(d)
    I = np.eye(len(d))
    lam = d.copy()
    assert np.all(E.residuals(P, lam, I.astype(complex)) == 0.0)
    t = 0.3
    x = I[:, 0] + t * I[:, 1]
    r = E.residuals(P, np.array([d[0]]), x[:, None].astype(complex))[0]
    assert np.isclose(r, t * abs(d[1] - d[0]) / (abs(d[0]) * np.hypot(1.0, t)), rtol=1e-14)
    # |lambda| < 1e-6: absolute residual over ||x||
    x = I[:, 3] + t * I[:, 4]
    r = E.residuals(P, np.array([0.0]), x[:, None].astype(complex))[0]
    assert np.isclose(r, t * abs(d[4]) / np.hypot(1.0, t), rtol=1e-14)


def test_residuals_structured_branch_matches_explicit_branch(monkeypatch):
    wl = W.config1()
    P = O.Pencil(wl)
    lam, X, _, _ = E.qz_nearest(P, wl.sigma, 6)
    Xp = X + 1e-6 * np.stack([W.random_vector(wl.n, 50 + i) for i in range(6)], axis=1) * P.bdiag[:, None]
    r_exp = E.residuals(P, lam, Xp)
    monkeypatch.setattr(E, "EXPLICIT_MAX_N", 0)
    r_str = E.residuals(P, lam, Xp)
    assert np.allclose(r_str, r_exp, rtol=1e-8)
    assert np.all(r_exp > 1e-9)


# ----------------------------------------------------------- order_nearest --
def test_order_nearest_brute_force():
    lam = np.array([3.0, 1 - 1j, 1 + 1j, 0.5, -0.5 + 0j, 2j, -2j, 1.0 + 1e-15])
    got = list(E.order_nearest(lam, 0.0))
    # by distance; equal distances (to 1e-12): Im > 0 first, then the given order
    assert got == [3, 4, 7, 2, 1, 5, 6, 0]
    got = list(E.order_nearest(lam, 1.0))
    assert got[:2] == [7, 3]


# ------------------------------------------------------------ parity.match --
def test_match_accepts_exact_set():
    ref = np.array([0.1 + 0.2j, 0.1 - 0.2j, 0.5, 1.0 + 1j])
    res, skipped = PAR.match(ref[[1, 0, 2]], ref)
    assert all(r["ok"] for r in res) and not skipped


def test_match_rejects_duplicates():
    ref = np.array([0.1 + 0.2j, 0.3, 0.5])
    res, skipped = PAR.match(np.array([0.1 + 0.2j, 0.1 + 0.2j]), ref)
    assert sum(r["ok"] for r in res) == 1
    assert not all(r["ok"] for r in res)


def test_match_reports_a_skipped_nearer_eigenvalue():
    ref = np.array([0.1, 0.2, 0.3, 0.4])
    res, skipped = PAR.match(np.array([0.2, 0.3, 0.4]), ref)
    assert all(r["ok"] for r in res)
    assert skipped == [0]


def test_match_conjugate_tie_is_not_a_skip():
    ref = np.array([1 + 1j, 1 - 1j, 3.0])
    res, skipped = PAR.match(np.array([1 - 1j]), ref, sigma=0.0)
    assert res[0]["ok"] and not skipped


def test_match_conditioning_bound():
    lam_ref = np.array([0.5 + 0.1j])
    got = lam_ref * (1 + 1e-9)
    res, _ = PAR.match(got, lam_ref, tol=1e-10)
    assert not res[0]["ok"]
    normA = 100.0
    # 10 kappa u ||A|| / |lambda| = 2e-9 > 1e-9: accepted as conditioning-limited
    kap = np.array([2e-9 * abs(lam_ref[0]) / (10 * U * normA)])
    res, _ = PAR.match(got, lam_ref, kap, normA, tol=1e-10)
    assert res[0]["ok"] and np.isclose(res[0]["bound"], 2e-9)
    res, _ = PAR.match(got, lam_ref, kap / 4, normA, tol=1e-10)
    assert not res[0]["ok"]


# ------------------------------------------------- row-built ILU(0) oracle --
@pytest.mark.parametrize("cfg,lines", [("c1", 1), ("c1", 4), ("c2", 3), ("ragged", 2)])
def test_row_built_line_block_ilu0_equals_assembled_one(cfg, lines):
    wl = EDGE[cfg]()
    P = O.Pencil(wl)
    sigma = wl.sigma
    b = W.random_vector(wl.n, 30) * P.bdiag
    ref = J.LineBlockILU0(P, sigma, lines).solve(b)
    got = J.LineBlockILU0Rows(P, sigma, lines).solve(b)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_row_built_ilu0_is_exact_lu_for_single_lines_and_drops_fill_for_more():
    """With one line per block the pattern is dense, so ILU(0) is the exact LU
    of the line block; with several lines the cross-line pattern is only the
    node diagonal and fill is dropped, so it differs from the exact solve."""
    wl = W.config1()
    P = O.Pencil(wl)
    sigma = wl.sigma
    b = W.random_vector(wl.n, 31) * P.bdiag
    y = J.LineBlockILU0Rows(P, sigma, 1).solve(b)
    C = (P.A - sigma * P.B).tocsr()
    for f in range(2):
        for k in range(P.Nxi):
            idx = (2 * np.arange(P.Ny) + f) * P.Nxi + k
            blk = C[idx][:, idx].toarray()
            assert np.linalg.norm(blk @ y[idx] - b[idx]) <= 1e-12 * (np.linalg.norm(b[idx]) + 1e-300)
    y4 = J.LineBlockILU0Rows(P, sigma, 4).solve(b)
    Kb = J.LineBlockILU0(P, sigma, 4)
    ex = np.empty_like(b)
    vp = b[Kb.perm]
    Cp = C[Kb.perm][:, Kb.perm].tocsr()
    out = np.empty_like(vp)
    for a, e, _ in Kb.blocks:
        out[a:e] = np.linalg.solve(Cp[a:e, a:e].toarray(), vp[a:e])
    ex[Kb.perm] = out
    assert np.linalg.norm(y4 - ex) > 1e-6 * np.linalg.norm(ex)


# ------------------------------------------- two-sided Rayleigh refinement --
def test_extended_structured_product_matches_fp64_within_rounding():
    wl = W.config1()
    P = O.Pencil(wl)
    x = W.random_vector(wl.n, 60)
    ref = P.A @ x
    got = O.apply_structured_extended(P, x).astype(complex)
    absA = abs(P.A) @ np.abs(x)
    assert np.all(np.abs(got - ref) <= 2 * (wl.Ny + 2 * wl.Nxi + 8) * U * absA + 1e-300)


def test_two_sided_rayleigh_quotient_is_second_order():
    """Vectors perturbed by 1e-6 give eigenvalues within ~1e-12 through the
    two-sided quotient, while the one-sided quotient x^H A x / x^H B x of the
    same vectors is off at first order."""
    wl = W.config1()
    P = O.Pencil(wl)
    lam, X, Y, _ = E.qz_all(P)
    idx = E.order_nearest(lam, wl.sigma)[:6]
    lam, X, Y = lam[idx], X[:, idx], Y[:, idx]
    rng = np.random.default_rng(9)
    pert = lambda M: M + 1e-6 * np.linalg.norm(M, axis=0) * (
        rng.standard_normal(M.shape) + 1j * rng.standard_normal(M.shape)) / np.sqrt(M.shape[0])
    Xp, Yp = pert(X), pert(Y)
    Xp[P.bc.ravel()] = 0.0
    rq = E.refine_two_sided(P, Xp, Yp)
    err2 = np.abs(rq - lam) / np.abs(lam)
    one = np.array([np.vdot(Xp[:, i], P.A @ Xp[:, i]) / np.vdot(Xp[:, i], P.bdiag * Xp[:, i])
                    for i in range(len(lam))])
    err1 = np.abs(one - lam) / np.abs(lam)
    kap = E.condition_numbers(P, lam, X, Y)
    print(err2, err1)
    assert np.all(err2 <= 1e-12 * kap ** 2 + 1e-13)
    assert np.all(err1 >= 100 * err2)
