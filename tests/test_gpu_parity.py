"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Every input is seeded and synthetic (paper_2607_27440_amd.workloads); every
expected value comes from oracle/.  Floating-point bounds are stated per test:
entrywise results use the dot-product error bound c * u * (|A| |x|)_i, solves use
the eigenpair matching rule of oracle.parity.
"""
import os

import numpy as np
import pytest

from paper_2607_27440_amd import workloads as W
from oracle import eig as E
from oracle import jd as OJ
from oracle import operator as O
from oracle import parity as PAR

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U = 2.0 ** -53
DEV = "cuda:0"


def _klst():
    from paper_2607_27440_amd import klst
    return klst


def _ctx(wl, **kw):
    klst = _klst()
    print(f"[case] {wl.name} n={wl.n} opts={kw}", flush=True)
    ctx = klst.Context(**kw)
    ctx.assemble(wl)
    return ctx


def _abs_bound(P, x, tau):
    """(|A - tau B| |x|)_i from the structured pieces (valid at every size)."""
    wl = P.wl
    ax = np.abs(x).reshape(P.Ny, 2, P.Nxi)
    y = np.einsum("jm,mfk->jfk", np.abs(P.Dx), ax) * np.abs(wl.xi_x)[None, None, :]
    y += np.abs(1j * wl.beta * wl.xi_y[None, None, :] + P.state["nu"][:, None, None] - tau) * ax
    m = np.einsum("jafk,jfk->ja", np.abs(P.M), ax)
    y += np.einsum("jfak,ja->jfk", np.abs(P.U), m)
    y[P.bc] = ax[P.bc]
    return y.ravel()


def _table_bound(P, x, eps_dx=1e-14, eps_nu=1e-14, eps_u=1e-13, eps_m=1e-13):
    """Entrywise bound of |(A_lib - A) x| when the library's own assembly lies
    within eps of the oracle's tables (the agreement the host-table test
    asserts: D_x and nu relative to their largest entry, U and M node by node
    relative to the node's largest entry); first order in the differences,
    zero on the boundary rows (y = x there)."""
    wl = P.wl
    ax = np.abs(x).reshape(P.Ny, 2, P.Nxi)
    aU, aM = np.abs(P.U), np.abs(P.M)
    dD = eps_dx * np.abs(P.Dx).max()
    dn = eps_nu * np.abs(P.state["nu"]).max()
    dU = eps_u * aU.max(axis=(1, 2, 3))                             # per node
    dM = eps_m * aM.max(axis=(1, 2, 3))
    y = np.broadcast_to(dD * ax.sum(axis=0)[None] * np.abs(wl.xi_x)[None, None, :], ax.shape).copy()
    y += dn * ax
    m = np.einsum("jafk,jfk->ja", aM, ax)                           # |M| |x| per node and moment
    y += (dU * m.sum(axis=1))[:, None, None]                        # |dU| |M| |x|
    y += (dM * ax.sum(axis=(1, 2)))[:, None, None] * aU.sum(axis=2)  # |U| |dM| |x|
    y[P.bc] = 0.0
    return y.ravel()


def _norm1_bound(P):
    """Upper bound of ||A||_1 (largest column sum of |A|) from the structured pieces,
    by the triangle inequality on every entry; needs no assembled matrix."""
    wl = P.wl
    nonbc = (~P.bc[:, 0, :]).astype(float)                       # [Ny, Nxi], same for both fields
    stream = np.einsum("jk,jm->mk", nonbc, np.abs(P.Dx)) * np.abs(wl.xi_x)[None, :]
    diag = np.abs(1j * wl.beta * wl.xi_y[None, :] + P.state["nu"][:, None]) * nonbc + (1 - nonbc)
    ucol = np.einsum("mk,mfak->ma", nonbc, np.abs(P.U))           # [Ny, r]
    coup = np.einsum("ma,mafk->mfk", ucol, np.abs(P.M))           # column (m, f, k)
    return float(np.max(stream[:, None, :] + diag[:, None, :] + coup))


def _gamma(P):
    """Deterministic dot-product error bound factor gamma_L = L u for the longest
    row (L = Ny - 1 + 2 Nxi entries plus the rank-r update)."""
    return (P.Ny + 2 * P.Nxi + P.r + 4) * U


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


CONFIGS = {"c1": W.config1, "c2": W.config2}


@pytest.mark.parametrize("cfg", ["c1", "c2"])
@pytest.mark.parametrize("tau", [0.0, 0.3 - 0.7j])
def test_apply_matches_oracle(cfg, tau):
    wl = CONFIGS[cfg]()
    P = O.Pencil(wl)
    x = W.random_vector(wl.n, 11)
    ctx = _ctx(wl)
    xd = _dev(x)
    yd = torch.empty_like(xd)
    ctx.apply(tau, xd, yd)
    torch.cuda.synchronize()
    y = yd.cpu().numpy()
    ref = P.apply(x, tau)
    bound = _gamma(P) * _abs_bound(P, x, tau) + 1e-300
    assert np.all(np.abs(y - ref) <= bound), np.max(np.abs(y - ref) / bound)


@pytest.mark.parametrize("cfg", ["c1", "c2"])
def test_apply_csr_matches_oracle(cfg):
    wl = CONFIGS[cfg]()
    P = O.Pencil(wl)
    x = W.random_vector(wl.n, 12)
    tau = 0.1 + 0.05j
    ctx = _ctx(wl)
    assert ctx.nnz == P.A.nnz == O.nnz_formula(P.Ny, P.Nxi, int(P.bc.sum()))
    xd = _dev(x)
    yd = torch.empty_like(xd)
    ctx.apply_csr(tau, xd, yd)
    torch.cuda.synchronize()
    y = yd.cpu().numpy()
    ref = P.apply(x, tau)
    bound = _gamma(P) * _abs_bound(P, x, tau) + 1e-300
    assert np.all(np.abs(y - ref) <= bound), np.max(np.abs(y - ref) / bound)


def test_apply_c3_full_shape():
    """M=4, Ny=96, Nxi=1464 (n = 281,088): every entry of one matrix-free apply
    against the oracle's structured apply."""
    wl = W.config3()
    P = O.Pencil(wl)
    x = W.random_vector(wl.n, 13)
    ctx = _ctx(wl)
    xd = _dev(x)
    yd = torch.empty_like(xd)
    ctx.apply(0.0, xd, yd)
    torch.cuda.synchronize()
    y = yd.cpu().numpy()
    ref = P.apply_structured(x, 0.0)
    bound = _gamma(P) * _abs_bound(P, x, 0.0) + 1e-300
    assert np.all(np.abs(y - ref) <= bound), np.max(np.abs(y - ref) / bound)


@pytest.mark.parametrize("cfg", ["c1", "c2", "c3"])
def test_apply_f32_matches_oracle(cfg):
    """The FP32 operator of the mixed-precision inner solve (klst_apply_f32: the
    tables rounded to FP32, the streaming sum on the FP32 matrix cores, FP32
    accumulation) against the oracle's FP64 product of the same FP32 input:
    every entry within 2 gamma_L(u32) (|A - tau B| |x|)_i, the dot-product bound
    doubled for the tables' own FP32 rounding."""
    wl = {"c1": W.config1, "c2": W.config2, "c3": W.config3}[cfg]()
    P = O.Pencil(wl)
    x = W.random_vector(wl.n, 14).astype(np.complex64)
    tau = 0.1 + 0.05j
    print(f"[case] FP32 operator {wl.name}", flush=True)
    ctx = _ctx(wl, precision=1, pc_kernel=2)
    xd = torch.from_numpy(x).to(DEV)
    yd = torch.empty_like(xd)
    ctx.apply_f32(tau, xd, yd)
    torch.cuda.synchronize()
    y = yd.cpu().numpy().astype(np.complex128)
    x64 = x.astype(np.complex128)
    ref = P.apply_structured(x64, tau) if wl.n > 60000 else P.apply(x64, tau)
    bound = 2 * (P.Ny + 2 * P.Nxi + P.r + 8) * 2.0 ** -24 * _abs_bound(P, x64, tau) + 1e-30
    assert np.all(np.abs(y - ref) <= bound), np.max(np.abs(y - ref) / bound)


@pytest.mark.parametrize("cfg,nvec", [("c2", 5), ("c2", 12), ("c3", 9)])
def test_apply_many_equals_single(cfg, nvec):
    """The batched operator (the many-vector kernels from 8 vectors on) gives every
    vector bit for bit what a single application gives it."""
    wl = {"c2": W.config2, "c3": W.config3}[cfg]()
    ctx = _ctx(wl)
    x = np.stack([W.random_vector(wl.n, 20 + i) for i in range(nvec)])
    xd = _dev(x.ravel())
    yd = torch.empty_like(xd)
    ctx.apply_many(0.2j, nvec, xd, yd)
    y1 = torch.empty(wl.n, dtype=torch.complex128, device=DEV)
    for i in range(nvec):
        ctx.apply(0.2j, xd[i * wl.n:(i + 1) * wl.n], y1)
        torch.cuda.synchronize()
        assert torch.equal(y1, yd[i * wl.n:(i + 1) * wl.n])


@pytest.mark.parametrize("pc_kernel", [0, 1])
@pytest.mark.parametrize("cfg,lines", [("c1", 1), ("c1", 4), ("c2", 3)])
def test_precond_matches_oracle(cfg, lines, pc_kernel):
    """Both application kernels of the block-Jacobi ILU(0) preconditioner (level-set
    triangular sweeps; stored block inverse) against the oracle's plain ILU(0)."""
    wl = CONFIGS[cfg]()
    P = O.Pencil(wl)
    sigma = wl.sigma
    K = OJ.LineBlockILU0(P, sigma, lines)
    b = W.random_vector(wl.n, 30) * P.bdiag
    ctx = _ctx(wl, lines_per_block=lines, pc_kernel=pc_kernel)
    ctx.precond_setup(sigma)
    bd = _dev(b)
    yd = torch.empty_like(bd)
    ctx.precond_apply(bd, yd)
    torch.cuda.synchronize()
    y = yd.cpu().numpy()
    ref = K.solve(b)
    err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    assert err <= 1e-11, err


@pytest.mark.parametrize("cfg", ["c1", "c2"])
def test_structured_inverse_matches_oracle(cfg):
    """Structured exact (A - sigma B)^{-1} (velocity-line inverses plus the moment
    capacitance) against the oracle's structured shift-invert solve: the GPU
    result's normwise backward error is at rounding level and it agrees with the
    oracle's solution."""
    wl = CONFIGS[cfg]()
    P = O.Pencil(wl)
    sigma = wl.sigma
    b = W.random_vector(wl.n, 31)
    ctx = _ctx(wl, pc_kernel=2)
    ctx.precond_setup(sigma)
    bd = _dev(b)
    yd = torch.empty_like(bd)
    ctx.precond_apply(bd, yd)
    torch.cuda.synchronize()
    y = yd.cpu().numpy()
    C = (P.A - sigma * P.B).tocsr()
    normC = abs(C).sum(axis=0).max()
    bwd = np.linalg.norm(C @ y - b) / (normC * np.linalg.norm(y) + np.linalg.norm(b))
    ref = E.ShiftInvert(P, sigma).solve(b)
    err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    print(f"backward error {bwd:.2e}, difference to oracle {err:.2e}", flush=True)
    assert bwd <= 1e-14, bwd
    assert err <= 1e-9, err


def _check_solve(wl, out, ref_lam, kappa=None, normA=None, tol=1e-10):
    lam = out["lam"]
    assert out["nconv"] == wl.nev, out["stats"]
    assert np.all(out["resid"] <= 1e-10), out["resid"]
    res, skipped = PAR.match(lam, ref_lam, kappa, normA, sigma=wl.sigma, tol=tol)
    bad = [r for r in res if not r["ok"]]
    assert not bad, bad
    assert not skipped, skipped


def test_solve_c1_matches_qz():
    wl = W.config1()
    P = O.Pencil(wl)
    lam_all, X, Y, ninf = E.qz_all(P)
    assert ninf == int(P.bc.sum())
    idx = E.order_nearest(lam_all, wl.sigma)[:wl.nev + 10]
    kap = E.condition_numbers(P, lam_all[idx], X[:, idx], Y[:, idx])
    normA = abs(P.A).sum(axis=0).max()
    ctx = _ctx(wl, pc_kernel=1, lines_per_block=4, m_max=40)
    out = ctx.solve(wl.sigma, wl.nev)
    print(out["stats"], flush=True)
    _check_solve(wl, out, lam_all[idx], kap, normA)
    # eigenvectors: residual with the oracle's explicit matrices
    r = E.residuals(P, out["lam"], out["X"])
    assert np.all(r <= 1e-10), r
    # convergence history: one row per correction equation, locked count never
    # decreasing (past nev while guard pairs confirm the nearest set, below the
    # 2 nev cap), every recorded residual above the locking threshold tol / 2
    h = ctx.history()
    assert h.shape[1] == 6 and 0 < len(h) <= out["stats"]["outer_iterations"]
    assert np.all(np.diff(h[:, 1]) >= 0) and h[-1, 1] < 2 * wl.nev
    assert np.all(h[:, 2] > 0.5e-10)
    assert np.all((h[:, 5] == 1) == (h[:, 2] <= 0.01))


@pytest.mark.parametrize("precision", [0, 1])
def test_solve_c1_structured_inverse(precision):
    """JD with the exact structured inverse as preconditioner (FP64, or FP32
    inside FP64 refinement) reaches the QZ eigenpairs."""
    wl = W.config1()
    P = O.Pencil(wl)
    lam_all, X, Y, _ = E.qz_all(P)
    idx = E.order_nearest(lam_all, wl.sigma)[:wl.nev + 10]
    kap = E.condition_numbers(P, lam_all[idx], X[:, idx], Y[:, idx])
    normA = abs(P.A).sum(axis=0).max()
    ctx = _ctx(wl, pc_kernel=2, m_max=40, precision=precision)
    out = ctx.solve(wl.sigma, wl.nev)
    print(out["stats"], flush=True)
    _check_solve(wl, out, lam_all[idx], kap, normA, tol=1e-10 if precision == 0 else 1e-8)
    r = E.residuals(P, out["lam"], out["X"])
    assert np.all(r <= 1e-10), r


@pytest.mark.parametrize("reorth", [0, 1])
def test_solve_c2_gram_schmidt_variants(reorth, c2_reference):
    """GMRES Arnoldi with two Gram-Schmidt passes always, or the second only when
    the on-device DGKS test asks for it: both reach the shift-invert eigenpairs."""
    wl, P, ref, kap, normA = c2_reference
    ctx = _ctx(wl, pc_kernel=2, m_max=60, reorth=reorth)
    out = ctx.solve(wl.sigma, wl.nev)
    print(out["stats"], flush=True)
    assert np.all(E.residuals(P, out["lam"], out["X"]) <= 1e-10)
    _check_solve(wl, out, ref, kap, normA, tol=1e-10)


@pytest.mark.parametrize("precision", [0, 1])
def test_solve_c1_restarted_gmres(precision):
    """Correction equations by GMRES(8) restarted up to 40 steps (FP64 residual
    restarts in mixed precision) reach the same eigenpairs as QZ."""
    wl = W.config1()
    P = O.Pencil(wl)
    lam_all, X, Y, _ = E.qz_all(P)
    idx = E.order_nearest(lam_all, wl.sigma)[:wl.nev + 10]
    kap = E.condition_numbers(P, lam_all[idx], X[:, idx], Y[:, idx])
    normA = abs(P.A).sum(axis=0).max()
    ctx = _ctx(wl, pc_kernel=1, lines_per_block=4, m_max=40, gmres_m=8, inner_max_it=40, precision=precision)
    out = ctx.solve(wl.sigma, wl.nev)
    print(out["stats"], flush=True)
    _check_solve(wl, out, lam_all[idx], kap, normA, tol=1e-10 if precision == 0 else 1e-8)
    r = E.residuals(P, out["lam"], out["X"])
    assert np.all(r <= 1e-10), r


@pytest.fixture(scope="module")
def c2_reference():
    """Oracle eigenvalues nearest the target at config 2 (structured shift-invert
    Arnoldi), their condition numbers from left eigenvectors (adjoint structured
    inverse) and ||A||_1, for the conditioning-aware parity rule."""
    wl = W.config2()
    P = O.Pencil(wl)
    ref, X = E.si_nearest(P, wl.sigma, wl.nev + 10)
    Y = E.left_vectors_si(P, ref, wl.sigma)
    BX = P.bdiag[:, None] * X
    kap = np.linalg.norm(Y, axis=0) * np.linalg.norm(X, axis=0) / np.abs(np.einsum("ij,ij->j", Y.conj(), BX))
    normA = abs(P.A).sum(axis=0).max()
    return wl, P, ref, kap, normA


@pytest.mark.parametrize("pc_kernel", [1, 0, 2])
def test_solve_c2_matches_shift_invert(pc_kernel, c2_reference):
    """20 eigenpairs nearest 0.05i (n = 12,288): relative error <= 1e-10, or within
    10 kappa u ||A||_1 / |lambda| for eigenvalues whose conditioning (kappa up to
    ~800 here) puts that floor above 1e-10."""
    wl, P, ref, kap, normA = c2_reference
    ctx = _ctx(wl, lines_per_block=3, m_max=60, pc_kernel=pc_kernel)
    out = ctx.solve(wl.sigma, wl.nev)
    print(out["stats"], flush=True)
    r = E.residuals(P, out["lam"], out["X"])
    assert np.all(r <= 1e-10), r
    _check_solve(wl, out, ref, kap, normA, tol=1e-10)


def test_solve_c1_mixed_precision():
    """FP32 inner GMRES (operator, preconditioner, Krylov vectors) inside FP64
    refinement: eigenpairs still meet the FP64 residual gate and match QZ."""
    wl = W.config1()
    P = O.Pencil(wl)
    lam_all, X, Y, _ = E.qz_all(P)
    idx = E.order_nearest(lam_all, wl.sigma)[:wl.nev + 10]
    kap = E.condition_numbers(P, lam_all[idx], X[:, idx], Y[:, idx])
    normA = abs(P.A).sum(axis=0).max()
    ctx = _ctx(wl, pc_kernel=1, lines_per_block=4, m_max=40, precision=1)
    out = ctx.solve(wl.sigma, wl.nev)
    print(out["stats"], flush=True)
    _check_solve(wl, out, lam_all[idx], kap, normA, tol=1e-8)
    res, _ = PAR.match(out["lam"], lam_all[idx], kap, normA, sigma=wl.sigma, tol=1e-8)
    print("mixed rel. errors:", [f"{r['err']:.2e}" for r in res], flush=True)


@pytest.mark.parametrize("pc_kernel", [1, 2])
def test_solve_c2_mixed_precision(pc_kernel, c2_reference):
    wl, P, ref, kap, normA = c2_reference
    ctx = _ctx(wl, pc_kernel=pc_kernel, lines_per_block=3, m_max=60, precision=1)
    out = ctx.solve(wl.sigma, wl.nev)
    print(out["stats"], flush=True)
    r = E.residuals(P, out["lam"], out["X"])
    assert np.all(r <= 1e-10), r
    _check_solve(wl, out, ref, kap, normA, tol=1e-8)
    res, _ = PAR.match(out["lam"], ref, kap, normA, sigma=wl.sigma, tol=1e-8)
    print("mixed rel. errors:", [f"{r['err']:.2e}" for r in res], flush=True)


@pytest.mark.parametrize("draw", [7, 27, 40])
def test_sweep_hard_draws_structured_inverse(draw):
    """Sweep draws on which block-Jacobi ILU(0) correction solves stall: the line
    blocks drop the collision-invariant coupling, so GMRES(20) barely reduces the
    correction residual.  With the exact structured inverse JD converges, and the
    eigenvalues match the oracle's shift-invert Arnoldi."""
    wl = W.sweep(seed=4, count=64, nev=8)[draw]
    P = O.Pencil(wl)
    ref, X = E.si_nearest(P, wl.sigma, wl.nev + 6)
    Y = E.left_vectors_si(P, ref, wl.sigma)
    kap = np.linalg.norm(Y, axis=0) * np.linalg.norm(X, axis=0) / np.abs(
        np.einsum("ij,ij->j", Y.conj(), P.bdiag[:, None] * X))
    normA = abs(P.A).sum(axis=0).max()
    ctx = _ctx(wl, pc_kernel=2, m_max=30)
    out = ctx.solve(wl.sigma, wl.nev)
    print(out["stats"], flush=True)
    assert np.all(E.residuals(P, out["lam"], out["X"]) <= 1e-10)
    _check_solve(wl, out, ref, kap, normA, tol=1e-10)


def test_guard_settles_above_tolerance():
    """Served-sweep draw 69 (seed 5): the 8 nearest lock within 50 outer
    iterations; the guard that follows (one of the pair 1.2283 +- 0.0037i,
    condition numbers ~1e4) stalls near relative residual 5e-8, above the
    locking tolerance.  A guard settled below 1e-6 beyond the 8th nearest
    completes the set (the solve used to run into its 2,000-iteration cap).  The
    8 eigenvalues match the oracle's shift-invert Arnoldi."""
    wl = W.sweep(seed=5, count=80, nev=8)[69]
    P = O.Pencil(wl)
    ref, X = E.si_nearest(P, wl.sigma, wl.nev + 6)
    Y = E.left_vectors_si(P, ref, wl.sigma)
    kap = np.linalg.norm(Y, axis=0) * np.linalg.norm(X, axis=0) / np.abs(
        np.einsum("ij,ij->j", Y.conj(), P.bdiag[:, None] * X))
    normA = abs(P.A).sum(axis=0).max()
    ctx = _ctx(wl, pc_kernel=2, m_max=30, m_min=6, gmres_m=20, max_it=2000)
    out = ctx.solve(wl.sigma, wl.nev)
    print(out["stats"], flush=True)
    assert out["stats"]["outer_iterations"] < 300, out["stats"]
    assert np.all(E.residuals(P, out["lam"], out["X"]) <= 1e-10)
    _check_solve(wl, out, ref, kap, normA, tol=1e-10)


def _assert_closed_under_conjugation(lam, rel=1e-9):
    """A real target on a reflection-symmetric problem: every returned complex
    eigenvalue's conjugate is returned too (the farthest pair may be split by
    the nev cut, so the two farthest values are exempt)."""
    lam = np.asarray(lam)
    far = np.argsort(np.abs(lam))[-2:]
    for i, lv in enumerate(lam):
        if i in far or abs(lv.imag) <= 1e-12 * abs(lv):
            continue
        assert np.min(np.abs(lam - np.conj(lv))) <= rel * abs(lv), (lv, lam)


def _c3_reference():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c3_m4_reference.txt")
    a = np.loadtxt(path)
    return a[:, 0] + 1j * a[:, 1], a[:, 3]


def test_solve_c3_matches_oracle_reference():
    """The 281,088-unknown Mach 4 bimodal shock, 10 eigenpairs nearest 0, FP64 JD
    with the exact structured inverse, against the oracle's stored shift-invert
    Arnoldi eigenvalues (tests/golden/c3_m4_reference.txt).  The 8 nearest are
    unique; the rest lie in a cluster of 16 eigenvalues within 1e-5 relative of
    each other, where any members are correct: each must match a distinct cluster
    member.  Residuals are recomputed by the oracle's structured operator."""
    wl = W.config3()
    P = O.Pencil(wl)
    ref, kap = _c3_reference()
    normA = _norm1_bound(P)
    ctx = _ctx(wl, pc_kernel=2, m_max=80, fix=1e-3, max_it=2000)
    out = ctx.solve(wl.sigma, wl.nev)
    print(out["stats"], flush=True)
    assert out["nconv"] == wl.nev, out["stats"]
    assert np.all(out["resid"] <= 1e-10), out["resid"]
    assert np.all(E.residuals(P, out["lam"], out["X"]) <= 1e-10)
    res, skipped = PAR.match(out["lam"], ref, kap, normA, sigma=wl.sigma, tol=1e-10, tie=1e-5)
    print("C3 rel. errors:", [f"{r['err']:.2e}/{r['bound']:.1e}" for r in res], flush=True)
    assert all(r["ok"] for r in res), res
    assert not skipped, skipped
    assert sorted(r["j"] for r in res)[:8] == list(range(8))
    # the reference eigenvalues are two-sided Rayleigh quotients in extended
    # precision (accurate far below 1e-10): the 8 unique ones meet the FP64 bar
    # itself, with no conditioning allowance
    assert all(r["err"] <= 1e-10 for r in res if r["j"] < 8), [r for r in res if r["j"] < 8]
    _assert_closed_under_conjugation(out["lam"])


def test_solve_c3_mixed_precision_matches_oracle_reference():
    """The Mach 4 pencil with FP32 inner solves (FP32 structured inverse and
    GMRES inside FP64 refinement of the correction equation): every eigenpair
    within the mixed-precision bar of 1e-8 of the oracle's reference, residuals
    gated in FP64."""
    wl = W.config3()
    P = O.Pencil(wl)
    ref, kap = _c3_reference()
    normA = _norm1_bound(P)
    ctx = _ctx(wl, pc_kernel=2, m_max=80, fix=1e-3, max_it=3000, precision=1)
    out = ctx.solve(wl.sigma, wl.nev)
    print(out["stats"], flush=True)
    assert out["nconv"] == wl.nev, out["stats"]
    assert np.all(out["resid"] <= 1e-10), out["resid"]
    assert np.all(E.residuals(P, out["lam"], out["X"]) <= 1e-10)
    res, skipped = PAR.match(out["lam"], ref, kap, normA, sigma=wl.sigma, tol=1e-8, tie=1e-5)
    print("C3 mixed rel. errors:", [f"{r['err']:.2e}" for r in res], flush=True)
    assert all(r["ok"] for r in res), res
    assert not skipped, skipped
    assert sorted(r["j"] for r in res)[:8] == list(range(8))


@pytest.mark.parametrize("workload", ["c2", "c3", "m4_gh48", "pb_q20", "pb_q24", "pb_q32"])
@pytest.mark.parametrize("krylov32", [0, 1])
def test_bench_configurations_match_oracle(workload, c2_reference, krylov32):
    """The solve exactly as bench.py times it (its workload options) against the
    oracle: config 2 against shift-invert Arnoldi, the other shapes against their
    stored references; the nearest set complete, residuals gated in FP64.  Also
    with the inner GMRES Krylov basis stored in FP32 (krylov32 = 1), which must
    meet the same FP64 bar."""
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import bench
    from paper_2607_27440_amd import workloads as WL
    gen, opts = bench.WORKLOADS[workload]
    wl = bench.make_workload(WL, gen)
    P = O.Pencil(wl)
    if workload == "c2":
        _, _, ref, kap, normA = c2_reference
        tie = 1e-8
    else:
        ref, kap = (_c3_reference() if workload == "c3" else _golden(workload))
        normA = _norm1_bound(P)
        tie = 1e-5 if workload == "c3" else 1e-8
    ctx = _ctx(wl, **opts, krylov32=krylov32)
    out = ctx.solve(wl.sigma, wl.nev)
    print(out["stats"], flush=True)
    assert out["nconv"] == wl.nev and np.all(out["resid"] <= 1e-10), out["stats"]
    assert np.all(E.residuals(P, out["lam"], out["X"]) <= 1e-10)
    res, skipped = PAR.match(out["lam"], ref, kap, normA, sigma=wl.sigma, tol=1e-10, tie=tie)
    print(workload, "max rel. error:", max(r["err"] for r in res), flush=True)
    assert all(r["ok"] for r in res), [r for r in res if not r["ok"]]
    assert not skipped, skipped
    if workload in ("c3", "m4_gh48"):
        # references refined by extended-precision two-sided Rayleigh quotients:
        # every isolated eigenvalue (no other reference eigenvalue within 1e-6
        # relative) meets the FP64 bar with no conditioning allowance
        for r in res:
            d = np.abs(ref - ref[r["j"]])
            d[r["j"]] = np.inf
            if np.min(d) > 1e-6 * abs(ref[r["j"]]):
                assert r["err"] <= 1e-10, (workload, r)
        if complex(wl.sigma).imag == 0.0:
            _assert_closed_under_conjugation(out["lam"])


# ---- shift-invert Krylov-Schur with the exact structured inverse --------------

def test_shift_invert_c1_matches_qz():
    wl = W.config1()
    P = O.Pencil(wl)
    lam_all, X, Y, _ = E.qz_all(P)
    idx = E.order_nearest(lam_all, wl.sigma)[:wl.nev + 10]
    kap = E.condition_numbers(P, lam_all[idx], X[:, idx], Y[:, idx])
    normA = abs(P.A).sum(axis=0).max()
    ctx = _ctx(wl, m_max=30, max_it=200)
    out = ctx.solve(wl.sigma, wl.nev, method="shift_invert")
    print(out["stats"], flush=True)
    _check_solve(wl, out, lam_all[idx], kap, normA)
    assert np.all(E.residuals(P, out["lam"], out["X"]) <= 1e-10)
    d = np.abs(out["lam"] - wl.sigma)
    assert np.all(np.diff(d) >= -1e-12 * d[1:])          # ordered by distance


def test_shift_invert_c2_matches_oracle(c2_reference):
    """Through klst_solve with method = 1 (options), config 2's 20 pairs."""
    wl, P, ref, kap, normA = c2_reference
    ctx = _ctx(wl, m_max=60, method=1)
    out = ctx.solve(wl.sigma, wl.nev)
    print(out["stats"], flush=True)
    assert np.all(E.residuals(P, out["lam"], out["X"]) <= 1e-10)
    _check_solve(wl, out, ref, kap, normA, tol=1e-10)


@pytest.mark.parametrize("draw", [7, 27, 40, 57])
def test_shift_invert_sweep_draws(draw):
    wl = W.sweep(seed=4, count=64, nev=8)[draw]
    P = O.Pencil(wl)
    ref, X = E.si_nearest(P, wl.sigma, wl.nev + 6)
    Y = E.left_vectors_si(P, ref, wl.sigma)
    kap = np.linalg.norm(Y, axis=0) * np.linalg.norm(X, axis=0) / np.abs(
        np.einsum("ij,ij->j", Y.conj(), P.bdiag[:, None] * X))
    normA = abs(P.A).sum(axis=0).max()
    ctx = _ctx(wl, m_max=30, max_it=200)
    out = ctx.solve(wl.sigma, wl.nev, method="shift_invert")
    print(out["stats"], flush=True)
    assert np.all(E.residuals(P, out["lam"], out["X"]) <= 1e-10)
    _check_solve(wl, out, ref, kap, normA, tol=1e-10)


def test_shift_invert_c3_matches_oracle_reference():
    """The 281,088-unknown Mach 4 pencil by shift-invert Krylov-Schur (search
    space 120, enough to resolve the 1e-6-wide cluster that holds the 9th and
    10th eigenvalues), against the stored oracle eigenvalues: the 8 nearest
    exactly, the rest as distinct cluster members."""
    wl = W.config3()
    P = O.Pencil(wl)
    ref, kap = _c3_reference()
    normA = _norm1_bound(P)
    ctx = _ctx(wl, m_max=120, max_it=100)
    out = ctx.solve(wl.sigma, wl.nev, method="shift_invert")
    print(out["stats"], flush=True)
    assert out["nconv"] == wl.nev, out["stats"]
    assert np.all(out["resid"] <= 1e-10), out["resid"]
    assert np.all(E.residuals(P, out["lam"], out["X"]) <= 1e-10)
    res, skipped = PAR.match(out["lam"], ref, kap, normA, sigma=wl.sigma, tol=1e-10, tie=1e-5)
    print("C3 rel. errors:", [f"{r['err']:.2e}/{r['bound']:.1e}" for r in res], flush=True)
    assert all(r["ok"] for r in res), res
    assert not skipped, skipped
    assert sorted(r["j"] for r in res)[:8] == list(range(8))


# ---- the paper's benchmark shape: Ny = 81, 20 x 20 Gauss-Hermite, 50 eigenpairs --

def _golden(name):
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"{name}_reference.txt")
    a = np.loadtxt(path)
    return a[:, 0] + 1j * a[:, 1], a[:, 3]


#: case -> (workload, JD options, shift-invert options)
PAPER_SHAPES = {
    "pb_q20": (lambda: W.paper_benchmark(20), dict(pc_kernel=2, m_max=150, m_min=30, max_it=3000),
               dict(m_max=150, max_it=100)),
    "pb_q24": (lambda: W.paper_benchmark(24), dict(pc_kernel=2, m_max=150, m_min=30, max_it=3000),
               dict(m_max=150, max_it=100)),
    "pb_q32": (lambda: W.paper_benchmark(32), dict(pc_kernel=2, m_max=150, m_min=30, max_it=3000),
               dict(m_max=150, max_it=100)),
    "m4_gh48": (W.paper_mach4, dict(pc_kernel=2, m_max=80, fix=1e-3, max_it=3000),
                dict(m_max=120, max_it=100)),
}


@pytest.mark.parametrize("method", ["jd", "shift_invert"])
@pytest.mark.parametrize("case", ["pb_q20", "pb_q24", "pb_q32", "m4_gh48"])
def test_solve_paper_shape_matches_oracle_reference(case, method):
    """Gauss-Hermite workloads at the paper's shapes against the oracle's stored
    structured shift-invert Arnoldi eigenvalues (tests/golden/<case>_reference.txt):
    pb_q20 is the M = 1.2 benchmark case (Sec. 4.3: N = 80, Q = 20, beta = 16,
    n = 64,800, the 50 eigenpairs nearest 1e-2, search space 150 as in App. C,
    restarts keeping 30: with 6 kept, a change of summation order in the basis
    rotation once left two conjugate pairs of the Q = 32 cloud unfound);
    m4_gh48 the Mach 4 shape (Sec. 4.4: Ny = 61, Q = 48, n = 281,088, 10 nearest
    0).  FP64; JD with the exact structured inverse, or shift-invert Krylov-Schur."""
    make, jd_opts, si_opts = PAPER_SHAPES[case]
    wl = make()
    P = O.Pencil(wl)
    ref, kap = _golden(case)
    normA = _norm1_bound(P)
    ctx = _ctx(wl, **(jd_opts if method == "jd" else si_opts))
    out = ctx.solve(wl.sigma, wl.nev, method=method)
    print(out["stats"], flush=True)
    assert out["nconv"] == wl.nev, out["stats"]
    assert np.all(out["resid"] <= 1e-10), out["resid"]
    assert np.all(E.residuals(P, out["lam"], out["X"]) <= 1e-10)
    res, skipped = PAR.match(out["lam"], ref, kap, normA, sigma=wl.sigma, tol=1e-10)
    print(case, "rel. errors (max):", max(r["err"] for r in res), flush=True)
    assert all(r["ok"] for r in res), [r for r in res if not r["ok"]]
    assert not skipped, skipped
    d = np.abs(out["lam"] - wl.sigma)
    assert np.all(np.diff(d) >= -1e-12 * d[1:])


def _ragged(Dv):
    """N_y = 40 (three row tiles, the last 8 rows long) at a velocity count whose
    2 N_xi is not a multiple of 16: D_v = 1 (N_xi = 7, rank 3, one partial
    column tile) or D_v = 2 (N_xi = 35, rank 4, five column tiles, the last 6
    columns wide, one partly filled column group)."""
    return W.make_workload(f"ragged_dv{Dv}_ny40", mach=2.0, Ny=40, Qx=7, Qy=5, beta=0.5,
                           sigma=0.0, nev=4, base="bimodal", delta=2.5, Dv=Dv)


@pytest.mark.parametrize("tile", [None, (1, 1), (2, 4), (3, 1), (0, 8)])
@pytest.mark.parametrize("Dv", [1, 2])
def test_apply_many_ragged_tiles(Dv, tile, tmp_path):
    """Ragged row and column tiles under every FP64 operator kernel (the tiled
    MFMA kernel at 1-3 row tiles and 1 or 4 wavefronts, the streaming kernel
    as (0, 8)): each vector of a 9-vector batch equals its single application
    bit for bit, and that is within the dot-product bound of the oracle."""
    klst = _klst()
    wl = _ragged(Dv)
    P = O.Pencil(wl)
    nvec, tau = 9, 0.2 - 0.4j
    x = np.stack([W.random_vector(wl.n, 200 + i) for i in range(nvec)])
    klst.tune_clear()
    try:
        ctx = _ctx(wl)
        xd = _dev(x.ravel())
        y1 = torch.empty_like(xd)
        for i in range(nvec):
            ctx.apply(tau, xd[i * wl.n:(i + 1) * wl.n], y1[i * wl.n:(i + 1) * wl.n])
        if tile is not None:
            path = tmp_path / "tile.txt"
            path.write_text(f"{wl.Ny} {wl.Nxi} {nvec} 0 {tile[0]} {tile[1]} 0 0\n")
            klst.tune_load(str(path))
        print(f"[case] ragged D_v={Dv} tiles {tile}", flush=True)
        y = torch.empty_like(xd)
        ctx.apply_many(tau, nvec, xd, y)
        torch.cuda.synchronize()
        assert torch.equal(y, y1)
        yh = y.cpu().numpy().reshape(nvec, wl.n)
        for i in range(nvec):
            ref = P.apply(x[i], tau)
            bound = _gamma(P) * _abs_bound(P, x[i], tau) + 1e-300
            assert np.all(np.abs(yh[i] - ref) <= bound), np.max(np.abs(yh[i] - ref) / bound)
    finally:
        klst.tune_clear()


@pytest.mark.parametrize("tile", [None, (1, 1), (3, 4), (2, 1), (0, 4), (0, 8), (0, 16)])
@pytest.mark.parametrize("Dv", [1, 2])
def test_apply_f32_ragged_tiles(Dv, tile, tmp_path):
    """The FP32 operator at ragged row and column tiles under each of its
    kernels (matrix-core tilings; the scalar kernel at 4, 8 or 16 rows per
    thread) against the oracle's FP64 product of the same FP32 input, within
    the FP32 dot-product bound doubled for the tables' rounding."""
    klst = _klst()
    wl = _ragged(Dv)
    P = O.Pencil(wl)
    x = W.random_vector(wl.n, 31).astype(np.complex64)
    tau = 0.1 + 0.05j
    klst.tune_clear()
    try:
        ctx = _ctx(wl, precision=1, pc_kernel=2)
        if tile is not None:
            path = tmp_path / "tile.txt"
            path.write_text(f"{wl.Ny} {wl.Nxi} 1 1 {tile[0]} {tile[1]} 0 0\n")
            klst.tune_load(str(path))
        print(f"[case] FP32 ragged D_v={Dv} tiles {tile}", flush=True)
        xd = torch.from_numpy(x).to(DEV)
        yd = torch.empty_like(xd)
        ctx.apply_f32(tau, xd, yd)
        torch.cuda.synchronize()
        y = yd.cpu().numpy().astype(np.complex128)
        x64 = x.astype(np.complex128)
        ref = P.apply(x64, tau)
        bound = 2 * (P.Ny + 2 * P.Nxi + P.r + 8) * 2.0 ** -24 * _abs_bound(P, x64, tau) + 1e-30
        assert np.all(np.abs(y - ref) <= bound), np.max(np.abs(y - ref) / bound)
    finally:
        klst.tune_clear()


@pytest.mark.parametrize("cfg,nvec", [("c2", 5), ("c3", 3), ("ragged2", 9)])
def test_apply_many_f32_matches_oracle(cfg, nvec):
    """The batched FP32 operator (klst_apply_many_f32: FP32 moments of every
    vector, then the FP32 matrix-core operator over all of them in one launch)
    against the oracle's FP64 product of each FP32 input vector, within the FP32
    dot-product bound doubled for the tables' own rounding."""
    wl = {"c2": W.config2, "c3": W.config3, "ragged2": lambda: _ragged(2)}[cfg]()
    P = O.Pencil(wl)
    x = np.stack([W.random_vector(wl.n, 60 + i) for i in range(nvec)]).astype(np.complex64)
    tau = -0.2 + 0.3j
    print(f"[case] batched FP32 operator {wl.name} x {nvec}", flush=True)
    ctx = _ctx(wl, precision=1, pc_kernel=2)
    xd = torch.from_numpy(x.ravel()).to(DEV)
    yd = torch.empty_like(xd)
    ctx.apply_many_f32(tau, nvec, xd, yd)
    torch.cuda.synchronize()
    y = yd.cpu().numpy().astype(np.complex128).reshape(nvec, wl.n)
    for i in range(nvec):
        x64 = x[i].astype(np.complex128)
        ref = P.apply_structured(x64, tau) if wl.n > 60000 else P.apply(x64, tau)
        bound = 2 * (P.Ny + 2 * P.Nxi + P.r + 8) * 2.0 ** -24 * _abs_bound(P, x64, tau) + 1e-30
        assert np.all(np.abs(y[i] - ref) <= bound), (i, np.max(np.abs(y[i] - ref) / bound))


@pytest.mark.parametrize("cfg", ["c3", "ragged1", "ragged2"])
def test_apply_many_f32_streaming_kernel(cfg, tmp_path):
    """The FP32 streaming many-vector kernel (chosen through the launch table
    as (0, 8)) against the tiled FP32 kernel at two row tiles and four
    wavefronts: both accumulate every entry's streaming sum over K in the same
    order on the FP32 matrix cores and form the epilogue with the same fused
    multiply-adds, so they agree bit for bit; and each vector is within the
    FP32 bound of the oracle's product."""
    klst = _klst()
    wl = {"c3": W.config3, "ragged1": lambda: _ragged(1), "ragged2": lambda: _ragged(2)}[cfg]()
    P = O.Pencil(wl)
    nvec, tau = 9, 0.15 - 0.25j
    x = np.stack([W.random_vector(wl.n, 300 + i) for i in range(nvec)]).astype(np.complex64)
    xd = torch.from_numpy(x.ravel()).to(DEV)
    out = {}
    klst.tune_clear()
    try:
        ctx = _ctx(wl, precision=1, pc_kernel=2)
        for name, tile in (("tiled", (2, 4)), ("stream", (0, 8))):
            path = tmp_path / f"{name}.txt"
            path.write_text(f"{wl.Ny} {wl.Nxi} {nvec} 1 {tile[0]} {tile[1]} 0 0\n")
            klst.tune_clear()
            klst.tune_load(str(path))
            print(f"[case] FP32 batched {name} {wl.name}", flush=True)
            yd = torch.empty_like(xd)
            ctx.apply_many_f32(tau, nvec, xd, yd)
            torch.cuda.synchronize()
            out[name] = yd
    finally:
        klst.tune_clear()
    assert torch.equal(out["stream"], out["tiled"])
    y = out["stream"].cpu().numpy().astype(np.complex128).reshape(nvec, wl.n)
    for i in range(nvec):
        x64 = x[i].astype(np.complex128)
        ref = P.apply_structured(x64, tau) if wl.n > 60000 else P.apply(x64, tau)
        bound = 2 * (P.Ny + 2 * P.Nxi + P.r + 8) * 2.0 ** -24 * _abs_bound(P, x64, tau) + 1e-30
        assert np.all(np.abs(y[i] - ref) <= bound), (i, np.max(np.abs(y[i] - ref) / bound))


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("Ny", [56, 72])
def test_apply_many_streaming_kernel_row_tiles(Ny, prec, tmp_path):
    """The streaming many-vector kernel at 4 and 5 row tiles, the last one 8
    rows long, where its LDS holds the x entries of only some row tiles for the
    epilogue in FP64 (three of four, three of five) and of all of them in FP32:
    bit for bit what the single-vector application (FP64) or the tiled FP32
    kernel gives, and within the oracle's product by the dot-product bound
    plus, in FP64, the bound of the two assemblies' table differences (at these
    shapes some small U entries differ by far more than the rounding of a dot
    product relative to themselves, though by under 1e-14 of the table)."""
    klst = _klst()
    wl = W.make_workload(f"stream_ny{Ny}", mach=2.0, Ny=Ny, Qx=7, Qy=5, beta=0.5,
                         sigma=0.0, nev=4, base="bimodal", delta=2.5, Dv=2)
    P = O.Pencil(wl)
    nvec, tau = 9, 0.3 - 0.1j
    x = np.stack([W.random_vector(wl.n, 500 + i) for i in range(nvec)])
    if prec:
        x = x.astype(np.complex64)
    xd = torch.from_numpy(x.ravel()).to(DEV)
    klst.tune_clear()
    try:
        ctx = _ctx(wl, precision=prec, pc_kernel=2)
        if prec:
            path = tmp_path / "tiled.txt"
            path.write_text(f"{wl.Ny} {wl.Nxi} {nvec} 1 2 4 0 0\n")
            klst.tune_load(str(path))
            y1 = torch.empty_like(xd)
            ctx.apply_many_f32(tau, nvec, xd, y1)
            klst.tune_clear()
        else:
            y1 = torch.empty_like(xd)
            for i in range(nvec):
                ctx.apply(tau, xd[i * wl.n:(i + 1) * wl.n], y1[i * wl.n:(i + 1) * wl.n])
        path = tmp_path / "stream.txt"
        path.write_text(f"{wl.Ny} {wl.Nxi} {nvec} {prec} 0 8 0 0\n")
        klst.tune_load(str(path))
        print(f"[case] streaming kernel N_y={Ny} precision {prec}", flush=True)
        y = torch.empty_like(xd)
        if prec:
            ctx.apply_many_f32(tau, nvec, xd, y)
        else:
            ctx.apply_many(tau, nvec, xd, y)
        torch.cuda.synchronize()
    finally:
        klst.tune_clear()
    assert torch.equal(y, y1)
    yh = y.cpu().numpy().astype(np.complex128).reshape(nvec, wl.n)
    for i in range(nvec):
        x64 = x[i].astype(np.complex128)
        ref = P.apply(x64, tau)
        if prec:
            bound = 2 * (P.Ny + 2 * P.Nxi + P.r + 8) * 2.0 ** -24 * _abs_bound(P, x64, tau) + 1e-30
        else:
            bound = _gamma(P) * _abs_bound(P, x64, tau) + _table_bound(P, x64) + 1e-300
        assert np.all(np.abs(yh[i] - ref) <= bound), (i, np.max(np.abs(yh[i] - ref) / bound))
