"""The result definition: the nev finite eigenvalues of A x = lambda B x nearest a
target sigma, with right eigenvectors (Sec. 4, eq. MatrixProblem; the paper asks
for the k eigenvalues closest to a target, Sec. 4.3).

Two routes, both plain:
  * qz_nearest       -- dense QZ of the full pencil (LAPACK zggev through SciPy);
                        eigenvalues with beta ~ 0 are the infinite ones.
  * ShiftInvert /    -- (A - sigma B)^{-1} applied exactly through its structure:
    si_nearest          A - sigma B = P - U M where P (streaming + diagonal +
                        inflow rows) is block diagonal over the velocity lines and
                        U M is the rank-(r Ny) moment coupling, so the Woodbury
                        identity P^-1 + P^-1 U (I - M P^-1 U)^-1 M P^-1 gives the
                        inverse; ARPACK then finds the largest eigenvalues mu of
                        (A - sigma B)^{-1} B and lambda = sigma + 1/mu.  This is the
                        shift-invert Arnoldi route of Sec. 4.1 with a structured
                        exact factorisation in place of a sparse LU.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla


def order_nearest(lam, sigma):
    """Indices ordered by |lambda - sigma|, ties (to 1e-12 relative) broken with
    Im lambda > 0 first (conjugate pairs are equally near a real target)."""
    d = np.abs(lam - sigma)
    scale = max(1.0, float(np.max(d))) if d.size else 1.0
    key = np.round(d / (1e-12 * scale))
    return np.lexsort((-np.sign(lam.imag), key))


def qz_all(P, left=True):
    """All eigenvalues of the pencil with left/right vectors; returns
    (lam_finite, X, Y, n_infinite)."""
    A, B = P.dense()
    (alpha, beta), Y, X = sla.eig(A, B, left=True, right=True, homogeneous_eigvals=True)
    finite = np.abs(beta) > 1e-10 * np.maximum(np.abs(alpha), 1.0)
    lam = alpha[finite] / beta[finite]
    return lam, X[:, finite], Y[:, finite], int(np.count_nonzero(~finite))


def condition_numbers(P, lam, X, Y):
    """kappa_i = ||y_i|| ||x_i|| / |y_i^H B x_i| for simple eigenvalues."""
    BX = P.B @ X
    num = np.linalg.norm(Y, axis=0) * np.linalg.norm(X, axis=0)
    den = np.abs(np.einsum("ij,ij->j", Y.conj(), BX))
    return num / den


def qz_nearest(P, sigma, nev):
    lam, X, Y, ninf = qz_all(P)
    idx = order_nearest(lam, sigma)[:nev]
    kap = condition_numbers(P, lam[idx], X[:, idx], Y[:, idx])
    return lam[idx], X[:, idx], kap, ninf


class ShiftInvert:
    """Exact (A - sigma B)^{-1} (or its adjoint) through velocity-line LUs and a
    rank-(r Ny) Woodbury capacitance."""

    def __init__(self, P, sigma, adjoint=False):
        wl = P.wl
        Ny, Nxi, r = P.Ny, P.Nxi, P.r
        self.P, self.sigma, self.adjoint = P, sigma, adjoint
        nu = P.state["nu"]
        bcl = P.bc[:, 0, :]          # inflow pattern is the same for both fields
        lines = np.empty((Nxi, Ny, Ny), complex)
        for k in range(Nxi):
            Pk = wl.xi_x[k] * P.Dx + np.diag(1j * wl.beta * wl.xi_y[k] + nu - sigma)
            Pk = Pk.astype(complex)
            for j in range(Ny):
                if bcl[j, k]:
                    Pk[j, :] = 0.0
                    Pk[j, j] = 1.0
            lines[k] = Pk.conj().T if adjoint else Pk
        self.lines = lines                                         # [k, j, m]
        self.lines_inv = np.linalg.inv(lines)                      # [k, j, m]
        U = P.U * (~P.bc)[:, :, None, :]                           # zero on inflow rows
        M = P.M
        if adjoint:
            # (P - U M)^H = P^H - M^H U^H: roles of U and M swap (conjugated).
            U, M = M.transpose(0, 2, 1, 3).conj(), U.transpose(0, 2, 1, 3).conj()
            # now U[j, f, a, k] and M[j, a, f, k] again
        self.U, self.M = U, M
        # capacitance C = I - M P^-1 U, index (j, a), (J, A)
        # sum over (f, k) of M[j,a,f,k] Pinv_k[j,J] U[J,f,A,k], as batched products
        MPU = np.zeros((Ny, Ny, r, r), complex)                  # [J, j, a, A]
        inv_t = self.lines_inv.transpose(2, 1, 0)                 # [J, j, k]
        for f in range(2):
            for J in range(Ny):
                Z = M[:, :, f, :] * inv_t[J][:, None, :]          # [j, a, k]
                MPU[J] += (Z.reshape(Ny * r, Nxi) @ U[J, f].T).reshape(Ny, r, r)
        MPU = MPU.transpose(1, 2, 0, 3)                           # [j, a, J, A]
        self.C = np.eye(Ny * r) - MPU.reshape(Ny * r, Ny * r)
        self.C_lu = sla.lu_factor(self.C)
        self.Ny, self.Nxi, self.r = Ny, Nxi, r

    def _pinv(self, b):
        Ny, Nxi = self.Ny, self.Nxi
        v = b.reshape(Ny, 2, Nxi).transpose(2, 0, 1)               # [k, m, f]
        return np.matmul(self.lines_inv, v).transpose(1, 2, 0).reshape(-1)

    def solve(self, b):
        Ny, Nxi, r = self.Ny, self.Nxi, self.r
        y = self._pinv(b)
        Y = y.reshape(Ny, 2, Nxi)
        m = (self.M * Y[:, None, :, :]).sum(axis=(2, 3)).reshape(-1)
        c = sla.lu_solve(self.C_lu, m).reshape(Ny, r)
        z = (self.U * c[:, None, :, None]).sum(axis=2).reshape(-1)
        return y + self._pinv(z)


def si_nearest(P, sigma, nev, ncv=None, tol=1e-14, v0=None):
    """nev eigenpairs nearest sigma by ARPACK on (A - sigma B)^{-1} B."""
    S = ShiftInvert(P, sigma)
    n = P.n
    Bd = P.bdiag
    op = spla.LinearOperator((n, n), matvec=lambda x: S.solve(Bd * x.ravel()), dtype=complex)
    k = min(nev + 6, n - 2)
    ncv = ncv or min(n - 1, max(2 * k + 1, 40))
    if v0 is None:
        v0 = Bd * (np.cos(np.arange(n) * 0.7) + 1j * np.sin(np.arange(n) * 1.3))
    mu, X = spla.eigs(op, k=k, which="LM", ncv=ncv, tol=tol, v0=v0, maxiter=20000)
    lam = sigma + 1.0 / mu
    idx = order_nearest(lam, sigma)[:nev]
    return lam[idx], X[:, idx]


def left_vectors_si(P, lam, sigma, tol=1e-14):
    """Left eigenvectors y (A^H y = conj(lambda) B^H y) by ARPACK on the adjoint
    structured inverse; used for condition numbers at sizes where QZ is too big."""
    S = ShiftInvert(P, sigma, adjoint=True)
    n = P.n
    Bd = P.bdiag
    op = spla.LinearOperator((n, n), matvec=lambda x: S.solve(Bd * x.ravel()), dtype=complex)
    k = min(len(lam) + 6, n - 2)
    mu, Y = spla.eigs(op, k=k, which="LM", ncv=min(n - 1, max(2 * k + 1, 40)), tol=tol)
    lam_l = np.conj(np.conj(sigma) + 1.0 / mu)
    out = np.empty((n, len(lam)), complex)
    for i, l in enumerate(lam):
        out[:, i] = Y[:, int(np.argmin(np.abs(lam_l - l)))]
    return out


#: largest n for which residuals() uses the assembled matrices; above it the
#: structured product of the row definition
EXPLICIT_MAX_N = 60000


def residuals(P, lam, X):
    """Relative residual ||A x - lambda B x|| / (|lambda| ||x||) (the acceptance
    test of Sec. 4.2; absolute residual over ||x|| when |lambda| < 1e-6)."""
    if P.n <= EXPLICIT_MAX_N:
        R = P.A @ X - (P.B @ X) * lam[None, :]
    else:
        R = np.stack([P.apply_structured(X[:, i], lam[i]) for i in range(len(lam))], axis=1)
    nr = np.linalg.norm(R, axis=0)
    nx = np.linalg.norm(X, axis=0)
    den = np.where(np.abs(lam) < 1e-6, 1.0, np.abs(lam)) * nx
    return nr / den


def refine_two_sided(P, X, Y):
    """Two-sided Rayleigh quotients lambda = (y^H A x) / (y^H B x) of right and
    left eigenvector approximations (columns of X and Y), with A x formed and
    both inner products accumulated in extended precision.  If x and y carry
    errors e_x and e_y, y^H (A - lambda B) x = e_y^H (A - lambda B) e_x, so the
    quotient's error is second order in the vector errors, and the extended
    arithmetic keeps the rounding of the quotient itself well below FP64's."""
    from .operator import apply_structured_extended
    cld = np.clongdouble
    out = np.empty(X.shape[1], complex)
    Bd = P.bdiag.astype(np.longdouble)
    for i in range(X.shape[1]):
        x = X[:, i]
        y = Y[:, i].astype(cld)
        ax = apply_structured_extended(P, x)
        num = np.sum(np.conj(y) * ax)
        den = np.sum(np.conj(y) * (Bd * x.astype(cld)))
        out[i] = complex(num / den)
    return out
