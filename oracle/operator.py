"""The discrete kLST pencil (A, B) for a 1-D normal shock (Sec. 2.2).

Unknowns q = [g_hat; h_hat] at every (spatial node j, field f, velocity node k);
the paper leaves the ordering open, this oracle uses idx(j, f, k) = (2j + f) Nxi + k.

Rows follow eqs. comp_ghat1Dshock / comp_hhat1Dshock with the left-hand side
written as A q = lambda B q, lambda = i*omega (eq. MatrixSystem):

  (A q)_{j,f,k} = xi_x,k sum_m (D_x)_{jm} q_{m,f,k} + (i beta xi_y,k + nu_j) q_{j,f,k}
                  - sum_a U_a(j,f,k) m_a(j),

with the perturbation-moment functionals of Sec. 2.2 (the integrals below
eq. Comp1DHarm, discretised as in eq. comp_ghat1Dshock)
  m_rho = sum W g,  m_u = sum W (xi_x - u) g / rho,  m_v = sum W xi_y g / rho,
  m_E   = sum W [(|xi|^2 - 2E) g + h] / (2 rho),
and U_a = G_a on g rows, H_a on h rows.  The G/H coefficients are deferred by the
paper to another work; here they are the exact linearisation of the discrete BGK
relaxation nu(m) (f^e(m) - f) about the base state, i.e. of eq. CompBGKtilde
with P = rho T / 2 and mu ~ T^s (the paper does not print them; this form is
pinned by a complex-step derivative of the nonlinear operator):
  G_a = nu [ C_ga + (g^e - g_c) Lambda_a ],  H_a = nu [ C_ha + (h^e - h_c) Lambda_a ],
  C_ga = d g^e / d a,  C_ha = d h^e / d a,  Lambda_a = d ln P/da - d ln mu/da.

Inflow rows (x = -s_inf with xi_x > 0, x = +s_inf with xi_x < 0; Sec. 2.2,
zero-perturbation Dirichlet conditions) are identity rows of A and zero rows of
B, so B = Z = diag(1 - bc): the diagonal boundary-condition matrix Z of the
nomenclature plays the role of B.
"""
import numpy as np
import scipy.sparse as sp

from . import grid as _grid


def rank(Dv):
    """Number of coupled moments: rho, u, (v,) E."""
    return 4 if Dv == 2 else 3


def equilibrium(rho, u, T, xi_x, xi_y, Dv):
    """Reduced Maxwellians g^e, h^e (Sec. 2.2, equilibrium definitions) with
    2RT -> T in these units and (K+1) = 3 - Dv: h^e = ((3 - Dv)/2) T g^e."""
    c2 = (xi_x[None, :] - u[:, None]) ** 2 + xi_y[None, :] ** 2
    ge = rho[:, None] / (np.pi * T[:, None]) ** (0.5 * Dv) * np.exp(-c2 / T[:, None])
    he = 0.5 * (3 - Dv) * T[:, None] * ge
    return ge, he


def moments(g, h, xi_x, xi_y, w):
    """Discrete macros of a reduced VDF pair: rho, u, v, E, T (Sec. 2.2)."""
    rho = g @ w
    u = (g * xi_x[None, :]) @ w / rho
    v = (g * xi_y[None, :]) @ w / rho
    E = 0.5 * ((g * (xi_x ** 2 + xi_y ** 2)[None, :] + h) @ w) / rho
    T = (4.0 / 3.0) * (E - 0.5 * (u ** 2 + v ** 2))
    return rho, u, v, E, T


def base_state(wl):
    """Base macros, collision rate and base VDFs.

    EQ mode (wl.mode == 0): macros are given and (g_c, h_c) := (g^e, h^e).
    NONEQ mode: macros are the discrete moments of the given (g_c, h_c), with the
    transverse velocity set to zero (the base flow is 1-D)."""
    xi_x, xi_y, w, Dv = wl.xi_x, wl.xi_y, wl.w, wl.Dv
    if wl.mode == 0:
        rho = np.asarray(wl.rho, float)
        u = np.asarray(wl.u, float)
        T = np.asarray(wl.T, float)
        E = 0.5 * u ** 2 + 0.75 * T
        ge, he = equilibrium(rho, u, T, xi_x, xi_y, Dv)
        gc, hc = ge, he
    else:
        gc = np.asarray(wl.g_c, float)
        hc = np.asarray(wl.h_c, float)
        rho, u, _v, E, _T = moments(gc, hc, xi_x, xi_y, w)
        T = (4.0 / 3.0) * (E - 0.5 * u ** 2)
        ge, he = equilibrium(rho, u, T, xi_x, xi_y, Dv)
    nu = wl.nu_inf * rho * T ** (1.0 - wl.s_visc)
    return dict(rho=rho, u=u, E=E, T=T, nu=nu, ge=ge, he=he, gc=gc, hc=hc)


def coefficients(wl, st=None):
    """Coupling columns U[j, f, a, k] and moment functionals M[j, a, f, p].

    a runs over (rho, u, v, E) for Dv = 2 and (rho, u, E) for Dv = 1."""
    st = base_state(wl) if st is None else st
    xi_x, xi_y, w, Dv, s = wl.xi_x, wl.xi_y, wl.w, wl.Dv, wl.s_visc
    rho, u, E, T, nu = st["rho"], st["u"], st["E"], st["T"], st["nu"]
    ge, he, gc, hc = st["ge"], st["he"], st["gc"], st["hc"]
    Ny, Nxi = ge.shape
    R = rho[:, None]
    U_ = u[:, None]
    T_ = T[:, None]
    cx = xi_x[None, :] - U_
    c2 = cx ** 2 + xi_y[None, :] ** 2
    dlng_dT = c2 / T_ ** 2 - 0.5 * Dv / T_
    zero = np.zeros_like(ge)
    # d g^e / d a for a = rho, u, v, E; T = (4/3)(E - (u^2 + v^2)/2), v = 0.
    dT = {"rho": zero, "u": -4.0 / 3.0 * U_ + zero, "v": zero, "E": 4.0 / 3.0 + zero}
    Cg = {"rho": ge / R,
          "u": ge * (2.0 * cx / T_ + dlng_dT * dT["u"]),
          "v": ge * (2.0 * xi_y[None, :] / T_),
          "E": ge * dlng_dT * dT["E"]}
    Ch = {a: 0.5 * (3 - Dv) * (T_ * Cg[a] + ge * dT[a]) for a in Cg}
    Lam = {"rho": 1.0 / R + zero,
           "u": (1.0 - s) * dT["u"] / T_,
           "v": zero,
           "E": (1.0 - s) * dT["E"] / T_}
    names = ["rho", "u", "v", "E"] if Dv == 2 else ["rho", "u", "E"]
    r = len(names)
    U = np.zeros((Ny, 2, r, Nxi))
    M = np.zeros((Ny, r, 2, Nxi))
    for ia, a in enumerate(names):
        U[:, 0, ia, :] = nu[:, None] * (Cg[a] + (ge - gc) * Lam[a])
        U[:, 1, ia, :] = nu[:, None] * (Ch[a] + (he - hc) * Lam[a])
    Wb = np.broadcast_to(w[None, :], (Ny, Nxi))
    func = {"rho": (Wb, 0 * Wb),
            "u": (Wb * cx / R, 0 * Wb),
            "v": (Wb * xi_y[None, :] / R, 0 * Wb),
            "E": (Wb * ((xi_x ** 2 + xi_y ** 2)[None, :] - 2.0 * E[:, None]) / (2.0 * R),
                  Wb / (2.0 * R))}
    for ia, a in enumerate(names):
        M[:, ia, 0, :] = func[a][0]
        M[:, ia, 1, :] = func[a][1]
    return U, M


def bc_mask(Ny, xi_x):
    """Inflow rows: j = N (x = -s_inf) with xi_x > 0 and j = 0 (x = +s_inf) with
    xi_x < 0, for both fields; returned as a [Ny, 2, Nxi] boolean array."""
    Nxi = xi_x.shape[0]
    bc = np.zeros((Ny, 2, Nxi), bool)
    bc[Ny - 1, :, :] = (xi_x > 0)[None, :]
    bc[0, :, :] = (xi_x < 0)[None, :]
    return bc


class Pencil:
    """Explicit sparse pencil plus the pieces it was built from."""

    def __init__(self, wl):
        self.wl = wl
        self.Ny, self.Nxi, self.Dv = wl.Ny, wl.xi_x.shape[0], wl.Dv
        self.n = 2 * self.Ny * self.Nxi
        self.x, self.dydx, self.Dx = _grid.mapped_grid(wl.Ny, wl.L, wl.s_inf)
        self.state = base_state(wl)
        self.U, self.M = coefficients(wl, self.state)
        self.bc = bc_mask(self.Ny, wl.xi_x)
        self.r = self.U.shape[2]
        self.bdiag = (~self.bc.ravel()).astype(float)
        self._AB = None

    @property
    def A(self):
        if self._AB is None:
            self._AB = self._assemble()
        return self._AB[0]

    @property
    def B(self):
        if self._AB is None:
            self._AB = self._assemble()
        return self._AB[1]

    def _assemble(self):
        wl, Ny, Nxi, n = self.wl, self.Ny, self.Nxi, self.n
        stream = sp.kron(sp.csr_matrix(self.Dx),
                         sp.kron(sp.identity(2), sp.diags(wl.xi_x)), format="csr")
        d = (1j * wl.beta * wl.xi_y[None, None, :] + self.state["nu"][:, None, None]
             + np.zeros((Ny, 2, Nxi)))
        blocks = []
        for j in range(Ny):
            Uj = self.U[j].transpose(0, 2, 1).reshape(2 * Nxi, self.r)   # rows (f,k)
            Mj = self.M[j].reshape(self.r, 2 * Nxi)                      # cols (f,p)
            blocks.append(Uj @ Mj)
        coup = sp.block_diag(blocks, format="csr")
        A = (stream + sp.diags(d.ravel()) - coup).tocsr().astype(complex)
        bcf = self.bc.ravel()
        keep = sp.diags((~bcf).astype(float))
        A = (keep @ A + sp.diags(bcf.astype(float))).tocsr()
        A.eliminate_zeros()
        B = sp.diags((~bcf).astype(float)).tocsr().astype(complex)
        return A, B

    def dense(self):
        return self.A.toarray(), self.B.toarray()

    def apply(self, x, tau=0.0):
        """(A - tau B) x with the explicit matrices."""
        return self.A @ x - tau * (self.B @ x)

    def apply_structured(self, x, tau=0.0):
        """(A - tau B) x from the row definition without forming A (for sizes where
        the explicit matrix does not fit): streaming D_x along j per (f, k), the
        diagonal, the rank-r moment coupling per node, and identity inflow rows."""
        wl = self.wl
        X = x.reshape(self.Ny, 2, self.Nxi)
        Y = np.einsum("jm,mfk->jfk", self.Dx, X) * wl.xi_x[None, None, :]
        Y += (1j * wl.beta * wl.xi_y[None, None, :] + self.state["nu"][:, None, None]) * X
        m = np.einsum("jafk,jfk->ja", self.M, X)
        Y -= np.einsum("jfak,ja->jfk", self.U, m)
        Y -= tau * X
        Y[self.bc] = X[self.bc]
        return Y.reshape(-1)


def apply_structured_extended(P, x, tau=0.0):
    """(A - tau B) x as Pencil.apply_structured, evaluated in x87 extended
    precision (64-bit significand, unit roundoff 5.4e-20) on the FP64 tables and
    the given vector: the same row definition, rounded about 2^11 times more
    finely.  Returns complex extended-precision values."""
    wl = P.wl
    ld, cld = np.longdouble, np.clongdouble
    X = np.asarray(x).astype(cld).reshape(P.Ny, 2, P.Nxi)
    Dx = P.Dx.astype(ld)
    Y = np.einsum("jm,mfk->jfk", Dx, X) * wl.xi_x.astype(ld)[None, None, :]
    diag = (1j * wl.beta * wl.xi_y.astype(ld))[None, None, :] + P.state["nu"].astype(ld)[:, None, None]
    Y += diag.astype(cld) * X
    m = np.einsum("jafk,jfk->ja", P.M.astype(ld), X)
    Y -= np.einsum("jfak,ja->jfk", P.U.astype(ld), m)
    Y -= cld(tau) * X
    Y[P.bc] = X[P.bc]
    return Y.reshape(-1)


def structural_pattern(Ny, xi_x):
    """Structural nonzero pattern of A, built from the row definition: a non-inflow
    row (j,f,k) touches (m,f,k) for every m (streaming, D_x is dense) and every
    unknown at node j (the moment coupling reaches both fields); an inflow row
    touches only its diagonal.  Returned as a boolean scipy CSR matrix."""
    Nxi = xi_x.shape[0]
    bc = bc_mask(Ny, xi_x).ravel()
    rows, cols = [], []
    for j in range(Ny):
        for f in range(2):
            for k in range(Nxi):
                i = (2 * j + f) * Nxi + k
                if bc[i]:
                    rows.append(i)
                    cols.append(i)
                    continue
                c = set((2 * m + f) * Nxi + k for m in range(Ny))
                c.update(range(2 * j * Nxi, (2 * j + 2) * Nxi))
                rows.extend([i] * len(c))
                cols.extend(sorted(c))
    n = 2 * Ny * Nxi
    return sp.csr_matrix((np.ones(len(rows), bool), (rows, cols)), shape=(n, n))


def nnz_formula(Ny, Nxi, n_bc):
    """nnz(A) = n (Ny - 1 + 2 Nxi) - n_bc (Ny - 2 + 2 Nxi): non-inflow rows carry
    Ny - 1 streaming off-diagonals plus 2 Nxi point-block entries, inflow rows one."""
    n = 2 * Ny * Nxi
    return n * (Ny - 1 + 2 * Nxi) - n_bc * (Ny - 2 + 2 * Nxi)


def collision_nonlinear(g, h, wl):
    """Nonlinear discrete BGK relaxation nu(m) (f^e(m) - f) for f = g, h, with the
    macros m the discrete moments of (g, h) and nu = nu_inf rho T^(1-s)
    (Sec. 2.1 BGK model with collision rate P/mu; Sec. 3.3 reduced equations).
    Written with analytic operations only, so that a complex-step perturbation
    yields its exact directional derivative."""
    xi_x, xi_y, w, Dv = wl.xi_x, wl.xi_y, wl.w, wl.Dv
    rho = g @ w
    ux = (g * xi_x[None, :]) @ w / rho
    uy = (g * xi_y[None, :]) @ w / rho
    E = 0.5 * ((g * (xi_x ** 2 + xi_y ** 2)[None, :] + h) @ w) / rho
    T = (4.0 / 3.0) * (E - 0.5 * (ux ** 2 + uy ** 2))
    c2 = (xi_x[None, :] - ux[:, None]) ** 2 + (xi_y[None, :] - uy[:, None]) ** 2
    ge = rho[:, None] / (np.pi * T[:, None]) ** (0.5 * Dv) * np.exp(-c2 / T[:, None])
    he = 0.5 * (3 - Dv) * T[:, None] * ge
    nu = wl.nu_inf * rho * T ** (1.0 - wl.s_visc)
    return nu[:, None] * (ge - g), nu[:, None] * (he - h)
