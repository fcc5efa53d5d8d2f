"""Plain CPU Jacobi-Davidson for A x = lambda B x near a target (Sec. 4.2).

The steps are those the paper lists for its JD solve: a block-Jacobi
preconditioner of (A - sigma B) is set up once; an initial search vector is
chosen; each outer iteration solves the small projected problem for a harmonic
Ritz (Petrov) pair nearest sigma, forms its residual, accepts and deflates it
when ||r|| < tol |theta|, and otherwise solves the correction equation
approximately with preconditioned GMRES, orthogonalises the correction against
the basis and appends it; at ncv vectors the basis is restarted to its k_min
best directions.

The paper's harmonic-Ritz formula is not legible in its text; this oracle uses
harmonic Petrov extraction with test space W = orth((I - Z Z^H)(A - sigma B) V)
and deflation through a partial generalized Schur form (Q, Z, S_A, S_B), the
JDQZ scheme of Fokkema, Sleijpen and van der Vorst (1998) that extends the
method of Sleijpen and van der Vorst (1996) cited by the paper.  Small
projected problems are solved with plain library calls (triangular solve,
eigendecomposition, QR).

This JD is the CPU *baseline* (timed beside the GPU solve), not a parity
reference: every parity test compares with the result definition in eig.py
(dense QZ, or exact shift-invert Arnoldi).  Beyond the paper's steps it carries
the library's rules for returning the nev nearest eigenvalues -- guard pairs
after nev locks, and a settled-guard stop next to a nearly defective pair --
so that the two stop on the same criterion and the timed rates are comparable.
It is written for clarity, not speed.
"""
import numpy as np
import scipy.linalg as sla


def splitmix64(z):
    """SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) on a uint64 array."""
    with np.errstate(over="ignore"):
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def start_vector(n, seed, stream=0):
    """Counter-based start vector (the paper leaves it unspecified): with key = seed * 0x100000001B3 +
    stream (mod 2^64) and U(c) = 2 * (splitmix64(key + c) >> 11) * 2^-53 - 1,
    entry i is U(2i) + i U(2i+1).  The caller masks inflow entries to zero."""
    key = np.uint64((int(seed) * 0x100000001B3 + int(stream)) % (1 << 64))
    c = np.arange(2 * n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        bits = splitmix64(c + key)
    u = (bits >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    u = 2.0 * u - 1.0
    return u[0::2] + 1j * u[1::2]


def _orth(X, v, passes=2):
    """Classical Gram-Schmidt against the columns of X, repeated (CGS2)."""
    c = np.zeros(X.shape[1], complex)
    for _ in range(passes):
        h = X.conj().T @ v
        v = v - X @ h
        c += h
    return v, c


def _sorted_schur(G):
    """Schur form G U = U T with |T_11| >= |T_22| >= ... (largest first), from the
    QR factorisation of the eigenvector matrix with sorted columns."""
    mu, X = np.linalg.eig(G)
    order = np.argsort(-np.abs(mu), kind="stable")
    Uq, _ = np.linalg.qr(X[:, order])
    T = Uq.conj().T @ G @ Uq
    return Uq, T, mu[order]


def gmres(apply, b, m, rtol):
    """GMRES(m), one cycle from x0 = 0, modified Gram-Schmidt Arnoldi; stops when
    the least-squares residual is below rtol ||b||.  Returns (x, steps)."""
    beta = np.linalg.norm(b)
    if beta == 0.0:
        return np.zeros_like(b), 0
    Vk = [b / beta]
    H = np.zeros((m + 1, m), complex)
    e1 = np.zeros(m + 1, complex)
    e1[0] = beta
    y = np.zeros(0)
    steps = 0
    for j in range(m):
        w = apply(Vk[j])
        for i in range(j + 1):
            H[i, j] = np.vdot(Vk[i], w)
            w = w - H[i, j] * Vk[i]
        H[j + 1, j] = np.linalg.norm(w)
        steps = j + 1
        y, *_ = np.linalg.lstsq(H[:j + 2, :j + 1], e1[:j + 2], rcond=None)
        res = np.linalg.norm(H[:j + 2, :j + 1] @ y - e1[:j + 2])
        if res <= rtol * beta or H[j + 1, j] == 0.0:
            break
        Vk.append(w / H[j + 1, j])
    x = np.zeros_like(b)
    for i in range(steps):
        x = x + y[i] * Vk[i]
    return x, steps


def gmres_restarted(apply, b, m, rtol, max_steps):
    """Restarted GMRES(m) from x0 = 0: cycles of at most m steps, each started
    from the true residual b - apply(x), until ||b - apply(x)|| <= rtol ||b|| or
    max_steps steps in total.  Returns (x, steps)."""
    x, steps = gmres(apply, b, min(m, max_steps), rtol)
    bnorm = np.linalg.norm(b)
    while steps < max_steps:
        res = b - apply(x)
        rn = np.linalg.norm(res)
        if rn <= rtol * bnorm:
            break
        dx, st = gmres(apply, res, min(m, max_steps - steps), rtol * bnorm / rn)
        x = x + dx
        steps += max(st, 1)
    return x, steps


def jd(P, sigma, nev, tol=1e-10, m_min=6, m_max=None, gmres_m=20, inner_rtol=1e-6,
       max_it=10000, seed=0, time_limit=None, verbose=False, fix=0.01, precond=None,
       inner_max_it=None):
    """Returns dict(lam, X, resid, outer, inner, nconv).  The correction equation
    is solved by GMRES restarted every gmres_m steps, until its residual is below
    inner_rtol times the initial one or inner_max_it steps are spent (App. C sets
    a restart length, a relative tolerance and an iteration cap); by default
    inner_max_it = gmres_m, one cycle."""
    import time
    t_start = time.perf_counter()
    n = P.n
    m_max = m_max or max(30, 3 * nev)
    Bd = P.bdiag
    A = P.A.tocsr()

    def op(x, tau):
        return A @ x - tau * (Bd * x)

    if precond is None:
        raise ValueError("jd needs a preconditioner of A - sigma B (an object with solve(v))")
    K = precond
    Q = np.zeros((n, 0), complex)
    Z = np.zeros((n, 0), complex)
    Yk = np.zeros((n, 0), complex)               # K^{-1} Z
    SA = np.zeros((0, 0), complex)
    SB = np.zeros((0, 0), complex)
    V = np.zeros((n, 0), complex)
    W = np.zeros((n, 0), complex)
    R = np.zeros((0, 0), complex)
    MB = np.zeros((0, 0), complex)
    t = Bd * start_vector(n, seed)
    outer = inner = 0
    restarts = 0
    # the result is the nev eigenvalues nearest sigma, and JD locks pairs in the
    # order they converge: after nev are locked, go on until max(1, nev // 25)
    # consecutive newly locked eigenvalues were not nearer than the nev-th nearest
    # locked one (beyond it, or tied as a conjugate partner is for a real target),
    # then keep the nev nearest
    kcap = min(2 * nev, 100, 250 - m_max)
    complete = False
    guard = {"run": max(1, nev // 25), "streak": 0}
    # a guard that never reaches tol (next to a nearly defective pair the attainable
    # residual is about sqrt(u)) completes the set once it stays below 1e-6 and not
    # nearer (by a margin of sqrt(residual)) than the nev-th nearest locked
    # eigenvalue for 50 outer iterations in a row
    settle = {"count": 0, "k": -1}

    def passed_nearest():
        d = np.abs(np.diag(SA) / np.diag(SB) - sigma)
        guard["streak"] = guard["streak"] + 1 if d[-1] >= np.sort(d)[nev - 1] * (1 - 1e-12) else 0
        return guard["streak"] >= guard["run"]

    while not complete and outer < max_it:
        if time_limit is not None and time.perf_counter() - t_start > time_limit:
            break
        outer += 1
        # --- restart
        m = V.shape[1]
        if m >= m_max:
            Uq, T, _ = _sorted_schur(np.linalg.solve(R, MB))
            UL, SR = np.linalg.qr(R @ Uq)
            V = V @ Uq[:, :m_min]
            W = W @ UL[:, :m_min]
            R = SR[:m_min, :m_min]
            MB = (UL.conj().T @ MB @ Uq)[:m_min, :m_min]
            restarts += 1
        # --- expand the search space with t, the test space with (A - sigma B) v
        v, _ = _orth(np.hstack([Q, V]), t)
        v = v / np.linalg.norm(v)
        w0 = op(v, sigma)
        w, c = _orth(np.hstack([Z, W]), w0)
        rho = np.linalg.norm(w)
        w = w / rho
        nz = Z.shape[1]
        m = V.shape[1]
        Rn = np.zeros((m + 1, m + 1), complex)
        Rn[:m, :m] = R
        Rn[:m, m] = c[nz:]
        Rn[m, m] = rho
        V = np.hstack([V, v[:, None]])
        W = np.hstack([W, w[:, None]])
        R = Rn
        MB = W.conj().T @ (Bd[:, None] * V)
        # --- extraction (repeated while pairs converge)
        while True:
            Uq, T, mu = _sorted_schur(np.linalg.solve(R, MB))
            UL, SR = np.linalg.qr(R @ Uq)
            theta = sigma + 1.0 / mu[0]
            u = V @ Uq[:, 0]
            z = W @ UL[:, 0]
            r = op(u, theta)
            r = r - Z @ (Z.conj().T @ r)
            rn = np.linalg.norm(r)
            scale = abs(theta) if abs(theta) >= 1e-6 else 1.0
            if verbose:
                print(f"it {outer} nconv {Q.shape[1]} m {V.shape[1]} theta {theta:.10f} res {rn/scale:.3e}")
            if rn > tol * scale:
                break
            # lock (u, z) into the partial Schur form and deflate V, W
            Qn = np.hstack([Q, u[:, None]])
            Zn = np.hstack([Z, z[:, None]])
            Au = op(u, 0.0)
            Bu = Bd * u
            k = Q.shape[1]
            SAn = np.zeros((k + 1, k + 1), complex)
            SBn = np.zeros((k + 1, k + 1), complex)
            SAn[:k, :k], SBn[:k, :k] = SA, SB
            SAn[:, k] = Zn.conj().T @ Au
            SBn[:, k] = Zn.conj().T @ Bu
            Q, Z, SA, SB = Qn, Zn, SAn, SBn
            Yk = np.hstack([Yk, K.solve(z)[:, None]])
            MBr = UL.conj().T @ MB @ Uq
            V = V @ Uq[:, 1:]
            W = W @ UL[:, 1:]
            R = SR[1:, 1:]
            MB = MBr[1:, 1:]
            k = Q.shape[1]
            if k >= kcap or (k > nev and passed_nearest()) or (k >= nev and V.shape[1] == 0):
                complete = True
                break
            if V.shape[1] == 0:
                rn = None
                break
        if complete:
            break
        if rn is None:            # search space emptied by deflation: fresh start
            t = Bd * start_vector(n, seed, stream=outer)
            continue
        k = Q.shape[1]
        if k >= nev:
            d = np.abs(np.diag(SA) / np.diag(SB) - sigma)
            # theta may be off by about sqrt(residual) (relative) from its eigenvalue
            beyond = abs(theta - sigma) - np.sqrt(rn / scale) * scale >= np.sort(d)[nev - 1] * (1 - 1e-12)
            if rn <= 1e-6 * scale and beyond:
                settle["count"] = settle["count"] + 1 if settle["k"] == k else 1
                settle["k"] = k
            else:
                settle["count"] = 0
            if settle["count"] >= 50:
                break
        # --- correction equation, preconditioned with K, projected with [Q u], [Z z]
        Qt = np.hstack([Q, u[:, None]])
        Yt = np.hstack([Yk, K.solve(z)[:, None]])
        Ht = Qt.conj().T @ Yt
        Hlu = sla.lu_factor(Ht)

        def proj(y):
            return y - Yt @ sla.lu_solve(Hlu, Qt.conj().T @ y)

        # the shift of the correction equation stays at the target until the
        # residual is below `fix` (relative), then follows the Petrov value
        shift = theta if rn <= fix * scale else sigma

        def F(x):
            return proj(K.solve(op(x, shift)))

        rhs = -proj(K.solve(r))
        t, steps = gmres_restarted(F, rhs, gmres_m, inner_rtol, inner_max_it or gmres_m)
        inner += steps
    # eigenpairs of the upper-triangular pencil (S_A, S_B), mapped back through Q;
    # the nev nearest the target are returned
    k = Q.shape[1]
    lam = np.array([SA[i, i] / SB[i, i] for i in range(k)])
    X = np.zeros((n, k), complex)
    for i in range(k):
        s = np.zeros(k, complex)
        s[i] = 1.0
        Mx = SA - lam[i] * SB
        for p in range(i - 1, -1, -1):
            s[p] = -(Mx[p, p + 1:i + 1] @ s[p + 1:i + 1]) / Mx[p, p]
        x = Q @ s
        x = x / np.linalg.norm(x)
        imax = int(np.argmax(np.abs(x)))
        x = x * (abs(x[imax]) / x[imax])
        X[:, i] = x
    keep = _nearest_first(lam, sigma)[:nev]
    lam, X = lam[keep], X[:, keep]
    res = np.linalg.norm(A @ X - (Bd[:, None] * X) * lam[None, :], axis=0)
    res = res / np.where(np.abs(lam) < 1e-6, 1.0, np.abs(lam))
    return dict(lam=lam, X=X, resid=res, outer=outer, inner=inner, nconv=len(lam),
                restarts=restarts, seconds=time.perf_counter() - t_start)


def _nearest_first(lam, sigma):
    """Indices by |lambda - sigma|; within 1e-12 relative, Im lambda > 0 first,
    then the given order."""
    d = np.abs(np.asarray(lam) - sigma)
    keys = [(d[i], i) for i in range(len(d))]
    out = []
    for _, i in sorted(keys):
        out.append(i)
    # stable pass for ties: group within 1e-12 relative, positive imaginary first
    res, g = [], []
    for i in out:
        if g and abs(d[i] - d[g[0]]) > 1e-12 * max(d[i], d[g[0]]):
            res += sorted(g, key=lambda j: (not np.imag(lam[j]) > 0, g.index(j)))
            g = []
        g.append(i)
    res += sorted(g, key=lambda j: (not np.imag(lam[j]) > 0, g.index(j)))
    return np.array(res, dtype=int)


class LineBlockILU0:
    """Block-Jacobi ILU(0) of (A - sigma B) with contiguous row blocks in the
    velocity-major ordering (field, velocity node, spatial node) -- the ordering
    implied by the banded sparsity extract of Sec. 4.3 -- so that each block holds
    `lines` whole velocity lines (eq. bjilu with ILU(0) per block, eq. ilu with
    fill level zero).  ILU(0) is done by plain elimination restricted to the
    structural pattern of the block."""

    def __init__(self, P, sigma, lines=1):
        from .operator import structural_pattern
        Ny, Nxi = P.Ny, P.Nxi
        nl_tot = 2 * Nxi
        # permutation: velocity-major position of canonical index (j, f, k)
        j, f, k = np.meshgrid(np.arange(Ny), np.arange(2), np.arange(Nxi), indexing="ij")
        vm = ((f * Nxi + k) * Ny + j).ravel()
        self.perm = np.argsort(vm)           # perm[vm_pos] = canonical index
        C = (P.A - sigma * P.B).tocsr()[self.perm][:, self.perm].tocsr()
        S = structural_pattern(Ny, P.wl.xi_x)[self.perm][:, self.perm].tocsr()
        self.blocks = []
        start = 0
        while start < nl_tot:
            stop = min(nl_tot, start + lines)
            a, b = start * Ny, stop * Ny
            Cb = C[a:b, a:b].toarray()
            Sb = S[a:b, a:b].toarray()
            self.blocks.append((a, b, self._ilu0(Cb, Sb)))
            start = stop

    @staticmethod
    def _ilu0(a, pat):
        a = a.copy()
        nb = a.shape[0]
        for i in range(1, nb):
            for kk in np.nonzero(pat[i, :i])[0]:
                a[i, kk] /= a[kk, kk]
                cols = np.nonzero(pat[i, kk + 1:])[0] + kk + 1
                a[i, cols] -= a[i, kk] * a[kk, cols]
        return a

    def solve(self, v):
        vp = v[self.perm]
        out = np.empty_like(vp)
        for a, b, F in self.blocks:
            y = sla.solve_triangular(F, vp[a:b], lower=True, unit_diagonal=True)
            out[a:b] = sla.solve_triangular(F, y, lower=False)
        res = np.empty_like(out)
        res[self.perm] = out
        return res


class LineBlockILU0Rows:
    """The block-Jacobi ILU(0) of LineBlockILU0 (eqs. ilu and bjilu: fill level
    zero, contiguous blocks of `lines` whole velocity lines in the velocity-major
    ordering), with every block built straight from the operator rows of Sec. 2.2
    instead of from the assembled matrix, for shapes where A is too large to
    form.  Block rows and columns are (line p, node j), line l = f Nxi + k:
      same line, any nodes j, m:  xi_x,k D_x[j, m] + [j = m](i beta xi_y,k + nu_j - sigma)
      same node j, any two lines: - sum_a U[j, f, a, k] M[j, a, f', k']
      inflow rows:                 the identity row
    and the ILU(0) pattern is exactly this set of positions (the inflow rows
    keep their diagonal only).  The factors come from right-looking elimination
    restricted to the pattern, all blocks of one size at once."""

    def __init__(self, P, sigma, lines=1):
        wl = P.wl
        Ny, Nxi = P.Ny, P.Nxi
        nu = P.state["nu"]
        self.Ny, self.Nxi = Ny, Nxi
        nl_tot = 2 * Nxi
        starts = list(range(0, nl_tot, lines))
        self.blocks = []                       # (first line, line count, factors)
        by_size = {}
        for l0 in starts:
            by_size.setdefault(min(lines, nl_tot - l0), []).append(l0)
        for nlb, firsts in by_size.items():
            nb = nlb * Ny
            F = np.zeros((len(firsts), nb, nb), complex)
            pat = np.zeros((len(firsts), nb, nb), bool)
            for bi, l0 in enumerate(firsts):
                for p in range(nlb):
                    f, k = divmod(l0 + p, Nxi)
                    rp = slice(p * Ny, (p + 1) * Ny)
                    F[bi, rp, rp] = wl.xi_x[k] * P.Dx
                    F[bi, rp, rp] += np.diag(1j * wl.beta * wl.xi_y[k] + nu - sigma)
                    pat[bi, rp, rp] = True
                    for q in range(nlb):
                        fq, kq = divmod(l0 + q, Nxi)
                        c = -np.einsum("ja,ja->j", P.U[:, f, :, k], P.M[:, :, fq, kq])
                        rows = p * Ny + np.arange(Ny)
                        cols = q * Ny + np.arange(Ny)
                        F[bi, rows, cols] += c
                        pat[bi, rows, cols] = True
                    for j in range(Ny):
                        if P.bc[j, f, k]:
                            row = p * Ny + j
                            F[bi, row, :] = 0.0
                            pat[bi, row, :] = False
                            F[bi, row, row] = 1.0
                            pat[bi, row, row] = True
            for kk in range(nb - 1):
                piv = F[:, kk, kk][:, None]
                below = F[:, kk + 1:, kk] / piv * pat[:, kk + 1:, kk]
                F[:, kk + 1:, kk] = below
                F[:, kk + 1:, kk + 1:] -= pat[:, kk + 1:, kk + 1:] * (below[:, :, None] * F[:, kk, None, kk + 1:])
            for bi, l0 in enumerate(firsts):
                self.blocks.append((l0, nlb, F[bi]))
        self.blocks.sort(key=lambda t: t[0])

    def _gather(self, v, l0, nlb):
        Ny, Nxi = self.Ny, self.Nxi
        V = v.reshape(Ny, 2, Nxi)
        return np.concatenate([V[:, (l0 + p) // Nxi, (l0 + p) % Nxi] for p in range(nlb)])

    def solve(self, v):
        Ny, Nxi = self.Ny, self.Nxi
        out = np.zeros((Ny, 2, Nxi), complex)
        for l0, nlb, F in self.blocks:
            b = self._gather(v, l0, nlb)
            y = sla.solve_triangular(F, b, lower=True, unit_diagonal=True)
            x = sla.solve_triangular(F, y, lower=False)
            for p in range(nlb):
                f, k = divmod(l0 + p, Nxi)
                out[:, f, k] = x[p * Ny:(p + 1) * Ny]
        return out.reshape(-1)
