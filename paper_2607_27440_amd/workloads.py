"""Seeded synthetic inputs for the kLST shock-stability path.

This module produces the *inputs* of the method -- a velocity node table and a
base flow sampled on the spatial nodes -- and nothing of the method itself: no
Chebyshev differentiation, no linearisation coefficients, no moment functionals
and no operator.  It stands in for the paper's base-flow producer (the BE-BGK
solver of Sec. 3.3), which the paper says generates its physical node positions
with the same algebraic map as the stability operator (Sec. 3.3, last
paragraphs); this module therefore carries its own copy of that node placement
(Sec. 3.1, eqs. ChebPoints and Chebmapping) so that it can sample profiles at
the nodes.  It imports neither the oracle nor the native library, so both sides
of every parity test consume exactly the same arrays.

Units follow Sec. 2.2: velocities in u_ref = sqrt(2 R T_inf), temperature in
T_inf, density in rho_inf, length in upstream mean free paths.

Workload recipe (the paper's BE-BGK base flows are not available):
  * Rankine-Hugoniot states for gamma = 5/3 (Sec. 2.1, the jump relations).
  * Weight w(x) = (1 + tanh(2x/Delta))/2, whose maximum slope 1/Delta matches the
    shock-thickness definition (Sec. 2.1, eq. ShockThickness).
  * "maxwellian" base: rho, u, T each blended with w (the paper's EQ case).
  * "bimodal" base: Mott-Smith mix g_c = (1-w) g_inf + w g_1 of the two
    Rankine-Hugoniot Maxwellians, same for h (the paper's NONEQ case, Sec. 5).
  * Velocity table: tensor-product trapezoid rule Q_x x Q_y on [-a, a]^2, or, for
    the shapes of the paper's benchmark tables (Sec. 4.3), the Q x Q tensor
    Gauss-Hermite rule of Sec. 3.2 converted to integrate plain functions.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

GAMMA = 5.0 / 3.0
#: Hard-sphere collision rate at the upstream state in mean-free-path units,
#: nu_inf = 8 / (5 sqrt(pi)) (mean free path definition of Sec. 2.1 with delta = 5).
NU_INF_HS = 8.0 / (5.0 * math.sqrt(math.pi))


@dataclasses.dataclass
class Workload:
    """One generalized-eigenproblem instance: grid, velocity table, base flow."""
    name: str
    Ny: int
    L: float
    s_inf: float
    Qx: int
    Qy: int
    vmax: float
    xi_x: np.ndarray          # [Nxi]
    xi_y: np.ndarray          # [Nxi]
    w: np.ndarray             # [Nxi] quadrature weights
    Dv: int                   # resolved velocity dimensions (2, or 1 with xi_y == 0)
    mode: int                 # 0 = EQ (macros given), 1 = NONEQ (VDF given)
    rho: Optional[np.ndarray]  # [Ny] EQ macros
    u: Optional[np.ndarray]
    T: Optional[np.ndarray]
    g_c: Optional[np.ndarray]  # [Ny, Nxi] NONEQ base VDFs
    h_c: Optional[np.ndarray]
    s_visc: float             # viscosity exponent, mu ~ T^s
    nu_inf: float             # upstream collision rate
    beta: float               # transverse wavenumber
    sigma: complex            # target, in lambda = i*omega space
    nev: int
    mach: float
    delta: float
    x: np.ndarray             # physical node positions (for reference / plots)

    @property
    def Nxi(self) -> int:
        return int(self.xi_x.shape[0])

    @property
    def n(self) -> int:
        return 2 * self.Ny * self.Nxi


def rankine_hugoniot(mach: float, gamma: float = GAMMA):
    """Downstream (rho1, u1, T1) and upstream speed u_inf for a normal shock.

    Upstream state is rho = T = 1; speeds are in units of sqrt(2 R T_inf), so the
    upstream sound speed is sqrt(gamma/2)."""
    m2 = mach * mach
    rho1 = (gamma + 1.0) * m2 / ((gamma - 1.0) * m2 + 2.0)
    p1 = 1.0 + 2.0 * gamma / (gamma + 1.0) * (m2 - 1.0)
    T1 = p1 / rho1
    u_inf = mach * math.sqrt(gamma / 2.0)
    return rho1, u_inf / rho1, T1, u_inf


def velocity_range(mach: float) -> float:
    """Half-width a of the velocity box: clamp(round(u_inf + 3 sqrt(T1)), 5, 10)."""
    _, _, T1, u_inf = rankine_hugoniot(mach)
    return float(min(max(round(u_inf + 3.0 * math.sqrt(T1)), 5), 10))


def trapezoid_table(Qx: int, Qy: int, a: float, Dv: int = 2):
    """Tensor-product trapezoid nodes/weights on [-a, a]^Dv, flattened p = ix*Qy + iy."""
    def line(Q):
        if Q == 1:
            return np.zeros(1), np.ones(1)
        z = np.linspace(-a, a, Q)
        z = 0.5 * (z - z[::-1])          # exactly symmetric about 0 (linspace is not, by an ulp)
        h = 2.0 * a / (Q - 1)
        wt = np.full(Q, h)
        wt[0] = wt[-1] = 0.5 * h
        return z, wt
    zx, wx = line(Qx)
    if Dv == 1:
        return zx.copy(), np.zeros(Qx), wx.copy()
    zy, wy = line(Qy)
    XX, YY = np.meshgrid(zx, zy, indexing="ij")
    WW = np.outer(wx, wy)
    return XX.ravel().copy(), YY.ravel().copy(), WW.ravel().copy()


def gauss_hermite_table(Q: int, scale: float = 1.0, Dv: int = 2):
    """Q x Q tensor Gauss-Hermite nodes/weights for integrating plain functions.

    Sec. 3.2 gives the rule for integrals of f(x) exp(-x^2); a base VDF is
    integrated as it stands, so each weight carries exp(x_i^2), and the nodes are
    stretched by `scale` (the paper prints neither conversion).  Flattened
    p = ix*Q + iy like the trapezoid table."""
    z, wz = np.polynomial.hermite.hermgauss(Q)
    z = scale * z
    wz = scale * wz * np.exp((z / scale) ** 2)
    if Dv == 1:
        return z.copy(), np.zeros(Q), wz.copy()
    XX, YY = np.meshgrid(z, z, indexing="ij")
    return XX.ravel().copy(), YY.ravel().copy(), np.outer(wz, wz).ravel().copy()


def gauss_hermite_scale(Q: int, mach: float) -> float:
    """Node stretch so that the Q-point rule reaches the velocity box a(M) of the
    trapezoid tables, and never shrinks below the free-stream thermal scale 1."""
    zmax = float(np.max(np.polynomial.hermite.hermgauss(Q)[0]))
    return max(1.0, velocity_range(mach) / zmax)


def node_positions(Ny: int, L: float, s_inf: float) -> np.ndarray:
    """Physical positions of the mapped Chebyshev-Gauss-Lobatto nodes (base-flow side)."""
    N = Ny - 1
    yc = np.cos(np.pi * np.arange(Ny) / N)
    s = (L / s_inf) ** 2
    return L * yc / np.sqrt(1.0 + s - yc * yc)


def _maxwell_vdf(rho, u, T, xi_x, xi_y, Dv):
    """Reduced Maxwellian pair (g, h) of a base-flow state (the producer's own)."""
    c2 = (xi_x[None, :] - u[:, None]) ** 2 + xi_y[None, :] ** 2
    g = rho[:, None] / (np.pi * T[:, None]) ** (0.5 * Dv) * np.exp(-c2 / T[:, None])
    return g, 0.5 * (3 - Dv) * T[:, None] * g


def make_workload(name: str, *, mach: float, Ny: int, Qx: int, Qy: int, beta: float,
                  sigma: complex, nev: int, base: str, delta: float,
                  s_visc: float = 0.5, nu_inf: float = NU_INF_HS, Dv: int = 2,
                  s_inf: Optional[float] = None, L: Optional[float] = None,
                  vmax: Optional[float] = None, velocity: str = "trapezoid") -> Workload:
    a = velocity_range(mach) if vmax is None else vmax
    s_inf = 5.0 * delta if s_inf is None else s_inf
    L = delta if L is None else L
    if velocity == "trapezoid":
        xi_x, xi_y, w = trapezoid_table(Qx, Qy, a, Dv)
    elif velocity == "gauss_hermite":
        if Qx != Qy:
            raise ValueError("the Gauss-Hermite table is Q x Q")
        xi_x, xi_y, w = gauss_hermite_table(Qx, gauss_hermite_scale(Qx, mach), Dv)
        a = float(np.max(xi_x))
    else:
        raise ValueError(velocity)
    x = node_positions(Ny, L, s_inf)
    wgt = 0.5 * (1.0 + np.tanh(2.0 * x / delta))      # 0 upstream (x<0), 1 downstream
    rho1, u1, T1, u_inf = rankine_hugoniot(mach)
    rho = rho_b = 1.0 + wgt * (rho1 - 1.0)
    u = u_inf + wgt * (u1 - u_inf)
    T = 1.0 + wgt * (T1 - 1.0)
    g_c = h_c = None
    if base == "maxwellian":
        mode = 0
    elif base == "bimodal":
        mode = 1
        one = np.ones(Ny)
        g0, h0 = _maxwell_vdf(one, one * u_inf, one, xi_x, xi_y, Dv)
        g1, h1 = _maxwell_vdf(one * rho1, one * u1, one * T1, xi_x, xi_y, Dv)
        g_c = (1.0 - wgt)[:, None] * g0 + wgt[:, None] * g1
        h_c = (1.0 - wgt)[:, None] * h0 + wgt[:, None] * h1
        rho = u = T = None
    else:
        raise ValueError(base)
    del rho_b
    return Workload(name=name, Ny=Ny, L=float(L), s_inf=float(s_inf), Qx=Qx, Qy=Qy,
                    vmax=float(a), xi_x=xi_x, xi_y=xi_y, w=w, Dv=Dv, mode=mode,
                    rho=rho, u=u, T=T, g_c=g_c, h_c=h_c, s_visc=float(s_visc),
                    nu_inf=float(nu_inf), beta=float(beta), sigma=complex(sigma),
                    nev=int(nev), mach=float(mach), delta=float(delta), x=x)


def config1() -> Workload:
    """M=1.2 argon shock, Maxwellian base, Ny=24, 4x4 velocities on [-5,5], n=768.

    Collision rate constant in temperature (s = 1): nu = nu_inf * rho."""
    return make_workload("c1_m1.2_ny24_nxi16", mach=1.2, Ny=24, Qx=4, Qy=4, beta=0.5,
                         sigma=0.0, nev=10, base="maxwellian", delta=2.0, s_visc=1.0,
                         s_inf=10.0, L=2.0)


def config2() -> Workload:
    """M=3 bimodal shock, Ny=64, 12x8 velocities on [-8,8], n=12,288, 20 nearest 0.05i."""
    delta = float(np.random.default_rng(2).uniform(2.0, 4.0))
    return make_workload("c2_m3_ny64_nxi96", mach=3.0, Ny=64, Qx=12, Qy=8, beta=0.5,
                         sigma=0.05j, nev=20, base="bimodal", delta=delta)


def config3() -> Workload:
    """M=4 bimodal shock, Ny=96, 61x24 velocities on [-10,10], n=281,088, 10 nearest 0."""
    delta = float(np.random.default_rng(3).uniform(2.0, 4.0))
    return make_workload("c3_m4_ny96_nxi1464", mach=4.0, Ny=96, Qx=61, Qy=24, beta=0.5,
                         sigma=0.0, nev=10, base="bimodal", delta=delta)


def paper_benchmark(Q: int = 20, Ny: int = 81) -> Workload:
    """Shape of the paper's benchmark cases (Sec. 4.3): M=1.2, N = 80 (Ny = 81),
    Q x Q Gauss-Hermite velocities, beta = 16, 50 eigenvalues nearest 1e-2.

    n = 2 Ny Q^2: 64,800 / 93,312 / 165,888 for Q = 20 / 24 / 32.  The BE-BGK base
    flow is replaced by the Mott-Smith bimodal mix with Delta ~ U(2, 4), seed 20 + Q."""
    delta = float(np.random.default_rng(20 + Q).uniform(2.0, 4.0))
    return make_workload(f"pb_m1.2_ny{Ny}_gh{Q}", mach=1.2, Ny=Ny, Qx=Q, Qy=Q, beta=16.0,
                         sigma=1e-2, nev=50, base="bimodal", delta=delta,
                         velocity="gauss_hermite")


def paper_mach4(Q: int = 48, Ny: int = 61, nev: int = 10) -> Workload:
    """Shape of the paper's Mach 4 production run (Sec. 4.4): Ny = 61, Q = 48
    Gauss-Hermite (n = 281,088), bimodal base with Delta ~ U(2, 4), seed 48,
    beta = 0.5, the eigenvalues nearest 0 (the paper does not state nev)."""
    delta = float(np.random.default_rng(48).uniform(2.0, 4.0))
    return make_workload(f"m4_ny{Ny}_gh{Q}", mach=4.0, Ny=Ny, Qx=Q, Qy=Q, beta=0.5,
                         sigma=0.0, nev=nev, base="bimodal", delta=delta,
                         velocity="gauss_hermite")


#: velocity counts of the batched sweep and their tensor factorisation Q_x x Q_y
_SWEEP_NXI = {16: (4, 4), 32: (8, 4), 64: (8, 8), 128: (16, 8)}


def sweep(seed: int = 4, count: int = 64, nev: int = 8):
    """Batched-sweep draws: Ny in {24,32,48,64}, Nxi in {16,32,64,128}, beta~U(0.1,2),
    Mach~U(1.2,4), Maxwellian or bimodal base with probability 1/2, Delta~U(2,4)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        Ny = int(rng.choice([24, 32, 48, 64]))
        Nxi = int(rng.choice([16, 32, 64, 128]))
        beta = float(rng.uniform(0.1, 2.0))
        mach = float(rng.uniform(1.2, 4.0))
        base = "maxwellian" if rng.uniform() < 0.5 else "bimodal"
        delta = float(rng.uniform(2.0, 4.0))
        Qx, Qy = _SWEEP_NXI[Nxi]
        out.append(make_workload(f"sweep{seed}_{i}", mach=mach, Ny=Ny, Qx=Qx, Qy=Qy,
                                 beta=beta, sigma=0.0, nev=nev, base=base, delta=delta))
    return out


def bgk_start(wl: Workload):
    """Initial state (g, h) [Ny, Nxi] of the base-flow relaxation: the Mott-Smith
    mix of the two Rankine-Hugoniot Maxwellians, with the two end nodes set to
    those Maxwellians exactly (node 0 downstream, node Ny-1 upstream)."""
    one = np.ones(wl.Ny)
    rho1, u1, T1, u_inf = rankine_hugoniot(wl.mach)
    g0, h0 = _maxwell_vdf(one, one * u_inf, one, wl.xi_x, wl.xi_y, wl.Dv)
    g1, h1 = _maxwell_vdf(one * rho1, one * u1, one * T1, wl.xi_x, wl.xi_y, wl.Dv)
    wgt = 0.5 * (1.0 + np.tanh(2.0 * wl.x / wl.delta))[:, None]
    g = (1.0 - wgt) * g0 + wgt * g1
    h = (1.0 - wgt) * h0 + wgt * h1
    g[0], h[0] = g1[0], h1[0]
    g[-1], h[-1] = g0[-1], h0[-1]
    return g, h


def bgk_start_from_profile(wl: Workload, rho, u, T):
    """Initial state (g, h) [Ny, Nxi] of the base-flow relaxation from a shock
    profile given at the nodes (rho, u, T normalised by the upstream state, as
    the continuum structure of Sec. 2.1 returns them): the local Maxwellians, with
    the two end nodes set to the Rankine-Hugoniot Maxwellians exactly."""
    rho1, u1, T1, u_inf = rankine_hugoniot(wl.mach)
    g, h = _maxwell_vdf(np.asarray(rho, float), np.asarray(u, float) * u_inf, np.asarray(T, float),
                        wl.xi_x, wl.xi_y, wl.Dv)
    one = np.ones(1)
    g1, h1 = _maxwell_vdf(one * rho1, one * u1, one * T1, wl.xi_x, wl.xi_y, wl.Dv)
    gi, hi = _maxwell_vdf(one, one * u_inf, one, wl.xi_x, wl.xi_y, wl.Dv)
    g[0], h[0] = g1[0], h1[0]
    g[-1], h[-1] = gi[0], hi[0]
    return g, h


def bgk_dt(wl: Workload, cfl: float = 0.4) -> float:
    """Time step of the relaxation: cfl x the smallest interior cell width
    (x_{i+1} - x_{i-1}) / 2 over the largest |xi_x|."""
    x = np.sort(wl.x)
    return float(cfl * np.min(0.5 * (x[2:] - x[:-2])) / np.max(np.abs(wl.xi_x)))


def random_vector(n: int, seed: int) -> np.ndarray:
    """Seeded complex test vector, uniform in [-1,1] for real and imaginary parts."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)
