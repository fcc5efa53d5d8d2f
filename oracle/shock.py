"""Continuum (Navier-Stokes) normal-shock structure of Gilbarg and Paolucci
(Sec. 2.1, eq. GB1DShockeqn), the start profile of the BE-BGK relaxation and
the source of the shock thickness Delta (eq. ShockThickness).

With m = rho u (mass flux), P = p + rho u^2 (momentum flux) and E = h + u^2/2
(total enthalpy), the normalised velocity and temperature are Omega = m u / P
and theta = m^2 R T / P^2 (the paper prints theta = (m/P) T; a dimensionless
temperature needs the square), and the shock strength is alpha = 2 E m^2/P^2 - 1.
Steady 1-D Navier-Stokes with viscous stress (4/3) mu u' and heat flux
kappa T', kappa = c_p mu / Pr, in z = x / l_inf (l_inf the upstream mean free
path of Sec. 2.1) reads

    (4/3) mu_h dOmega/dz           = Omega + theta/Omega - 1,
    (gamma mu_h / Pr) dtheta/dz    = theta - g [(1 - Omega)^2 + alpha],   g = (gamma - 1)/2,

with mu_h = mu / (m l_inf) = mu_h_inf (theta/theta_inf)^s and
mu_h_inf = (delta/16) sqrt(2 pi / gamma) / M_inf.  For gamma = 5/3 and
Pr = 2/3 these are the printed equations (the ratio of the two gives the
printed 8/15 in dtheta/dOmega), with beta / M_inf = mu_h_inf and
M_bar_inf = 3 M_inf / 4; the paper sets Pr = 1 for its G&P flows (Sec. 5),
which changes only the factor gamma / Pr.

The two end states are the zeros of both right-hand sides, the Rankine-Hugoniot
states.  The downstream state is a saddle: the shock is its separatrix, traced
here in the phase plane, dtheta/dOmega = (4 Pr / (3 gamma)) Omega (theta - g[.])
/ (Omega^2 - Omega + theta), from the downstream state toward the upstream one
(the direction the paper integrates), and z(Omega) by quadrature of
dz/dOmega = (4/3) mu_h / (Omega + theta/Omega - 1).
"""
import numpy as np
from scipy.integrate import solve_ivp


class GPShock:
    def __init__(self, mach, gamma=5.0 / 3.0, Pr=1.0, s_visc=0.5, delta=5.0):
        self.mach, self.gamma, self.Pr, self.s, self.delta = mach, gamma, Pr, s_visc, delta
        g = 0.5 * (gamma - 1.0)
        self.g = g
        # upstream state in units rho_inf = 1, R T_inf = 1 (p_inf = 1), u_inf = M sqrt(gamma)
        u0 = mach * np.sqrt(gamma)
        m = u0
        P = 1.0 + u0 ** 2
        E = gamma / (gamma - 1.0) + 0.5 * u0 ** 2
        self.m, self.P, self.E = m, P, E
        self.alpha = 2.0 * E * m ** 2 / P ** 2 - 1.0
        self.Om_inf, self.th_inf = m * u0 / P, m ** 2 / P ** 2
        # the other zero of both right-hand sides: (1 + g) W^2 - (1 + 2 g) W + g (1 + alpha) = 0
        a, b, c = 1.0 + g, -(1.0 + 2.0 * g), g * (1.0 + self.alpha)
        disc = np.sqrt(b * b - 4 * a * c)
        roots = np.array([(-b - disc) / (2 * a), (-b + disc) / (2 * a)])
        self.Om_1 = roots[np.argmin(np.abs(roots - self.Om_inf)) ^ 1]
        self.th_1 = self.Om_1 * (1.0 - self.Om_1)
        self.mu_inf = (delta / 16.0) * np.sqrt(2.0 * np.pi / gamma) / mach
        self._trace()

    # right-hand sides in z
    def mu_h(self, th):
        return self.mu_inf * (th / self.th_inf) ** self.s

    def dOm_dz(self, Om, th):
        return (Om + th / Om - 1.0) / (4.0 / 3.0 * self.mu_h(th))

    def dth_dz(self, Om, th):
        return (th - self.g * ((1.0 - Om) ** 2 + self.alpha)) / (self.gamma * self.mu_h(th) / self.Pr)

    def _slope(self, Om, th):
        c = 4.0 * self.Pr / (3.0 * self.gamma)
        return c * Om * (th - self.g * ((1.0 - Om) ** 2 + self.alpha)) / (Om * Om - Om + th)

    def _trace(self):
        O1, t1, g = self.Om_1, self.th_1, self.g
        c = 4.0 * self.Pr / (3.0 * self.gamma)
        # separatrix slopes at the downstream saddle: k^2 + (2 O1 - 1 - c O1) k - 2 c g O1 (1 - O1) = 0;
        # the shock leaves it with theta falling as Omega rises toward the upstream state
        B = 2 * O1 - 1 - c * O1
        C = -2 * c * g * O1 * (1 - O1)
        ks = np.roots([1.0, B, C]).real
        k = ks[ks < 0][0] if np.any(ks < 0) else ks.min()
        span = self.Om_inf - O1
        eps = 1e-10 * span
        sol = solve_ivp(lambda O, t: [self._slope(O, t[0])], (O1 + eps, self.Om_inf - 1e-9 * span),
                        [t1 + k * eps], method="DOP853", rtol=1e-12, atol=1e-15, dense_output=True)
        self.sol = sol
        self.Om_lo, self.Om_hi = O1 + eps, self.Om_inf - 1e-9 * span
        # steepest point: max |dOmega/dz| along the separatrix
        Om = np.linspace(self.Om_lo, self.Om_hi, 20001)
        th = sol.sol(Om)[0]
        w = np.abs(self.dOm_dz(Om, th))
        i = int(np.argmax(w))
        from scipy.optimize import minimize_scalar
        lo, hi = Om[max(0, i - 1)], Om[min(len(Om) - 1, i + 1)]
        r = minimize_scalar(lambda o: -abs(self.dOm_dz(o, sol.sol(o)[0])), bounds=(lo, hi), method="bounded",
                            options={"xatol": 1e-14 * span})
        self.Om_star = r.x
        self.max_slope = -r.fun
        self.thickness = span / self.max_slope        # Delta / l_inf (eq. ShockThickness)

    def theta_of_omega(self, Om):
        return self.sol.sol(Om)[0]

    def _z_dense(self):
        """z(Omega) from the steepest point to both ends, as dense outputs."""
        if not hasattr(self, "_zlo"):
            f = lambda o, z: [4.0 / 3.0 * self.mu_h(self.sol.sol(o)[0]) / (o + self.sol.sol(o)[0] / o - 1.0)]
            kw = dict(method="DOP853", rtol=1e-11, atol=1e-13, dense_output=True)
            self._zhi = solve_ivp(f, (self.Om_star, self.Om_hi), [0.0], **kw).sol
            self._zlo = solve_ivp(f, (self.Om_star, self.Om_lo), [0.0], **kw).sol
        return self._zlo, self._zhi

    def z_of_omega(self, Om):
        """z(Omega) with z = 0 at the steepest point, by quadrature of dz/dOmega."""
        lo, hi = self._z_dense()
        Om = np.atleast_1d(np.asarray(Om, float))
        return np.array([(hi if o >= self.Om_star else lo)(o)[0] for o in Om])

    def profile(self, z):
        """(rho / rho_inf, u / u_inf, T / T_inf) at positions z = x / l_inf
        measured from the steepest point (upstream at negative z), from the
        separatrix and z(Omega) inverted by bisection."""
        z = np.atleast_1d(np.asarray(z, float))
        Om = np.empty_like(z)
        for i, zz in enumerate(z):
            lo, hi = self.Om_lo, self.Om_hi        # z(Omega) decreases from +inf (downstream) to -inf
            for _ in range(200):
                mid = 0.5 * (lo + hi)
                if self.z_of_omega(mid)[0] > zz:
                    lo = mid
                else:
                    hi = mid
                if hi - lo <= 1e-13 * (self.Om_hi - self.Om_lo):
                    break
            Om[i] = 0.5 * (lo + hi)
        th = self.theta_of_omega(Om)
        u = Om / self.Om_inf
        return 1.0 / u, u, th / self.th_inf
