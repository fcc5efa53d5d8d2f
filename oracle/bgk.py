"""BE-BGK base-flow relaxation (Sec. 3.3), the step before the stability
operator: the reduced 1D2V BGK equations for (g, h) marched in time to a steady
shock.  Test infrastructure: the CPU definition the device solver is checked
against.

  d g/dt = nu (g^e - g) - xi_x d g/dx,  d h/dt = nu (h^e - h) - xi_x d h/dx
  (Sec. 3.3, eq. BoltzmannBGK_reduced; the right-hand side RHS(q) below it)

  * x-derivative: finite volumes on the mapped Chebyshev nodes (cell i spans
    the midpoints to its neighbours, width (x_{i+1} - x_{i-1}) / 2), interface
    values by MUSCL reconstruction upwinded on the sign of xi_x with the minmod
    limiter evaluated as minmod(a, b) = (sgn a + sgn b)/2 min(|a|, |b|) of the
    backward and forward differences (Sec. 3.3):
        xi_x >= 0: phi_{i+1/2} = phi_i     + minmod(phi_i - phi_{i-1}, phi_{i+1} - phi_i) / 2
        xi_x <  0: phi_{i+1/2} = phi_{i+1} - minmod(phi_{i+2} - phi_{i+1}, phi_{i+1} - phi_i) / 2
    and xi_x (phi_{i+1/2} - phi_{i-1/2}) / dx_i at the interior nodes.  Values
    beyond the two end nodes repeat the end node (the paper does not say).
  * collision: g^e, h^e at the node's discrete macros (rho, u, E from g and h,
    T = (4/3)(E - u^2/2), transverse velocity 0), nu = nu_inf rho T^(1 - s).
  * the two end nodes hold their initial (Rankine-Hugoniot) states: Dirichlet.
  * time: classical fourth-order Runge-Kutta with a fixed step.

Arrays are [Ny, Nxi] in the node order of the grid (node 0 at x = +s_inf).
"""
import numpy as np

from . import operator as O


def minmod(a, b):
    return 0.5 * (np.sign(a) + np.sign(b)) * np.minimum(np.abs(a), np.abs(b))


def interface_values(phi, xi_x):
    """phi_{i+1/2} for i = 0..Ny-2 with x increasing along axis 0: [Ny-1, Nxi]."""
    p = np.concatenate([phi[:1], phi, phi[-1:]], axis=0)      # p[i + 1] = phi[i]
    i = np.arange(phi.shape[0] - 1)
    ph_m, ph_0, ph_p, ph_pp = p[i], p[i + 1], p[i + 2], p[i + 3]
    left = ph_0 + 0.5 * minmod(ph_0 - ph_m, ph_p - ph_0)
    right = ph_p - 0.5 * minmod(ph_pp - ph_p, ph_p - ph_0)
    return np.where(xi_x[None, :] >= 0, left, right)


def streaming(phi, xi_x, x):
    """-xi_x d phi / dx at the interior nodes (zero rows at the two ends), for
    phi on nodes with x increasing along axis 0."""
    face = interface_values(phi, xi_x)
    dx = 0.5 * (x[2:] - x[:-2])
    out = np.zeros_like(phi)
    out[1:-1] = -xi_x[None, :] * (face[1:] - face[:-1]) / dx[:, None]
    return out


def macros(g, h, xi_x, xi_y, w):
    rho = g @ w
    u = (g * xi_x[None, :]) @ w / rho
    E = 0.5 * ((g * (xi_x ** 2 + xi_y ** 2)[None, :] + h) @ w) / rho
    T = (4.0 / 3.0) * (E - 0.5 * u ** 2)
    return rho, u, E, T


def rhs(g, h, x, xi_x, xi_y, w, Dv, nu_inf, s_visc):
    """RHS(q) on nodes with x increasing; zero at the two end nodes."""
    rho, u, E, T = macros(g, h, xi_x, xi_y, w)
    nu = nu_inf * rho * T ** (1.0 - s_visc)
    ge, he = O.equilibrium(rho, u, T, xi_x, xi_y, Dv)
    rg = nu[:, None] * (ge - g) + streaming(g, xi_x, x)
    rh = nu[:, None] * (he - h) + streaming(h, xi_x, x)
    rg[[0, -1]] = 0.0
    rh[[0, -1]] = 0.0
    return rg, rh


def relax(x, xi_x, xi_y, w, Dv, nu_inf, s_visc, g0, h0, dt, steps):
    """`steps` RK4 steps from (g0, h0); arrays and x in the grid's node order.
    Returns (g, h, max |RHS| of the final state)."""
    flip = x[0] > x[-1]
    sl = slice(None, None, -1) if flip else slice(None)
    xs, g, h = x[sl], np.array(g0[sl], float), np.array(h0[sl], float)
    args = (xs, xi_x, xi_y, w, Dv, nu_inf, s_visc)
    for _ in range(steps):
        k1 = rhs(g, h, *args)
        k2 = rhs(g + 0.5 * dt * k1[0], h + 0.5 * dt * k1[1], *args)
        k3 = rhs(g + 0.5 * dt * k2[0], h + 0.5 * dt * k2[1], *args)
        k4 = rhs(g + dt * k3[0], h + dt * k3[1], *args)
        g = g + (dt / 6.0) * (k1[0] + 2 * k2[0] + 2 * k3[0] + k4[0])
        h = h + (dt / 6.0) * (k1[1] + 2 * k2[1] + 2 * k3[1] + k4[1])
    r = rhs(g, h, *args)
    res = max(np.abs(r[0]).max(), np.abs(r[1]).max())
    return g[sl], h[sl], res
