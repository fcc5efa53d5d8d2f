"""Post-processing of eigenvectors and base flows (test infrastructure: the CPU
definition the device kernels are checked against; nothing in the library path
imports it).

perturbation_macros -- macroscopic perturbations of a reduced-VDF perturbation
    (g_hat, h_hat) at every spatial node, from the velocity integrals that define
    them (Sec. 2.2, the integrals after the linearised BGK equations), linearised
    about the base state consistently with the operator:
        rho_hat = sum W g_hat
        u_hat   = (sum W xi_x g_hat - u rho_hat) / rho
        v_hat   =  sum W xi_y g_hat / rho                       (base v = 0)
        E_hat   = (sum W (|xi|^2 g_hat + h_hat) / 2 - E rho_hat) / rho
        T_hat   = (4/3) (E_hat - u u_hat)                (T = (4/3)(E - |u|^2/2))
    and the velocity-perturbation amplitude |U_hat| = sqrt(|u_hat|^2 + |v_hat|^2)
    of Sec. 5 (eq. Unormpert), reported divided by its maximum over the nodes
    as the paper plots it.
noneq_level -- the translational non-equilibrium level of the base flow,
    E_neq(x_j) = sqrt(sum_k W_k (g_c - g^e)^2) (Sec. 5, eq. L2norm), with the
    reduced g in place of f and g^e the reduced Maxwellian at the node's macros.
"""
import numpy as np

from . import operator as O


def perturbation_macros(wl, X):
    """X: [n] or [n, nvec] complex in the (2j + f) Nxi + k ordering.
    Returns macros [nvec, Ny, 5] (rho, u, v, E, T hats) and |U_hat| / max [nvec, Ny]."""
    st = O.base_state(wl)
    X = np.asarray(X).reshape(wl.n, -1)
    nvec = X.shape[1]
    Ny, Nxi = wl.Ny, wl.Nxi
    w, xx, xy = wl.w, wl.xi_x, wl.xi_y
    mac = np.zeros((nvec, Ny, 5), complex)
    um = np.zeros((nvec, Ny))
    for v in range(nvec):
        q = X[:, v].reshape(Ny, 2, Nxi)
        g, h = q[:, 0, :], q[:, 1, :]
        rho_h = g @ w
        mx = (g * xx[None, :]) @ w
        my = (g * xy[None, :]) @ w
        e2 = 0.5 * ((g * (xx ** 2 + xy ** 2)[None, :] + h) @ w)
        u_h = (mx - st["u"] * rho_h) / st["rho"]
        v_h = my / st["rho"] if wl.Dv == 2 else np.zeros(Ny, complex)
        E_h = (e2 - st["E"] * rho_h) / st["rho"]
        T_h = (4.0 / 3.0) * (E_h - st["u"] * u_h)
        mac[v] = np.stack([rho_h, u_h, v_h, E_h, T_h], axis=1)
        a = np.sqrt(np.abs(u_h) ** 2 + np.abs(v_h) ** 2)
        um[v] = a / a.max() if a.max() > 0 else a
    return mac, um


def noneq_level(wl):
    """E_neq at every spatial node [Ny] (zero for an EQ base flow)."""
    st = O.base_state(wl)
    d = st["gc"] - st["ge"]
    return np.sqrt((d * d) @ wl.w)
