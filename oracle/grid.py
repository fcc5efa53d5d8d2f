"""Chebyshev collocation in x with the algebraic map (Sec. 3.1).

Pinned by tests/test_oracle_pins.py: exact differentiation of polynomials of
degree <= N at the nodes, and the mapped derivative against the chain rule and a
finite difference of the map.
"""
import numpy as np


def cheb_nodes(N):
    """y_i = cos(i pi / N), i = 0..N (eq. ChebPoints)."""
    return np.cos(np.arange(N + 1) * np.pi / N)


def cheb_diff(N):
    """(N+1)x(N+1) Chebyshev derivative matrix written entry by entry from
    eqs. ChebOffDiag (off-diagonal, with c_0 = c_N = 2), ChebDiag (interior
    diagonal) and ChebBC (the two corner entries)."""
    y = cheb_nodes(N)
    c = np.ones(N + 1)
    c[0] = c[N] = 2.0
    D = np.zeros((N + 1, N + 1))
    for j in range(N + 1):
        for m in range(N + 1):
            if j != m:
                D[j, m] = (c[j] / c[m]) * (-1.0) ** (j + m) / (y[j] - y[m])
    for j in range(1, N):
        D[j, j] = -y[j] / (2.0 * (1.0 - y[j] ** 2))
    D[0, 0] = (2.0 * N * N + 1.0) / 6.0
    D[N, N] = -(2.0 * N * N + 1.0) / 6.0
    return D


def mapped_grid(Ny, L, s_inf):
    """Algebraic map x = L y / sqrt(1 + s - y^2), s = (L/s_inf)^2 (eq. Chebmapping).

    Returns (x, dy/dx, D_x) with (D_x)_ij = (dy/dx)_i (D_y)_ij.  Node j = 0 sits
    at x = +s_inf (downstream), node N at x = -s_inf (upstream)."""
    N = Ny - 1
    y = cheb_nodes(N)
    s = (L / s_inf) ** 2
    x = L * y / np.sqrt(1.0 + s - y ** 2)
    dydx = np.sqrt(1.0 + s) * L ** 2 / (L ** 2 + x ** 2) ** 1.5
    Dx = dydx[:, None] * cheb_diff(N)
    return x, dydx, Dx
