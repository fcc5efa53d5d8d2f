"""Micro-velocity quadrature (Sec. 3.2).

Gauss-Hermite nodes and weights by the Golub-Welsch construction: eigenvalues of
the symmetric tridiagonal Jacobi matrix of the monic Hermite recurrence
(off-diagonal sqrt(k/2)) are the nodes, and sqrt(pi) times the squared first
eigenvector components are the weights.  Pinned against the exactness property
stated in Sec. 3.2 (polynomials up to degree 2n-1 against exp(-x^2)).
"""
import numpy as np


def gauss_hermite(n):
    k = np.arange(1, n)
    off = np.sqrt(k / 2.0)
    J = np.diag(off, 1) + np.diag(off, -1)
    x, V = np.linalg.eigh(J)
    w = np.sqrt(np.pi) * V[0, :] ** 2
    return x, w


def gauss_hermite_plain(n, scale=1.0):
    """Nodes/weights for integrating a plain function f(x) dx (not f e^{-x^2}):
    W_i exp(x_i^2), with nodes stretched by `scale` (reading of Sec. 3.2: the
    paper does not print this conversion)."""
    x, w = gauss_hermite(n)
    return scale * x, scale * w * np.exp(x ** 2)


def tensor_table(zx, wx, zy, wy):
    """Flattened 2-D table p = ix*Qy + iy of a tensor-product rule."""
    XX, YY = np.meshgrid(zx, zy, indexing="ij")
    return XX.ravel().copy(), YY.ravel().copy(), np.outer(wx, wy).ravel().copy()
