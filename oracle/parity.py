"""Eigenpair matching rule used by the parity tests.

Each computed eigenvalue is matched greedily (nearest first) to a distinct
reference eigenvalue from a pool of the reference's nearest ones; the relative
error e_i = |lambda_i - lambda_ref| / |lambda_ref| must be below `tol`, or, for an
eigenvalue whose conditioning limits the attainable accuracy, below
10 kappa_i u ||A||_1 / |lambda_i| (kappa from left/right reference vectors).  The
computed set may not skip a reference eigenvalue nearer the target than the
farthest computed one, except within `tie` relative distance (clusters and
conjugate pairs equidistant from a real target).
"""
import numpy as np

U_ROUND = 2.0 ** -53


def match(lam, ref, kappa=None, normA=None, sigma=0.0, tol=1e-10, tie=1e-8):
    lam = np.asarray(lam)
    ref = np.asarray(ref)
    used = np.zeros(len(ref), bool)
    out = []
    order = np.argsort(np.abs(lam - sigma))
    for i in order:
        d = np.abs(ref - lam[i])
        d[used] = np.inf
        j = int(np.argmin(d))
        used[j] = True
        e = abs(lam[i] - ref[j]) / abs(ref[j])
        bound = tol
        if kappa is not None and normA is not None:
            bound = max(tol, 10 * kappa[j] * U_ROUND * normA / abs(ref[j]))
        out.append(dict(i=int(i), j=j, err=e, bound=bound, ok=bool(e <= bound)))
    far = max(np.abs(lam - sigma)) if len(lam) else 0.0
    skipped = [int(j) for j in range(len(ref))
               if not used[j] and np.abs(ref[j] - sigma) < far * (1 - tie)]
    return out, skipped
