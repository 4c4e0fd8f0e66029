"""Chebyshev-in-time coefficients of a prescribed exterior state for the
library (test helper: input preparation only)."""
import numpy as np


def chebyshev_coefficients(g, X, t_a, t_b, nt, nfields=1):
    """[nfields][E_bdy][Np][nt] coefficients of g(x, y, t, field) at the
    points X [E_bdy][Np][2], interpolated at nt Chebyshev points of
    [t_a, t_b] in tau = (2t - t_a - t_b) / (t_b - t_a)."""
    k = np.arange(nt)
    tau = np.cos(np.pi * (k + 0.5) / nt)
    ts = 0.5 * (t_a + t_b) + 0.5 * (t_b - t_a) * tau
    out = []
    for f in range(nfields):
        vals = np.stack([np.asarray(g(X[..., 0], X[..., 1], t, f), dtype=np.float64) for t in ts])
        c = np.polynomial.chebyshev.chebfit(tau, vals.reshape(nt, -1), nt - 1)   # [nt, n]
        out.append(c.T.reshape(X.shape[0], X.shape[1], nt))
    return np.stack(out)
