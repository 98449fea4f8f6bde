"""Esirkepov's charge-conserving current for first-order (CIC) particles,
and the EZ scheme: Esirkepov's decomposition applied to each segment of the
ZigZag split (the alternatives the paper names beside ZigZag in Sec. 2.5).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``; plain numpy, FP64,
periodic grids.

Esirkepov (2001).  A CIC particle at xi (cell units) has weight
S_a(i) = max(0, 1 - |xi_a - i|) at node i of axis a.  For a move xi0 -> xi1
the change of the node density S_x S_y S_z splits into W_x + W_y + W_z with

    W_x = dS_x (S0_y S0_z + dS_y S0_z / 2 + S0_y dS_z / 2 + dS_y dS_z / 3),

W_y and W_z cyclically, S0 = S(xi0), dS = S(xi1) - S(xi0).  Discrete
continuity then fixes the current on the x edges (i + 1/2, j, k) as the
running sum J_x(i) = J_x(i - 1) - q dx W_x(i, j, k) / (dt dV), starting from
zero below the particle's nodes (and returning to zero above them).

EZ (Steiniger et al. 2023): split the move at the ZigZag relay point, so that
each segment stays in one cell, and apply the decomposition to each segment.
For CIC shapes a segment inside one cell gives W_x = dxi_x (w_y w_z +
dxi_y dxi_z / 12) on its edges (w the bilinear weights at the segment's
mid-point), which is the ZigZag segment weight of the step: the test pins
the two against each other.
"""
from __future__ import annotations

import numpy as np


def _shape(x, lo, order=1, count=3):
    """Weights of position x (cell units) on the nodes lo .. lo + count - 1:
    CIC max(0, 1 - |x - i|) (order 1) or the quadratic B-spline (order 2)."""
    t = np.abs(x - (lo + np.arange(count)))
    if order == 1:
        return np.maximum(0.0, 1.0 - t)
    return np.where(t <= 0.5, 0.75 - t * t, np.where(t < 1.5, 0.5 * (1.5 - t) ** 2, 0.0))


def esirkepov(n, d, dt, xi0, xi1, q, J, order=1):
    """Add the current of one particle of charge q moving xi0 -> xi1 (cell
    units, |xi1 - xi0| < 1 per axis, xi0 inside the periodic box) into J
    ([3][n_z][n_y][n_x], J_a on its edges); order 1 (CIC) or 2 (b_2)."""
    xi0 = np.asarray(xi0, dtype=np.float64)
    xi1 = np.asarray(xi1, dtype=np.float64)
    if order == 1:
        lo = np.minimum(np.floor(xi0), np.floor(xi1)).astype(np.int64)
        K = 3
    else:
        lo = np.minimum(np.floor(xi0 + 0.5), np.floor(xi1 + 0.5)).astype(np.int64) - 1
        K = 4
    S0 = [_shape(xi0[a], lo[a], order, K) for a in range(3)]
    dS = [_shape(xi1[a], lo[a], order, K) - S0[a] for a in range(3)]
    dV = d[0] * d[1] * d[2]
    idx = [np.mod(lo[a] + np.arange(K), n[a]) for a in range(3)]
    for c in range(3):
        b1, b2 = (c + 1) % 3, (c + 2) % 3
        # transverse factor on the (b1, b2) node pairs
        T = (np.outer(S0[b1], S0[b2]) + 0.5 * np.outer(dS[b1], S0[b2])
             + 0.5 * np.outer(S0[b1], dS[b2]) + np.outer(dS[b1], dS[b2]) / 3.0)
        W = np.zeros((K, K, K))  # [x][y][z] over the particle's nodes
        for l in range(K):
            sl = [slice(None)] * 3
            sl[c] = l
            # T is indexed [b1][b2]; place it on the axes (b1, b2) of W
            Tc = T if b1 < b2 else T.T
            W[tuple(sl)] = dS[c][l] * Tc
        Jloc = -q * d[c] / (dt * dV) * np.cumsum(W, axis=c)
        ix, iy, iz = np.meshgrid(idx[0], idx[1], idx[2], indexing="ij")
        np.add.at(J[c], (iz, iy, ix), Jloc)
    return J


def relay(xi0, xi1):
    """ZigZag relay point per axis (Umeda et al. 2003): min(min(i0, i1) + 1,
    max(max(i0, i1), mid-point))."""
    xi0 = np.asarray(xi0, dtype=np.float64)
    xi1 = np.asarray(xi1, dtype=np.float64)
    i0, i1 = np.floor(xi0), np.floor(xi1)
    return np.minimum(np.minimum(i0, i1) + 1.0, np.maximum(np.maximum(i0, i1), 0.5 * (xi0 + xi1)))


def ez(n, d, dt, xi0, xi1, q, J):
    """EZ current: Esirkepov's decomposition on each ZigZag segment."""
    xr = relay(xi0, xi1)
    esirkepov(n, d, dt, xi0, xr, q, J)
    # the second segment starts at the relay point, which may sit on the far
    # face of the first cell; shift into the box for the node indices
    esirkepov(n, d, dt, xr, xi1, q, J)
    return J
