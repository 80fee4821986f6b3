"""Brute-force references written from the mathematics, for pinning the oracle.

Nothing here is shared with the oracle or the HIP path: the shape function is
taken from its piecewise definition and evaluated node by node over every
periodic image, time integrals are done by Gauss-Legendre quadrature, and
differences are whole-array rolls.
"""
from __future__ import annotations

import math

import numpy as np


def s2(d):
    """Quadratic B-spline: 3/4 - d^2 (|d| <= 1/2), (3/2 - |d|)^2 / 2 (1/2 <= |d| <= 3/2), else 0."""
    a = np.abs(np.asarray(d, dtype=np.float64))
    return np.where(a <= 0.5, 0.75 - a * a, np.where(a <= 1.5, 0.5 * (1.5 - a) ** 2, 0.0))


def shape_on_axis(xi, n, stag=0, periodic=True):
    """S2(xi - stag/2 - i) for every node i of an axis of n cells, summed over
    periodic images (or without images on an open axis with n + 1 nodes)."""
    if periodic:
        nodes = np.arange(n, dtype=np.float64)
        tot = np.zeros(n)
        for img in (-2, -1, 0, 1, 2):
            tot += s2(xi - 0.5 * stag - nodes - img * n)
        return tot
    nodes = np.arange(n + 1 - stag, dtype=np.float64)
    return s2(xi - 0.5 * stag - nodes)


def rho_2d(x, y, w, q, n, periodic=(True, True)):
    """Charge density on primal nodes, shape (ny_nodes, nx_nodes)."""
    out = None
    for xi, yi, wi in zip(x, y, w):
        sx = shape_on_axis(xi, n[0], 0, periodic[0])
        sy = shape_on_axis(yi, n[1], 0, periodic[1])
        term = q * wi * np.outer(sy, sx)
        out = term if out is None else out + term
    return out


def gather_2d(fields, xi, eta, n):
    """Brute-force gather on a periodic 2-D grid: sum over every node (and its
    images) of F * S2 * S2 with each component's own staggering."""
    stag = [(1, 0), (0, 1), (0, 0), (0, 1), (1, 0), (1, 1)]
    out = []
    for c in range(6):
        sx = shape_on_axis(xi, n[0], stag[c][0])
        sy = shape_on_axis(eta, n[1], stag[c][1])
        out.append(float(np.sum(fields[c] * np.outer(sy, sx))))
    return np.array(out)


GL2 = ((0.5 - 0.5 / math.sqrt(3.0), 0.5), (0.5 + 0.5 / math.sqrt(3.0), 0.5))


def esirkepov_quadrature_2d(x0, x1, w, q, vz, d, dt, n):
    """Currents of one particle moving x0 -> x1 on a periodic 2-D grid from the
    time integral of the linearly interpolated shape factors (two-point
    Gauss-Legendre, exact for the quadratic-in-t integrands), with the
    longitudinal currents obtained by running sums started far from the
    particle.  Returns Jx (dual x), Jy (dual y), Jz (primal), each (ny, nx)."""
    S0x = shape_on_axis(x0[0], n[0])
    S1x = shape_on_axis(x1[0], n[0])
    S0y = shape_on_axis(x0[1], n[1])
    S1y = shape_on_axis(x1[1], n[1])
    DSx, DSy = S1x - S0x, S1y - S0y
    Wx = np.zeros((n[1], n[0]))
    Wy = np.zeros((n[1], n[0]))
    Wz = np.zeros((n[1], n[0]))
    for t, wt in GL2:
        Sx_t = S0x + t * DSx
        Sy_t = S0y + t * DSy
        Wx += wt * np.outer(Sy_t, DSx)
        Wy += wt * np.outer(DSy, Sx_t)
        Wz += wt * np.outer(Sy_t, Sx_t)
    # running sums along the axis, starting at the node opposite the particle
    sx = (int(math.floor(x0[0])) + n[0] // 2) % n[0]
    sy = (int(math.floor(x0[1])) + n[1] // 2) % n[1]
    Jx = np.zeros((n[1], n[0]))
    Jy = np.zeros((n[1], n[0]))
    cx = -q * w * d[0] / dt
    cy = -q * w * d[1] / dt
    acc = np.zeros(n[1])
    for k in range(n[0]):
        i = (sx + k) % n[0]
        acc = acc + cx * Wx[:, i]
        Jx[:, i] = acc  # dual node i + 1/2
    acc = np.zeros(n[0])
    for k in range(n[1]):
        j = (sy + k) % n[1]
        acc = acc + cy * Wy[j, :]
        Jy[j, :] = acc
    Jz = q * w * vz * Wz
    return Jx, Jy, Jz


def div_dual_2d(Jx, Jy, d):
    """Backward-difference divergence of dual-located currents onto primal nodes."""
    return (Jx - np.roll(Jx, 1, axis=1)) / d[0] + (Jy - np.roll(Jy, 1, axis=0)) / d[1]


# ---------------------------------------------------------------------------
# 3-D (periodic) references, arrays shaped (nz, ny, nx)

STAG3 = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (0, 1, 1), (1, 0, 1), (1, 1, 0)]


def _outer3(sx, sy, sz):
    return sz[:, None, None] * sy[None, :, None] * sx[None, None, :]


def gather_3d(fields, xi, n):
    """Brute-force gather on a periodic 3-D grid: sum over every node (and its
    images) of F * S2 * S2 * S2 with each component's own staggering
    (Ex, Ey, Ez half a cell up along their own axis; Bx, By, Bz half a cell
    up along the two other axes)."""
    out = []
    for c in range(6):
        s = [shape_on_axis(xi[a], n[a], STAG3[c][a]) for a in range(3)]
        out.append(float(np.sum(fields[c] * _outer3(*s))))
    return np.array(out)


def rho_3d(xs, w, q, n):
    """Charge density on primal nodes of a periodic 3-D grid."""
    out = np.zeros((n[2], n[1], n[0]))
    for k in range(len(w)):
        s = [shape_on_axis(xs[a][k], n[a]) for a in range(3)]
        out += q * w[k] * _outer3(*s)
    return out


def esirkepov_quadrature_3d(x0, x1, w, q, d, dt, n):
    """Currents of one particle moving x0 -> x1 on a periodic 3-D grid: W_a is
    the time integral of DS_a times the linearly interpolated transverse
    shapes (two-point Gauss-Legendre, exact for the quadratic-in-t
    integrand); J_a is the running sum of -q w (d_a/dt) W_a along axis a,
    started far from the particle.  Returns [Jx, Jy, Jz], each (nz, ny, nx)."""
    S0 = [shape_on_axis(x0[a], n[a]) for a in range(3)]
    DS = [shape_on_axis(x1[a], n[a]) - S0[a] for a in range(3)]
    out = []
    for a in range(3):
        Wa = np.zeros((n[2], n[1], n[0]))
        for t, wt in GL2:
            s = [S0[b] + t * DS[b] for b in range(3)]
            s[a] = DS[a]
            Wa += wt * _outer3(*s)
        coef = -q * w * d[a] / dt
        axis = 2 - a  # array axis of grid axis a
        start = (int(math.floor(x0[a])) + n[a] // 2) % n[a]
        Ja = np.zeros_like(Wa)
        acc = np.zeros(np.delete(Wa.shape, axis))
        for k in range(n[a]):
            i = (start + k) % n[a]
            acc = acc + coef * np.take(Wa, i, axis=axis)
            idx = [slice(None)] * 3
            idx[axis] = i
            Ja[tuple(idx)] = acc
        out.append(Ja)
    return out


def div_dual_3d(J, d):
    """Backward-difference divergence of dual-located currents onto primal nodes."""
    return sum((J[a] - np.roll(J[a], 1, axis=2 - a)) / d[a] for a in range(3))


# ---------------------------------------------------------------------------
# particle merging: weighted Lloyd k-means in momentum, one crowded cell

def lloyd_cell(u, w, k, iters):
    """Weighted Lloyd iterations on momenta u (n x 3) with weights w, k
    centroids started at members floor(j n / k).  Every round assigns each
    member to its nearest centroid (squared distance, lowest index on ties)
    and moves every non-empty centroid to the weighted mean of its members,
    summed in member order.  Returns (assignment, centroids after each
    round)."""
    u = np.asarray(u, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    n = len(w)
    cen = np.array([u[(j * n) // k] for j in range(k)])
    history = []
    asg = np.zeros(n, dtype=np.int64)
    for _ in range(iters):
        d2 = ((u[:, None, :] - cen[None, :, :]) ** 2).sum(axis=2)
        asg = np.argmin(d2, axis=1)  # first minimum: lowest index on ties
        new = cen.copy()
        for j in range(k):
            sw, su = 0.0, np.zeros(3)
            for i in range(n):
                if asg[i] == j:
                    sw += w[i]
                    su = su + w[i] * u[i]
            if sw > 0.0:
                new[j] = su / sw
        cen = new
        history.append(cen.copy())
    return asg, history


def merge_pair(u, w, x, ids):
    """The two particles that replace a cluster: half its weight each, at its
    weighted mean position, with the cluster's mean Lorentz factor and total
    momentum, split symmetrically about the momentum direction."""
    u = np.asarray(u, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    W = w.sum()
    g = np.sqrt(1.0 + (u * u).sum(axis=1))
    gt = (w * g).sum() / W
    ut = np.sqrt(max(gt * gt - 1.0, 0.0))
    P = (w[:, None] * u).sum(axis=0)
    pn = np.linalg.norm(P)
    e1 = P / pn if pn > 0 else np.array([1.0, 0.0, 0.0])
    ax = int(np.argmin(np.abs(e1)))
    e2 = np.zeros(3)
    e2[ax] = 1.0
    e2 -= e2 @ e1 * e1
    e2 /= np.linalg.norm(e2)
    ct = min(pn / (W * ut), 1.0) if ut > 0 else 0.0
    st = np.sqrt(1.0 - ct * ct)
    X = (w[:, None] * np.asarray(x, dtype=np.float64)).sum(axis=0) / W
    lo = sorted(ids)[:2]
    return [(X, ut * (ct * e1 + st * e2), 0.5 * W, lo[0]),
            (X, ut * (ct * e1 - st * e2), 0.5 * W, lo[1])]
