"""Brute-force ray tracer through spherical shells (test reference for the
curved-atmosphere variant; shares nothing with the oracle's integrals).

The atmosphere between consecutive table nodes is cut into m thin shells of
constant index (n at the shell's mid altitude, psi linear in altitude between
nodes).  A ray goes in straight lines from sphere to sphere and is refracted
at each sphere by the vector form of Snell's law about the local radial
normal.  A virtual interface at the emission point (from n_e) and one at the
ground (into n_obs) make the discrete medium keep the ray invariant exactly,
so only the path between the spheres carries the O(1/m^2) discretisation
error, which two values of m and Richardson extrapolation remove.
"""

import math

import numpy as np

C_LIGHT = 0.299792458  # m / ns


def _refract(d, nrm, n1, n2):
    """Direction after crossing from index n1 into n2; nrm the unit normal
    pointing against d (into the medium the ray leaves).  None: total
    internal reflection."""
    cos_i = -(d[0] * nrm[0] + d[1] * nrm[1] + d[2] * nrm[2])
    eta = n1 / n2
    k = 1.0 - eta * eta * (1.0 - cos_i * cos_i)
    if k < 0.0:
        return None
    f = eta * cos_i - math.sqrt(k)
    out = [eta * d[a] + f * nrm[a] for a in range(3)]
    norm = math.sqrt(out[0] ** 2 + out[1] ** 2 + out[2] ** 2)
    return [c / norm for c in out]


def trace(R, grid, psi, h_obs, P, D, m):
    """One ray from P = (x, y, z) (z along the origin's vertical, the centre at
    (0, 0, -R)) with unit direction D = (u, v, -w).  Returns (x_g, y_g,
    u_o, v_o, T) at the sphere of altitude h_obs, or None if the ray does
    not get there."""
    def n_at(h):
        return math.sqrt(1.0 + float(np.interp(h, grid, psi)))

    x, y, z = P
    rz = R + z
    r_e = math.sqrt(x * x + y * y + rz * rz)
    h_e = r_e - R
    # shell boundaries below the emission point, top to bottom
    i = int(np.searchsorted(grid, h_e, side="right")) - 1
    cells = [(h_e, float(grid[i]))] + [(float(grid[j]), float(grid[j - 1])) for j in range(i, 0, -1)]
    bounds = [h_e]
    for top, bot in cells:
        if top == bot:
            continue
        for q in range(1, m + 1):
            bounds.append(top + (bot - top) * q / m)
    # positions relative to the centre
    p = [x, y, rz]
    d = list(D)
    n_cur = n_at(h_e)
    opt = 0.0
    r_cur = r_e
    for k in range(len(bounds) - 1):
        h_top, h_bot = bounds[k], bounds[k + 1]
        n_layer = n_at(0.5 * (h_top + h_bot))
        nrm = [p[a] / r_cur for a in range(3)]
        d = _refract(d, nrm, n_cur, n_layer)
        if d is None:
            return None
        r_next = R + h_bot
        b = p[0] * d[0] + p[1] * d[1] + p[2] * d[2]
        c0 = (r_cur - r_next) * (r_cur + r_next)
        disc = b * b - c0
        if b >= 0.0 or disc < 0.0:
            return None            # moving outward, or misses the inner sphere: turns
        t = c0 / (-b + math.sqrt(disc))
        p = [p[a] + t * d[a] for a in range(3)]
        opt += n_layer * t
        r_cur = r_next
        n_cur = n_layer
    n_obs = n_at(h_obs)
    nrm = [p[a] / r_cur for a in range(3)]
    d = _refract(d, nrm, n_cur, n_obs)
    return p[0], p[1], d[0], d[1], opt / C_LIGHT


def trace_extrapolated(R, grid, psi, h_obs, P, D, m=8):
    """Richardson extrapolation of trace() over m and 2m shells per cell."""
    a = trace(R, grid, psi, h_obs, P, D, m)
    b = trace(R, grid, psi, h_obs, P, D, 2 * m)
    if a is None or b is None:
        return None
    return tuple((4.0 * vb - va) / 3.0 for va, vb in zip(a, b))
