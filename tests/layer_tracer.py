"""Brute-force ray tracing through a stratified medium, used to pin the oracle.

Independent of the oracle's moment-table series: the ray is followed cell by
cell with Snell's invariant p = n sin(theta), and the horizontal advance and
travel time of each cell are integrated in closed form for psi = n^2 - 1
linear in altitude inside the cell:

  advance  = 2 p dz / (s_t + s_b),
  c * time = (2/3) dz (s_t^2 + s_t s_b + s_b^2) / (s_t + s_b) + 2 p^2 dz / (s_t + s_b),

with s = sqrt(1 + psi - p^2) at the cell's top and bottom.
"""

import numpy as np

C_LIGHT = 0.299792458


def trace(grid_h, grid_psi, h_e, sin_theta_e):
    """Horizontal advance [m] and c*travel-time [m] from h_e down to grid_h[0].

    grid_h: uniform node altitudes (ascending), grid_psi: psi at the nodes;
    psi is linear between nodes.  sin_theta_e: sine of the zenith angle of the
    ray at emission (the ray goes downward)."""
    psi_e = np.interp(h_e, grid_h, grid_psi)
    p = np.sqrt(1.0 + psi_e) * sin_theta_e
    i_top = np.searchsorted(grid_h, h_e, side="right") - 1
    # node list from the bottom to the emission altitude
    hs = np.concatenate([grid_h[: i_top + 1], [h_e]])
    ps = np.concatenate([grid_psi[: i_top + 1], [psi_e]])
    if hs[-1] == hs[-2]:
        hs, ps = hs[:-1], ps[:-1]
    dz = np.diff(hs)
    s = np.sqrt(1.0 + ps - p * p)
    sb, st = s[:-1], s[1:]
    adv = np.sum(2.0 * p * dz / (st + sb))
    ct = np.sum((2.0 / 3.0) * dz * (st * st + st * sb + sb * sb) / (st + sb)
                + 2.0 * p * p * dz / (st + sb))
    return adv, ct
