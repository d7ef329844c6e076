"""Seeded synthetic inputs: atmospheres, telescope layouts and track segments.

This module produces *inputs only*. It holds none of the Cherenkov
generation / propagation arithmetic; both the HIP library and the CPU
oracle consume what it returns.

The paper measures on CTA production gamma showers from CORSIKA (sec. 3.2,
sec. 5.2: 2500 showers, CTA standard parameters).  Those input cards,
atmospheric profiles and array layouts are not available, so seeded
stand-ins with the same structure are generated here:

* segments  - charged-particle track steps (sec. 2 / App. A: each particle
  track is cut into steps and Cherenkov light is computed per step); start
  altitude drawn from a Gaisser-Hillas longitudinal profile, lateral offset
  exponential around the shower axis, direction uniform in a cone around the
  axis, total energy and step length log-uniform;
* atmosphere - tabulated n-1 versus altitude (sec. 3.3.1 atmospheric
  tables; sec. 2 external profiles), exponential or layered exponential;
* telescopes - fiducial spheres on the ground (sec. 2).

Frame: x, y horizontal [m], h altitude [m].  Directions are stored as
(u, v, w) = (dx/ds, dy/ds, -dh/ds), so w > 0 means downward.
Units: m, ns, MeV.
"""

from __future__ import annotations

import dataclasses
import math
import os
from concurrent.futures import ThreadPoolExecutor
from typing import Callable, List, Optional, Sequence

import numpy as np

C_LIGHT_M_PER_NS = 0.299792458
# vertical-depth normalisation of the synthetic atmospheres: density is taken
# proportional to n-1 with n-1 = 2.9e-4 <-> rho = 1.225e-3 g/cm^3 at sea level
ETA_SEA = 2.9e-4
RHO_SEA_G_CM3 = 1.225e-3
PTYPE_ELECTRON = 0
PTYPE_MUON = 1
TOP_OF_ATMOSPHERE_M = 100_000.0
GH_LAMBDA_G_CM2 = 70.0
METHOD_SEED = 0x0000000000014927


# ----------------------------------------------------------------------------
# atmospheres
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Atmosphere:
    alt: np.ndarray   # [m], strictly increasing
    eta: np.ndarray   # n - 1 >= 0
    obs_level: float  # [m]

    def vertical_depth(self) -> np.ndarray:
        """Vertical depth X(h) [g/cm^2] at each tabulated altitude.

        Density is taken as eta * RHO_SEA/ETA_SEA and integrated from the top of
        the table downward, treating eta as log-linear between nodes (exact for
        the exponential profiles used here)."""
        a, e = self.alt, self.eta
        dz_cm = np.diff(a) * 100.0
        e0, e1 = e[:-1], e[1:]
        with np.errstate(divide="ignore", invalid="ignore"):
            r = np.log(e0 / e1)
            cell = np.where(np.abs(r) > 1e-12, (e0 - e1) / r, 0.5 * (e0 + e1)) * dz_cm
        cell = cell * (RHO_SEA_G_CM3 / ETA_SEA)
        x = np.zeros_like(a)
        x[:-1] = np.cumsum(cell[::-1])[::-1]
        # above the table: continue the top cell's scale height
        if e[-1] > 0 and e[-2] > e[-1]:
            h_top = (a[-1] - a[-2]) / math.log(e[-2] / e[-1]) * 100.0
            x += e[-1] * (RHO_SEA_G_CM3 / ETA_SEA) * h_top
        return x

    def altitude_of_depth(self, xv: np.ndarray) -> np.ndarray:
        """Inverse of vertical_depth by log-linear interpolation."""
        xd = self.vertical_depth()
        lx = np.log(np.maximum(xd, 1e-300))
        # xd decreases with altitude: interpolate on reversed arrays
        return np.interp(np.log(np.maximum(xv, 1e-300)), lx[::-1], self.alt[::-1])


def exponential_atmosphere(eta0: float = ETA_SEA, scale_m: float = 8400.0,
                           h_max: float = 100_000.0, step: float = 100.0,
                           obs_level: float = 2200.0) -> Atmosphere:
    """n-1 = eta0 * exp(-h/H) tabulated every `step` metres from 0 to h_max."""
    n = int(round(h_max / step)) + 1
    alt = np.arange(n, dtype=np.float64) * step
    return Atmosphere(alt, eta0 * np.exp(-alt / scale_m), obs_level)


def layered_atmosphere(bounds_km: Sequence[float] = (0, 4, 10, 40, 100, 120),
                       scales_km: Sequence[float] = (9.5, 8.5, 6.4, 7.2, 6.0),
                       eta0: float = ETA_SEA, step: float = 50.0,
                       obs_level: float = 2200.0) -> Atmosphere:
    """Continuous layered exponential: d ln(n-1)/dh = -1/H_l inside layer l."""
    b = np.asarray(bounds_km, dtype=np.float64) * 1000.0
    hs = np.asarray(scales_km, dtype=np.float64) * 1000.0
    n = int(round((b[-1] - b[0]) / step)) + 1
    alt = b[0] + np.arange(n, dtype=np.float64) * step
    log_eta = np.empty_like(alt)
    base = math.log(eta0)
    for l in range(len(hs)):
        lo, hi = b[l], b[l + 1]
        m = (alt >= lo) & (alt <= hi)
        log_eta[m] = base - (alt[m] - lo) / hs[l]
        base -= (hi - lo) / hs[l]
    return Atmosphere(alt, np.exp(log_eta), obs_level)


# ----------------------------------------------------------------------------
# telescopes
# ----------------------------------------------------------------------------

def sparse_atmosphere(obs_level: float = 2200.0) -> Atmosphere:
    """The 5-layer profile tabulated at 57 non-uniform altitudes, the way
    atmospheric-profile files give it (about 55 points, denser low down):
    every 0.5 km to 10 km, every 1 km to 30 km, every 3 km to 60 km, every
    10 km to 120 km."""
    fine = layered_atmosphere(step=50.0, obs_level=obs_level)
    alt = np.concatenate([np.arange(0.0, 10000.0, 500.0), np.arange(10000.0, 30000.0, 1000.0),
                          np.arange(30000.0, 60000.0, 3000.0), np.arange(60000.0, 120001.0, 10000.0)])
    eta = np.interp(alt, fine.alt, fine.eta)
    return Atmosphere(alt, eta, obs_level)


@dataclasses.dataclass
class Telescopes:
    x: np.ndarray
    y: np.ndarray
    r: np.ndarray

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def telescopes_grid(n_side: int = 3, pitch: float = 100.0, radius: float = 12.0) -> Telescopes:
    c = (np.arange(n_side) - (n_side - 1) / 2.0) * pitch
    xx, yy = np.meshgrid(c, c, indexing="ij")
    x = xx.ravel().astype(np.float64)
    return Telescopes(x, yy.ravel().astype(np.float64), np.full(x.shape, radius))


def telescopes_disk(n: int = 100, disk_radius: float = 1000.0, r_min: float = 6.0,
                    r_max: float = 12.0, seed: int = 2006) -> Telescopes:
    """Uniform in a disk with rejection on overlap (centre distance >= Ri+Rj+1 m)."""
    rng = np.random.default_rng(seed)
    xs, ys, rs = [], [], []
    while len(xs) < n:
        rr = rng.uniform(r_min, r_max)
        a = rng.uniform(0.0, 2.0 * math.pi)
        d = disk_radius * math.sqrt(rng.uniform())
        x, y = d * math.cos(a), d * math.sin(a)
        ok = all((x - xo) ** 2 + (y - yo) ** 2 >= (rr + ro + 1.0) ** 2
                 for xo, yo, ro in zip(xs, ys, rs))
        if ok:
            xs.append(x), ys.append(y), rs.append(rr)
    return Telescopes(np.array(xs), np.array(ys), np.array(rs))


# ----------------------------------------------------------------------------
# segments
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Segments:
    """Structure-of-arrays track segments, grouped by shower."""
    x0: np.ndarray
    y0: np.ndarray
    h0: np.ndarray
    u: np.ndarray
    v: np.ndarray
    w: np.ndarray
    length: np.ndarray
    t0: np.ndarray
    energy: np.ndarray
    ptype: np.ndarray          # uint8
    seg_offsets: np.ndarray    # int64 [n_showers + 1]
    t_ref: np.ndarray          # float64 [n_showers]
    shower_ids: np.ndarray     # uint32 [n_showers] (RNG counter word)

    FIELDS = ("x0", "y0", "h0", "u", "v", "w", "length", "t0", "energy")

    @property
    def n(self) -> int:
        return int(self.x0.shape[0])

    @property
    def n_showers(self) -> int:
        return int(self.t_ref.shape[0])

    def take(self, idx: np.ndarray) -> "Segments":
        """Subset of segments (single-shower view keeps shower bookkeeping)."""
        out = {f: getattr(self, f)[idx] for f in self.FIELDS}
        return Segments(**out, ptype=self.ptype[idx],
                        seg_offsets=np.array([0, len(idx)], dtype=np.int64),
                        t_ref=self.t_ref[:1].copy(), shower_ids=self.shower_ids[:1].copy())

    def take_shower(self, shower: int, local_idx: np.ndarray) -> "Segments":
        """Steps local_idx (indices inside the shower) of one shower, as a one-shower input."""
        base = int(self.seg_offsets[shower])
        idx = base + np.asarray(local_idx, dtype=np.int64)
        out = {f: getattr(self, f)[idx] for f in self.FIELDS}
        return Segments(**out, ptype=self.ptype[idx],
                        seg_offsets=np.array([0, len(idx)], dtype=np.int64),
                        t_ref=self.t_ref[shower:shower + 1].copy(),
                        shower_ids=self.shower_ids[shower:shower + 1].copy())

    @staticmethod
    def concat(parts: List["Segments"], consume: bool = False) -> "Segments":
        """Showers of all parts in order.  consume=True empties `parts` while
        copying, so that large inputs are not held twice."""
        total = sum(p.n for p in parts)
        out = {f: np.empty(total, dtype=np.float64) for f in Segments.FIELDS}
        ptype = np.empty(total, dtype=np.uint8)
        offs, t_ref, sids = [0], [], []
        at = 0
        for i in range(len(parts)):
            p = parts[i]
            for f in Segments.FIELDS:
                out[f][at:at + p.n] = getattr(p, f)
            ptype[at:at + p.n] = p.ptype
            at += p.n
            for s in range(p.n_showers):
                offs.append(offs[-1] + int(p.seg_offsets[s + 1] - p.seg_offsets[s]))
            t_ref.append(p.t_ref)
            sids.append(p.shower_ids)
            if consume:
                parts[i] = None
        return Segments(**out, ptype=ptype, seg_offsets=np.array(offs, dtype=np.int64),
                        t_ref=np.concatenate(t_ref), shower_ids=np.concatenate(sids).astype(np.uint32))

    @staticmethod
    def join_blocks(blocks: List["Segments"]) -> "Segments":
        """Blocks of one shower (same t_ref and shower id) as a single shower."""
        one = Segments.concat(blocks, consume=True)
        return Segments(**{f: getattr(one, f) for f in Segments.FIELDS}, ptype=one.ptype,
                        seg_offsets=np.array([0, one.n], dtype=np.int64),
                        t_ref=one.t_ref[:1].copy(), shower_ids=one.shower_ids[:1].copy())


def _orthonormal_pair(ax: np.ndarray):
    """Two unit vectors perpendicular to the unit vector ax (3,)."""
    helper = np.array([1.0, 0.0, 0.0]) if abs(ax[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(ax, helper)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(ax, e1)
    return e1, e2


def _sample_gaisser_hillas(rng, n, xmax, x_limit):
    """Slant depths X in (0, x_limit] from N(X) ~ (X/Xmax)^(Xmax/lam) e^((Xmax-X)/lam)."""
    grid = np.linspace(0.0, x_limit, 8193)
    with np.errstate(divide="ignore"):
        logn = (xmax / GH_LAMBDA_G_CM2) * np.log(np.maximum(grid, 1e-300) / xmax) \
            + (xmax - grid) / GH_LAMBDA_G_CM2
    pdf = np.exp(logn - np.max(logn))
    pdf[0] = 0.0
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (pdf[1:] + pdf[:-1]) * np.diff(grid))])
    cdf /= cdf[-1]
    return np.interp(rng.uniform(size=n), cdf, grid)


def shower_segments(shower: int, n_seg: int, atmo: Atmosphere, *, zenith_deg: float = 0.0,
                    azimuth_deg: float = 0.0, core=(0.0, 0.0), xmax: float = 300.0,
                    e_range_mev=(20.0, 1000.0), cone_deg: float = 3.0,
                    lateral_mean: float = 30.0, ptype: int = PTYPE_ELECTRON,
                    len_range=(1.0, 100.0), muon_fraction: float = 0.0,
                    muon_e_range_mev=(1000.0, 100000.0), muon_cone_deg: float = 15.0,
                    muon_xmax: float = 450.0, muon_lateral_mean: float = 150.0,
                    shower_id: Optional[int] = None, block: Optional[int] = None) -> Segments:
    """Segments of one synthetic shower, seeded by SeedSequence(2006, spawn_key=(shower,)),
    or, for one block of a large shower, spawn_key=(shower, block)."""
    key = (shower,) if block is None else (shower, block)
    rng = np.random.default_rng(np.random.SeedSequence(2006, spawn_key=key))
    h_obs = atmo.obs_level
    th, ph = math.radians(zenith_deg), math.radians(azimuth_deg)
    axis = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), -math.cos(th)])
    w0 = math.cos(th)
    e1, e2 = _orthonormal_pair(axis)

    n_mu = int(round(n_seg * muon_fraction))
    kinds = np.zeros(n_seg, dtype=np.uint8)
    kinds[n_seg - n_mu:] = PTYPE_MUON if muon_fraction > 0 else ptype
    if muon_fraction == 0:
        kinds[:] = ptype
    rng.shuffle(kinds)
    is_mu = kinds == PTYPE_MUON

    x_obs_vert = float(atmo.vertical_depth()[np.searchsorted(atmo.alt, h_obs)])
    x_limit = x_obs_vert / w0

    def per_kind(mask, xm, lat_mean, cone, erange):
        m = int(mask.sum())
        if m == 0:
            return
        pos = np.empty((m, 3))
        todo = np.arange(m)
        while todo.size:
            k = todo.size
            xs = _sample_gaisser_hillas(rng, k, xm, x_limit)
            h_axis = atmo.altitude_of_depth(xs * w0)
            s_up = (h_axis - h_obs) / w0
            foot = np.stack([core[0] - axis[0] * s_up, core[1] - axis[1] * s_up, h_axis], axis=1)
            r = rng.exponential(lat_mean, size=k)
            a = rng.uniform(0.0, 2.0 * math.pi, size=k)
            p = foot + (r * np.cos(a))[:, None] * e1 + (r * np.sin(a))[:, None] * e2
            pos[todo] = p
            todo = todo[p[:, 2] < h_obs + 1.0]
        cosg = rng.uniform(math.cos(math.radians(cone)), 1.0, size=m)
        sing = np.sqrt(1.0 - cosg * cosg)
        az = rng.uniform(0.0, 2.0 * math.pi, size=m)
        d = cosg[:, None] * axis + (sing * np.cos(az))[:, None] * e1 + (sing * np.sin(az))[:, None] * e2
        d /= np.linalg.norm(d, axis=1)[:, None]
        energy = np.exp(rng.uniform(math.log(erange[0]), math.log(erange[1]), size=m))
        length = np.exp(rng.uniform(math.log(len_range[0]), math.log(len_range[1]), size=m))
        w = -d[:, 2]
        length = np.minimum(length, (pos[:, 2] - h_obs) / w)
        # time: slant distance along the axis from its 100 km crossing to the foot
        s_foot = (pos - np.array([core[0], core[1], h_obs])) @ (-axis)
        t0 = ((TOP_OF_ATMOSPHERE_M - h_obs) / w0 - s_foot) / C_LIGHT_M_PER_NS
        out = dict(x0=pos[:, 0], y0=pos[:, 1], h0=pos[:, 2], u=d[:, 0], v=d[:, 1], w=w,
                   length=length, t0=t0, energy=energy)
        for key, val in out.items():
            cols[key][mask] = val

    cols = {f: np.empty(n_seg, dtype=np.float64) for f in Segments.FIELDS}
    if muon_fraction > 0:
        per_kind(~is_mu, xmax, lateral_mean, cone_deg, e_range_mev)
        per_kind(is_mu, muon_xmax, muon_lateral_mean, muon_cone_deg, muon_e_range_mev)
    elif ptype == PTYPE_MUON:
        per_kind(is_mu, xmax, lateral_mean, cone_deg, e_range_mev)
    else:
        per_kind(~is_mu, xmax, lateral_mean, cone_deg, e_range_mev)
    t_ref = (TOP_OF_ATMOSPHERE_M - h_obs) / (w0 * C_LIGHT_M_PER_NS)
    sid = shower if shower_id is None else shower_id
    return Segments(**cols, ptype=kinds, seg_offsets=np.array([0, n_seg], dtype=np.int64),
                    t_ref=np.array([t_ref]), shower_ids=np.array([sid], dtype=np.uint32))


# ----------------------------------------------------------------------------
# the workloads
# ----------------------------------------------------------------------------

# showers above this many steps are generated as independently seeded blocks
BLOCK_SEGMENTS = 4_000_000


def default_workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _pmap(fn: Callable, items, workers: Optional[int]):
    """Map in threads (numpy releases the GIL in the bulk of the generator);
    results in input order."""
    items = list(items)
    w = default_workers() if workers is None else workers
    if w <= 1 or len(items) <= 1:
        return [fn(x) for x in items]
    with ThreadPoolExecutor(min(w, len(items))) as ex:
        return list(ex.map(fn, items))


def large_shower(shower: int, n_seg: int, atmo: Atmosphere, workers: Optional[int] = None,
                 **kw) -> Segments:
    """One shower; above BLOCK_SEGMENTS steps it is the concatenation of blocks of
    BLOCK_SEGMENTS steps, block b seeded by spawn_key=(shower, b)."""
    if n_seg <= BLOCK_SEGMENTS:
        return shower_segments(shower, n_seg, atmo, **kw)
    sizes = [min(BLOCK_SEGMENTS, n_seg - b0) for b0 in range(0, n_seg, BLOCK_SEGMENTS)]
    blocks = _pmap(lambda b: shower_segments(shower, sizes[b], atmo, block=b, **kw),
                   range(len(sizes)), workers)
    return Segments.join_blocks(blocks)

@dataclasses.dataclass
class Workload:
    name: str
    atmo: Atmosphere
    tels: Telescopes
    segs: Segments
    bunch_size: float = 5.0
    lambda_min: float = 300.0
    lambda_max: float = 600.0
    seed: int = METHOD_SEED
    fine_step: float = 0.0   # 0: keep the tabulated step


def vertical_gamma(n_seg: int = 20_000) -> Workload:
    """1 vertical gamma shower, 2e4 e+- segments, Xmax 300, exponential atmosphere
    tabulated every 100 m, 3x3 telescopes of 12 m at 100 m pitch."""
    atmo = exponential_atmosphere(step=100.0, h_max=100_000.0, obs_level=2200.0)
    segs = shower_segments(0, n_seg, atmo, zenith_deg=0.0, xmax=300.0)
    return Workload("vertical_gamma_2e4", atmo, telescopes_grid(), segs)


def single_tev(n_seg: int = 2_000_000) -> Workload:
    """1 TeV gamma-like shower at 20 deg: 2e6 segments, Xmax 400, 5-layer
    atmosphere on a 50 m grid to 120 km, 100 telescopes (6-12 m) in a 1 km disk."""
    atmo = layered_atmosphere()
    segs = shower_segments(0, n_seg, atmo, zenith_deg=20.0, azimuth_deg=0.0, xmax=400.0)
    return Workload(f"single_tev_20deg_{n_seg:.0e}".replace("+0", ""), atmo,
                    telescopes_disk(), segs)


def inclined(zenith_deg: float, n_seg: int = 2_000_000) -> Workload:
    """The TeV gamma-like shower of single_tev at a large zenith angle (core at
    the array centre, Xmax 400 g/cm^2 along the axis), for the curved
    atmosphere: at 70 deg its light is emitted 10-60 km from the array."""
    atmo = layered_atmosphere()
    segs = shower_segments(0, n_seg, atmo, zenith_deg=zenith_deg, azimuth_deg=0.0, xmax=400.0)
    return Workload(f"inclined_{int(zenith_deg)}deg_{n_seg:.0e}".replace("+0", ""), atmo,
                    telescopes_disk(), segs)


def batched_showers(n_showers: int = 256, seg_scale: float = 1.0, seed: int = 2006,
                    workers: Optional[int] = None) -> Workload:
    """Many showers of uneven size: E log-uniform 30 GeV..30 TeV,
    n_seg = min(4e6, 1e4 E/30 GeV) x seg_scale, zenith U[0,60], cores in the 1 km disk."""
    atmo = layered_atmosphere()
    rng = np.random.default_rng(seed)
    energy = np.exp(rng.uniform(math.log(30.0), math.log(30000.0), size=n_showers))  # GeV
    zen = rng.uniform(0.0, 60.0, size=n_showers)
    az = rng.uniform(0.0, 360.0, size=n_showers)
    rc = 1000.0 * np.sqrt(rng.uniform(size=n_showers))
    ac = rng.uniform(0.0, 2 * math.pi, size=n_showers)

    def one(s):
        n_seg = max(1, int(round(min(4e6, 1e4 * energy[s] / 30.0) * seg_scale)))
        xm = 400.0 + 80.0 * math.log10(energy[s] / 1000.0)
        return shower_segments(s, n_seg, atmo, zenith_deg=float(zen[s]), azimuth_deg=float(az[s]),
                               core=(rc[s] * math.cos(ac[s]), rc[s] * math.sin(ac[s])), xmax=xm)

    parts = _pmap(one, range(n_showers), workers)
    return Workload(f"batched_{n_showers}", atmo, telescopes_disk(),
                    Segments.concat(parts, consume=True))


def hadron_like(zenith_deg: float, n_seg: int = 50_000_000, shower: int = 0,
                workers: Optional[int] = None) -> Workload:
    """90% e+- (Xmax 550, lateral mean 60 m) + 10% muons (1-100 GeV, 15 deg cone)."""
    atmo = layered_atmosphere()
    segs = large_shower(shower, n_seg, atmo, workers, zenith_deg=zenith_deg, xmax=550.0,
                        lateral_mean=60.0, muon_fraction=0.1)
    return Workload(f"hadron_like_{int(zenith_deg)}deg", atmo, telescopes_disk(), segs)


def grazing_tracks(n_seg: int = 20_000, seed: int = 86) -> Workload:
    """Near-horizontal electron steps low above the observation level (step w
    0.02-0.14, heading +x, 30-400 m up), so their photons arrive with w on both
    sides of 0.1 (and some upward); 400 spheres of 12 m on a line along +x
    (100 m - 10.1 km, 25 m apart) catch them."""
    atmo = layered_atmosphere()
    rng = np.random.default_rng(seed)
    h_obs = atmo.obs_level
    w = rng.uniform(0.02, 0.14, n_seg)
    az = rng.normal(0.0, 0.002, n_seg)
    s = np.sqrt(1.0 - w * w)
    u, v = s * np.cos(az), s * np.sin(az)
    h0 = h_obs + rng.uniform(30.0, 400.0, n_seg)
    x0 = rng.uniform(-200.0, 200.0, n_seg)
    y0 = rng.normal(0.0, 4.0, n_seg)
    length = np.minimum(np.exp(rng.uniform(math.log(1.0), math.log(100.0), n_seg)), (h0 - h_obs) / w)
    energy = np.exp(rng.uniform(math.log(100.0), math.log(2000.0), n_seg))
    t0 = rng.uniform(0.0, 100.0, n_seg)
    segs = Segments(x0, y0, h0, u, v, w, length, t0, energy, np.zeros(n_seg, np.uint8),
                    np.array([0, n_seg], dtype=np.int64), np.zeros(1), np.zeros(1, np.uint32))
    xs = 100.0 + 25.0 * np.arange(400)
    tels = Telescopes(xs, np.zeros(400), np.full(400, 12.0))
    return Workload("grazing_tracks", atmo, tels, segs)


# ----------------------------------------------------------------------------
# differentiation workload: parameterised atmosphere, target from perturbed
# parameters (common random numbers: same steps, same seed)
# ----------------------------------------------------------------------------

DIFF_LAYER_BOUNDS_M = tuple(1000.0 * b for b in (0, 2, 4, 7, 10, 15, 25, 40, 120))
DIFF_BASE_SCALE_M = tuple(1000.0 * h for h in (9.5, 9.5, 8.5, 8.5, 6.4, 6.4, 6.4, 7.2))
DIFF_N_KNOTS = 64
DIFF_KNOT_TOP_M = 60_000.0


@dataclasses.dataclass
class DiffWorkload:
    name: str
    segs: Segments
    tels: Telescopes
    eta0: float
    layer_bounds: np.ndarray
    n_knots: int
    knot_top: float
    obs_level: float
    step: float
    top: float
    theta0: np.ndarray          # 64 knots (log n-1 offsets), then 8 scale heights [m]
    theta_target: np.ndarray
    sigma: float = 0.5          # soft sphere edge [m]
    bunch_size: float = 5.0
    lambda_min: float = 300.0
    lambda_max: float = 600.0
    seed: int = METHOD_SEED


def diff_showers(n_showers: int = 64, n_seg: int = 500_000, seed: int = 4927,
                 zenith_deg: float = 20.0) -> DiffWorkload:
    """Gamma-like showers at 20 deg (or zenith_deg), Xmax 400, cores uniform within
    300 m of the array centre; theta0 = (knots 0, base scale heights), target theta*
    with knots 0.05 sin(2 pi j/16 + 0.3) and scale heights x (1 + 0.02 (-1)^l)."""
    place = layered_atmosphere()
    rng = np.random.default_rng(seed)
    rc = 300.0 * np.sqrt(rng.uniform(size=n_showers))
    ac = rng.uniform(0.0, 2 * math.pi, size=n_showers)
    parts = _pmap(lambda s: shower_segments(s, n_seg, place, zenith_deg=zenith_deg, azimuth_deg=0.0,
                                            core=(rc[s] * math.cos(ac[s]), rc[s] * math.sin(ac[s])),
                                            xmax=400.0),
                  range(n_showers), None)
    j = np.arange(DIFF_N_KNOTS)
    l = np.arange(len(DIFF_BASE_SCALE_M))
    base = np.array(DIFF_BASE_SCALE_M)
    theta0 = np.concatenate([np.zeros(DIFF_N_KNOTS), base])
    target = np.concatenate([0.05 * np.sin(2 * math.pi * j / 16.0 + 0.3),
                             base * (1.0 + 0.02 * (-1.0) ** l)])
    name = f"diff_{n_showers}x{n_seg}" + ("" if zenith_deg == 20.0 else f"_{int(zenith_deg)}deg")
    return DiffWorkload(name, Segments.concat(parts, consume=True),
                        telescopes_disk(),
                        ETA_SEA, np.array(DIFF_LAYER_BOUNDS_M), DIFF_N_KNOTS, DIFF_KNOT_TOP_M,
                        2200.0, 50.0, 120_000.0, theta0, target)
