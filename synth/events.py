"""Seeded synthetic TPC cluster sets with the shapes of the paper's workloads.

Charged particles move on helices in a uniform solenoidal field.  A cluster is
where a helix crosses a pad-row plane inside a sector, optionally moved by a
smooth radial space-charge distortion, smeared by the cluster resolution, and
mixed with uniformly distributed noise clusters.  Time-frame slices overlap
many collisions in drift time (paper, Section 1: continuous read-out, about
five Pb-Pb collisions per 100 us drift time).

The module knows the detector description and helix kinematics only; it holds
no part of the tracking method.  Random numbers come from numpy's PCG64 with
one spawned sub-stream per purpose, so every set is reproducible from its seed.
Heavy geometry runs in float64 on a torch device (CPU by default) in chunks.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

from . import geometry as G


# ----------------------------------------------------------------------------
# particles
# ----------------------------------------------------------------------------
@dataclass
class Tracks:
    """Truth kinematics, float64; one entry per particle."""
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    pt: np.ndarray      # GeV/c
    phi: np.ndarray     # azimuth of the momentum at the vertex
    tanl: np.ndarray    # pz / pT = sinh(eta)
    q: np.ndarray       # charge sign, +-1
    t_us: np.ndarray    # collision time inside the time frame

    def __len__(self):
        return len(self.pt)

    @staticmethod
    def concat(parts):
        return Tracks(*[np.concatenate([getattr(p, f) for p in parts])
                        for f in ("vx", "vy", "vz", "pt", "phi", "tanl", "q", "t_us")])


def _primaries(rng, n, pt, eta, phi, t_us=0.0):
    z0 = np.zeros(n)
    return Tracks(z0.copy(), z0.copy(), z0.copy(), pt, phi, np.sinh(eta),
                  rng.choice(np.array([-1.0, 1.0]), size=n), np.full(n, float(t_us)))


def _secondaries(rng, n, pt, eta, phi, rv_max=60.0, t_us=0.0):
    rv = rng.uniform(0.0, rv_max, size=n)
    t = _primaries(rng, n, pt, eta, phi, t_us)
    t.vx = rv * np.cos(phi)
    t.vy = rv * np.sin(phi)
    t.vz = rv * np.sinh(eta)
    return t


def pt_exponential(rng, n, mean_above_floor=0.5, floor=0.1):
    """pT = floor + Exp(mean): mean pT 0.6 GeV/c with a 0.1 GeV/c floor."""
    return floor + rng.exponential(mean_above_floor, size=n)


# ----------------------------------------------------------------------------
# distortion
# ----------------------------------------------------------------------------
@dataclass
class RadialDistortion:
    """Measured radius = true radius - amp * (r0 / r)^2 at unchanged angle and z."""
    amp_cm: float = 10.0
    r0_cm: float = 85.0

    def shift(self, r):
        return self.amp_cm * (self.r0_cm / r) ** 2


# ----------------------------------------------------------------------------
# helix / pad-row-plane crossings
# ----------------------------------------------------------------------------
def _psi_exit(cx, cy, R, q, theta0, r_out):
    """Turning angle at which the helix first reaches the outer radius."""
    cabs = torch.sqrt(cx * cx + cy * cy)
    beta = torch.atan2(cy, cx)
    qq = (r_out * r_out - cabs * cabs - R * R) / (2.0 * R * cabs)
    two_pi = 2.0 * math.pi
    res = torch.full_like(R, two_pi)
    reach = qq.abs() <= 1.0
    ac = torch.acos(qq.clamp(-1.0, 1.0))
    for sgn in (1.0, -1.0):
        th = beta + sgn * ac
        psi = torch.remainder(q * (theta0 - th), two_pi)
        psi = torch.where(psi <= 0.0, torch.full_like(psi, two_pi), psi)
        res = torch.where(reach, torch.minimum(res, psi), res)
    return res


def helix_crossings(tr: Tracks, distortion: RadialDistortion | None = None,
                    device="cpu", chunk=2048, as_numpy=True):
    """All crossings of the helices with the pad-row planes of every sector.

    A helix is followed for at most one full turn in the transverse plane
    (outgoing and returning leg), until it reaches the outer radius, and while
    |z| <= z_max.  Returns a dict of arrays over crossings (numpy, or torch
    tensors on ``device``): track, sector, row, y (local, as measured), z, psi
    (turning angle from the vertex), y_true (local y of the undistorted point).
    """
    dt = torch.float64
    xr = torch.tensor(G.row_x_f64(), dtype=dt, device=device)          # [152]
    tanh = G.tan_half_opening()
    kap = G.C_LIGHT_GEV * G.BZ_TESLA
    out = {k: [] for k in ("track", "sector", "row", "y", "z", "psi", "y_true")}
    n = len(tr)
    for c0 in range(0, n, chunk):
        sl = slice(c0, min(n, c0 + chunk))
        T = lambda a: torch.tensor(a[sl], dtype=dt, device=device)
        vx, vy, vz, pt, phi, tl, q = (T(tr.vx), T(tr.vy), T(tr.vz), T(tr.pt),
                                      T(tr.phi), T(tr.tanl), T(tr.q))
        R = pt / kap
        cx = vx + q * R * torch.sin(phi)
        cy = vy - q * R * torch.cos(phi)
        theta0 = torch.atan2(vy - cy, vx - cx)
        psi_end = _psi_exit(cx, cy, R, q, theta0, G.OUTER_RADIUS_CM)
        side_a = (tl > 0) | ((tl == 0) & (vz >= 0))
        # the 18 sectors of the track's own side
        sec_local = torch.arange(G.SECTORS_PER_SIDE, device=device)
        sec = sec_local[None, :] + torch.where(side_a, 0, G.SECTORS_PER_SIDE)[:, None]  # [T,18]
        alpha = (sec_local.to(dt) + 0.5) * (2.0 * math.pi / G.SECTORS_PER_SIDE)        # [18]
        ca, sa = torch.cos(alpha), torch.sin(alpha)
        cxl = cx[:, None] * ca + cy[:, None] * sa                                      # [T,18]
        cyl = -cx[:, None] * sa + cy[:, None] * ca
        d = xr[None, None, :] - cxl[:, :, None]                                        # [T,18,152]
        disc = R[:, None, None] ** 2 - d * d
        ok0 = disc >= 0.0
        h = torch.sqrt(disc.clamp_min(0.0))
        for br in (1.0, -1.0):
            Y = cyl[:, :, None] + br * h
            th = torch.atan2(Y - cyl[:, :, None], d) + alpha[None, :, None]
            psi = torch.remainder(q[:, None, None] * (theta0[:, None, None] - th), 2.0 * math.pi)
            z = vz[:, None, None] + tl[:, None, None] * R[:, None, None] * psi
            ok = (ok0 & (Y.abs() <= xr[None, None, :] * tanh) & (psi > 0.0)
                  & (psi < psi_end[:, None, None]) & (z.abs() <= G.Z_MAX_CM)
                  & ((z >= 0.0) == side_a[:, None, None]))
            if distortion is not None:
                # loose pre-selection; validity is decided after the distortion
                margin = 2.0 * distortion.amp_cm
                ok = (ok0 & (Y.abs() <= xr[None, None, :] * tanh + margin) & (psi > 0.0)
                      & (psi < psi_end[:, None, None] + 0.5)
                      & (z.abs() <= G.Z_MAX_CM + margin * tl.abs().max().clamp_min(1.0)))
            idx = ok.nonzero(as_tuple=True)
            if idx[0].numel() == 0:
                continue
            ti, si, ri = idx
            if distortion is not None:
                Yd, zd, psid, okd, Yt = _distorted_crossing(
                    xr[ri], cxl[ti, si], cyl[ti, si], R[ti], q[ti], theta0[ti], alpha[si],
                    vz[ti], tl[ti], br, distortion)
                okd = (okd & (Yd.abs() <= xr[ri] * tanh) & (psid > 0.0)
                       & (psid < psi_end[ti]) & (zd.abs() <= G.Z_MAX_CM)
                       & ((zd >= 0.0) == side_a[ti]))
                sel = okd.nonzero(as_tuple=True)[0]
                ti, si, ri = ti[sel], si[sel], ri[sel]
                Yv, zv, pv, Yt = Yd[sel], zd[sel], psid[sel], Yt[sel]
            else:
                Yv, zv, pv = Y[idx], z[idx], psi[idx]
                Yt = Yv
            out["track"].append(ti + c0)
            out["sector"].append(sec[ti, si])
            out["row"].append(ri)
            out["y"].append(Yv)
            out["z"].append(zv)
            out["psi"].append(pv)
            out["y_true"].append(Yt)
    res = {}
    for k, v in out.items():
        if v:
            res[k] = torch.cat(v)
        else:
            res[k] = torch.zeros(0, dtype=dt if k in ("y", "z", "psi", "y_true") else torch.int64,
                                 device=device)
    if as_numpy:
        res = {k: v.cpu().numpy() for k, v in res.items()}
    return res


def _distorted_crossing(x_row, cxl, cyl, R, q, theta0, alpha, vz, tl, br, dist, n_iter=40):
    """True point whose radially distorted image lies on the row plane x_row.

    Fixed-point iteration on the plane X the true helix crosses:
    X <- x_row / (1 - delta(r)/r), r the radius of the crossing with plane X.
    Returns the measured local y (the image), z, turning angle, validity and
    the true local y.
    """
    X = x_row.clone()
    ok = torch.ones_like(X, dtype=torch.bool)
    for _ in range(n_iter):
        d = X - cxl
        disc = R * R - d * d
        ok = ok & (disc >= 0.0)
        Y = cyl + br * torch.sqrt(disc.clamp_min(0.0))
        r = torch.sqrt(X * X + Y * Y)
        X = x_row / (1.0 - dist.shift(r) / r)
    d = X - cxl
    disc = R * R - d * d
    ok = ok & (disc >= 0.0)
    Y = cyl + br * torch.sqrt(disc.clamp_min(0.0))
    r = torch.sqrt(X * X + Y * Y)
    scale = 1.0 - dist.shift(r) / r
    th = torch.atan2(Y - cyl, d) + alpha
    psi = torch.remainder(q * (theta0 - th), 2.0 * math.pi)
    z = vz + tl * R * psi
    return Y * scale, z, psi, ok, Y


# ----------------------------------------------------------------------------
# cluster sets
# ----------------------------------------------------------------------------
@dataclass
class ClusterSet:
    """Clusters grouped by (unit, row); caller index = cluster id.

    row_begin[u*N_ROWS + r] .. row_begin[u*N_ROWS + r + 1] is the range of
    unit u, row r.  Within a range the order is a seeded shuffle.
    """
    n_units: int
    unit_sector: np.ndarray          # int32 [n_units]
    row_begin: np.ndarray            # int64 [n_units*N_ROWS+1]
    y: np.ndarray                    # float32 [N]
    z: np.ndarray                    # float32 [N]
    truth_track: np.ndarray          # int64 [N], -1 for noise
    truth_y: np.ndarray              # float64 [N] true local y (before distortion and smearing)
    truth_z: np.ndarray
    truth_psi: np.ndarray            # float64 [N] turning angle from the vertex (nan for noise)
    tracks: Tracks
    meta: dict = field(default_factory=dict)

    @property
    def n_clusters(self):
        return int(self.y.shape[0])

    def row_of(self):
        """Row index of every cluster (host helper for tests)."""
        cnt = np.diff(self.row_begin)
        return np.repeat(np.tile(np.arange(G.N_ROWS), self.n_units), cnt).astype(np.int32)

    def unit_of(self):
        cnt = np.diff(self.row_begin)
        return np.repeat(np.repeat(np.arange(self.n_units), G.N_ROWS), cnt).astype(np.int32)


def build_clusters(tracks: Tracks, sectors, rng_seed, smear_sigma=0.1, noise_frac=0.0,
                   distortion=None, drift_offsets=False, device="cpu", meta=None, truth=True):
    """Turn particles into a ClusterSet over the given sectors (one unit each).

    Random numbers for smearing, noise and the in-row order come from a torch
    generator on ``device`` seeded from ``rng_seed``: a seed reproduces the same
    set on the same kind of device.
    """
    dev = torch.device(device)
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(rng_seed) % (2**63))
    dt = torch.float64
    sectors = np.asarray(sectors, dtype=np.int32)
    unit_of_sector = torch.full((G.N_SECTORS,), -1, dtype=torch.int64, device=dev)
    unit_of_sector[torch.as_tensor(sectors, dtype=torch.int64, device=dev)] = torch.arange(
        len(sectors), device=dev)

    cr = helix_crossings(tracks, distortion, device=dev, as_numpy=False)
    unit = unit_of_sector[cr["sector"]]
    keep = unit >= 0
    trk = cr["track"][keep]
    unit = unit[keep]
    row = cr["row"][keep].to(torch.int64)
    my0 = cr["y"][keep]
    ty = cr["y_true"][keep]
    tz = cr["z"][keep]
    tpsi = cr["psi"][keep]
    if drift_offsets:
        # continuous read-out: the drift coordinate of a cluster is shifted by
        # the collision time, towards the read-out plane of its own side
        t_us = torch.as_tensor(tracks.t_us, dtype=dt, device=dev)
        sgn = torch.where(tz >= 0.0, 1.0, -1.0)
        tz = tz - sgn * G.DRIFT_CM_PER_US * t_us[trk]
    n_sig = int(trk.numel())
    if smear_sigma > 0:
        my = my0 + smear_sigma * torch.randn(n_sig, generator=gen, device=dev, dtype=dt)
        mz = tz + smear_sigma * torch.randn(n_sig, generator=gen, device=dev, dtype=dt)
    else:
        my, mz = my0.clone(), tz.clone()

    n_noise = int(round(noise_frac * n_sig))
    if n_noise:
        nu = torch.randint(0, len(sectors), (n_noise,), generator=gen, device=dev)
        nr = torch.randint(0, G.N_ROWS, (n_noise,), generator=gen, device=dev)
        xr = torch.as_tensor(G.row_x_f64(), dtype=dt, device=dev)[nr]
        ny = (torch.rand(n_noise, generator=gen, device=dev, dtype=dt) * 2.0 - 1.0) * xr * G.tan_half_opening()
        side_a = torch.as_tensor(G.sector_side_is_a(sectors), device=dev)[nu]
        t_max = float(tracks.t_us.max()) if (drift_offsets and len(tracks)) else 0.0
        span = G.DRIFT_CM_PER_US * t_max
        u01 = torch.rand(n_noise, generator=gen, device=dev, dtype=dt)
        nz = torch.where(side_a, -span + u01 * (G.Z_MAX_CM + span),
                         -G.Z_MAX_CM + u01 * (G.Z_MAX_CM + span))
        trk = torch.cat([trk, torch.full((n_noise,), -1, dtype=torch.int64, device=dev)])
        unit = torch.cat([unit, nu])
        row = torch.cat([row, nr])
        ty = torch.cat([ty, ny])
        tz = torch.cat([tz, nz])
        my = torch.cat([my, ny])
        mz = torch.cat([mz, nz])
        tpsi = torch.cat([tpsi, torch.full((n_noise,), float("nan"), dtype=dt, device=dev)])

    # group by (unit, row); seeded shuffle inside each group
    key = unit * G.N_ROWS + row
    perm = torch.randperm(key.numel(), generator=gen, device=dev)
    order = perm[torch.argsort(key[perm], stable=True)]
    counts = torch.bincount(key, minlength=len(sectors) * G.N_ROWS)
    row_begin = np.zeros(len(sectors) * G.N_ROWS + 1, dtype=np.int64)
    np.cumsum(counts.cpu().numpy(), out=row_begin[1:])
    h = lambda t: t[order].cpu().numpy()
    if not truth:
        # measured clusters only (large inputs: no per-cluster truth on the host)
        return ClusterSet(len(sectors), sectors, row_begin, h(my.to(torch.float32)),
                          h(mz.to(torch.float32)), None, None, None, None, tracks, dict(meta or {}))
    return ClusterSet(len(sectors), sectors, row_begin, h(my.to(torch.float32)),
                      h(mz.to(torch.float32)), h(trk), h(ty), h(tz), h(tpsi), tracks,
                      dict(meta or {}))


# ----------------------------------------------------------------------------
# the workloads
# ----------------------------------------------------------------------------
def single_sector(seed=1, n_tracks=200, noise_frac=0.05, smear_sigma=0.1, device="cpu"):
    """One side-A sector: primaries from the origin, pT log-uniform 0.2-10 GeV/c,
    0 <= eta < 0.9, azimuth uniform across sector 0, 5 % uniform noise."""
    ss = np.random.SeedSequence(seed)
    rt, rc = [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(2)]
    pt = np.exp(rt.uniform(math.log(0.2), math.log(10.0), n_tracks))
    eta = rt.uniform(0.0, 0.9, n_tracks)
    a0 = float(G.sector_alpha(0))
    phi = rt.uniform(a0 - G.HALF_OPENING_RAD, a0 + G.HALF_OPENING_RAD, n_tracks)
    tr = _primaries(rt, n_tracks, pt, eta, phi)
    return build_clusters(tr, [0], int(rc.integers(2**63)), smear_sigma, noise_frac,
                          device=device, meta=dict(workload="single-sector", seed=seed))


def central_event(seed=2, n_primaries=10_000, secondary_frac=0.2, noise_frac=0.10,
                  smear_sigma=0.1, distortion=None, device="cpu"):
    """Full TPC (36 sectors), central Pb-Pb-like multiplicity."""
    ss = np.random.SeedSequence(seed)
    rt, rc = [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(2)]
    tr = _event_tracks(rt, n_primaries, secondary_frac, 0.0)
    return build_clusters(tr, np.arange(G.N_SECTORS), int(rc.integers(2**63)), smear_sigma,
                          noise_frac, distortion=distortion, device=device,
                          meta=dict(workload="central-event", seed=seed))


def _event_tracks(rng, n_prim, secondary_frac, t_us):
    n_sec = int(round(secondary_frac * n_prim))
    p = _primaries(rng, n_prim, pt_exponential(rng, n_prim), rng.uniform(-0.9, 0.9, n_prim),
                   rng.uniform(0.0, 2.0 * math.pi, n_prim), t_us)
    s = _secondaries(rng, n_sec, pt_exponential(rng, n_sec), rng.uniform(-0.9, 0.9, n_sec),
                     rng.uniform(0.0, 2.0 * math.pi, n_sec), t_us=t_us)
    return Tracks.concat([p, s])


def timeframe_slice(seed=3000, n_collisions=128, mean_primaries=2500.0, secondary_frac=0.2,
                    noise_frac=0.10, smear_sigma=0.1, rate_per_us=0.05,
                    distortion=RadialDistortion(), device="cpu", truth=True):
    """Overlapping minimum-bias collisions in continuous drift time.

    Collision times form a Poisson process (5 per 100 us); multiplicities are
    exponential with a mean of a quarter of the central event.
    """
    ss = np.random.SeedSequence(seed)
    rt, rc = [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(2)]
    times = np.cumsum(rt.exponential(1.0 / rate_per_us, n_collisions))
    mult = np.maximum(1, np.round(rt.exponential(mean_primaries, n_collisions))).astype(np.int64)
    parts = [_event_tracks(rt, int(m), secondary_frac, float(t)) for m, t in zip(mult, times)]
    tr = Tracks.concat(parts)
    return build_clusters(tr, np.arange(G.N_SECTORS), int(rc.integers(2**63)), smear_sigma,
                          noise_frac, distortion=distortion, drift_offsets=True, device=device,
                          meta=dict(workload="timeframe-slice", seed=seed, n_collisions=n_collisions),
                          truth=truth)


def slice_batch_collisions(seed=4000, n_slices=16, lo=32, hi=160):
    """Collision counts of a batch of time-frame slices: uniform in [lo, hi]."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    return [int(v) for v in rng.integers(lo, hi + 1, n_slices)]


def exact_tracks(seed, n_tracks=10, pt_range=(0.5, 5.0), eta_range=(0.05, 0.85), sector=0):
    """Noise-free, unsmeared primaries aimed into one sector (recovery pins)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    pt = np.exp(rng.uniform(math.log(pt_range[0]), math.log(pt_range[1]), n_tracks))
    eta = rng.uniform(eta_range[0], eta_range[1], n_tracks)
    a0 = float(G.sector_alpha(sector))
    phi = rng.uniform(a0 - 0.7 * G.HALF_OPENING_RAD, a0 + 0.7 * G.HALF_OPENING_RAD, n_tracks)
    tr = _primaries(rng, n_tracks, pt, eta, phi)
    return build_clusters(tr, [sector], seed + 17, smear_sigma=0.0, noise_frac=0.0,
                          meta=dict(workload="exact-tracks", seed=seed))
