"""Seeded synthetic TPC events: helix tracks crossing the pad-row planes of the
36 sector instances, with Gaussian cluster smearing and uniform noise.

This module is the one input source shared by the CPU oracle and the GPU path.
It holds detector geometry and exact circle/plane geometry of the generated
(true) trajectories only; none of the tracker's arithmetic (series
propagation, Kalman filter, neighbour scores, grid) lives here.

Workloads (the paper's reference time frame is not available, so these stand
in for it; the paper only fixes the context: Pb-Pb collisions, a 32-orbit time
frame of roughly 3 ms, TPC processing dominating the GPU load -- Introduction):

  config 1  one 20-degree sector wedge, 50 tracks from the origin
  config 2  36 sector instances, one central collision, 8000 tracks
  config 3  36 sector instances, 128 collisions overlapping in drift time
  config 4  256 independent wedge instances, cluster counts log-uniform 1e3..4e5
  config 5  found-track hit lists for the Kalman refit under a distortion map

Every random draw comes from numpy's PCG64 generator seeded with
``0x7C0000 + config`` (+ ``0x100 * rep``).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

N_ROWS = 152
X_INNER, X_OUTER = 85.0, 247.0
Z_MAX = 250.0
N_PHI = 18
SECTOR_DEG = 20.0
B_TESLA = 0.5
C_LIGHT = 0.299792458e-2          # GeV / (T cm)
V_DRIFT = 2.58                    # cm / us
SIGMA_Y, SIGMA_Z = 0.1, 0.15      # cm
SEED_BASE = 0x7C0000


def geometry() -> dict:
    """Detector description handed to both implementations as input data."""
    row_x = np.array([X_INNER + r * ((X_OUTER - X_INNER) / (N_ROWS - 1)) for r in range(N_ROWS)],
                     dtype=np.float64).astype(np.float32)
    return dict(n_rows=N_ROWS, row_x=row_x, bz=np.float32(B_TESLA),
                tan_half=np.float32(np.tan(np.radians(SECTOR_DEG / 2))),
                sigma_y2=np.float32(0.01), sigma_z2=np.float32(0.0225))


@dataclass
class Event:
    name: str
    seed: int
    x: np.ndarray            # f32[N] local x of the pad row the cluster is on
    y: np.ndarray            # f32[N] local y (measured)
    z: np.ndarray            # f32[N] z (measured; drift-shifted in config 3)
    row: np.ndarray          # u16[N]
    charge: np.ndarray       # u16[N]
    inst_off: np.ndarray     # i64[n_inst+1]
    label: np.ndarray        # i32[N] MC track id, -1 for noise
    sector: np.ndarray       # u8[N] phi-sector 0..17 of the cluster
    inst_sector: np.ndarray  # i32[n_inst]
    tracks: dict = field(default_factory=dict)   # MC truth per track
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.inst_off[-1])

    @property
    def n_inst(self) -> int:
        return len(self.inst_off) - 1

    def clusters(self) -> dict:
        return dict(x=self.x, y=self.y, z=self.z, row=self.row, charge=self.charge)


# ---------------------------------------------------------------------------
# true trajectories


def _wrap2pi(a):
    return np.mod(a, 2 * np.pi)


def _crossings(q, pt, phi0, tanl, vx, vy, vz, row_x, sectors=None, dist=None):
    """First crossing of each track with each (row, sector) pad-row plane.

    Tracks are circles of radius pt/(c B) in the transverse plane (positive
    charges turn clockwise seen from +z for B along +z), and z grows linearly
    with the transverse arc length (slope tan(lambda)).  Only the outgoing
    leg is kept: from the vertex up to the point farthest from the beam axis.
    A plane of sector k at row r is the line ``p . n_k = x_r (+ dist[r, k])``
    with n_k the sector axis; the crossing must lie inside the wedge
    (|y_local| <= x_r tan 10deg) and at |z_true| <= 250 cm.

    Returns a dict of flat arrays (one entry per crossing).
    """
    T = len(q)
    R = pt / (C_LIGHT * B_TESLA)
    cx = vx + q * R * np.sin(phi0)
    cy = vy - q * R * np.cos(phi0)
    th_v = np.arctan2(vy - cy, vx - cx)
    rc = np.hypot(cx, cy)
    fx = cx + R * cx / rc
    fy = cy + R * cy / rc
    psi_far = _wrap2pi(q * (th_v - np.arctan2(fy - cy, fx - cx)))
    psi_far = np.where(psi_far == 0, 2 * np.pi, psi_far)

    rx = row_x.astype(np.float64)
    # where the circle crosses radius x_r (fixes the candidate phi sectors)
    rho = rx[None, :]
    a = (rho * rho - (R * R)[:, None] + (rc * rc)[:, None]) / (2 * rc[:, None])
    h2 = rho * rho - a * a
    ok_rho = h2 >= 0
    hh = np.sqrt(np.where(ok_rho, h2, 0))
    ux, uy = (cx / rc)[:, None], (cy / rc)[:, None]
    best_phi = np.full((T, N_ROWS), np.nan)
    best_psi = np.full((T, N_ROWS), np.inf)
    for sgn in (1.0, -1.0):
        px = a * ux - sgn * hh * uy
        py = a * uy + sgn * hh * ux
        psi = _wrap2pi(q[:, None] * (th_v[:, None] - np.arctan2(py - cy[:, None], px - cx[:, None])))
        good = ok_rho & (psi > 0) & (psi <= psi_far[:, None]) & (psi < best_psi)
        best_psi = np.where(good, psi, best_psi)
        best_phi = np.where(good, np.arctan2(py, px), best_phi)
    has = np.isfinite(best_psi)
    k0 = np.floor(_wrap2pi(np.where(has, best_phi, 0)) / np.radians(SECTOR_DEG)).astype(np.int64) % N_PHI

    tt, rr = np.nonzero(has)
    kk0 = k0[tt, rr]
    out = {key: [] for key in ("trk", "row", "sec", "y", "z", "psi", "snp")}
    tan_half = np.tan(np.radians(SECTOR_DEG / 2))
    for dk in (-1, 0, 1):
        k = (kk0 + dk) % N_PHI
        if sectors is not None:
            sel = np.isin(k, sectors)
            t_, r_, k_ = tt[sel], rr[sel], k[sel]
        else:
            t_, r_, k_ = tt, rr, k
        alpha = np.radians(SECTOR_DEG) * (k_ + 0.5)
        nx, ny = np.cos(alpha), np.sin(alpha)
        xp = rx[r_] + (dist[r_, k_] if dist is not None else 0.0)
        d = xp - (nx * cx[t_] + ny * cy[t_])
        disc = R[t_] ** 2 - d * d
        okd = disc >= 0
        hd = np.sqrt(np.where(okd, disc, 0))
        psi_b = np.full(len(t_), np.inf)
        y_b = np.zeros(len(t_))
        px_b = np.zeros(len(t_))
        py_b = np.zeros(len(t_))
        for sgn in (1.0, -1.0):
            px = cx[t_] + d * nx - sgn * hd * ny
            py = cy[t_] + d * ny + sgn * hd * nx
            psi = _wrap2pi(q[t_] * (th_v[t_] - np.arctan2(py - cy[t_], px - cx[t_])))
            yl = -px * ny + py * nx
            good = okd & (psi > 0) & (psi <= psi_far[t_]) & (np.abs(yl) <= rx[r_] * tan_half) & (psi < psi_b)
            psi_b = np.where(good, psi, psi_b)
            y_b = np.where(good, yl, y_b)
            px_b = np.where(good, px, px_b)
            py_b = np.where(good, py, py_b)
        z = vz[t_] + tanl[t_] * R[t_] * np.where(np.isfinite(psi_b), psi_b, 0)
        keep = np.isfinite(psi_b) & (np.abs(z) <= Z_MAX)
        # direction of motion -> local sin(phi)
        dxr = (py_b - cy[t_]) * q[t_] / R[t_]
        dyr = -(px_b - cx[t_]) * q[t_] / R[t_]
        snp = -dxr * ny + dyr * nx
        for key, val in (("trk", t_), ("row", r_), ("sec", k_), ("y", y_b), ("z", z),
                         ("psi", psi_b), ("snp", snp)):
            out[key].append(val[keep])
    return {key: np.concatenate(v) for key, v in out.items()}


def _draw_pt_central(rng, n):
    """Exponential (mean 0.5 GeV) below 2 GeV, a p_T^-6 power-law tail above."""
    pt = rng.exponential(0.5, n)
    tail = pt > 2.0
    pt[tail] = 2.0 * rng.uniform(0, 1, int(tail.sum())) ** (-1.0 / 5.0)
    return pt


def _central_tracks(rng, n, vz):
    pt = _draw_pt_central(rng, n)
    eta = rng.uniform(-0.9, 0.9, n)
    phi0 = rng.uniform(0, 2 * np.pi, n)
    q = rng.choice(np.array([-1.0, 1.0]), n)
    vx = np.zeros(n)
    vy = np.zeros(n)
    sec = rng.uniform(0, 1, n) < 0.10
    ns = int(sec.sum())
    rad = rng.uniform(1.0, 50.0, ns)
    ang = rng.uniform(0, 2 * np.pi, ns)
    vx[sec] = rad * np.cos(ang)
    vy[sec] = rad * np.sin(ang)
    return dict(q=q, pt=pt, phi0=phi0, tanl=np.sinh(eta), vx=vx, vy=vy, vz=np.full(n, vz),
                secondary=sec)


def _wedge_tracks(rng, n):
    """Config-1-like tracks: from the origin, azimuth at r=166 cm uniform in sector 0."""
    pt = np.exp(rng.uniform(np.log(0.2), np.log(5.0), n))
    eta = rng.uniform(-0.9, 0.9, n)
    q = rng.choice(np.array([-1.0, 1.0]), n)
    R = pt / (C_LIGHT * B_TESLA)
    phi_t = rng.uniform(0, np.radians(SECTOR_DEG), n)
    phi0 = phi_t + q * np.arcsin(np.minimum(1.0, 166.0 / (2 * R)))
    z0 = np.zeros(n)
    return dict(q=q, pt=pt, phi0=phi0, tanl=np.sinh(eta), vx=z0.copy(), vy=z0.copy(), vz=z0.copy(),
                secondary=np.zeros(n, bool))


def _cat_tracks(parts):
    return {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}


def _assemble(rng, name, seed, geom, inst_of, n_inst, inst_sector, cr, zmeas, trk_id,
              noise_frac, z_range, tracks, smear=True):
    """Smear crossings into clusters, add per-instance noise, shuffle per instance."""
    row_x = geom["row_x"]
    tan_half = float(np.tan(np.radians(SECTOR_DEG / 2)))
    n_sig = len(cr["row"])
    truth = np.stack([cr["y"], zmeas, cr["snp"]], axis=1)
    ys = cr["y"] + (rng.normal(0, SIGMA_Y, n_sig) if smear else 0.0)
    zs = zmeas + (rng.normal(0, SIGMA_Z, n_sig) if smear else 0.0)
    cnt = np.bincount(inst_of, minlength=n_inst)
    parts = []
    for i in range(n_inst):
        sel = np.nonzero(inst_of == i)[0]
        nf = noise_frac[i] if np.ndim(noise_frac) else noise_frac
        n_noise = int(round(cnt[i] * nf))
        nr = rng.integers(0, N_ROWS, n_noise)
        ny_ = rng.uniform(-1, 1, n_noise) * row_x[nr].astype(np.float64) * tan_half
        zlo, zhi = z_range[i]
        nz_ = rng.uniform(zlo, zhi, n_noise)
        row = np.concatenate([cr["row"][sel], nr]).astype(np.uint16)
        y = np.concatenate([ys[sel], ny_])
        z = np.concatenate([zs[sel], nz_])
        lab = np.concatenate([trk_id[sel], np.full(n_noise, -1)]).astype(np.int32)
        secs = np.concatenate([cr["sec"][sel], np.full(n_noise, inst_sector[i])]).astype(np.uint8)
        tru = np.concatenate([truth[sel], np.full((n_noise, 3), np.nan)])
        order = rng.permutation(len(row))
        parts.append((row[order], y[order], z[order], lab[order], secs[order], tru[order]))
    row = np.concatenate([p[0] for p in parts]) if parts else np.zeros(0, np.uint16)
    y = np.concatenate([p[1] for p in parts]).astype(np.float32)
    z = np.concatenate([p[2] for p in parts]).astype(np.float32)
    lab = np.concatenate([p[3] for p in parts])
    secs = np.concatenate([p[4] for p in parts])
    inst_off = np.zeros(n_inst + 1, np.int64)
    inst_off[1:] = np.cumsum([len(p[0]) for p in parts])
    x = row_x[row]
    charge = rng.integers(20, 400, len(row)).astype(np.uint16)
    ev = Event(name=name, seed=seed, x=x, y=y, z=z, row=row, charge=charge, inst_off=inst_off,
               label=lab, sector=secs, inst_sector=np.asarray(inst_sector, np.int32),
               tracks=tracks)
    ev.extra["truth"] = np.concatenate([p[5] for p in parts]) if parts else np.zeros((0, 3))
    return ev


def _chunked_crossings(trk, row_x, sectors=None, dist=None, chunk=8192):
    outs = []
    n = len(trk["q"])
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        c = _crossings(trk["q"][a:b], trk["pt"][a:b], trk["phi0"][a:b], trk["tanl"][a:b],
                       trk["vx"][a:b], trk["vy"][a:b], trk["vz"][a:b], row_x, sectors, dist)
        c["trk"] = c["trk"] + a
        outs.append(c)
    return {k: np.concatenate([o[k] for o in outs]) for k in outs[0]}


def config1(rep=0, n_tracks=50, noise=0.05, smear=True) -> Event:
    """One 20-degree wedge (sector 0, both z sides) with 50 tracks from the origin."""
    seed = SEED_BASE + 1 + 0x100 * rep
    rng = np.random.Generator(np.random.PCG64(seed))
    geom = geometry()
    trk = _wedge_tracks(rng, n_tracks)
    cr = _chunked_crossings(trk, geom["row_x"], sectors=[0])
    inst = np.zeros(len(cr["row"]), np.int64)
    return _assemble(rng, "config1", seed, geom, inst, 1, [0], cr, cr["z"], cr["trk"], noise,
                     [(-Z_MAX, Z_MAX)], trk, smear=smear)


def _sector_instances(cr):
    """36 instances: phi-sector k on side A (z>=0) is k, on side C it is 18+k."""
    side = (cr["z"] < 0).astype(np.int64)
    return cr["sec"] + N_PHI * side


def config2(rep=0, n_tracks=8000, noise=0.10, smear=True) -> Event:
    """One central collision over the 36 sector instances."""
    seed = SEED_BASE + 2 + 0x100 * rep
    rng = np.random.Generator(np.random.PCG64(seed))
    geom = geometry()
    vz = rng.normal(0, 5.0)
    trk = _central_tracks(rng, n_tracks, vz)
    cr = _chunked_crossings(trk, geom["row_x"])
    inst = _sector_instances(cr)
    zr = [(0.0, Z_MAX)] * N_PHI + [(-Z_MAX, 0.0)] * N_PHI
    return _assemble(rng, "config2", seed, geom, inst, 2 * N_PHI, list(range(N_PHI)) * 2, cr,
                     cr["z"], cr["trk"], noise, zr, trk, smear=smear)


def config3(rep=0, n_coll=128, mean_tracks=1500.0, t_window_us=3000.0, noise=0.10) -> Event:
    """A time-frame slice: collisions at uniform times, z shifted by the drift."""
    seed = SEED_BASE + 3 + 0x100 * rep
    rng = np.random.Generator(np.random.PCG64(seed))
    geom = geometry()
    parts, t0 = [], []
    for _ in range(n_coll):
        t = rng.uniform(0, t_window_us)
        n = int(round(rng.exponential(mean_tracks)))
        if n == 0:
            continue
        parts.append(_central_tracks(rng, n, rng.normal(0, 5.0)))
        t0.append(np.full(n, t))
    trk = _cat_tracks(parts)
    trk["t0"] = np.concatenate(t0)
    cr = _chunked_crossings(trk, geom["row_x"])
    inst = _sector_instances(cr)
    zmeas = cr["z"] - np.sign(cr["z"]) * V_DRIFT * trk["t0"][cr["trk"]]
    shift = V_DRIFT * t_window_us
    zr = [(-shift, Z_MAX)] * N_PHI + [(-Z_MAX, shift)] * N_PHI
    return _assemble(rng, "config3", seed, geom, inst, 2 * N_PHI, list(range(N_PHI)) * 2, cr,
                     zmeas, cr["trk"], noise, zr, trk)


def config4(rep=0, n_inst=256, n_min=1e3, n_max=4e5, scale=1.0) -> Event:
    """256 independent wedge instances of very uneven occupancy.

    Per instance: a target count N ~ logU(n_min, n_max) (times ``scale``) and a
    noise fraction f ~ U(0, 0.2); config-1-like tracks are added until the
    signal reaches N(1-f), then noise brings the instance to about N.
    """
    seed = SEED_BASE + 4 + 0x100 * rep
    rng = np.random.Generator(np.random.PCG64(seed))
    geom = geometry()
    target = np.exp(rng.uniform(np.log(n_min), np.log(n_max), n_inst)) * scale
    frac = rng.uniform(0, 0.2, n_inst)
    parts_trk, parts_cr, inst_parts = [], [], []
    id0 = 0
    for i in range(n_inst):
        want = target[i] * (1 - frac[i])
        est = max(4, int(want / 90.0 * 1.3))
        trk = _wedge_tracks(rng, est)
        cr = _chunked_crossings(trk, geom["row_x"], sectors=[0])
        per = np.bincount(cr["trk"], minlength=est)
        ntk = int(np.searchsorted(np.cumsum(per), want) + 1)
        while ntk > est:      # not enough: draw more
            more = _wedge_tracks(rng, est)
            trk = _cat_tracks([trk, more])
            cr = _chunked_crossings(trk, geom["row_x"], sectors=[0])
            est = len(trk["q"])
            per = np.bincount(cr["trk"], minlength=est)
            ntk = int(np.searchsorted(np.cumsum(per), want) + 1)
        keep = cr["trk"] < ntk
        cr = {k: v[keep] for k, v in cr.items()}
        trk = {k: v[:ntk] for k, v in trk.items()}
        cr["trk"] = cr["trk"] + id0
        id0 += ntk
        parts_trk.append(trk)
        parts_cr.append(cr)
        inst_parts.append(np.full(len(cr["row"]), i))
    trk = _cat_tracks(parts_trk)
    cr = {k: np.concatenate([c[k] for c in parts_cr]) for k in parts_cr[0]}
    inst = np.concatenate(inst_parts)
    nf = frac / (1 - frac)
    ev = _assemble(rng, "config4", seed, geom, inst, n_inst, [0] * n_inst, cr, cr["z"], cr["trk"],
                   nf, [(-Z_MAX, Z_MAX)] * n_inst, trk)
    ev.extra["target"] = target
    ev.extra["noise_frac"] = frac
    return ev


def distortion_map(rng, amp=1.0) -> np.ndarray:
    """Smooth random radial distortion D[row][phi-sector] (cm), max |D| = amp."""
    r = np.arange(N_ROWS)[:, None] / (N_ROWS - 1)
    k = np.arange(N_PHI)[None, :]
    D = np.zeros((N_ROWS, N_PHI))
    for m in range(3):
        for n in range(3):
            a = rng.normal()
            pr, pk = rng.uniform(0, 2 * np.pi, 2)
            D += a * np.cos(np.pi * m * r + pr) * np.cos(2 * np.pi * n * k / N_PHI + pk)
    return D * (amp / np.abs(D).max())


def config5(rep=0, n_found=200_000, min_hits=10, smear=True, amp=1.0) -> Event:
    """Found-track hit lists (MC truth, one list per track and sector instance,
    the part of the outgoing leg with |snp| < 0.95) for the Kalman refit; true
    hits lie on planes x_r + D_true[r][k] while the clusters record x_r."""
    seed = SEED_BASE + 5 + 0x100 * rep
    rng = np.random.Generator(np.random.PCG64(seed))
    geom = geometry()
    D = distortion_map(rng, amp)
    segs_cr, parts_trk = [], []
    got, id0 = 0, 0
    while got < n_found:
        trk = _central_tracks(rng, 8000, rng.normal(0, 5.0))
        cr = _chunked_crossings(trk, geom["row_x"], dist=D)
        # a tracker follows a track while |snp| stays well below 1 (loopers
        # turn over at the end of the outgoing leg): keep that part
        keep = np.abs(cr["snp"]) < 0.95
        cr = {k: v[keep] for k, v in cr.items()}
        cr["trk"] = cr["trk"] + id0
        id0 += 8000
        parts_trk.append(trk)
        key = (cr["trk"] * 64 + _sector_instances(cr)).astype(np.int64)
        order = np.lexsort((cr["row"], key))
        cr = {k: v[order] for k, v in cr.items()}
        key = key[order]
        uk, start, cnt = np.unique(key, return_index=True, return_counts=True)
        ok = cnt >= min_hits
        sel_start, sel_cnt = start[ok], cnt[ok]
        take = min(len(sel_start), n_found - got)
        sel_start, sel_cnt = sel_start[:take], sel_cnt[:take]
        idx = np.concatenate([np.arange(s, s + c) for s, c in zip(sel_start, sel_cnt)]) \
            if take else np.zeros(0, np.int64)
        segs_cr.append(({k: v[idx] for k, v in cr.items()}, sel_cnt))
        got += take
    trk = _cat_tracks(parts_trk)
    cr = {k: np.concatenate([s[0][k] for s in segs_cr]) for k in segs_cr[0][0]}
    cnt = np.concatenate([s[1] for s in segs_cr])
    n = len(cr["row"])
    hit_off = np.zeros(len(cnt) + 1, np.int64)
    hit_off[1:] = np.cumsum(cnt)
    row_x = geom["row_x"]
    y = (cr["y"] + (rng.normal(0, SIGMA_Y, n) if smear else 0.0)).astype(np.float32)
    z = (cr["z"] + (rng.normal(0, SIGMA_Z, n) if smear else 0.0)).astype(np.float32)
    row = cr["row"].astype(np.uint16)
    first = hit_off[:-1]
    q = trk["q"][cr["trk"][first]]
    pt = trk["pt"][cr["trk"][first]]
    seed_par = np.zeros((len(cnt), 5), np.float32)
    seed_par[:, 0] = y[first]
    seed_par[:, 1] = z[first]
    seed_par[:, 2] = cr["snp"][first]
    seed_par[:, 3] = trk["tanl"][cr["trk"][first]]
    seed_par[:, 4] = q / pt
    ev = Event(name="config5", seed=seed, x=row_x[row], y=y, z=z, row=row,
               charge=rng.integers(20, 400, n).astype(np.uint16),
               inst_off=np.array([0, n], np.int64), label=cr["trk"].astype(np.int32),
               sector=cr["sec"].astype(np.uint8), inst_sector=np.zeros(1, np.int32), tracks=trk)
    ev.extra.update(hit_off=hit_off.astype(np.int32), hit_clu=np.arange(n, dtype=np.int32),
                    seed_par=seed_par, D_true=D.astype(np.float32))
    return ev


def make(config: int, **kw) -> Event:
    return {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}[config](**kw)


# ---------------------------------------------------------------------------
# readout encoding for the cluster coordinate transformation (f3)

T_BIN_US = 0.2                    # time-bin length (5 MHz sampling)
PAD_W_INNER, PAD_W_OUTER = 0.42, 0.60   # pad widths [cm], rows < 63 and >= 63
N_ROWS_INNER = 63


def transform_geometry(nu=16, nv=9, nw=26, t0_us=0.0) -> dict:
    """Readout description of the pad rows and the drift (detector data for
    both implementations): pad width and centre pad per row, time-bin
    length, drift velocity and length, the call's time offset, and the
    residual-correction grid (nu nodes over the rows, nv over y/x beyond the
    sector edges, nw over the drift distance)."""
    g = geometry()
    r = np.arange(N_ROWS)
    pad_w = np.where(r < N_ROWS_INNER, PAD_W_INNER, PAD_W_OUTER)
    tan_half = np.tan(np.radians(SECTOR_DEG / 2))
    n_pads = 2 * np.ceil((g["row_x"].astype(np.float64) * tan_half + 2.0) / pad_w)
    vmax = 1.05 * tan_half
    return dict(row_x=g["row_x"], pad_w=pad_w.astype(np.float32),
                pad_c=((n_pads - 1) / 2).astype(np.float32), n_pads=n_pads.astype(np.int32),
                tbin=np.float32(T_BIN_US), vdrift=np.float32(V_DRIFT), zlen=np.float32(Z_MAX),
                t0=np.float32(t0_us), nu=nu, nv=nv, nw=nw,
                u0=np.float32(0.0), iu=np.float32((nu - 1) / (N_ROWS - 1)),
                v0=np.float32(-vmax), iv=np.float32((nv - 1) / (2 * vmax)),
                w0=np.float32(0.0), iw=np.float32((nw - 1) / Z_MAX))


def cluster_sides(ev: Event) -> np.ndarray:
    """Readout side of every cluster (1 = C, negative z): the instance's side
    where instances are (sector, side) pairs, else the sign of z."""
    if ev.n_inst == 2 * N_PHI and ev.name in ("config2", "config3"):
        inst = np.repeat(np.arange(ev.n_inst), np.diff(ev.inst_off))
        return (inst >= N_PHI).astype(np.uint8)
    return (ev.z < 0).astype(np.uint8)


class Distortion:
    """A smooth space-point distortion per sector instance (36): each
    transverse component (y, z) is a sum of three products of cosines in the
    row fraction, y/x and the drift distance, with seeded amplitudes and
    phases, at most `amp` cm.  Physics of the generator, not of the
    method: measured position = true position + d(true position)."""

    def __init__(self, amp=0.5, seed=SEED_BASE + 0x31):
        rng = np.random.Generator(np.random.PCG64(seed))
        self.amp = amp
        self.k = rng.integers(1, 4, (36, 3, 3, 3)).astype(np.float64)
        self.ph = rng.uniform(0, 2 * np.pi, (36, 3, 3, 3))
        self.a = rng.uniform(-1, 1, (36, 3, 3)) * amp / 3
        # no radial component: a cluster is read on its pad row's plane
        # (radial plane displacements are the refit's map D)
        self.a[:, 0, :] = 0.0

    def __call__(self, s, x, y, z):
        """d(x, y, z) of sector instances s (arrays): [3, n] in cm."""
        s = np.asarray(s, np.int64)
        u = (np.asarray(x, np.float64) - X_INNER) / (X_OUTER - X_INNER)
        v = np.asarray(y, np.float64) / np.asarray(x, np.float64) / np.tan(np.radians(10)) / 2
        w = (Z_MAX - np.abs(np.asarray(z, np.float64))) / Z_MAX
        out = np.zeros((3, len(s)))
        for q in range(3):
            for m in range(3):
                k, ph = self.k[s, q, m], self.ph[s, q, m]
                out[q] += self.a[s, q, m] * (np.cos(np.pi * k[:, 0] * u + ph[:, 0])
                                             * np.cos(np.pi * k[:, 1] * v + ph[:, 1])
                                             * np.cos(np.pi * k[:, 2] * w + ph[:, 2]))
        return out


def calibration_map(tg: dict, dist: Distortion) -> np.ndarray:
    """The residual-correction map that undoes `dist` to first order: minus
    the distortion at the grid nodes, float32 [36, nu, nv, nw, 4]."""
    nu, nv, nw = tg["nu"], tg["nv"], tg["nw"]
    u = np.float64(tg["u0"]) + np.arange(nu) / np.float64(tg["iu"])
    v = np.float64(tg["v0"]) + np.arange(nv) / np.float64(tg["iv"])
    w = np.float64(tg["w0"]) + np.arange(nw) / np.float64(tg["iw"])
    U, V, W = np.meshgrid(u, v, w, indexing="ij")
    x = X_INNER + U * (X_OUTER - X_INNER) / (N_ROWS - 1)
    y = V * x
    out = np.zeros((36, nu, nv, nw, 4), np.float32)
    for s in range(36):
        zs = (Z_MAX - W) * (-1.0 if s >= N_PHI else 1.0)
        d = dist(np.full(x.size, s), x.ravel(), y.ravel(), zs.ravel())
        for q in range(3):
            out[s, ..., q] = (-d[q]).reshape(U.shape)
    return out


def encode_raw(ev: Event, tg: dict, dist: Distortion | None = None,
               dmap: np.ndarray | None = None) -> dict:
    """Readout coordinates of the event's clusters (binary64, rounded to
    binary32 at the end): sector instance k + 18 side, row, pad, time.  With
    `dist` the clusters are first displaced by the distortion (their
    measured position); with `dmap` their plane is taken at x_r + D[r][k]
    (a radial displacement the transformation's radial offset undoes)."""
    side = cluster_sides(ev)
    s = ev.sector.astype(np.int64) + N_PHI * side.astype(np.int64)
    x = tg["row_x"][ev.row].astype(np.float64)
    y = ev.y.astype(np.float64)
    z = ev.z.astype(np.float64)
    if dist is not None:
        d = dist(s, x, y, z)
        y = y + d[1]
        z = z + d[2]
    pad = y / tg["pad_w"][ev.row].astype(np.float64) + tg["pad_c"][ev.row].astype(np.float64)
    sgn = np.where(side == 1, -1.0, 1.0)
    drift = np.float64(tg["zlen"]) - sgn * z
    time = (drift / np.float64(tg["vdrift"]) + np.float64(tg["t0"])) / np.float64(tg["tbin"])
    return dict(sector=s.astype(np.uint8), row=ev.row.copy(), pad=pad.astype(np.float32),
                time=time.astype(np.float32))


# ---------------------------------------------------------------------------
# tracks through a non-uniform field and material (refit with f2)

M_PION = 0.13957                  # GeV


def field_map(nzb=25, amp=0.03) -> np.ndarray:
    """A smooth solenoid field [T] per (row, z bin): 0.5 T, varying by up to
    1.5 `amp` (relative) with radius and z, not symmetric in z --
    piecewise constant per cell, as the refit reads it."""
    g = geometry()
    xr = g["row_x"].astype(np.float64)
    zc = -Z_MAX + (np.arange(nzb) + 0.5) * (2 * Z_MAX / nzb)
    u = (xr - X_INNER) / (X_OUTER - X_INNER)
    return (B_TESLA * (1 + amp * np.cos(np.pi * u)[:, None] * np.cos(np.pi * zc / Z_MAX)[None, :]
                       + 0.5 * amp * np.sin(np.pi * zc / (2 * Z_MAX))[None, :])).astype(np.float32)


def material_map(scale=1.0):
    """Inverse radiation length [1/cm] and mean energy loss at minimum
    ionisation [GeV/cm] per row: a Ne-CO2-N2-like gas (X0 ~ 86 m, about
    3.2 MeV per metre), times `scale`."""
    ix0 = np.full(N_ROWS, scale / 8600.0, np.float32)
    eloss = np.full(N_ROWS, scale * 3.2e-6, np.float32)
    return ix0, eloss


def _zbin(z, nzb):
    f = np.floor((z + Z_MAX) * nzb / (2 * Z_MAX))
    return np.clip(np.where(np.isfinite(f), f, 0), 0, nzb - 1).astype(np.int64)


def material_tracks(n=400, rep=0, bz=None, ix0=None, eloss=None, smear=True, pt_range=(0.15, 2.0),
                    with_material=True) -> Event:
    """Tracks of one sector (the local frame of sector 0, side A), simulated
    row by row in binary64: an exact helix step between the pad-row planes
    in the field of the destination cell (`bz` [152, nzb], or 0.5 T), then,
    with material, a random multiple-scattering kick (Highland width without
    its logarithm, both directions perpendicular to the track) and the mean
    energy loss (dE/dx = K / beta^2, exact in energy), for pions.  One hit
    per row, smeared; a track stops at |sin phi| > 0.95, the sector edge or
    |z| > 250 cm.  Returns an Event with the refit's hit lists, the true
    (snp, tgl, q/pt) at the first hit as seeds and the true q/pt at the
    last hit (extra "qpt_last")."""
    seed = SEED_BASE + 0x52 + 0x100 * rep
    rng = np.random.Generator(np.random.PCG64(seed))
    g = geometry()
    xr = g["row_x"].astype(np.float64)
    tan_half = np.tan(np.radians(SECTOR_DEG / 2))
    ys, zs, rows, counts, seeds, truth_qpt = [], [], [], [], [], []   # q/pt at the last hit
    while len(counts) < n:
        pt = np.exp(rng.uniform(np.log(pt_range[0]), np.log(pt_range[1])))
        q = rng.choice([-1.0, 1.0])
        lam = np.arctan(np.sinh(rng.uniform(-0.9, 0.9)))
        phi = rng.uniform(-0.3, 0.3)
        p = pt / np.cos(lam)
        y = rng.uniform(-0.1, 0.1) * xr[0]
        z = rng.uniform(-20, 20)
        hy, hz, hr = [y], [z], [0]
        sd = (np.sin(phi), np.tan(lam), q / (p * np.cos(lam)))
        for r in range(1, N_ROWS):
            B = float(bz[r, _zbin(np.array([z]), bz.shape[1])[0]]) if bz is not None else B_TESLA
            C = -C_LIGHT * B * q / (p * np.cos(lam))
            dx = xr[r] - xr[r - 1]
            s1 = np.sin(phi) + C * dx
            if abs(s1) > 0.95:
                break
            phi1 = np.arcsin(s1)
            if abs(C) > 1e-12:
                y = y + (np.cos(phi) - np.cos(phi1)) / C
                arc = (phi1 - phi) / C
            else:
                y = y + dx * np.tan(phi)
                arc = dx / np.cos(phi)
            z = z + np.tan(lam) * arc
            phi = phi1
            if abs(y) > xr[r] * tan_half or abs(z) > Z_MAX:
                break
            if with_material and ix0 is not None:
                path = abs(arc) / np.cos(lam)
                e = np.sqrt(p * p + M_PION ** 2)
                beta2 = p * p / (e * e)
                th = np.sqrt(0.0136 ** 2 * path * float(ix0[r]) / (beta2 * p * p))
                phi += rng.normal(0, th) / np.cos(lam)
                lam += rng.normal(0, th)
                e -= float(eloss[r]) / beta2 * path
                if e <= M_PION * 1.01:
                    break
                p = np.sqrt(e * e - M_PION ** 2)
            hy.append(y)
            hz.append(z)
            hr.append(r)
        if len(hr) < 20:
            continue
        ys += hy
        zs += hz
        rows += hr
        counts.append(len(hr))
        seeds.append(sd)
        truth_qpt.append(q / (p * np.cos(lam)))
    m = len(rows)
    hit_off = np.zeros(n + 1, np.int64)
    hit_off[1:] = np.cumsum(counts)
    y = np.array(ys) + (rng.normal(0, SIGMA_Y, m) if smear else 0.0)
    z = np.array(zs) + (rng.normal(0, SIGMA_Z, m) if smear else 0.0)
    row = np.array(rows, np.uint16)
    sp = np.zeros((n, 5), np.float32)
    first = hit_off[:-1]
    sp[:, 0] = y[first]
    sp[:, 1] = z[first]
    sp[:, 2:] = np.array(seeds)
    ev = Event(name="material", seed=seed, x=g["row_x"][row], y=y.astype(np.float32),
               z=z.astype(np.float32), row=row, charge=np.zeros(m, np.uint16),
               inst_off=np.array([0, m], np.int64), label=np.repeat(np.arange(n), counts),
               sector=np.zeros(m, np.uint8), inst_sector=np.zeros(1, np.int32))
    ev.extra.update(hit_off=hit_off.astype(np.int32), hit_clu=np.arange(m, dtype=np.int32),
                    seed_par=sp, qpt_last=np.array(truth_qpt))
    return ev
