"""CPU oracle of the TPC sector tracker -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package; the product library never does.  It wraps ``liboracle.so``
(built from ``tpc_oracle.c`` twice: binary32 without FP contraction for the
bit-exact comparison, binary64 for accuracy references) with numpy arrays.

Stages follow the readings documented with the C source: grid (a1),
neighbours (a2), cleaner (a3), start hits (a4), tracklets (a5), selection
(a6), refit and adjoint (a8/a9).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.environ.get("TPC_ORACLE_LIB", os.path.join(HERE, "liboracle.so"))
N_ROWS_MAX = 152

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-Wall",
          "-Wno-unused-function"]


def build(force: bool = True, out: str | None = None, srcdir: str | None = None,
          extra: tuple = ()) -> str:
    """Compile liboracle.so with gcc (binary32 and binary64 objects; the
    refit also as complex binary64) from the C sources in `srcdir`; `extra`
    flags go to every compile and the link (e.g. sanitizers)."""
    out = out or LIB
    if not force and os.path.exists(out):
        return out
    srcdir = srcdir or HERE
    objs = []
    for name, tags in (("tpc_oracle.c", (("f32", []), ("f64", ["-DORC_F64"]),
                                         ("f32c", ["-DORC_F32C", "-mfma",
                                                   "-ffp-contract=fast"]))),
                       ("tpc_refit.c", (("rf32", []), ("rf64", ["-DORC_F64"]),
                                        ("rc128", ["-DORC_C128"]))),
                       ("tpc_transform.c", (("tf32", []), ("tf64", ["-DORC_F64"]))),
                       ("tpc_merge.c", (("mf32", []), ("mf64", ["-DORC_F64"])))):
        for tag, defs in tags:
            obj = out + f".{tag}.o"
            subprocess.run(["gcc", *CFLAGS, *extra, *defs, "-I", srcdir, "-c",
                            os.path.join(srcdir, name), "-o", obj], check=True)
            objs.append(obj)
    tmp = out + ".tmp"
    subprocess.run(["gcc", "-shared", *extra, "-o", tmp, *objs, "-lm"], check=True)
    os.replace(tmp, out)
    for o in objs:
        os.remove(o)
    return out


class Geom(C.Structure):
    _fields_ = [("n_rows", C.c_int32), ("row_x", C.c_float * N_ROWS_MAX), ("bz", C.c_float),
                ("tan_half", C.c_float), ("sigma_y2", C.c_float), ("sigma_z2", C.c_float)]


class Params(C.Structure):
    _fields_ = [("nf_win_y", C.c_float), ("nf_win_z", C.c_float), ("nf_chi2_max", C.c_float),
                ("tc_chi2_pick", C.c_float), ("snp_max", C.c_float),
                ("grid_occupancy", C.c_float), ("edge_margin", C.c_float),
                ("search_margin", C.c_float), ("y_valid_margin", C.c_float),
                ("min_chain", C.c_int32), ("tc_max_miss", C.c_int32),
                ("min_tracklet_hits", C.c_int32), ("min_track_hits", C.c_int32)]


DEFAULT_PARAMS = dict(nf_win_y=3.0, nf_win_z=3.5, nf_chi2_max=13.8, tc_chi2_pick=13.8,
                      snp_max=0.99, grid_occupancy=2.0, edge_margin=1.0, search_margin=0.01,
                      y_valid_margin=2.0, min_chain=3, tc_max_miss=10, min_tracklet_hits=10,
                      min_track_hits=10)


def make_geom(geom: dict) -> Geom:
    g = Geom()
    g.n_rows = int(geom["n_rows"])
    rx = np.asarray(geom["row_x"], np.float32)
    for r in range(g.n_rows):
        g.row_x[r] = float(rx[r])
    g.bz = float(geom["bz"])
    g.tan_half = float(geom["tan_half"])
    g.sigma_y2 = float(geom["sigma_y2"])
    g.sigma_z2 = float(geom["sigma_z2"])
    return g


def make_params(**over) -> Params:
    p = Params()
    d = dict(DEFAULT_PARAMS)
    d.update(over)
    for k, v in d.items():
        setattr(p, k, v)
    return p


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = C.CDLL(LIB)
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _dt(prec):
    return np.float64 if prec == 64 else np.float32


def _fn(name, prec):
    # prec 32, 64, or "32c" (binary32 with fused multiply-add)
    return getattr(lib(), f"{name}_f{prec}")


@dataclass
class Grid:
    sseg: np.ndarray
    row_off: np.ndarray
    meta_i: np.ndarray
    meta_f: np.ndarray
    bin_off: np.ndarray
    perm: np.ndarray
    ys: np.ndarray
    zs: np.ndarray
    n_bad: int
    n_bins: int


def grid_build(geom, params, inst_off, y, z, row, prec=32) -> Grid:
    g, P = make_geom(geom), params if isinstance(params, Params) else make_params(**params)
    n_inst = len(inst_off) - 1
    n = int(inst_off[-1])
    nr = g.n_rows
    inst_off = np.ascontiguousarray(inst_off, np.int64)
    y = np.ascontiguousarray(y, np.float32)
    z = np.ascontiguousarray(z, np.float32)
    row = np.ascontiguousarray(row, np.uint16)
    dt = _dt(prec)
    sseg = np.empty(n, np.int32)
    perm = np.empty(n, np.int32)
    ys = np.empty(n, dt)
    zs = np.empty(n, dt)
    row_off = np.empty(n_inst * (nr + 1), np.int32)
    meta_i = np.empty((n_inst * nr, 4), np.int32)
    meta_f = np.empty((n_inst * nr, 4), dt)
    cap = int(np.ceil(5.0 * n / P.grid_occupancy)) + 10 * nr * n_inst + 16
    bin_off = np.empty(cap, np.int32)
    nbad = C.c_int64(0)
    f = _fn("orc_grid_build", prec)
    f.restype = C.c_int64
    used = f(C.byref(g), C.byref(P), C.c_int32(n_inst), _p(inst_off), _p(y), _p(z), _p(row),
             _p(sseg), _p(row_off), _p(meta_i), _p(meta_f), _p(bin_off), C.c_int64(cap),
             _p(perm), _p(ys), _p(zs), C.byref(nbad))
    if used < 0:
        raise RuntimeError("oracle grid: bin capacity exceeded")
    return Grid(sseg, row_off, meta_i, meta_f, bin_off[:used].copy(), perm, ys, zs,
                int(nbad.value), int(used))


def neighbours(geom, params, grid: Grid, prec=32, brute=False):
    g, P = make_geom(geom), params if isinstance(params, Params) else make_params(**params)
    n = len(grid.sseg)
    up = np.empty(n, np.int32)
    dn = np.empty(n, np.int32)
    f = _fn("orc_neighbours", prec)
    f.restype = None
    f(C.byref(g), C.byref(P), C.c_int64(n), _p(grid.sseg), _p(grid.row_off), _p(grid.meta_i),
      _p(grid.meta_f), _p(grid.bin_off), _p(grid.perm), _p(grid.ys), _p(grid.zs), _p(up), _p(dn),
      C.c_int(1 if brute else 0))
    return up, dn


def clean(up, dn, prec=32):
    n = len(up)
    up2 = np.empty(n, np.int32)
    dn2 = np.empty(n, np.int32)
    f = _fn("orc_clean", prec)
    f.restype = None
    f(C.c_int64(n), _p(np.ascontiguousarray(up, np.int32)), _p(np.ascontiguousarray(dn, np.int32)),
      _p(up2), _p(dn2))
    return up2, dn2


def start_hits(params, up2, dn2, prec=32):
    P = params if isinstance(params, Params) else make_params(**params)
    n = len(up2)
    st = np.empty(max(1, n), np.int32)
    f = _fn("orc_start_hits", prec)
    f.restype = C.c_int64
    S = f(C.byref(P), C.c_int64(n), _p(up2), _p(dn2), _p(st))
    return st[:S].copy()


@dataclass
class Tracklets:
    par: np.ndarray     # [S,5]
    cov: np.ndarray     # [S,15]
    chi2: np.ndarray
    nhit: np.ndarray
    rmin: np.ndarray
    rmax: np.ndarray
    hit: np.ndarray     # [S, n_rows]
    status: np.ndarray


def tracklets(geom, params, grid: Grid, start, up2, prec=32) -> Tracklets:
    g, P = make_geom(geom), params if isinstance(params, Params) else make_params(**params)
    S = len(start)
    dt = _dt(prec)
    nr = g.n_rows
    Sa = max(S, 1)
    out = Tracklets(np.zeros((Sa, 5), dt), np.zeros((Sa, 15), dt), np.zeros(Sa, dt),
                    np.zeros(Sa, np.int32), np.zeros(Sa, np.int32), np.zeros(Sa, np.int32),
                    np.full((Sa, nr), -1, np.int32), np.zeros(Sa, np.int32))
    f = _fn("orc_tracklets", prec)
    f.restype = None
    f(C.byref(g), C.byref(P), C.c_int64(S), _p(np.ascontiguousarray(start, np.int32)),
      _p(up2), _p(grid.sseg), _p(grid.row_off), _p(grid.meta_i), _p(grid.meta_f),
      _p(grid.bin_off), _p(grid.perm), _p(grid.ys), _p(grid.zs), _p(out.par), _p(out.cov),
      _p(out.chi2), _p(out.nhit), _p(out.rmin), _p(out.rmax), _p(out.hit), _p(out.status))
    if S == 0:
        out = Tracklets(*(a[:0] for a in (out.par, out.cov, out.chi2, out.nhit, out.rmin,
                                          out.rmax, out.hit, out.status)))
    return out


@dataclass
class Tracks:
    par: np.ndarray
    cov: np.ndarray
    chi2: np.ndarray
    ndf: np.ndarray
    x_ref: np.ndarray
    hit_off: np.ndarray
    hit_clu: np.ndarray
    clu2trk: np.ndarray
    owner: np.ndarray
    need_tracks: int
    need_hits: int


def select(geom, params, inst_off, grid: Grid, start, tl: Tracklets, prec=32,
           cap_tracks=None, cap_hits=None) -> Tracks:
    g, P = make_geom(geom), params if isinstance(params, Params) else make_params(**params)
    n = len(grid.sseg)
    S = len(start)
    dt = _dt(prec)
    ct = S if cap_tracks is None else cap_tracks
    ch = n if cap_hits is None else cap_hits
    owner = np.zeros(max(n, 1), np.uint64)
    tpar = np.zeros((max(ct, 1), 5), dt)
    tcov = np.zeros((max(ct, 1), 15), dt)
    tchi2 = np.zeros(max(ct, 1), dt)
    tndf = np.zeros(max(ct, 1), np.int32)
    txref = np.zeros(max(ct, 1), np.float32)
    thoff = np.zeros(ct + 1, np.int32)
    thclu = np.zeros(max(ch, 1), np.int32)
    clu2trk = np.full(max(n, 1), -1, np.int32)
    nh = C.c_int64(0)
    need_t = C.c_int64(0)
    need_h = C.c_int64(0)
    Sa = max(S, 1)

    def arr(a, dtp, shape):
        return np.ascontiguousarray(a, dtp) if S else np.zeros(shape, dtp)

    f = _fn("orc_select", prec)
    f.restype = C.c_int64
    nt = f(C.byref(g), C.byref(P), C.c_int64(n), C.c_int64(S),
           _p(np.ascontiguousarray(inst_off, np.int64)), _p(arr(start, np.int32, Sa)),
           _p(grid.sseg), _p(grid.perm), _p(arr(tl.par, dt, (Sa, 5))),
           _p(arr(tl.cov, dt, (Sa, 15))), _p(arr(tl.chi2, dt, Sa)), _p(arr(tl.nhit, np.int32, Sa)),
           _p(arr(tl.rmin, np.int32, Sa)), _p(arr(tl.rmax, np.int32, Sa)),
           _p(arr(tl.hit, np.int32, (Sa, g.n_rows))), _p(arr(tl.status, np.int32, Sa)),
           _p(owner), C.c_int64(ct), C.c_int64(ch), _p(tpar), _p(tcov), _p(tchi2), _p(tndf),
           _p(txref), _p(thoff), _p(thclu), _p(clu2trk), C.byref(nh), C.byref(need_t),
           C.byref(need_h))
    return Tracks(tpar[:nt], tcov[:nt], tchi2[:nt], tndf[:nt], txref[:nt], thoff[:nt + 1],
                  thclu[:nh.value], clu2trk[:n], owner[:n], int(need_t.value), int(need_h.value))


@dataclass
class ChainResult:
    grid: Grid
    up: np.ndarray
    dn: np.ndarray
    up2: np.ndarray
    dn2: np.ndarray
    start: np.ndarray
    tracklets: Tracklets
    tracks: Tracks


def track(geom, params, inst_off, y, z, row, prec=32) -> ChainResult:
    """The whole sector-tracking chain a1..a6, one stage after the other."""
    gr = grid_build(geom, params, inst_off, y, z, row, prec)
    up, dn = neighbours(geom, params, gr, prec)
    up2, dn2 = clean(up, dn, prec)
    st = start_hits(params, up2, dn2, prec)
    tl = tracklets(geom, params, gr, st, up2, prec)
    tr = select(geom, params, inst_off, gr, st, tl, prec)
    return ChainResult(gr, up, dn, up2, dn2, st, tl, tr)


def replay(geom, params, r0, rmin, rmax, hy, hz, has, prec=64):
    """Re-run a tracklet's filter sequence on a fixed per-row hit list."""
    g, P = make_geom(geom), params if isinstance(params, Params) else make_params(**params)
    dt = _dt(prec)
    par = np.zeros(5, dt)
    cov = np.zeros(15, dt)
    chi2 = (C.c_double if prec == 64 else C.c_float)(0)
    f = _fn("orc_replay", prec)
    f.restype = C.c_int
    ok = f(C.byref(g), C.byref(P), C.c_int(int(r0)), C.c_int(int(rmin)), C.c_int(int(rmax)),
           _p(np.ascontiguousarray(hy, np.float32)), _p(np.ascontiguousarray(hz, np.float32)),
           _p(np.ascontiguousarray(has, np.uint8)), _p(par), _p(cov), C.byref(chi2))
    return bool(ok), par, cov, float(chi2.value)


def propagate(geom, params, p, c, x1, x2, prec=64):
    """One R7/R8 step of state p[5] and lower-triangular covariance c[15]."""
    g, P = make_geom(geom), params if isinstance(params, Params) else make_params(**params)
    dt = _dt(prec)
    p = np.array(p, dt)
    c = np.array(c, dt)
    f = _fn("orc_propagate", prec)
    f.restype = C.c_int
    sc = C.c_double if prec == 64 else C.c_float
    ok = f(C.byref(g), C.byref(P), _p(p), _p(c), sc(x1), sc(x2))
    return bool(ok), p, c


def update(geom, p, c, my, mz, prec=64):
    """One R9 measurement update; returns (chi2, p, c)."""
    g = make_geom(geom)
    dt = _dt(prec)
    p = np.array(p, dt)
    c = np.array(c, dt)
    f = _fn("orc_update", prec)
    sc = C.c_double if prec == 64 else C.c_float
    f.restype = sc
    ch = f(C.byref(g), _p(p), _p(c), sc(my), sc(mz))
    return float(ch), p, c


def underflow_raised(clear: bool = True) -> bool:
    """The IEEE underflow flag of this thread (R29: no operation of the
    binary32 reference may deliver a subnormal); clear resets it."""
    f = lib().orc_underflow_raised
    f.restype = C.c_int
    return bool(f(C.c_int(1 if clear else 0)))


# ----------------------------------------------------------------------------
# refit (a8) and its adjoint (a9)

def _refit_args(geom, params, ev_like, hit_off, hit_clu, seed, dmap):
    g, P = make_geom(geom), params if isinstance(params, Params) else make_params(**params)
    arrs = dict(hit_off=np.ascontiguousarray(hit_off, np.int32),
                hit_clu=np.ascontiguousarray(hit_clu, np.int32),
                sector=np.ascontiguousarray(ev_like.sector, np.uint8),
                x=np.ascontiguousarray(ev_like.x, np.float32),
                y=np.ascontiguousarray(ev_like.y, np.float32),
                z=np.ascontiguousarray(ev_like.z, np.float32),
                row=np.ascontiguousarray(ev_like.row, np.uint16),
                seed=np.ascontiguousarray(seed, np.float32),
                dmap=np.ascontiguousarray(dmap, np.float32))
    return g, P, arrs


def refit(geom, params, ev_like, hit_off, hit_clu, seed, dmap, prec=32, mat=None):
    """Forward refit: (chi2[n], status[n], ckpt[n_hits, 20]).  status 1: the
    propagation failed; 2: a hit names no cluster or a row beyond the map.
    `mat`: field map and material (R42-R44), see _material."""
    g, P, a = _refit_args(geom, params, ev_like, hit_off, hit_clu, seed, dmap)
    M = _material(mat)
    n = len(a["hit_off"]) - 1
    nh = int(a["hit_off"][-1])
    dt = _dt(prec)
    chi2 = np.zeros(max(n, 1), dt)
    status = np.zeros(max(n, 1), np.int32)
    ckpt = np.zeros((max(nh, 1), 20), dt)
    f = _fn("orc_refit", prec)
    f.restype = None
    f(C.byref(g), C.byref(P), C.byref(M), C.c_int64(n), _p(a["hit_off"]), _p(a["hit_clu"]), _p(a["sector"]),
      _p(a["x"]), _p(a["y"]), _p(a["z"]), _p(a["row"]), C.c_int64(len(a["x"])), _p(a["seed"]),
      _p(a["dmap"]), _p(chi2), _p(status), _p(ckpt))
    return chi2[:n], status[:n], ckpt[:nh]


class Material(C.Structure):
    _fields_ = [("bz", C.c_void_p), ("nzb", C.c_int32), ("ix0", C.c_void_p),
                ("eloss", C.c_void_p)]


def _material(mat):
    """orc_material from a dict with any of bz [152, nzb], ix0 [152],
    eloss [152] (None: uniform field, no material); the arrays are kept
    alive on the returned structure."""
    m = Material()
    if not mat:
        return m
    keep = []
    if mat.get("bz") is not None:
        b = np.ascontiguousarray(mat["bz"], np.float32)
        keep.append(b)
        m.bz, m.nzb = b.ctypes.data, b.shape[1]
    for name in ("ix0", "eloss"):
        if mat.get(name) is not None:
            a = np.ascontiguousarray(mat[name], np.float32)
            keep.append(a)
            setattr(m, name, a.ctypes.data)
    m._keep = keep
    return m


REFIT_WHICH = {"x": 0, "y": 1, "z": 2, "map": 3}


def refit_loss(geom, params, ev_like, hit_off, hit_clu, seed, dmap, w, which=None, idx=-1,
               h=0.0, mode="f64", mat=None):
    """sum_t w_t chi2_t with one input perturbed by h (mode f64 / f32), or
    the complex-step derivative w.r.t. that input (mode c128)."""
    g, P, a = _refit_args(geom, params, ev_like, hit_off, hit_clu, seed, dmap)
    M = _material(mat)
    n = len(a["hit_off"]) - 1
    w = np.ascontiguousarray(w, np.float64)
    f = getattr(lib(), f"orc_refit_loss_{mode}")
    f.restype = C.c_double
    return f(C.byref(g), C.byref(P), C.byref(M), C.c_int64(n), _p(a["hit_off"]), _p(a["hit_clu"]),
             _p(a["sector"]), _p(a["x"]), _p(a["y"]), _p(a["z"]), _p(a["row"]),
             C.c_int64(len(a["x"])), _p(a["seed"]), _p(a["dmap"]), _p(w), C.c_int(-1 if which is None else REFIT_WHICH[which]),
             C.c_int64(idx), C.c_double(h))


def refit_grad(geom, params, ev_like, hit_off, hit_clu, seed, dmap, w=None, ckpt=None,
               status=None, mat=None):
    """binary64 forward + reverse pass: (chi2, status, gmap[152,18], gx, gy, gz).
    With ckpt/status given (e.g. a binary32 forward's checkpoints) the reverse
    pass runs on those instead of the binary64 forward's."""
    chi2, st64, ck64 = refit(geom, params, ev_like, hit_off, hit_clu, seed, dmap, prec=64,
                             mat=mat)
    M = _material(mat)
    ckpt = ck64 if ckpt is None else ckpt
    status = st64 if status is None else status
    g, P, a = _refit_args(geom, params, ev_like, hit_off, hit_clu, seed, dmap)
    n = len(a["hit_off"]) - 1
    nc = len(a["x"])
    w = np.ones(n) if w is None else np.ascontiguousarray(w, np.float64)
    gmap = np.zeros(g.n_rows * 18)
    gx = np.zeros(max(nc, 1))
    gy = np.zeros(max(nc, 1))
    gz = np.zeros(max(nc, 1))
    f = lib().orc_refit_grad_f64
    f.restype = None
    ck = np.ascontiguousarray(ckpt, np.float64) if len(ckpt) else np.zeros((1, 20))
    f(C.byref(g), C.byref(P), C.byref(M), C.c_int64(n), _p(a["hit_off"]), _p(a["hit_clu"]), _p(a["sector"]),
      _p(a["x"]), _p(a["y"]), _p(a["z"]), _p(a["row"]), _p(a["seed"]), _p(a["dmap"]), _p(ck),
      _p(np.ascontiguousarray(status, np.int32)), _p(w), C.c_int64(nc), _p(gmap), _p(gx), _p(gy),
      _p(gz))
    return chi2, status, gmap.reshape(g.n_rows, 18), gx[:nc], gy[:nc], gz[:nc]


# ----------------------------------------------------------------------------
# cluster coordinate transformation (f3)

class TGeom(C.Structure):
    _fields_ = [("row_x", C.c_float * N_ROWS_MAX), ("pad_w", C.c_float * N_ROWS_MAX),
                ("pad_c", C.c_float * N_ROWS_MAX), ("tbin", C.c_float), ("vdrift", C.c_float),
                ("zlen", C.c_float), ("t0", C.c_float), ("nu", C.c_int32), ("nv", C.c_int32),
                ("nw", C.c_int32), ("u0", C.c_float), ("iu", C.c_float), ("v0", C.c_float),
                ("iv", C.c_float), ("w0", C.c_float), ("iw", C.c_float)]


def make_tgeom(tg: dict) -> TGeom:
    t = TGeom()
    for name in ("row_x", "pad_w", "pad_c"):
        arr = np.asarray(tg[name], np.float32)
        for r in range(N_ROWS_MAX):
            getattr(t, name)[r] = float(arr[r])
    for name in ("tbin", "vdrift", "zlen", "t0", "u0", "iu", "v0", "iv", "w0", "iw"):
        setattr(t, name, float(np.float32(tg[name])))
    for name in ("nu", "nv", "nw"):
        setattr(t, name, int(tg[name]))
    return t


def transform(tg: dict, sector, row, pad, time, dmap=None, rmap=None, prec=32):
    """R31-R34: raw clusters (sector, row, pad, time) to tracker inputs
    (x, y, z, row); dmap [152, 18] radial offsets, rmap [36, nu, nv, nw, 4]
    residual corrections (None: not applied)."""
    T = make_tgeom(tg)
    n = len(row)
    dt = _dt(prec)
    sector = np.ascontiguousarray(sector, np.uint8)
    row = np.ascontiguousarray(row, np.uint16)
    pad = np.ascontiguousarray(pad, np.float32)
    time = np.ascontiguousarray(time, np.float32)
    dm = None if dmap is None else np.ascontiguousarray(dmap, np.float32)
    rm = None if rmap is None else np.ascontiguousarray(rmap, np.float32)
    x = np.empty(max(n, 1), dt)
    y = np.empty(max(n, 1), dt)
    z = np.empty(max(n, 1), dt)
    ro = np.empty(max(n, 1), np.uint16)
    f = getattr(lib(), f"orc_transform_f{prec}")
    f.restype = None
    f(C.byref(T), C.c_int64(n), _p(sector), _p(row), _p(pad), _p(time),
      _p(dm) if dm is not None else None, _p(rm) if rm is not None else None,
      _p(x), _p(y), _p(z), _p(ro))
    return x[:n], y[:n], z[:n], ro[:n]


# ----------------------------------------------------------------------------
# sector-track merging and the global refit (f1)

class MParams(C.Structure):
    _fields_ = [("max_dz", C.c_float), ("max_dist", C.c_float), ("chi2_max", C.c_float),
                ("cos_a", C.c_float * 18), ("sin_a", C.c_float * 18), ("cos_d", C.c_float),
                ("sin_d", C.c_float)]


DEFAULT_MERGE = dict(max_dz=20.0, max_dist=40.0, chi2_max=30.0)


def make_mparams(**over) -> MParams:
    d = dict(DEFAULT_MERGE)
    d.update(over)
    m = MParams()
    m.max_dz, m.max_dist, m.chi2_max = d["max_dz"], d["max_dist"], d["chi2_max"]
    for k in range(18):
        a = np.radians(20.0 * (k + 0.5))
        m.cos_a[k] = float(np.float32(np.cos(a)))
        m.sin_a[k] = float(np.float32(np.sin(a)))
    m.cos_d = float(np.float32(np.cos(np.radians(20.0))))
    m.sin_d = float(np.float32(np.sin(np.radians(20.0))))
    return m


@dataclass
class Merged:
    out_ok: np.ndarray
    out_p: np.ndarray
    out_c: np.ndarray
    out_x: np.ndarray
    succ: np.ndarray
    pred: np.ndarray
    succ_chi2: np.ndarray
    pred_chi2: np.ndarray
    next: np.ndarray
    chain_off: np.ndarray
    chain_seg: np.ndarray
    hit_off: np.ndarray
    hit_clu: np.ndarray
    par: np.ndarray
    cov: np.ndarray
    chi2: np.ndarray
    ndf: np.ndarray
    status: np.ndarray
    k: np.ndarray
    x_ref: np.ndarray


def merge(geom, inst_off, y, z, row, tracks, prec=32, **mover) -> Merged:
    """R35-R41 on the sector tracker's tracks (an oracle.Tracks, or any
    object with par, cov, x_ref, hit_off, hit_clu) of the 36 sector
    instances."""
    g = make_geom(geom)
    M = make_mparams(**mover)
    dt = _dt(prec)
    n = len(tracks.hit_off) - 1
    na = max(n, 1)
    par = np.ascontiguousarray(tracks.par, dt).reshape(-1)
    cov = np.ascontiguousarray(tracks.cov, dt).reshape(-1)
    xr = np.ascontiguousarray(tracks.x_ref, np.float32)
    ho = np.ascontiguousarray(tracks.hit_off, np.int32)
    hc = np.ascontiguousarray(tracks.hit_clu, np.int32)
    nh = int(ho[-1])
    r = Merged(np.zeros(na, np.int32), np.zeros((na, 5), dt), np.zeros((na, 15), dt),
               np.zeros(na, dt), np.zeros(na, np.int32), np.zeros(na, np.int32), np.zeros(na, dt),
               np.zeros(na, dt), np.zeros(na, np.int32), np.zeros(na + 1, np.int32),
               np.zeros(na, np.int32), np.zeros(na + 1, np.int32), np.zeros(max(nh, 1), np.int32),
               np.zeros((na, 5), dt), np.zeros((na, 15), dt), np.zeros(na, dt),
               np.zeros(na, np.int32), np.zeros(na, np.int32), np.zeros(na, np.int32),
               np.zeros(na, np.float32))
    f = _fn("orc_merge", prec)
    f.restype = C.c_int64
    nc = f(C.byref(g), C.byref(M), C.c_int64(n), _p(par if n else np.zeros(5, dt)),
           _p(cov if n else np.zeros(15, dt)), _p(xr if n else np.zeros(1, np.float32)), _p(ho),
           _p(hc if nh else np.zeros(1, np.int32)), _p(np.ascontiguousarray(inst_off, np.int64)),
           _p(np.ascontiguousarray(row, np.uint16)), _p(np.ascontiguousarray(y, np.float32)),
           _p(np.ascontiguousarray(z, np.float32)), _p(r.out_ok), _p(r.out_p), _p(r.out_c),
           _p(r.out_x), _p(r.succ), _p(r.pred), _p(r.succ_chi2), _p(r.pred_chi2), _p(r.next),
           _p(r.chain_off), _p(r.chain_seg), _p(r.hit_off), _p(r.hit_clu), _p(r.par), _p(r.cov),
           _p(r.chi2), _p(r.ndf), _p(r.status), _p(r.k), _p(r.x_ref))
    cut = lambda a, m: a[:m]  # noqa: E731
    return Merged(cut(r.out_ok, n), cut(r.out_p, n), cut(r.out_c, n), cut(r.out_x, n),
                  cut(r.succ, n), cut(r.pred, n), cut(r.succ_chi2, n), cut(r.pred_chi2, n),
                  cut(r.next, n), r.chain_off[:nc + 1], cut(r.chain_seg, n), r.hit_off[:nc + 1],
                  r.hit_clu[:nh], cut(r.par, nc), cut(r.cov, nc), cut(r.chi2, nc), cut(r.ndf, nc),
                  cut(r.status, nc), cut(r.k, nc), cut(r.x_ref, nc))


def rotate(geom, p, c, x, up, prec=64):
    """R36 on one state: rotation into the next (up) or previous phi
    sector's frame; returns (ok, p, c, x_new)."""
    g = make_geom(geom)
    M = make_mparams()
    dt = _dt(prec)
    p = np.array(p, dt)
    c = np.array(c, dt)
    xn = np.zeros(1, dt)
    f = _fn("orc_rotate", prec)
    f.restype = C.c_int
    sc = C.c_double if prec == 64 else C.c_float
    ok = f(C.byref(g), C.byref(M), _p(p), _p(c), sc(x), C.c_int(1 if up else 0), _p(xn))
    return bool(ok), p, c, float(xn[0])


def chi2_5(S15, d, prec=64):
    """R37's chi2 d^T S^-1 d (S as a lower triangle in the tracker's order)."""
    dt = _dt(prec)
    f = _fn("orc_chi2_5", prec)
    f.restype = C.c_double if prec == 64 else C.c_float
    return float(f(_p(np.ascontiguousarray(S15, dt)), _p(np.ascontiguousarray(d, dt))))
