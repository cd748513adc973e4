"""Python binding of libtpcca.so, the MI355X TPC sector tracker.

Argument marshalling only: torch tensors supply device memory and the
current HIP stream; every step of the tracking chain runs in the library's
HIP kernels.  The names mirror the C ABI in include/tpcca.h:
``grid_build`` -> tpc_grid_build, ``sector_track`` -> tpc_sector_track.
If the library is not built, loading it raises RuntimeError; there is no
fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtpcca.so")
N_ROWS = 152
FLAG_DETERMINISTIC = 1
FLAG_GENERIC = 8
FLAG_COUNT_CANDIDATES = 16

_lib = None


def lib() -> C.CDLL:
    """The loaded libtpcca.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2511_17018_amd.build` (hipcc, gfx950)")
        _lib = C.CDLL(LIB_PATH)
        _lib.tpc_status_string.restype = C.c_char_p
        _lib.tpc_grid_bin_capacity.restype = C.c_int64
        _lib.tpc_grid_workspace_bytes.restype = C.c_size_t
        _lib.tpc_track_workspace_bytes.restype = C.c_size_t
        _lib.tpc_track_workspace_layout.restype = C.c_int
        _lib.tpc_grid_build.restype = C.c_int
        _lib.tpc_sector_track.restype = C.c_int
        _lib.tpc_standard_configuration.restype = C.c_int32
    return _lib


def standard_configuration(geom: dict, params: Params) -> bool:
    """Whether sector tracking runs the kernels compiled for the standard
    configuration (same results as the generic ones)."""
    g = make_geometry(geom)
    return lib().tpc_standard_configuration(C.byref(g), C.byref(params)) == 1


class Geometry(C.Structure):
    _fields_ = [("n_rows", C.c_int32), ("row_x", C.c_float * N_ROWS), ("bz_tesla", C.c_float),
                ("tan_half_sector", C.c_float), ("sigma_y2", C.c_float), ("sigma_z2", C.c_float)]


class Params(C.Structure):
    _fields_ = [("nf_win_y", C.c_float), ("nf_win_z", C.c_float), ("nf_chi2_max", C.c_float),
                ("tc_chi2_pick", C.c_float), ("snp_max", C.c_float),
                ("grid_occupancy", C.c_float), ("edge_margin", C.c_float),
                ("search_margin", C.c_float), ("y_valid_margin", C.c_float),
                ("min_chain", C.c_int32), ("tc_max_miss", C.c_int32),
                ("min_tracklet_hits", C.c_int32), ("min_track_hits", C.c_int32),
                ("flags", C.c_uint32), ("tl_chunk", C.c_int32)]


class Clusters(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p), ("row", C.c_void_p),
                ("charge", C.c_void_p)]


class GridStruct(C.Structure):
    _fields_ = [("sseg", C.c_void_p), ("row_off", C.c_void_p), ("meta", C.c_void_p),
                ("bin_off", C.c_void_p), ("perm", C.c_void_p), ("yz", C.c_void_p),
                ("bin_cap", C.c_int64)]


class TracksStruct(C.Structure):
    _fields_ = [("param", C.c_void_p), ("cov", C.c_void_p), ("chi2", C.c_void_p),
                ("ndf", C.c_void_p), ("x_ref", C.c_void_p), ("hit_off", C.c_void_p),
                ("hit_clu", C.c_void_p), ("clu2trk", C.c_void_p), ("cap_tracks", C.c_int64),
                ("cap_hits", C.c_int64), ("hit_data", C.c_void_p)]


class TrackWsLayout(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "up", "dn", "up2", "dn2", "start", "tl_par", "tl_cov", "tl_chi2", "tl_nhit", "tl_rmin",
        "tl_rmax", "tl_status", "tl_hit", "tl_ncand", "owner", "scratch", "total",
        "cap_tracklets")]


RESULT_DTYPE = np.dtype([(n, np.int64) for n in (
    "n_valid", "n_bad", "n_bins", "n_start", "n_tracklets_kept", "n_tracks", "n_hits",
    "need_tracklets", "need_tracks", "need_hits")] + [("overflow", np.int32), ("reserved", np.int32)])
RESULT_BYTES = RESULT_DTYPE.itemsize


class TpcError(RuntimeError):
    pass


def _check(st: int, what: str):
    if st != 0:
        raise TpcError(f"{what}: {lib().tpc_status_string(st).decode()} ({st})")


def make_geometry(geom: dict) -> Geometry:
    g = Geometry()
    g.n_rows = int(geom["n_rows"])
    rx = np.asarray(geom["row_x"], np.float32)
    C.memmove(g.row_x, rx.ctypes.data, 4 * N_ROWS)
    g.bz_tesla = float(geom["bz"])
    g.tan_half_sector = float(geom["tan_half"])
    g.sigma_y2 = float(geom["sigma_y2"])
    g.sigma_z2 = float(geom["sigma_z2"])
    return g


def make_params(det: bool = True, generic: bool = False, count: bool = False, **over) -> Params:
    """Default parameters with overrides; `generic` keeps the library from
    using its kernels compiled for the standard configuration; `count` runs
    the instrumented tracklet kernel (window candidates in tl_ncand)."""
    p = Params()
    lib().tpc_default_params(C.byref(p))
    for k, v in over.items():
        setattr(p, k, v)
    p.flags = (p.flags | FLAG_DETERMINISTIC) if det else (p.flags & ~FLAG_DETERMINISTIC)
    if generic:
        p.flags |= FLAG_GENERIC
    if count:
        p.flags |= FLAG_COUNT_CANDIDATES
    return p


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else C.c_void_p(0)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclass
class Batch:
    """Clusters of several sector instances resident on the GPU."""
    x: torch.Tensor
    y: torch.Tensor
    z: torch.Tensor
    row: torch.Tensor      # int16 storage of uint16 row numbers
    charge: torch.Tensor
    inst_off_host: np.ndarray
    inst_off: torch.Tensor

    @property
    def n(self) -> int:
        return int(self.inst_off_host[-1])

    @property
    def n_inst(self) -> int:
        return len(self.inst_off_host) - 1

    def struct(self) -> Clusters:
        return Clusters(_ptr(self.x), _ptr(self.y), _ptr(self.z), _ptr(self.row), _ptr(self.charge))

    def slice(self, i: int) -> "Batch":
        """Instance i alone (views, no copies of the cluster arrays)."""
        a, b = int(self.inst_off_host[i]), int(self.inst_off_host[i + 1])
        off = np.array([0, b - a], np.int64)
        return Batch(self.x[a:b], self.y[a:b], self.z[a:b], self.row[a:b], self.charge[a:b],
                     off, torch.from_numpy(off).to(self.x.device))


def upload(x, y, z, row, charge, inst_off, device="cuda") -> Batch:
    off = np.ascontiguousarray(inst_off, np.int64)
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a).view(dt)).to(device)  # noqa: E731
    return Batch(t(x, np.float32), t(y, np.float32), t(z, np.float32), t(row, np.int16),
                 t(charge, np.int16), off, torch.from_numpy(off).to(device))


def upload_device(x: torch.Tensor, y: torch.Tensor, z: torch.Tensor, row: torch.Tensor,
                  inst_off, charge: torch.Tensor | None = None) -> Batch:
    """A batch from clusters already on the device (e.g. the output of
    cluster_transform); inst_off is host data."""
    off = np.ascontiguousarray(inst_off, np.int64)
    if charge is None:
        charge = torch.zeros_like(row)
    return Batch(x, y, z, row, charge, off, torch.from_numpy(off).to(row.device))


@dataclass
class Grid:
    sseg: torch.Tensor
    row_off: torch.Tensor
    meta: torch.Tensor      # int32 [n_inst*152, 8]: ny, nz, bin_base, count, y0, z0, iwy, iwz (bits)
    bin_off: torch.Tensor
    perm: torch.Tensor
    yz: torch.Tensor        # float32 [n, 2]: (y, z) of each position

    def struct(self) -> GridStruct:
        return GridStruct(_ptr(self.sseg), _ptr(self.row_off), _ptr(self.meta), _ptr(self.bin_off),
                          _ptr(self.perm), _ptr(self.yz), self.bin_off.numel())


@dataclass
class Tracks:
    param: torch.Tensor
    cov: torch.Tensor
    chi2: torch.Tensor
    ndf: torch.Tensor
    x_ref: torch.Tensor
    hit_off: torch.Tensor
    hit_clu: torch.Tensor
    clu2trk: torch.Tensor
    # optional float32 [cap_hits, 4]: each hit's row plane x, y, z and phi
    # sector (the merging reads its segments' hits from here when present)
    hit_data: torch.Tensor | None = None

    def struct(self) -> TracksStruct:
        return TracksStruct(_ptr(self.param), _ptr(self.cov), _ptr(self.chi2), _ptr(self.ndf),
                            _ptr(self.x_ref), _ptr(self.hit_off), _ptr(self.hit_clu),
                            _ptr(self.clu2trk), self.param.shape[0], self.hit_clu.numel(),
                            _ptr(self.hit_data))


def alloc_grid(n_inst: int, n: int, device="cuda", params: Params | None = None) -> Grid:
    p = params if params is not None else make_params()
    cap = int(lib().tpc_grid_bin_capacity(C.byref(p), C.c_int32(n_inst), C.c_int64(n)))
    i32 = dict(dtype=torch.int32, device=device)
    return Grid(torch.empty(n, **i32), torch.empty(n_inst * (N_ROWS + 1), **i32),
                torch.empty((n_inst * N_ROWS, 8), **i32), torch.empty(cap, **i32),
                torch.empty(n, **i32), torch.empty((n, 2), dtype=torch.float32, device=device))


def alloc_tracks(n: int, cap_tracks: int | None = None, cap_hits: int | None = None,
                 device="cuda", hit_data: bool = False) -> Tracks:
    ct = max(1, n // 10 + 16) if cap_tracks is None else cap_tracks
    ch = n if cap_hits is None else cap_hits
    f32 = dict(dtype=torch.float32, device=device)
    i32 = dict(dtype=torch.int32, device=device)
    return Tracks(torch.empty((ct, 5), **f32), torch.empty((ct, 15), **f32), torch.empty(ct, **f32),
                  torch.empty(ct, **i32), torch.empty(ct, **f32), torch.empty(ct + 1, **i32),
                  torch.empty(ch, **i32), torch.empty(n, **i32),
                  torch.empty((ch, 4), **f32) if hit_data and ch > 0 else None)


class Workspace:
    """Device scratch of one tracking call (grid and tracking parts)."""

    def __init__(self, n_inst: int, n: int, cap_tracklets: int = 0, device="cuda",
                 params: Params | None = None):
        L = lib()
        self.n_inst, self.n, self.cap_tracklets = n_inst, n, cap_tracklets
        p = params if params is not None else make_params()
        gb = int(L.tpc_grid_workspace_bytes(C.byref(p), C.c_int32(n_inst), C.c_int64(n)))
        tb = int(L.tpc_track_workspace_bytes(C.c_int32(n_inst), C.c_int64(n),
                                             C.c_int64(cap_tracklets)))
        self.grid_ws = torch.empty(max(gb, 256), dtype=torch.uint8, device=device)
        self.track_ws = torch.empty(max(tb, 256), dtype=torch.uint8, device=device)
        self.layout = TrackWsLayout()
        _check(L.tpc_track_workspace_layout(C.c_int32(n_inst), C.c_int64(n),
                                            C.c_int64(cap_tracklets), C.byref(self.layout)),
               "tpc_track_workspace_layout")
        self.result = torch.zeros(RESULT_BYTES, dtype=torch.uint8, device=device)

    def view(self, name: str, dtype, count: int) -> torch.Tensor:
        off = getattr(self.layout, name)
        nbytes = count * torch.empty(0, dtype=dtype).element_size()
        return self.track_ws[off:off + nbytes].view(dtype)

    def read_result(self) -> np.void:
        return np.frombuffer(self.result.cpu().numpy().tobytes(), RESULT_DTYPE)[0]


def grid_build(geom: Geometry, params: Params, batch: Batch, grid: Grid, ws: Workspace) -> None:
    """tpc_grid_build on the current stream (asynchronous)."""
    gs = grid.struct()
    _check(lib().tpc_grid_build(
        C.byref(geom), C.byref(params), C.c_int32(batch.n_inst),
        batch.inst_off_host.ctypes.data_as(C.c_void_p), _ptr(batch.inst_off), batch.struct(),
        C.byref(gs), _ptr(ws.result), _ptr(ws.grid_ws), C.c_size_t(ws.grid_ws.numel()),
        _stream()), "tpc_grid_build")


def sector_track(geom: Geometry, params: Params, batch: Batch, grid: Grid, tracks: Tracks,
                 ws: Workspace) -> None:
    """tpc_sector_track on the current stream (asynchronous)."""
    gs = grid.struct()
    ts = tracks.struct()
    _check(lib().tpc_sector_track(
        C.byref(geom), C.byref(params), C.c_int32(batch.n_inst),
        batch.inst_off_host.ctypes.data_as(C.c_void_p), _ptr(batch.inst_off), batch.struct(),
        C.byref(gs), C.byref(ts), _ptr(ws.result), _ptr(ws.track_ws),
        C.c_size_t(ws.track_ws.numel()), C.c_int64(ws.cap_tracklets), _stream()),
        "tpc_sector_track")


@dataclass
class TrackRun:
    grid: Grid
    tracks: Tracks
    ws: Workspace
    result: np.void


def track(geom: dict, batch: Batch, det: bool = True, cap_tracks=None, cap_hits=None,
          cap_tracklets: int = 0, hit_data: bool = False, **param_over) -> TrackRun:
    """Grid + sector tracking of a batch; synchronises and returns the result.
    hit_data: also write each hit's plane, position and sector (for merging)."""
    g = make_geometry(geom)
    p = make_params(det, **param_over)
    dev = batch.x.device
    grid = alloc_grid(batch.n_inst, batch.n, dev, p)
    tracks = alloc_tracks(batch.n, cap_tracks, cap_hits, dev, hit_data)
    ws = Workspace(batch.n_inst, batch.n, cap_tracklets, dev, p)
    grid_build(g, p, batch, grid, ws)
    sector_track(g, p, batch, grid, tracks, ws)
    torch.cuda.synchronize()
    return TrackRun(grid, tracks, ws, ws.read_result())


# ----------------------------------------------------------------------------
# differentiable refit (tpc_refit / tpc_refit_backward)

N_PHI = 18


class RefitTracksStruct(C.Structure):
    _fields_ = [("hit_off", C.c_void_p), ("hit_clu", C.c_void_p), ("sector", C.c_void_p),
                ("seed", C.c_void_p), ("n_tracks", C.c_int64), ("n_hits", C.c_int64)]


@dataclass
class RefitTracks:
    """Found tracks on the GPU: CSR hit lists (cluster indices, ascending row),
    per-cluster phi-sector, seeds (y, z, snp, tgl, qpt)."""
    hit_off: torch.Tensor   # int32 [n_tracks+1]
    hit_clu: torch.Tensor   # int32 [n_hits]
    sector: torch.Tensor    # uint8 [n_clusters]
    seed: torch.Tensor      # float32 [n_tracks, 5]

    @property
    def n_tracks(self) -> int:
        return self.hit_off.numel() - 1

    @property
    def n_hits(self) -> int:
        return self.hit_clu.numel()

    def struct(self) -> RefitTracksStruct:
        return RefitTracksStruct(_ptr(self.hit_off), _ptr(self.hit_clu), _ptr(self.sector),
                                 _ptr(self.seed), self.n_tracks, self.n_hits)


def upload_refit_tracks(hit_off, hit_clu, sector, seed, device="cuda") -> RefitTracks:
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dt)).to(device)  # noqa: E731
    return RefitTracks(t(hit_off, np.int32), t(hit_clu, np.int32), t(sector, np.uint8),
                       t(seed, np.float32))


def _xyz_struct(xyz: torch.Tensor, row: torch.Tensor) -> Clusters:
    return Clusters(_ptr(xyz[0]), _ptr(xyz[1]), _ptr(xyz[2]), _ptr(row), C.c_void_p(0))


class MaterialStruct(C.Structure):
    _fields_ = [("bz", C.c_void_p), ("nzb", C.c_int32), ("ix0", C.c_void_p),
                ("eloss", C.c_void_p)]


@dataclass
class Material:
    """Field map and material of the refit (tpc_material): device tensors,
    any of them None -- bz float32 [152, nzb] field [T] per row and z bin,
    ix0 float32 [152] inverse radiation length [1/cm], eloss float32 [152]
    mean energy loss at minimum ionisation [GeV/cm]."""
    bz: torch.Tensor | None = None
    ix0: torch.Tensor | None = None
    eloss: torch.Tensor | None = None

    def struct(self) -> MaterialStruct:
        for t in (self.bz, self.ix0, self.eloss):
            assert t is None or (t.dtype == torch.float32 and t.is_contiguous())
        nzb = self.bz.shape[1] if self.bz is not None else 0
        return MaterialStruct(_ptr(self.bz) if self.bz is not None else None, nzb,
                              _ptr(self.ix0) if self.ix0 is not None else None,
                              _ptr(self.eloss) if self.eloss is not None else None)


def upload_material(bz=None, ix0=None, eloss=None, device="cuda") -> Material:
    t = (lambda a: None if a is None
         else torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device))  # noqa: E731
    return Material(t(bz), t(ix0), t(eloss))


def _mat_ref(mat: Material | None):
    """(pointer argument, the struct kept alive by the caller)"""
    if mat is None:
        return None, None
    m = mat.struct()
    return C.byref(m), m


def checkpoint_index(hit_off) -> np.ndarray:
    """Float indices into the refit's flat checkpoint array of each hit's 20
    values, for the hits in hit order: ckpt.reshape(-1)[checkpoint_index(
    hit_off)] is [n_hits, 20] in hit order.  tpc_refit's layout: groups of 64
    consecutive tracks; in a group, by hit number j, the a_j tracks with more
    than j hits share 80 * a_j bytes starting at entry E_j (the group's first
    hit plus sum_k min(L_k, j)), as five runs of 16-byte parts, part q of the
    track of rank r at float4 5 E_j + q a_j + r."""
    ho = np.asarray(hit_off, np.int64)
    n = len(ho) - 1
    L = np.diff(ho)
    trk = np.repeat(np.arange(n, dtype=np.int64), L)
    j = np.arange(int(ho[-1]), dtype=np.int64) - np.repeat(ho[:-1], L)
    g = trk // 64
    # rank among the group's tracks with more than j hits, and their count:
    # the hits sorted by (group, j, track) enumerate each (group, j) run
    order = np.lexsort((trk, j, g))
    key = g[order] * (int(L.max(initial=0)) + 1) + j[order]
    first = np.r_[True, key[1:] != key[:-1]]
    run_start = np.maximum.accumulate(np.where(first, np.arange(len(key)), 0))
    rank = np.empty(len(trk), np.int64)
    rank[order] = np.arange(len(key)) - run_start
    run_len = np.diff(np.r_[np.nonzero(first)[0], len(key)])
    act = np.empty(len(trk), np.int64)
    act[order] = np.repeat(run_len, run_len)
    # E_j: the run's first entry (the hits before it in the same order)
    e0 = np.empty(len(trk), np.int64)
    e0[order] = run_start
    q = np.arange(5, dtype=np.int64)
    f4 = 5 * e0[:, None] + q[None, :] * act[:, None] + rank[:, None]
    return (4 * f4[:, :, None] + np.arange(4)[None, None, :]).reshape(len(trk), 20)


def refit(geom: dict, xyz: torch.Tensor, row: torch.Tensor, trk: RefitTracks,
          dist_map: torch.Tensor, det: bool = True, mat: Material | None = None):
    """tpc_refit on the current stream: (chi2[n], status[n], ckpt[n_hits, 20]);
    ckpt in the library's layout (checkpoint_index gives the hit order).
    mat: field map and material (None: uniform field, no material)."""
    assert xyz.dtype == torch.float32 and xyz.is_contiguous() and xyz.shape[0] == 3
    dev = xyz.device
    n = trk.n_tracks
    chi2 = torch.empty(max(n, 1), dtype=torch.float32, device=dev)
    status = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    ckpt = torch.empty((max(trk.n_hits, 1), 20), dtype=torch.float32, device=dev)
    g = make_geometry(geom)
    p = make_params(det)
    L = lib()
    L.tpc_refit.restype = C.c_int
    mref, _keep = _mat_ref(mat)
    _check(L.tpc_refit(C.byref(g), C.byref(p), C.c_int64(xyz.shape[1]), _xyz_struct(xyz, row),
                       trk.struct(), _ptr(dist_map.contiguous()), mref, _ptr(chi2),
                       _ptr(status), _ptr(ckpt), _stream()), "tpc_refit")
    return chi2[:n], status[:n], ckpt[:trk.n_hits]


def refit_backward(geom: dict, xyz: torch.Tensor, row: torch.Tensor, trk: RefitTracks,
                   dist_map: torch.Tensor, ckpt: torch.Tensor, status: torch.Tensor,
                   grad_chi2: torch.Tensor, mat: Material | None = None):
    """tpc_refit_backward: (grad_map[152, 18], grad_xyz[3, n_clusters])."""
    dev = xyz.device
    nc = xyz.shape[1]
    gmap = torch.empty((N_ROWS, N_PHI), dtype=torch.float32, device=dev)
    gxyz = torch.empty((3, max(nc, 1)), dtype=torch.float32, device=dev)
    L = lib()
    L.tpc_refit_workspace_bytes.restype = C.c_size_t
    L.tpc_refit_backward.restype = C.c_int
    ws = torch.empty(int(L.tpc_refit_workspace_bytes()), dtype=torch.uint8, device=dev)
    g = make_geometry(geom)
    p = make_params(True)
    ckpt_p = _ptr(ckpt) if trk.n_hits else C.c_void_p(0)
    mref, _keep = _mat_ref(mat)
    _check(L.tpc_refit_backward(
        C.byref(g), C.byref(p), C.c_int64(nc), _xyz_struct(xyz, row), trk.struct(),
        _ptr(dist_map.contiguous()), mref, ckpt_p, _ptr(status), _ptr(grad_chi2.contiguous()),
        _ptr(gmap), _ptr(gxyz[0]), _ptr(gxyz[1]), _ptr(gxyz[2]), _ptr(ws),
        C.c_size_t(ws.numel()), _stream()), "tpc_refit_backward")
    return gmap, gxyz[:, :nc]


def refit_backward_noalloc(geom: dict, xyz: torch.Tensor, row: torch.Tensor, trk: RefitTracks,
                           dist_map: torch.Tensor, ckpt: torch.Tensor, status: torch.Tensor,
                           grad_chi2: torch.Tensor, gmap: torch.Tensor, gxyz: torch.Tensor,
                           mat: Material | None = None):
    """tpc_refit_backward_noalloc into caller-given outputs grad_map[152, 18]
    and grad_xyz[3, >= n_clusters] (the library allocates nothing)."""
    nc = xyz.shape[1]
    assert gmap.is_contiguous() and gmap.numel() == N_ROWS * N_PHI
    assert gxyz.is_contiguous() and gxyz.shape[0] == 3 and gxyz.shape[1] >= max(nc, 1)
    L = lib()
    L.tpc_refit_backward_noalloc.restype = C.c_int
    g = make_geometry(geom)
    p = make_params(True)
    ckpt_p = _ptr(ckpt) if trk.n_hits else C.c_void_p(0)
    mref, _keep = _mat_ref(mat)
    _check(L.tpc_refit_backward_noalloc(
        C.byref(g), C.byref(p), C.c_int64(nc), _xyz_struct(xyz, row), trk.struct(),
        _ptr(dist_map.contiguous()), mref, ckpt_p, _ptr(status), _ptr(grad_chi2.contiguous()),
        _ptr(gmap), _ptr(gxyz[0]), _ptr(gxyz[1]), _ptr(gxyz[2]), _stream()),
        "tpc_refit_backward_noalloc")
    return gmap, gxyz[:, :nc]


class TpcRefit(torch.autograd.Function):
    """chi2[t] of every found track under the distortion map, differentiable
    with respect to the cluster coordinates xyz[3, N] and the map [152, 18].

        chi2 = TpcRefit.apply(xyz, dist_map, row, tracks, geom)
        chi2.sum().backward()   # xyz.grad, dist_map.grad
    """

    @staticmethod
    def forward(ctx, xyz, dist_map, row, tracks, geom, det=True, mat=None):
        xyz_c = xyz.detach().contiguous()
        map_c = dist_map.detach().contiguous()
        chi2, status, ckpt = refit(geom, xyz_c, row, tracks, map_c, det, mat)
        ctx.save_for_backward(xyz_c, map_c, ckpt, status)
        ctx.row, ctx.tracks, ctx.geom, ctx.mat = row, tracks, geom, mat
        return chi2

    @staticmethod
    def backward(ctx, grad_chi2):
        xyz_c, map_c, ckpt, status = ctx.saved_tensors
        gmap, gxyz = refit_backward(ctx.geom, xyz_c, ctx.row, ctx.tracks, map_c, ckpt, status,
                                    grad_chi2.float().contiguous(), ctx.mat)
        return gxyz, gmap, None, None, None, None, None


# ----------------------------------------------------------------------------
# cluster coordinate transformation (tpc_cluster_transform)

class TransformGeometry(C.Structure):
    _fields_ = [("row_x", C.c_float * N_ROWS), ("pad_w", C.c_float * N_ROWS),
                ("pad_c", C.c_float * N_ROWS), ("tbin_us", C.c_float), ("vdrift_cm_us", C.c_float),
                ("zlen_cm", C.c_float), ("t0_us", C.c_float), ("nu", C.c_int32), ("nv", C.c_int32),
                ("nw", C.c_int32), ("u0", C.c_float), ("iu", C.c_float), ("v0", C.c_float),
                ("iv", C.c_float), ("w0", C.c_float), ("iw", C.c_float)]


class RawClusters(C.Structure):
    _fields_ = [("sector", C.c_void_p), ("row", C.c_void_p), ("pad", C.c_void_p),
                ("time", C.c_void_p)]


def make_transform_geometry(tg: dict) -> TransformGeometry:
    t = TransformGeometry()
    for name in ("row_x", "pad_w", "pad_c"):
        arr = np.asarray(tg[name], np.float32)
        for r in range(N_ROWS):
            getattr(t, name)[r] = float(arr[r])
    t.tbin_us, t.vdrift_cm_us = float(tg["tbin"]), float(tg["vdrift"])
    t.zlen_cm, t.t0_us = float(tg["zlen"]), float(tg["t0"])
    t.nu, t.nv, t.nw = int(tg["nu"]), int(tg["nv"]), int(tg["nw"])
    for name in ("u0", "iu", "v0", "iv", "w0", "iw"):
        setattr(t, name, float(np.float32(tg[name])))
    return t


def cluster_transform(tg: dict, sector: torch.Tensor, row: torch.Tensor, pad: torch.Tensor,
                      time: torch.Tensor, dist_map=None, corr_map=None, det: bool = True,
                      out=None):
    """tpc_cluster_transform on the current stream: (x, y, z, row) tensors
    (row int16-typed, holding the uint16 row or 0xFFFF).  `out` may give the
    four output tensors."""
    n = row.numel()
    dev = row.device
    if out is None:
        out = (torch.empty(max(n, 1), dtype=torch.float32, device=dev),
               torch.empty(max(n, 1), dtype=torch.float32, device=dev),
               torch.empty(max(n, 1), dtype=torch.float32, device=dev),
               torch.empty(max(n, 1), dtype=torch.int16, device=dev))
    x, y, z, ro = out
    t = make_transform_geometry(tg)
    L = lib()
    L.tpc_cluster_transform.restype = C.c_int
    raw = RawClusters(_ptr(sector), _ptr(row), _ptr(pad), _ptr(time))
    dm = _ptr(dist_map) if dist_map is not None else C.c_void_p(0)
    cm = _ptr(corr_map) if corr_map is not None else C.c_void_p(0)
    _check(L.tpc_cluster_transform(C.byref(t), C.c_uint32(FLAG_DETERMINISTIC if det else 0),
                                   C.c_int64(n), raw, dm, cm, _ptr(x), _ptr(y), _ptr(z), _ptr(ro),
                                   _stream()), "tpc_cluster_transform")
    return x[:n], y[:n], z[:n], ro[:n]


# ----------------------------------------------------------------------------
# sector-track merging and global refit (tpc_merge_tracks)

class MergeParams(C.Structure):
    _fields_ = [("max_dz", C.c_float), ("max_dist", C.c_float), ("chi2_max", C.c_float),
                ("cos_a", C.c_float * N_PHI), ("sin_a", C.c_float * N_PHI), ("cos_d", C.c_float),
                ("sin_d", C.c_float)]


class MergedStruct(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in ("param", "cov", "chi2", "ndf", "status", "sector",
                                          "x_ref", "hit_off", "hit_clu", "seg_off", "seg", "next",
                                          "counts")] + [("cap_tracks", C.c_int64),
                                                        ("cap_hits", C.c_int64)]


def default_merge_params(**over) -> MergeParams:
    m = MergeParams()
    lib().tpc_default_merge_params(C.byref(m))
    for k, v in over.items():
        setattr(m, k, v)
    return m


@dataclass
class Merged:
    param: torch.Tensor
    cov: torch.Tensor
    chi2: torch.Tensor
    ndf: torch.Tensor
    status: torch.Tensor
    sector: torch.Tensor
    x_ref: torch.Tensor
    hit_off: torch.Tensor
    hit_clu: torch.Tensor
    seg_off: torch.Tensor
    seg: torch.Tensor
    next: torch.Tensor
    counts: torch.Tensor
    ws: torch.Tensor

    def struct(self) -> MergedStruct:
        return MergedStruct(*[_ptr(getattr(self, f)) for f in (
            "param", "cov", "chi2", "ndf", "status", "sector", "x_ref", "hit_off", "hit_clu",
            "seg_off", "seg", "next", "counts")], self.param.shape[0], self.hit_clu.numel())

    def host(self) -> dict:
        nc, nh = (int(v) for v in self.counts.cpu().tolist())
        h = lambda t: t.cpu().numpy()  # noqa: E731
        return dict(n=nc, param=h(self.param[:nc]), cov=h(self.cov[:nc]), chi2=h(self.chi2[:nc]),
                    ndf=h(self.ndf[:nc]), status=h(self.status[:nc]), sector=h(self.sector[:nc]),
                    x_ref=h(self.x_ref[:nc]), hit_off=h(self.hit_off[:nc + 1]),
                    hit_clu=h(self.hit_clu[:nh]), seg_off=h(self.seg_off[:nc + 1]),
                    seg=h(self.seg[:int(self.seg_off[nc].item())]), next=h(self.next))


def alloc_merged(cap_tracks: int, cap_hits: int, device="cuda") -> Merged:
    f32 = dict(dtype=torch.float32, device=device)
    i32 = dict(dtype=torch.int32, device=device)
    ct = max(cap_tracks, 1)
    L = lib()
    L.tpc_merge_workspace_bytes.restype = C.c_size_t
    wsb = int(L.tpc_merge_workspace_bytes(C.c_int64(cap_tracks), C.c_int64(cap_hits)))
    return Merged(torch.empty((ct, 5), **f32), torch.empty((ct, 15), **f32), torch.empty(ct, **f32),
                  torch.empty(ct, **i32), torch.empty(ct, **i32), torch.empty(ct, **i32),
                  torch.empty(ct, **f32), torch.empty(ct + 1, **i32),
                  torch.empty(max(cap_hits, 1), **i32), torch.empty(ct + 1, **i32),
                  torch.empty(ct, **i32), torch.empty(ct, **i32),
                  torch.zeros(2, dtype=torch.int64, device=device),
                  torch.empty(max(wsb, 256), dtype=torch.uint8, device=device))


def merge_tracks(geom: dict, batch: Batch, tracks: Tracks, result: torch.Tensor, det: bool = True,
                 out: Merged | None = None, mp: MergeParams | None = None) -> Merged:
    """tpc_merge_tracks on the current stream (asynchronous): the sector
    tracker's tracks of a 36-sector batch merged across sector edges and the
    central membrane, and refitted.  `result` is the tracker's device result
    word (Workspace.result)."""
    g = make_geometry(geom)
    p = make_params(det)
    mp = mp if mp is not None else default_merge_params()
    out = out if out is not None else alloc_merged(tracks.param.shape[0], tracks.hit_clu.numel(),
                                                   batch.x.device)
    ts = tracks.struct()
    ms = out.struct()
    L = lib()
    L.tpc_merge_tracks.restype = C.c_int
    _check(L.tpc_merge_tracks(C.byref(g), C.byref(p), C.byref(mp), C.c_int32(batch.n_inst),
                              _ptr(batch.inst_off), batch.struct(), C.byref(ts), _ptr(result),
                              C.byref(ms), _ptr(out.ws), C.c_size_t(out.ws.numel()), _stream()),
           "tpc_merge_tracks")
    return out
