"""Host-side checks of the C ABI (no GPU work): the library loads, exports
every function include/tpcca.h declares, fills defaults, sizes workspaces and
rejects bad arguments before enqueueing anything."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2511_17018_amd as tpc
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "tpcca.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tpc_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    names = _declared()
    assert "tpc_grid_build" in names and "tpc_sector_track" in names
    L = tpc.lib()
    for n in names:
        assert hasattr(L, n), n


def test_default_params_match_readings():
    p = tpc.make_params(det=True)
    assert (p.nf_win_y, p.nf_win_z) == (3.0, 3.5)
    assert p.nf_chi2_max == pytest.approx(13.8) and p.tc_chi2_pick == pytest.approx(13.8)
    assert p.snp_max == pytest.approx(0.99) and p.grid_occupancy == 2.0
    assert (p.min_chain, p.tc_max_miss, p.min_tracklet_hits, p.min_track_hits) == (3, 10, 10, 10)
    assert p.flags == tpc.FLAG_DETERMINISTIC
    assert tpc.make_params(det=False).flags == 0


def test_status_strings():
    L = tpc.lib()
    assert L.tpc_status_string(0) == b"ok"
    assert L.tpc_status_string(-1) == b"invalid argument"
    assert L.tpc_status_string(-4) == b"workspace too small"


def test_workspace_sizes_grow_and_layout_is_ordered():
    L = tpc.lib()
    a = L.tpc_track_workspace_bytes(C.c_int32(1), C.c_int64(1000), C.c_int64(0))
    b = L.tpc_track_workspace_bytes(C.c_int32(1), C.c_int64(100000), C.c_int64(0))
    assert 0 < a < b
    lay = tpc.TrackWsLayout()
    assert L.tpc_track_workspace_layout(C.c_int32(4), C.c_int64(5000), C.c_int64(0), C.byref(lay)) == 0
    assert lay.cap_tracklets == 5000 // 3 + 4
    offs = [getattr(lay, f) for f in ("up", "dn", "up2", "dn2", "start", "tl_par", "tl_cov",
                                      "tl_chi2", "tl_nhit", "tl_rmin", "tl_rmax", "tl_status",
                                      "tl_hit", "tl_ncand", "owner", "scratch", "total")]
    assert offs == sorted(offs) and all(o % 256 == 0 for o in offs)
    assert lay.tl_hit + 4 * 152 * lay.cap_tracklets <= lay.tl_ncand
    # the merging's workspace grows with the segment capacity and, for the
    # merged-order hit data, by 16 bytes per hit slot (size_t beyond 2^31)
    L.tpc_merge_workspace_bytes.restype = C.c_size_t
    m0 = L.tpc_merge_workspace_bytes(C.c_int64(1000), C.c_int64(0))
    m1 = L.tpc_merge_workspace_bytes(C.c_int64(1000), C.c_int64(50000))
    assert 0 < m0 and m1 - m0 >= 16 * 50000
    assert L.tpc_merge_workspace_bytes(C.c_int64(2000), C.c_int64(0)) > m0
    assert L.tpc_merge_workspace_bytes(C.c_int64(-1), C.c_int64(0)) == 0
    assert L.tpc_merge_workspace_bytes(C.c_int64(1000), C.c_int64(-1)) == 0
    assert L.tpc_merge_workspace_bytes(C.c_int64(1 << 26), C.c_int64(1 << 28)) > 1 << 32
    p = tpc.make_params()
    assert L.tpc_grid_bin_capacity(C.byref(p), C.c_int32(2), C.c_int64(100)) >= 5 * 50 + 2 * 152 * 9
    p.grid_occupancy = 0.5
    assert L.tpc_grid_bin_capacity(C.byref(p), C.c_int32(2), C.c_int64(100)) >= 5 * 200 + 2 * 152 * 9


def _args(geom=None, n_inst=1, off=(0, 10)):
    g = tpc.make_geometry(geom or synth.geometry())
    p = tpc.make_params()
    off = np.array(off, np.int64)
    dummy = C.c_void_p(0x1000)   # never dereferenced: validation fails first
    cl = tpc.Clusters(dummy, dummy, dummy, dummy, dummy)
    gs = tpc.GridStruct(dummy, dummy, dummy, dummy, dummy, dummy, 100)
    return g, p, off, cl, gs, dummy


@pytest.mark.parametrize("case", ["rows", "offset0", "negative", "huge_instance", "min_chain",
                                  "null_geom", "row_order", "workspace", "tl_chunk"])
def test_invalid_arguments_rejected_on_host(case):
    L = tpc.lib()
    g, p, off, cl, gs, dummy = _args()
    ws_bytes = 1 << 40
    n_inst = 1
    if case == "rows":
        g.n_rows = 151
    elif case == "offset0":
        off = np.array([1, 10], np.int64)
    elif case == "negative":
        off = np.array([0, 10, 5], np.int64)
        n_inst = 2
    elif case == "huge_instance":
        off = np.array([0, 1 << 24], np.int64)
    elif case == "min_chain":
        p.min_chain = 2
    elif case == "row_order":
        g.row_x[10] = g.row_x[9]
    elif case == "workspace":
        ws_bytes = 16
    elif case == "tl_chunk":
        p.tl_chunk = 96
    gp = None if case == "null_geom" else C.byref(g)
    st = L.tpc_grid_build(gp, C.byref(p), C.c_int32(n_inst), off.ctypes.data_as(C.c_void_p), dummy,
                          cl, C.byref(gs), dummy, dummy, C.c_size_t(ws_bytes), C.c_void_p(0))
    want = -4 if case == "workspace" else -1
    assert st == want


def test_standard_configuration_matches_generator_geometry():
    # the compile-time constants equal the generator's detector description
    # and the default parameters bit for bit; any other setting, or the
    # generic flag, selects the generic kernels
    g = synth.geometry()
    assert tpc.standard_configuration(g, tpc.make_params(True))
    assert tpc.standard_configuration(g, tpc.make_params(False))
    assert tpc.standard_configuration(g, tpc.make_params(True, grid_occupancy=0.5, tl_chunk=64))
    assert not tpc.standard_configuration(g, tpc.make_params(True, generic=True))
    assert not tpc.standard_configuration(g, tpc.make_params(True, tc_max_miss=8))
    assert not tpc.standard_configuration(g, tpc.make_params(True, nf_win_y=2.5))
    g2 = dict(g, bz=np.float32(0.2))
    assert not tpc.standard_configuration(g2, tpc.make_params(True))
    g3 = dict(g, row_x=g["row_x"].copy())
    g3["row_x"][100] = np.nextafter(g3["row_x"][100], np.float32(1e9))
    assert not tpc.standard_configuration(g3, tpc.make_params(True))


@pytest.mark.parametrize("case", ["unknown_flag", "bin_table_over_int32"])
def test_grid_and_track_reject_unknown_flags_and_oversized_bin_tables(case):
    L = tpc.lib()
    g, p, off, cl, gs, dummy = _args()
    n_inst = 1
    if case == "unknown_flag":
        p.flags |= 2          # no such flag
    else:
        # 2^27 clusters in 16 instances at occupancy 0.25: the bin table the
        # size query asks for exceeds the 32-bit bin offsets
        n_inst = 16
        off = np.arange(17, dtype=np.int64) * ((1 << 24) - 1)
        p.grid_occupancy = 0.25
        assert L.tpc_grid_bin_capacity(C.byref(p), C.c_int32(n_inst), C.c_int64(int(off[-1]))) > 2**31 - 1
    st = L.tpc_grid_build(C.byref(g), C.byref(p), C.c_int32(n_inst), off.ctypes.data_as(C.c_void_p),
                          dummy, cl, C.byref(gs), dummy, dummy, C.c_size_t(1 << 50), C.c_void_p(0))
    assert st == -1
    tr = tpc.TracksStruct(dummy, dummy, dummy, dummy, dummy, dummy, dummy, dummy, 10, 10)
    st = L.tpc_sector_track(C.byref(g), C.byref(p), C.c_int32(n_inst),
                            off.ctypes.data_as(C.c_void_p), dummy, cl, C.byref(gs), C.byref(tr),
                            dummy, dummy, C.c_size_t(1 << 50), C.c_int64(0), C.c_void_p(0))
    assert st == -1


@pytest.mark.parametrize("case", ["unknown_flag", "clusters_over_int32", "null_map", "rows",
                                  "field_bins_zero", "field_bins_over"])
def test_refit_rejects_bad_arguments_on_host(case):
    L = tpc.lib()
    g = tpc.make_geometry(synth.geometry())
    p = tpc.make_params(True)
    dummy = C.c_void_p(0x1000)   # never dereferenced: validation fails first
    cl = tpc.Clusters(dummy, dummy, dummy, dummy, dummy)
    trk = tpc.RefitTracksStruct(dummy, dummy, dummy, dummy, 4, 40)
    nc = 1000
    dmap = dummy
    if case == "unknown_flag":
        p.flags |= 4
    elif case == "clusters_over_int32":
        nc = 1 << 31
    elif case == "null_map":
        dmap = C.c_void_p(0)
    elif case == "rows":
        g.n_rows = 150
    mat = None
    if case.startswith("field_bins"):
        # a field map with no z bin, or more than the 65536 the header allows
        mat = C.byref(tpc.MaterialStruct(dummy, 0 if case == "field_bins_zero" else 65537,
                                         None, None))
    L.tpc_refit.restype = C.c_int
    L.tpc_refit_backward.restype = C.c_int
    L.tpc_refit_backward_noalloc.restype = C.c_int
    st = L.tpc_refit(C.byref(g), C.byref(p), C.c_int64(nc), cl, trk, dmap, mat, dummy, dummy,
                     C.c_void_p(0x2000), C.c_void_p(0))
    assert st == -1
    st = L.tpc_refit_backward(C.byref(g), C.byref(p), C.c_int64(nc), cl, trk, dmap, mat,
                              C.c_void_p(0x2000), dummy, dummy, dummy, dummy, dummy, dummy,
                              C.c_void_p(0x3000), C.c_size_t(1 << 20), C.c_void_p(0))
    assert st == -1
    st = L.tpc_refit_backward_noalloc(C.byref(g), C.byref(p), C.c_int64(nc), cl, trk, dmap, mat,
                                      C.c_void_p(0x2000), dummy, dummy, dummy, dummy, dummy,
                                      dummy, C.c_void_p(0))
    assert st == -1
