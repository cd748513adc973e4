"""Pins of the cluster-transformation oracle (f3, readings R31-R34).

P17 the nominal transformation inverts the generator's readout encoding
(closed form: pad and time from the true position) to the rounding of the
binary32 readout values; hand cases (centre pad, zero drift, sides).
P18 the residual map's interpolation is exact on trilinear functions of the
grid coordinates, reproduces node values at nodes and continues the
boundary values outside the grid.
P19 a smooth distortion is undone by its calibration map to well within
the distortion (first-order inverse plus interpolation error).
P20 order of the corrections: the residual map reads y / x after the radial
offset.  Invalid raw clusters come out as invalid tracker inputs (R34).
"""
import numpy as np
import pytest

import oracle
import synth

TG = synth.transform_geometry()


def _raw(n, rng, tg=TG):
    s = rng.integers(0, 36, n).astype(np.uint8)
    r = rng.integers(0, 152, n).astype(np.uint16)
    pad = rng.uniform(0, 2 * tg["pad_c"][r]).astype(np.float32)
    time = rng.uniform(0, float(tg["zlen"]) / float(tg["vdrift"]) / float(tg["tbin"]),
                       n).astype(np.float32)
    return s, r, pad, time


def test_nominal_transform_inverts_the_readout_encoding():
    ev = synth.config2(n_tracks=400)
    raw = synth.encode_raw(ev, TG)
    x, y, z, ro = oracle.transform(TG, raw["sector"], raw["row"], raw["pad"], raw["time"], prec=64)
    assert np.array_equal(ro, ev.row)
    assert np.array_equal(x, TG["row_x"][ev.row].astype(np.float64))
    # the readout values are binary32: pad to ~1e-5 pads, time to ~3e-5 bins
    assert np.abs(y - ev.y).max() <= 1e-5 and np.abs(z - ev.z).max() <= 2e-5
    x32, y32, z32, _ = oracle.transform(TG, raw["sector"], raw["row"], raw["pad"], raw["time"])
    assert np.abs(y32 - y).max() <= 4e-6 and np.abs(z32 - z).max() <= 4e-5
    # the side of a cluster decides the sign of z (up to the smearing of
    # clusters next to the central membrane)
    side = raw["sector"] >= 18
    assert np.all(z[side] <= 1.0) and np.all(z[~side] >= -1.0)


def test_nominal_transform_hand_cases():
    tg = dict(TG, t0=np.float32(2.0))
    r = np.array([0, 62, 63, 151], np.uint16)
    pad = tg["pad_c"][r].copy()
    pad[2] += 1.0                                     # one pad right of the centre
    t_full = np.float32((250.0 / 2.58 + 2.0) / 0.2)  # the whole drift length
    time = np.array([(2.0 / 0.2), 0.0, t_full, (2.0 + 100.0 / 2.58) / 0.2], np.float32)
    s = np.array([3, 20, 0, 35], np.uint8)
    x, y, z, ro = oracle.transform(tg, s, r, pad, time, prec=64)
    assert np.allclose(y, [0, 0, 0.60, 0], atol=1e-6)
    # zero drift: z = +-250 (time 0 is t0 = 2 us before zero drift: 5.16 cm
    # beyond); full drift: z = 0; 100 cm of drift on side C
    assert z[0] == pytest.approx(250.0, abs=1e-4) and z[1] == pytest.approx(-250.0 - 2.58 * 2.0, abs=1e-4)
    assert z[2] == pytest.approx(0.0, abs=1e-4) and z[3] == pytest.approx(-150.0, abs=1e-4)
    assert np.array_equal(ro, r) and np.array_equal(x, tg["row_x"][r].astype(np.float64))


def _node_coords(tg):
    u = np.float64(tg["u0"]) + np.arange(tg["nu"]) / np.float64(tg["iu"])
    v = np.float64(tg["v0"]) + np.arange(tg["nv"]) / np.float64(tg["iv"])
    w = np.float64(tg["w0"]) + np.arange(tg["nw"]) / np.float64(tg["iw"])
    return u, v, w


def _trilinear_map(tg, coef):
    """Nodes holding f_q(u, v, w) = sum of coef[q] * (1, u, v, w, uv, vw, uw, uvw)."""
    u, v, w = _node_coords(tg)
    U, V, W = np.meshgrid(u, v, w, indexing="ij")
    basis = np.stack([np.ones_like(U), U, V, W, U * V, V * W, U * W, U * V * W])
    m = np.zeros((36, tg["nu"], tg["nv"], tg["nw"], 4), np.float64)
    for s in range(36):
        for q in range(3):
            m[s, ..., q] = np.tensordot(coef[s, q], basis, axes=1)
    return m


def test_residual_map_exact_on_trilinear_functions():
    rng = np.random.default_rng(5)
    # nodes must be exact binary32 values for an exact comparison in binary64:
    # powers-of-two coefficients on a grid with dyadic spacing
    tg = dict(TG, nu=5, nv=3, nw=9, u0=np.float32(0.0), iu=np.float32(1 / 32),
              v0=np.float32(-0.25), iv=np.float32(4.0), w0=np.float32(0.0), iw=np.float32(1 / 32),
              tbin=np.float32(0.25), vdrift=np.float32(2.0))
    coef = rng.integers(-4, 5, (36, 3, 8)) * np.array([2.0 ** -3, 2.0 ** -9, 2.0 ** -4, 2.0 ** -10,
                                                       2.0 ** -9, 2.0 ** -8, 2.0 ** -14, 2.0 ** -14])
    rm = _trilinear_map(tg, coef)
    assert np.array_equal(rm.astype(np.float32).astype(np.float64), rm)
    s, r, pad, time = _raw(4000, rng, tg)
    x0, y0, z0, _ = oracle.transform(tg, s, r, pad, time, prec=64)
    x, y, z, _ = oracle.transform(tg, s, r, pad, time, rmap=rm.astype(np.float32), prec=64)
    side = np.where(s >= 18, -1.0, 1.0)
    # the map's coordinates of every cluster, clamped to the grid
    u = np.clip(r.astype(np.float64), 0, 4 * 32)
    v = np.clip(y0 / x0, -0.25, 0.25)
    w = np.clip((250.0 - side * z0), 0, 8 * 32)
    basis = np.stack([np.ones_like(u), u, v, w, u * v, v * w, u * w, u * v * w])
    for q, (got, base) in enumerate(((x, x0), (y, y0), (z, z0))):
        want = np.einsum("nk,kn->n", coef[s, q], basis)
        assert np.abs((got - base) - want).max() <= 1e-9, q
    # a cluster on a node gets the node's value: row 64 is u node 2, the
    # centre pad is y = 0 (v node 1), a drift of 64 cm is w node 2
    s1 = np.array([7, 25], np.uint8)
    r1 = np.array([64, 64], np.uint16)
    p1 = tg["pad_c"][r1].astype(np.float32)
    t1 = np.array([128.0, 128.0], np.float32)          # 128 bins x 0.25 us x 2 cm/us
    xb, yb, zb, _ = oracle.transform(tg, s1, r1, p1, t1, prec=64)
    x1, y1, z1, _ = oracle.transform(tg, s1, r1, p1, t1, rmap=rm.astype(np.float32), prec=64)
    assert np.array_equal(x1 - xb, rm[s1, 2, 1, 2, 0])
    assert np.array_equal(y1 - yb, rm[s1, 2, 1, 2, 1])
    assert np.array_equal(z1 - zb, rm[s1, 2, 1, 2, 2])


def test_calibration_map_undoes_a_smooth_distortion():
    ev = synth.config2(n_tracks=800)
    dist = synth.Distortion(amp=1.0)
    raw_d = synth.encode_raw(ev, TG, dist=dist)
    rm = synth.calibration_map(TG, dist)
    x, y, z, _ = oracle.transform(TG, raw_d["sector"], raw_d["row"], raw_d["pad"], raw_d["time"],
                                  rmap=rm, prec=64)
    xu, yu, zu, _ = oracle.transform(TG, raw_d["sector"], raw_d["row"], raw_d["pad"],
                                     raw_d["time"], prec=64)
    x_true = TG["row_x"][ev.row].astype(np.float64)
    err_u = np.sqrt(np.mean((yu - ev.y) ** 2 + (zu - ev.z) ** 2))
    err_c = np.sqrt(np.mean((x - x_true) ** 2 + (y - ev.y) ** 2 + (z - ev.z) ** 2))
    assert err_u > 0.1
    # first-order inverse (|grad d| |d|) plus interpolation error: ~0.1 of
    # the distortion; a sign or axis mistake leaves at least the distortion
    assert err_c < 0.2 * err_u


def test_residual_map_reads_y_over_x_after_the_radial_offset():
    rng = np.random.default_rng(6)
    s, r, pad, time = _raw(500, rng)
    D = rng.uniform(-1, 1, (152, 18)).astype(np.float32)
    coef = np.zeros((36, 3, 8))
    coef[:, 1, 2] = 0.5                                # dy = v / 2
    rm = _trilinear_map(TG, coef).astype(np.float32)
    x0, y0, z0, _ = oracle.transform(TG, s, r, pad, time, prec=64)
    x, y, z, _ = oracle.transform(TG, s, r, pad, time, dmap=D, rmap=rm, prec=64)
    k = s.astype(np.int64) % 18
    xd = x0 + D[r, k].astype(np.float64)
    v = np.clip(y0 / xd, float(TG["v0"]), -float(TG["v0"]))
    assert np.abs(x - xd).max() <= 1e-12
    assert np.abs((y - y0) - 0.5 * v).max() <= 1e-7
    assert np.abs(z - z0).max() <= 1e-12


def test_invalid_raw_clusters_become_invalid_tracker_inputs():
    s = np.array([0, 36, 5, 40, 3], np.uint8)
    r = np.array([10, 10, 152, 200, 20], np.uint16)
    pad = np.array([10, 10, 10, 10, np.nan], np.float32)
    time = np.array([100, 100, 100, 100, 100], np.float32)
    x, y, z, ro = oracle.transform(TG, s, r, pad, time)
    assert list(ro[:4]) == [10, 0xFFFF, 0xFFFF, 0xFFFF]
    assert ro[4] == 20 and np.isnan(y[4])
