"""Pins of the CPU oracle against what geometry, the Kalman filter's
statistics and brute force fix independently of the oracle itself.

P1 generator on the analytic circle; P2 propagation vs the exact helix;
P3 Jacobian vs finite differences, arc series vs asin; P4 Kalman filter
(noise-free truth, chi2/ndf, pulls, Gluckstern's curvature resolution);
P5 grid invariants; P6 neighbour finder vs brute force at several grid
sizes; P7 cleaner / start-hit definitions; P8 tracklet cases; P9 selection
vs brute-force ownership; P10 efficiency floor.
"""
import numpy as np
import pytest

import oracle
import synth
from tests import helix

G = synth.geometry()
P = dict(oracle.DEFAULT_PARAMS)
RX = G["row_x"].astype(np.float64)


def _cov0():
    c = np.zeros(15)
    c[0], c[2], c[5], c[9], c[14] = 0.01, 0.0225, 1.0, 1.0, 100.0
    return c


# ---------------------------------------------------------------- P1 generator
def test_generator_points_on_circle():
    rng = np.random.default_rng(1)
    n = 40
    trk = dict(q=rng.choice([-1.0, 1.0], n), pt=rng.uniform(0.2, 5, n),
               phi0=rng.uniform(0, 2 * np.pi, n), tanl=rng.uniform(-1, 1, n),
               vx=np.zeros(n), vy=np.zeros(n), vz=rng.normal(0, 5, n))
    cr = synth._crossings(trk["q"], trk["pt"], trk["phi0"], trk["tanl"], trk["vx"], trk["vy"],
                          trk["vz"], G["row_x"])
    t = cr["trk"]
    R = trk["pt"][t] / (synth.C_LIGHT * synth.B_TESLA)
    cx = trk["q"][t] * R * np.sin(trk["phi0"][t])
    cy = -trk["q"][t] * R * np.cos(trk["phi0"][t])
    a = np.radians(20.0) * (cr["sec"] + 0.5)
    X = RX[cr["row"]] * np.cos(a) - cr["y"] * np.sin(a)
    Y = RX[cr["row"]] * np.sin(a) + cr["y"] * np.cos(a)
    assert np.max(np.abs(np.hypot(X - cx, Y - cy) - R)) < 1e-9
    # z linear in the transverse arc length with slope tan(lambda)
    assert np.max(np.abs(cr["z"] - trk["vz"][t] - trk["tanl"][t] * R * cr["psi"])) < 1e-9
    # every crossing lies inside its wedge
    assert np.all(np.abs(cr["y"]) <= RX[cr["row"]] * np.tan(np.radians(10)) + 1e-12)


# --------------------------------------------------------------- P2 propagation
def _random_states(rng, n, qmax=5.0, smax=0.5):
    st = np.zeros((n, 5))
    st[:, 0] = rng.uniform(-10, 10, n)
    st[:, 1] = rng.uniform(-100, 100, n)
    st[:, 2] = rng.uniform(-smax, smax, n)
    st[:, 3] = rng.uniform(-1, 1, n)
    st[:, 4] = rng.uniform(-qmax, qmax, n)
    return st


@pytest.mark.parametrize("prec,tol", [(64, 1e-8), (32, 1e-3)])
def test_propagation_matches_exact_helix(prec, tol):
    rng = np.random.default_rng(2)
    for st in _random_states(rng, 12, qmax=1.5, smax=0.2):
        # stays below snp_max over all rows
        y1, z1, s1 = helix.at(st, RX[0], RX[-1])
        if abs(s1) > 0.9:
            continue
        p, c = st.copy(), _cov0()
        for r in range(151):
            ok, p, c = oracle.propagate(G, P, p, c, RX[r], RX[r + 1], prec=prec)
            assert ok
        assert abs(p[0] - y1) < tol and abs(p[1] - z1) < tol
        assert abs(p[2] - s1) < tol * 1e-2
        # back to the start row: the step is reversible
        for r in range(151, 0, -1):
            ok, p, c = oracle.propagate(G, P, p, c, RX[r], RX[r - 1], prec=prec)
        assert np.allclose(p, st, atol=tol)


def test_walk_back_step_over_eight_rows_matches_helix_and_single_rows():
    # R16 walks the state back to the start row in steps of up to 8 rows:
    # one step over 8 rows lands on the exact helix (the arc-length series'
    # truncation aside) and carries the covariance as the 8 single-row steps
    # do, for curvatures down to pT = 0.1 GeV and |snp| up to the limit
    rng = np.random.default_rng(31)
    worst_pos = worst_cov = 0.0
    n = 0
    for st in _random_states(rng, 400, qmax=10.0, smax=0.97):
        for r in (151, 100, 40, 9):
            with np.errstate(invalid="ignore"):
                y1, z1, s1 = helix.at(st, RX[r], RX[r - 8])
            if not abs(s1) < 0.99:
                continue
            ok, p, c = oracle.propagate(G, P, st, _cov0(), RX[r], RX[r - 8], prec=64)
            if not ok:
                continue
            n += 1
            worst_pos = max(worst_pos, abs(p[0] - y1), abs(p[1] - z1))
            assert abs(p[2] - s1) < 1e-9
            q, cq = st.copy(), _cov0()
            for k in range(8):
                ok1, q, cq = oracle.propagate(G, P, q, cq, RX[r - k], RX[r - k - 1], prec=64)
                assert ok1
            assert np.allclose(p, q, rtol=0, atol=1e-3)
            worst_cov = max(worst_cov, np.max(np.abs(c - cq)) / np.max(np.abs(cq)))
    assert n > 1000
    assert worst_pos < 1e-3 and worst_cov < 1e-3, (worst_pos, worst_cov)


def test_propagation_straight_line_exact():
    st = np.array([1.0, 2.0, 0.3, 0.5, 0.0])
    ok, p, _ = oracle.propagate(G, P, st, _cov0(), 100.0, 110.0, prec=64)
    assert ok
    y, z, snp = helix.at(st, 100.0, 110.0)
    assert abs(p[0] - y) < 1e-12 and abs(p[1] - z) < 1e-12 and p[2] == 0.3


def test_propagation_refuses_snp_overflow():
    st = np.array([0.0, 0.0, 0.985, 0.1, -5.0])     # curvature drives snp past 0.99
    ok, p, c = oracle.propagate(G, P, st, _cov0(), 100.0, 102.0, prec=64)
    assert not ok and np.array_equal(p, st)


def test_propagation_refuses_state_outside_domain():
    # cos(phi) = sqrt(1 - snp^2) must exist at the start of the step too: an
    # update can leave |snp| >= snp_max, and a step that brings it back into
    # range must still fail (it would otherwise return NaN for y and z)
    # (kB < 0: q/pt of the sign of snp turns it back towards zero, so the
    # end point of each of these steps is inside the domain)
    for snp0 in (0.995, 1.02, -1.03):
        st = np.array([1.0, 2.0, snp0, 0.1, np.sign(snp0) * 20.0])
        for prec in (32, 64):
            ok, p, c = oracle.propagate(G, P, st, _cov0(), 100.0, 102.0, prec=prec)
            assert not ok and np.array_equal(p, st.astype(p.dtype)), (snp0, prec)
    # just inside the domain the step is taken
    st = np.array([1.0, 2.0, 0.989, 0.1, 20.0])
    ok, p, _ = oracle.propagate(G, P, st, _cov0(), 100.0, 102.0, prec=64)
    assert ok and np.isfinite(p).all() and p[2] < 0.989


def test_dense_event_outputs_are_finite():
    # a dense wedge (1500 tracks) where updates push some states past
    # |snp| = 1: every accepted tracklet and every track has finite
    # parameters, covariance and chi2
    ev = synth.config1(n_tracks=1500)
    o = oracle.track(G, P, ev.inst_off, ev.y, ev.z, ev.row)
    tl = o.tracklets
    acc = tl.status == 0
    assert acc.sum() > 1000
    assert np.isfinite(tl.par[acc]).all() and np.isfinite(tl.cov[acc]).all()
    assert np.isfinite(tl.chi2[acc]).all()
    T = o.tracks
    assert np.isfinite(T.par).all() and np.isfinite(T.cov).all() and np.isfinite(T.chi2).all()


# --------------------------------------------------------------- P3 Jacobian
def _jacobian(st, x1, x2, prec=64):
    F = np.zeros((5, 5))
    for i in range(5):
        c = np.zeros(15)
        c[oracle_ci(i, i)] = 1.0
        ok, _, c2 = oracle.propagate(G, P, st, c, x1, x2, prec=prec)
        assert ok
        for j in range(5):
            F[j, i] = c2[oracle_ci(j, i)]
    return F


def oracle_ci(i, j):
    return i * (i + 1) // 2 + j if i >= j else j * (j + 1) // 2 + i


def _fd(st, x1, x2, i, h):
    vals = []
    for k in (-2, -1, 1, 2):
        s = st.copy()
        s[i] += k * h
        ok, p, _ = oracle.propagate(G, P, s, _cov0(), x1, x2, prec=64)
        assert ok
        vals.append(p)
    return (vals[0] - 8 * vals[1] + 8 * vals[2] - vals[3]) / (12 * h)


@pytest.mark.parametrize("dx", [1.0728, -1.0728, 12.0])
def test_jacobian_matches_finite_differences(dx):
    rng = np.random.default_rng(3)
    steps = [1e-3, 1e-3, 1e-4, 1e-4, 1e-4]
    worst = 0.0
    for st in _random_states(rng, 150, qmax=5.0, smax=0.6):
        x1 = 120.0
        F = _jacobian(st, x1, x1 + dx)
        Ffd = np.stack([_fd(st, x1, x1 + dx, i, steps[i]) for i in range(5)], axis=1)
        err = np.abs(F - Ffd) / np.maximum(np.abs(Ffd), 1e-3)
        worst = max(worst, err.max())
    assert worst < 1e-6, worst


def test_jacobian_structure():
    """Entries the model fixes exactly: identity where nothing couples."""
    st = np.array([1.0, 5.0, 0.2, 0.4, 1.3])
    F = _jacobian(st, 100.0, 101.0728)
    kB = helix.kB()
    assert F[2, 4] == pytest.approx(kB * 1.0728, rel=1e-12)
    for (i, j) in [(0, 1), (1, 0), (2, 0), (2, 1), (2, 3), (3, 0), (3, 1), (3, 2), (3, 4),
                   (4, 0), (4, 1), (4, 2), (4, 3), (0, 3)]:
        assert F[i, j] == 0.0, (i, j)
    assert np.all(np.diag(F) == 1.0)


def test_arc_series_matches_asin():
    rng = np.random.default_rng(4)
    worst = 0.0
    for _ in range(300):
        st = np.array([0.0, 0.0, rng.uniform(-0.7, 0.7), 1.0, rng.uniform(-15.6, 15.6)])
        x1, x2 = 100.0, 100.0 + 1.0728
        ok, p, _ = oracle.propagate(G, P, st, _cov0(), x1, x2, prec=64)
        if not ok:
            continue
        arc = helix.exact_arc(st, x1, x2)
        worst = max(worst, abs(p[1] / arc - 1))
    assert worst < 1e-11, worst


# --------------------------------------------------------------- P4 Kalman
def _smeared_track(rng, st, rows, sy=0.1, sz=0.15):
    y, z, snp = helix.at(st, RX[rows[0]], RX[rows])
    return (y + rng.normal(0, sy, len(rows))).astype(np.float32), \
        (z + rng.normal(0, sz, len(rows))).astype(np.float32), y, z, snp


def test_kf_noise_free_truth_init():
    rng = np.random.default_rng(5)
    for st in _random_states(rng, 10, qmax=2.0, smax=0.3):
        rows = np.arange(152)
        y, z, snp = helix.at(st, RX[0], RX[rows])
        if np.max(np.abs(snp)) > 0.9:
            continue
        p, c = st.copy(), _cov0()
        for r in range(1, 152):
            ok, p, c = oracle.propagate(G, P, p, c, RX[r - 1], RX[r], prec=64)
            assert ok
            _, p, c = oracle.update(G, p, c, y[r], z[r], prec=64)
        truth = np.array([y[-1], z[-1], snp[-1], st[3], st[4]])
        assert np.all(np.abs(p - truth) <= 1e-9 * np.maximum(np.abs(truth), 1.0))


def test_kf_noise_free_r13_init_converges():
    rng = np.random.default_rng(6)
    for st in _random_states(rng, 10, qmax=2.0, smax=0.3):
        y, z, snp = helix.at(st, RX[0], RX)
        if np.max(np.abs(snp)) > 0.9:
            continue
        has = np.ones(152, np.uint8)
        ok, par, cov, chi2 = oracle.replay(G, P, 0, 0, 151, y, z, has, prec=64)
        assert ok
        truth = np.array([y[0], z[0], snp[0], st[3], st[4]])
        # hits were rounded to binary32, so compare at the float32 input level
        assert np.all(np.abs(par - truth) <= 1e-4 * np.maximum(np.abs(truth), 0.05)), (par, truth)


def test_kf_chi2_and_pulls():
    rng = np.random.default_rng(7)
    n_trk = 4000
    chi2n, pulls = [], []
    ndf_tot = 0
    chi2_tot = 0.0
    while len(pulls) < n_trk:
        st = np.array([rng.uniform(-5, 5), rng.uniform(-50, 50), rng.uniform(-0.3, 0.3),
                       rng.uniform(-1, 1), rng.choice([-1, 1]) * rng.uniform(0.2, 2.0)])
        y0, z0, snp = helix.at(st, RX[0], RX)
        if np.max(np.abs(snp)) > 0.8:
            continue
        ys, zs, yt, zt, _ = _smeared_track(rng, st, np.arange(152))
        ok, par, cov, chi2 = oracle.replay(G, P, 0, 0, 151, ys, zs, np.ones(152, np.uint8), prec=64)
        if not ok:
            continue
        ndf = 2 * 152 - 5
        chi2_tot += chi2
        ndf_tot += ndf
        truth = np.array([yt[0], zt[0], snp[0], st[3], st[4]])
        sig = np.sqrt(cov[[0, 2, 5, 9, 14]])
        pulls.append((par - truth) / sig)
    pulls = np.array(pulls)
    assert abs(chi2_tot / ndf_tot - 1) < 0.01
    mean = pulls.mean(axis=0)
    width = pulls.std(axis=0)
    assert np.all(np.abs(mean) < 0.05), mean
    assert np.all((width > 0.96) & (width < 1.04)), width


def test_kf_gluckstern_curvature_resolution():
    """sqrt(C_qpt) * |kB| vs Gluckstern's sigma_kappa for equally spaced points."""
    sy = 0.1
    N = 152
    Lproj = RX[-1] - RX[0]
    sk = sy / Lproj ** 2 * np.sqrt(720.0 * N ** 3 / ((N - 1) * (N + 1) * (N + 2) * (N + 3)))
    for qpt in (0.2, -0.5, 0.8):
        snp0 = -helix.kB() * qpt * Lproj / 2          # symmetric about snp = 0
        st = np.array([0.0, 0.0, snp0, 0.3, qpt])
        y, z, snp = helix.at(st, RX[0], RX)
        assert np.max(np.abs(snp)) <= 0.1
        ok, par, cov, chi2 = oracle.replay(G, P, 0, 0, 151, y, z, np.ones(152, np.uint8), prec=64)
        assert ok
        s = np.sqrt(cov[14]) * abs(helix.kB())
        assert abs(s / sk - 1) < 0.02, (s, sk)


# --------------------------------------------------------------- P5 grid
def _with_bad(ev):
    y = ev.y.copy()
    z = ev.z.copy()
    row = ev.row.copy()
    y[3] = np.nan
    row[5] = 200
    y[7] = 1e4
    z[11] = np.inf
    return y, z, row


def test_grid_invariants():
    ev = synth.config1()
    y, z, row = _with_bad(ev)
    gr = oracle.grid_build(G, P, ev.inst_off, y, z, row)
    assert gr.n_bad == 4
    valid = np.ones(ev.n, bool)
    valid[[3, 5, 7, 11]] = False
    n_valid = int(valid.sum())
    perm = gr.perm[:n_valid]
    assert np.all(gr.perm[n_valid:] == -1) and np.all(gr.sseg[n_valid:] == -1)
    assert np.array_equal(np.sort(perm), np.nonzero(valid)[0])
    assert np.array_equal(row[perm], gr.sseg[:n_valid] % 152)
    assert np.array_equal(gr.ys[:n_valid], y[perm]) and np.array_equal(gr.zs[:n_valid], z[perm])
    ro = gr.row_off[:153]
    assert np.array_equal(np.diff(ro), np.bincount(row[valid], minlength=152))
    for r in range(152):
        ny, nz, base, cnt = gr.meta_i[r]
        bo = gr.bin_off[base:base + ny * nz + 1]
        assert bo[0] == ro[r] and bo[-1] == ro[r + 1] and np.all(np.diff(bo) >= 0)
        nb = max(1, cnt // 2)
        assert ny * nz <= 3 * nb + 8
        # bin id of every sorted position of the row
        b = np.repeat(np.arange(ny * nz), np.diff(bo))
        iy, iz = b % ny, b // ny
        yy, zz, pp = gr.ys[ro[r]:ro[r + 1]], gr.zs[ro[r]:ro[r + 1]], perm[ro[r]:ro[r + 1]]
        # input order inside a bin
        for k in range(ny * nz):
            seg = pp[bo[k] - ro[r]:bo[k + 1] - ro[r]]
            assert np.all(np.diff(seg) > 0)
        # the data box spans the bins: the row's smallest coordinate lands in
        # column 0 and its largest in the last column
        for ax_i, ax_v, n_ax in ((iy, yy, ny), (iz, zz, nz)):
            if len(ax_v):
                assert ax_i[np.argmin(ax_v)] == 0 and ax_i[np.argmax(ax_v)] == n_ax - 1
        # monotone binning: higher bin column => not smaller coordinate
        for ax_i, ax_v, n_ax in ((iy, yy, ny), (iz, zz, nz)):
            for k in range(n_ax - 1):
                lo, hi = ax_v[ax_i == k], ax_v[ax_i == k + 1]
                if len(lo) and len(hi):
                    assert lo.max() <= hi.min()


# --------------------------------------------------------------- P6 neighbours
def _tiny_event(rng, n_tracks=6, n_noise=30, rows=range(40, 45)):
    rows = np.array(list(rows))
    ys, zs, rs, lab = [], [], [], []
    for t in range(n_tracks):
        st = np.array([rng.uniform(-8, 8), rng.uniform(-10, 10), rng.uniform(-0.4, 0.4),
                       rng.uniform(-0.8, 0.8), rng.uniform(-3, 3)])
        y, z, _ = helix.at(st, RX[rows[0]], RX[rows])
        ys.append(y + rng.normal(0, 0.1, len(rows)))
        zs.append(z + rng.normal(0, 0.15, len(rows)))
        rs.append(rows)
        lab.append(np.full(len(rows), t))
    ys.append(rng.uniform(-12, 12, n_noise))
    zs.append(rng.uniform(-15, 15, n_noise))
    rs.append(rng.choice(rows, n_noise))
    lab.append(np.full(n_noise, -1))
    y = np.concatenate(ys).astype(np.float32)
    z = np.concatenate(zs).astype(np.float32)
    r = np.concatenate(rs).astype(np.uint16)
    lab = np.concatenate(lab)
    o = rng.permutation(len(y))
    return y[o], z[o], r[o], lab[o]


def _links_by_input(gr, up, dn):
    """(up, down) as input indices, indexed by input index."""
    n = len(gr.perm)
    U = np.full(n, -1)
    D = np.full(n, -1)
    v = gr.perm >= 0
    U[gr.perm[v]] = np.where(up[v] >= 0, gr.perm[up[v]], -1)
    D[gr.perm[v]] = np.where(dn[v] >= 0, gr.perm[dn[v]], -1)
    return U, D


def _python_brute_nf(y, z, row):
    """All-triples neighbour search in binary32 arithmetic, plain Python."""
    f = np.float32
    ivy = f(1.0 / (1.5 * float(G["sigma_y2"])))
    ivz = f(1.0 / (1.5 * float(G["sigma_z2"])))
    rx = G["row_x"]
    n = len(y)
    U = np.full(n, -1)
    D = np.full(n, -1)
    for h in range(n):
        r = int(row[h])
        if r == 0 or r == 151:
            continue
        t = (rx[r] - rx[r - 1]) / (rx[r + 1] - rx[r - 1])
        best = None
        for u in np.nonzero(row == r + 1)[0]:
            if not (abs(y[u] - y[h]) <= f(3.0) and abs(z[u] - z[h]) <= f(3.5)):
                continue
            for d in np.nonzero(row == r - 1)[0]:
                if not (abs(y[d] - y[h]) <= f(3.0) and abs(z[d] - z[h]) <= f(3.5)):
                    continue
                ey = y[h] - (y[d] + (y[u] - y[d]) * t)
                ez = z[h] - (z[d] + (z[u] - z[d]) * t)
                sc = (ey * ey) * ivy + (ez * ez) * ivz
                if sc <= f(13.8) and (best is None or (sc, u, d) < best):
                    best = (sc, u, d)
        if best is not None:
            U[h], D[h] = best[1], best[2]
    return U, D


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_neighbours_brute_force_and_grid_independence(seed):
    rng = np.random.default_rng(seed)
    y, z, row, lab = _tiny_event(rng)
    io = np.array([0, len(y)], np.int64)
    Ub, Db = _python_brute_nf(y, z, row)
    assert (Ub >= 0).sum() > 0
    for occ in (0.25, 1.0, 2.0, 8.0, 64.0):
        Pq = dict(P, grid_occupancy=occ)
        gr = oracle.grid_build(G, Pq, io, y, z, row)
        for brute in (False, True):
            up, dn = oracle.neighbours(G, Pq, gr, brute=brute)
            U, D = _links_by_input(gr, up, dn)
            assert np.array_equal(U, Ub) and np.array_equal(D, Db), (occ, brute)


def test_neighbours_isolated_tracks_link_true_neighbours():
    rng = np.random.default_rng(14)
    rows = np.arange(20, 60)
    ys, zs, rs, ls = [], [], [], []
    for t, z0 in enumerate((-100.0, -50.0, 0.0, 50.0, 100.0)):   # well separated in z
        st = np.array([rng.uniform(-5, 5), z0, rng.uniform(-0.3, 0.3), rng.uniform(-0.3, 0.3),
                       rng.uniform(-3, 3)])
        yy, zz, _ = helix.at(st, RX[rows[0]], RX[rows])
        ys.append(yy + rng.normal(0, 0.1, len(rows)))
        zs.append(zz + rng.normal(0, 0.15, len(rows)))
        rs.append(rows)
        ls.append(np.full(len(rows), t))
    o = rng.permutation(5 * len(rows))
    y = np.concatenate(ys).astype(np.float32)[o]
    z = np.concatenate(zs).astype(np.float32)[o]
    row = np.concatenate(rs).astype(np.uint16)[o]
    lab = np.concatenate(ls)[o]
    io = np.array([0, len(y)], np.int64)
    gr = oracle.grid_build(G, P, io, y, z, row)
    up, dn = oracle.neighbours(G, P, gr)
    U, D = _links_by_input(gr, up, dn)
    inner = (row > 20) & (row < 59)
    for h in np.nonzero(inner)[0]:
        if U[h] >= 0:
            assert lab[U[h]] == lab[h] and row[U[h]] == row[h] + 1
            assert lab[D[h]] == lab[h] and row[D[h]] == row[h] - 1
    assert (U[inner] >= 0).mean() > 0.9


# --------------------------------------------------------------- P7 clean/start
def test_clean_and_start_hits_definitions():
    ev = synth.config2(n_tracks=300)
    r = oracle.track(G, P, ev.inst_off, ev.y, ev.z, ev.row)
    up, dn, up2, dn2 = r.up, r.dn, r.up2, r.dn2
    n = len(up)
    for h in range(n):
        if up2[h] >= 0:
            assert dn[up2[h]] == h and up[h] == up2[h]
        else:
            assert up[h] < 0 or dn[up[h]] != h
        if dn2[h] >= 0:
            assert up[dn2[h]] == h and dn[h] == dn2[h]
    want = [h for h in range(n) if dn2[h] == -1 and up2[h] >= 0 and up2[up2[h]] >= 0]
    assert list(r.start) == want


# --------------------------------------------------------------- P8 tracklets
def _single_track_event(st, rows, smear, rng):
    y, z, snp = helix.at(st, RX[rows[0]], RX[rows])
    if smear:
        y = y + rng.normal(0, 0.1, len(rows))
        z = z + rng.normal(0, 0.15, len(rows))
    return y.astype(np.float32), z.astype(np.float32), rows.astype(np.uint16), snp


def test_tracklet_single_noise_free_track():
    rng = np.random.default_rng(21)
    st = np.array([2.0, 10.0, 0.1, 0.5, 1.2])
    rows = np.arange(152)
    y, z, row, snp = _single_track_event(st, rows, False, rng)
    o = rng.permutation(152)
    io = np.array([0, 152], np.int64)
    for prec in (32, 64):
        r = oracle.track(G, P, io, y[o], z[o], row[o], prec=prec)
        assert len(r.tracks.chi2) == 1
        assert r.tracks.hit_off[1] == 152
        assert np.array_equal(np.sort(r.tracks.hit_clu), np.arange(152))
        truth = np.array([y[0], z[0], snp[0], st[3], st[4]])
        tol = 1e-4 if prec == 64 else 2e-3
        assert np.all(np.abs(r.tracks.par[0] - truth) <= tol * np.maximum(np.abs(truth), 0.05))


def test_tracklets_two_crossing_tracks():
    rng = np.random.default_rng(22)
    rows = np.arange(30, 130)
    a = np.array([0.0, 0.0, 0.15, 0.3, 2.0])
    # second track passes through the same (y, z) at row 80 with other slopes
    ya, za, _ = helix.at(a, RX[30], RX[80])
    b80 = np.array([ya, za, -0.2, 0.25, -1.5], dtype=np.float64)
    yb, zb, _ = helix.at(b80, RX[80], RX[rows])
    y1, z1, r1, _ = _single_track_event(a, rows, True, rng)
    y2 = (yb + rng.normal(0, 0.1, len(rows))).astype(np.float32)
    z2 = (zb + rng.normal(0, 0.15, len(rows))).astype(np.float32)
    y = np.concatenate([y1, y2])
    z = np.concatenate([z1, z2])
    row = np.concatenate([r1, rows.astype(np.uint16)])
    lab = np.repeat([0, 1], len(rows))
    r = oracle.track(G, P, np.array([0, len(y)], np.int64), y, z, row)
    T = r.tracks
    assert len(T.chi2) == 2
    for k in range(2):
        l = lab[T.hit_clu[T.hit_off[k]:T.hit_off[k + 1]]]
        assert np.all(l == l[0]) and len(l) >= 0.95 * len(rows)


def test_tracklet_stops_at_sector_edge():
    rng = np.random.default_rng(23)
    st = np.array([10.0, 0.0, 0.25, 0.2, -1.0])      # bends out through the +y edge
    rows = np.arange(0, 152)
    y, z, snp = helix.at(st, RX[0], RX[rows])
    inside = (np.abs(y) <= RX[rows] * np.tan(np.radians(10))) & (np.abs(snp) < 0.99)
    last = np.nonzero(~inside)[0][0]
    assert 30 <= last < 140
    rows = rows[:last]
    y, z, row, _ = _single_track_event(st, rows, True, rng)
    r = oracle.track(G, P, np.array([0, len(y)], np.int64), y, z, row)
    assert len(r.tracks.chi2) == 1
    tl = r.tracklets
    k = np.nonzero(tl.status == 0)[0][0]
    assert tl.rmax[k] == rows[-1]


def _first_chain_tracklet(y, z, row):
    """Chain result and the tracklet of the lowest start hit (single instance)."""
    r = oracle.track(G, P, np.array([0, len(y)], np.int64), y, z, row)
    t = int(np.argmin(r.grid.sseg[r.start]))
    return r, t


def test_tracklet_search_stops_after_consecutive_misses_only():
    # R15: the upward search ends at the tc_max_miss-th consecutive row without
    # a hit; a found hit starts the count again.  The links end at row 38
    # (rows 40.. are missing), so rows from 39 up are reached by the search.
    rng = np.random.default_rng(24)
    st = np.array([1.0, 5.0, 0.05, 0.4, 0.8])
    rows = np.arange(152)
    y, z, row, _ = _single_track_event(st, rows, False, rng)
    m = P["tc_max_miss"]
    for gap, top in ((m - 1, 151), (m, 39)):
        keep = (rows < 40) | (rows >= 40 + gap)
        r, t = _first_chain_tracklet(y[keep], z[keep], row[keep])
        assert r.tracklets.rmax[t] == top
    # 2m scattered misses (every other row of 60..100), never m in a row
    keep = ~((rows >= 60) & (rows <= 100) & (rows % 2 == 0))
    assert (~keep).sum() >= 2 * m
    r, t = _first_chain_tracklet(y[keep], z[keep], row[keep])
    assert r.tracklets.rmax[t] == 151 and r.tracklets.nhit[t] == keep.sum()


def test_tracklet_kept_from_min_tracklet_hits():
    # R17: a tracklet is kept iff it has at least min_tracklet_hits hits.  A
    # noise-free track on rows 50..50+k-1 only gives one tracklet of k hits.
    rng = np.random.default_rng(25)
    st = np.array([-3.0, 20.0, -0.05, 0.3, 0.5])
    k = P["min_tracklet_hits"]
    for nrow, status in ((k - 1, 1), (k, 0)):
        rows = np.arange(50, 50 + nrow)
        y, z, row, _ = _single_track_event(st, rows, False, rng)
        r, t = _first_chain_tracklet(y, z, row)
        assert r.tracklets.nhit[t] == nrow and r.tracklets.status[t] == status
    # the kept one is the track: two measurements per hit less five
    # parameters, state given at the innermost hit's plane (R17)
    T = r.tracks
    assert len(T.chi2) == 1 and T.hit_off[1] == k
    assert T.ndf[0] == 2 * k - 5 and T.x_ref[0] == np.float32(G["row_x"][50])


def test_tracklet_search_tie_goes_to_lower_input_index():
    # R15: two clusters at the same (y, z) of row 100 give the search an exact
    # chi2 tie, which the lower input index wins.  Row 70 is missing, so the
    # first chain's tracklet reaches row 100 by searching, not by links.
    rng = np.random.default_rng(26)
    st = np.array([0.5, -8.0, 0.08, -0.35, -0.6])
    rows = np.arange(152)
    y, z, row, _ = _single_track_event(st, rows, False, rng)
    keep = rows != 70
    y, z, row = y[keep], z[keep], row[keep]
    i100 = int(np.nonzero(row == 100)[0][0])
    for dup_first in (True, False):
        # the copy of the row-100 cluster goes before or after all others
        if dup_first:
            yy, zz, rr = (np.concatenate([[y[i100]], y]), np.concatenate([[z[i100]], z]),
                          np.concatenate([[row[i100]], row]))
            lo = 0
        else:
            yy, zz, rr = (np.append(y, y[i100]), np.append(z, z[i100]),
                          np.append(row, row[i100]))
            lo = i100
        r, t = _first_chain_tracklet(yy.astype(np.float32), zz.astype(np.float32),
                                     rr.astype(np.uint16))
        assert r.grid.sseg[r.start[t]] % 152 < 70
        assert r.grid.perm[r.tracklets.hit[t, 100]] == lo


def test_tracklet_search_window_follows_each_axis_variance():
    # R15: the search window is sqrt(pick * S) + margin per axis, with S00 for
    # y and S11 for z.  The row-100 hit of a noise-free track is moved 0.5 cm
    # in z: chi2 ~ 0.25 / S11 ~ 11 <= 13.8, beyond the y-sized half-width
    # (~0.4 cm) but inside the z-sized one (~0.58 cm).  A 40 x 40 cm lattice of
    # other clusters on that row (kept 2 cm away from the track) makes 1 cm
    # bins with an edge 0.44 cm above the true z, so a z window of the y size
    # never reaches the moved hit's bin.  Row 70 is missing: the first chain's
    # tracklet reaches row 100 by searching.
    rng = np.random.default_rng(27)
    st = np.array([0.5, -8.0, 0.08, -0.35, -0.6])
    rows = np.arange(152)
    y, z, row, _ = _single_track_event(st, rows, False, rng)
    yt, zt = float(y[100]), float(z[100])
    z = z.copy()
    z[100] = np.float32(zt + 0.5)
    keep = rows != 70
    y, z, row = y[keep], z[keep], row[keep]
    moved = int(np.nonzero(row == 100)[0][0])
    y0, z0 = np.float32(yt - 20.3), np.float32(zt + 0.44 - 20)
    ly, lz = np.meshgrid(y0 + np.float32(40) * np.arange(40, dtype=np.float32) / 39,
                         z0 + np.float32(40) * np.arange(40, dtype=np.float32) / 39)
    ly, lz = ly.ravel().astype(np.float32), lz.ravel().astype(np.float32)
    far = np.hypot(ly - yt, lz - zt) > 2.0
    ly, lz = ly[far], lz[far]
    extra = 1601 - 1 - len(ly)                          # at least 1600 clusters on the row
    ly = np.append(ly, np.full(extra, y0 + 0.5, np.float32))
    lz = np.append(lz, z0 + 0.5 + 0.01 * np.arange(extra, dtype=np.float32))
    yy = np.concatenate([y, ly]).astype(np.float32)
    zz = np.concatenate([z, lz]).astype(np.float32)
    rr = np.concatenate([row, np.full(len(ly), 100, np.uint16)])
    p = dict(P, grid_occupancy=1.0)
    r = oracle.track(G, p, np.array([0, len(yy)], np.int64), yy, zz, rr)
    ny, nz = r.grid.meta_i[100][:2]
    assert (ny, nz) == (40, 40) and r.grid.meta_f[100][1] == z0 and r.grid.meta_f[100][3] == 1
    t = int(np.argmin(r.grid.sseg[r.start]))
    assert r.grid.sseg[r.start[t]] % 152 < 70
    assert r.grid.perm[r.tracklets.hit[t, 100]] == moved


def test_tracklets_independent_of_the_grid():
    # R15's window holds every cluster with chi2 <= tc_chi2_pick (the bounding
    # box of that ellipse plus a margin), and ties go by input index, so the
    # tracklets do not depend on the bin size; one bin per row is a full scan.
    ev = synth.config2(n_tracks=300)
    ref = None
    for occ in (0.5, 2.0, 1e9):
        r = oracle.track(G, dict(P, grid_occupancy=occ), ev.inst_off, ev.y, ev.z, ev.row)
        tl, perm = r.tracklets, r.grid.perm
        got = {}
        for t in range(len(r.start)):
            hits = tuple(int(perm[h]) if h >= 0 else -1
                         for h in tl.hit[t, tl.rmin[t]:tl.rmax[t] + 1])
            got[int(perm[r.start[t]])] = (tl.status[t], tl.nhit[t], tl.rmin[t], hits,
                                          tl.chi2[t].tobytes(), tl.par[t].tobytes())
        if ref is None:
            ref = got
        else:
            assert got == ref


# --------------------------------------------------------------- P9 selection
def test_selection_matches_brute_force_ownership():
    ev = synth.config2(n_tracks=600)
    r = oracle.track(G, P, ev.inst_off, ev.y, ev.z, ev.row)
    tl, st = r.tracklets, r.start
    n = len(r.up)
    best = {}
    for t in range(len(st)):
        if tl.status[t] != 0:
            continue
        inst = r.grid.sseg[st[t]] // 152
        key = (int(tl.nhit[t]), -float(np.float32(tl.chi2[t])),
               -(int(r.grid.perm[st[t]]) - int(ev.inst_off[inst])))
        for rr in range(tl.rmin[t], tl.rmax[t] + 1):
            h = tl.hit[t, rr]
            if h >= 0 and (h not in best or key > best[h][0]):
                best[h] = (key, t)
    own = {}
    for h, (_, t) in best.items():
        own.setdefault(t, []).append(h)
    tracks = [t for t in range(len(st)) if len(own.get(t, [])) >= P["min_track_hits"]]
    T = r.tracks
    assert len(T.chi2) == len(tracks)
    for k, t in enumerate(tracks):
        got = T.hit_clu[T.hit_off[k]:T.hit_off[k + 1]]
        want = r.grid.perm[sorted(own[t], key=lambda h: r.grid.sseg[h])]
        assert np.array_equal(got, want)
    # each cluster belongs to at most one track, and clu2trk agrees
    assert len(np.unique(T.hit_clu)) == len(T.hit_clu)
    c2t = np.full(n, -1)
    for k in range(len(T.chi2)):
        c2t[T.hit_clu[T.hit_off[k]:T.hit_off[k + 1]]] = k
    assert np.array_equal(c2t, T.clu2trk)


def test_selection_merges_broken_chain_clone():
    rng = np.random.default_rng(31)
    st = np.array([1.0, 5.0, 0.05, 0.4, 0.8])
    rows = np.arange(152)
    y, z, row, _ = _single_track_event(st, rows, True, rng)
    keep = rows != 70             # delete one hit: two link chains
    y, z, row = y[keep], z[keep], row[keep]
    r = oracle.track(G, P, np.array([0, len(y)], np.int64), y, z, row)
    assert len(r.start) >= 2
    assert len(r.tracks.chi2) == 1
    assert r.tracks.hit_off[1] == len(y)


@pytest.mark.parametrize("lower_first", [True, False])
def test_selection_exact_key_tie_goes_to_lower_start_index(lower_first):
    # R20: two tracklets with the same hit count and bit-identical chi2 share
    # the hits of rows 40..59; each also holds a hit of its own on row 39,
    # which is its start hit.  The tie goes to the start hit with the lower
    # input index, whatever the tracklets' order in the list: that tracklet
    # owns 21 hits and becomes the one track, the other owns one.
    ev = synth.config1()
    gr = oracle.grid_build(G, P, ev.inst_off, ev.y, ev.z, ev.row)
    ro = gr.row_off
    assert np.all(np.diff(ro[39:61]) >= 1) and ro[40] - ro[39] >= 2
    a, b = int(ro[39]), int(ro[39]) + 1
    lo, hi = (a, b) if gr.perm[a] < gr.perm[b] else (b, a)
    starts = [lo, hi] if lower_first else [hi, lo]
    nr = G["n_rows"]
    hit = np.full((2, nr), -1, np.int32)
    for t, s0 in enumerate(starts):
        hit[t, 39] = s0
        hit[t, 40:60] = ro[40:60]
    cov = np.zeros((2, 15), np.float32)
    cov[:, [0, 2, 5, 9, 14]] = 1.0
    tl = oracle.Tracklets(np.zeros((2, 5), np.float32), cov,
                          np.full(2, 3.25, np.float32), np.full(2, 21, np.int32),
                          np.full(2, 39, np.int32), np.full(2, 59, np.int32), hit,
                          np.zeros(2, np.int32))
    T = oracle.select(G, P, ev.inst_off, gr, np.array(starts, np.int32), tl)
    assert len(T.chi2) == 1 and T.hit_off[1] == 21
    assert gr.perm[lo] in T.hit_clu and gr.perm[hi] not in T.hit_clu
    assert T.clu2trk[gr.perm[lo]] == 0 and T.clu2trk[gr.perm[hi]] == -1


def test_selection_capacity_truncates_in_order():
    ev = synth.config2(n_tracks=300)
    full = oracle.track(G, P, ev.inst_off, ev.y, ev.z, ev.row)
    nt = len(full.tracks.chi2)
    cut = oracle.select(G, P, ev.inst_off, full.grid, full.start, full.tracklets,
                        cap_tracks=nt // 2, cap_hits=10 ** 9)
    assert len(cut.chi2) == nt // 2 and cut.need_tracks == nt
    assert np.array_equal(cut.hit_off, full.tracks.hit_off[:nt // 2 + 1])
    h = int(full.tracks.hit_off[nt // 3]) + 1
    cut2 = oracle.select(G, P, ev.inst_off, full.grid, full.start, full.tracklets,
                         cap_tracks=nt, cap_hits=h)
    assert len(cut2.chi2) == nt // 3 and cut2.need_hits == full.tracks.hit_off[-1]


# --------------------------------------------------------------- P10 physics
def test_config1_efficiency_floor():
    ev = synth.config1()
    r = oracle.track(G, P, ev.inst_off, ev.y, ev.z, ev.row)
    T = r.tracks
    lab = ev.label
    found = set()
    for k in range(len(T.chi2)):
        l = lab[T.hit_clu[T.hit_off[k]:T.hit_off[k + 1]]]
        u, c = np.unique(l, return_counts=True)
        j = c.argmax()
        if u[j] >= 0 and c[j] > 0.5 * len(l):
            found.add(u[j])
    u, c = np.unique(lab[lab >= 0], return_counts=True)
    good = u[c >= 30]
    assert np.mean([g in found for g in good]) >= 0.9


def test_oracle_is_deterministic():
    ev = synth.config1()
    a = oracle.track(G, P, ev.inst_off, ev.y, ev.z, ev.row)
    b = oracle.track(G, P, ev.inst_off, ev.y, ev.z, ev.row)
    assert np.array_equal(a.tracklets.par, b.tracklets.par)
    assert np.array_equal(a.tracks.clu2trk, b.tracks.clu2trk)


def test_oracle_matches_stored_golden_summary():
    """Regression of the oracle itself (values written by tests/golden/make_golden.py)."""
    import json
    import os
    from tests.golden.make_golden import summary
    with open(os.path.join(os.path.dirname(__file__), "golden", "config1_oracle.json")) as f:
        want = json.load(f)
    assert summary() == want


def test_neighbours_non_uniform_rows_and_exact_ties():
    """Uneven row pitch fixes which row spacing the midpoint fraction uses;
    duplicated clusters give exact score ties, which go to the lower input
    index of u, then of d."""
    rng = np.random.default_rng(41)
    g2 = dict(G)
    rx = G["row_x"].astype(np.float64).copy()
    rx[41] += 0.4                      # rows 40, 41, 42 no longer evenly spaced
    rx[43] -= 0.3
    g2["row_x"] = rx.astype(np.float32)
    y, z, row, lab = _tiny_event(rng, n_tracks=8, n_noise=20)
    # duplicate some clusters on rows 42 and 40 (identical coordinates)
    dup = np.nonzero((row == 42) | (row == 40))[0][:6]
    y = np.concatenate([y, y[dup]])
    z = np.concatenate([z, z[dup]])
    row = np.concatenate([row, row[dup]])
    io = np.array([0, len(y)], np.int64)

    f = np.float32
    ivy = f(1.0 / (1.5 * float(G["sigma_y2"])))
    ivz = f(1.0 / (1.5 * float(G["sigma_z2"])))
    X = g2["row_x"]
    n = len(y)
    Ub = np.full(n, -1)
    Db = np.full(n, -1)
    ties = 0
    for h in range(n):
        r = int(row[h])
        t = (X[r] - X[r - 1]) / (X[r + 1] - X[r - 1])
        cands = []
        for u in np.nonzero(row == r + 1)[0]:
            if abs(y[u] - y[h]) <= f(3.0) and abs(z[u] - z[h]) <= f(3.5):
                for d in np.nonzero(row == r - 1)[0]:
                    if abs(y[d] - y[h]) <= f(3.0) and abs(z[d] - z[h]) <= f(3.5):
                        ey = y[h] - (y[d] + (y[u] - y[d]) * t)
                        ez = z[h] - (z[d] + (z[u] - z[d]) * t)
                        sc = (ey * ey) * ivy + (ez * ez) * ivz
                        if sc <= f(13.8):
                            cands.append((sc, u, d))
        if cands:
            best = min(cands)
            ties += sum(1 for c in cands if c[0] == best[0]) > 1
            Ub[h], Db[h] = best[1], best[2]
    assert ties > 0
    gr = oracle.grid_build(g2, P, io, y, z, row)
    up, dn = oracle.neighbours(g2, P, gr)
    U, D = _links_by_input(gr, up, dn)
    assert np.array_equal(U, Ub) and np.array_equal(D, Db)


def test_replay_straight_line_three_hits_exact():
    """A noise-free straight track: the start estimate (slopes from the first
    and third hit over the chord) is exact, so every later residual is zero."""
    st = np.array([3.0, -20.0, 0.5, 0.7, 0.0])
    rows = np.arange(10, 13)
    y, z, snp = helix.at(st, RX[10], RX[rows])
    hy = np.zeros(152)
    hz = np.zeros(152)
    has = np.zeros(152, np.uint8)
    hy[rows], hz[rows], has[rows] = y, z, 1
    # use binary32-exact inputs so that the check is exact in binary64
    hy = hy.astype(np.float32)
    hz = hz.astype(np.float32)
    ok, par, cov, chi2 = oracle.replay(G, P, 10, 10, 12, hy, hz, has, prec=64)
    assert ok
    dxi = RX[12] - RX[10]
    dyi = float(hy[12]) - float(hy[10])
    dzi = float(hz[12]) - float(hz[10])
    L = np.hypot(dxi, dyi)
    assert par[3] == pytest.approx(dzi / L, rel=1e-12, abs=1e-12)
    assert par[2] == pytest.approx(dyi / L, rel=1e-12, abs=1e-12)
    assert chi2 < 1e-10


def test_tracklet_straight_line_start_state_exact():
    """R13 through the tracker itself: clusters exactly on a straight line
    (no field bending, qpt = 0) with both slopes nonzero.  The start state
    takes snp and tgl from the chord of the first and third hit, so it is
    the line's own direction: every update has zero residual, the fit's
    chi2 vanishes, and the output keeps snp = dy/L and tgl = dz/L with
    L the transverse chord.  A start tgl of dz/dx instead of dz/L would be
    off by the factor 1/cos(phi) and leave residuals at the next hits."""
    geo = dict(G, bz=0.0)
    rows = np.arange(152)
    x = G["row_x"].astype(np.float32)
    # binary32-exact points: multiplying by powers of two rounds nothing
    y = (np.float32(0.125) * x).astype(np.float32)
    z = (np.float32(-0.5) * x).astype(np.float32)
    o = np.random.default_rng(31).permutation(152)
    io = np.array([0, 152], np.int64)
    r = oracle.track(geo, P, io, y[o], z[o], rows.astype(np.uint16)[o], prec=64)
    tl = r.tracklets
    kept = np.nonzero(tl.status == 0)[0]
    assert len(kept) >= 1
    slope_y, slope_z = 0.125, -0.5
    snp = slope_y / np.hypot(1.0, slope_y)
    tgl = slope_z / np.hypot(1.0, slope_y)
    for t in kept:
        assert tl.chi2[t] <= 1e-10
        assert abs(tl.par[t, 2] - snp) <= 1e-12 and abs(tl.par[t, 3] - tgl) <= 1e-12
        assert abs(tl.par[t, 4]) <= 1e-10
        r0 = tl.rmin[t]
        assert abs(tl.par[t, 0] - float(y[r0])) <= 1e-10
        assert abs(tl.par[t, 1] - float(z[r0])) <= 1e-10
    assert len(r.tracks.chi2) == 1 and r.tracks.hit_off[1] == 152


@pytest.mark.parametrize("occ", [0.5, 1.0, 2.0])
def test_grid_bins_hold_the_requested_occupancy(occ):
    """R10 as a property: a row of n clusters asks for nb = floor(n / occ)
    square bins over its data box.  Where the area term sets the width
    (w^2 = dy dz / nb above both of its floors), ceil on each axis gives at
    least nb bins, and one rounding step per axis stays within a small
    factor of nb; over all rows the mean number of clusters per bin then
    lies between occ / 2.5 and occ.  A width taken without the square root
    would leave one or two bins per row."""
    evs = (synth.config1(), synth.config2(n_tracks=2000))
    for ev in evs:
        Pk = dict(P, grid_occupancy=occ)
        gr = oracle.grid_build(G, Pk, ev.inst_off, ev.y, ev.z, ev.row, prec=32)
        tot_c = tot_b = 0
        n_area = 0
        for i in range(len(ev.inst_off) - 1):
            a, b = int(ev.inst_off[i]), int(ev.inst_off[i + 1])
            ys, zs, rs = ev.y[a:b].astype(np.float64), ev.z[a:b].astype(np.float64), ev.row[a:b]
            for r in range(152):
                ny, nz, _, cnt = gr.meta_i[i * 152 + r]
                if cnt == 0:
                    continue
                sel = rs == r
                dy = ys[sel].max() - ys[sel].min()
                dz = zs[sel].max() - zs[sel].min()
                nb = max(1, int(np.floor(cnt / occ)))
                assert ny * nz <= 5 * nb + 4
                if np.sqrt(dy * dz / nb) > max(1.0, max(dy, dz) / nb) * 1.001:
                    n_area += 1
                    assert nb <= ny * nz <= 2 * nb + 4, (i, r, ny, nz, nb)
                tot_c += cnt
                tot_b += ny * nz
        assert n_area > 100
        assert occ / 2.5 <= tot_c / tot_b <= occ
