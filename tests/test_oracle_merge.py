"""Pins of the merging and global-refit oracle (f1, readings R35-R41).

P21 the rotation of a state into the next sector's frame is exact on a
helix (closed form: the same point and direction seen from the rotated
axes, computed with trigonometric functions); up then down is the identity.
P22 the rotated covariance equals J C J^T with J the finite-difference
Jacobian of (rotate, then propagate to the nominal new plane).
P23 the LDL^T chi2 equals d^T S^-1 d from a library solve; in binary32 it
does not fall below the single-component bound d_i^2 / S_ii that the pair
search uses to skip transports (by more than 1e-3, on strongly correlated
covariances).
P24 noise-free helices crossing sector edges: every segment link joins
segments of one particle, and the merged refit stays on the helix (chi2
~ 0, parameters at the first hit equal the truth).
P25 smeared events: links are pure and find most crossings; the merged
refit has chi2/ndf ~ 1 and unit-width q/pt pulls; every segment is in
exactly one output track, chains follow the mutual links.
"""
import numpy as np
import pytest

import oracle
import synth
from tests import helix

G = synth.geometry()
P = dict(oracle.DEFAULT_PARAMS)
D20 = np.radians(20.0)


def _cov(rng):
    a = rng.normal(0, 1, (5, 5)) * np.array([0.1, 0.15, 0.01, 0.01, 0.05])[:, None]
    C = a @ a.T + np.diag([0.01, 0.02, 1e-4, 1e-4, 1e-3])
    return C[np.tril_indices(5)] if False else np.array([C[i, j] for i in range(5) for j in range(i + 1)])


def _full(c15):
    C = np.zeros((5, 5))
    k = 0
    for i in range(5):
        for j in range(i + 1):
            C[i, j] = C[j, i] = c15[k]
            k += 1
    return C


@pytest.mark.parametrize("up", [True, False])
def test_rotation_exact_on_a_helix(up):
    rng = np.random.default_rng(1)
    for _ in range(50):
        x = rng.uniform(90, 240)
        st = np.array([rng.uniform(-0.15, 0.15) * x, rng.uniform(-200, 200), rng.uniform(-0.6, 0.6),
                       rng.uniform(-1, 1), rng.uniform(-3, 3)])
        c15 = _cov(rng)
        ok, p, c, xn = oracle.rotate(G, st, c15, x, up)
        assert ok
        # the sector angle's cosine and sine are binary32 constants (relative
        # error ~3e-8): positions agree to ~1e-5 cm, directions to ~1e-7
        d = D20 if up else -D20
        phi = np.arcsin(st[2])
        assert xn == pytest.approx(x * np.cos(d) + st[0] * np.sin(d), abs=1e-5)
        assert p[0] == pytest.approx(-x * np.sin(d) + st[0] * np.cos(d), abs=1e-5)
        assert p[2] == pytest.approx(np.sin(phi - d), abs=1e-7)
        assert np.array_equal(p[[1, 3, 4]], st[[1, 3, 4]])
        # up then down: the identity, covariance included
        ok2, p2, c2, x2 = oracle.rotate(G, p, c, xn, not up)
        assert ok2 and x2 == pytest.approx(x, abs=1e-5)
        assert np.allclose(p2, st, atol=1e-5)
        assert np.allclose(c2, c15, rtol=1e-6, atol=1e-12)
    # a helix seen from the next sector: the exact crossing of the rotated
    # plane equals the rotated state moved along the helix to that plane
    st = np.array([10.0, 20.0, 0.3, 0.4, 1.5])
    x = 150.0
    ok, p, c, xn = oracle.rotate(G, st, _cov(rng), x, True)
    Xp = xn + 3.0
    ok, p3, _ = oracle.propagate(G, P, p, c, xn, Xp)
    # exact: the global circle through the point with the direction
    gx, gy = x, st[0]
    y3, z3, s3 = helix.at(np.array([p[0], p[1], p[2], p[3], p[4]]), xn, np.array([Xp]))
    assert p3[0] == pytest.approx(y3[0], abs=1e-7) and p3[2] == pytest.approx(s3[0], abs=1e-9)


def test_rotation_covariance_is_first_order_exact():
    rng = np.random.default_rng(2)
    for up in (True, False):
        for _ in range(20):
            x = rng.uniform(90, 240)
            st = np.array([rng.uniform(-0.15, 0.15) * x, rng.uniform(-100, 100),
                           rng.uniform(-0.5, 0.5), rng.uniform(-1, 1), rng.uniform(-4, 4)])
            c15 = _cov(rng)
            ok, p0, c1, X0 = oracle.rotate(G, st, c15, x, up)
            J = np.zeros((5, 5))
            for i in range(5):
                h = 1e-6 * max(1.0, abs(st[i]))
                cols = []
                for sgn in (1, -1):
                    s = st.copy()
                    s[i] += sgn * h
                    ok, q, _, xq = oracle.rotate(G, s, c15, x, up)
                    ok2, q2, _ = oracle.propagate(G, P, q, c15, xq, X0)
                    assert ok and ok2
                    cols.append(q2)
                J[:, i] = (cols[0] - cols[1]) / (2 * h)
            want = J @ _full(c15) @ J.T
            assert np.allclose(_full(c1), want, rtol=1e-6, atol=1e-9)


def test_ldl_chi2_equals_library_solve():
    rng = np.random.default_rng(3)
    for _ in range(200):
        c15 = _cov(rng)
        d = rng.normal(0, 1, 5) * np.array([0.1, 0.2, 0.01, 0.01, 0.03])
        want = d @ np.linalg.solve(_full(c15), d)
        assert oracle.chi2_5(c15, d) == pytest.approx(want, rel=1e-10)
    S = _full(_cov(rng))
    S[0, 0] = -1.0
    assert oracle.chi2_5(np.array([S[i, j] for i in range(5) for j in range(i + 1)]),
                         np.ones(5)) < 0


@pytest.mark.parametrize("floor", [1e-2, 1e-4, 1e-6])
def test_ldl_chi2_in_binary32_keeps_the_single_component_bound(floor):
    # The pair search skips the transport of a pair whose bound
    # max(d_3^2 / S_33, d_4^2 / S_44) exceeds 1.5 times the cut, which is
    # exact only if the binary32 LDL^T chi2 never falls below a third of
    # d^T S^-1 d >= d_i^2 / S_ii.  Covariances of track-like scales, strongly
    # correlated (the diagonal floor sets how nearly singular they are):
    # the binary32 chi2 stays within 1e-3 of the bound or above it.
    rng = np.random.default_rng(11)
    scale = np.array([0.1, 0.15, 0.01, 0.01, 0.05])
    worst = np.inf
    for _ in range(4000):
        a = rng.normal(0, 1, (5, 3)) * scale[:, None]
        C = a @ a.T + np.diag(floor * scale ** 2)
        c15 = np.array([C[i, j] for i in range(5) for j in range(i + 1)], np.float32)
        d = (rng.normal(0, 1, 5) * scale * rng.uniform(0.1, 30)).astype(np.float32)
        S = _full(c15.astype(np.float64))
        exact = d.astype(np.float64) @ np.linalg.solve(S, d.astype(np.float64))
        bound = max(float(np.float32(d[3] * d[3]) / c15[9]), float(np.float32(d[4] * d[4]) / c15[14]))
        assert exact >= bound * (1 - 1e-5)
        got = oracle.chi2_5(c15, d, prec=32)
        worst = min(worst, got / bound)
    assert worst >= 1 - 1e-3, worst


def _segments(ev, tracks):
    T = tracks
    return np.array([np.bincount(np.maximum(ev.label[T.hit_clu[T.hit_off[k]:T.hit_off[k + 1]]], 0)).argmax()
                     for k in range(len(T.chi2))])


def _possible_links(lab):
    u, c = np.unique(lab, return_counts=True)
    return int((c - 1).sum())


def test_noise_free_crossings_merge_and_stay_on_the_helix():
    ev = synth.config2(n_tracks=600, noise=0.0, smear=False)
    r = oracle.track(G, P, ev.inst_off, ev.y, ev.z, ev.row, prec=64)
    m = oracle.merge(G, ev.inst_off, ev.y, ev.z, ev.row, r.tracks, prec=64)
    lab = _segments(ev, r.tracks)
    nl = (m.next >= 0).sum()
    assert nl > 50
    assert all(lab[a] == lab[m.next[a]] for a in np.nonzero(m.next >= 0)[0])
    trk = ev.tracks
    multi = np.nonzero(np.diff(m.chain_off) > 1)[0]
    good = multi[m.status[multi] == 0]
    assert len(good) >= 0.9 * len(multi)
    for c in good:
        a, b = m.hit_off[c], m.hit_off[c + 1]
        assert m.chi2[c] / (2 * (b - a) - 5) < 1e-6
        h0 = m.hit_clu[a]
        t = lab[m.chain_seg[m.chain_off[c]]]
        qpt = trk["q"][t] / trk["pt"][t]
        assert m.par[c, 0] == pytest.approx(float(ev.y[h0]), abs=1e-4)
        assert m.par[c, 1] == pytest.approx(float(ev.z[h0]), abs=1e-4)
        assert m.par[c, 2] == pytest.approx(ev.extra["truth"][h0, 2], abs=1e-5)
        assert m.par[c, 3] == pytest.approx(trk["tanl"][t], abs=1e-5)
        assert m.par[c, 4] == pytest.approx(qpt, abs=1e-4 * max(1.0, abs(qpt)))


def test_smeared_event_links_pure_refit_calibrated_partition_complete():
    ev = synth.config2(n_tracks=2500)
    r = oracle.track(G, P, ev.inst_off, ev.y, ev.z, ev.row)
    T = r.tracks
    m = oracle.merge(G, ev.inst_off, ev.y, ev.z, ev.row, T)
    lab = _segments(ev, T)
    linked = np.nonzero(m.next >= 0)[0]
    assert np.mean(lab[linked] == lab[m.next[linked]]) >= 0.999
    assert len(linked) >= 0.85 * _possible_links(lab)
    # mutual best: a link is both ends' best choice, and only such pairs link
    for a in range(len(m.next)):
        b = m.succ[a]
        assert m.next[a] == (b if b >= 0 and m.pred[b] == a else -1)
    # every segment in exactly one chain, chains follow the links
    assert np.array_equal(np.sort(m.chain_seg), np.arange(len(T.chi2)))
    for c in range(len(m.chain_off) - 1):
        segs = m.chain_seg[m.chain_off[c]:m.chain_off[c + 1]]
        assert np.all(m.next[segs[:-1]] == segs[1:])
        assert m.next[segs[-1]] < 0 or m.next[segs[-1]] in segs
        hits = np.concatenate([T.hit_clu[T.hit_off[s]:T.hit_off[s + 1]] for s in segs])
        assert np.array_equal(m.hit_clu[m.hit_off[c]:m.hit_off[c + 1]], hits)
    ok = m.status == 0
    assert ok.mean() > 0.95
    # the binary32 refit keeps its covariances positive definite
    for c in np.nonzero(ok)[0]:
        assert np.all(np.linalg.eigvalsh(_full(m.cov[c].astype(np.float64))) > 0), c
    # chi2/ndf of the merged refit: the merged tracks (the sector tracker's
    # own output carries a few junk tracks of huge chi2 among the single
    # segments, so the median is taken there)
    multi = np.nonzero((np.diff(m.chain_off) > 1) & ok)[0]
    assert m.chi2[multi].sum() / m.ndf[multi].sum() == pytest.approx(1.0, abs=0.1)
    assert np.median(m.chi2[ok] / m.ndf[ok]) == pytest.approx(1.0, abs=0.05)
    # q/pt pulls of merged multi-segment tracks against the truth
    t = lab[m.chain_seg[m.chain_off[multi]]]
    qpt = ev.tracks["q"][t] / ev.tracks["pt"][t]
    pull = (m.par[multi, 4] - qpt) / np.sqrt(m.cov[multi, 14])
    assert len(multi) > 300
    assert abs(np.median(pull)) < 0.15 and 0.8 < np.std(np.clip(pull, -6, 6)) < 1.3
