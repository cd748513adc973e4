"""Pins of the refit oracle (a8) and its adjoint (a9).

P13 noise-free hits on the true distorted planes give chi2 ~ 0, smeared hits
chi2/ndf ~ 1; P14 the binary64 adjoint against central finite differences
(h = 1e-3 cm); P15 against complex-step derivatives of the same forward code
(a derivative independent of the hand-written reverse pass); P16 the map
gradient points from D = 0 towards the true distortion and nearly vanishes
at the truth.
"""
import numpy as np
import pytest

import oracle
import synth

G = synth.geometry()
P = dict(oracle.DEFAULT_PARAMS)


def _ev(n=60, smear=True, seed=0):
    return synth.config5(n_found=n, smear=smear, rep=seed)


def _args(ev):
    return ev.extra["hit_off"], ev.extra["hit_clu"], ev.extra["seed_par"], ev.extra["D_true"]


def test_refit_noise_free_true_map_chi2_vanishes():
    ev = _ev(40, smear=False)
    ho, hc, seed, D = _args(ev)
    chi2, st, _ = oracle.refit(G, P, ev, ho, hc, seed, D, prec=64)
    assert np.all(st == 0)
    # hits are rounded to binary32 (~1e-5 cm): chi2 per hit stays ~1e-8
    assert chi2.sum() < 1e-6 * ev.n
    chi2_0, _, _ = oracle.refit(G, P, ev, ho, hc, seed, np.zeros_like(D), prec=64)
    assert chi2_0.sum() > 100 * chi2.sum() + 1.0


def test_refit_smeared_chi2_per_ndf():
    ev = _ev(400)
    ho, hc, seed, D = _args(ev)
    chi2, st, ckpt = oracle.refit(G, P, ev, ho, hc, seed, D, prec=64)
    ok = st == 0
    assert ok.mean() > 0.99
    n = np.diff(ho)[ok]
    ndf = (2 * n - 5).sum()
    assert abs(chi2[ok].sum() / ndf - 1) < 0.05
    # checkpoint of the last hit = the final filtered state; first = the seed
    assert np.allclose(ckpt[ho[:-1][ok], 2:5], seed[ok, 2:5].astype(np.float64))


def test_refit_binary32_close_to_binary64():
    ev = _ev(100)
    ho, hc, seed, D = _args(ev)
    c32, s32, _ = oracle.refit(G, P, ev, ho, hc, seed, D, prec=32)
    c64, s64, _ = oracle.refit(G, P, ev, ho, hc, seed, D, prec=64)
    ok = (s32 == 0) & (s64 == 0)
    assert np.all(np.abs(c32[ok] - c64[ok]) <= 1e-3 * np.maximum(c64[ok], 1.0))


@pytest.fixture(scope="module")
def grad_case():
    ev = _ev(60)
    ho, hc, seed, D = _args(ev)
    rng = np.random.default_rng(3)
    w = rng.uniform(0.5, 1.5, len(ho) - 1)
    r = oracle.refit_grad(G, P, ev, ho, hc, seed, D, w)
    return ev, (ho, hc, seed, D), w, r, rng


def _cells(ev):
    return np.unique(ev.row.astype(np.int64) * 18 + ev.sector % 18)


def test_adjoint_matches_complex_step(grad_case):
    ev, (ho, hc, seed, D), w, (chi2, st, gmap, gx, gy, gz), rng = grad_case
    worst = 0.0
    for which, arr, idx in (("x", gx, rng.choice(ev.n, 40, replace=False)),
                            ("y", gy, rng.choice(ev.n, 40, replace=False)),
                            ("z", gz, rng.choice(ev.n, 40, replace=False)),
                            ("map", gmap.reshape(-1), rng.choice(_cells(ev), 25, replace=False))):
        for i in idx:
            cs = oracle.refit_loss(G, P, ev, ho, hc, seed, D, w, which, int(i), 1e-30, mode="c128")
            worst = max(worst, abs(arr[i] - cs) / max(abs(cs), 1e-9))
    assert worst < 1e-9, worst


def test_adjoint_matches_central_differences(grad_case):
    ev, (ho, hc, seed, D), w, (chi2, st, gmap, gx, gy, gz), rng = grad_case
    h = 1e-3
    errs = []
    for which, arr, idx in (("x", gx, rng.choice(ev.n, 60, replace=False)),
                            ("y", gy, rng.choice(ev.n, 60, replace=False)),
                            ("z", gz, rng.choice(ev.n, 60, replace=False)),
                            ("map", gmap.reshape(-1), rng.choice(_cells(ev), 20, replace=False))):
        for i in idx:
            fp = oracle.refit_loss(G, P, ev, ho, hc, seed, D, w, which, int(i), h)
            fm = oracle.refit_loss(G, P, ev, ho, hc, seed, D, w, which, int(i), -h)
            fd = (fp - fm) / (2 * h)
            errs.append(abs(arr[i] - fd) / max(abs(fd), 1e-2))
    # the O(h^2) truncation of the difference itself reaches ~3e-5 at h = 1e-3 cm
    assert max(errs) < 1e-4, max(errs)


def test_adjoint_of_failed_track_is_zero():
    ev = _ev(30, smear=False)
    ho, hc, seed, D = _args(ev)
    seed = seed.copy()
    seed[0, 2] = 0.98          # first track starts next to |snp| = 0.99: fails
    seed[0, 4] = -20.0
    chi2, st, gmap, gx, gy, gz = oracle.refit_grad(G, P, ev, ho, hc, seed, D)
    assert st[0] == 1 and chi2[0] == 0
    c = hc[ho[0]:ho[1]]
    assert np.all(gx[c] == 0) and np.all(gy[c] == 0) and np.all(gz[c] == 0)


@pytest.mark.parametrize("smear", [False, True])
def test_map_gradient_quadratic_relation_and_zero_at_truth(smear):
    """chi2 is close to quadratic in the map: with g0 the gradient at D = 0,
    <g0, D_true> = -2 (chi2(0) - chi2(D_true)); for noise-free hits the
    gradient vanishes at the true map."""
    ev = _ev(400, smear=smear)
    ho, hc, seed, D = _args(ev)
    c0, s0, g0, *_ = oracle.refit_grad(G, P, ev, ho, hc, seed, np.zeros_like(D))
    ct, st, gt, *_ = oracle.refit_grad(G, P, ev, ho, hc, seed, D)
    assert np.all(s0 == 0) and np.all(st == 0)
    lhs = float((g0 * D.astype(np.float64)).sum())
    rhs = -2.0 * (c0.sum() - ct.sum())
    assert abs(lhs / rhs - 1) < 0.03, (lhs, rhs)
    if not smear:
        assert np.linalg.norm(gt) < 1e-3 * np.linalg.norm(g0)


def test_refit_rejects_tracks_with_invalid_hits():
    """A hit naming no cluster, or a cluster on a row beyond the map, has no
    measurement plane: its track is rejected as a whole (status 2, chi2 0,
    zero gradient) and the other tracks are untouched."""
    ev = _ev(12)
    ho, hc, seed, D = _args(ev)
    ref_chi2, ref_st, _ = oracle.refit(G, P, ev, ho, hc, seed, D, prec=64)
    hc = hc.copy()
    row = ev.row.copy()
    hc[ho[3] + 2] = ev.n            # index past the last cluster
    hc[ho[5]] = -1                  # negative index
    row[hc[ho[7] + 4]] = 152        # row beyond the map
    import copy
    ev2 = copy.copy(ev)
    ev2.row = row
    for prec in (32, 64):
        chi2, st, _ = oracle.refit(G, P, ev2, ho, hc, seed, D, prec=prec)
        bad = [3, 5, 7]
        assert np.all(st[bad] == 2) and np.all(chi2[bad] == 0)
        good = np.setdiff1d(np.arange(len(st)), bad)
        if prec == 64:
            assert np.array_equal(chi2[good], ref_chi2[good]) and np.array_equal(st[good], ref_st[good])
    _, st, gm, gx, gy, gz = oracle.refit_grad(G, P, ev2, ho, hc, seed, D)
    for t in (3, 5, 7):
        cl = hc[ho[t]:ho[t + 1]]
        cl = cl[(cl >= 0) & (cl < ev.n)]
        assert np.all(gx[cl] == 0) and np.all(gy[cl] == 0) and np.all(gz[cl] == 0)
    loss = oracle.refit_loss(G, P, ev2, ho, hc, seed, D, np.ones(len(st)))
    assert loss == pytest.approx(ref_chi2[st == 0].sum(), rel=1e-12)


# ---------------------------------------------------------------- field map and material (f2)

@pytest.fixture(scope="module")
def material_case():
    bz = synth.field_map(amp=0.1)
    ix0, el = synth.material_map(scale=20.0)
    ev = synth.material_tracks(60, bz=bz, ix0=ix0, eloss=el, rep=3)
    mat = dict(bz=bz, ix0=ix0, eloss=el)
    ho, hc, seed = ev.extra["hit_off"], ev.extra["hit_clu"], ev.extra["seed_par"]
    D = (np.random.default_rng(8).uniform(-0.3, 0.3, (152, 18))).astype(np.float32)
    w = np.random.default_rng(9).uniform(0.5, 1.5, len(ho) - 1)
    res = oracle.refit_grad(G, P, ev, ho, hc, seed, D, w, mat=mat)
    return ev, (ho, hc, seed, D), w, mat, res


def test_material_adjoint_matches_complex_step_and_differences(material_case):
    """P26: with the field map, multiple scattering and energy loss, the
    binary64 adjoint equals complex-step derivatives of the same forward
    code (independent of the reverse pass) and central differences."""
    ev, (ho, hc, seed, D), w, mat, (chi2, st, gmap, gx, gy, gz) = material_case
    assert np.all(st == 0)
    rng = np.random.default_rng(10)
    worst_cs, worst_fd = 0.0, 0.0
    cells = np.unique(ev.row.astype(np.int64) * 18)
    for which, arr, idx in (("x", gx, rng.choice(ev.n, 25, replace=False)),
                            ("y", gy, rng.choice(ev.n, 25, replace=False)),
                            ("z", gz, rng.choice(ev.n, 25, replace=False)),
                            ("map", gmap.reshape(-1), rng.choice(cells, 15, replace=False))):
        for i in idx:
            cs = oracle.refit_loss(G, P, ev, ho, hc, seed, D, w, which, int(i), 1e-30,
                                   mode="c128", mat=mat)
            worst_cs = max(worst_cs, abs(arr[i] - cs) / max(abs(cs), 1e-9))
            fp = oracle.refit_loss(G, P, ev, ho, hc, seed, D, w, which, int(i), 1e-3, mat=mat)
            fm = oracle.refit_loss(G, P, ev, ho, hc, seed, D, w, which, int(i), -1e-3, mat=mat)
            fd = (fp - fm) / 2e-3
            worst_fd = max(worst_fd, abs(arr[i] - fd) / max(abs(fd), 1e-2))
    assert worst_cs < 1e-9, worst_cs
    assert worst_fd < 1e-4, worst_fd


def _chi2_ndf(ev, mat, prec=64):
    ho, hc, seed = ev.extra["hit_off"], ev.extra["hit_clu"], ev.extra["seed_par"]
    c, s, _ = oracle.refit(G, P, ev, ho, hc, seed, np.zeros((152, 18), np.float32), prec=prec,
                           mat=mat)
    ok = s == 0
    assert ok.mean() > 0.99
    return c[ok].sum() / (2 * np.diff(ho)[ok] - 5).sum()


def test_field_map_and_material_make_the_fit_consistent():
    """P27: tracks simulated through a field varying by 10 % (no material)
    fit with chi2/ndf ~ 1 under the map and clearly above 1 under the
    uniform field; tracks simulated through twenty times the gas material
    fit with chi2/ndf ~ 1 with the multiple-scattering and energy-loss
    model and far above 1 without it."""
    bz = synth.field_map(amp=0.1)
    ev = synth.material_tracks(400, bz=bz, with_material=False, pt_range=(0.15, 1.0))
    assert _chi2_ndf(ev, dict(bz=bz)) == pytest.approx(1.0, abs=0.02)
    assert _chi2_ndf(ev, None) > 1.08
    ix0, el = synth.material_map(scale=20.0)
    ev = synth.material_tracks(400, bz=bz, ix0=ix0, eloss=el, rep=1)
    assert _chi2_ndf(ev, dict(bz=bz, ix0=ix0, eloss=el)) == pytest.approx(1.0, abs=0.03)
    assert _chi2_ndf(ev, dict(bz=bz)) > 1.4
    # energy loss: q/pt at the last hit is unbiased with it and biased
    # towards the track's mean without it (the free q/pt absorbs part of the
    # loss, so the chi2 barely shows it); tracks with energy loss only, since
    # scattering adds a bias of its own to a ratio estimate
    ev = synth.material_tracks(1000, bz=bz, ix0=np.zeros(152, np.float32), eloss=el, rep=1)
    ho, hc, seed = ev.extra["hit_off"], ev.extra["hit_clu"], ev.extra["seed_par"]
    truth = ev.extra["qpt_last"]
    bias = {}
    for name, m in (("with", dict(bz=bz, eloss=el)), ("without", dict(bz=bz))):
        _, st, ck = oracle.refit(G, P, ev, ho, hc, seed, np.zeros((152, 18), np.float32),
                                 prec=64, mat=m)
        fit = ck[ho[1:] - 1, 4]
        ok = st == 0
        bias[name] = np.mean((fit[ok] - truth[ok]) / truth[ok])
    assert abs(bias["with"]) < 0.003 and bias["without"] < -0.008, bias


def test_neutral_maps_change_nothing():
    """P28: a field map holding the geometry's field everywhere and zero
    material reproduce the plain refit bit for bit (binary32)."""
    ev = synth.material_tracks(80, rep=4)
    ho, hc, seed = ev.extra["hit_off"], ev.extra["hit_clu"], ev.extra["seed_par"]
    D = np.zeros((152, 18), np.float32)
    base = oracle.refit(G, P, ev, ho, hc, seed, D)
    flat = dict(bz=np.full((152, 7), np.float32(G["bz"])), ix0=np.zeros(152, np.float32),
                eloss=np.zeros(152, np.float32))
    got = oracle.refit(G, P, ev, ho, hc, seed, D, mat=flat)
    for a, b in zip(base, got):
        assert np.array_equal(a, b)
