"""GPU parity of the refit (a8) and its reverse pass (a9) through the C ABI.

Deterministic forward: chi2, status and checkpoints equal the binary32 oracle
bit for bit (R28).  Gradient: against the binary64 oracle adjoint (which the
CPU pins tie to complex-step derivatives) within R27: norm-wise relative
error <= 1e-3 and element-wise |g - g_ref| <= 1e-3 * max(|g_ref|,
1e-2 * rms(g_ref)); bit-identical from run to run.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2511_17018_amd as tpc
import synth

pytestmark = pytest.mark.gpu

G = synth.geometry()
P = dict(oracle.DEFAULT_PARAMS)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _gpu(ev, dmap, det=True):
    xyz = torch.from_numpy(np.stack([ev.x, ev.y, ev.z]).astype(np.float32)).cuda()
    row = torch.from_numpy(ev.row.view(np.int16)).cuda()
    trk = tpc.upload_refit_tracks(ev.extra["hit_off"], ev.extra["hit_clu"], ev.sector,
                                  ev.extra["seed_par"])
    m = torch.from_numpy(np.ascontiguousarray(dmap, np.float32)).cuda()
    return xyz, row, trk, m


def _args(ev):
    return ev.extra["hit_off"], ev.extra["hit_clu"], ev.extra["seed_par"]


def _hit_order(ckpt, hit_off):
    """The GPU checkpoints in hit order (the library stores them by group
    of 64 tracks and hit number, in parts of 16 bytes)."""
    return ckpt.cpu().numpy().reshape(-1)[tpc.checkpoint_index(hit_off)]


def _r27_elements(g, ref):
    g = np.asarray(g, np.float64).reshape(-1)
    ref = np.asarray(ref, np.float64).reshape(-1)
    rms = np.sqrt(np.mean(ref ** 2))
    return np.abs(g - ref) / np.maximum(np.abs(ref), 1e-2 * rms + 1e-30)


def _r27(g, ref):
    g = np.asarray(g, np.float64).reshape(-1)
    ref = np.asarray(ref, np.float64).reshape(-1)
    nrm = np.linalg.norm(g - ref) / max(np.linalg.norm(ref), 1e-30)
    rms = np.sqrt(np.mean(ref ** 2)) if len(ref) else 0.0
    el = np.abs(g - ref) / np.maximum(np.abs(ref), 1e-2 * rms + 1e-30)
    return nrm, float(el.max()) if len(el) else 0.0


@pytest.mark.parametrize("n_found,smear", [(300, True), (60, False)])
def test_refit_forward_bit_exact(n_found, smear):
    ev = synth.config5(n_found=n_found, smear=smear)
    _say(f"[refit fwd] tracks={n_found} hits={ev.n}")
    ho, hc, seed = _args(ev)
    for dmap in (ev.extra["D_true"], np.zeros_like(ev.extra["D_true"])):
        xyz, row, trk, m = _gpu(ev, dmap)
        chi2, status, ckpt = tpc.refit(G, xyz, row, trk, m, det=True)
        torch.cuda.synchronize()
        c_o, s_o, k_o = oracle.refit(G, P, ev, ho, hc, seed, dmap, prec=32)
        assert np.array_equal(status.cpu().numpy(), s_o)
        assert np.array_equal(chi2.cpu().numpy().view(np.int32), c_o.view(np.int32))
        ok = np.repeat(s_o == 0, np.diff(ho))
        assert np.array_equal(_hit_order(ckpt, ho)[ok].view(np.int32), k_o[ok].view(np.int32))


def test_refit_backward_matches_binary64_adjoint():
    ev = synth.config5(n_found=400)
    ho, hc, seed = _args(ev)
    rng = np.random.default_rng(4)
    w = rng.uniform(0.5, 1.5, len(ho) - 1)
    for dmap in (ev.extra["D_true"], np.zeros_like(ev.extra["D_true"])):
        xyz, row, trk, m = _gpu(ev, dmap)
        chi2, status, ckpt = tpc.refit(G, xyz, row, trk, m)
        gmap, gxyz = tpc.refit_backward(G, xyz, row, trk, m, ckpt, status,
                                        torch.from_numpy(w.astype(np.float32)).cuda())
        torch.cuda.synchronize()
        w32 = w.astype(np.float32).astype(np.float64)
        _, st, rmap, rx, ry, rz = oracle.refit_grad(G, P, ev, ho, hc, seed, dmap, w32)
        # the binary64 adjoint on the binary32 trajectory: the oracle's own
        # binary32 forward, which the GPU forward equals bit for bit
        c_o, s_o, k_o = oracle.refit(G, P, ev, ho, hc, seed, dmap, prec=32)
        ok = np.repeat(s_o == 0, np.diff(ho))
        assert np.array_equal(status.cpu().numpy(), s_o)
        assert np.array_equal(_hit_order(ckpt, ho)[ok].view(np.int32), k_o[ok].view(np.int32))
        _, _, _, sx, sy, sz = oracle.refit_grad(G, P, ev, ho, hc, seed, dmap, w32,
                                                ckpt=k_o, status=s_o)
        gx, gy, gz = gxyz.cpu().numpy()
        fails = []
        for name, a, b, bs in (("x", gx, rx, sx), ("y", gy, ry, sy), ("z", gz, rz, sz)):
            nrm, _ = _r27(a, b)
            _, el = _r27(a, bs)
            _say(f"[refit bwd] {name}: norm-wise vs binary64 {nrm:.2e}; element-wise vs "
                 f"binary64 adjoint of the binary32 trajectory {el:.2e}")
            if not (nrm <= 1e-3 and el <= 1e-6):
                fails.append(name)
        # a map cell is a sum over its hits: its rounding scale is the sum of
        # the magnitudes of the terms, not the (possibly cancelling) total
        cell = ev.row.astype(np.int64) * 18 + ev.sector % 18
        scale = np.bincount(cell, weights=np.abs(rx), minlength=152 * 18)
        a = gmap.cpu().numpy().reshape(-1).astype(np.float64)
        nrm, _ = _r27(a, rmap)
        el = float((np.abs(a - rmap.reshape(-1)) / np.maximum(scale, 1e-30))[scale > 0].max())
        _say(f"[refit bwd] map: norm-wise {nrm:.2e} element-wise (term scale) {el:.2e}")
        if not (nrm <= 1e-3 and el <= 1e-3):
            fails.append("map")
        assert not fails, fails


def test_refit_backward_deterministic_and_map_is_sum_of_x_gradients():
    ev = synth.config5(n_found=500)
    dmap = ev.extra["D_true"]
    xyz, row, trk, m = _gpu(ev, dmap)
    chi2, status, ckpt = tpc.refit(G, xyz, row, trk, m)
    ones = torch.ones_like(chi2)
    a = tpc.refit_backward(G, xyz, row, trk, m, ckpt, status, ones)
    b = tpc.refit_backward(G, xyz, row, trk, m, ckpt, status, ones)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    # every hit's dL/dX enters both its cluster's x gradient and its map cell
    cell = ev.row.astype(np.int64) * 18 + ev.sector % 18
    gx = a[1][0].cpu().numpy().astype(np.float64)
    want = np.bincount(cell, weights=gx, minlength=152 * 18)
    got = a[0].cpu().numpy().reshape(-1)
    assert np.allclose(got, want, rtol=1e-5, atol=1e-4 * np.abs(want).max())


def test_autograd_function_matches_direct_calls():
    ev = synth.config5(n_found=200)
    xyz, row, trk, m = _gpu(ev, ev.extra["D_true"] * 0.5)
    xyz.requires_grad_(True)
    m.requires_grad_(True)
    chi2 = tpc.TpcRefit.apply(xyz, m, row, trk, G)
    (chi2 * 2.0).sum().backward()
    c2, st, ck = tpc.refit(G, xyz.detach(), row, trk, m.detach())
    gm, gxyz = tpc.refit_backward(G, xyz.detach(), row, trk, m.detach(), ck, st,
                                  torch.full_like(c2, 2.0))
    torch.cuda.synchronize()
    assert torch.equal(chi2.detach(), c2)
    assert torch.equal(xyz.grad, gxyz) and torch.equal(m.grad, gm)


def test_refit_prod_close_to_binary64():
    ev = synth.config5(n_found=300)
    ho, hc, seed = _args(ev)
    dmap = ev.extra["D_true"]
    xyz, row, trk, m = _gpu(ev, dmap)
    chi2, status, _ = tpc.refit(G, xyz, row, trk, m, det=False)
    c64, s64, _ = oracle.refit(G, P, ev, ho, hc, seed, dmap, prec=64)
    c = chi2.cpu().numpy()
    ok = (status.cpu().numpy() == 0) & (s64 == 0)
    assert np.all(np.abs(c[ok] - c64[ok]) <= 1e-3 * np.maximum(c64[ok], 1.0))


def test_refit_rejects_tracks_with_invalid_hits_like_the_oracle():
    """Hits past the last cluster, negative, or on a row beyond the map:
    status 2 (also when a propagation failure comes first), chi2 0, no
    gradient, and every other track bit-exact with the oracle."""
    ev = synth.config5(n_found=300)
    ho, hc, seed = _args(ev)
    hc = hc.copy()
    row = ev.row.copy()
    hc[ho[3] + 2] = ev.n
    hc[ho[5]] = -7
    row[hc[ho[7] + 4]] = 152
    hc[ho[11 + 1] - 1] = ev.n + 100           # last hit of track 11
    seed = seed.copy()
    seed[11, 2], seed[11, 4] = 0.9895, -5.0   # its first propagation fails too
    import copy
    ev2 = copy.copy(ev)
    ev2.row = row
    ev2.extra = dict(ev.extra, hit_clu=hc, seed_par=seed)
    dmap = ev.extra["D_true"]
    _say(f"[refit invalid hits] tracks={len(ho) - 1}")
    c_o, s_o, k_o = oracle.refit(G, P, ev2, ho, hc, seed, dmap, prec=32)
    assert np.all(s_o[[3, 5, 7, 11]] == 2)
    xyz, rw, trk, m = _gpu(ev2, dmap)
    chi2, status, ckpt = tpc.refit(G, xyz, rw, trk, m, det=True)
    gmap, gxyz = tpc.refit_backward(G, xyz, rw, trk, m, ckpt, status, torch.ones_like(chi2))
    torch.cuda.synchronize()
    assert np.array_equal(status.cpu().numpy(), s_o)
    assert np.array_equal(chi2.cpu().numpy().view(np.int32), c_o.view(np.int32))
    ok = np.repeat(s_o == 0, np.diff(ho))
    assert np.array_equal(_hit_order(ckpt, ho)[ok].view(np.int32), k_o[ok].view(np.int32))
    g = gxyz.cpu().numpy()
    for t in (3, 5, 7, 11):
        cl = hc[ho[t]:ho[t + 1]]
        cl = cl[(cl >= 0) & (cl < ev.n)]
        assert np.all(g[:, cl] == 0)
    assert np.isfinite(gmap.cpu().numpy()).all()


def test_refit_gradient_matches_finite_differences_and_complex_step():
    """The target stated for the refit: gradients within 1e-3 relative error
    of finite differences.  On sampled cluster coordinates and map cells the
    GPU gradient is compared with binary64 central differences (h = 1e-3 cm)
    and with complex-step derivatives of the binary64 forward (exact to
    rounding), none of which uses the adjoint code: norm-wise over the
    sample <= 1e-3; element-wise |g - ref| <= 1e-3 * max(|ref|, rms), i.e.
    relative to the element or, for elements below the gradient's rms, to
    that scale: the binary32 trajectory leaves an absolute spread of about
    2e-4 rms (measured on the CPU), which is a large relative error only on
    elements near zero."""
    ev = synth.config5(n_found=400)
    ho, hc, seed = _args(ev)
    dmap = ev.extra["D_true"] * 0.5
    rng = np.random.default_rng(11)
    w = rng.uniform(0.5, 1.5, len(ho) - 1).astype(np.float32)
    w64 = w.astype(np.float64)
    xyz, row, trk, m = _gpu(ev, dmap)
    chi2, status, ckpt = tpc.refit(G, xyz, row, trk, m)
    gmap, gxyz = tpc.refit_backward(G, xyz, row, trk, m, ckpt, status, torch.from_numpy(w).cuda())
    torch.cuda.synchronize()
    gxyz = gxyz.cpu().numpy().astype(np.float64)
    gmap = gmap.cpu().numpy().reshape(-1).astype(np.float64)
    on_track = np.zeros(ev.n, bool)
    on_track[hc] = True
    clus = rng.choice(np.nonzero(on_track)[0], 40, replace=False)
    cells_used = np.nonzero(np.bincount(ev.row.astype(np.int64)[hc] * 18 + ev.sector[hc] % 18,
                                        minlength=152 * 18))[0]
    cells = rng.choice(cells_used, 30, replace=False)

    def loss(which, i, h, mode):
        return oracle.refit_loss(G, P, ev, ho, hc, seed, dmap, w64, which=which, idx=int(i), h=h,
                                 mode=mode)

    fails = []
    for name, ax, idx in (("x", 0, clus), ("y", 1, clus), ("z", 2, clus), ("map", None, cells)):
        g = gmap[idx] if ax is None else gxyz[ax, idx]
        allg = gmap if ax is None else gxyz[ax]
        rms = np.sqrt(np.mean(allg[allg != 0] ** 2))
        cs = np.array([loss(name, i, 1e-30, "c128") for i in idx])
        fd = np.array([(loss(name, i, 1e-3, "f64") - loss(name, i, -1e-3, "f64")) / 2e-3
                       for i in idx])
        # the difference quotient's own truncation error (measured up to 3e-5)
        assert np.all(np.abs(fd - cs) <= 1e-4 * np.maximum(np.abs(cs), 1e-2 * rms)), name
        for rname, ref in (("fd", fd), ("cs", cs)):
            nrm = np.linalg.norm(g - ref) / np.linalg.norm(ref)
            el = float((np.abs(g - ref) / np.maximum(np.abs(ref), rms)).max())
            _say(f"[refit grad vs {rname}] {name}: norm-wise {nrm:.2e} element-wise {el:.2e}")
            if not (nrm <= 1e-3 and el <= 1e-3):
                fails.append((name, rname, nrm, el))
    assert not fails, fails


# ---------------------------------------------------------------- field map and material (f2)

def _material_case(n, rep, kind):
    """Tracks simulated through a 10 % field variation and twenty times the
    gas material; `kind` selects what the refit is given."""
    bz = synth.field_map(amp=0.1)
    ix0, el = synth.material_map(scale=20.0)
    ev = synth.material_tracks(n, bz=bz, ix0=ix0, eloss=el, rep=rep)
    mat = {"all": dict(bz=bz, ix0=ix0, eloss=el), "field": dict(bz=bz),
           "material": dict(ix0=ix0, eloss=el), "loss": dict(eloss=el),
           "scatter": dict(bz=bz, ix0=ix0)}[kind]
    D = np.random.default_rng(rep).uniform(-0.3, 0.3, (152, 18)).astype(np.float32)
    return ev, mat, D


@pytest.mark.parametrize("kind", ["all", "field", "material", "loss", "scatter"])
def test_material_refit_forward_bit_exact(kind):
    """f2 forward (R42-R44): with the field map and any part of the material,
    the deterministic GPU refit's chi2, status and checkpoints equal the
    binary32 oracle bit for bit."""
    ev, mat, D = _material_case(300, 5, kind)
    _say(f"[refit mat fwd] kind={kind} tracks=300 hits={ev.n}")
    ho, hc, seed = _args(ev)
    xyz, row, trk, m = _gpu(ev, D)
    gm = tpc.upload_material(**mat)
    chi2, status, ckpt = tpc.refit(G, xyz, row, trk, m, det=True, mat=gm)
    torch.cuda.synchronize()
    c_o, s_o, k_o = oracle.refit(G, P, ev, ho, hc, seed, D, prec=32, mat=mat)
    assert (s_o == 0).mean() > 0.95
    assert np.array_equal(status.cpu().numpy(), s_o)
    assert np.array_equal(chi2.cpu().numpy().view(np.int32), c_o.view(np.int32))
    ok = np.repeat(s_o == 0, np.diff(ho))
    assert np.array_equal(_hit_order(ckpt, ho)[ok].view(np.int32), k_o[ok].view(np.int32))
    # the production build stays close to the binary64 fit of the same model
    c_p, s_p, _ = tpc.refit(G, xyz, row, trk, m, det=False, mat=gm)
    c_64, s_64, _ = oracle.refit(G, P, ev, ho, hc, seed, D, prec=64, mat=mat)
    both = (s_p.cpu().numpy() == 0) & (s_64 == 0)
    rel = np.abs(c_p.cpu().numpy()[both] - c_64[both]) / np.maximum(c_64[both], 1.0)
    assert both.mean() > 0.95 and np.quantile(rel, 0.99) < 1e-3, np.quantile(rel, 0.99)


def test_material_refit_backward_matches_adjoint_and_derivatives():
    """f2 reverse pass: the GPU gradient of sum_t w_t chi2_t with the field
    map, scattering and energy loss equals the binary64 oracle adjoint on the
    same binary32 checkpoints (element-wise 1e-6, map cells against their
    terms' magnitude 1e-6), and matches complex-step derivatives and central
    differences (h = 1e-3 cm) of the binary64 forward on sampled coordinates
    and cells within 1e-3 (norm-wise; element-wise relative to max(|ref|,
    rms) as in the uniform-field test)."""
    ev, mat, D = _material_case(400, 6, "all")
    ho, hc, seed = _args(ev)
    _say(f"[refit mat bwd] tracks=400 hits={ev.n}")
    rng = np.random.default_rng(12)
    w = rng.uniform(0.5, 1.5, len(ho) - 1).astype(np.float32)
    w64 = w.astype(np.float64)
    xyz, row, trk, m = _gpu(ev, D)
    gm = tpc.upload_material(**mat)
    chi2, status, ckpt = tpc.refit(G, xyz, row, trk, m, mat=gm)
    gmap, gxyz = tpc.refit_backward(G, xyz, row, trk, m, ckpt, status,
                                    torch.from_numpy(w).cuda(), mat=gm)
    gmap2, gxyz2 = tpc.refit_backward(G, xyz, row, trk, m, ckpt, status,
                                      torch.from_numpy(w).cuda(), mat=gm)
    torch.cuda.synchronize()
    assert torch.equal(gmap, gmap2) and torch.equal(gxyz, gxyz2)
    c_o, s_o, k_o = oracle.refit(G, P, ev, ho, hc, seed, D, prec=32, mat=mat)
    assert np.array_equal(status.cpu().numpy(), s_o)
    _, _, smap, sx, sy, sz = oracle.refit_grad(G, P, ev, ho, hc, seed, D, w64, ckpt=k_o,
                                               status=s_o, mat=mat)
    g = gxyz.cpu().numpy().astype(np.float64)
    gmp = gmap.cpu().numpy().reshape(-1).astype(np.float64)
    fails = []
    for name, a, b in (("x", g[0], sx), ("y", g[1], sy), ("z", g[2], sz)):
        _, el = _r27(a, b)
        _say(f"[refit mat bwd] {name}: element-wise vs binary64 adjoint {el:.2e}")
        if not el <= 1e-6:
            fails.append(name)
    cell = ev.row.astype(np.int64) * 18 + ev.sector % 18
    scale = np.bincount(cell, weights=np.abs(sx), minlength=152 * 18)
    el = float((np.abs(gmp - smap.reshape(-1)) / np.maximum(scale, 1e-30))[scale > 0].max())
    _say(f"[refit mat bwd] map: element-wise (term scale) {el:.2e}")
    if not el <= 1e-6:
        fails.append("map")
    assert not fails, fails

    def loss(which, i, h, mode):
        return oracle.refit_loss(G, P, ev, ho, hc, seed, D, w64, which=which, idx=int(i), h=h,
                                 mode=mode, mat=mat)

    clus = rng.choice(ev.n, 30, replace=False)
    cells = rng.choice(np.nonzero(scale)[0], 20, replace=False)
    for name, ax, idx in (("x", 0, clus), ("y", 1, clus), ("z", 2, clus), ("map", None, cells)):
        gs = gmp[idx] if ax is None else g[ax, idx]
        allg = gmp if ax is None else g[ax]
        rms = np.sqrt(np.mean(allg[allg != 0] ** 2))
        cs = np.array([loss(name, i, 1e-30, "c128") for i in idx])
        fd = np.array([(loss(name, i, 1e-3, "f64") - loss(name, i, -1e-3, "f64")) / 2e-3
                       for i in idx])
        for rname, ref in (("fd", fd), ("cs", cs)):
            nrm = np.linalg.norm(gs - ref) / np.linalg.norm(ref)
            el = float((np.abs(gs - ref) / np.maximum(np.abs(ref), rms)).max())
            _say(f"[refit mat grad vs {rname}] {name}: norm-wise {nrm:.2e} element-wise {el:.2e}")
            if not (nrm <= 1e-3 and el <= 1e-3):
                fails.append((name, rname, nrm, el))
    assert not fails, fails


def test_material_neutral_maps_equal_plain_refit_on_gpu():
    """A field map holding the geometry's field everywhere with zero material
    gives the plain refit's outputs bit for bit (forward) and the same
    gradient (reverse pass)."""
    ev = synth.material_tracks(200, rep=7)
    ho, hc, seed = _args(ev)
    D = np.zeros((152, 18), np.float32)
    xyz, row, trk, m = _gpu(ev, D)
    flat = tpc.upload_material(bz=np.full((152, 9), np.float32(G["bz"])),
                               ix0=np.zeros(152, np.float32), eloss=np.zeros(152, np.float32))
    a = tpc.refit(G, xyz, row, trk, m)
    b = tpc.refit(G, xyz, row, trk, m, mat=flat)
    ones = torch.ones_like(a[0])
    ga = tpc.refit_backward(G, xyz, row, trk, m, a[2], a[1], ones)
    gb = tpc.refit_backward(G, xyz, row, trk, m, b[2], b[1], ones, mat=flat)
    torch.cuda.synchronize()
    for u, v in zip(a, b):
        assert torch.equal(u, v)
    # the same arithmetic in a differently scheduled kernel (fast math):
    # equal up to the last bits of the binary64 sums
    for u, v in zip(ga, gb):
        assert torch.allclose(u, v, rtol=1e-6, atol=1e-9 * float(u.abs().max()))


def test_refit_checkpoints_of_tracks_longer_than_the_layout_table():
    """Checkpoint layout beyond the per-wave table of 160 hit numbers: hit
    lists that run along a track, back and out again (up to 454 hits, the
    same clusters visited three times), in two groups of 64 tracks mixed with
    ordinary ones -- forward bit-exact with the binary32 oracle after
    decoding the layout, map gradient within R27 of the binary64 adjoint of
    those checkpoints (the map sums every hit; cluster gradients are not
    defined for a cluster hit more than once)."""
    ev = synth.config5(n_found=150, rep=3)
    ho0, hc0, seed = _args(ev)
    lists = []
    for t in range(len(ho0) - 1):
        h = hc0[ho0[t]:ho0[t + 1]]
        lists.append(np.concatenate([h, h[::-1][1:], h[1:]]) if t % 3 == 0 else h)
    ho = np.concatenate([[0], np.cumsum([len(x) for x in lists])]).astype(np.int32)
    hc = np.concatenate(lists).astype(np.int32)
    assert np.diff(ho).max() > 160
    ev2 = synth.Event(**{**ev.__dict__})
    ev2.extra = dict(ev.extra, hit_off=ho, hit_clu=hc)
    dmap = ev.extra["D_true"]
    _say(f"[refit long tracks] tracks={len(ho) - 1} longest={np.diff(ho).max()}")
    xyz, row, trk, m = _gpu(ev2, dmap)
    chi2, status, ckpt = tpc.refit(G, xyz, row, trk, m, det=True)
    w = torch.ones_like(chi2)
    gmap, _ = tpc.refit_backward(G, xyz, row, trk, m, ckpt, status, w)
    torch.cuda.synchronize()
    c_o, s_o, k_o = oracle.refit(G, P, ev2, ho, hc, seed, dmap, prec=32)
    long_ok = (np.diff(ho) > 160) & (s_o == 0)
    assert long_ok.sum() >= 10
    assert np.array_equal(status.cpu().numpy(), s_o)
    assert np.array_equal(chi2.cpu().numpy().view(np.int32), c_o.view(np.int32))
    ok = np.repeat(s_o == 0, np.diff(ho))
    assert np.array_equal(_hit_order(ckpt, ho)[ok].view(np.int32), k_o[ok].view(np.int32))
    _, _, smap, _, _, _ = oracle.refit_grad(G, P, ev2, ho, hc, seed, dmap, np.ones(len(ho) - 1),
                                            ckpt=k_o, status=s_o)
    nrm, _ = _r27(gmap.cpu().numpy(), smap)
    _say(f"[refit long tracks] map gradient norm-wise {nrm:.2e}")
    assert nrm <= 1e-6
