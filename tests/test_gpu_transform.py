"""GPU parity of the cluster coordinate transformation (f3) through the C
ABI: deterministic outputs equal the binary32 oracle bit for bit (with and
without each correction map, ragged and unaligned sizes, invalid raw
clusters, the empty input); the production build within a few binary32
roundings; the transformed clusters tracked by the GPU equal the oracle's
whole chain; and at the benchmark's size (15.65 M clusters, the launch
the benchmark times) sampled clusters equal the oracle's."""
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2511_17018_amd as tpc
import synth
from tests import parity

pytestmark = pytest.mark.gpu

TG = synth.transform_geometry()


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(raw):
    return (torch.from_numpy(raw["sector"]).cuda(), torch.from_numpy(raw["row"].view(np.int16)).cuda(),
            torch.from_numpy(raw["pad"]).cuda(), torch.from_numpy(raw["time"]).cuda())


def _maps(seed=3):
    rng = np.random.default_rng(seed)
    D = rng.uniform(-0.8, 0.8, (152, 18)).astype(np.float32)
    rm = synth.calibration_map(TG, synth.Distortion(amp=1.0, seed=seed))
    return D, rm


def _compare(raw, D, rm, sl=slice(None)):
    s, r, p, t = _dev(raw)
    s, r, p, t = s[sl], r[sl], p[sl], t[sl]
    Dd = torch.from_numpy(D).cuda() if D is not None else None
    rmd = torch.from_numpy(rm).cuda() if rm is not None else None
    x, y, z, ro = tpc.cluster_transform(TG, s, r, p, t, Dd, rmd, det=True)
    torch.cuda.synchronize()
    ox, oy, oz, oro = oracle.transform(TG, raw["sector"][sl], raw["row"][sl], raw["pad"][sl],
                                       raw["time"][sl], D, rm, prec=32)
    for name, g, o in (("x", x, ox), ("y", y, oy), ("z", z, oz)):
        assert np.array_equal(parity.bits(g.cpu().numpy()), parity.bits(o)), name
    assert np.array_equal(ro.cpu().numpy().view(np.uint16), oro)


@pytest.mark.parametrize("maps", ["none", "radial", "residual", "both"])
def test_transform_bit_exact(maps):
    ev = synth.config2(n_tracks=1500)
    raw = synth.encode_raw(ev, TG, dist=synth.Distortion(amp=1.0))
    D, rm = _maps()
    D = D if maps in ("radial", "both") else None
    rm = rm if maps in ("residual", "both") else None
    _say(f"[transform] n={ev.n} maps={maps}")
    _compare(raw, D, rm)
    # ragged length and a start that breaks the four-cluster alignment
    _compare(raw, D, rm, slice(1, ev.n - 2))
    _compare(raw, D, rm, slice(0, 7))


def test_transform_edge_cases():
    rng = np.random.default_rng(9)
    n = 4099
    raw = dict(sector=rng.integers(0, 40, n).astype(np.uint8),
               row=rng.integers(0, 160, n).astype(np.uint16),
               pad=rng.uniform(-20, 300, n).astype(np.float32),
               time=rng.uniform(-100, 1500, n).astype(np.float32))
    raw["pad"][::97] = np.nan
    raw["time"][5::89] = np.inf
    D, rm = _maps(5)
    _say(f"[transform edge] n={n}")
    _compare(raw, D, rm)
    # the empty input enqueues nothing and returns
    e = torch.empty(0, dtype=torch.float32, device="cuda")
    x, y, z, ro = tpc.cluster_transform(TG, e.to(torch.uint8), e.to(torch.int16), e, e)
    torch.cuda.synchronize()
    assert x.numel() == 0


def test_transform_prod_close_to_det():
    ev = synth.config2(n_tracks=1500)
    raw = synth.encode_raw(ev, TG, dist=synth.Distortion(amp=1.0))
    D, rm = _maps()
    s, r, p, t = _dev(raw)
    Dd, rmd = torch.from_numpy(D).cuda(), torch.from_numpy(rm).cuda()
    a = tpc.cluster_transform(TG, s, r, p, t, Dd, rmd, det=True)
    b = tpc.cluster_transform(TG, s, r, p, t, Dd, rmd, det=False)
    torch.cuda.synchronize()
    for u, v in zip(a[:3], b[:3]):
        u, v = u.cpu().numpy().astype(np.float64), v.cpu().numpy().astype(np.float64)
        # contraction and the fast division change a few roundings of values
        # up to 250 cm
        assert np.abs(u - v).max() <= 1e-4
    assert torch.equal(a[3], b[3])


def test_transformed_clusters_track_like_the_oracle():
    """f3 then a1-a6 on the GPU equals the oracle's transformation then its
    tracking chain, bit for bit."""
    ev = synth.config2(n_tracks=1200)
    raw = synth.encode_raw(ev, TG, dist=synth.Distortion(amp=1.0))
    D, rm = _maps()
    D[:] = 0.0
    s, r, p, t = _dev(raw)
    x, y, z, ro = tpc.cluster_transform(TG, s, r, p, t, torch.from_numpy(D).cuda(),
                                        torch.from_numpy(rm).cuda(), det=True)
    batch = tpc.upload_device(x, y, z, ro, ev.inst_off)
    run = tpc.track(parity.G, batch, det=True)
    g = parity.gpu_arrays(run, ev.n)
    ox, oy, oz, oro = oracle.transform(TG, raw["sector"], raw["row"], raw["pad"], raw["time"], D,
                                       rm, prec=32)
    o = oracle.track(parity.G, parity.P, ev.inst_off, oy, oz, oro)
    errs = parity.compare_det(g, o)
    assert not errs, errs
    _say(f"[transform+track] {len(g['param'])} tracks bit-exact")


def test_transform_full_size_sampled():
    """The benchmark's launch: 15.65 M clusters (config 4) with both maps;
    200 000 sampled clusters against the oracle, bit for bit."""
    ev = synth.config4()
    raw = synth.encode_raw(ev, TG, dist=synth.Distortion(amp=1.0))
    D, rm = _maps()
    _say(f"[transform full] n={ev.n}")
    s, r, p, t = _dev(raw)
    x, y, z, ro = tpc.cluster_transform(TG, s, r, p, t, torch.from_numpy(D).cuda(),
                                        torch.from_numpy(rm).cuda(), det=True)
    torch.cuda.synchronize()
    idx = np.sort(np.random.default_rng(1).choice(ev.n, 200_000, replace=False))
    ox, oy, oz, oro = oracle.transform(TG, raw["sector"][idx], raw["row"][idx], raw["pad"][idx],
                                       raw["time"][idx], D, rm, prec=32)
    ii = torch.from_numpy(idx).cuda()
    for name, g, o in (("x", x, ox), ("y", y, oy), ("z", z, oz)):
        assert np.array_equal(parity.bits(g[ii].cpu().numpy()), parity.bits(o)), name
    assert np.array_equal(ro[ii].cpu().numpy().view(np.uint16), oro)
