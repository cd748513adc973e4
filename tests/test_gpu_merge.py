"""GPU parity of sector-track merging and the global refit (f1) through the
C ABI: on the deterministic tracker's output for 36-sector events, the
kept links, the chains, the merged hit lists and the refitted parameters,
covariances, chi2, ndf, status and frames equal the binary32 oracle bit for
bit; the production build keeps a valid partition of the segments."""
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2511_17018_amd as tpc
import synth
from tests import parity

pytestmark = pytest.mark.gpu

G = synth.geometry()


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _check_hit_data(run, ev):
    # the tracker's optional per-hit output: the row plane, the cluster's y
    # and z, and the instance's phi sector of every hit, bit for bit
    nh = int(run.result["n_hits"])
    hc = run.tracks.hit_clu[:nh].cpu().numpy()
    hd = run.tracks.hit_data[:nh].cpu().numpy()
    inst = np.searchsorted(ev.inst_off, hc, side="right") - 1
    want = np.stack([G["row_x"][ev.row[hc]], ev.y[hc], ev.z[hc], (inst % 18).astype(np.float32)], 1)
    assert np.array_equal(parity.bits(hd), parity.bits(want.astype(np.float32)))


def _run(ev, det=True, hit_data=True):
    batch = tpc.upload(ev.x, ev.y, ev.z, ev.row, ev.charge, ev.inst_off, "cuda")
    run = tpc.track(G, batch, det=det, hit_data=hit_data)
    if hit_data:
        _check_hit_data(run, ev)
    m = tpc.merge_tracks(G, batch, run.tracks, run.ws.result, det=det)
    torch.cuda.synchronize()
    return run, m.host()


def _oracle_segments(run, ev):
    g = parity.gpu_arrays(run, ev.n)

    class S:
        par, cov, x_ref = g["param"], g["cov"], g["x_ref"]
        hit_off, hit_clu = g["hit_off"], g["hit_clu"]
    return S


def _compare(h, m):
    nc = len(m.chi2)
    assert h["n"] == nc
    assert np.array_equal(h["next"][:len(m.next)], m.next)
    assert np.array_equal(h["seg_off"], m.chain_off) and np.array_equal(h["seg"], m.chain_seg)
    assert np.array_equal(h["hit_off"], m.hit_off) and np.array_equal(h["hit_clu"], m.hit_clu)
    assert np.array_equal(h["status"], m.status) and np.array_equal(h["ndf"], m.ndf)
    assert np.array_equal(h["sector"], m.k)
    for name, a, b in (("param", h["param"], m.par), ("cov", h["cov"], m.cov),
                       ("chi2", h["chi2"], m.chi2), ("x_ref", h["x_ref"], m.x_ref)):
        assert np.array_equal(parity.bits(a), parity.bits(b)), name


@pytest.mark.parametrize("n_tracks,hit_data", [(300, True), (2500, True), (8000, True),
                                               (8000, False)])
def test_merge_bit_exact(n_tracks, hit_data):
    # hit_data: the segments' hits read from the tracker's per-hit output
    # (contiguous) or through the cluster arrays; the result is the same
    ev = synth.config2(n_tracks=n_tracks)
    _say(f"[merge] config2 tracks={n_tracks} clusters={ev.n} hit_data={hit_data}")
    run, h = _run(ev, hit_data=hit_data)
    S = _oracle_segments(run, ev)
    m = oracle.merge(G, ev.inst_off, ev.y, ev.z, ev.row, S)
    _say(f"[merge] segments={len(S.hit_off) - 1} merged={len(m.chi2)} "
         f"links={(m.next >= 0).sum()}")
    _compare(h, m)


def test_merge_bit_exact_pileup():
    """Collisions overlapping in drift time (the time-frame workload at a
    tenth of its collisions): many segments share each sector edge's z and
    distance window, so the bucketed pair search and its pre-transport
    bound reject most candidates -- the result still equals the oracle's
    search over all pairs."""
    ev = synth.config3(n_coll=12)
    _say(f"[merge] pile-up collisions=12 clusters={ev.n}")
    run, h = _run(ev)
    S = _oracle_segments(run, ev)
    m = oracle.merge(G, ev.inst_off, ev.y, ev.z, ev.row, S)
    _say(f"[merge] segments={len(S.hit_off) - 1} merged={len(m.chi2)} "
         f"links={(m.next >= 0).sum()}")
    _compare(h, m)


def test_merge_run_to_run_identical():
    """The pair-search buckets are filled in atomic order, which varies from
    run to run; the deterministic output does not (ten runs)."""
    ev = synth.config3(n_coll=4)
    batch = tpc.upload(ev.x, ev.y, ev.z, ev.row, ev.charge, ev.inst_off, "cuda")
    run = tpc.track(G, batch, det=True)
    n_seg = int(run.result["n_tracks"])
    first = None
    for _ in range(10):
        h = tpc.merge_tracks(G, batch, run.tracks, run.ws.result, det=True).host()
        torch.cuda.synchronize()
        h["next"] = h["next"][:n_seg]
        if first is None:
            first = h
            continue
        for k in ("next", "seg_off", "seg", "hit_off", "hit_clu", "status", "sector"):
            assert np.array_equal(h[k], first[k]), k
        for k in ("param", "cov", "chi2", "x_ref"):
            assert np.array_equal(parity.bits(h[k]), parity.bits(first[k])), k


def test_merge_crossing_the_membrane_and_empty_input():
    # noise-free tracks of shallow dip cross z = 0 (segments on both sides)
    ev = synth.config2(n_tracks=1500, noise=0.0)
    run, h = _run(ev)
    S = _oracle_segments(run, ev)
    m = oracle.merge(G, ev.inst_off, ev.y, ev.z, ev.row, S)
    _compare(h, m)
    # no tracks at all (five scattered clusters per sector): nothing merged
    rng = np.random.default_rng(3)
    n = 36 * 5
    row = rng.integers(0, 152, n).astype(np.uint16)
    x = G["row_x"][row]
    y = (rng.uniform(-0.1, 0.1, n) * x).astype(np.float32)
    z = rng.uniform(-200, 200, n).astype(np.float32)
    off = np.arange(37, dtype=np.int64) * 5
    batch = tpc.upload(x, y, z, row, np.zeros(n, np.uint16), off, "cuda")
    run = tpc.track(G, batch, det=True)
    assert int(run.result["n_tracks"]) == 0
    h = tpc.merge_tracks(G, batch, run.tracks, run.ws.result).host()
    assert h["n"] == 0 and h["hit_off"][0] == 0


def test_merge_prod_partition_valid():
    ev = synth.config2()
    run, h = _run(ev, det=False)
    n_seg = int(run.result["n_tracks"])
    seg = h["seg"]
    assert np.array_equal(np.sort(seg), np.arange(n_seg))
    ho = run.tracks.hit_off[:n_seg + 1].cpu().numpy()
    hc = run.tracks.hit_clu[:int(ho[-1])].cpu().numpy()
    for c in range(h["n"]):
        segs = seg[h["seg_off"][c]:h["seg_off"][c + 1]]
        want = np.concatenate([hc[ho[s]:ho[s + 1]] for s in segs])
        assert np.array_equal(h["hit_clu"][h["hit_off"][c]:h["hit_off"][c + 1]], want)
    ok = h["status"] == 0
    assert ok.mean() > 0.95
    assert np.median(h["chi2"][ok] / h["ndf"][ok]) == pytest.approx(1.0, abs=0.05)
