"""Batching (a10): graph-captured chains replay the eager result bit for bit
(with eager work between replays), per-instance chains in one graph equal
the batched chain, and autotuner candidates leave the output unchanged."""
import numpy as np
import pytest
import torch

import paper_2511_17018_amd as tpc
import synth
from paper_2511_17018_amd import autotune
from paper_2511_17018_amd.runtime import Chain, GraphChain, plain_chains, same_outputs

pytestmark = pytest.mark.gpu
G = synth.geometry()


def _batch(n_inst=12):
    ev = synth.config4(n_inst=n_inst, n_min=500, n_max=3e4)
    return ev, tpc.upload(ev.x, ev.y, ev.z, ev.row, ev.charge, ev.inst_off)


def test_graph_replay_equals_eager_with_work_between():
    ev, b = _batch()
    s = torch.cuda.Stream()
    eager = Chain(G, b, True, s)
    with torch.cuda.stream(s):
        eager.enqueue()
    s.synchronize()
    ref = eager.outputs()
    gc = Chain(G, b, True, s)
    graph = GraphChain([gc], s)
    other = Chain(G, b, False, s)
    for i in range(4):
        # clobber the graph's outputs and run unrelated work eagerly in between
        gc.tracks.hit_clu.fill_(-5)
        gc.tracks.clu2trk.fill_(-5)
        with torch.cuda.stream(s):
            other.enqueue()
            _ = (torch.ones(1 << 20, device="cuda") * i).sum()
        graph.replay()
        s.synchronize()
        assert same_outputs(gc.outputs(), ref), f"replay {i}"


def test_plain_chains_in_one_graph_equal_batched():
    ev, b = _batch(8)
    s = torch.cuda.Stream()
    whole = Chain(G, b, True, s)
    with torch.cuda.stream(s):
        whole.enqueue()
    s.synchronize()
    w = whole.outputs()
    chains = plain_chains(G, b, True, s)
    graph = GraphChain(chains, s)
    graph.replay()
    s.synchronize()
    hit_clu, c2t, nt = [], np.full(b.n, -1), 0
    for i, c in enumerate(chains):
        o = c.outputs()
        a = int(ev.inst_off[i])
        hit_clu.append(o["hit_clu"] + a)
        m = o["clu2trk"] >= 0
        c2t[a:a + len(m)][m] = o["clu2trk"][m] + nt
        nt += len(o["param"])
    assert np.array_equal(np.concatenate(hit_clu), w["hit_clu"])
    assert np.array_equal(c2t, w["clu2trk"])


def test_autotune_candidates_keep_output(tmp_path, monkeypatch):
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "tune.json"))
    ev, b = _batch(10)
    entry = autotune.tune(G, b, steps=2, candidates=[(0.5, 64), (1.0, 128), (4.0, 256)],
                          use_cache=False)
    assert all(t["identical"] for t in entry["trials"])
    assert (tmp_path / "tune.json").exists()
