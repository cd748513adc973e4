"""The quality figures (efficiency, fakes, clones) against a plain loop over
the tracks on the oracle's config-1 output, and on hand-made cases."""
import numpy as np

import oracle
import synth
from synth.quality import track_quality

G = synth.geometry()


def _loop(label, inst_off, ho, hc, min_hits):
    inst = np.searchsorted(inst_off, np.arange(len(label)), side="right") - 1
    match = []
    for k in range(len(ho) - 1):
        l = label[hc[ho[k]:ho[k + 1]]]
        u, c = np.unique(l, return_counts=True)
        j = int(np.argmax(c))
        match.append((int(u[j]), int(inst[hc[ho[k]]])) if u[j] >= 0 and 2 * c[j] > len(l) else None)
    good = {(int(p), int(i)) for p, i in zip(label, inst) if p >= 0}
    good = {g for g in good if np.sum((label == g[0]) & (inst == g[1])) >= min_hits}
    got = [m for m in match if m is not None]
    eff = np.mean([g in set(got) for g in good])
    return eff, np.mean([m is None for m in match]), (len(got) - len(set(got))) / max(1, len(got))


def test_quality_matches_loop_on_oracle_output():
    ev = synth.config1()
    T = oracle.track(G, oracle.DEFAULT_PARAMS, ev.inst_off, ev.y, ev.z, ev.row).tracks
    q = track_quality(ev.label, ev.inst_off, T.hit_off, T.hit_clu, 30)
    e, f, c = _loop(ev.label, ev.inst_off, T.hit_off, T.hit_clu, 30)
    assert abs(q["efficiency"] - e) < 1e-12 and abs(q["fake_rate"] - f) < 1e-12
    assert abs(q["clone_rate"] - c) < 1e-12 and q["efficiency"] >= 0.9


def test_quality_hand_made():
    # two instances; particle 0 in both, particle 1 only in the second
    label = np.array([0, 0, 0, 0, -1, 0, 0, 0, 1, 1, 1, 1])
    inst_off = np.array([0, 5, 12])
    # track A: clusters 0-3 (p0, inst 0); B: 5,6,7 (p0, inst 1); C: 8,9,10 (p1);
    # D: 9,10,11 (p1 again: a clone); E: 4,8 (noise + p1: no majority -> fake)
    hc = np.array([0, 1, 2, 3, 5, 6, 7, 8, 9, 10, 9, 10, 11, 4, 8])
    ho = np.array([0, 4, 7, 10, 13, 15])
    q = track_quality(label, inst_off, ho, hc, min_hits=3)
    assert q["reconstructable"] == 3 and q["tracks"] == 5
    assert q["efficiency"] == 1.0 and q["fake_rate"] == 0.2 and q["clone_rate"] == 0.25
