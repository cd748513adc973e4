"""Tracking quality against the generator's Monte-Carlo truth (evaluation
only; none of the tracker's arithmetic).

A found track matches MC particle p when more than half of its clusters
carry p's label.  A (particle, instance) pair is reconstructable when the
instance holds at least `min_hits` of its clusters.  Efficiency is the
fraction of reconstructable pairs matched by at least one found track of
that instance; the fake rate is the fraction of found tracks that match
nothing; the clone rate is the fraction of matched tracks beyond the first
one per pair.
"""
from __future__ import annotations

import numpy as np


def track_quality(label: np.ndarray, inst_off: np.ndarray, hit_off: np.ndarray,
                  hit_clu: np.ndarray, min_hits: int = 30) -> dict:
    label = np.asarray(label, np.int64)
    n = len(label)
    inst = np.searchsorted(np.asarray(inst_off), np.arange(n), side="right") - 1
    nt = len(hit_off) - 1
    nl = int(label.max()) + 2 if n else 1
    match = np.full(nt, -1, np.int64)
    if nt:
        lens = np.diff(hit_off)
        trk = np.repeat(np.arange(nt), lens)
        lab = label[hit_clu[:hit_off[-1]]]
        keys, cnt = np.unique(trk * nl + (lab + 1), return_counts=True)
        kt, kl = keys // nl, keys % nl - 1
        order = np.lexsort((-cnt, kt))          # per track, the largest count first
        first = np.ones(len(order), bool)
        first[1:] = kt[order][1:] != kt[order][:-1]
        top = order[first]
        ok = (kl[top] >= 0) & (2 * cnt[top] > lens[kt[top]])
        match[kt[top][ok]] = kl[top][ok]
    sig = label >= 0
    pair = label * (len(inst_off)) + inst
    u, c = np.unique(pair[sig], return_counts=True)
    good = u[c >= min_hits]
    m = match >= 0
    tpair = np.full(nt, -1, np.int64)
    if nt:
        tinst = inst[hit_clu[hit_off[:-1]]]
        tpair[m] = match[m] * len(inst_off) + tinst[m]
    found = np.unique(tpair[m])
    n_match = int(m.sum())
    return {
        "efficiency": float(np.isin(good, found).mean()) if len(good) else float("nan"),
        "fake_rate": float((~m).mean()) if nt else 0.0,
        "clone_rate": float((n_match - len(found)) / n_match) if n_match else 0.0,
        "reconstructable": int(len(good)),
        "tracks": int(nt),
        "min_hits": int(min_hits),
    }
