"""Writes tests/golden/config1_oracle.json from the CPU oracle alone.

The stored counts and digests pin the oracle's binary32 output on the seeded
config-1 event (one sector wedge, 50 tracks) so that any later change of the
oracle's arithmetic shows up as a failing test and has to be justified.
Run:  python tests/golden/make_golden.py
"""
import hashlib
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth   # noqa: E402


def digest(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def summary():
    ev = synth.config1()
    r = oracle.track(synth.geometry(), oracle.DEFAULT_PARAMS, ev.inst_off, ev.y, ev.z, ev.row)
    kept = r.tracklets.status == 0
    return {
        "event": "config1 seed 0x7C0001",
        "n_clusters": int(ev.n),
        "input_sha256": digest(ev.y, ev.z, ev.row, ev.inst_off),
        "n_bad": r.grid.n_bad,
        "n_bins": r.grid.n_bins,
        "n_links": int((r.up >= 0).sum()),
        "n_clean_links": int((r.up2 >= 0).sum()),
        "n_start": int(len(r.start)),
        "n_kept": int(kept.sum()),
        "n_tracks": int(len(r.tracks.chi2)),
        "n_assigned": int((r.tracks.clu2trk >= 0).sum()),
        "grid_sha256": digest(r.grid.perm, r.grid.bin_off),
        "links_sha256": digest(r.up, r.dn, r.up2, r.dn2, r.start),
        "tracklets_sha256": digest(r.tracklets.par, r.tracklets.cov, r.tracklets.chi2,
                                   r.tracklets.nhit),
        "tracks_sha256": digest(r.tracks.hit_off, r.tracks.hit_clu, r.tracks.par),
    }


if __name__ == "__main__":
    with open(os.path.join(HERE, "config1_oracle.json"), "w") as f:
        json.dump(summary(), f, indent=1)
        f.write("\n")
