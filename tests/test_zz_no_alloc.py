"""The allocation-free reverse pass (tpc_refit_backward_noalloc) against
tpc_refit_backward through the C ABI: two calls in a row on one GPU, the
second on a smaller input, each equal to the workspace entry point's output
bit for bit (same kernels, exact fixed-point map sums)."""
import sys

import numpy as np
import pytest
import torch

import paper_2511_17018_amd as tpc
import synth

pytestmark = pytest.mark.gpu

G = synth.geometry()


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _inputs(n_found, rep):
    ev = synth.config5(n_found=n_found, rep=rep)
    xyz = torch.from_numpy(np.stack([ev.x, ev.y, ev.z]).astype(np.float32)).cuda()
    row = torch.from_numpy(ev.row.view(np.int16)).cuda()
    trk = tpc.upload_refit_tracks(ev.extra["hit_off"], ev.extra["hit_clu"], ev.sector,
                                  ev.extra["seed_par"])
    m = torch.from_numpy(np.ascontiguousarray(ev.extra["D_true"] * 0.7, np.float32)).cuda()
    w = torch.from_numpy(np.random.default_rng(rep).uniform(0.5, 1.5, len(ev.extra["hit_off"]) - 1)
                         .astype(np.float32)).cuda()
    return xyz, row, trk, m, w


def test_noalloc_reverse_pass_equals_workspace_entry_point_twice():
    # the outputs of both calls are allocated up front, at the larger size
    nmax = 0
    cases = [(600, 1), (150, 2)]
    ins = [_inputs(n, r) for n, r in cases]
    nmax = max(x[0].shape[1] for x in ins)
    gmap = torch.empty((152, 18), dtype=torch.float32, device="cuda")
    gxyz = torch.empty((3, nmax), dtype=torch.float32, device="cuda")
    for (n, r), (xyz, row, trk, m, w) in zip(cases, ins):
        _say(f"[noalloc] tracks={n} clusters={xyz.shape[1]}")
        chi2, status, ckpt = tpc.refit(G, xyz, row, trk, m)
        ref_map, ref_xyz = tpc.refit_backward(G, xyz, row, trk, m, ckpt, status, w)
        gxyz.fill_(float("nan"))
        got_map, got_xyz = tpc.refit_backward_noalloc(G, xyz, row, trk, m, ckpt, status, w,
                                                      gmap, gxyz)
        torch.cuda.synchronize()
        assert torch.equal(got_map, ref_map)
        assert torch.equal(got_xyz, ref_xyz)
        assert torch.count_nonzero(got_map) > 0
