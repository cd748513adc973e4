"""Launch plans over the C ABI: pre-marshalled call chains and their capture
into a HIP graph.

A ``Chain`` holds the buffers and the ctypes argument tuples of one
tpc_grid_build + tpc_sector_track pair (one batch, or one instance in the
per-instance "plain" mode), so that enqueueing costs two foreign calls.  A
``GraphChain`` captures any list of chains on one stream into a HIP graph
(through torch's graph API, which drives hipStreamBeginCapture): the calls
only enqueue kernels -- no memsets, no host synchronisation -- so the
captured graph replays the same work.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import (Batch, Workspace, _ptr, alloc_grid, alloc_tracks, lib, make_geometry, make_params)


class Chain:
    """One grid build + sector tracking call with its own outputs."""

    def __init__(self, geom: dict, batch: Batch, det: bool = True, stream=None,
                 cap_tracklets: int = 0, hit_data: bool = False, **param_over):
        dev = batch.x.device
        self.batch = batch
        self.geom = make_geometry(geom)
        self.params = make_params(det, **param_over)
        self.grid = alloc_grid(batch.n_inst, batch.n, dev, self.params)
        self.tracks = alloc_tracks(batch.n, device=dev, hit_data=hit_data)
        self.ws = Workspace(batch.n_inst, batch.n, cap_tracklets, dev, self.params)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        sp = C.c_void_p(self.stream.cuda_stream)
        self._keep = (self.grid.struct(), self.tracks.struct(), batch.struct())
        gs, ts, cs = self._keep
        off_h = batch.inst_off_host.ctypes.data_as(C.c_void_p)
        self._ga = (C.byref(self.geom), C.byref(self.params), C.c_int32(batch.n_inst), off_h,
                    _ptr(batch.inst_off), cs, C.byref(gs), _ptr(self.ws.result),
                    _ptr(self.ws.grid_ws), C.c_size_t(self.ws.grid_ws.numel()), sp)
        self._ta = (C.byref(self.geom), C.byref(self.params), C.c_int32(batch.n_inst), off_h,
                    _ptr(batch.inst_off), cs, C.byref(gs), C.byref(ts), _ptr(self.ws.result),
                    _ptr(self.ws.track_ws), C.c_size_t(self.ws.track_ws.numel()),
                    C.c_int64(cap_tracklets), sp)
        self._lib = lib()

    def enqueue(self) -> None:
        st = self._lib.tpc_grid_build(*self._ga)
        st2 = self._lib.tpc_sector_track(*self._ta)
        if st or st2:
            raise RuntimeError(f"tracker call failed: grid {st}, track {st2}")

    def result(self):
        return self.ws.read_result()

    def outputs(self) -> dict:
        """Tracks and association on the host (for comparisons)."""
        r = self.result()
        nt, nh = int(r["n_tracks"]), int(r["n_hits"])
        t = self.tracks
        return dict(hit_off=t.hit_off[:nt + 1].cpu().numpy(), hit_clu=t.hit_clu[:nh].cpu().numpy(),
                    param=t.param[:nt].cpu().numpy(), clu2trk=t.clu2trk.cpu().numpy())


def plain_chains(geom: dict, batch: Batch, det: bool = True, stream=None, **param_over):
    """One chain per instance (the per-instance launch mode)."""
    return [Chain(geom, batch.slice(i), det, stream, **param_over) for i in range(batch.n_inst)]


class GraphChain:
    """A list of chains captured into one HIP graph on `stream`."""

    def __init__(self, chains: list, stream: torch.cuda.Stream):
        for c in chains:
            if c.stream.cuda_stream != stream.cuda_stream:
                raise ValueError("every chain must be prepared on the capture stream")
        self.chains = chains
        self.stream = stream
        # warm up on the capture stream, then capture
        with torch.cuda.stream(stream):
            for c in chains:
                c.enqueue()
        stream.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph, stream=stream):
            for c in chains:
                c.enqueue()

    def replay(self) -> None:
        with torch.cuda.stream(self.stream):
            self.graph.replay()


def canonical_tracks(o: dict) -> dict:
    """Tracks as {tuple of input indices: parameter bits}: equal for two runs
    whose outputs differ only in track order (e.g. another grid bin size)."""
    ho, hc, par = o["hit_off"], o["hit_clu"], o["param"]
    return {tuple(hc[ho[k]:ho[k + 1]].tolist()): par[k].view(np.int32).tobytes()
            for k in range(len(ho) - 1)}


def same_outputs(a: dict, b: dict) -> bool:
    """Same tracks (hit sets, parameter bits) and the same cluster partition."""
    if canonical_tracks(a) != canonical_tracks(b):
        return False
    ca, cb = a["clu2trk"], b["clu2trk"]
    if not np.array_equal(ca < 0, cb < 0):
        return False
    m = ca >= 0
    pairs = np.unique(np.stack([ca[m], cb[m]], 1), axis=0)
    return len(pairs) == len(np.unique(ca[m])) == len(np.unique(cb[m]))
