"""Element-by-element comparison of a GPU tracking run with the CPU oracle
(test infrastructure: used by the GPU tests and the smoke check)."""
from __future__ import annotations

import numpy as np
import torch

import oracle
import paper_2511_17018_amd as tpc
import synth

G = synth.geometry()
P = dict(oracle.DEFAULT_PARAMS)
NR = 152


def bits(a):
    """Bit patterns of a binary32 array, with every NaN as one canonical
    pattern: IEEE 754 leaves the sign and payload of the NaN an invalid
    operation delivers to the implementation (x86 gives a negative quiet
    NaN, the GPU a positive one), so only NaN-ness is compared."""
    a = np.ascontiguousarray(a)
    if a.dtype != np.float32:
        return a
    b = a.view(np.int32).copy()
    b[np.isnan(a)] = 0x7FC00000
    return b


def run_gpu(ev_or_arrays, det=True, device="cuda", **kw):
    a = ev_or_arrays
    batch = tpc.upload(a.x, a.y, a.z, a.row, a.charge, a.inst_off, device)
    return tpc.track(G, batch, det=det, **kw)


def gpu_arrays(run: tpc.TrackRun, n: int) -> dict:
    """Everything a run produced, on the host."""
    res = run.result
    ws = run.ws
    cap = ws.layout.cap_tracklets
    S = int(min(res["n_start"], cap))
    nb = int(res["n_bins"])
    nt, nh = int(res["n_tracks"]), int(res["n_hits"])
    h = lambda t: t.cpu().numpy()  # noqa: E731
    i32, f32 = torch.int32, torch.float32
    out = dict(
        sseg=h(run.grid.sseg), perm=h(run.grid.perm), ys=h(run.grid.yz)[:, 0].copy(),
        zs=h(run.grid.yz)[:, 1].copy(),
        row_off=h(run.grid.row_off), meta=h(run.grid.meta), bin_off=h(run.grid.bin_off)[:nb],
        up=h(ws.view("up", i32, n)), dn=h(ws.view("dn", i32, n)),
        up2=h(ws.view("up2", i32, n)), dn2=h(ws.view("dn2", i32, n)),
        start=h(ws.view("start", i32, cap))[:S],
        tl_par=h(ws.view("tl_par", f32, 5 * cap)).reshape(5, cap)[:, :S].T.copy(),
        tl_cov=h(ws.view("tl_cov", f32, 15 * cap)).reshape(15, cap)[:, :S].T.copy(),
        tl_chi2=h(ws.view("tl_chi2", f32, cap))[:S],
        tl_nhit=h(ws.view("tl_nhit", i32, cap))[:S],
        tl_rmin=h(ws.view("tl_rmin", i32, cap))[:S],
        tl_rmax=h(ws.view("tl_rmax", i32, cap))[:S],
        tl_status=h(ws.view("tl_status", i32, cap))[:S],
        tl_hit=h(ws.view("tl_hit", i32, NR * cap)).reshape(NR, cap)[:, :S].T.copy(),
        param=h(run.tracks.param)[:nt], cov=h(run.tracks.cov)[:nt], chi2=h(run.tracks.chi2)[:nt],
        ndf=h(run.tracks.ndf)[:nt], x_ref=h(run.tracks.x_ref)[:nt],
        hit_off=h(run.tracks.hit_off)[:nt + 1], hit_clu=h(run.tracks.hit_clu)[:nh],
        clu2trk=h(run.tracks.clu2trk)[:n], result=res)
    return out


def _eq(name, a, b, errors):
    a = np.asarray(a)
    b = np.asarray(b)
    if a.shape != b.shape:
        errors.append(f"{name}: shape {a.shape} vs {b.shape}")
        return
    if not np.array_equal(bits(a), bits(b)):
        k = int(np.argmax((bits(a) != bits(b)).reshape(-1)))
        errors.append(f"{name}: {int((bits(a) != bits(b)).sum())} differ, first flat index {k}: "
                      f"{a.reshape(-1)[k]!r} vs {b.reshape(-1)[k]!r}")


def compare_det(g: dict, o: oracle.ChainResult) -> list:
    """Bit-exact comparison (deterministic mode) of every stage; returns errors."""
    e = []
    res = g["result"]
    gr = o.grid
    if int(res["n_bad"]) != gr.n_bad:
        e.append(f"n_bad {res['n_bad']} vs {gr.n_bad}")
    if int(res["n_bins"]) != gr.n_bins:
        e.append(f"n_bins {res['n_bins']} vs {gr.n_bins}")
        return e
    if int(res["overflow"]) != 0:
        e.append(f"overflow {res['overflow']}")
    _eq("sseg", g["sseg"], gr.sseg, e)
    _eq("perm", g["perm"], gr.perm, e)
    _eq("ys", g["ys"], gr.ys, e)
    _eq("zs", g["zs"], gr.zs, e)
    _eq("row_off", g["row_off"], gr.row_off, e)
    _eq("meta_i", g["meta"][:, :4], gr.meta_i, e)
    _eq("meta_f", g["meta"][:, 4:], gr.meta_f.view(np.int32), e)
    _eq("bin_off", g["bin_off"], gr.bin_off, e)
    for k, v in (("up", o.up), ("dn", o.dn), ("up2", o.up2), ("dn2", o.dn2), ("start", o.start)):
        _eq(k, g[k], v, e)
    if e:
        return e
    tl = o.tracklets
    _eq("tl_status", g["tl_status"], tl.status, e)
    _eq("tl_nhit", g["tl_nhit"], tl.nhit, e)
    _eq("tl_rmin", g["tl_rmin"], tl.rmin, e)
    _eq("tl_rmax", g["tl_rmax"], tl.rmax, e)
    if e:
        return e
    _eq("tl_par", g["tl_par"], tl.par, e)
    _eq("tl_cov", g["tl_cov"], tl.cov, e)
    _eq("tl_chi2", g["tl_chi2"], tl.chi2, e)
    rows = np.arange(NR)[None, :]
    m = (rows >= tl.rmin[:, None]) & (rows <= tl.rmax[:, None])
    _eq("tl_hit", np.where(m, g["tl_hit"], -7), np.where(m, tl.hit, -7), e)
    # outside [rmin, rmax] every slot reads -1 (the selection scans whole rows)
    _eq("tl_hit outside the row range", np.where(m, -1, g["tl_hit"]),
        np.full(g["tl_hit"].shape, -1, g["tl_hit"].dtype), e)
    T = o.tracks
    if int(res["need_tracks"]) != T.need_tracks or int(res["need_hits"]) != T.need_hits:
        e.append(f"need {res['need_tracks']},{res['need_hits']} vs {T.need_tracks},{T.need_hits}")
    for k, v in (("param", T.par), ("cov", T.cov), ("chi2", T.chi2), ("ndf", T.ndf),
                 ("x_ref", T.x_ref), ("hit_off", T.hit_off), ("hit_clu", T.hit_clu),
                 ("clu2trk", T.clu2trk)):
        _eq(k, g[k], v, e)
    return e


def match_tracks(hit_off_a, hit_clu_a, hit_off_b, hit_clu_b, n):
    """Match tracks of two outputs by shared clusters (>= 50 % of the smaller);
    returns the fraction of clusters assigned differently (R30)."""
    ca = np.full(n, -1)
    cb = np.full(n, -1)
    for k in range(len(hit_off_a) - 1):
        ca[hit_clu_a[hit_off_a[k]:hit_off_a[k + 1]]] = k
    for k in range(len(hit_off_b) - 1):
        cb[hit_clu_b[hit_off_b[k]:hit_off_b[k + 1]]] = k
    both = (ca >= 0) & (cb >= 0)
    pairs, shared = np.unique(np.stack([ca[both], cb[both]], 1), axis=0, return_counts=True)
    la = np.diff(hit_off_a)
    lb = np.diff(hit_off_b)
    match = {}
    order = np.argsort(-shared, kind="stable")
    used_b = set()
    for i in order:
        a, b = pairs[i]
        if a in match or b in used_b:
            continue
        if shared[i] >= 0.5 * min(la[a], lb[b]):
            match[a] = b
            used_b.add(b)
    mapped = np.array([match.get(k, -2) for k in range(len(la))] + [-1])
    diff = np.where(ca >= 0, mapped[ca], -1) != cb
    return float(diff.mean()) if n else 0.0


def check_structure(g: dict, row: np.ndarray, min_track_hits: int = 10) -> list:
    """Validity of a tracking output whatever its order (production mode):
    hit_off ascending from 0; every track holds at least min_track_hits
    clusters in strictly ascending row; no cluster on two tracks; clu2trk
    names exactly the track of every listed cluster and -1 elsewhere; the
    counts agree with the result word and nothing overflowed."""
    e = []
    res = g["result"]
    ho, hc, c2t = g["hit_off"], g["hit_clu"], g["clu2trk"]
    nt = len(ho) - 1
    if int(res["overflow"]) != 0:
        e.append(f"overflow {res['overflow']}")
    if nt != int(res["n_tracks"]) or nt != int(res["need_tracks"]):
        e.append(f"tracks {nt} vs n_tracks {res['n_tracks']} need {res['need_tracks']}")
    if len(hc) != int(res["n_hits"]) or len(hc) != int(res["need_hits"]) or ho[-1] != len(hc):
        e.append(f"hits {len(hc)} vs n_hits {res['n_hits']} need {res['need_hits']} end {ho[-1]}")
        return e
    if ho[0] != 0 or np.any(np.diff(ho) < min_track_hits):
        e.append("hit_off not ascending by at least min_track_hits")
        return e
    if len(hc) and (hc.min() < 0 or hc.max() >= len(c2t)):
        e.append("hit list names a cluster out of range")
        return e
    if len(np.unique(hc)) != len(hc):
        e.append(f"{len(hc) - len(np.unique(hc))} clusters on more than one track")
    trk = np.repeat(np.arange(nt), np.diff(ho))
    if not np.array_equal(c2t[hc], trk):
        e.append("clu2trk disagrees with the hit lists")
    listed = np.zeros(len(c2t), bool)
    listed[hc] = True
    if np.any(c2t[~listed] != -1):
        e.append("clu2trk names a track for an unlisted cluster")
    r = row[hc].astype(np.int64)
    same = trk[1:] == trk[:-1]
    if np.any(r[1:][same] <= r[:-1][same]):
        e.append("rows not strictly ascending within a track")
    return e


# Production error allowed per component, in units of the track's binary32
# rounding-noise scale: the production build rounds each operation to within
# about 2 ulp (fast reciprocal and square root) against 0.5 ulp, a factor 4
# in the noise scale, and 5 standard deviations of that keep a sample of
# 10^4 tracks clear of the tail.
K_PROD = 20.0
N_NOISE = 8     # perturbed binary32 replays per track for its noise scale


def prod_param_errors(g: dict, kept=None):
    """Per kept tracklet and parameter, against the binary64 replay of its
    hit list and relative to max(|p64|, floor): the production error, and
    the binary32 filter's rounding-noise scale on that list -- the largest
    of the deterministic binary32 error, the error of a binary32 replay with
    fused multiply-adds (another rounding of the same formulas) and the RMS
    error of N_NOISE binary32 replays with every hit moved by a random +-1
    ulp (a single binary32 error can be small by chance, so one draw alone is
    no scale)."""
    e_prod = replay_params(g, kept=kept)
    e_32 = replay_params(g, kept=kept, against=32)
    e_c = replay_params(g, kept=kept, against="32c")
    e_n = replay_params(g, kept=kept, against="noise")
    return e_prod, np.maximum(np.maximum(e_32, e_c), e_n)


def prod_bound_violations(e_prod, e_32, k=K_PROD, base=1e-4):
    """Tracklets whose production error exceeds max(base, k * binary32
    rounding-noise scale) in some parameter."""
    bound = np.maximum(base, k * e_32)
    return np.nonzero(np.any(e_prod > bound, axis=1))[0]


def replay_params(g: dict, prec=64, kept=None, against=None):
    """binary64 replay of every kept GPU tracklet on its own hit list:
    relative errors of the GPU parameters (or, with against=32, of the
    binary32 replay of the same list) with respect to it."""
    floor = np.array([1, 1, 0.01, 0.01, 0.01])
    rel = []
    ts = np.nonzero(g["tl_status"] == 0)[0] if kept is None else kept
    for t in ts:
        h0 = g["start"][t]
        r0 = int(g["sseg"][h0] % NR)
        rmin, rmax = int(g["tl_rmin"][t]), int(g["tl_rmax"][t])
        hy = np.zeros(NR, np.float32)
        hz = np.zeros(NR, np.float32)
        has = np.zeros(NR, np.uint8)
        rows = np.arange(rmin, rmax + 1)
        hh = g["tl_hit"][t, rows]
        m = hh >= 0
        hy[rows[m]] = g["ys"][hh[m]]
        hz[rows[m]] = g["zs"][hh[m]]
        has[rows[m]] = 1
        ok, par, cov, chi2 = oracle.replay(G, P, r0, rmin, rmax, hy, hz, has, prec=prec)
        if not ok:
            rel.append(np.full(5, np.nan))
            continue
        if against in (32, "32c"):
            ok32, p32, _, _ = oracle.replay(G, P, r0, rmin, rmax, hy, hz, has, prec=against)
            cand = p32.astype(np.float64) if ok32 else np.full(5, np.inf)
        elif against == "noise":
            rng = np.random.default_rng(int(t))
            sq = np.zeros(5)
            for _ in range(N_NOISE):
                up = rng.integers(0, 2, (2, NR)).astype(bool)
                hy2 = np.where(up[0], np.nextafter(hy, np.float32(np.inf)),
                               np.nextafter(hy, np.float32(-np.inf))).astype(np.float32)
                hz2 = np.where(up[1], np.nextafter(hz, np.float32(np.inf)),
                               np.nextafter(hz, np.float32(-np.inf))).astype(np.float32)
                okn, pn, _, _ = oracle.replay(G, P, r0, rmin, rmax, hy2, hz2, has, prec=32)
                d = (pn.astype(np.float64) - par) if okn else np.full(5, np.inf)
                sq += d * d
            rel.append(np.sqrt(sq / N_NOISE) / np.maximum(np.abs(par), floor))
            continue
        else:
            cand = g["tl_par"][t]
        rel.append(np.abs(cand - par) / np.maximum(np.abs(par), floor))
    return np.array(rel).reshape(-1, 5)
