"""Planted mistakes: each one alone in a copy of the oracle's C sources must
make at least one pin of the oracle fail.

This checks the pins, not the oracle: a pin set that lets a dropped term, a
swapped index, a wrong sign, an off-by-one threshold or a reversed tie order
pass would also let such a mistake in the oracle itself go unseen.  Each
mutant is built with gcc into a temporary library, and the pin files run
against it in a child pytest (the oracle package loads the library named by
TPC_ORACLE_LIB).  Mutants are built and checked in parallel worker threads.
"""
import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_DIR = os.path.join(ROOT, "oracle")
TRACK = ["tests/test_oracle_pins.py"]
# A digest of the oracle's own output fails on any change of its arithmetic
# and so pins nothing; the planted mistakes must be caught without it.
NOT_PINS = ["--deselect", "tests/test_oracle_pins.py::test_oracle_matches_stored_golden_summary"]
REFIT = ["tests/test_oracle_refit.py"]
BOTH = TRACK + REFIT
TRANSFORM = ["tests/test_oracle_transform.py"]
MERGE = ["tests/test_oracle_merge.py"]

# (source file, pin files, what is planted, original text, planted text)
MUTATIONS = [
    ("kalman.h", BOTH, "drop L*kB in du2q", "du2q = hlc * (dLq * cc + L * kB);", "du2q = hlc * (dLq * cc);"),
    ("kalman.h", BOTH, "wrong sign Si01", "q.si01 = -(S01 / det);", "q.si01 = (S01 / det);"),
    ("kalman.h", BOTH, "transpose k0 index", "k0[i] = CC(s, i, 0) * q.si00 + CC(s, i, 1) * q.si01;", "k0[i] = CC(s, i, 1) * q.si00 + CC(s, i, 0) * q.si01;"),
    ("kalman.h", BOTH, "cov B1 d/e swap", "B1[j] = ((CC(s, 1, j) + d * CC(s, 2, j)) + e * CC(s, 3, j)) + gq * CC(s, 4, j);", "B1[j] = ((CC(s, 1, j) + e * CC(s, 2, j)) + d * CC(s, 3, j)) + gq * CC(s, 4, j);"),
    ("kalman.h", BOTH, "series 3/40 term dropped", "real g = one + u2 * (K_SIXTH + u2 * K_3_40);", "real g = one + u2 * K_SIXTH;"),
    ("kalman.h", BOTH, "dg wrong", "real dg = K_SIXTH + u2 * K_3_20;", "real dg = K_SIXTH + u2 * K_3_40;"),
    ("kalman.h", BOTH, "f formula", "real f = (snp + s2) / (c1 + c2);", "real f = (snp + s2) / (c1 - c2 + 2);"),
    ("kalman.h", BOTH, "update hc uses C row 0", "hc1[i] = CC(s, 1, i);", "hc1[i] = CC(s, 0, i);"),
    ("kalman.h", BOTH, "chi2 weight si00 for si11", "return r0 * (q->si00 * r0 + q->si01 * r1) + r1 * (q->si01 * r0 + q->si11 * r1);", "return r0 * (q->si00 * r0 + q->si01 * r1) + r1 * (q->si01 * r0 + q->si00 * r1);"),
    ("kalman.h", BOTH, "cov update sign", "s->c[ci(i, j)] = s->c[ci(i, j)] - (k0[i] * hc0[j] + k1[i] * hc1[j]);", "s->c[ci(i, j)] = s->c[ci(i, j)] - (k0[i] * hc0[j] + k1[i] * hc0[j]);"),
    ("tpc_oracle.c", TRACK, "nf t index", "real t = (x0 - xm) / (xp - xm);", "real t = (xp - x0) / (xp - xm);"),
    ("tpc_oracle.c", TRACK, "nf ez uses y", "real ez = zh - (zs[d] + (zs[u] - zs[d]) * t);", "real ez = zh - (zs[d] + (zs[u] - ys[d]) * t);"),
    ("tpc_oracle.c", TRACK, "nf tie break reversed", "(sc == bs && (perm[u] < perm[bu] ||", "(sc == bs && (perm[u] > perm[bu] ||"),
    ("tpc_oracle.c", TRACK, "clean not mutual", "up2[h] = (u >= 0 && dn[u] == h) ? u : -1;", "up2[h] = (u >= 0) ? u : -1;"),
    ("tpc_oracle.c", TRACK, "start hit admits short chains", "if (len >= P->min_chain) start[S++]", "if (len >= P->min_chain - 1) start[S++]"),
    ("tpc_oracle.c", TRACK, "start hit ignores down link", "if (dn2[h] != -1 || up2[h] < 0) continue;", "if (up2[h] < 0) continue;"),
    ("tpc_oracle.c", TRACK, "key chi2 not inverted", "((uint64_t)(~bits & 0x7FFFFFFFu) << 25)", "((uint64_t)(bits & 0x7FFFFFFFu) << 25)"),
    ("tpc_oracle.c", TRACK, "key index not reversed", "(uint64_t)(0x1FFFFFFu - (uint64_t)lid)", "(uint64_t)(lid)"),
    ("tpc_oracle.c", TRACK, "track threshold off by one", "if (own < P->min_track_hits) continue;", "if (own < P->min_track_hits - 1) continue;"),
    ("tpc_oracle.c", TRACK, "init tgl uses dx", "st.p[3] = dzi / Li;", "st.p[3] = dzi / dxi;"),
    ("tpc_oracle.c", TRACK, "grid bin off by one", "if (f >= (real)(n - 1)) return n - 1;", "if (f >= (real)(n - 2) && n > 1) return n - 2;"),
    ("tpc_oracle.c", TRACK, "phase 3 no downward search", "      int miss = 0;\n      while (r > 0) {", "      int miss = 0;\n      while (r > 1000) {"),
    ("tpc_refit.c", REFIT, "map sign in plane x", "return (real)x[c] + (real)dmap[", "return (real)x[c] - (real)dmap["),
    ("tpc_refit.c", REFIT, "adjoint X carry sign", "gX_next = -dxb;", "gX_next = dxb;"),
    ("tpc_refit.c", REFIT, "adjoint gy from z", "gy[c] = mb[0];", "gy[c] = mb[1];"),
    ("tpc_refit.c", REFIT, "adjoint z propagation uses snp", "pp[1] = p0[1] + p0[3] * q.ds;", "pp[1] = p0[1] + p0[2] * q.ds;"),
    ("tpc_refit.c", REFIT, "adjoint symmetric factor dropped", "const double Fb[6] = {2 * XFC[0][2],", "const double Fb[6] = {XFC[0][2],"),
    ("tpc_refit.c", REFIT, "adjoint first hit map gradient dropped", "gmap[(int64_t)row[c0] * NPHI + sector[c0] % NPHI] += gX_next;", "(void)0;"),
    ("tpc_oracle.c", TRACK, "nf z window uses y width", "FABS(zs[pos] - zh) <= wz)", "FABS(zs[pos] - zh) <= wy)"),
    ("tpc_oracle.c", TRACK, "nf chi2 cut dropped", "if (!(sc <= cmax)) continue;", "(void)0;"),
    ("tpc_oracle.c", TRACK, "nf weights swapped", "real sc = (ey * ey) * ivy + (ez * ez) * ivz;", "real sc = (ey * ey) * ivz + (ez * ez) * ivy;"),
    ("tpc_oracle.c", TRACK, "validity margin dropped", "* (real)g->tan_half + (real)P->y_valid_margin;", "* (real)g->tan_half;"),
    ("tpc_oracle.c", TRACK, "grid width without sqrt", "real w = SQRT((dy * dz) / nb);", "real w = (dy * dz) / nb;"),
    ("tpc_oracle.c", TRACK, "phase2 miss not reset", "save = st;\n          miss = 0;", "save = st;"),
    ("tpc_oracle.c", TRACK, "phase2 save not updated", "save = st;\n          miss = 0;", "miss = 0;"),
    ("tpc_oracle.c", TRACK, "phase3 out not updated", "out = st;\n          miss = 0;", "miss = 0;"),
    ("tpc_oracle.c", TRACK, "edge check sign", "if (!(FABS(st.p[0]) <= X[r] * tanh_ + edge)) break;", "if (!(FABS(st.p[0]) <= X[r] * tanh_ - edge)) break;"),
    ("tpc_oracle.c", TRACK, "search tie reversed", "G->perm[pos] < G->perm[best]", "G->perm[pos] > G->perm[best]"),
    ("tpc_oracle.c", TRACK, "search z window from S00", "real wz = SQRT(pick * q->S11) + margin;", "real wz = SQRT(pick * q->S00) + margin;"),
    ("tpc_oracle.c", TRACK, "search pick cut dropped", "if (ch <= pick && (best < 0", "if ((best < 0"),
    ("tpc_oracle.c", TRACK, "tracklet min hits off by one", "if (n < P->min_tracklet_hits) stat = 1;", "if (n < P->min_tracklet_hits - 1) stat = 1;"),
    ("tpc_oracle.c", TRACK, "miss limit off by one", "if (++miss >= P->tc_max_miss) break;", "if (++miss > P->tc_max_miss) break;"),
    ("tpc_oracle.c", TRACK, "ndf off by one", "tndf[nt] = 2 * nhit[t] - 5;", "tndf[nt] = 2 * nhit[t] - 4;"),
    ("tpc_oracle.c", TRACK, "x_ref at rmax", "txref[nt] = g->row_x[rmin[t]];", "txref[nt] = g->row_x[rmax[t]];"),
    ("tpc_oracle.c", TRACK, "hit capacity strict", "nh + own <= cap_hits", "nh + own < cap_hits"),
    ("tpc_oracle.c", TRACK, "hit list positions", "thit_clu[j++] = perm[h];", "thit_clu[j++] = h;"),
    ("tpc_refit.c", REFIT, "refit drops last hit", "for (int64_t k = a + 1; k < b; k++) {\n    const int64_t c = hit_clu[k];\n    const real xk", "for (int64_t k = a + 1; k < b - 1; k++) {\n    const int64_t c = hit_clu[k];\n    const real xk"),
    ("tpc_refit.c", REFIT, "refit seed snp from tgl", "st.p[2] = (real)seed5[2];", "st.p[2] = (real)seed5[3];"),
    ("tpc_refit.c", REFIT, "refit x not advanced", "    xprev = xk;\n", "    (void)xk;\n"),
    ("tpc_transform.c", TRANSFORM, "lerp reversed", "return a + (b - a) * t;", "return b + (a - b) * t;"),
    ("tpc_transform.c", TRANSFORM, "cell fraction not clamped", "  if (t > 1) t = 1;\n", "\n"),
    ("tpc_transform.c", TRANSFORM, "map v from the nominal plane", "cell(yc / xc,", "cell(yc / (real)T->row_x[r],"),
    ("tpc_transform.c", TRANSFORM, "side sign", "real zc = side ? -za : za;", "real zc = side ? za : -za;"),
    ("tpc_transform.c", TRANSFORM, "pad centre sign", "((real)pad[c] - (real)T->pad_c[r])", "((real)pad[c] + (real)T->pad_c[r])"),
    ("tpc_transform.c", TRANSFORM, "time offset sign", "(real)T->tbin - (real)T->t0)", "(real)T->tbin + (real)T->t0)"),
    ("tpc_transform.c", TRANSFORM, "map w from z", "cell(d, (real)T->w0,", "cell(za, (real)T->w0,"),
    ("tpc_transform.c", TRANSFORM, "dz correction sign", "zc = zc + corr[2];", "zc = zc - corr[2];"),
    ("tpc_transform.c", TRANSFORM, "map u and w lerp swapped", "corr[q] = lerp(f0, f1, au);", "corr[q] = lerp(f0, f1, aw);"),
    ("tpc_refit.c", REFIT, "scattering without 1/beta^2", "const real th2 = ((real)K_MS * (path * ix0)) * (w * bg);", "const real th2 = ((real)K_MS * (path * ix0)) * w;"),
    ("tpc_refit.c", REFIT, "scattering snp noise without 1+tgl^2", "th2 * (((one - snp) * (one + snp)) * t2)", "th2 * ((one - snp) * (one + snp))"),
    ("tpc_refit.c", REFIT, "scattering tgl-qpt correlation sign", "s->c[13] = s->c[13] + th2 * (t2 * qt);", "s->c[13] = s->c[13] - th2 * (t2 * qt);"),
    ("tpc_refit.c", REFIT, "energy loss sign", "(SQRT(w * bg) * (K * bg)) * (path * sgn)", "(SQRT(w * bg) * (K * bg)) * (path * -sgn)"),
    ("tpc_refit.c", REFIT, "energy loss q/pt variance scaled once", "s->c[14] = (s->c[14] * f) * f;", "s->c[14] = s->c[14] * f;"),
    ("tpc_refit.c", REFIT, "adjoint scattering path term dropped", "pathb += A * K_MS * m->ix0 * m->w * m->bg;", "(void)0;"),
    ("tpc_refit.c", REFIT, "adjoint energy loss sqrt term dropped", "wb += wbgb * m->bg;", "(void)0;"),
    ("tpc_refit.c", REFIT, "field bin from |z|", "floor(((double)z + 250.0) *", "floor((fabs((double)z) + 250.0) *"),
    ("tpc_merge.c", MERGE, "rotated y sign", "s->p[0] = y * ca - x * sa;", "s->p[0] = y * ca + x * sa;"),
    ("tpc_merge.c", MERGE, "rotation jacobian j00 sign", "const real j00 = ca - sa * (snn / csn);", "const real j00 = ca + sa * (snn / csn);"),
    ("tpc_merge.c", MERGE, "rotation jacobian curvature term dropped", "const real j20 = -(kB * s->p[4]) * sa;", "const real j20 = 0;"),
    ("tpc_merge.c", MERGE, "rotation jacobian j22 inverted", "const real j22 = csn / csp;", "const real j22 = csp / csn;"),
    ("tpc_merge.c", MERGE, "ldl forward substitution sign", "v = v - L[i][k] * w[k];", "v = v + L[i][k] * w[k];"),
    ("tpc_merge.c", MERGE, "links not mutual", "if (succ[A] >= 0 && pred[succ[A]] == A) {", "if (succ[A] >= 0) {"),
    ("tpc_merge.c", MERGE, "inward covariance not inflated", "s.c[j] = s.c[j] * (real)INWARD_SCALE;", "(void)0;"),
    ("tpc_merge.c", MERGE, "chains start anywhere", "(pass == 0 && has_pred[t])", "(pass == 0 && 0)"),
    ("tpc_merge.c", MERGE, "outer state without the segment's hits", "&s, &x, &k, hit_clu, a + 1, b - a - 1, 1,", "&s, &x, &k, hit_clu, a + 1, 0, 1,"),
    ("tpc_merge.c", MERGE, "global refit seed from the last segment", "m_seed(g, &s, y, z, m_hit_clu[a], par + t0 * 5);", "m_seed(g, &s, y, z, m_hit_clu[a], par + chain_seg[chain_off[m + 1] - 1] * 5);"),
]


def _run_mutant(m):
    fname, pins, name, before, after = m
    d = tempfile.mkdtemp(prefix="orc_mutant_")
    try:
        for f in os.listdir(ORACLE_DIR):
            if f.endswith((".c", ".h")):
                shutil.copy(os.path.join(ORACLE_DIR, f), d)
        path = os.path.join(d, fname)
        text = open(path).read()
        if before not in text:
            return name, "pattern not found"
        open(path, "w").write(text.replace(before, after, 1))
        lib = oracle.build(out=os.path.join(d, "liboracle.so"), srcdir=d)
        env = dict(os.environ, TPC_ORACLE_LIB=lib)
        r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                            *NOT_PINS, *pins], cwd=ROOT, env=env, capture_output=True, text=True,
                           timeout=600)
        return name, "caught" if r.returncode != 0 else "missed"
    finally:
        shutil.rmtree(d, ignore_errors=True)


def test_every_planted_mistake_fails_a_pin():
    workers = max(1, min(8, os.cpu_count() or 1))
    with ThreadPoolExecutor(workers) as ex:
        res = list(ex.map(_run_mutant, MUTATIONS))
    bad = [(n, s) for n, s in res if s != "caught"]
    assert not bad, bad
    assert len(res) == len(MUTATIONS) == len({m[2] for m in MUTATIONS})
