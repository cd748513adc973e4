/*
 * CPU oracle of the TPC sector tracker -- TEST INFRASTRUCTURE ONLY
 * (loaded by the tests, the smoke check and the benchmark's CPU-baseline leg,
 * never by the product library).  See tpc_oracle.h for the conventions.
 *
 * The paper (Rohr, "Improvements of the GPU Processing Framework for ALICE")
 * does not spell out the tracking algorithm; it fixes the deterministic-mode
 * contract (Sec. 2: total-order sorting, no FMA, no fast math, IEEE results
 * comparable bit by bit between CPU and GPU) and the workload (TPC sector
 * tracking with cluster-to-track association, Sec. 1-2; track propagation in
 * a magnetic field, Sec. 4).  The algorithm readings implemented here are
 * numbered R1..R30 and listed in the design notes; each function names the
 * readings it follows.
 *
 * Floating point: every expression is evaluated in the order written, in
 * `real`, with no contraction (build flag -ffp-contract=off) and only
 * + - * / sqrt, all of which IEEE-754 rounds correctly.
 */
#include "tpc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "kalman.h"

#define NROWS_MAX ORC_MAX_ROWS
/* R16: rows per propagation step of the walk back to the start row (no
 * updates on the way, so the steps may span several rows) */
#define WALK_ROWS 8

/* ------------------------------------------------------------------------ */
/* derived constants (R3, R9, R11): computed once in binary64 from the inputs */

static real kB_of(const orc_geom* g) { return (real)(-0.299792458e-2 * (double)g->bz); }
static real nf_ivy(const orc_geom* g) { return (real)(1.0 / (1.5 * (double)g->sigma_y2)); }
static real nf_ivz(const orc_geom* g) { return (real)(1.0 / (1.5 * (double)g->sigma_z2)); }

/* ------------------------------------------------------------------------ */
/* R10: bin coordinate of q on one grid axis (monotone in q) */
static int bin_coord(real q, real q0, real iw, int n)
{
  real f = (q - q0) * iw;
  if (!(f > 0)) return 0;
  if (f >= (real)(n - 1)) return n - 1;
  return (int)f;
}

static int axis_bins(real d, real w)
{
  real t = CEIL(d / w);
  if (t < 1) return 1;
  if (t > 65535) return 65535;
  return (int)t;
}

/* validity of an input cluster (bad inputs are counted and ignored) */
static int cluster_valid(const orc_geom* g, const orc_params* P, float y, float z, int row)
{
  if (row >= g->n_rows) return 0;
  real lim = (real)g->row_x[row] * (real)g->tan_half + (real)P->y_valid_margin;
  if (!(FABS((real)y) <= lim)) return 0;
  if (!(FABS((real)z) <= (real)1.0e5)) return 0;
  return 1;
}

/*
 * a1 -- per (instance, row) cluster grid, R10.
 * Row geometry from the data box of the row's valid clusters; every valid
 * cluster goes to bin iz*ny + iy; the instance's valid clusters are ordered
 * by (row, bin, input index) -- a total order (Sec. 2, first compile-time
 * item) -- via a stable counting sort in input order.
 * Returns the number of bin_off entries used, or -1 if bin_cap is too small.
 */
int64_t SFX(orc_grid_build)(const orc_geom* g, const orc_params* P, int32_t n_inst,
                            const int64_t* inst_off, const float* y, const float* z,
                            const uint16_t* row, int32_t* sseg, int32_t* row_off,
                            int32_t* meta_i, real* meta_f, int32_t* bin_off, int64_t bin_cap,
                            int32_t* perm, real* ys, real* zs, int64_t* n_bad)
{
  const int NR = g->n_rows;
  int64_t base = 0;
  int64_t bad = 0;
  for (int i = 0; i < n_inst; i++) {
    int64_t a = inst_off[i], b = inst_off[i + 1];
    int64_t cnt[NROWS_MAX];
    real ymin[NROWS_MAX], ymax[NROWS_MAX], zmin[NROWS_MAX], zmax[NROWS_MAX];
    for (int r = 0; r < NR; r++) cnt[r] = 0;
    for (int64_t c = a; c < b; c++) {
      if (!cluster_valid(g, P, y[c], z[c], row[c])) { bad++; continue; }
      int r = row[c];
      real yc = (real)y[c], zc = (real)z[c];
      if (cnt[r] == 0) { ymin[r] = ymax[r] = yc; zmin[r] = zmax[r] = zc; }
      else {
        if (yc < ymin[r]) ymin[r] = yc;
        if (yc > ymax[r]) ymax[r] = yc;
        if (zc < zmin[r]) zmin[r] = zc;
        if (zc > zmax[r]) zmax[r] = zc;
      }
      cnt[r]++;
    }
    int64_t pos = a;
    const int64_t inst_base = base;
    for (int r = 0; r < NR; r++) {
      int64_t s = (int64_t)i * NR + r;
      int ny = 1, nz = 1;
      real y0 = 0, z0 = 0, iwy = 0, iwz = 0;
      if (cnt[r] > 0) {
        /* one canonical zero: a -0 extreme of the data box becomes +0 */
        real ylo = ymin[r] + (real)0, yhi = ymax[r] + (real)0;
        real zlo = zmin[r] + (real)0, zhi = zmax[r] + (real)0;
        real dy = yhi - ylo, dz = zhi - zlo;
        real nb = FLOOR((real)cnt[r] / (real)P->grid_occupancy);
        if (nb < 1) nb = 1;
        real w = SQRT((dy * dz) / nb);
        if (w < 1) w = 1;
        real m = (dy > dz ? dy : dz) / nb;
        if (w < m) w = m;
        ny = axis_bins(dy, w);
        nz = axis_bins(dz, w);
        iwy = dy > 0 ? (real)ny / dy : 0;
        iwz = dz > 0 ? (real)nz / dz : 0;
        y0 = ylo;
        z0 = zlo;
      }
      meta_i[s * 4 + 0] = ny;
      meta_i[s * 4 + 1] = nz;
      meta_i[s * 4 + 2] = (int32_t)base;
      meta_i[s * 4 + 3] = (int32_t)cnt[r];
      meta_f[s * 4 + 0] = y0;
      meta_f[s * 4 + 1] = z0;
      meta_f[s * 4 + 2] = iwy;
      meta_f[s * 4 + 3] = iwz;
      row_off[(int64_t)i * (NR + 1) + r] = (int32_t)pos;
      int64_t nbins = (int64_t)ny * nz;
      if (base + nbins + 1 > bin_cap) return -1;
      for (int64_t k = 0; k <= nbins; k++) bin_off[base + k] = 0;
      base += nbins + 1;
      pos += cnt[r];
    }
    row_off[(int64_t)i * (NR + 1) + NR] = (int32_t)pos;
    /* bin histogram */
    for (int64_t c = a; c < b; c++) {
      if (!cluster_valid(g, P, y[c], z[c], row[c])) continue;
      int64_t s = (int64_t)i * NR + row[c];
      const int32_t* mi = meta_i + s * 4;
      const real* mf = meta_f + s * 4;
      int iy = bin_coord((real)y[c], mf[0], mf[2], mi[0]);
      int iz = bin_coord((real)z[c], mf[1], mf[3], mi[1]);
      bin_off[mi[2] + (int64_t)iz * mi[0] + iy]++;
    }
    /* exclusive scan per row -> global positions; sentinel = row end */
    for (int r = 0; r < NR; r++) {
      int64_t s = (int64_t)i * NR + r;
      const int32_t* mi = meta_i + s * 4;
      int64_t nbins = (int64_t)mi[0] * mi[1];
      int32_t acc = row_off[(int64_t)i * (NR + 1) + r];
      for (int64_t k = 0; k < nbins; k++) {
        int32_t c = bin_off[mi[2] + k];
        bin_off[mi[2] + k] = acc;
        acc += c;
      }
      bin_off[mi[2] + nbins] = acc;
    }
    /* stable scatter in input order */
    for (int64_t p = a; p < b; p++) { sseg[p] = -1; perm[p] = -1; ys[p] = 0; zs[p] = 0; }
    int32_t* cur = (int32_t*)malloc(sizeof(int32_t) * (size_t)(base - inst_base));
    memcpy(cur, bin_off + inst_base, sizeof(int32_t) * (size_t)(base - inst_base));
    for (int64_t c = a; c < b; c++) {
      if (!cluster_valid(g, P, y[c], z[c], row[c])) continue;
      int64_t s = (int64_t)i * NR + row[c];
      const int32_t* mi = meta_i + s * 4;
      const real* mf = meta_f + s * 4;
      int iy = bin_coord((real)y[c], mf[0], mf[2], mi[0]);
      int iz = bin_coord((real)z[c], mf[1], mf[3], mi[1]);
      int32_t p = cur[mi[2] - inst_base + (int64_t)iz * mi[0] + iy]++;
      sseg[p] = (int32_t)s;
      perm[p] = (int32_t)c;
      ys[p] = (real)y[c];
      zs[p] = (real)z[c];
    }
    free(cur);
  }
  *n_bad = bad;
  return base;
}

/* ------------------------------------------------------------------------ */
/* grid window query: visit the sorted positions of every bin of row segment s
 * that overlaps [qy0,qy1] x [qz0,qz1] */
typedef struct {
  const int32_t* meta_i;
  const real* meta_f;
  const int32_t* bin_off;
  const int32_t* row_off;
  const int32_t* perm;
  const real* ys;
  const real* zs;
  int n_rows;
} gridv;

#define GRID_FOREACH(G, s, qy0, qy1, qz0, qz1, POS, ...)                               \
  do {                                                                                \
    const int32_t* mi_ = (G)->meta_i + (int64_t)(s) * 4;                              \
    const real* mf_ = (G)->meta_f + (int64_t)(s) * 4;                                 \
    int ylo_ = bin_coord((qy0), mf_[0], mf_[2], mi_[0]);                             \
    int yhi_ = bin_coord((qy1), mf_[0], mf_[2], mi_[0]);                             \
    int zlo_ = bin_coord((qz0), mf_[1], mf_[3], mi_[1]);                             \
    int zhi_ = bin_coord((qz1), mf_[1], mf_[3], mi_[1]);                             \
    for (int iz_ = zlo_; iz_ <= zhi_; iz_++) {                                        \
      int64_t b0_ = mi_[2] + (int64_t)iz_ * mi_[0];                                   \
      for (int32_t POS = (G)->bin_off[b0_ + ylo_]; POS < (G)->bin_off[b0_ + yhi_ + 1]; \
           POS++) {                                                                   \
        __VA_ARGS__                                                                   \
      }                                                                               \
    }                                                                                 \
  } while (0)

/*
 * a2 -- NeighboursFinder, R11.  For each cluster h on row r (1 <= r <= n_rows-2)
 * take every pair (u on r+1, d on r-1) inside the |dy| <= nf_win_y,
 * |dz| <= nf_win_z boxes; the midpoint residual of h w.r.t. the straight line
 * d-u gives score = ey^2/(1.5 sy2) + ez^2/(1.5 sz2); keep the pair with the
 * lowest score <= nf_chi2_max, ties broken by (input index of u, input index
 * of d) so that the choice is a total order independent of the grid.
 * brute != 0 scans the whole neighbour rows instead of the grid window.
 */
void SFX(orc_neighbours)(const orc_geom* g, const orc_params* P, int64_t n, const int32_t* sseg,
                         const int32_t* row_off, const int32_t* meta_i, const real* meta_f,
                         const int32_t* bin_off, const int32_t* perm, const real* ys,
                         const real* zs, int32_t* up, int32_t* dn, int brute)
{
  const int NR = g->n_rows;
  gridv G = {meta_i, meta_f, bin_off, row_off, perm, ys, zs, NR};
  real ivy = nf_ivy(g), ivz = nf_ivz(g);
  real wy = (real)P->nf_win_y, wz = (real)P->nf_win_z;
  real wym = wy + (real)P->search_margin, wzm = wz + (real)P->search_margin;
  real cmax = (real)P->nf_chi2_max;
  int32_t* ucand = (int32_t*)malloc(sizeof(int32_t) * 1);
  int32_t* dcand = (int32_t*)malloc(sizeof(int32_t) * 1);
  int64_t ucap = 1, dcap = 1;
  for (int64_t h = 0; h < n; h++) {
    up[h] = -1;
    dn[h] = -1;
    int32_t s = sseg[h];
    if (s < 0) continue;
    int i = s / NR, r = s % NR;
    if (r == 0 || r == NR - 1) continue;
    real yh = ys[h], zh = zs[h];
    int64_t nu = 0, nd = 0;
    for (int side = 0; side < 2; side++) {
      int32_t s2 = s + (side == 0 ? 1 : -1);
      int32_t** lst = side == 0 ? &ucand : &dcand;
      int64_t* cnt = side == 0 ? &nu : &nd;
      int64_t* cap = side == 0 ? &ucap : &dcap;
#define NF_TAKE                                                       \
  if (FABS(ys[pos] - yh) <= wy && FABS(zs[pos] - zh) <= wz) {         \
    if (*cnt == *cap) {                                               \
      *cap *= 2;                                                      \
      *lst = (int32_t*)realloc(*lst, sizeof(int32_t) * (size_t)*cap); \
    }                                                                 \
    (*lst)[(*cnt)++] = pos;                                           \
  }
      if (brute) {
        int r2 = s2 % NR;
        for (int32_t pos = row_off[(int64_t)i * (NR + 1) + r2];
             pos < row_off[(int64_t)i * (NR + 1) + r2 + 1]; pos++) {
          NF_TAKE
        }
      } else {
        GRID_FOREACH(&G, s2, yh - wym, yh + wym, zh - wzm, zh + wzm, pos, NF_TAKE);
      }
#undef NF_TAKE
    }
    if (nu == 0 || nd == 0) continue;
    real xm = (real)g->row_x[r - 1], x0 = (real)g->row_x[r], xp = (real)g->row_x[r + 1];
    real t = (x0 - xm) / (xp - xm);
    int32_t bu = -1, bd = -1;
    real bs = 0;
    for (int64_t a = 0; a < nu; a++) {
      int32_t u = ucand[a];
      for (int64_t b = 0; b < nd; b++) {
        int32_t d = dcand[b];
        real ey = yh - (ys[d] + (ys[u] - ys[d]) * t);
        real ez = zh - (zs[d] + (zs[u] - zs[d]) * t);
        real sc = (ey * ey) * ivy + (ez * ez) * ivz;
        if (!(sc <= cmax)) continue;
        int better = bu < 0 || sc < bs ||
                     (sc == bs && (perm[u] < perm[bu] || (perm[u] == perm[bu] && perm[d] < perm[bd])));
        if (better) { bu = u; bd = d; bs = sc; }
      }
    }
    up[h] = bu;
    dn[h] = bd;
  }
  free(ucand);
  free(dcand);
}

/* a3 -- NeighboursCleaner: keep only mutual links (reads the uncleaned arrays). */
void SFX(orc_clean)(int64_t n, const int32_t* up, const int32_t* dn, int32_t* up2, int32_t* dn2)
{
  for (int64_t h = 0; h < n; h++) {
    int32_t u = up[h], d = dn[h];
    up2[h] = (u >= 0 && dn[u] == h) ? u : -1;
    dn2[h] = (d >= 0 && up[d] == h) ? d : -1;
  }
}

/* a4 -- StartHitsFinder, R12: no cleaned down link and a cleaned up-chain of at
 * least min_chain hits; the list is in ascending sorted position. */
int64_t SFX(orc_start_hits)(const orc_params* P, int64_t n, const int32_t* up2, const int32_t* dn2,
                            int32_t* start)
{
  int64_t S = 0;
  for (int64_t h = 0; h < n; h++) {
    if (dn2[h] != -1 || up2[h] < 0) continue;
    int32_t q = (int32_t)h;
    int len = 1;
    while (len < P->min_chain && up2[q] >= 0) { q = up2[q]; len++; }
    if (len >= P->min_chain) start[S++] = (int32_t)h;
  }
  return S;
}

/* R15: best cluster of row segment s for the predicted state st (chi2 <= pick,
 * ties to the lower input index); -1 if none */
static int32_t k_search(const gridv* G, int32_t s, const kst* st, const kinn* q, real pick,
                        real margin)
{
  real y = st->p[0], z = st->p[1];
  real wy = SQRT(pick * q->S00) + margin;
  real wz = SQRT(pick * q->S11) + margin;
  int32_t best = -1;
  real bchi = 0;
  GRID_FOREACH(G, s, y - wy, y + wy, z - wz, z + wz, pos, {
    real r0 = G->ys[pos] - y, r1 = G->zs[pos] - z;
    real ch = k_chi2(q, r0, r1);
    if (ch <= pick && (best < 0 || ch < bchi || (ch == bchi && G->perm[pos] < G->perm[best]))) {
      best = pos;
      bchi = ch;
    }
  });
  return best;
}

/*
 * a5 -- TrackletConstructor, R13-R19.  One tracklet per start hit, in start
 * list order.  Outputs (per tracklet t):
 *   par[t*5..], cov[t*15..]  state at the innermost hit (R17)
 *   chi2[t], nhit[t], rmin[t], rmax[t]
 *   hit[t*n_rows + r]        sorted position of the hit on row r, -1 if none
 *                            (defined for rmin <= r <= rmax)
 *   status[t]                0 kept, 1 too few hits, 2 back-propagation
 *                            failure, 3 non-finite or negative chi2
 */
void SFX(orc_tracklets)(const orc_geom* g, const orc_params* P, int64_t S, const int32_t* start,
                        const int32_t* up2, const int32_t* sseg, const int32_t* row_off,
                        const int32_t* meta_i, const real* meta_f, const int32_t* bin_off,
                        const int32_t* perm, const real* ys, const real* zs, real* par,
                        real* cov, real* chi2o, int32_t* nhito, int32_t* rmino, int32_t* rmaxo,
                        int32_t* hit, int32_t* status)
{
  const int NR = g->n_rows;
  gridv G = {meta_i, meta_f, bin_off, row_off, perm, ys, zs, NR};
  const real kB = kB_of(g);
  const real vy = (real)g->sigma_y2, vz = (real)g->sigma_z2;
  const real smax = (real)P->snp_max, pick = (real)P->tc_chi2_pick;
  const real margin = (real)P->search_margin, edge = (real)P->edge_margin;
  const real tanh_ = (real)g->tan_half;
  real X[NROWS_MAX];
  for (int r = 0; r < NR; r++) X[r] = (real)g->row_x[r];
  for (int64_t t = 0; t < S; t++) {
    int32_t* H = hit + t * NR;
    for (int r = 0; r < NR; r++) H[r] = -1;
    int32_t h0 = start[t];
    int32_t seg0 = sseg[h0];
    int32_t segbase = seg0 - seg0 % NR;
    int r0 = seg0 % NR;
    int32_t h2 = up2[up2[h0]];
    kst st;
    {
      real dxi = X[r0 + 2] - X[r0];
      real dyi = ys[h2] - ys[h0];
      real dzi = zs[h2] - zs[h0];
      real Li = SQRT(dxi * dxi + dyi * dyi);
      st.p[0] = ys[h0];
      st.p[1] = zs[h0];
      st.p[2] = dyi / Li;
      st.p[3] = dzi / Li;
      st.p[4] = 0;
      k_init_cov(&st, vy, vz);
    }
    real chi2 = 0;
    int n = 1, rmax = r0, rmin = r0, stat = 0;
    H[r0] = h0;
    int r = r0;
    int32_t h = h0;
    int ok_up = 1;
    /* phase 1: follow the cleaned up links, update without a cut (R14) */
    while (up2[h] >= 0) {
      int32_t hn = up2[h];
      if (!k_propagate(&st, X[r], X[r + 1], kB, smax)) { ok_up = 0; break; }
      r++;
      chi2 += k_update(&st, ys[hn], zs[hn], vy, vz);
      H[r] = hn;
      n++;
      rmax = r;
      h = hn;
    }
    kst save = st;
    /* phase 2: extend upward by grid search (R15) */
    if (ok_up) {
      int miss = 0;
      while (r < NR - 1) {
        if (!k_propagate(&st, X[r], X[r + 1], kB, smax)) break;
        r++;
        if (!(FABS(st.p[0]) <= X[r] * tanh_ + edge)) break;
        kinn q = k_innov(&st, vy, vz);
        int32_t b = k_search(&G, segbase + r, &st, &q, pick, margin);
        if (b >= 0) {
          chi2 += k_update(&st, ys[b], zs[b], vy, vz);
          H[r] = b;
          n++;
          rmax = r;
          save = st;
          miss = 0;
        } else {
          H[r] = -1;
          if (++miss >= P->tc_max_miss) break;
        }
      }
    }
    /* phase 3: back down to the start row without updates, in steps of at
     * most WALK_ROWS rows, then extend downward (R16); the output state is
     * the one at the innermost hit */
    st = save;
    r = rmax;
    while (r > r0) {
      int rn = r - WALK_ROWS > r0 ? r - WALK_ROWS : r0;
      if (!k_propagate(&st, X[r], X[rn], kB, smax)) { stat = 2; break; }
      r = rn;
    }
    kst out = st;
    if (stat == 0) {
      int miss = 0;
      while (r > 0) {
        if (!k_propagate(&st, X[r], X[r - 1], kB, smax)) break;
        r--;
        if (!(FABS(st.p[0]) <= X[r] * tanh_ + edge)) break;
        kinn q = k_innov(&st, vy, vz);
        int32_t b = k_search(&G, segbase + r, &st, &q, pick, margin);
        if (b >= 0) {
          chi2 += k_update(&st, ys[b], zs[b], vy, vz);
          H[r] = b;
          n++;
          rmin = r;
          out = st;
          miss = 0;
        } else {
          H[r] = -1;
          if (++miss >= P->tc_max_miss) break;
        }
      }
      if (n < P->min_tracklet_hits) stat = 1;
      else if (!(chi2 >= 0 && chi2 <= (real)3.0e38)) stat = 3;
    }
    for (int k = 0; k < 5; k++) par[t * 5 + k] = out.p[k];
    for (int k = 0; k < 15; k++) cov[t * 15 + k] = out.c[k];
    chi2o[t] = chi2;
    nhito[t] = n;
    rmino[t] = rmin;
    rmaxo[t] = rmax;
    status[t] = stat;
  }
}

/* ------------------------------------------------------------------------ */
/* a6 -- TrackletSelector, R20.  key = (nhit, smaller chi2, smaller
 * instance-local input index of the start hit: independent of the grid);
 * each hit is owned by the kept tracklet
 * with the largest key; a tracklet owning >= min_track_hits hits becomes a
 * track.  Tracks are emitted in tracklet order with their owned hits in
 * ascending row order (input indices); clu2trk[input index] = track or -1. */
static uint64_t ts_key(int32_t nhit, real chi2, int64_t lid)
{
  float c = (float)chi2;
  uint32_t bits;
  memcpy(&bits, &c, 4);
  return ((uint64_t)(uint32_t)nhit << 56) | ((uint64_t)(~bits & 0x7FFFFFFFu) << 25) |
         (uint64_t)(0x1FFFFFFu - (uint64_t)lid);
}

int64_t SFX(orc_select)(const orc_geom* g, const orc_params* P, int64_t n, int64_t S,
                        const int64_t* inst_off, const int32_t* start, const int32_t* sseg,
                        const int32_t* perm, const real* par, const real* cov, const real* chi2,
                        const int32_t* nhit, const int32_t* rmin, const int32_t* rmax,
                        const int32_t* hit, const int32_t* status, uint64_t* owner,
                        int64_t cap_tracks, int64_t cap_hits, real* tpar, real* tcov,
                        real* tchi2, int32_t* tndf, float* txref, int32_t* thit_off,
                        int32_t* thit_clu, int32_t* clu2trk, int64_t* n_hits_out,
                        int64_t* need_tracks, int64_t* need_hits)
{
  const int NR = g->n_rows;
  for (int64_t h = 0; h < n; h++) owner[h] = 0;
  uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(S > 0 ? S : 1));
  for (int64_t t = 0; t < S; t++) {
    keys[t] = 0;
    if (status[t] != 0) continue;
    int32_t s0 = sseg[start[t]];
    int64_t lid = perm[start[t]] - inst_off[s0 / NR];
    keys[t] = ts_key(nhit[t], chi2[t], lid);
    for (int r = rmin[t]; r <= rmax[t]; r++) {
      int32_t h = hit[t * NR + r];
      if (h >= 0 && keys[t] > owner[h]) owner[h] = keys[t];
    }
  }
  for (int64_t c = 0; c < n; c++) clu2trk[c] = -1;
  int64_t nt = 0, nh = 0, wt = 0, wh = 0;
  int full = 0;
  if (cap_tracks >= 0) thit_off[0] = 0;
  for (int64_t t = 0; t < S; t++) {
    if (status[t] != 0) continue;
    int own = 0;
    for (int r = rmin[t]; r <= rmax[t]; r++) {
      int32_t h = hit[t * NR + r];
      if (h >= 0 && owner[h] == keys[t]) own++;
    }
    if (own < P->min_track_hits) continue;
    if (!full && nt < cap_tracks && nh + own <= cap_hits) {
      for (int k = 0; k < 5; k++) tpar[nt * 5 + k] = par[t * 5 + k];
      for (int k = 0; k < 15; k++) tcov[nt * 15 + k] = cov[t * 15 + k];
      tchi2[nt] = chi2[t];
      tndf[nt] = 2 * nhit[t] - 5;
      txref[nt] = g->row_x[rmin[t]];
      int64_t j = nh;
      for (int r = rmin[t]; r <= rmax[t]; r++) {
        int32_t h = hit[t * NR + r];
        if (h >= 0 && owner[h] == keys[t]) {
          thit_clu[j++] = perm[h];
          clu2trk[perm[h]] = (int32_t)nt;
        }
      }
      thit_off[nt + 1] = (int32_t)(nh + own);
      wt = nt + 1;
      wh = nh + own;
    } else {
      full = 1;
    }
    nt++;
    nh += own;
  }
  free(keys);
  *n_hits_out = wh;
  *need_tracks = nt;
  *need_hits = nh;
  return wt;
}

/* Replay of a tracklet's filter sequence on a fixed hit list (used to give
 * the binary64 reference of the parameters of any fitted hit list, R30):
 * init at r0 from the hits on r0 and r0+2, update upward at every row with a
 * hit up to rmax, propagate back to r0, then update downward to rmin.
 * hy/hz/has are indexed by row.  Returns 0 on a propagation failure. */
int SFX(orc_replay)(const orc_geom* g, const orc_params* P, int r0, int rmin, int rmax,
                    const float* hy, const float* hz, const uint8_t* has, real* par, real* cov,
                    real* chi2o)
{
  const real kB = kB_of(g);
  const real vy = (real)g->sigma_y2, vz = (real)g->sigma_z2;
  const real smax = (real)P->snp_max;
  real X[NROWS_MAX];
  for (int r = 0; r < g->n_rows; r++) X[r] = (real)g->row_x[r];
  kst st;
  real dxi = X[r0 + 2] - X[r0];
  real dyi = (real)hy[r0 + 2] - (real)hy[r0];
  real dzi = (real)hz[r0 + 2] - (real)hz[r0];
  real Li = SQRT(dxi * dxi + dyi * dyi);
  st.p[0] = (real)hy[r0];
  st.p[1] = (real)hz[r0];
  st.p[2] = dyi / Li;
  st.p[3] = dzi / Li;
  st.p[4] = 0;
  k_init_cov(&st, vy, vz);
  real chi2 = 0;
  for (int r = r0 + 1; r <= rmax; r++) {
    if (!k_propagate(&st, X[r - 1], X[r], kB, smax)) return 0;
    if (has[r]) chi2 += k_update(&st, (real)hy[r], (real)hz[r], vy, vz);
  }
  for (int r = rmax; r > r0;) {
    int rn = r - WALK_ROWS > r0 ? r - WALK_ROWS : r0;
    if (!k_propagate(&st, X[r], X[rn], kB, smax)) return 0;
    r = rn;
  }
  kst out = st;
  for (int r = r0 - 1; r >= rmin; r--) {
    if (!k_propagate(&st, X[r + 1], X[r], kB, smax)) return 0;
    if (has[r]) {
      chi2 += k_update(&st, (real)hy[r], (real)hz[r], vy, vz);
      out = st;
    }
  }
  for (int k = 0; k < 5; k++) par[k] = out.p[k];
  for (int k = 0; k < 15; k++) cov[k] = out.c[k];
  *chi2o = chi2;
  return 1;
}

/* Bare propagation + update helpers exposed for the closed-form pins. */
int SFX(orc_propagate)(const orc_geom* g, const orc_params* P, real* p, real* c, real x1, real x2)
{
  kst s;
  memcpy(s.p, p, sizeof(s.p));
  memcpy(s.c, c, sizeof(s.c));
  int ok = k_propagate(&s, x1, x2, kB_of(g), (real)P->snp_max);
  memcpy(p, s.p, sizeof(s.p));
  memcpy(c, s.c, sizeof(s.c));
  return ok;
}

real SFX(orc_update)(const orc_geom* g, real* p, real* c, real my, real mz)
{
  kst s;
  memcpy(s.p, p, sizeof(s.p));
  memcpy(s.c, c, sizeof(s.c));
  real chi2 = k_update(&s, my, mz, (real)g->sigma_y2, (real)g->sigma_z2);
  memcpy(p, s.p, sizeof(s.p));
  memcpy(c, s.c, sizeof(s.c));
  return chi2;
}

#if !defined(ORC_F64) && !defined(ORC_F32C)
#include <fenv.h>
/* R29 check: whether an operation since the last clear delivered a tiny
 * (subnormal or flushed) inexact result -- the IEEE underflow flag of the
 * calling thread.  clear != 0 resets the flag after reading it. */
int orc_underflow_raised(int clear)
{
  const int r = fetestexcept(FE_UNDERFLOW) != 0;
  if (clear) feclearexcept(FE_UNDERFLOW);
  return r;
}
#endif
