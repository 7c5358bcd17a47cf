/*
 * Eikonal oracle -- TEST INFRASTRUCTURE ONLY (see eik_oracle.h).
 *
 * Every routine here is the plain serial form of a method in Chacon &
 * Vladimirsky, "Fast two-scale methods for Eikonal equations"; each cites the
 * section, equation or algorithm it follows.  Build with -ffp-contract=off so
 * that no multiply-add is fused.  Readings of passages where the paper is
 * silent are marked READING and listed with their justification in the
 * design notes of the repository.
 */
#include "eik_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define INF HUGE_VAL

/* ------------------------------------------------------------------------ */
/* Problem set-up                                                           */
/* ------------------------------------------------------------------------ */

typedef struct {
  int nx, ny;
  long n;
  double h;
  const double* F;
  double* delta;        /* h / F at every accessible node                    */
  unsigned char* acc;   /* 1 = accessible                                    */
  unsigned char* src;   /* 1 = node of the exit set Q (kept fixed at q)      */
  double* qv;           /* q at sources (min over duplicates)                */
} grid_t;

static void grid_free(grid_t* g) {
  free(g->delta);
  free(g->acc);
  free(g->src);
  free(g->qv);
  memset(g, 0, sizeof *g);
}

/* Validates the boundary-value problem of the introduction (|grad u| F = 1,
   u = q on Q, state constraint elsewhere on the boundary). */
static int grid_init(grid_t* g, const orc_problem* p) {
  memset(g, 0, sizeof *g);
  if (!p || p->nx < 1 || p->ny < 1 || !(p->h > 0.0) || !isfinite(p->h) || !p->F ||
      p->nsrc < 1 || !p->src)
    return -1;
  g->nx = p->nx;
  g->ny = p->ny;
  g->n = (long)p->nx * (long)p->ny;
  g->h = p->h;
  g->F = p->F;
  g->delta = (double*)malloc(sizeof(double) * g->n);
  g->acc = (unsigned char*)malloc(g->n);
  g->src = (unsigned char*)calloc(g->n, 1);
  g->qv = (double*)malloc(sizeof(double) * g->n);
  if (!g->delta || !g->acc || !g->src || !g->qv) {
    grid_free(g);
    return -2;
  }
  for (long k = 0; k < g->n; ++k) {
    g->acc[k] = p->mask ? (p->mask[k] != 0) : 1;
    g->qv[k] = INF;
    if (g->acc[k]) {
      double f = p->F[k];
      if (!(f > 0.0) || !isfinite(f)) {
        grid_free(g);
        return -1;
      }
      g->delta[k] = p->h / f;
    } else {
      g->delta[k] = INF;
    }
  }
  for (int s = 0; s < p->nsrc; ++s) {
    long k = (long)p->src[s];
    double q = p->q ? p->q[s] : 0.0;
    if (k < 0 || k >= g->n || !g->acc[k] || !isfinite(q)) {
      grid_free(g);
      return -1;
    }
    g->src[k] = 1;
    if (q < g->qv[k]) g->qv[k] = q;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Local update (Section 2: upwind discretisation, one- and two-sided        */
/* updates, and the remark that only min(U_S,U_N), min(U_E,U_W) matter)      */
/* ------------------------------------------------------------------------ */

/* The two-sided quadrant root U >= max(a, b) of
   ((U-a)/h)^2 + ((U-b)/h)^2 = 1/F^2 exists iff |a-b| <= delta = h/F; at
   equality it coincides with the one-sided value min(a,b) + delta, so the
   one-sided branch is taken for |a-b| >= delta.  Infinite inputs never meet
   in a subtraction.  Expression order is fixed (READING). */
double orc_update(double a, double b, double delta) {
  double lo = a < b ? a : b;
  if (lo == INF) return INF;
  double d = a - b;
  if (fabs(d) >= delta) return lo + delta;
  return 0.5 * (a + b + sqrt(2.0 * delta * delta - d * d));
}

static double nb(const grid_t* g, const double* V, int i, int j) {
  if (i < 0 || j < 0 || i >= g->nx || j >= g->ny) return INF;
  return V[(long)j * g->nx + i];
}

/* Temporary value of node (i,j) from its four neighbours (eq. Eik_discr);
   outside-grid and obstacle neighbours count as +inf. */
static double node_update(const grid_t* g, const double* V, int i, int j) {
  double uW = nb(g, V, i - 1, j), uE = nb(g, V, i + 1, j);
  double uS = nb(g, V, i, j - 1), uN = nb(g, V, i, j + 1);
  double a = uW < uE ? uW : uE;
  double b = uS < uN ? uS : uN;
  return orc_update(a, b, g->delta[(long)j * g->nx + i]);
}

static void init_values(const grid_t* g, double* V) {
  for (long k = 0; k < g->n; ++k) V[k] = g->src[k] ? g->qv[k] : INF;
}

/* ------------------------------------------------------------------------ */
/* Binary heap keyed by (key, index), with positions for decrease-key        */
/* ------------------------------------------------------------------------ */

typedef struct {
  long* a;
  long* pos; /* -1 when absent */
  long n;
  const double* key;
} heap_t;

static int heap_less(const heap_t* H, long x, long y) {
  double kx = H->key[x], ky = H->key[y];
  return kx < ky || (kx == ky && x < y);
}

static void heap_swap(heap_t* H, long i, long j) {
  long t = H->a[i];
  H->a[i] = H->a[j];
  H->a[j] = t;
  H->pos[H->a[i]] = i;
  H->pos[H->a[j]] = j;
}

static void heap_up(heap_t* H, long i) {
  while (i > 0) {
    long p = (i - 1) / 2;
    if (!heap_less(H, H->a[i], H->a[p])) break;
    heap_swap(H, i, p);
    i = p;
  }
}

static void heap_down(heap_t* H, long i) {
  for (;;) {
    long l = 2 * i + 1, r = l + 1, m = i;
    if (l < H->n && heap_less(H, H->a[l], H->a[m])) m = l;
    if (r < H->n && heap_less(H, H->a[r], H->a[m])) m = r;
    if (m == i) break;
    heap_swap(H, i, m);
    i = m;
  }
}

static void heap_push(heap_t* H, long x) {
  H->a[H->n] = x;
  H->pos[x] = H->n;
  H->n++;
  heap_up(H, H->n - 1);
}

static long heap_pop(heap_t* H) {
  long x = H->a[0];
  H->n--;
  if (H->n > 0) {
    H->a[0] = H->a[H->n];
    H->pos[H->a[0]] = 0;
    heap_down(H, 0);
  }
  H->pos[x] = -1;
  return x;
}

static int heap_init(heap_t* H, long cap, const double* key) {
  H->a = (long*)malloc(sizeof(long) * (cap > 0 ? cap : 1));
  H->pos = (long*)malloc(sizeof(long) * (cap > 0 ? cap : 1));
  H->n = 0;
  H->key = key;
  if (!H->a || !H->pos) {
    free(H->a);
    free(H->pos);
    return -2;
  }
  for (long k = 0; k < cap; ++k) H->pos[k] = -1;
  return 0;
}

static void heap_free(heap_t* H) {
  free(H->a);
  free(H->pos);
}

/* ------------------------------------------------------------------------ */
/* Fast Marching (Algorithm FMM)                                             */
/* ------------------------------------------------------------------------ */

enum { FAR = 0, CONSIDERED = 1, ACCEPTED = 2 };

static int fmm_grid(const grid_t* g, double* V, int64_t* order, int64_t* nacc) {
  unsigned char* lab = (unsigned char*)calloc(g->n, 1);
  long* srcs = (long*)malloc(sizeof(long) * g->n);
  heap_t H;
  if (!lab || !srcs || heap_init(&H, g->n, V)) {
    free(lab);
    free(srcs);
    return -2;
  }
  init_values(g, V);
  long ns = 0, na = 0;
  /* Initialisation: Q is Accepted (in (q, index) order, READING), its Far
     neighbours become Considered with a temporary value. */
  {
    heap_t Q;
    if (heap_init(&Q, g->n, g->qv)) {
      free(lab);
      free(srcs);
      heap_free(&H);
      return -2;
    }
    for (long k = 0; k < g->n; ++k)
      if (g->src[k]) heap_push(&Q, k);
    while (Q.n > 0) srcs[ns++] = heap_pop(&Q);
    heap_free(&Q);
  }
  for (long s = 0; s < ns; ++s) {
    lab[srcs[s]] = ACCEPTED;
    if (order) order[na] = srcs[s];
    na++;
  }
  static const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
  for (long s = 0; s < ns; ++s) {
    long k = srcs[s];
    int i = (int)(k % g->nx), j = (int)(k / g->nx);
    for (int e = 0; e < 4; ++e) {
      int ii = i + di[e], jj = j + dj[e];
      if (ii < 0 || jj < 0 || ii >= g->nx || jj >= g->ny) continue;
      long kk = (long)jj * g->nx + ii;
      if (!g->acc[kk] || lab[kk] == ACCEPTED) continue;
      double t = node_update(g, V, ii, jj);
      if (t < V[kk]) V[kk] = t;
      if (lab[kk] == FAR) {
        lab[kk] = CONSIDERED;
        heap_push(&H, kk);
      } else {
        heap_up(&H, H.pos[kk]);
      }
    }
  }
  /* Main loop: accept the smallest Considered node, update its neighbours. */
  while (H.n > 0) {
    long k = heap_pop(&H);
    lab[k] = ACCEPTED;
    if (order) order[na] = k;
    na++;
    int i = (int)(k % g->nx), j = (int)(k / g->nx);
    for (int e = 0; e < 4; ++e) {
      int ii = i + di[e], jj = j + dj[e];
      if (ii < 0 || jj < 0 || ii >= g->nx || jj >= g->ny) continue;
      long kk = (long)jj * g->nx + ii;
      if (!g->acc[kk] || lab[kk] == ACCEPTED) continue;
      double t = node_update(g, V, ii, jj);
      if (t < V[kk]) V[kk] = t;
      if (lab[kk] == FAR) {
        lab[kk] = CONSIDERED;
        heap_push(&H, kk);
      } else {
        heap_up(&H, H.pos[kk]);
      }
    }
  }
  if (nacc) *nacc = na;
  free(lab);
  free(srcs);
  heap_free(&H);
  return 0;
}

int orc_fmm(const orc_problem* p, double* V, int64_t* order, int64_t* nacc) {
  grid_t g;
  int rc = grid_init(&g, p);
  if (rc) return rc;
  rc = fmm_grid(&g, V, order, nacc);
  grid_free(&g);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Fast Sweeping (Algorithms FSM_order and FSM) and Locking Sweeping         */
/* ------------------------------------------------------------------------ */

/* Sweep direction d = sweepNumber mod 4: 0 i,j ascending (from SW);
   1 i ascending, j descending (NW); 2 both descending (NE); 3 i descending,
   j ascending (SE).  i (the x index) is the outer loop. */
static void dir_steps(int d, int* sx, int* sy) {
  *sx = (d == 0 || d == 1) ? 1 : -1;
  *sy = (d == 0 || d == 3) ? 1 : -1;
}

/* One Gauss-Seidel sweep in direction d over the node box [x0,x1)x[y0,y1);
   neighbours outside the box are read from V as they stand (the box's halo).
   directional = 1 uses only the two upwind neighbours of the sweep (the
   sweep-directional update of FMSM); otherwise the quadrant shortcut. */
static int sweep_box(const grid_t* g, double* V, int d, int x0, int x1, int y0,
                     int y1, int directional) {
  int sx, sy, changed = 0;
  dir_steps(d, &sx, &sy);
  for (int ii = 0; ii < x1 - x0; ++ii) {
    int i = sx > 0 ? x0 + ii : x1 - 1 - ii;
    for (int jj = 0; jj < y1 - y0; ++jj) {
      int j = sy > 0 ? y0 + jj : y1 - 1 - jj;
      long k = (long)j * g->nx + i;
      if (!g->acc[k] || g->src[k]) continue;
      double t;
      if (directional)
        t = orc_update(nb(g, V, i - sx, j), nb(g, V, i, j - sy), g->delta[k]);
      else
        t = node_update(g, V, i, j);
      if (t < V[k]) {
        V[k] = t;
        changed = 1;
      }
    }
  }
  return changed;
}

/* Change record of one sweep: largest decrease (+inf when a node leaves
   +inf) and number of nodes that decreased. */
static void note_change(double before, double after, double* mx, int64_t* cnt) {
  if (!(after < before)) return;
  double d = before == INF ? INF : before - after;
  if (d > *mx) *mx = d;
  (*cnt)++;
}

int orc_fsm_sweep(const orc_problem* p, double* V, int32_t sweep, double* max_change,
                  int64_t* n_changed) {
  grid_t g;
  int rc = grid_init(&g, p);
  if (rc) return rc;
  int sx, sy;
  double mx = 0.0;
  int64_t cnt = 0;
  dir_steps(sweep % 4, &sx, &sy);
  for (int ii = 0; ii < g.nx; ++ii) {
    int i = sx > 0 ? ii : g.nx - 1 - ii;
    for (int jj = 0; jj < g.ny; ++jj) {
      int j = sy > 0 ? jj : g.ny - 1 - jj;
      long k = (long)j * g.nx + i;
      if (!g.acc[k] || g.src[k]) continue;
      double t = node_update(&g, V, i, j);
      if (t < V[k]) {
        note_change(V[k], t, &mx, &cnt);
        V[k] = t;
      }
    }
  }
  if (max_change) *max_change = mx;
  if (n_changed) *n_changed = cnt;
  grid_free(&g);
  return 0;
}

int orc_fsm(const orc_problem* p, double* V, int32_t* nsweeps) {
  grid_t g;
  int rc = grid_init(&g, p);
  if (rc) return rc;
  init_values(&g, V);
  int sweep = 0, changed;
  do {
    changed = sweep_box(&g, V, sweep % 4, 0, g.nx, 0, g.ny, 0);
    sweep++;
  } while (changed);
  if (nsweeps) *nsweeps = sweep;
  grid_free(&g);
  return 0;
}

/* LSM sweep over a box: visit unlocked nodes only; a node that decreases
   unlocks its larger neighbours inside the box; every visited node is locked
   (Section 2, remark on locking flags). */
static int lsm_sweep_box(const grid_t* g, double* V, unsigned char* unl, int d,
                         int x0, int x1, int y0, int y1) {
  int sx, sy, changed = 0;
  static const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
  dir_steps(d, &sx, &sy);
  for (int ii = 0; ii < x1 - x0; ++ii) {
    int i = sx > 0 ? x0 + ii : x1 - 1 - ii;
    for (int jj = 0; jj < y1 - y0; ++jj) {
      int j = sy > 0 ? y0 + jj : y1 - 1 - jj;
      long k = (long)j * g->nx + i;
      if (!unl[k]) continue;
      unl[k] = 0;
      double t = node_update(g, V, i, j);
      if (t < V[k]) {
        V[k] = t;
        changed = 1;
        for (int e = 0; e < 4; ++e) {
          int a = i + di[e], b = j + dj[e];
          if (a < x0 || b < y0 || a >= x1 || b >= y1) continue;
          long kk = (long)b * g->nx + a;
          if (g->acc[kk] && !g->src[kk] && V[kk] > V[k]) unl[kk] = 1;
        }
      }
    }
  }
  return changed;
}

/* Locking Sweeping's start: the accessible non-exit neighbours of exit
   nodes are unlocked, every other node locked. */
static void lsm_unlock_init(const grid_t* g, unsigned char* unl) {
  static const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
  if (g->n > 0) memset(unl, 0, (size_t)g->n);
  for (long k = 0; k < g->n; ++k) {
    if (!g->src[k]) continue;
    int i = (int)(k % g->nx), j = (int)(k / g->nx);
    for (int e = 0; e < 4; ++e) {
      int a = i + di[e], b = j + dj[e];
      if (a < 0 || b < 0 || a >= g->nx || b >= g->ny) continue;
      long kk = (long)b * g->nx + a;
      if (g->acc[kk] && !g->src[kk]) unl[kk] = 1;
    }
  }
}

int orc_sweep_init(const orc_problem* p, double* V, uint8_t* unlocked) {
  grid_t g;
  int rc = grid_init(&g, p);
  if (rc) return rc;
  init_values(&g, V);
  if (unlocked) lsm_unlock_init(&g, unlocked);
  grid_free(&g);
  return 0;
}

int orc_lsm_sweep(const orc_problem* p, double* V, uint8_t* unlocked, int32_t sweep,
                  double* max_change, int64_t* n_changed) {
  grid_t g;
  int rc = grid_init(&g, p);
  if (rc) return rc;
  static const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
  int sx, sy;
  double mx = 0.0;
  int64_t cnt = 0;
  dir_steps(sweep % 4, &sx, &sy);
  for (int ii = 0; ii < g.nx; ++ii) {
    int i = sx > 0 ? ii : g.nx - 1 - ii;
    for (int jj = 0; jj < g.ny; ++jj) {
      int j = sy > 0 ? jj : g.ny - 1 - jj;
      long k = (long)j * g.nx + i;
      if (!unlocked[k]) continue;
      unlocked[k] = 0;
      double t = node_update(&g, V, i, j);
      if (t < V[k]) {
        note_change(V[k], t, &mx, &cnt);
        V[k] = t;
        for (int e = 0; e < 4; ++e) {
          int a = i + di[e], b = j + dj[e];
          if (a < 0 || b < 0 || a >= g.nx || b >= g.ny) continue;
          long kk = (long)b * g.nx + a;
          if (g.acc[kk] && !g.src[kk] && V[kk] > V[k]) unlocked[kk] = 1;
        }
      }
    }
  }
  if (max_change) *max_change = mx;
  if (n_changed) *n_changed = cnt;
  grid_free(&g);
  return 0;
}

int orc_lsm(const orc_problem* p, double* V, int32_t* nsweeps) {
  grid_t g;
  int rc = grid_init(&g, p);
  if (rc) return rc;
  unsigned char* unl = (unsigned char*)calloc(g.n, 1);
  if (!unl) {
    grid_free(&g);
    return -2;
  }
  init_values(&g, V);
  static const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
  /* all nodes but those adjacent to Q start locked */
  for (long k = 0; k < g.n; ++k) {
    if (!g.src[k]) continue;
    int i = (int)(k % g.nx), j = (int)(k / g.nx);
    for (int e = 0; e < 4; ++e) {
      int a = i + di[e], b = j + dj[e];
      if (a < 0 || b < 0 || a >= g.nx || b >= g.ny) continue;
      long kk = (long)b * g.nx + a;
      if (g.acc[kk] && !g.src[kk]) unl[kk] = 1;
    }
  }
  int sweep = 0, changed;
  do {
    changed = lsm_sweep_box(&g, V, unl, sweep % 4, 0, g.nx, 0, g.ny);
    sweep++;
  } while (changed);
  if (nsweeps) *nsweeps = sweep;
  free(unl);
  grid_free(&g);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Value iteration (Section 1 on graphs, applied to eq. Eik_discr) and the   */
/* fixed-point residual                                                     */
/* ------------------------------------------------------------------------ */

int orc_jacobi(const orc_problem* p, double* V, int32_t* niters) {
  grid_t g;
  int rc = grid_init(&g, p);
  if (rc) return rc;
  double* W = (double*)malloc(sizeof(double) * g.n);
  if (!W) {
    grid_free(&g);
    return -2;
  }
  init_values(&g, V);
  int it = 0, changed;
  do {
    changed = 0;
    for (int j = 0; j < g.ny; ++j)
      for (int i = 0; i < g.nx; ++i) {
        long k = (long)j * g.nx + i;
        W[k] = V[k];
        if (!g.acc[k] || g.src[k]) continue;
        double t = node_update(&g, V, i, j);
        if (t < V[k]) {
          W[k] = t;
          changed = 1;
        }
      }
    memcpy(V, W, sizeof(double) * g.n);
    it++;
  } while (changed);
  if (niters) *niters = it;
  free(W);
  grid_free(&g);
  return 0;
}

double orc_residual(const orc_problem* p, const double* V, double* r) {
  grid_t g;
  if (grid_init(&g, p)) return -1.0;
  double mx = 0.0;
  for (int j = 0; j < g.ny; ++j)
    for (int i = 0; i < g.nx; ++i) {
      long k = (long)j * g.nx + i;
      double rk = 0.0;
      if (g.acc[k] && !g.src[k]) {
        double t = node_update(&g, V, i, j);
        if (V[k] == INF)
          rk = (t == INF) ? 0.0 : INF;
        else
          rk = fabs(t - V[k]) / V[k];
      }
      if (r) r[k] = rk;
      if (rk > mx) mx = rk;
    }
  grid_free(&g);
  return mx;
}

/* ------------------------------------------------------------------------ */
/* Cells                                                                    */
/* ------------------------------------------------------------------------ */

/* READING: K = ceil(n/s) cells per axis, cell k = [k s, min((k+1) s, n));
   a last cell that would be one node wide is merged into its predecessor. */
int32_t orc_tiling(int32_t n, int32_t s, int32_t* lo) {
  if (n < 1 || s < 1) return 0;
  int32_t K = (n + s - 1) / s;
  if (K > 1 && n % s == 1) K--;
  if (lo) {
    for (int32_t k = 0; k < K; ++k) lo[k] = k * s;
    lo[K] = n;
  }
  return K;
}

typedef struct {
  int Kx, Ky;
  long J;
  int32_t* xl; /* Kx+1 */
  int32_t* yl; /* Ky+1 */
} cells_t;

static int cells_init(cells_t* C, const grid_t* g, int s) {
  C->Kx = orc_tiling(g->nx, s, NULL);
  C->Ky = orc_tiling(g->ny, s, NULL);
  C->J = (long)C->Kx * C->Ky;
  C->xl = (int32_t*)malloc(sizeof(int32_t) * (C->Kx + 1));
  C->yl = (int32_t*)malloc(sizeof(int32_t) * (C->Ky + 1));
  if (!C->xl || !C->yl) {
    free(C->xl);
    free(C->yl);
    return -2;
  }
  orc_tiling(g->nx, s, C->xl);
  orc_tiling(g->ny, s, C->yl);
  return 0;
}

static void cells_free(cells_t* C) {
  free(C->xl);
  free(C->yl);
}

/* Sides of a cell: 0 W, 1 E, 2 S, 3 N.  Direction bits: 0 SW, 1 NW, 2 NE,
   3 SE.  A neighbour on side W (resp. E, S, N) that influences a cell calls
   for the sweeps that start on that side: SW+NW (NE+SE, SW+SE, NW+NE). */
static const int side_dirs[4] = {(1 << 0) | (1 << 1), (1 << 2) | (1 << 3),
                                 (1 << 0) | (1 << 3), (1 << 1) | (1 << 2)};
/* The side of the neighbour cell facing back towards us. */
static const int opposite[4] = {1, 0, 3, 2};

static long cell_nbr(const cells_t* C, long c, int side) {
  int cx = (int)(c % C->Kx), cy = (int)(c / C->Kx);
  if (side == 0) cx--;
  if (side == 1) cx++;
  if (side == 2) cy--;
  if (side == 3) cy++;
  if (cx < 0 || cy < 0 || cx >= C->Kx || cy >= C->Ky) return -1;
  return (long)cy * C->Kx + cx;
}

static void cell_box(const cells_t* C, long c, int* x0, int* x1, int* y0, int* y1) {
  int cx = (int)(c % C->Kx), cy = (int)(c / C->Kx);
  *x0 = C->xl[cx];
  *x1 = C->xl[cx + 1];
  *y0 = C->yl[cy];
  *y1 = C->yl[cy + 1];
}

/* Pairs (x_i in c on `side`, x_j across it): the t-th pair, t < len. */
static void side_pair(const cells_t* C, const grid_t* g, long c, int side, int t,
                      long* ki, long* kj) {
  int x0, x1, y0, y1;
  cell_box(C, c, &x0, &x1, &y0, &y1);
  int i, j, oi = 0, oj = 0;
  if (side == 0) { i = x0; j = y0 + t; oi = -1; }
  else if (side == 1) { i = x1 - 1; j = y0 + t; oi = 1; }
  else if (side == 2) { i = x0 + t; j = y0; oj = -1; }
  else { i = x0 + t; j = y1 - 1; oj = 1; }
  *ki = (long)j * g->nx + i;
  *kj = (long)(j + oj) * g->nx + (i + oi);
}

static int side_len(const cells_t* C, long c, int side) {
  int x0, x1, y0, y1;
  cell_box(C, c, &x0, &x1, &y0, &y1);
  return (side <= 1) ? (y1 - y0) : (x1 - x0);
}

/* Eq. cell_value: with x_i the largest finite value on c's side line facing
   c_k and y_i the point (1 + w_k)/2 nodes beyond x_i towards c_k (w_k = c_k's
   width across that side, so y_i lies on c_k's centre line), the estimate is
   V_i + ((1 + w_k)/2) h / F(y_i).  READING: F(y_i) is the node value at an
   integer offset and the mean of the two straddling accessible nodes at a
   half-integer one; no finite value or no accessible node => no estimate. */
static int cell_value_estimate(const cells_t* C, const grid_t* g, const double* V,
                               long c, int side, long ck, double* est) {
  int len = side_len(C, c, side);
  double vmax = -INF;
  long kmax = -1;
  for (int t = 0; t < len; ++t) {
    long ki, kj;
    side_pair(C, g, c, side, t, &ki, &kj);
    if (V[ki] != INF && (kmax < 0 || V[ki] > vmax)) {
      vmax = V[ki];
      kmax = ki;
    }
  }
  if (kmax < 0) return 0;
  int xk0, xk1, yk0, yk1;
  cell_box(C, ck, &xk0, &xk1, &yk0, &yk1);
  int wk = (side <= 1) ? (xk1 - xk0) : (yk1 - yk0);
  int i = (int)(kmax % g->nx), j = (int)(kmax / g->nx);
  int dir = (side == 1 || side == 3) ? 1 : -1;
  int along = (side <= 1) ? i : j;
  /* twice the position of y_i along the axis */
  int twice = 2 * along + dir * (1 + wk);
  int na = 0, nbk = 0;
  int pa[2];
  if (twice % 2 == 0) {
    pa[na++] = twice / 2;
  } else {
    int lo = (twice - 1) / 2; /* exact: twice - 1 is even */
    pa[na++] = lo;
    pa[na++] = lo + 1;
  }
  double fs = 0.0;
  for (int m = 0; m < na; ++m) {
    int ii = (side <= 1) ? pa[m] : i, jj = (side <= 1) ? j : pa[m];
    if (ii < 0 || jj < 0 || ii >= g->nx || jj >= g->ny) continue;
    long kk = (long)jj * g->nx + ii;
    if (!g->acc[kk]) continue;
    fs += g->F[kk];
    nbk++;
  }
  if (nbk == 0) return 0;
  double fy = fs / nbk;
  *est = vmax + (0.5 * (1 + wk) * g->h) / fy;
  return 1;
}

/* FHCM monotonicity check on c's side line facing the neighbour (finite
   values only).  Along the line ordered N->S for W/E sides and W->E for S/N
   sides: non-decreasing selects one sweep, non-increasing the other, a
   constant line counts as monotone and keeps both (READING). */
static int monotone_dirs(const cells_t* C, const grid_t* g, const double* V, long c,
                         int side, int* ok) {
  int len = side_len(C, c, side);
  int nondec = 1, noninc = 1, have = 0;
  double prev = 0.0;
  for (int u = 0; u < len; ++u) {
    /* W/E lines are walked from north to south, S/N lines from west to east */
    int t = (side <= 1) ? (len - 1 - u) : u;
    long ki, kj;
    side_pair(C, g, c, side, t, &ki, &kj);
    double v = V[ki];
    if (v == INF) continue;
    if (have) {
      if (v < prev) nondec = 0;
      if (v > prev) noninc = 0;
    }
    prev = v;
    have = 1;
  }
  /* dirs seen from the receiving cell: c lies on side opposite[side] of it */
  int recv_side = opposite[side];
  int both = side_dirs[recv_side];
  *ok = nondec || noninc;
  if (nondec && noninc) return both;
  if (recv_side == 0) return nondec ? (1 << 1) : noninc ? (1 << 0) : both;  /* from W */
  if (recv_side == 1) return nondec ? (1 << 2) : noninc ? (1 << 3) : both;  /* from E */
  if (recv_side == 3) return nondec ? (1 << 1) : noninc ? (1 << 2) : both;  /* from N */
  return nondec ? (1 << 0) : noninc ? (1 << 3) : both;                      /* from S */
}

/* HCM cell solver (Section 3.2.2 items 1-3): Locking Sweeping on c with its
   halo fixed, preferred directions first (flagged ones in canonical order,
   then the others), afterwards the canonical loop; stops at the first sweep
   that changes nothing.  Returns the number of sweeps. */
static int hcm_cell_solve(const grid_t* g, double* V, unsigned char* unl,
                          int x0, int x1, int y0, int y1, int flags) {
  static const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
  /* unlock nodes next to the halo and next to sources inside the cell */
  for (int j = y0; j < y1; ++j)
    for (int i = x0; i < x1; ++i) {
      long k = (long)j * g->nx + i;
      if (!g->acc[k] || g->src[k]) continue;
      int u = (i == x0 || i == x1 - 1 || j == y0 || j == y1 - 1);
      for (int e = 0; e < 4 && !u; ++e) {
        int a = i + di[e], b = j + dj[e];
        if (a >= x0 && b >= y0 && a < x1 && b < y1 && g->src[(long)b * g->nx + a]) u = 1;
      }
      if (u) unl[k] = 1;
    }
  int sched[4], ns = 0;
  for (int d = 0; d < 4; ++d)
    if (flags & (1 << d)) sched[ns++] = d;
  for (int d = 0; d < 4; ++d)
    if (!(flags & (1 << d))) sched[ns++] = d;
  int sweeps = 0, changed;
  do {
    int d = sweeps < 4 ? sched[sweeps] : sweeps % 4;
    changed = lsm_sweep_box(g, V, unl, d, x0, x1, y0, y1);
    sweeps++;
  } while (changed);
  return sweeps;
}

/* Heap-Cell Methods: Algorithm generic_LC_cells with the cell values of eq.
   cell_value and a heap (HCM, Section 3.2.2), or Algorithm FHCM (fast = 1,
   Section 3.2.3). */
int orc_hcm(const orc_problem* p, int32_t s, int32_t fast, double* V,
            orc_cell_stats* st) {
  grid_t g;
  cells_t C;
  int rc = grid_init(&g, p);
  if (rc) return rc;
  if (s < 1) {
    grid_free(&g);
    return -1;
  }
  if ((rc = cells_init(&C, &g, s))) {
    grid_free(&g);
    return rc;
  }
  long J = C.J;
  double* key = (double*)malloc(sizeof(double) * J);
  unsigned char* flags = (unsigned char*)calloc(J, 1);
  long* visits = (long*)calloc(J, sizeof(long));
  unsigned char* unl = (unsigned char*)calloc(g.n, 1);
  double* start = (double*)malloc(sizeof(double) * g.n);
  heap_t H;
  if (!key || !flags || !visits || !unl || !start || heap_init(&H, J, key)) {
    free(key); free(flags); free(visits); free(unl); free(start);
    cells_free(&C);
    grid_free(&g);
    return -2;
  }
  orc_cell_stats S;
  memset(&S, 0, sizeof S);
  S.cells = J;
  /* Cell initialisation: HCM keys max q over c & Q, FHCM key 0 and all four
     flags raised; other cells key +inf and not listed. */
  for (long c = 0; c < J; ++c) key[c] = INF;
  for (long c = 0; c < J; ++c) {
    int x0, x1, y0, y1, has = 0;
    double qmax = -INF;
    cell_box(&C, c, &x0, &x1, &y0, &y1);
    for (int j = y0; j < y1; ++j)
      for (int i = x0; i < x1; ++i) {
        long k = (long)j * g.nx + i;
        if (g.src[k]) {
          has = 1;
          if (g.qv[k] > qmax) qmax = g.qv[k];
        }
      }
    if (has) {
      key[c] = fast ? 0.0 : qmax;
      if (fast) flags[c] = 0xF;
      heap_push(&H, c);
    }
  }
  init_values(&g, V);
  while (H.n > 0) {
    long c = heap_pop(&H);
    int first = (visits[c] == 0);
    visits[c]++;
    S.removals++;
    int x0, x1, y0, y1;
    cell_box(&C, c, &x0, &x1, &y0, &y1);
    for (int j = y0; j < y1; ++j)
      memcpy(start + (long)j * g.nx + x0, V + (long)j * g.nx + x0,
             sizeof(double) * (x1 - x0));
    int fl = flags[c];
    flags[c] = 0;
    if (!fast) {
      S.sweeps += hcm_cell_solve(&g, V, unl, x0, x1, y0, y1, fl);
    } else {
      /* one non-directional sweep per flagged direction, canonical order */
      for (int d = 0; d < 4; ++d)
        if (fl & (1 << d)) {
          sweep_box(&g, V, d, x0, x1, y0, y1, 0);
          S.sweeps++;
        }
    }
    for (int side = 0; side < 4; ++side) {
      long ck = cell_nbr(&C, c, side);
      if (ck < 0) continue;
      int add = 0, len = side_len(&C, c, side);
      for (int t = 0; t < len && !add; ++t) {
        long ki, kj;
        side_pair(&C, &g, c, side, t, &ki, &kj);
        int changed = V[ki] < start[ki] || (first && g.src[ki]);
        if (changed && g.acc[kj] && !g.src[kj] && V[ki] < V[kj]) add = 1;
      }
      double est;
      if (cell_value_estimate(&C, &g, V, c, side, ck, &est) && est < key[ck]) {
        key[ck] = est;
        if (H.pos[ck] >= 0) heap_up(&H, H.pos[ck]);
      }
      if (add) {
        int dirs;
        if (fast) {
          int ok;
          dirs = monotone_dirs(&C, &g, V, c, side, &ok);
          S.mon_checks++;
          S.mon_ok += ok;
        } else {
          dirs = side_dirs[opposite[side]];
        }
        flags[ck] |= (unsigned char)dirs;
        if (H.pos[ck] < 0) heap_push(&H, ck);
      }
    }
  }
  if (st) *st = S;
  heap_free(&H);
  free(key); free(flags); free(visits); free(unl); free(start);
  cells_free(&C);
  grid_free(&g);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Fast Marching-Sweeping Method (Algorithm FMSM, remark on Modified Fast    */
/* Sweeping, figure on coarse sweep choice)                                 */
/* ------------------------------------------------------------------------ */

/* READING of the figure: A = sides with an earlier-accepted neighbour.  With
   vertical and horizontal members, sweep from each corner XY with X in
   A & {N,S} and Y in A & {E,W}; only horizontal members Y: NY and SY; only
   vertical members X: XE and XW. */
int32_t orc_fmsm_dirs(int32_t sides) {
  int W = sides & 1, E = (sides >> 1) & 1, S = (sides >> 2) & 1, N = (sides >> 3) & 1;
  int hor = W || E, ver = S || N, d = 0;
  /* direction bits: 0 SW, 1 NW, 2 NE, 3 SE */
  if (hor && ver) {
    if (S && W) d |= 1 << 0;
    if (N && W) d |= 1 << 1;
    if (N && E) d |= 1 << 2;
    if (S && E) d |= 1 << 3;
  } else if (hor) {
    if (W) d |= (1 << 0) | (1 << 1);
    if (E) d |= (1 << 2) | (1 << 3);
  } else if (ver) {
    if (S) d |= (1 << 0) | (1 << 3);
    if (N) d |= (1 << 1) | (1 << 2);
  }
  return d;
}

int orc_fmsm(const orc_problem* p, int32_t s, double* V, int64_t* order_out,
             double* coarse_u, orc_cell_stats* st) {
  grid_t g;
  cells_t C;
  int rc = grid_init(&g, p);
  if (rc) return rc;
  if (s < 1) {
    grid_free(&g);
    return -1;
  }
  if ((rc = cells_init(&C, &g, s))) {
    grid_free(&g);
    return rc;
  }
  long J = C.J;
  double* Fc = (double*)malloc(sizeof(double) * J);
  uint8_t* mc = (uint8_t*)calloc(J, 1);
  int64_t* csrc = (int64_t*)malloc(sizeof(int64_t) * J);
  double* cq = (double*)malloc(sizeof(double) * J);
  double* Uc = (double*)malloc(sizeof(double) * J);
  int64_t* P = (int64_t*)malloc(sizeof(int64_t) * J);
  long* rank = (long*)malloc(sizeof(long) * J);
  unsigned char* issrc = (unsigned char*)calloc(J, 1);
  if (!Fc || !mc || !csrc || !cq || !Uc || !P || !rank || !issrc) {
    rc = -2;
    goto done;
  }
  /* Part I.  Coarse grid of cell centres, h^c = s h (Section 3.1: a coarse
     gridpoint is the centre of its cell, and Fast Marching runs on the coarse
     grid).  READING: the coarse speed is F at the cell centre: the centre
     node for an odd side, else the mean of the two or four accessible nodes
     around the centre, added in the order (x ascending, then y ascending
     within each x).  If none of those is accessible, the mean of F over the
     cell's accessible nodes, summed column by column (each column bottom to
     top, then the column sums left to right); an all-obstacle cell is a
     coarse obstacle.  A cell holding sources is a coarse source with the
     smallest of their q. */
  long nsc = 0;
  for (long c = 0; c < J; ++c) {
    int x0, x1, y0, y1, cnt = 0, has = 0;
    double sum = 0.0, qmin = INF;
    cell_box(&C, c, &x0, &x1, &y0, &y1);
    for (int i = x0; i < x1; ++i) {
      double col = 0.0;
      for (int j = y0; j < y1; ++j) {
        long k = (long)j * g.nx + i;
        if (!g.acc[k]) continue;
        col += g.F[k];
        cnt++;
        if (g.src[k]) {
          has = 1;
          if (g.qv[k] < qmin) qmin = g.qv[k];
        }
      }
      sum += col;
    }
    mc[c] = cnt > 0;
    Fc[c] = cnt > 0 ? sum / cnt : 1.0;
    {
      int is[2] = {(x0 + x1 - 1) / 2, (x0 + x1) / 2}, js[2] = {(y0 + y1 - 1) / 2, (y0 + y1) / 2};
      int ni = is[0] == is[1] ? 1 : 2, nj = js[0] == js[1] ? 1 : 2, nc = 0;
      double sc = 0.0;
      for (int a = 0; a < ni; ++a)
        for (int b = 0; b < nj; ++b) {
          long k = (long)js[b] * g.nx + is[a];
          if (!g.acc[k]) continue;
          sc += g.F[k];
          nc++;
        }
      if (nc > 0) Fc[c] = sc / nc;
    }
    if (has) {
      csrc[nsc] = c;
      cq[nsc] = qmin;
      nsc++;
      issrc[c] = 1;
    }
  }
  {
    orc_problem cp;
    cp.nx = C.Kx;
    cp.ny = C.Ky;
    cp.h = (double)s * g.h;
    cp.F = Fc;
    cp.mask = mc;
    cp.nsrc = (int32_t)nsc;
    cp.src = csrc;
    cp.q = cq;
    int64_t na = 0;
    if ((rc = orc_fmm(&cp, Uc, P, &na))) goto done;
    /* accessible cells the coarse front never reaches follow, by index */
    for (long c = 0; c < J; ++c)
      if (mc[c] && Uc[c] == INF) P[na++] = c;
    for (long c = 0; c < J; ++c) rank[c] = -1;
    for (long t = 0; t < na; ++t) rank[P[t]] = t;
    /* Part II.  Fine initialisation, then cells in the order P. */
    init_values(&g, V);
    orc_cell_stats S;
    memset(&S, 0, sizeof S);
    S.cells = J;
    for (long t = 0; t < na; ++t) {
      long c = P[t];
      int x0, x1, y0, y1;
      cell_box(&C, c, &x0, &x1, &y0, &y1);
      S.removals++;
      if (issrc[c] || Uc[c] == INF) {
        /* plain FSM to convergence on the cell */
        int sw = 0, ch;
        do {
          ch = sweep_box(&g, V, sw % 4, x0, x1, y0, y1, 0);
          sw++;
        } while (ch);
        S.sweeps += sw;
      } else {
        int sides = 0;
        for (int side = 0; side < 4; ++side) {
          long ck = cell_nbr(&C, c, side);
          if (ck >= 0 && rank[ck] >= 0 && rank[ck] < t) sides |= 1 << side;
        }
        int dirs = orc_fmsm_dirs(sides);
        for (int d = 0; d < 4; ++d)
          if (dirs & (1 << d)) {
            sweep_box(&g, V, d, x0, x1, y0, y1, 1);
            S.sweeps++;
          }
      }
    }
    if (order_out)
      for (long t = 0; t < J; ++t) order_out[t] = t < na ? P[t] : -1;
    if (coarse_u) memcpy(coarse_u, Uc, sizeof(double) * J);
    if (st) *st = S;
  }
done:
  free(Fc); free(mc); free(csrc); free(cq); free(Uc); free(P); free(rank); free(issrc);
  cells_free(&C);
  grid_free(&g);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Three dimensions: the same methods on a 3-D grid with six neighbours      */
/* ------------------------------------------------------------------------ */

typedef struct {
  int nx, ny, nz;
  long n;
  double* delta;
  unsigned char* acc;
  unsigned char* src;
  double* qv;
} grid3_t;

static void grid3_free(grid3_t* g) {
  free(g->delta);
  free(g->acc);
  free(g->src);
  free(g->qv);
}

static int grid3_init(grid3_t* g, const orc3_problem* p) {
  memset(g, 0, sizeof *g);
  if (!p || p->nx < 1 || p->ny < 1 || p->nz < 1 || !(p->h > 0.0) || !isfinite(p->h) || !p->F ||
      p->nsrc < 1 || !p->src)
    return -1;
  g->nx = p->nx;
  g->ny = p->ny;
  g->nz = p->nz;
  g->n = (long)p->nx * p->ny * p->nz;
  g->delta = (double*)malloc(sizeof(double) * g->n);
  g->acc = (unsigned char*)malloc(g->n);
  g->src = (unsigned char*)calloc(g->n, 1);
  g->qv = (double*)malloc(sizeof(double) * g->n);
  if (!g->delta || !g->acc || !g->src || !g->qv) {
    grid3_free(g);
    return -2;
  }
  for (long k = 0; k < g->n; ++k) {
    g->acc[k] = p->mask ? (p->mask[k] != 0) : 1;
    g->qv[k] = INF;
    if (g->acc[k]) {
      double f = p->F[k];
      if (!(f > 0.0) || !isfinite(f)) {
        grid3_free(g);
        return -1;
      }
      g->delta[k] = p->h / f;
    } else {
      g->delta[k] = INF;
    }
  }
  for (int s = 0; s < p->nsrc; ++s) {
    long k = (long)p->src[s];
    double q = p->q ? p->q[s] : 0.0;
    if (k < 0 || k >= g->n || !g->acc[k] || !isfinite(q)) {
      grid3_free(g);
      return -1;
    }
    g->src[k] = 1;
    if (q < g->qv[k]) g->qv[k] = q;
  }
  return 0;
}

double orc3_update(double a, double b, double c, double delta) {
  double lo = a < b ? a : b, hi = a < b ? b : a;
  double m1 = lo < c ? lo : c, mid = lo < c ? c : lo;
  double m2 = hi < mid ? hi : mid, m3 = hi < mid ? mid : hi;
  if (m1 == INF) return INF;
  double d = m1 - m2;
  if (fabs(d) >= delta) return m1 + delta;
  double u2 = 0.5 * (m1 + m2 + sqrt(2.0 * delta * delta - d * d));
  if (u2 <= m3) return u2;
  double d13 = m1 - m3, d23 = m2 - m3;
  double disc = 3.0 * delta * delta - (d * d + d13 * d13 + d23 * d23);
  if (!(disc >= 0.0)) return u2; /* rounding guard: the two-sided root */
  return (m1 + m2 + m3 + sqrt(disc)) / 3.0;
}

static double nb3(const grid3_t* g, const double* V, int i, int j, int k) {
  if (i < 0 || j < 0 || k < 0 || i >= g->nx || j >= g->ny || k >= g->nz) return INF;
  return V[((long)k * g->ny + j) * g->nx + i];
}

/* Temporary value of node (i,j,k) from its six neighbours. */
static double node_update3(const grid3_t* g, const double* V, int i, int j, int k) {
  double uW = nb3(g, V, i - 1, j, k), uE = nb3(g, V, i + 1, j, k);
  double uS = nb3(g, V, i, j - 1, k), uN = nb3(g, V, i, j + 1, k);
  double uD = nb3(g, V, i, j, k - 1), uU = nb3(g, V, i, j, k + 1);
  double a = uW < uE ? uW : uE;
  double b = uS < uN ? uS : uN;
  double c = uD < uU ? uD : uU;
  return orc3_update(a, b, c, g->delta[((long)k * g->ny + j) * g->nx + i]);
}

static void init_values3(const grid3_t* g, double* V) {
  for (long k = 0; k < g->n; ++k) V[k] = g->src[k] ? g->qv[k] : INF;
}

/* Fast Marching: as in two dimensions (sources accepted first in (q, index)
   order, then the smallest (value, index) considered node). */
int orc3_fmm(const orc3_problem* p, double* V, int64_t* order, int64_t* nacc) {
  grid3_t g;
  int rc = grid3_init(&g, p);
  if (rc) return rc;
  unsigned char* lab = (unsigned char*)calloc(g.n, 1);
  long* srcs = (long*)malloc(sizeof(long) * g.n);
  heap_t H, Q;
  if (!lab || !srcs || heap_init(&H, g.n, V)) {
    free(lab);
    free(srcs);
    grid3_free(&g);
    return -2;
  }
  if (heap_init(&Q, g.n, g.qv)) {
    free(lab);
    free(srcs);
    heap_free(&H);
    grid3_free(&g);
    return -2;
  }
  init_values3(&g, V);
  long ns = 0, na = 0;
  for (long k = 0; k < g.n; ++k)
    if (g.src[k]) heap_push(&Q, k);
  while (Q.n > 0) srcs[ns++] = heap_pop(&Q);
  heap_free(&Q);
  for (long s = 0; s < ns; ++s) {
    lab[srcs[s]] = ACCEPTED;
    if (order) order[na] = srcs[s];
    na++;
  }
  static const int di[6] = {-1, 1, 0, 0, 0, 0}, dj[6] = {0, 0, -1, 1, 0, 0}, dk[6] = {0, 0, 0, 0, -1, 1};
  long pos = 0;  /* sources first, then the heap */
  for (;;) {
    long x;
    if (pos < ns) {
      x = srcs[pos++];
    } else {
      if (H.n == 0) break;
      x = heap_pop(&H);
      lab[x] = ACCEPTED;
      if (order) order[na] = x;
      na++;
    }
    int i = (int)(x % g.nx), j = (int)((x / g.nx) % g.ny), k = (int)(x / ((long)g.nx * g.ny));
    for (int e = 0; e < 6; ++e) {
      int a = i + di[e], b = j + dj[e], c = k + dk[e];
      if (a < 0 || b < 0 || c < 0 || a >= g.nx || b >= g.ny || c >= g.nz) continue;
      long kk = ((long)c * g.ny + b) * g.nx + a;
      if (!g.acc[kk] || lab[kk] == ACCEPTED) continue;
      double t = node_update3(&g, V, a, b, c);
      if (t < V[kk]) V[kk] = t;
      if (lab[kk] == FAR) {
        lab[kk] = CONSIDERED;
        heap_push(&H, kk);
      } else {
        heap_up(&H, H.pos[kk]);
      }
    }
  }
  if (nacc) *nacc = na;
  free(lab);
  free(srcs);
  heap_free(&H);
  grid3_free(&g);
  return 0;
}

int orc3_fsm(const orc3_problem* p, double* V, int32_t* nsweeps) {
  grid3_t g;
  int rc = grid3_init(&g, p);
  if (rc) return rc;
  init_values3(&g, V);
  int sweep = 0, changed;
  do {
    int d = sweep % 8;
    int sx = (d & 1) ? -1 : 1, sy = (d & 2) ? -1 : 1, sz = (d & 4) ? -1 : 1;
    changed = 0;
    for (int kk = 0; kk < g.nz; ++kk) {
      int k = sz > 0 ? kk : g.nz - 1 - kk;
      for (int jj = 0; jj < g.ny; ++jj) {
        int j = sy > 0 ? jj : g.ny - 1 - jj;
        for (int ii = 0; ii < g.nx; ++ii) {
          int i = sx > 0 ? ii : g.nx - 1 - ii;
          long x = ((long)k * g.ny + j) * g.nx + i;
          if (!g.acc[x] || g.src[x]) continue;
          double t = node_update3(&g, V, i, j, k);
          if (t < V[x]) {
            V[x] = t;
            changed = 1;
          }
        }
      }
    }
    sweep++;
  } while (changed);
  if (nsweeps) *nsweeps = sweep;
  grid3_free(&g);
  return 0;
}

/* Fast Marching-Sweeping in three dimensions (Algorithm FMSM extended as
   Section 5 proposes).  Cells of s x s x s nodes, cell c covering
   [c s, min((c + 1) s, n)) along each axis (no merging of a last one-node
   cell).  Part I: Fast Marching on the grid of cell centres.  Part II: the
   cells in that acceptance order, each swept once in every ordering its
   earlier-accepted neighbours allow, with the update restricted to the
   sweep's upwind neighbours; cells holding exit nodes and cells the coarse
   front never reaches are swept to convergence with the standard update. */

/* Canonical order of the eight orderings (bit 0 x descending, bit 1 y
   descending, bit 2 z descending): z ascending first, and within a z
   direction the two-dimensional order SW, NW, NE, SE. */
static const int fmsm3_seq[8] = {0, 2, 3, 1, 4, 6, 7, 5};

static void cell3_box(long c, const int* K, int s, const grid3_t* g, int* lo, int* hi) {
  int ci[3] = {(int)(c % K[0]), (int)((c / K[0]) % K[1]), (int)(c / ((long)K[0] * K[1]))};
  int n[3] = {g->nx, g->ny, g->nz};
  for (int a = 0; a < 3; ++a) {
    lo[a] = ci[a] * s;
    hi[a] = (ci[a] + 1) * s < n[a] ? (ci[a] + 1) * s : n[a];
  }
}

/* One Gauss-Seidel sweep of the box in ordering d; directional: the update
   from the three upwind neighbours of the ordering only. */
static int sweep3_box(const grid3_t* g, double* V, int d, const int* lo, const int* hi,
                      int directional) {
  int sx = (d & 1) ? -1 : 1, sy = (d & 2) ? -1 : 1, sz = (d & 4) ? -1 : 1, changed = 0;
  for (int kk = 0; kk < hi[2] - lo[2]; ++kk) {
    int k = sz > 0 ? lo[2] + kk : hi[2] - 1 - kk;
    for (int jj = 0; jj < hi[1] - lo[1]; ++jj) {
      int j = sy > 0 ? lo[1] + jj : hi[1] - 1 - jj;
      for (int ii = 0; ii < hi[0] - lo[0]; ++ii) {
        int i = sx > 0 ? lo[0] + ii : hi[0] - 1 - ii;
        long x = ((long)k * g->ny + j) * g->nx + i;
        if (!g->acc[x] || g->src[x]) continue;
        double t = directional ? orc3_update(nb3(g, V, i - sx, j, k), nb3(g, V, i, j - sy, k),
                                             nb3(g, V, i, j, k - sz), g->delta[x])
                               : node_update3(g, V, i, j, k);
        if (t < V[x]) {
          V[x] = t;
          changed = 1;
        }
      }
    }
  }
  return changed;
}

/* READING of the sweep choice in three dimensions (the figure on coarse
   sweep choice, per axis): an axis with an earlier-accepted neighbour on its
   low (high) face contributes the ascending (descending) direction, both when
   both; an axis without one contributes both directions; an axis along which
   the grid is one node thick contributes the ascending one only (both visit
   its node in the same order from the same neighbours).  The orderings are
   the combinations, in canonical order.  Returns a mask over ordering codes. */
int32_t orc3_fmsm_orderings(int32_t faces, int32_t thin_axes) {
  int allow[3];
  for (int a = 0; a < 3; ++a) {
    int lo = (faces >> (2 * a)) & 1, hi = (faces >> (2 * a + 1)) & 1;
    if ((thin_axes >> a) & 1) allow[a] = 1;
    else if (lo || hi) allow[a] = (lo ? 1 : 0) | (hi ? 2 : 0);
    else allow[a] = 3;
  }
  int32_t m = 0;
  for (int d = 0; d < 8; ++d) {
    int ok = 1;
    for (int a = 0; a < 3; ++a) ok &= (allow[a] >> ((d >> a) & 1)) & 1;
    if (ok) m |= 1 << d;
  }
  return m;
}

int orc3_fmsm(const orc3_problem* p, int32_t s, double* V, int64_t* order_out, double* coarse_u,
              orc_cell_stats* st) {
  grid3_t g;
  int rc = grid3_init(&g, p);
  if (rc) return rc;
  if (s < 1) {
    grid3_free(&g);
    return -1;
  }
  int K[3] = {(g.nx + s - 1) / s, (g.ny + s - 1) / s, (g.nz + s - 1) / s};
  long J = (long)K[0] * K[1] * K[2];
  double* Fc = (double*)malloc(sizeof(double) * J);
  uint8_t* mc = (uint8_t*)calloc(J, 1);
  int64_t* csrc = (int64_t*)malloc(sizeof(int64_t) * J);
  double* cq = (double*)malloc(sizeof(double) * J);
  double* Uc = (double*)malloc(sizeof(double) * J);
  int64_t* P = (int64_t*)malloc(sizeof(int64_t) * J);
  long* rank = (long*)malloc(sizeof(long) * J);
  unsigned char* issrc = (unsigned char*)calloc(J, 1);
  if (!Fc || !mc || !csrc || !cq || !Uc || !P || !rank || !issrc) {
    rc = -2;
    goto done3;
  }
  {
    /* Part I.  Coarse speed (READING, as in two dimensions): F at the cell
       centre -- the centre node along an axis of odd extent, the two around
       it otherwise -- the mean of those that are accessible, added x
       outermost, then y, then z; if none is, the mean of F over the cell's
       accessible nodes, summed plane by plane (each x-plane y outer, z
       inner, then the plane sums x ascending).  Coarse exit cost: min q of
       the cell's exit nodes; all-obstacle cells are coarse obstacles. */
    long nsc = 0;
    int thin = (g.nx == 1 ? 1 : 0) | (g.ny == 1 ? 2 : 0) | (g.nz == 1 ? 4 : 0);
    for (long c = 0; c < J; ++c) {
      int lo[3], hi[3], cnt = 0, has = 0;
      double sum = 0.0, qmin = INF;
      cell3_box(c, K, s, &g, lo, hi);
      for (int i = lo[0]; i < hi[0]; ++i) {
        double pl = 0.0;
        for (int j = lo[1]; j < hi[1]; ++j)
          for (int k = lo[2]; k < hi[2]; ++k) {
            long x = ((long)k * g.ny + j) * g.nx + i;
            if (!g.acc[x]) continue;
            pl += p->F[x];
            cnt++;
            if (g.src[x]) {
              has = 1;
              if (g.qv[x] < qmin) qmin = g.qv[x];
            }
          }
        sum += pl;
      }
      mc[c] = cnt > 0;
      Fc[c] = cnt > 0 ? sum / cnt : 1.0;
      int is[2] = {(lo[0] + hi[0] - 1) / 2, (lo[0] + hi[0]) / 2};
      int js[2] = {(lo[1] + hi[1] - 1) / 2, (lo[1] + hi[1]) / 2};
      int ks[2] = {(lo[2] + hi[2] - 1) / 2, (lo[2] + hi[2]) / 2};
      int ni = is[0] == is[1] ? 1 : 2, nj = js[0] == js[1] ? 1 : 2, nk = ks[0] == ks[1] ? 1 : 2;
      int nc = 0;
      double sc = 0.0;
      for (int a = 0; a < ni; ++a)
        for (int b = 0; b < nj; ++b)
          for (int e = 0; e < nk; ++e) {
            long x = ((long)ks[e] * g.ny + js[b]) * g.nx + is[a];
            if (!g.acc[x]) continue;
            sc += p->F[x];
            nc++;
          }
      if (nc > 0) Fc[c] = sc / nc;
      if (has) {
        csrc[nsc] = c;
        cq[nsc] = qmin;
        nsc++;
        issrc[c] = 1;
      }
    }
    orc3_problem cp;
    cp.nx = K[0];
    cp.ny = K[1];
    cp.nz = K[2];
    cp.h = (double)s * p->h;
    cp.F = Fc;
    cp.mask = mc;
    cp.nsrc = (int32_t)nsc;
    cp.src = csrc;
    cp.q = cq;
    int64_t na = 0;
    if ((rc = orc3_fmm(&cp, Uc, P, &na))) goto done3;
    for (long c = 0; c < J; ++c)
      if (mc[c] && Uc[c] == INF) P[na++] = c;
    for (long c = 0; c < J; ++c) rank[c] = -1;
    for (long t = 0; t < na; ++t) rank[P[t]] = t;
    /* Part II */
    init_values3(&g, V);
    orc_cell_stats S;
    memset(&S, 0, sizeof S);
    S.cells = J;
    for (long t = 0; t < na; ++t) {
      long c = P[t];
      int lo[3], hi[3];
      cell3_box(c, K, s, &g, lo, hi);
      S.removals++;
      if (issrc[c] || Uc[c] == INF) {
        int sw = 0, ch;
        do {
          ch = sweep3_box(&g, V, fmsm3_seq[sw % 8], lo, hi, 0);
          sw++;
        } while (ch);
        S.sweeps += sw;
      } else {
        int ci[3] = {(int)(c % K[0]), (int)((c / K[0]) % K[1]), (int)(c / ((long)K[0] * K[1]))};
        long stride[3] = {1, K[0], (long)K[0] * K[1]};
        int faces = 0;
        for (int a = 0; a < 3; ++a) {
          if (ci[a] > 0 && rank[c - stride[a]] >= 0 && rank[c - stride[a]] < t) faces |= 1 << (2 * a);
          if (ci[a] + 1 < K[a] && rank[c + stride[a]] >= 0 && rank[c + stride[a]] < t)
            faces |= 1 << (2 * a + 1);
        }
        int32_t m = orc3_fmsm_orderings(faces, thin);
        for (int q = 0; q < 8; ++q)
          if (m & (1 << fmsm3_seq[q])) {
            sweep3_box(&g, V, fmsm3_seq[q], lo, hi, 1);
            S.sweeps++;
          }
      }
    }
    if (order_out)
      for (long t = 0; t < J; ++t) order_out[t] = t < na ? P[t] : -1;
    if (coarse_u) memcpy(coarse_u, Uc, sizeof(double) * J);
    if (st) *st = S;
  }
done3:
  free(Fc); free(mc); free(csrc); free(cq); free(Uc); free(P); free(rank); free(issrc);
  grid3_free(&g);
  return rc;
}

int orc3_jacobi(const orc3_problem* p, double* V, int32_t* niters) {
  grid3_t g;
  int rc = grid3_init(&g, p);
  if (rc) return rc;
  double* W = (double*)malloc(sizeof(double) * g.n);
  if (!W) {
    grid3_free(&g);
    return -2;
  }
  init_values3(&g, V);
  int it = 0, changed;
  do {
    changed = 0;
    for (int k = 0; k < g.nz; ++k)
      for (int j = 0; j < g.ny; ++j)
        for (int i = 0; i < g.nx; ++i) {
          long x = ((long)k * g.ny + j) * g.nx + i;
          W[x] = V[x];
          if (!g.acc[x] || g.src[x]) continue;
          double t = node_update3(&g, V, i, j, k);
          if (t < W[x]) {
            W[x] = t;
            changed = 1;
          }
        }
    memcpy(V, W, sizeof(double) * g.n);
    it++;
  } while (changed);
  if (niters) *niters = it;
  free(W);
  grid3_free(&g);
  return 0;
}

double orc3_residual(const orc3_problem* p, const double* V, double* r) {
  grid3_t g;
  if (grid3_init(&g, p)) return -1.0;
  double mx = 0.0;
  for (int k = 0; k < g.nz; ++k)
    for (int j = 0; j < g.ny; ++j)
      for (int i = 0; i < g.nx; ++i) {
        long x = ((long)k * g.ny + j) * g.nx + i;
        double res = 0.0;
        if (g.acc[x] && !g.src[x]) {
          double t = node_update3(&g, V, i, j, k);
          if (V[x] == INF) res = t == INF ? 0.0 : INF;
          else res = fabs(t - V[x]) / V[x];
        }
        if (r) r[x] = res;
        if (res > mx) mx = res;
      }
  grid3_free(&g);
  return mx;
}
