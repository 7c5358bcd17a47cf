/*
 * Eikonal oracle: plain, serial, fp64 reference implementations of the
 * methods of Chacon & Vladimirsky, "Fast two-scale methods for Eikonal
 * equations" (arXiv 1110.6220).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this code.  The GPU library never
 * links, includes or calls it, and it shares no code with the GPU library.
 *
 * Conventions (shared with the problem statement, not with any code):
 *   - node (i, j) <-> linear index j*nx + i, x fastest; x_i = x0 + i*h;
 *   - F > 0 is the speed, mask 1 = accessible, 0 = obstacle (NULL = all 1);
 *   - src[] are linear node indices of the exit set Q, q[] their exit costs
 *     (NULL = all zero); duplicate sources take the smallest q;
 *   - outputs are +inf on obstacles and on nodes with no path to Q.
 */
#ifndef EIK_ORACLE_H
#define EIK_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t nx, ny;
  double h;
  const double* F;
  const uint8_t* mask;
  int32_t nsrc;
  const int64_t* src;
  const double* q;
} orc_problem;

typedef struct {
  int64_t cells;        /* number of cells J in the decomposition           */
  int64_t removals;     /* heap removals (AvHR = removals / cells)          */
  int64_t sweeps;       /* sweeps incl. final no-change ones (AvS = /cells) */
  int64_t mon_checks;   /* FHCM monotonicity checks performed               */
  int64_t mon_ok;       /* ... of which the side line was monotone          */
} orc_cell_stats;

/* Error codes: 0 ok, -1 invalid input, -2 out of memory. */

/* Local update from the quadrant shortcut: a = min(U_W,U_E), b = min(U_S,U_N),
   delta = h/F.  Returns +inf when both a and b are infinite. */
double orc_update(double a, double b, double delta);

/* Fast Marching with a binary heap keyed by (value, linear index).
   order (optional, nx*ny entries): acceptance order, sources first (sorted by
   (q, index)); *naccepted receives its length. */
int orc_fmm(const orc_problem* p, double* V, int64_t* order, int64_t* naccepted);
/* Fast Sweeping: alternating Gauss-Seidel sweeps until a sweep changes nothing.
   *nsweeps counts every sweep including the final one. */
int orc_fsm(const orc_problem* p, double* V, int32_t* nsweeps);
/* Locking Sweeping: the same sweeps, visiting only unlocked nodes. */
int orc_lsm(const orc_problem* p, double* V, int32_t* nsweeps);
/* One sweep at a time, for the early-termination study (Section 4 remark on
   stopping sweeping methods before convergence).  orc_sweep_init sets V to q
   on exit nodes and +inf elsewhere and, when unlocked is not NULL, unlocks
   the accessible non-exit neighbours of exit nodes (Locking Sweeping's
   start).  orc_fsm_sweep performs sweep number `sweep` (direction sweep mod
   4, as in orc_fsm) over the whole grid; orc_lsm_sweep the same sweep of
   Locking Sweeping, visiting only unlocked nodes.  Both report the largest
   decrease of a node (+inf when a node leaves +inf; 0 when none decreased)
   and the number of nodes that decreased. */
int orc_sweep_init(const orc_problem* p, double* V, uint8_t* unlocked);
int orc_fsm_sweep(const orc_problem* p, double* V, int32_t sweep, double* max_change,
                  int64_t* n_changed);
int orc_lsm_sweep(const orc_problem* p, double* V, uint8_t* unlocked, int32_t sweep,
                  double* max_change, int64_t* n_changed);
/* Value iteration V <- min(V, T V), all nodes at once, to a fixed point. */
int orc_jacobi(const orc_problem* p, double* V, int32_t* niters);
/* Fixed-point residual r_k = |T(V)_k - V_k| / V_k on accessible non-source
   nodes with finite V (inf where V is inf but T(V) is finite); r may be NULL.
   Returns max r, or -1 on invalid input. */
double orc_residual(const orc_problem* p, const double* V, double* r);

/* Heap-Cell Method (fast = 0) and Fast Heap-Cell Method (fast = 1) with
   square cells of side s. */
int orc_hcm(const orc_problem* p, int32_t s, int32_t fast, double* V,
            orc_cell_stats* st);
/* Fast Marching-Sweeping Method with cells of side s.  order (optional, J
   entries) receives the cell processing order, coarse_u (optional, J) the
   coarse Fast Marching values. */
int orc_fmsm(const orc_problem* p, int32_t s, double* V, int64_t* order,
             double* coarse_u, orc_cell_stats* st);

/* Cell tiling along one axis of n nodes with nominal side s:
   returns the number of cells K; lo (K+1 entries, optional) the starts. */
int32_t orc_tiling(int32_t n, int32_t s, int32_t* lo);
/* FMSM sweep directions (bit d = direction d; 0 SW, 1 NW, 2 NE, 3 SE) for a
   cell whose earlier-accepted neighbours are the sides in `sides`
   (bit 0 W, 1 E, 2 S, 3 N). */
int32_t orc_fmsm_dirs(int32_t sides);

/* ---------------------------------------------------------------------- */
/* Three dimensions (the extension the paper names for its cell methods):  */
/* node (i, j, k) <-> (k*ny + j)*nx + i, six neighbours.                   */
/* ---------------------------------------------------------------------- */
typedef struct {
  int32_t nx, ny, nz;
  double h;
  const double* F;
  const uint8_t* mask;
  int32_t nsrc;
  const int64_t* src;
  const double* q;
} orc3_problem;

/* First-order upwind update from a = min(U_W,U_E), b = min(U_S,U_N),
   c = min(U_D,U_U) with delta = h/F: sorted m1 <= m2 <= m3, one-sided
   m1 + delta when m2 - m1 >= delta, else the two-sided root of
   (U-m1)^2 + (U-m2)^2 = delta^2 when it does not exceed m3, else the
   three-sided root of (U-m1)^2 + (U-m2)^2 + (U-m3)^2 = delta^2.  With
   c = +inf it equals orc_update(a, b, delta) bit for bit. */
double orc3_update(double a, double b, double c, double delta);
int orc3_fmm(const orc3_problem* p, double* V, int64_t* order, int64_t* naccepted);
/* Gauss-Seidel sweeps in the eight orderings (sweep number mod 8: bit 0
   x descending, bit 1 y descending, bit 2 z descending) until a sweep
   changes nothing. */
int orc3_fsm(const orc3_problem* p, double* V, int32_t* nsweeps);
int orc3_jacobi(const orc3_problem* p, double* V, int32_t* niters);
double orc3_residual(const orc3_problem* p, const double* V, double* r);
/* Fast Marching-Sweeping on cells of s x s x s nodes (cell c covering
   [c s, min((c+1) s, n)) per axis): Fast Marching on the grid of cell
   centres (h^c = s h, coarse speed F at the centre), then the cells in its
   acceptance order, each swept once in the orderings of
   orc3_fmsm_orderings (directional update); cells holding exit nodes and
   cells the coarse front never reaches are swept to convergence.
   order_out: J cell indices (-1 after the processed ones); coarse_u: J. */
int orc3_fmsm(const orc3_problem* p, int32_t s, double* V, int64_t* order_out, double* coarse_u,
              orc_cell_stats* st);
/* Orderings (mask over codes 0..7) for a cell whose earlier-accepted
   neighbours lie on `faces` (bit 2 axis + side, side 1 = high face) in a
   grid that is one node thick along the axes of `thin_axes` (bit axis). */
int32_t orc3_fmsm_orderings(int32_t faces, int32_t thin_axes);

#ifdef __cplusplus
}
#endif
#endif
