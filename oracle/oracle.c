/*
 * oracle.c -- plain, slow, FP64 CPU oracle for the FIRE 2.0 hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the HIP library; the two meet only through the
 * seeded input arrays.
 *
 * What it computes (Guenole et al., "Assessment and optimization of the fast
 * inertial relaxation engine (FIRE) for energy minimization in atomistic
 * simulations and its implementation in LAMMPS"):
 *   - E(x) and F = -grad E (Sec. 2.1, the definition under Eq. (1)) for
 *     * energy-shifted 12-6 Lennard-Jones,
 *     * the second-moment (Gupta / RGL) EAM-form potential of Sec. 5.2
 *       (pair term plus embedding F(rho) = -xi sqrt(rho)), with a cubic taper,
 *     * the Stillinger-Weber two- plus three-body potential of the Si test
 *       case (Sec. 5.1, case 5 of Sec. 5.3; original parameterisation),
 *     * an anisotropic quadratic well (test potential),
 *     as sums over the pairs closer than the cutoff under the minimum image;
 *     each atom's sums run over its partners in index order.  The pair set
 *     is found by testing every pair, or (same pairs, same order, same bits)
 *     through a cell grid for large systems,
 *   - the analytic Hessian-vector product H u of the same energies,
 *   - the FIRE 2.0 loop (Algorithm 2) with the semi-implicit Euler integrator
 *     and the mixing placed after the kick (Algorithm 4, Sec. 3.3), the
 *     Table 1 parameter semantics, and the stop criteria of Sec. 3.4; the
 *     original FIRE loop (Algorithm 1) and the explicit-Euler / velocity-Verlet
 *     integrators (Algorithms 3 and 6) as options.
 *
 * The OpenMP loops are over atoms only; every per-atom sum runs in a fixed
 * order and global sums are serial, so results do not depend on the thread
 * count.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_E_ARG -1
#define OR_E_BOX -2
#define OR_E_NONFINITE -3
#define OR_E_OVERLAP -4

#define OR_POT_LJ 1
#define OR_POT_GUPTA 2
#define OR_POT_HARMONIC 3
#define OR_POT_SW 4

typedef struct {
  double lo[3];
  double len[3];
  int periodic[3];
} or_box;

typedef struct {
  int kind;
  int convention; /* Gupta: 0 = every ordered pair carries phi (RGL), 1 = half sum */
  double eps, sigma, rc;
  double A, p, q, xi, r0, r_in, r_out;
  double k[3];
  double sw_B, sw_a, sw_lambda, sw_gamma; /* Stillinger-Weber (with eps, sigma, A, p, q) */
} or_pot;

int oracle_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ---------------------------------------------------------------- geometry */

/* Minimum-image separation d = x_i - x_j on periodic axes. */
static void min_image(const double *xi, const double *xj, const or_box *b, double d[3]) {
  for (int a = 0; a < 3; ++a) {
    double t = xi[a] - xj[a];
    if (b->periodic[a]) t -= b->len[a] * nearbyint(t / b->len[a]);
    d[a] = t;
  }
}

static double pot_cutoff(const or_pot *p) {
  if (p->kind == OR_POT_LJ) return p->rc;
  if (p->kind == OR_POT_GUPTA) return p->r_out;
  if (p->kind == OR_POT_SW) return p->sw_a * p->sigma;
  return 0.0;
}

static int check_inputs(long n, const double *pos, const or_box *b, const or_pot *p) {
  if (n <= 0 || !pos || !b || !p) return OR_E_ARG;
  for (long i = 0; i < 3 * n; ++i)
    if (!isfinite(pos[i])) return OR_E_NONFINITE;
  double rc = pot_cutoff(p);
  for (int a = 0; a < 3; ++a)
    if (b->periodic[a] && (!(b->len[a] > 0.0) || !(rc < 0.5 * b->len[a]))) return OR_E_BOX;
  return OR_OK;
}

/* -------------------------------------------------------- pair enumeration
 *
 * The energy is a sum over the atom pairs closer than the cutoff (Sec. 2.1).
 * Every force loop below reads that pair set from a table: for each atom i,
 * the atoms j != i with |x_i - x_j|^2 < rc^2 under the minimum image, in
 * increasing j.  Two ways of finding the set fill the table:
 *   - brute force (the default): every j is tested, O(n^2);
 *   - cells: atoms are binned into cells at least rc wide, and only the atoms
 *     of the (up to) 27 cells around i's cell are tested; the found j are
 *     then sorted.
 * Both test each candidate with the same min_image() and the same strict
 * "< rc^2", so they find the same j in the same order and every sum below is
 * bit-identical between them; the cells only make large systems affordable.
 */

static int g_use_cells = 0;

void oracle_set_cells(int on) { g_use_cells = on ? 1 : 0; }
int oracle_get_cells(void) { return g_use_cells; }

typedef struct {
  long n;
  long *start; /* n + 1 offsets into idx */
  long *idx;   /* neighbours of atom i: idx[start[i] .. start[i+1]-1], increasing */
} or_pairs;

static void pairs_free(or_pairs *t) {
  free(t->start);
  free(t->idx);
  t->start = NULL;
  t->idx = NULL;
}

/* One growable list per atom while searching. */
typedef struct {
  long m, cap;
  long *j;
} or_list;

static void list_push(or_list *l, long j) {
  if (l->m == l->cap) {
    l->cap = l->cap ? 2 * l->cap : 32;
    l->j = (long *)realloc(l->j, sizeof(long) * l->cap);
  }
  l->j[l->m++] = j;
}

static int cmp_long(const void *a, const void *b) {
  long x = *(const long *)a, y = *(const long *)b;
  return (x > y) - (x < y);
}

/* The candidate test shared by both searches; returns 1 for a pair, 0 for
 * none, OR_E_OVERLAP for two atoms at the same place. */
static int in_range(const double *pos, const or_box *b, long i, long j, double rc2) {
  double d[3];
  min_image(pos + 3 * i, pos + 3 * j, b, d);
  double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  if (r2 == 0.0) return OR_E_OVERLAP;
  return r2 < rc2;
}

/* Cell grid: per axis the number of cells, the origin and the cell width.
 * Periodic axes span the box; free axes span the atoms' extent.  Cells are
 * made slightly wider than rc so that rounding in the binning cannot push a
 * pair closer than rc two cells apart. */
typedef struct {
  long nc[3];
  double lo[3], w[3];
} or_grid;

static long cell_coord(const or_grid *g, const or_box *b, int a, double x) {
  double t = (x - g->lo[a]) / (g->w[a] * g->nc[a]); /* fraction of the grid's span */
  if (b->periodic[a]) t -= floor(t);
  long c = (long)floor(t * g->nc[a]);
  if (c < 0) c = 0;
  if (c >= g->nc[a]) c = g->nc[a] - 1;
  return c;
}

static void make_grid(long n, const double *pos, const or_box *b, double rc, or_grid *g) {
  long total = 1;
  for (int a = 0; a < 3; ++a) {
    double lo, ext;
    if (b->periodic[a]) {
      lo = b->lo[a];
      ext = b->len[a];
    } else {
      double mn = pos[a], mx = pos[a];
      for (long i = 1; i < n; ++i) {
        mn = fmin(mn, pos[3 * i + a]);
        mx = fmax(mx, pos[3 * i + a]);
      }
      lo = mn;
      ext = mx - mn;
    }
    long nc = (long)floor(ext / (rc * (1.0 + 1e-9)));
    if (nc < 1) nc = 1;
    if (nc > 4096) nc = 4096;
    g->nc[a] = nc;
    g->lo[a] = lo;
    g->w[a] = ext > 0.0 ? ext / nc : rc;
    total *= nc;
  }
  /* a sparse system in a wide box: coarser cells (more candidates, same pairs) */
  while (total > 8 * n + 64) {
    int a = 0;
    for (int q = 1; q < 3; ++q)
      if (g->nc[q] > g->nc[a]) a = q;
    g->w[a] *= (double)g->nc[a] / ((g->nc[a] + 1) / 2);
    g->nc[a] = (g->nc[a] + 1) / 2;
    total = g->nc[0] * g->nc[1] * g->nc[2];
  }
}

static int pairs_cells(long n, const double *pos, const or_box *b, double rc, or_list *lists) {
  double rc2 = rc * rc;
  or_grid g;
  make_grid(n, pos, b, rc, &g);
  long ncell = g.nc[0] * g.nc[1] * g.nc[2];
  long *cell = (long *)malloc(sizeof(long) * n);
  long *head = (long *)malloc(sizeof(long) * (ncell + 1));
  long *member = (long *)malloc(sizeof(long) * n);
  for (long c = 0; c <= ncell; ++c) head[c] = 0;
  for (long i = 0; i < n; ++i) {
    long cx = cell_coord(&g, b, 0, pos[3 * i]);
    long cy = cell_coord(&g, b, 1, pos[3 * i + 1]);
    long cz = cell_coord(&g, b, 2, pos[3 * i + 2]);
    cell[i] = cx + g.nc[0] * (cy + g.nc[1] * cz);
    head[cell[i] + 1] += 1;
  }
  for (long c = 0; c < ncell; ++c) head[c + 1] += head[c];
  {
    long *fill = (long *)malloc(sizeof(long) * ncell);
    for (long c = 0; c < ncell; ++c) fill[c] = head[c];
    for (long i = 0; i < n; ++i) member[fill[cell[i]]++] = i;
    free(fill);
  }
  int err = OR_OK;
#pragma omp parallel for schedule(dynamic, 256)
  for (long i = 0; i < n; ++i) {
    long c = cell[i];
    long cc[3] = {c % g.nc[0], (c / g.nc[0]) % g.nc[1], c / (g.nc[0] * g.nc[1])};
    /* the distinct neighbouring cells along each axis */
    long nb[3][3];
    int nnb[3];
    for (int a = 0; a < 3; ++a) {
      nnb[a] = 0;
      for (int o = -1; o <= 1; ++o) {
        long t = cc[a] + o;
        if (b->periodic[a]) t = ((t % g.nc[a]) + g.nc[a]) % g.nc[a];
        else if (t < 0 || t >= g.nc[a]) continue;
        int dup = 0;
        for (int k = 0; k < nnb[a]; ++k) dup |= nb[a][k] == t;
        if (!dup) nb[a][nnb[a]++] = t;
      }
    }
    for (int z = 0; z < nnb[2]; ++z)
      for (int y = 0; y < nnb[1]; ++y)
        for (int x = 0; x < nnb[0]; ++x) {
          long q = nb[0][x] + g.nc[0] * (nb[1][y] + g.nc[1] * nb[2][z]);
          for (long k = head[q]; k < head[q + 1]; ++k) {
            long j = member[k];
            if (j == i) continue;
            int r = in_range(pos, b, i, j, rc2);
            if (r < 0) {
#pragma omp atomic write
              err = r;
            } else if (r) {
              list_push(&lists[i], j);
            }
          }
        }
    qsort(lists[i].j, (size_t)lists[i].m, sizeof(long), cmp_long);
  }
  free(cell);
  free(head);
  free(member);
  return err;
}

static int pairs_brute(long n, const double *pos, const or_box *b, double rc, or_list *lists) {
  double rc2 = rc * rc;
  int err = OR_OK;
#pragma omp parallel for schedule(dynamic, 64)
  for (long i = 0; i < n; ++i)
    for (long j = 0; j < n; ++j) {
      if (j == i) continue;
      int r = in_range(pos, b, i, j, rc2);
      if (r < 0) {
#pragma omp atomic write
        err = r;
      } else if (r) {
        list_push(&lists[i], j);
      }
    }
  return err;
}

/* Fill t with the pair set of cutoff rc; returns 0 or OR_E_OVERLAP. */
static int pairs_build(long n, const double *pos, const or_box *b, double rc, or_pairs *t) {
  or_list *lists = (or_list *)calloc((size_t)n, sizeof(or_list));
  int err = g_use_cells ? pairs_cells(n, pos, b, rc, lists) : pairs_brute(n, pos, b, rc, lists);
  t->n = n;
  t->start = (long *)malloc(sizeof(long) * (n + 1));
  t->start[0] = 0;
  for (long i = 0; i < n; ++i) t->start[i + 1] = t->start[i] + lists[i].m;
  t->idx = (long *)malloc(sizeof(long) * (t->start[n] > 0 ? t->start[n] : 1));
#pragma omp parallel for schedule(static)
  for (long i = 0; i < n; ++i) {
    if (lists[i].m) memcpy(t->idx + t->start[i], lists[i].j, sizeof(long) * lists[i].m);
    free(lists[i].j);
  }
  free(lists);
  if (err) pairs_free(t);
  return err;
}

/* Number of pairs of each atom (for tests of the two searches). */
int oracle_pair_counts(long n, const double *pos, const or_box *b, double rc, long *count, long *total_out) {
  if (n <= 0 || !pos || !b || !count) return OR_E_ARG;
  or_pairs t;
  int err = pairs_build(n, pos, b, rc, &t);
  if (err) return err;
  for (long i = 0; i < n; ++i) count[i] = t.start[i + 1] - t.start[i];
  if (total_out) *total_out = t.start[n];
  pairs_free(&t);
  return OR_OK;
}

/* The pair set itself: idx_out receives, atom after atom, each atom's
 * partners in increasing order (capacity cap entries; total_out the size). */
int oracle_pair_list(long n, const double *pos, const or_box *b, double rc, long cap, long *start_out,
                     long *idx_out, long *total_out) {
  if (n <= 0 || !pos || !b || !start_out) return OR_E_ARG;
  or_pairs t;
  int err = pairs_build(n, pos, b, rc, &t);
  if (err) return err;
  memcpy(start_out, t.start, sizeof(long) * (n + 1));
  if (total_out) *total_out = t.start[n];
  if (idx_out && t.start[n] <= cap) memcpy(idx_out, t.idx, sizeof(long) * t.start[n]);
  err = (idx_out && t.start[n] > cap) ? OR_E_ARG : OR_OK;
  pairs_free(&t);
  return err;
}

/* ------------------------------------------------------------ pair kernels */

/* Lennard-Jones: phi(r) = 4 eps [(s/r)^12 - (s/r)^6]; derivatives by r. */
static void lj_phi(const or_pot *p, double r, double *phi, double *d1, double *d2) {
  double sr = p->sigma / r;
  double s6 = pow(sr, 6.0), s12 = s6 * s6;
  *phi = 4.0 * p->eps * (s12 - s6);
  *d1 = 4.0 * p->eps * (-12.0 * s12 + 6.0 * s6) / r;
  *d2 = 4.0 * p->eps * (156.0 * s12 - 42.0 * s6) / (r * r);
}

/* Cubic smoothstep S(r): 1 below r_in, (1-s)^2 (1+2s) between, 0 above r_out. */
static void taper(const or_pot *p, double r, double *s0, double *s1, double *s2) {
  if (r <= p->r_in) {
    *s0 = 1.0; *s1 = 0.0; *s2 = 0.0;
    return;
  }
  if (r >= p->r_out) {
    *s0 = 0.0; *s1 = 0.0; *s2 = 0.0;
    return;
  }
  double w = p->r_out - p->r_in;
  double s = (r - p->r_in) / w;
  *s0 = (1.0 - s) * (1.0 - s) * (1.0 + 2.0 * s);
  *s1 = -6.0 * s * (1.0 - s) / w;
  *s2 = -6.0 * (1.0 - 2.0 * s) / (w * w);
}

/* Gupta pair term phi_t = A exp(-p (r/r0 - 1)) S(r), with first and second
 * derivatives by r. */
static void gupta_phi(const or_pot *p, double r, double *f0, double *f1, double *f2) {
  double s0, s1, s2;
  taper(p, r, &s0, &s1, &s2);
  double e = p->A * exp(-p->p * (r / p->r0 - 1.0));
  double k = -p->p / p->r0;
  *f0 = e * s0;
  *f1 = k * e * s0 + e * s1;
  *f2 = k * k * e * s0 + 2.0 * k * e * s1 + e * s2;
}

/* Gupta density term rho_t = exp(-2q (r/r0 - 1)) S(r) and derivatives. */
static void gupta_rho(const or_pot *p, double r, double *f0, double *f1, double *f2) {
  double s0, s1, s2;
  taper(p, r, &s0, &s1, &s2);
  double e = exp(-2.0 * p->q * (r / p->r0 - 1.0));
  double k = -2.0 * p->q / p->r0;
  *f0 = e * s0;
  *f1 = k * e * s0 + e * s1;
  *f2 = k * k * e * s0 + 2.0 * k * e * s1 + e * s2;
}

/* Embedding F(rho) = -xi sqrt(rho) and its derivatives; 0 for an empty
 * neighbourhood. */
static void embed(const or_pot *p, double rho, double *f0, double *f1, double *f2) {
  if (rho <= 0.0) {
    *f0 = 0.0; *f1 = 0.0; *f2 = 0.0;
    return;
  }
  double s = sqrt(rho);
  *f0 = -p->xi * s;
  *f1 = -0.5 * p->xi / s;
  *f2 = 0.25 * p->xi / (rho * s);
}

/* ------------------------------------------------- per-atom brute-force sums */

/* Density of atom i: sum over its pairs (all j != i inside r_out). */
static double gupta_density_atom(const double *pos, const or_box *b, const or_pot *p, const or_pairs *t, long i) {
  double rho = 0.0;
  for (long k = t->start[i]; k < t->start[i + 1]; ++k) {
    long j = t->idx[k];
    double d[3];
    min_image(pos + 3 * i, pos + 3 * j, b, d);
    double f0, f1, f2;
    gupta_rho(p, sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]), &f0, &f1, &f2);
    rho += f0;
  }
  return rho;
}

/* ------------------------------------------------- Stillinger-Weber (Si)
 *
 * E = sum_{i<j} phi2(r_ij) + sum_i sum_{j<k; j,k != i} h(r_ij, r_ik, theta_jik)
 *   phi2(r) = eps A [B (s/r)^p - (s/r)^q] exp(s / (r - a s))          r < a s
 *   h       = lambda eps (cos theta_jik + 1/3)^2 g(r_ij) g(r_ik)
 *   g(r)    = exp(gamma s / (r - a s))                                 r < a s
 * (s = sigma; every term vanishes smoothly at the cutoff a s). */

static void sw_phi2(const or_pot *p, double r, double *f0, double *f1) {
  double s = p->sigma, rc = p->sw_a * s;
  if (!(r < rc)) {
    *f0 = *f1 = 0.0;
    return;
  }
  double sr = s / r;
  double bp = p->sw_B * pow(sr, p->p), bq = pow(sr, p->q);
  double poly = bp - bq;
  double dpoly = (-p->p * bp + p->q * bq) / r;
  double ex = exp(s / (r - rc));
  double dex = -s / ((r - rc) * (r - rc)) * ex;
  *f0 = p->eps * p->A * poly * ex;
  *f1 = p->eps * p->A * (dpoly * ex + poly * dex);
}

static void sw_g(const or_pot *p, double r, double *g0, double *g1) {
  double s = p->sigma, rc = p->sw_a * s;
  if (!(r < rc)) {
    *g0 = *g1 = 0.0;
    return;
  }
  *g0 = exp(p->sw_gamma * s / (r - rc));
  *g1 = -p->sw_gamma * s / ((r - rc) * (r - rc)) * *g0;
}

/* Three-body term of the triplet centred at c with ends a and b, given
 * u = x_a - x_c and w = x_b - x_c (both shorter than the cutoff); returns h
 * and its gradients dh/du, dh/dw. */
static double sw_h(const or_pot *p, const double u[3], const double w[3], double dhu[3], double dhw[3]) {
  double ru = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  double rw = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
  double gu, gu1, gw, gw1;
  sw_g(p, ru, &gu, &gu1);
  sw_g(p, rw, &gw, &gw1);
  double c = (u[0] * w[0] + u[1] * w[1] + u[2] * w[2]) / (ru * rw);
  double t = c + 1.0 / 3.0;
  double le = p->sw_lambda * p->eps;
  for (int a = 0; a < 3; ++a) {
    double dcu = w[a] / (ru * rw) - c * u[a] / (ru * ru); /* d cos / du */
    double dcw = u[a] / (ru * rw) - c * w[a] / (rw * rw);
    dhu[a] = le * (2.0 * t * dcu * gu * gw + t * t * gu1 * (u[a] / ru) * gw);
    dhw[a] = le * (2.0 * t * dcw * gu * gw + t * t * gu * gw1 * (w[a] / rw));
  }
  return le * t * t * gu * gw;
}

typedef struct {
  long j;
  double d[3]; /* x_j - x_i, minimum image */
  double r;
} sw_nb;

/* Neighbours of atom i (its pairs), in index order, with x_j - x_i and r,
 * into *out (malloc'd, caller frees); returns the count. */
static long sw_neighbours(const double *pos, const or_box *b, const or_pairs *t, long i, sw_nb **out) {
  long m = t->start[i + 1] - t->start[i];
  sw_nb *l = (sw_nb *)malloc(sizeof(sw_nb) * (m > 0 ? m : 1));
  for (long k = 0; k < m; ++k) {
    long j = t->idx[t->start[i] + k];
    double d[3];
    min_image(pos + 3 * j, pos + 3 * i, b, d);
    l[k].j = j;
    l[k].d[0] = d[0];
    l[k].d[1] = d[1];
    l[k].d[2] = d[2];
    l[k].r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  }
  *out = l;
  return m;
}

/* F_i = -dE/dx_i collects every term that contains x_i: the pairs (i, j),
 * the triplets centred at i, and the triplets centred at a neighbour m of i
 * with i as one end.  e_i = 1/2 sum_j phi2 + the triplets centred at i. */
static void sw_atom_force(const double *pos, const or_box *b, const or_pot *p, const or_pairs *t, long i,
                          double f[3], double *e) {
  sw_nb *ni = NULL;
  long cnt = sw_neighbours(pos, b, t, i, &ni);
  double fi[3] = {0.0, 0.0, 0.0}, ei = 0.0;
  for (long a = 0; a < cnt; ++a) {
    double f0, f1;
    sw_phi2(p, ni[a].r, &f0, &f1);
    ei += 0.5 * f0;
    for (int k = 0; k < 3; ++k) fi[k] += f1 * ni[a].d[k] / ni[a].r;
  }
  for (long a = 0; a < cnt; ++a)
    for (long c = a + 1; c < cnt; ++c) {
      double dhu[3], dhw[3];
      ei += sw_h(p, ni[a].d, ni[c].d, dhu, dhw);
      for (int k = 0; k < 3; ++k) fi[k] += dhu[k] + dhw[k];
    }
  for (long a = 0; a < cnt; ++a) {
    long m = ni[a].j;
    sw_nb *nm = NULL;
    long cm = sw_neighbours(pos, b, t, m, &nm);
    double u[3] = {-ni[a].d[0], -ni[a].d[1], -ni[a].d[2]}; /* x_i - x_m */
    for (long c = 0; c < cm; ++c) {
      if (nm[c].j == i) continue;
      double dhu[3], dhw[3];
      sw_h(p, u, nm[c].d, dhu, dhw);
      for (int k = 0; k < 3; ++k) fi[k] -= dhu[k];
    }
    free(nm);
  }
  free(ni);
  f[0] = fi[0]; f[1] = fi[1]; f[2] = fi[2];
  *e = ei;
}

/* E straight from its definition for small systems: every pair i < j and
 * every triplet (i; j < k) by a plain triple loop, no neighbour lists. */
int oracle_sw_energy_direct(long n, const double *pos, const or_box *b, const or_pot *p, double *energy) {
  int rc = check_inputs(n, pos, b, p);
  if (rc) return rc;
  if (p->kind != OR_POT_SW) return OR_E_ARG;
  double cut = pot_cutoff(p);
  double E = 0.0;
  for (long i = 0; i < n; ++i)
    for (long j = i + 1; j < n; ++j) {
      double d[3], f0, f1;
      min_image(pos + 3 * j, pos + 3 * i, b, d);
      sw_phi2(p, sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]), &f0, &f1);
      E += f0;
    }
  for (long i = 0; i < n; ++i)
    for (long j = 0; j < n; ++j) {
      if (j == i) continue;
      double u[3];
      min_image(pos + 3 * j, pos + 3 * i, b, u);
      if (!(sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) < cut)) continue;
      for (long k = j + 1; k < n; ++k) {
        if (k == i) continue;
        double w[3], dhu[3], dhw[3];
        min_image(pos + 3 * k, pos + 3 * i, b, w);
        if (!(sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]) < cut)) continue;
        E += sw_h(p, u, w, dhu, dhw);
      }
    }
  *energy = E;
  return OR_OK;
}

/* Force and energy share of atom i from its pairs.  For Gupta, rho[] must
 * hold the densities of i and of its partners.  e_i: LJ 1/2 sum_j phi_s;
 * Gupta c_e sum_j phi_t + F(rho_i). */
static void atom_force(const double *pos, const or_box *b, const or_pot *p, const or_pairs *t, const double *rho,
                       long i, double f[3], double *e) {
  double fx = 0.0, fy = 0.0, fz = 0.0, ei = 0.0;
  if (p->kind == OR_POT_HARMONIC) {
    const double *x = pos + 3 * i;
    f[0] = -p->k[0] * x[0];
    f[1] = -p->k[1] * x[1];
    f[2] = -p->k[2] * x[2];
    *e = 0.5 * (p->k[0] * x[0] * x[0] + p->k[1] * x[1] * x[1] + p->k[2] * x[2] * x[2]);
    return;
  }
  if (p->kind == OR_POT_SW) {
    sw_atom_force(pos, b, p, t, i, f, e);
    return;
  }
  double shift = 0.0;
  if (p->kind == OR_POT_LJ) {
    double d1, d2;
    lj_phi(p, p->rc, &shift, &d1, &d2);
  }
  double cpair = (p->kind == OR_POT_GUPTA && p->convention == 0) ? 2.0 : 1.0;
  double epair = (p->kind == OR_POT_GUPTA && p->convention == 0) ? 1.0 : 0.5;
  double Fi0 = 0.0, Fi1 = 0.0, Fi2 = 0.0;
  if (p->kind == OR_POT_GUPTA) embed(p, rho[i], &Fi0, &Fi1, &Fi2);
  for (long k = t->start[i]; k < t->start[i + 1]; ++k) {
    long j = t->idx[k];
    double d[3];
    min_image(pos + 3 * i, pos + 3 * j, b, d);
    double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double dEdr; /* derivative of the energy terms coupling i and j along r_ij */
    if (p->kind == OR_POT_LJ) {
      double phi, d1, d2;
      lj_phi(p, r, &phi, &d1, &d2);
      ei += 0.5 * (phi - shift);
      dEdr = d1;
    } else {
      double ph0, ph1, ph2, rh0, rh1, rh2, Fj0, Fj1, Fj2;
      gupta_phi(p, r, &ph0, &ph1, &ph2);
      gupta_rho(p, r, &rh0, &rh1, &rh2);
      embed(p, rho[j], &Fj0, &Fj1, &Fj2);
      ei += epair * ph0;
      dEdr = cpair * ph1 + (Fi1 + Fj1) * rh1;
    }
    /* F_i = -dE/dx_i = -dE/dr * d/r */
    fx -= dEdr * d[0] / r;
    fy -= dEdr * d[1] / r;
    fz -= dEdr * d[2] / r;
  }
  if (p->kind == OR_POT_GUPTA) ei += Fi0;
  f[0] = fx; f[1] = fy; f[2] = fz;
  *e = ei;
}

static int has_pairs(const or_pot *p) { return p->kind != OR_POT_HARMONIC; }

/*
 * Energy and forces of the whole system.  forces: (n, 3) or NULL;
 * atom_energy: (n) or NULL; rho_out: (n) or NULL (Gupta densities).
 * Returns 0 or a negative error code.
 */
int oracle_energy_forces(long n, const double *pos, const or_box *b, const or_pot *p, double *energy,
                         double *forces, double *atom_energy, double *rho_out) {
  int rc = check_inputs(n, pos, b, p);
  if (rc) return rc;
  or_pairs t = {0, NULL, NULL};
  if (has_pairs(p)) {
    rc = pairs_build(n, pos, b, pot_cutoff(p), &t);
    if (rc) return rc;
  }
  double *rho = NULL;
  if (p->kind == OR_POT_GUPTA) {
    rho = (double *)malloc(sizeof(double) * n);
#pragma omp parallel for schedule(dynamic, 64)
    for (long i = 0; i < n; ++i) rho[i] = gupta_density_atom(pos, b, p, &t, i);
    if (rho_out) memcpy(rho_out, rho, sizeof(double) * n);
  }
  double *ebuf = (double *)malloc(sizeof(double) * n);
  double *fbuf = (double *)malloc(sizeof(double) * 3 * n);
#pragma omp parallel for schedule(dynamic, 64)
  for (long i = 0; i < n; ++i) atom_force(pos, b, p, &t, rho, i, fbuf + 3 * i, ebuf + i);
  double etot = 0.0;
  for (long i = 0; i < n; ++i) etot += ebuf[i];
  if (energy) *energy = etot;
  if (forces) memcpy(forces, fbuf, sizeof(double) * 3 * n);
  if (atom_energy) memcpy(atom_energy, ebuf, sizeof(double) * n);
  free(rho); free(ebuf); free(fbuf);
  pairs_free(&t);
  return OR_OK;
}

/* Pair lists of the atoms flagged in need[] only, each found by testing every
 * other atom (O(n) per flagged atom); the other atoms get empty lists. */
static int pairs_build_some(long n, const double *pos, const or_box *b, double rc, const char *need, or_pairs *t) {
  or_list *lists = (or_list *)calloc((size_t)n, sizeof(or_list));
  double rc2 = rc * rc;
  int err = OR_OK;
#pragma omp parallel for schedule(dynamic, 1)
  for (long i = 0; i < n; ++i) {
    if (!need[i]) continue;
    for (long j = 0; j < n; ++j) {
      if (j == i) continue;
      int r = in_range(pos, b, i, j, rc2);
      if (r < 0) {
#pragma omp atomic write
        err = r;
      } else if (r) {
        list_push(&lists[i], j);
      }
    }
  }
  t->n = n;
  t->start = (long *)malloc(sizeof(long) * (n + 1));
  t->start[0] = 0;
  for (long i = 0; i < n; ++i) t->start[i + 1] = t->start[i] + lists[i].m;
  t->idx = (long *)malloc(sizeof(long) * (t->start[n] > 0 ? t->start[n] : 1));
  for (long i = 0; i < n; ++i) {
    if (lists[i].m) memcpy(t->idx + t->start[i], lists[i].j, sizeof(long) * lists[i].m);
    free(lists[i].j);
  }
  free(lists);
  if (err) pairs_free(t);
  return err;
}

/*
 * Forces and energy shares of a sample of atoms, computed from their own
 * pairs in O(n) per atom (Gupta: also the densities of their partners, each
 * from that partner's pairs).  idx: (m); forces: (m, 3); atom_energy: (m) or
 * NULL.  The same sums as oracle_energy_forces for these atoms.
 */
int oracle_sample_forces(long n, const double *pos, const or_box *b, const or_pot *p, long m,
                         const long *idx, double *forces, double *atom_energy) {
  int rc = check_inputs(n, pos, b, p);
  if (rc) return rc;
  for (long s = 0; s < m; ++s)
    if (idx[s] < 0 || idx[s] >= n) return OR_E_ARG;
  char *need = (char *)calloc((size_t)n, 1);
  for (long s = 0; s < m; ++s) need[idx[s]] = 1;
  or_pairs t = {0, NULL, NULL};
  double *rho = NULL;
  if (has_pairs(p)) {
    rc = pairs_build_some(n, pos, b, pot_cutoff(p), need, &t);
    if (!rc && (p->kind == OR_POT_GUPTA || p->kind == OR_POT_SW)) {
      /* the partners' densities (Gupta) or lists (Stillinger-Weber) too */
      for (long s = 0; s < m; ++s)
        for (long k = t.start[idx[s]]; k < t.start[idx[s] + 1]; ++k) need[t.idx[k]] = 1;
      pairs_free(&t);
      rc = pairs_build_some(n, pos, b, pot_cutoff(p), need, &t);
    }
  }
  if (rc) {
    free(need);
    return rc;
  }
  if (p->kind == OR_POT_GUPTA) {
    rho = (double *)calloc((size_t)n, sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < n; ++i)
      if (need[i]) rho[i] = gupta_density_atom(pos, b, p, &t, i);
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (long s = 0; s < m; ++s) {
    double ei;
    atom_force(pos, b, p, &t, rho, idx[s], forces + 3 * s, &ei);
    if (atom_energy) atom_energy[s] = ei;
  }
  free(rho);
  free(need);
  pairs_free(&t);
  return OR_OK;
}

/* ----------------------------------------------------------- Hessian * u */

/* Pair-block action: for a pair potential g(r) with derivatives g1, g2 along
 * d = x_i - x_j, the Hessian block applied to w = u_i - u_j is
 * g2 (dh.w) dh + (g1 / r) (w - (dh.w) dh). */
static void pair_block(double g1, double g2, double r, const double dh[3], const double w[3], double out[3]) {
  double dw = dh[0] * w[0] + dh[1] * w[1] + dh[2] * w[2];
  for (int a = 0; a < 3; ++a) out[a] = g2 * dw * dh[a] + (g1 / r) * (w[a] - dw * dh[a]);
}

/*
 * Analytic Hessian-vector product Hu = (d^2 E / dx dx) u.  u, hu: (n, 3).
 */
int oracle_hvp(long n, const double *pos, const double *u, const or_box *b, const or_pot *p, double *hu) {
  int rc = check_inputs(n, pos, b, p);
  if (rc) return rc;
  if (p->kind == OR_POT_SW) return OR_E_ARG; /* pair potentials and the well only */
  if (p->kind == OR_POT_HARMONIC) {
    for (long i = 0; i < n; ++i)
      for (int a = 0; a < 3; ++a) hu[3 * i + a] = p->k[a] * u[3 * i + a];
    return OR_OK;
  }
  or_pairs t;
  rc = pairs_build(n, pos, b, pot_cutoff(p), &t);
  if (rc) return rc;
  double *rho = NULL, *s = NULL;
  if (p->kind == OR_POT_GUPTA) {
    rho = (double *)malloc(sizeof(double) * n);
    s = (double *)malloc(sizeof(double) * n);
    /* rho_i and s_i = d rho_i / d eps along u = sum_j rho'(r_ij) dh_ij . (u_i - u_j) */
#pragma omp parallel for schedule(dynamic, 64)
    for (long i = 0; i < n; ++i) {
      double ri = 0.0, si = 0.0;
      for (long k = t.start[i]; k < t.start[i + 1]; ++k) {
        long j = t.idx[k];
        double d[3];
        min_image(pos + 3 * i, pos + 3 * j, b, d);
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]), f0, f1, f2;
        gupta_rho(p, r, &f0, &f1, &f2);
        ri += f0;
        double w = 0.0;
        for (int a = 0; a < 3; ++a) w += (d[a] / r) * (u[3 * i + a] - u[3 * j + a]);
        si += f1 * w;
      }
      rho[i] = ri;
      s[i] = si;
    }
  }
  double cpair = (p->kind == OR_POT_GUPTA && p->convention == 0) ? 2.0 : 1.0;
#pragma omp parallel for schedule(dynamic, 64)
  for (long i = 0; i < n; ++i) {
    double acc[3] = {0.0, 0.0, 0.0};
    double Fi0 = 0, Fi1 = 0, Fi2 = 0;
    if (p->kind == OR_POT_GUPTA) embed(p, rho[i], &Fi0, &Fi1, &Fi2);
    for (long k = t.start[i]; k < t.start[i + 1]; ++k) {
      long j = t.idx[k];
      double d[3];
      min_image(pos + 3 * i, pos + 3 * j, b, d);
      double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      double dh[3] = {d[0] / r, d[1] / r, d[2] / r};
      double w[3] = {u[3 * i] - u[3 * j], u[3 * i + 1] - u[3 * j + 1], u[3 * i + 2] - u[3 * j + 2]};
      double out[3];
      if (p->kind == OR_POT_LJ) {
        double phi, d1, d2;
        lj_phi(p, r, &phi, &d1, &d2);
        pair_block(d1, d2, r, dh, w, out);
        for (int a = 0; a < 3; ++a) acc[a] += out[a];
      } else {
        double ph0, ph1, ph2, rh0, rh1, rh2, Fj0, Fj1, Fj2;
        gupta_phi(p, r, &ph0, &ph1, &ph2);
        gupta_rho(p, r, &rh0, &rh1, &rh2);
        embed(p, rho[j], &Fj0, &Fj1, &Fj2);
        /* pair part */
        pair_block(cpair * ph1, cpair * ph2, r, dh, w, out);
        for (int a = 0; a < 3; ++a) acc[a] += out[a];
        /* embedding part: (F'_i + F'_j) B_rho w + (F''_i s_i + F''_j s_j) rho' dh */
        pair_block((Fi1 + Fj1) * rh1, (Fi1 + Fj1) * rh2, r, dh, w, out);
        double c = (Fi2 * s[i] + Fj2 * s[j]) * rh1;
        for (int a = 0; a < 3; ++a) acc[a] += out[a] + c * dh[a];
      }
    }
    hu[3 * i] = acc[0];
    hu[3 * i + 1] = acc[1];
    hu[3 * i + 2] = acc[2];
  }
  free(rho);
  free(s);
  pairs_free(&t);
  return OR_OK;
}

/* -------------------------------------------------------------- FIRE 2.0 */

typedef struct {
  double dt_start, tmax, tmin, dtgrow, dtshrink, alpha0, alphashrink, f2a;
  int delaystep, vdfmax, halfstepback, initialdelay;
  int integrator; /* 0 semi-implicit Euler, 1 explicit Euler, 2 velocity Verlet */
  int criterion;  /* 0 max per-atom |F_i|, 1 Euclidean norm of the 3N force vector */
  int variant;    /* 0 FIRE 2.0 (Algorithm 2), 1 original FIRE (Algorithm 1) */
  int pad;
  double dmax;    /* > 0: largest displacement of any atom in one drift (see drift()) */
} or_fire;

typedef struct {
  int stop; /* 1 converged, 2 max steps, 3 MAXVDOTF, <0 error */
  long iterations, force_evals;
  double energy, fmax, f2norm, dt, alpha;
  long n_pos, n_neg;
} or_result;

#define OR_STOP_CONVERGED 1
#define OR_STOP_MAX_STEPS 2
#define OR_STOP_MAXVDOTF 3

#define OR_TRACE_COLS 9

static double dot3n(long n, const double *a, const double *b) {
  double s = 0.0;
  for (long i = 0; i < 3 * n; ++i) s += a[i] * b[i];
  return s;
}

static double max_atom_norm(long n, const double *f) {
  double m = 0.0;
  for (long i = 0; i < n; ++i) {
    double t = sqrt(f[3 * i] * f[3 * i] + f[3 * i + 1] * f[3 * i + 1] + f[3 * i + 2] * f[3 * i + 2]);
    if (t > m) m = t;
  }
  return m;
}

/* v <- (1 - alpha) v + alpha |v| F / |F|  (the FIRE mixing of Sec. 2.1) */
static void mix(long n, double *v, const double *f, double alpha) {
  double vn = sqrt(dot3n(n, v, v)), fn = sqrt(dot3n(n, f, f));
  if (fn == 0.0) return;
  for (long i = 0; i < 3 * n; ++i) v[i] = (1.0 - alpha) * v[i] + alpha * vn * f[i] / fn;
}

/* Frozen degrees of freedom (bit d of frozen[i] set: component d of atom i)
 * have their force held at zero, so FIRE never moves them (the frozen borders
 * of the test cases in Sec. 5.3). */
static void apply_frozen(long n, double *f, const unsigned char *frozen) {
  if (!frozen) return;
  for (long i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d)
      if (frozen[i] & (1 << d)) f[3 * i + d] = 0.0;
}

/* The step length a move x += c dt v may use.  Without dmax it is dt.  With
 * dmax (the maximum atomic displacement per step the paper's melt case
 * needed, Sec. 5.3; the paper names the setting but not its mechanism) it is
 * shortened so that the fastest atom moves at most dmax per full step:
 * min(dt, dmax / max_i |v_i|), with v the velocity of that move.  It applies
 * to the drift and to the half step back (half of such a step); dt itself,
 * the FIRE state and the kicks are unchanged. */
static double capped_step(long n, const double *v, double dt, double dmax) {
  if (!(dmax > 0.0)) return dt;
  double vmax2 = 0.0;
  for (long i = 0; i < n; ++i) {
    double s = v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] + v[3 * i + 2] * v[3 * i + 2];
    if (s > vmax2) vmax2 = s;
  }
  double vmax = sqrt(vmax2);
  return vmax * dt > dmax ? dmax / vmax : dt;
}

static void drift(long n, double *pos, const double *v, double dt, double dmax) {
  double dtx = capped_step(n, v, dt, dmax);
  for (long k = 0; k < 3 * n; ++k) pos[k] += dtx * v[k];
}

/* The kick of one component: v += (c s_i) F with c the step's kick factor
 * (dt f2a, or half of it) and s_i = 1 / m_i the atom's inverse mass relative
 * to the mass f2a implies (1 without a mass array). */
static void kick(long n, double *v, const double *f, double c, const double *inv_mass) {
  for (long k = 0; k < 3 * n; ++k) v[k] += (inv_mass ? c * inv_mass[k / 3] : c) * f[k];
}

/* The FIRE state carried from one iteration to the next. */
typedef struct {
  double dt, alpha;
  long npos; /* consecutive iterations with P > 0 */
  long nneg; /* consecutive iterations with P <= 0 (counted by FIRE 2.0 only) */
} or_state;

/* What the sign of the power P = F.v decides at the start of an iteration. */
typedef struct {
  int uphill;       /* P <= 0: the velocities restart from zero */
  int stop;         /* FIRE 2.0: one uphill step more than allowed (MAXVDOTF) */
  double alpha_mix; /* FIRE: weight of the mixing done before the MD step, the alpha
                       in force before this iteration's decay */
} or_adapt;

/* Adapt dt, alpha and the counters to P at iteration i (Sec. 2.1 for FIRE,
 * Sec. 3.2 and Table 1 for FIRE 2.0).
 *   Downhill (P > 0): one more downhill step in a row; once there have been
 *   more than N_delay of them, dt grows by f_inc (capped at dt_max) and
 *   alpha decays by f_alpha.
 *   Uphill (P <= 0): the downhill count restarts and alpha returns to
 *   alpha_start as dt shrinks by f_dec.  FIRE 2.0 also counts uphill steps
 *   in a row (beyond N_{P<=0,max} the run stops), leaves dt and alpha alone
 *   during the initial delay (i < N_delay with initialdelay), and keeps dt
 *   if shrinking would take it below dt_min (alpha still resets). */
static or_adapt fire_adapt(const or_fire *fp, or_state *s, double P, long i) {
  or_adapt a = {0, 0, s->alpha};
  int fire2 = fp->variant == 0;
  if (P > 0.0) {
    s->npos += 1;
    if (fire2) s->nneg = 0;
    if (s->npos > fp->delaystep) {
      s->dt = fmin(s->dt * fp->dtgrow, fp->tmax * fp->dt_start);
      s->alpha *= fp->alphashrink;
    }
    return a;
  }
  a.uphill = 1;
  s->npos = 0;
  if (!fire2) {
    s->dt *= fp->dtshrink;
    s->alpha = fp->alpha0;
    return a;
  }
  s->nneg += 1;
  if (s->nneg > fp->vdfmax) {
    a.stop = 1;
    return a;
  }
  int in_initial_delay = fp->initialdelay && i < fp->delaystep;
  if (!in_initial_delay) {
    if (s->dt * fp->dtshrink >= fp->tmin * fp->dt_start) s->dt *= fp->dtshrink;
    s->alpha = fp->alpha0;
  }
  return a;
}

/* One MD step from (x, v, F) with step dt (kick factor dtf = dt f2a), the
 * FIRE mixing with weight alpha placed where each integrator puts it
 * (alpha < 0: no mixing), ending with the new force in f and energy in *E:
 *   semi-implicit Euler (Algorithm 4): kick, mix, drift, force;
 *   explicit Euler (Algorithm 3): mix, drift with that v, kick with the old
 *     force, force;
 *   velocity Verlet (Algorithm 6): half kick, mix, drift, force, half kick
 *     with the new force. */
static int md_step(long n, double *pos, double *v, double *f, double *fnew, double *E, const or_box *b,
                   const or_pot *p, const or_fire *fp, const unsigned char *frozen, const double *inv_mass,
                   double dt, double alpha) {
  double dtf = dt * fp->f2a;
  int rc;
  if (fp->integrator == 0) {
    kick(n, v, f, dtf, inv_mass);
    if (alpha >= 0.0) mix(n, v, f, alpha);
    drift(n, pos, v, dt, fp->dmax);
    rc = oracle_energy_forces(n, pos, b, p, E, f, NULL, NULL);
    apply_frozen(n, f, frozen);
  } else if (fp->integrator == 1) {
    if (alpha >= 0.0) mix(n, v, f, alpha);
    drift(n, pos, v, dt, fp->dmax);
    kick(n, v, f, dtf, inv_mass);
    rc = oracle_energy_forces(n, pos, b, p, E, f, NULL, NULL);
    apply_frozen(n, f, frozen);
  } else {
    kick(n, v, f, 0.5 * dtf, inv_mass);
    if (alpha >= 0.0) mix(n, v, f, alpha);
    drift(n, pos, v, dt, fp->dmax);
    rc = oracle_energy_forces(n, pos, b, p, E, fnew, NULL, NULL);
    memcpy(f, fnew, sizeof(double) * 3 * n);
    apply_frozen(n, f, frozen);
    kick(n, v, f, 0.5 * dtf, inv_mass);
  }
  return rc;
}

static double criterion_value(const or_fire *fp, long n, const double *f) {
  return fp->criterion == 0 ? max_atom_norm(n, f) : sqrt(dot3n(n, f, f));
}

static void trace_row(double *t, long i, double E, long n, const double *f, double P, const or_state *s,
                      int branch) {
  t[0] = (double)i;
  t[1] = E;
  t[2] = max_atom_norm(n, f);
  t[3] = sqrt(dot3n(n, f, f));
  t[4] = P;
  t[5] = s->dt;
  t[6] = s->alpha;
  t[7] = branch;
  t[8] = (double)s->npos;
}

/*
 * Minimise E from pos (in/out) with FIRE 2.0 (Algorithm 2) or FIRE
 * (Algorithm 1).  Each iteration: the power P = F.v decides the adaptation
 * (fire_adapt); uphill, FIRE 2.0 first moves the atoms back by half a step
 * of the just-adapted dt (halfstepback) and both zero v; FIRE mixes v
 * toward F here when downhill; then one MD step (md_step, where FIRE 2.0
 * mixes) and the convergence test on the new force.  tol applies to the
 * chosen criterion with a strict "<".  trace (nullable) receives one row per
 * iteration i = 0..it: {i, E, fmax, f2norm, P, dt, alpha,
 * branch(+1 P>0 / -1 P<=0 / 0 initial), n_pos} where E, fmax, f2norm are
 * those after the force evaluation of row i, and P, dt, alpha, branch are
 * those that led to it.  vel_out (nullable): final v.
 */
int oracle_fire_minimize_ex(long n, double *pos, const or_box *b, const or_pot *p, const or_fire *fp,
                            const unsigned char *frozen, const double *mass, double tol, long max_steps,
                            or_result *res, double *trace, double *vel_out) {
  int rc = check_inputs(n, pos, b, p);
  if (rc) return rc;
  double *inv_mass = NULL;
  if (mass) {
    inv_mass = (double *)malloc(sizeof(double) * n);
    for (long i = 0; i < n; ++i) {
      if (!(mass[i] > 0.0) || !isfinite(mass[i])) {
        free(inv_mass);
        return OR_E_ARG;
      }
      inv_mass[i] = 1.0 / mass[i];
    }
  }
  double *v = (double *)calloc((size_t)(3 * n), sizeof(double));
  double *f = (double *)malloc(sizeof(double) * 3 * n);
  double *fnew = (double *)malloc(sizeof(double) * 3 * n);
  double E;
  long evals = 0;
  or_state st = {fp->dt_start, fp->alpha0, 0, 0};
  memset(res, 0, sizeof(*res));

  rc = oracle_energy_forces(n, pos, b, p, &E, f, NULL, NULL);
  evals++;
  if (rc) goto done;
  apply_frozen(n, f, frozen);
  if (trace) trace_row(trace, 0, E, n, f, 0.0, &st, 0);

  int stop = criterion_value(fp, n, f) < tol ? OR_STOP_CONVERGED : 0;
  long it = 0;
  for (long i = 1; i <= max_steps && !stop; ++i) {
    double P = dot3n(n, f, v);
    or_adapt ad = fire_adapt(fp, &st, P, i);
    if (ad.stop) {
      stop = OR_STOP_MAXVDOTF;
      break;
    }
    if (ad.uphill) {
      if (fp->variant == 0 && fp->halfstepback) {
        double dth = capped_step(n, v, st.dt, fp->dmax);
        for (long k = 0; k < 3 * n; ++k) pos[k] -= 0.5 * dth * v[k];
      }
      memset(v, 0, sizeof(double) * 3 * n);
    } else if (fp->variant == 1) {
      mix(n, v, f, ad.alpha_mix);
    }
    rc = md_step(n, pos, v, f, fnew, &E, b, p, fp, frozen, inv_mass, st.dt, fp->variant == 0 ? st.alpha : -1.0);
    evals++;
    it = i;
    if (rc) goto done;
    if (trace) trace_row(trace + OR_TRACE_COLS * i, i, E, n, f, P, &st, ad.uphill ? -1 : 1);
    if (criterion_value(fp, n, f) < tol) stop = OR_STOP_CONVERGED;
  }
  if (!stop) stop = OR_STOP_MAX_STEPS;
  res->stop = stop;
  res->iterations = it;
  res->force_evals = evals;
  res->energy = E;
  res->fmax = max_atom_norm(n, f);
  res->f2norm = sqrt(dot3n(n, f, f));
  res->dt = st.dt;
  res->alpha = st.alpha;
  res->n_pos = st.npos;
  res->n_neg = st.nneg;
  if (vel_out) memcpy(vel_out, v, sizeof(double) * 3 * n);
done:
  free(v);
  free(f);
  free(fnew);
  free(inv_mass);
  return rc;
}

int oracle_fire_minimize(long n, double *pos, const or_box *b, const or_pot *p, const or_fire *fp, double tol,
                         long max_steps, or_result *res, double *trace, double *vel_out) {
  return oracle_fire_minimize_ex(n, pos, b, p, fp, NULL, NULL, tol, max_steps, res, trace, vel_out);
}
