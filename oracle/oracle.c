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
 *     by brute force over every atom pair under the minimum image; each atom's
 *     sums run over all other atoms in index order (no cell list, no pruning),
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

/* Density of atom i: sum over all j != i inside r_out. */
static int gupta_density_atom(long n, const double *pos, const or_box *b, const or_pot *p, long i,
                              double *rho_out) {
  double rc2 = p->r_out * p->r_out, rho = 0.0;
  for (long j = 0; j < n; ++j) {
    if (j == i) continue;
    double d[3];
    min_image(pos + 3 * i, pos + 3 * j, b, d);
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (r2 == 0.0) return OR_E_OVERLAP;
    if (r2 < rc2) {
      double f0, f1, f2;
      gupta_rho(p, sqrt(r2), &f0, &f1, &f2);
      rho += f0;
    }
  }
  *rho_out = rho;
  return OR_OK;
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

/* Neighbours of atom i closer than the cutoff, in index order, into *out
 * (malloc'd, caller frees); returns the count or a negative error code. */
static long sw_neighbours(long n, const double *pos, const or_box *b, const or_pot *p, long i, sw_nb **out) {
  double rc = pot_cutoff(p), rc2 = rc * rc;
  long cap = 16, m = 0;
  sw_nb *l = (sw_nb *)malloc(sizeof(sw_nb) * cap);
  for (long j = 0; j < n; ++j) {
    if (j == i) continue;
    double d[3];
    min_image(pos + 3 * j, pos + 3 * i, b, d);
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (r2 == 0.0) {
      free(l);
      return OR_E_OVERLAP;
    }
    if (!(r2 < rc2)) continue;
    if (m == cap) {
      cap *= 2;
      l = (sw_nb *)realloc(l, sizeof(sw_nb) * cap);
    }
    l[m].j = j;
    l[m].d[0] = d[0];
    l[m].d[1] = d[1];
    l[m].d[2] = d[2];
    l[m].r = sqrt(r2);
    ++m;
  }
  *out = l;
  return m;
}

/* F_i = -dE/dx_i collects every term that contains x_i: the pairs (i, j),
 * the triplets centred at i, and the triplets centred at a neighbour m of i
 * with i as one end.  e_i = 1/2 sum_j phi2 + the triplets centred at i. */
static int sw_atom_force(long n, const double *pos, const or_box *b, const or_pot *p, long i, double f[3],
                         double *e) {
  sw_nb *ni = NULL;
  long cnt = sw_neighbours(n, pos, b, p, i, &ni);
  if (cnt < 0) return (int)cnt;
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
  int err = OR_OK;
  for (long a = 0; a < cnt && !err; ++a) {
    long m = ni[a].j;
    sw_nb *nm = NULL;
    long cm = sw_neighbours(n, pos, b, p, m, &nm);
    if (cm < 0) {
      err = (int)cm;
      break;
    }
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
  return err;
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

/* Force and energy share of atom i.  For Gupta, rho[] must hold all
 * densities.  e_i: LJ 1/2 sum_j phi_s; Gupta c_e sum_j phi_t + F(rho_i). */
static int atom_force(long n, const double *pos, const or_box *b, const or_pot *p, const double *rho,
                      long i, double f[3], double *e) {
  double fx = 0.0, fy = 0.0, fz = 0.0, ei = 0.0;
  if (p->kind == OR_POT_HARMONIC) {
    const double *x = pos + 3 * i;
    f[0] = -p->k[0] * x[0];
    f[1] = -p->k[1] * x[1];
    f[2] = -p->k[2] * x[2];
    *e = 0.5 * (p->k[0] * x[0] * x[0] + p->k[1] * x[1] * x[1] + p->k[2] * x[2] * x[2]);
    return OR_OK;
  }
  if (p->kind == OR_POT_SW) return sw_atom_force(n, pos, b, p, i, f, e);
  double rc = pot_cutoff(p), rc2 = rc * rc;
  double shift = 0.0;
  if (p->kind == OR_POT_LJ) {
    double d1, d2;
    lj_phi(p, p->rc, &shift, &d1, &d2);
  }
  double cpair = (p->kind == OR_POT_GUPTA && p->convention == 0) ? 2.0 : 1.0;
  double epair = (p->kind == OR_POT_GUPTA && p->convention == 0) ? 1.0 : 0.5;
  double Fi0 = 0.0, Fi1 = 0.0, Fi2 = 0.0;
  if (p->kind == OR_POT_GUPTA) embed(p, rho[i], &Fi0, &Fi1, &Fi2);
  for (long j = 0; j < n; ++j) {
    if (j == i) continue;
    double d[3];
    min_image(pos + 3 * i, pos + 3 * j, b, d);
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (r2 == 0.0) return OR_E_OVERLAP;
    if (!(r2 < rc2)) continue;
    double r = sqrt(r2);
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
  return OR_OK;
}

/*
 * Energy and forces of the whole system.  forces: (n, 3) or NULL;
 * atom_energy: (n) or NULL; rho_out: (n) or NULL (Gupta densities).
 * Returns 0 or a negative error code.
 */
int oracle_energy_forces(long n, const double *pos, const or_box *b, const or_pot *p, double *energy,
                         double *forces, double *atom_energy, double *rho_out) {
  int rc = check_inputs(n, pos, b, p);
  if (rc) return rc;
  double *rho = NULL;
  int err = OR_OK;
  if (p->kind == OR_POT_GUPTA) {
    rho = (double *)malloc(sizeof(double) * n);
    if (!rho) return OR_E_ARG;
#pragma omp parallel for schedule(dynamic, 64)
    for (long i = 0; i < n; ++i) {
      int e = gupta_density_atom(n, pos, b, p, i, &rho[i]);
      if (e) {
#pragma omp atomic write
        err = e;
      }
    }
    if (err) {
      free(rho);
      return err;
    }
    if (rho_out) memcpy(rho_out, rho, sizeof(double) * n);
  }
  double *ebuf = (double *)malloc(sizeof(double) * n);
  double *fbuf = (double *)malloc(sizeof(double) * 3 * n);
  if (!ebuf || !fbuf) {
    free(rho); free(ebuf); free(fbuf);
    return OR_E_ARG;
  }
#pragma omp parallel for schedule(dynamic, 64)
  for (long i = 0; i < n; ++i) {
    int e = atom_force(n, pos, b, p, rho, i, fbuf + 3 * i, ebuf + i);
    if (e) {
#pragma omp atomic write
      err = e;
    }
  }
  if (!err) {
    double etot = 0.0;
    for (long i = 0; i < n; ++i) etot += ebuf[i];
    if (energy) *energy = etot;
    if (forces) memcpy(forces, fbuf, sizeof(double) * 3 * n);
    if (atom_energy) memcpy(atom_energy, ebuf, sizeof(double) * n);
  }
  free(rho); free(ebuf); free(fbuf);
  return err;
}

/*
 * Forces and energy shares of a sample of atoms, each computed on its own in
 * O(n) (Gupta: O(n * neighbours), for the densities of atom i and of its
 * neighbours).  idx: (m); forces: (m, 3); atom_energy: (m) or NULL.
 */
int oracle_sample_forces(long n, const double *pos, const or_box *b, const or_pot *p, long m,
                         const long *idx, double *forces, double *atom_energy) {
  int rc = check_inputs(n, pos, b, p);
  if (rc) return rc;
  int err = OR_OK;
  double rcut = pot_cutoff(p), rc2 = rcut * rcut;
#pragma omp parallel for schedule(dynamic, 1)
  for (long s = 0; s < m; ++s) {
    long i = idx[s];
    double *rho = NULL;
    if (p->kind == OR_POT_GUPTA) {
      /* a full density array is the plainest way to serve atom_force; only the
       * entries of i and of its neighbours are filled in */
      rho = (double *)calloc((size_t)n, sizeof(double));
      int e = gupta_density_atom(n, pos, b, p, i, &rho[i]);
      for (long j = 0; j < n && !e; ++j) {
        if (j == i) continue;
        double d[3];
        min_image(pos + 3 * i, pos + 3 * j, b, d);
        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (r2 < rc2) e = gupta_density_atom(n, pos, b, p, j, &rho[j]);
      }
      if (e) {
#pragma omp atomic write
        err = e;
      }
    }
    double ei;
    int e = atom_force(n, pos, b, p, rho, i, forces + 3 * s, &ei);
    if (atom_energy) atom_energy[s] = ei;
    if (e) {
#pragma omp atomic write
      err = e;
    }
    free(rho);
  }
  return err;
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
  double rcut = pot_cutoff(p), rc2 = rcut * rcut;
  double *rho = NULL, *s = NULL;
  int err = OR_OK;
  if (p->kind == OR_POT_GUPTA) {
    rho = (double *)malloc(sizeof(double) * n);
    s = (double *)malloc(sizeof(double) * n);
    /* rho_i and s_i = d rho_i / d eps along u = sum_j rho'(r_ij) dh_ij . (u_i - u_j) */
#pragma omp parallel for schedule(dynamic, 64)
    for (long i = 0; i < n; ++i) {
      double ri = 0.0, si = 0.0;
      for (long j = 0; j < n; ++j) {
        if (j == i) continue;
        double d[3];
        min_image(pos + 3 * i, pos + 3 * j, b, d);
        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (r2 == 0.0) {
#pragma omp atomic write
          err = OR_E_OVERLAP;
          continue;
        }
        if (!(r2 < rc2)) continue;
        double r = sqrt(r2), f0, f1, f2;
        gupta_rho(p, r, &f0, &f1, &f2);
        ri += f0;
        double w = 0.0;
        for (int a = 0; a < 3; ++a) w += (d[a] / r) * (u[3 * i + a] - u[3 * j + a]);
        si += f1 * w;
      }
      rho[i] = ri;
      s[i] = si;
    }
    if (err) {
      free(rho); free(s);
      return err;
    }
  }
  double shift = 0.0;
  (void)shift;
  double cpair = (p->kind == OR_POT_GUPTA && p->convention == 0) ? 2.0 : 1.0;
#pragma omp parallel for schedule(dynamic, 64)
  for (long i = 0; i < n; ++i) {
    double acc[3] = {0.0, 0.0, 0.0};
    double Fi0 = 0, Fi1 = 0, Fi2 = 0;
    if (p->kind == OR_POT_GUPTA) embed(p, rho[i], &Fi0, &Fi1, &Fi2);
    for (long j = 0; j < n; ++j) {
      if (j == i) continue;
      double d[3];
      min_image(pos + 3 * i, pos + 3 * j, b, d);
      double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      if (r2 == 0.0 || !(r2 < rc2)) continue;
      double r = sqrt(r2);
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
  return err;
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

/*
 * Minimise E from pos (in/out).  tol applies to the chosen criterion with a
 * strict "<".  trace (nullable) receives one row per iteration i = 0..it:
 * {i, E, fmax, f2norm, P, dt, alpha, branch(+1 P>0 / -1 P<=0 / 0 initial), n_pos}
 * where E, fmax, f2norm are those after the force evaluation of row i, and P,
 * dt, alpha, branch are those that led to it.  vel_out (nullable): final v.
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
  double alpha = fp->alpha0, dt = fp->dt_start;
  double dtmax = fp->tmax * fp->dt_start, dtmin = fp->tmin * fp->dt_start;
  long npos = 0, nneg = 0;
  memset(res, 0, sizeof(*res));

  rc = oracle_energy_forces(n, pos, b, p, &E, f, NULL, NULL);
  evals++;
  if (rc) goto done;
  apply_frozen(n, f, frozen);

#define CRIT() (fp->criterion == 0 ? max_atom_norm(n, f) : sqrt(dot3n(n, f, f)))
  if (trace) {
    double *t = trace;
    t[0] = 0; t[1] = E; t[2] = max_atom_norm(n, f); t[3] = sqrt(dot3n(n, f, f));
    t[4] = 0; t[5] = dt; t[6] = alpha; t[7] = 0; t[8] = 0;
  }
  int stop = 0;
  long it = 0;
  if (CRIT() < tol) stop = OR_STOP_CONVERGED;
  for (long i = 1; i <= max_steps && !stop; ++i) {
    double P = dot3n(n, f, v);
    int branch;
    if (fp->variant == 0) {
      /* Algorithm 2 */
      if (P > 0.0) {
        branch = 1;
        npos += 1;
        nneg = 0;
        if (npos > fp->delaystep) {
          dt = fmin(dt * fp->dtgrow, dtmax);
          alpha *= fp->alphashrink;
        }
      } else {
        branch = -1;
        npos = 0;
        nneg += 1;
        if (nneg > fp->vdfmax) {
          stop = OR_STOP_MAXVDOTF;
          break;
        }
        if (!(fp->initialdelay && i < fp->delaystep)) {
          if (dt * fp->dtshrink >= dtmin) dt *= fp->dtshrink;
          alpha = fp->alpha0;
        }
        if (fp->halfstepback) {
          double dth = capped_step(n, v, dt, fp->dmax);
          for (long k = 0; k < 3 * n; ++k) pos[k] -= 0.5 * dth * v[k];
        }
        memset(v, 0, sizeof(double) * 3 * n);
      }
    } else {
      /* Algorithm 1: mixing at the start of a P > 0 step, plain shrink */
      if (P > 0.0) {
        branch = 1;
        npos += 1;
        mix(n, v, f, alpha);
        if (npos > fp->delaystep) {
          dt = fmin(dt * fp->dtgrow, dtmax);
          alpha *= fp->alphashrink;
        }
      } else {
        branch = -1;
        npos = 0;
        memset(v, 0, sizeof(double) * 3 * n);
        dt *= fp->dtshrink;
        alpha = fp->alpha0;
      }
    }
    double dtf = dt * fp->f2a;
    int mixing = (fp->variant == 0);
    if (fp->integrator == 0) {
      /* Algorithm 4: kick, mix, drift */
      kick(n, v, f, dtf, inv_mass);
      if (mixing) mix(n, v, f, alpha);
      drift(n, pos, v, dt, fp->dmax);
      rc = oracle_energy_forces(n, pos, b, p, &E, f, NULL, NULL);
      apply_frozen(n, f, frozen);
    } else if (fp->integrator == 1) {
      /* Algorithm 3: mix, drift with the old v, kick with the old force */
      if (mixing) mix(n, v, f, alpha);
      drift(n, pos, v, dt, fp->dmax);
      kick(n, v, f, dtf, inv_mass);
      rc = oracle_energy_forces(n, pos, b, p, &E, f, NULL, NULL);
      apply_frozen(n, f, frozen);
    } else {
      /* Algorithm 6: half kick, mix, drift, force, half kick */
      kick(n, v, f, 0.5 * dtf, inv_mass);
      if (mixing) mix(n, v, f, alpha);
      drift(n, pos, v, dt, fp->dmax);
      rc = oracle_energy_forces(n, pos, b, p, &E, fnew, NULL, NULL);
      memcpy(f, fnew, sizeof(double) * 3 * n);
      apply_frozen(n, f, frozen);
      kick(n, v, f, 0.5 * dtf, inv_mass);
    }
    evals++;
    it = i;
    if (rc) goto done;
    if (trace) {
      double *t = trace + OR_TRACE_COLS * i;
      t[0] = (double)i; t[1] = E; t[2] = max_atom_norm(n, f); t[3] = sqrt(dot3n(n, f, f));
      t[4] = P; t[5] = dt; t[6] = alpha; t[7] = branch; t[8] = (double)npos;
    }
    if (CRIT() < tol) stop = OR_STOP_CONVERGED;
  }
  if (!stop) stop = OR_STOP_MAX_STEPS;
  res->stop = stop;
  res->iterations = it;
  res->force_evals = evals;
  res->energy = E;
  res->fmax = max_atom_norm(n, f);
  res->f2norm = sqrt(dot3n(n, f, f));
  res->dt = dt;
  res->alpha = alpha;
  res->n_pos = npos;
  res->n_neg = nneg;
  if (vel_out) memcpy(vel_out, v, sizeof(double) * 3 * n);
#undef CRIT
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
