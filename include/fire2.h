/*
 * fire2.h -- C ABI of the MI355X (gfx950) FIRE 2.0 energy-minimisation library.
 *
 * The library minimises the potential energy E(x) of N atoms over their 3N
 * coordinates (Guenole et al., FIRE 2.0, Sec. 1 and Sec. 2.1) with the
 * FIRE 2.0 pseudo-dynamics of Algorithm 2, integrated by semi-implicit Euler
 * with the velocity mixing placed after the kick (Algorithm 4, Sec. 3.3).
 * Forces F = -grad E (Sec. 2.1) come from hand-written HIP kernels over a
 * cell-sorted neighbour list: energy-shifted Lennard-Jones, or the
 * second-moment (Gupta/RGL) EAM form of Sec. 5.2 (pair term plus embedding
 * F(rho) = -xi sqrt(rho)).
 *
 * Conventions for every entry point:
 *   - Positions, forces and direction fields are row-major double[n][3] in the
 *     caller's atom order.  Energies are in the potential's units.
 *   - Host-pointer calls copy in and out and return when the result is on the
 *     host.  *_dev calls take device pointers and a hipStream_t passed as
 *     void* (NULL is the legacy default stream, as in HIP); they enqueue on
 *     that stream, after the work already queued there.
 *     fire_energy_forces_dev and fire_hvp_dev do not synchronise;
 *     fire_minimize_dev and fire_minimize_batched_dev poll small status
 *     words and return when done.
 *   - The caller owns every array it passes; the context owns its device
 *     work buffers and reuses them across calls.  A context is not
 *     thread-safe: calls on one context must not overlap.
 *   - Return value: FIRE_OK (0) or a negative FIRE_E_* code; the message is
 *     available from fire_last_error().  On error no output is written,
 *     except that fire_minimize may have advanced positions before a device
 *     error was detected.
 *   - Periodic axes require rc + skin < len/2 (minimum image); free axes ignore
 *     box.lo/len.  Positions returned on periodic axes are wrapped into
 *     [lo, lo + len).
 */
#ifndef FIRE2_H
#define FIRE2_H

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------- codes */
#define FIRE_OK 0
#define FIRE_E_ARG -1         /* NULL pointer, n <= 0, bad enum or parameter */
#define FIRE_E_BOX -2         /* len <= 0, or cutoff + skin >= len/2 on a periodic axis */
#define FIRE_E_NONFINITE -3   /* NaN/Inf in positions or in a computed energy/force */
#define FIRE_E_OVERLAP -4     /* two atoms at distance 0 */
#define FIRE_E_DEVICE -5      /* HIP runtime error or no gfx950 device */
#define FIRE_E_OOM -6         /* device allocation failed */

/* Stop reasons of a minimisation (not errors). */
#define FIRE_STOP_CONVERGED 1 /* criterion < tol after a force evaluation (Algorithm 2, "converged") */
#define FIRE_STOP_MAX_STEPS 2 /* max_steps iterations done */
#define FIRE_STOP_MAXVDOTF 3  /* more than vdfmax consecutive P <= 0 steps (Sec. 3.4, MAXVDOTF) */

#define FIRE_POT_LJ 1         /* 4 eps [(s/r)^12 - (s/r)^6] - phi(rc) for r < rc */
#define FIRE_POT_GUPTA 2      /* sum_j A e^{-p(r/r0-1)} S(r) - xi sqrt(sum_j e^{-2q(r/r0-1)} S(r)) */
#define FIRE_POT_HARMONIC 3   /* 1/2 sum_i sum_d k_d x_id^2 (test well, no pairs) */
#define FIRE_POT_SW 4         /* Stillinger-Weber: sum_{i<j} phi2(r_ij) + sum_i sum_{j<k} h(r_ij, r_ik, theta_jik) */

#define FIRE_GUPTA_RGL 0      /* every ordered pair carries phi: E = sum_i [sum_j phi + F(rho_i)] */
#define FIRE_GUPTA_HALF 1     /* EAM half sum: E = 1/2 sum_i sum_j phi + sum_i F(rho_i) */

#define FIRE_FP64 0           /* pair terms, accumulation, reductions and update in FP64 */
#define FIRE_MIXED 1          /* FP32 pair terms and per-atom accumulation from FP64 separations;
                                 FP64 reductions, update and stop test; switches to FP64 pair terms
                                 once the criterion falls below mixed_switch */
#define FIRE_FP32 2           /* FP32 pair terms throughout (no switch) */

#define FIRE_INT_EULER_IMPLICIT 0 /* Algorithm 4 (default, Table 1) */
#define FIRE_INT_EULER_EXPLICIT 1 /* Algorithm 3 */
#define FIRE_INT_VERLET 2         /* Algorithm 6 */

#define FIRE_CRIT_FMAX 0      /* max_i |F_i| (per-atom Euclidean norm) */
#define FIRE_CRIT_F2NORM 1    /* Euclidean norm of the 3N force vector (Sec. 3.4, f2norm) */

#define FIRE_VARIANT_FIRE2 0  /* Algorithm 2 */
#define FIRE_VARIANT_FIRE1 1  /* Algorithm 1 (original FIRE) */

/* ------------------------------------------------------------ records */

/* Opaque context: device, streams, work buffers and captured graphs. */
typedef struct fire_ctx fire_ctx;

/* Orthorhombic box with per-axis periodicity (the paper's test cases mix
 * periodic and free axes, Sec. 5.3). */
typedef struct {
  double lo[3];
  double len[3];
  int periodic[3];
} fire_box;

/* Interatomic model.  LJ uses eps, sigma, rc.  Gupta uses A, p, q, xi, r0 and
 * the cubic taper S(r) = 1 (r <= r_in), (1-s)^2 (1+2s) with
 * s = (r - r_in)/(r_out - r_in), 0 (r >= r_out); r_out is the cutoff.
 * HARMONIC uses k[3].  SW (the Si test case of Sec. 5.3) uses eps, sigma, A,
 * p, q and the sw_* fields, with s = sigma and cutoff a s:
 *   phi2(r) = eps A [B (s/r)^p - (s/r)^q] exp(s / (r - a s)),
 *   h       = lambda eps (cos theta_jik + 1/3)^2 g(r_ij) g(r_ik),
 *   g(r)    = exp(gamma s / (r - a s)),  all zero for r >= a s.
 * The SW path runs in FP64 whatever the precision setting, and has no
 * Hessian product and no batched form. */
typedef struct {
  int kind;        /* FIRE_POT_* */
  int convention;  /* FIRE_GUPTA_RGL or FIRE_GUPTA_HALF */
  double eps, sigma, rc;
  double A, p, q, xi, r0, r_in, r_out;
  double k[3];
  double sw_B, sw_a, sw_lambda, sw_gamma;
} fire_potential;

/* FIRE parameters.  The first twelve fields are Table 1 of the paper
 * (min_modify arguments); dt_start is the LAMMPS timestep and f2a the
 * force-to-acceleration factor 1/m (times a unit conversion), neither of
 * which has a paper default. */
typedef struct {
  double dt_start;     /* initial timestep */
  double tmax;         /* dt_max = tmax * dt_start */
  double tmin;         /* dt_min = tmin * dt_start */
  double dtgrow;       /* f_inc */
  double dtshrink;     /* f_dec */
  double alpha0;       /* alpha_start */
  double alphashrink;  /* f_alpha */
  double f2a;          /* 1/m */
  int delaystep;       /* N_delay */
  int vdfmax;          /* N_{P<=0,max} */
  int halfstepback;    /* 1: x -= dt v / 2 on P <= 0 */
  int initialdelay;    /* 1: no dt/alpha change on P <= 0 while i < N_delay */
  int integrator;      /* FIRE_INT_* */
  int criterion;       /* FIRE_CRIT_* */
  int variant;         /* FIRE_VARIANT_* */
  int precision;       /* FIRE_FP64 / FIRE_MIXED / FIRE_FP32 */
  double mixed_switch; /* FIRE_MIXED: criterion value below which pair terms go to FP64;
                          <= 0 selects 100 * tol */
  double skin;         /* neighbour-list skin in length units; <= 0 selects 0.12 * cutoff,
                          clamped to fit the box.  Affects speed only: lists are rebuilt
                          as soon as an atom has moved more than skin/2, so every pair
                          within the cutoff is always seen */
  double dmax;         /* > 0: displacement cap (the maximum atomic displacement per step of
                          the melt case, Sec. 5.3).  The drift uses the step
                          min(dt, dmax / max_i |v_i|), v the velocity it moves the atoms
                          with, so no atom drifts more than dmax; the half step back undoes
                          half of such a step of the velocity being zeroed (at most dmax/2).
                          dt itself and the kicks are unchanged.  0 (default): no cap.  Not
                          available in the batched form. */
} fire_params;

/* Outcome of a minimisation.  iterations counts integration steps
 * (force_evals = iterations + 1). */
typedef struct {
  int stop_reason;          /* FIRE_STOP_*; in the batched form, a system that failed
                               reports its FIRE_E_* code (< 0) here instead */
  int precision_switched;   /* FIRE_MIXED: 1 once the run moved to FP64 pair terms */
  long long iterations;
  long long force_evals;
  long long iterations_low; /* iterations done with FP32 pair terms */
  long long rebuilds;       /* neighbour-list builds, including the first */
  double energy;            /* E at the final positions */
  double energy_per_atom;
  double fmax;              /* max_i |F_i| */
  double f2norm;            /* |F| over 3N */
  double dt;                /* dt at the stop (before the final reset of Algorithm 2) */
  double alpha;
} fire_result;

/* Per-atom properties of a minimisation, in the caller's atom order (n
 * entries each); either pointer may be NULL.
 *   frozen: bit d (d = 0, 1, 2) of frozen[i] holds component d of atom i
 *           fixed.  Its force component is set to zero after every force
 *           evaluation, so its velocity and coordinate never change, and it
 *           counts as zero in P, |F|, max|F_i| and the stop test (the frozen
 *           borders of the test cases in Sec. 5.3).  Other bits are ignored.
 *   mass:   mass[i] > 0 and finite, relative to the mass that f2a implies:
 *           atom i is kicked with dt f2a / mass[i] instead of dt f2a (the
 *           m in the update steps of Algorithms 3, 4 and 6).  The mixing of
 *           Algorithm 2 uses the 3N-vector norms |v| and |F| as without
 *           masses.
 * Both arrays are read during the call only. */
typedef struct {
  const unsigned char* frozen;
  const double* mass;
} fire_atoms;

/* Fill p with the Table 1 defaults (eulerimplicit, tmax 10, tmin 0.02,
 * delaystep 20, dtgrow 1.1, dtshrink 0.5, alpha0 0.25, alphashrink 0.99,
 * vdfmax 2000, halfstepback yes, initialdelay yes), dt_start = f2a = 1,
 * criterion FMAX, variant FIRE2, precision FP64, automatic switch and skin. */
void fire_params_default(fire_params* p);

/* Create a context on HIP device `device`.  params may be NULL (defaults).
 * Fails with FIRE_E_DEVICE when the device is not gfx950. */
int fire_init(fire_ctx** ctx, int device, const fire_params* params);
void fire_finalize(fire_ctx* ctx);
int fire_set_params(fire_ctx* ctx, const fire_params* params);
int fire_get_params(const fire_ctx* ctx, fire_params* params);
const char* fire_last_error(const fire_ctx* ctx);
/* The speed-only choices of the last minimisation on ctx, as text.  After
 * a single-system call: the list order of the EAM form and the LDS
 * reservation of its tile blocks, timed on the system's start positions the
 * first time a class of systems is seen
 * (potential, starting precision, size in powers of two, periodic axes) and
 * cached per context and in $FIRE_TUNE_CACHE.single (default
 * ~/.cache/fire2_tune_single.txt).  After a batched call: the team size of
 * the persistent kernel and its chunk length, timed or from
 * $FIRE_TUNE_CACHE, and the launch plan (workgroups, and how many pairs of
 * them share the systems of most estimated work).  Single-system results
 * differ between choices only by summation order; batched results do not
 * depend on the plan.  The pointer stays valid until the next call on ctx. */
const char* fire_tuning_info(const fire_ctx* ctx);
const char* fire_stop_name(int stop_reason);

/* One force evaluation (Sec. 2.1): *energy = E(pos), forces = -grad E
 * (forces may be NULL).  Precision follows the context's params
 * (FIRE_MIXED evaluates with FP32 pair terms). */
int fire_energy_forces(fire_ctx* ctx, long long n, const double* pos, const fire_box* box,
                       const fire_potential* pot, double* energy, double* forces);

/* FIRE 2.0 minimisation (Algorithm 2 with the context's integrator) of pos
 * (in/out) until the criterion is < tol, max_steps iterations, or MAXVDOTF. */
int fire_minimize(fire_ctx* ctx, long long n, double* pos, const fire_box* box, const fire_potential* pot,
                  double tol, long long max_steps, fire_result* out);

/* As fire_minimize, and writes one row per force evaluation i = 0..iterations
 * into trace (capacity max_steps + 1 rows of FIRE_TRACE_COLS doubles):
 * {i, E, fmax, f2norm, P, dt, alpha, branch (+1: P > 0, -1: P <= 0, 0: initial), N_P>0}. */
#define FIRE_TRACE_COLS 9
int fire_minimize_traced(fire_ctx* ctx, long long n, double* pos, const fire_box* box,
                         const fire_potential* pot, double tol, long long max_steps, fire_result* out,
                         double* trace);

/* fire_minimize with per-atom properties (atoms may be NULL: then exactly
 * fire_minimize).  trace (NULL: none) is as for fire_minimize_traced and then
 * requires out.  FIRE_E_ARG if a mass is not positive and finite. */
int fire_minimize_ex(fire_ctx* ctx, long long n, double* pos, const fire_box* box, const fire_potential* pot,
                     const fire_atoms* atoms, double tol, long long max_steps, fire_result* out, double* trace);

/* Hessian-vector product hu = (d^2 E / dx dx) u at pos, FP64 (u, hu: [n][3]). */
int fire_hvp(fire_ctx* ctx, long long n, const double* pos, const double* u, const fire_box* box,
             const fire_potential* pot, double* hu);

/* Lowest curvature of E at pos along directions orthogonal to rigid
 * translations: k iterations of Lanczos on the Hessian (HVP kernel, full
 * re-orthogonalisation), started from the seeded direction u0 ([n][3],
 * NULL = built-in).  *lambda_min is the smallest Ritz value theta, the
 * Rayleigh quotient of its Ritz vector z, so the Hessian's lowest eigenvalue
 * is <= theta.  residual (may be NULL) receives |H z - theta z| (|z| = 1):
 * some eigenvalue lies within it of theta, so theta - residual > 0 shows a
 * positive curvature there; theta < 0 shows an unstable direction (a
 * saddle).  Whether theta has reached the lowest eigenvalue depends on k
 * and the spectrum's gaps. */
int fire_lowest_curvature(fire_ctx* ctx, long long n, const double* pos, const fire_box* box,
                          const fire_potential* pot, const double* u0, int k, double* lambda_min,
                          double* residual);

/* Independent minimisations of nsys systems in one persistent launch.
 * System s owns atoms offsets[s] .. offsets[s+1]-1 of pos ([offsets[nsys]][3],
 * in/out), the box boxes[s], and the FIRE state of its own; per_sys (NULL =
 * the context's params for all) gives each system its parameters.  All
 * systems share pot.  out has nsys entries.
 * A system that fails on its own -- two of its atoms at one place, a
 * non-finite position or force -- stops with out[s].stop_reason set to
 * FIRE_E_OVERLAP or FIRE_E_NONFINITE and its positions as they were at its
 * last force evaluation; every other system runs to its own stop exactly as
 * without it (the same bits), and the call returns FIRE_OK.  How the launch
 * shares out the work -- a system of more than 1.5 team widths of atoms may
 * be split over a pair of workgroups on two CUs -- changes no result either.
 * Errors of the call itself (arguments, the device, FIRE_E_DEVICE if the two
 * workgroups of a pair lose each other at a barrier for more than two
 * seconds) are returned as usual and then no output is written. */
int fire_minimize_batched(fire_ctx* ctx, int nsys, const long long* offsets, double* pos,
                          const fire_box* boxes, const fire_potential* pot, const fire_params* per_sys,
                          double tol, long long max_steps, fire_result* out);

/* Device-pointer variants (see the conventions above). */
int fire_energy_forces_dev(fire_ctx* ctx, long long n, const double* d_pos, const fire_box* box,
                           const fire_potential* pot, double* d_energy, double* d_forces, void* stream);
int fire_hvp_dev(fire_ctx* ctx, long long n, const double* d_pos, const double* d_u, const fire_box* box,
                 const fire_potential* pot, double* d_hu, void* stream);
int fire_minimize_dev(fire_ctx* ctx, long long n, double* d_pos, const fire_box* box,
                      const fire_potential* pot, double tol, long long max_steps, fire_result* out,
                      void* stream);
/* fire_minimize_ex on device positions; d_atoms is a host record whose
 * frozen and mass arrays are device pointers (n entries each). */
int fire_minimize_ex_dev(fire_ctx* ctx, long long n, double* d_pos, const fire_box* box,
                         const fire_potential* pot, const fire_atoms* d_atoms, double tol, long long max_steps,
                         fire_result* out, void* stream);
/* fire_minimize_batched on device positions d_pos ([offsets[nsys]][3], in
 * place); offsets, boxes, per_sys and out stay in host memory.  Returns when
 * every system has stopped.  Per-system failures are reported as in
 * fire_minimize_batched. */
int fire_minimize_batched_dev(fire_ctx* ctx, int nsys, const long long* offsets, double* d_pos,
                              const fire_box* boxes, const fire_potential* pot, const fire_params* per_sys,
                              double tol, long long max_steps, fire_result* out, void* stream);

/* For callers that cannot allocate device memory (work of their own under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc):
 * fire_minimize_batched_dev with no device allocation, graph or event in
 * the call.  Its work buffers are carved out of one 64 MiB device array that
 * each GPU the library runs on holds until the process ends (its address is
 * taken once per device by fire_init).  Limits: at most 1,024 systems, and
 * the batch's per-atom state plus neighbour lists must fit the array (about
 * 160,000 atoms of the EAM-form crystals, 130,000 of the LJ ones); beyond them FIRE_E_ARG, with
 * nothing written.  The context's device must be current (FIRE_E_DEVICE
 * otherwise).  Every call on one GPU uses the same array: calls that
 * overlap in time on one GPU, from any context or thread, race, and the
 * caller must serialise them.  Each call rewrites every part of the array
 * it reads before reading it.  Results, per-system failures and errors are
 * those of fire_minimize_batched_dev: the same kernels, with the team shape
 * of FIRE_BATCH_TEAM or of the context's cached tuning (1,024 threads if
 * there is none), so the bits match whenever both calls use one shape. */
int fire_minimize_batched_noalloc(fire_ctx* ctx, int nsys, const long long* offsets, double* d_pos,
                                  const fire_box* boxes, const fire_potential* pot, const fire_params* per_sys,
                                  double tol, long long max_steps, fire_result* out, void* stream);

/* Measurement hook: re-run the force evaluation (density and force passes for
 * the EAM form) of the system left by the last call on ctx, at its current
 * positions and neighbour list, reps times on stream, with the same kernels
 * and launch shapes as one iteration inside fire_minimize (where the update
 * is folded into the first pass, that pass with a zero update, writing the
 * context's second state set) and the precision of the context's params.
 * The system's positions, velocities, forces and FIRE state do not change.
 * FIRE_E_ARG if no system has been evaluated yet. */
int fire_repeat_forces_dev(fire_ctx* ctx, int reps, void* stream);

#ifdef __cplusplus
}
#endif
#endif
