// fire2_device.h -- device code shared by the single-system (fire2.hip) and
// batched (batched.hip) paths: wave reductions, fast reciprocals, and the
// scalar FIRE 2.0 control step.
#pragma once
#include <hip/hip_runtime.h>

#include "fire2.h"
#include "fire2_internal.h"

namespace fire {

// A double moved across lanes by a DPP control (two 32-bit moves).  Lanes
// in rows that ROWS leaves out receive id.
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ double dpp_d(double v, double id) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned long long o = __builtin_bit_cast(unsigned long long, id);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)o, (int)(unsigned)b, CTRL, ROWS, 0xf, false);
  const unsigned hi =
      (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)(o >> 32), (int)(unsigned)(b >> 32), CTRL, ROWS, 0xf, false);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ double lane63(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, 63);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), 63);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Sum (max) over the 64 lanes, returned to every lane.  Register-to-register
// lane moves in a fixed order: neighbours in a quad (lane ^ 1, lane ^ 2),
// the mirrored half row and row (eight, then sixteen lanes), then lane 15 of
// each row into the next row and lane 31 into the upper two rows; lane 63
// then holds the total.  The same order every time, so results repeat bit
// for bit.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<0xB1>(v, 0.0);        // quad_perm [1, 0, 3, 2]
  v += dpp_d<0x4E>(v, 0.0);        // quad_perm [2, 3, 0, 1]
  v += dpp_d<0x141>(v, 0.0);       // row_half_mirror
  v += dpp_d<0x140>(v, 0.0);       // row_mirror
  v += dpp_d<0x142, 0xa>(v, 0.0);  // row_bcast:15 into rows 1 and 3
  v += dpp_d<0x143, 0xc>(v, 0.0);  // row_bcast:31 into rows 2 and 3
  return lane63(v);
}
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_d<0xB1>(v, -INFINITY));
  v = fmax(v, dpp_d<0x4E>(v, -INFINITY));
  v = fmax(v, dpp_d<0x141>(v, -INFINITY));
  v = fmax(v, dpp_d<0x140>(v, -INFINITY));
  v = fmax(v, dpp_d<0x142, 0xa>(v, -INFINITY));
  v = fmax(v, dpp_d<0x143, 0xc>(v, -INFINITY));
  return lane63(v);
}

// 1/x and 1/sqrt(x) from the hardware estimates plus Newton steps (one step
// for the reciprocal squares the estimate's relative error, which is far
// below 1e-8, to round-off level).
__device__ __forceinline__ double rcp_d(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  return fma(y, fma(-x, y, 1.0), y);
}
__device__ __forceinline__ double rsqrt_d(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  return y * fma(-h * y, y, 1.5);
}
__device__ __forceinline__ float rcp_f(float x) { return __builtin_amdgcn_rcpf(x); }

// True in every lane when any active lane has c (a wave-uniform branch).
__device__ __forceinline__ bool wave_any(bool c) { return __builtin_amdgcn_ballot_w64(c) != 0; }

// e^x in FP64 for the pair terms (arguments of a few tens at most): with
// k = rint(x / ln 2) and r = x - k ln 2, |r| <= ln(2)/2, e^x = 2^k e^r and
// e^r is its Taylor series to r^13 (the remainder is below 1e-17 of the
// result).  ln 2 enters as a 32-bit leading part, whose product with k is
// exact, plus the rest (Cody and Waite's reduction).  No special cases:
// callers keep x finite and far from the overflow and underflow limits.
__device__ __forceinline__ double exp_d(double x) {
  constexpr double kLog2e = 1.4426950408889634074;
  constexpr double kLn2Hi = 6.93147180369123816490e-01;  // ln 2 to 32 bits
  constexpr double kLn2Lo = 1.90821492927058770002e-10;  // ln 2 - kLn2Hi
  const double k = __builtin_rint(x * kLog2e);
  const double r = fma(-k, kLn2Lo, fma(-k, kLn2Hi, x));
  double p = 1.0 / 6227020800.0;  // 1/13!
  p = fma(p, r, 1.0 / 479001600.0);
  p = fma(p, r, 1.0 / 39916800.0);
  p = fma(p, r, 1.0 / 3628800.0);
  p = fma(p, r, 1.0 / 362880.0);
  p = fma(p, r, 1.0 / 40320.0);
  p = fma(p, r, 1.0 / 5040.0);
  p = fma(p, r, 1.0 / 720.0);
  p = fma(p, r, 1.0 / 120.0);
  p = fma(p, r, 1.0 / 24.0);
  p = fma(p, r, 1.0 / 6.0);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return __builtin_ldexp(p, (int)k);
}

// 2^(j/32), j = 0..31, each rounded to the nearest double: the table of the
// FP64 exponential below.  Blocks that use it copy it to LDS first.
static __constant__ double kExp2Frac32[32] = {
    0x1.0000000000000p+0, 0x1.059b0d3158574p+0, 0x1.0b5586cf9890fp+0, 0x1.11301d0125b51p+0,
    0x1.172b83c7d517bp+0, 0x1.1d4873168b9aap+0, 0x1.2387a6e756238p+0, 0x1.29e9df51fdee1p+0,
    0x1.306fe0a31b715p+0, 0x1.371a7373aa9cbp+0, 0x1.3dea64c123422p+0, 0x1.44e086061892dp+0,
    0x1.4bfdad5362a27p+0, 0x1.5342b569d4f82p+0, 0x1.5ab07dd485429p+0, 0x1.6247eb03a5585p+0,
    0x1.6a09e667f3bcdp+0, 0x1.71f75e8ec5f74p+0, 0x1.7a11473eb0187p+0, 0x1.82589994cce13p+0,
    0x1.8ace5422aa0dbp+0, 0x1.93737b0cdc5e5p+0, 0x1.9c49182a3f090p+0, 0x1.a5503b23e255dp+0,
    0x1.ae89f995ad3adp+0, 0x1.b7f76f2fb5e47p+0, 0x1.c199bdd85529cp+0, 0x1.cb720dcef9069p+0,
    0x1.d5818dcfba487p+0, 0x1.dfc97337b9b5fp+0, 0x1.ea4afa2a490dap+0, 0x1.f50765b6e4540p+0,
};

// Threads 0..31 copy the table to the block's LDS array t; the caller's
// next barrier publishes it.
__device__ __forceinline__ void exp_table_fill(double* t) {
  if (threadIdx.x < 32) t[threadIdx.x] = kExp2Frac32[threadIdx.x];
}

// e^x in FP64 for the pair terms, table-driven (Tang's method, 1989): with
// k = rint(32 x / ln 2) = 32 m + j (0 <= j < 32) and r = x - k ln 2 / 32,
// |r| <= ln 2 / 64 and e^x = 2^m 2^(j/32) e^r.  e^r - 1 is its Taylor series
// to r^6 (the remainder is below 4e-18) and joins the table entry in one
// fma.  ln 2 / 32 enters as a leading part of 32 bits, whose product with k
// is exact, plus the rest (Cody and Waite's reduction).  No special cases:
// callers keep x finite and far from the overflow and underflow limits.
// tab: the LDS copy of the table.
__device__ __forceinline__ double exp_t(double x, const double* __restrict__ tab) {
  constexpr double kScale = 46.166241308446829036;              // 32 / ln 2
  constexpr double kHi = 6.93147180369123816490e-01 / 32;      // exact: ln 2 to 32 bits, over 32
  constexpr double kLo = 1.90821492927058770002e-10 / 32;
  const double kd = __builtin_rint(x * kScale);
  const double r = fma(-kd, kLo, fma(-kd, kHi, x));
  const int k = (int)kd;
  double q = 1.0 / 720.0;
  q = fma(q, r, 1.0 / 120.0);
  q = fma(q, r, 1.0 / 24.0);
  q = fma(q, r, 1.0 / 6.0);
  q = fma(q, r, 0.5);
  q = fma(q, r, 1.0);
  q *= r;  // e^r - 1
  const double t = tab[k & 31];
  return __builtin_ldexp(fma(t, q, t), k >> 5);
}

// FP32 pair terms: the hardware square root (within 1 ulp; the arguments
// are squared separations of a few A^2, far from denormals).
__device__ __forceinline__ float sqrt_f(float x) { return __builtin_amdgcn_sqrtf(x); }

// e^x in FP32 for the pair terms: x log2(e) as the rounded product plus its
// rounding error (one fma) and the error of log2(e) in float, the integer
// part applied by ldexp and 2^(the rest) by the hardware base-2 exponential.
// Arguments stay within a few tens, so there is no overflow or underflow
// handling.
__device__ __forceinline__ float exp_f(float x) {
  constexpr float kL = 1.44269502162933349609375f;  // log2(e) rounded to float
  constexpr float kLlo = 1.925962991126617e-8f;     // log2(e) - kL
  const float ph = x * kL;
  const float pl = fmaf(x, kL, -ph) + x * kLlo;
  const float e = __builtin_rintf(ph);
  return __builtin_ldexpf(__builtin_amdgcn_exp2f((ph - e) + pl), (int)e);
}

__device__ __forceinline__ float rsqrt_f(float x) {
  float y = __builtin_amdgcn_rsqf(x);
  return y * fmaf(-0.5f * x * y, y, 1.5f);
}

// What the P test at the start of iteration i decides (Algorithm 2, or
// Algorithm 1 for the original FIRE): the new dt and alpha, the alpha the
// original FIRE mixes with (the one before this test), the counters of
// consecutive P > 0 and P <= 0 steps, and whether P <= 0 has now held more
// than N_P<=0max times in a row (the MAXVDOTF stop).
struct Adapt {
  double dt, alpha, alpha_mix;
  long long npos, nneg;
  int neg, stop;
};

__device__ inline Adapt fire_adapt(const Ctrl& c, double P, long long i) {
  Adapt a{c.dt, c.alpha, c.alpha, c.npos, c.nneg, P > 0.0 ? 0 : 1, 0};
  if (!a.neg) {
    a.npos += 1;
    a.nneg = 0;
    if (a.npos > c.delaystep) {
      a.dt = fmin(a.dt * c.dtgrow, c.dtmax);
      a.alpha *= c.alphashrink;
    }
    return a;
  }
  a.npos = 0;
  if (c.variant != FIRE_VARIANT_FIRE2) {  // original FIRE: shrink and reset at once
    a.dt *= c.dtshrink;
    a.alpha = c.alpha0;
    return a;
  }
  a.nneg += 1;
  if (a.nneg > c.vdfmax) {
    a.stop = 1;
    return a;
  }
  if (!(c.initialdelay && i < c.delaystep)) {  // no shrink during the initial delay
    if (a.dt * c.dtshrink >= c.dtmin) a.dt *= c.dtshrink;
    a.alpha = c.alpha0;
  }
  return a;
}

// Coefficients of the next update for the chosen integrator (Algorithms 3,
// 4, 6): kick before the drift (k1), kick with the drift's old force (k2,
// explicit Euler), kick after the new force (k3), and the mixing
// v <- cv v + cf |v| F / |F|, applied after the first kick (FIRE 2.0) or at
// the start of the step (original FIRE, mix_first).
struct UpdCoefs {
  double k1, k2, k3, cv, cf;
  int mix_first;
};

__device__ inline UpdCoefs fire_coefficients(const Ctrl& c, const Adapt& a, double V2, double F2, double SvF,
                                             double SFF) {
  const double dtf = a.dt * c.f2a;
  UpdCoefs u{dtf, 0.0, 0.0, 0.0, 0.0, 0};
  if (c.integrator == FIRE_INT_EULER_EXPLICIT) {
    u.k1 = 0.0;
    u.k2 = dtf;
  } else if (c.integrator == FIRE_INT_VERLET) {
    u.k1 = 0.5 * dtf;
    u.k3 = 0.5 * dtf;
  }
  const double fn = sqrt(F2);
  if (c.variant == FIRE_VARIANT_FIRE2) {
    // |v| of the velocity being mixed, from the reductions: the kick gives
    // atom i v_i + k1 s_i F_i, so |v|^2 = V2 + 2 k1 sum s v.F + k1^2 sum s^2 F^2
    // (after P <= 0 the velocities are zero: V2 and sum s v.F drop out)
    const double V2e = a.neg ? 0.0 : V2, SvFe = a.neg ? 0.0 : SvF;
    const double vn = sqrt(fmax(V2e + 2.0 * u.k1 * SvFe + u.k1 * u.k1 * SFF, 0.0));
    u.cv = 1.0 - a.alpha;
    u.cf = fn > 0.0 ? a.alpha * vn / fn : 0.0;
  } else {
    u.mix_first = 1;
    u.cv = a.neg ? 1.0 : 1.0 - a.alpha_mix;
    u.cf = (a.neg || !(fn > 0.0)) ? 0.0 : a.alpha_mix * sqrt(V2) / fn;
  }
  return u;
}

// The scalar FIRE logic (one thread) on the reduced E, P, |F|^2, |v|^2,
// max|F_i|^2, max|v_i|^2, sum s_i v_i.F_i, sum s_i^2 |F_i|^2 of the force
// evaluation just finished (the last two equal P and |F|^2 when every
// s_i = 1/m_i is 1): stop tests, then the P test for the next iteration and
// the coefficients of the next update.  c is a snapshot of *cp taken by the
// caller (one load of the whole record, so no field costs a memory round
// trip of its own); the fields this step changes are written to *cp.
__device__ inline void fire_control(const Ctrl c, Ctrl* __restrict__ cp, const double (&r)[kCtl],
                                    double* __restrict__ trace) {
  const double E = r[0], P = r[1], F2 = r[2], V2 = r[3], fm = sqrt(r[4]), vm = sqrt(r[5]);
  cp->energy = E;
  cp->P = P;
  cp->F2 = F2;
  cp->v2 = V2;
  cp->fmax = fm;
  cp->f2norm = sqrt(F2);
  cp->vmax = vm;
  cp->evals = c.evals + 1;
  const long long it = c.iter;
  if (c.precision) cp->iter_low = c.iter_low + (it > 0);
  if (c.error & ERR_OVERLAP) {
    cp->status = FIRE_E_OVERLAP;
    return;
  }
  if (!isfinite(E) || !isfinite(F2) || (c.error & ERR_NONFINITE)) {
    cp->status = FIRE_E_NONFINITE;
    return;
  }
  if (c.eval_only) return;
  if (trace && it < c.trace_cap) {
    double* t = trace + (size_t)FIRE_TRACE_COLS * it;
    t[0] = (double)it;
    t[1] = E;
    t[2] = fm;
    t[3] = sqrt(F2);
    t[4] = c.P_used;
    t[5] = c.dt;
    t[6] = c.alpha;
    t[7] = (double)c.branch;
    t[8] = (double)c.npos;
  }
  const double crit = c.criterion == FIRE_CRIT_FMAX ? fm : sqrt(F2);
  if (crit < c.tol) {
    cp->status = FIRE_STOP_CONVERGED;
    return;
  }
  if (it >= c.max_steps) {
    cp->status = FIRE_STOP_MAX_STEPS;
    return;
  }
  int pause = 0;
  if (c.precision && c.mode == FIRE_MIXED && crit < c.switch_tol) {
    cp->precision = 0;
    pause |= PAUSE_PRECISION;
  }
  const Adapt a = fire_adapt(c, P, it + 1);
  cp->npos = a.npos;
  cp->nneg = a.nneg;
  if (a.stop) {
    cp->status = FIRE_STOP_MAXVDOTF;
    return;
  }
  const UpdCoefs u = fire_coefficients(c, a, V2, F2, r[R_SVF], r[R_SFF]);
  cp->dt = a.dt;
  cp->alpha = a.alpha;
  cp->branch = a.neg ? -1 : 1;
  cp->P_used = P;
  cp->neg = a.neg;
  cp->mix_first = u.mix_first;
  // the half step back undoes half of a step; with a displacement cap that
  // step is min(dt, dmax / max_i |v_i|) of the velocity being undone
  const double dth = (c.dmax > 0.0 && vm * a.dt > c.dmax) ? c.dmax / vm : a.dt;
  cp->hsb = (a.neg && c.variant == FIRE_VARIANT_FIRE2 && c.halfstepback) ? 0.5 * dth : 0.0;
  cp->kick1 = u.k1;
  cp->kick2 = u.k2;
  cp->kick3 = u.k3;
  cp->cv = u.cv;
  cp->cf = u.cf;
  cp->dtx = a.dt;
  cp->iter = it + 1;
  if (pause) {
    cp->pause = pause;
    cp->status = ST_PAUSED;
  }
}

}  // namespace fire
