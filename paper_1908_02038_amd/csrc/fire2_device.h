// fire2_device.h -- device code shared by the single-system (fire2.hip) and
// batched (batched.hip) paths: wave reductions, fast reciprocals, and the
// scalar FIRE 2.0 control step.
#pragma once
#include <hip/hip_runtime.h>

#include "fire2.h"
#include "fire2_internal.h"

namespace fire {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
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
__device__ __forceinline__ float rsqrt_f(float x) {
  float y = __builtin_amdgcn_rsqf(x);
  return y * fmaf(-0.5f * x * y, y, 1.5f);
}

// The scalar FIRE logic (one thread) on the reduced E, P, |F|^2, |v|^2,
// max|F_i|^2, max|v_i|^2, sum s_i v_i.F_i, sum s_i^2 |F_i|^2 of the force
// evaluation just finished (the last two equal P and |F|^2 when every
// s_i = 1/m_i is 1): stop tests, then the branch of Algorithm 2 (or 1) for
// the next iteration and the coefficients of the next update.
__device__ inline void fire_control(Ctrl* __restrict__ c, const double (&r)[kCtl], double* __restrict__ trace) {
  const double E = r[0], P = r[1], F2 = r[2], V2 = r[3], fm = sqrt(r[4]), vm = sqrt(r[5]);
  c->energy = E;
  c->P = P;
  c->F2 = F2;
  c->v2 = V2;
  c->fmax = fm;
  c->f2norm = sqrt(F2);
  c->vmax = vm;
  c->evals += 1;
  const long long it = c->iter;
  if (c->precision) c->iter_low += (it > 0);
  if (c->error & ERR_OVERLAP) {
    c->status = FIRE_E_OVERLAP;
    return;
  }
  if (!isfinite(E) || !isfinite(F2) || (c->error & ERR_NONFINITE)) {
    c->status = FIRE_E_NONFINITE;
    return;
  }
  if (c->eval_only) return;
  if (trace && it < c->trace_cap) {
    double* t = trace + (size_t)FIRE_TRACE_COLS * it;
    t[0] = (double)it;
    t[1] = E;
    t[2] = fm;
    t[3] = sqrt(F2);
    t[4] = c->P_used;
    t[5] = c->dt;
    t[6] = c->alpha;
    t[7] = (double)c->branch;
    t[8] = (double)c->npos;
  }
  const double crit = c->criterion == FIRE_CRIT_FMAX ? fm : sqrt(F2);
  if (crit < c->tol) {
    c->status = FIRE_STOP_CONVERGED;
    return;
  }
  if (it >= c->max_steps) {
    c->status = FIRE_STOP_MAX_STEPS;
    return;
  }
  int pause = 0;
  if (c->precision && c->mode == FIRE_MIXED && crit < c->switch_tol) {
    c->precision = 0;
    pause |= PAUSE_PRECISION;
  }
  // ---- start of iteration i = it + 1: the branch of Algorithm 2 (or 1)
  const long long i = it + 1;
  double dt = c->dt, alpha = c->alpha;
  const double alpha_mix = alpha;  // Algorithm 1 mixes before alpha decays
  int neg;
  if (P > 0.0) {
    neg = 0;
    c->npos += 1;
    c->nneg = 0;
    if (c->npos > c->delaystep) {
      dt = fmin(dt * c->dtgrow, c->dtmax);
      alpha *= c->alphashrink;
    }
  } else {
    neg = 1;
    c->npos = 0;
    if (c->variant == FIRE_VARIANT_FIRE2) {
      c->nneg += 1;
      if (c->nneg > c->vdfmax) {
        c->status = FIRE_STOP_MAXVDOTF;
        return;
      }
      if (!(c->initialdelay && i < c->delaystep)) {
        if (dt * c->dtshrink >= c->dtmin) dt *= c->dtshrink;
        alpha = c->alpha0;
      }
    } else {
      dt *= c->dtshrink;
      alpha = c->alpha0;
    }
  }
  const double dtf = dt * c->f2a;
  const double fn = sqrt(F2);
  const double V2e = neg ? 0.0 : V2, SvFe = neg ? 0.0 : r[R_SVF], SFF = r[R_SFF];
  double k1, k2, k3, cv, cf;
  int mix_first = 0;
  if (c->integrator == FIRE_INT_EULER_EXPLICIT) {
    k1 = 0.0;
    k2 = dtf;
    k3 = 0.0;
  } else if (c->integrator == FIRE_INT_VERLET) {
    k1 = 0.5 * dtf;
    k2 = 0.0;
    k3 = 0.5 * dtf;
  } else {
    k1 = dtf;
    k2 = 0.0;
    k3 = 0.0;
  }
  if (c->variant == FIRE_VARIANT_FIRE2) {
    // |v| of the velocity being mixed, from the reductions: the kick gives
    // atom i v_i + k1 s_i F_i, so |v|^2 = V2 + 2 k1 sum s v.F + k1^2 sum s^2 F^2
    const double vn = sqrt(fmax(V2e + 2.0 * k1 * SvFe + k1 * k1 * SFF, 0.0));
    cv = 1.0 - alpha;
    cf = fn > 0.0 ? alpha * vn / fn : 0.0;
  } else {
    mix_first = 1;
    cv = neg ? 1.0 : 1.0 - alpha_mix;
    cf = (neg || !(fn > 0.0)) ? 0.0 : alpha_mix * sqrt(V2) / fn;
  }
  c->dt = dt;
  c->alpha = alpha;
  c->branch = neg ? -1 : 1;
  c->P_used = P;
  c->neg = neg;
  c->mix_first = mix_first;
  // the half step back undoes half of a step; with a displacement cap that
  // step is min(dt, dmax / max_i |v_i|) of the velocity being undone
  const double dth = (c->dmax > 0.0 && vm * dt > c->dmax) ? c->dmax / vm : dt;
  c->hsb = (neg && c->variant == FIRE_VARIANT_FIRE2 && c->halfstepback) ? 0.5 * dth : 0.0;
  c->kick1 = k1;
  c->kick2 = k2;
  c->kick3 = k3;
  c->cv = cv;
  c->cf = cf;
  c->dtx = dt;
  c->iter = i;
  if (pause) {
    c->pause = pause;
    c->status = ST_PAUSED;
  }
}

}  // namespace fire
