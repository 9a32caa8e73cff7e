// batched.hip -- many independent FIRE 2.0 relaxations in one persistent launch.
//
// One workgroup ("team") relaxes one system at a time: the system's positions
// live in LDS (up to 4096 atoms), velocities, forces and the skin reference in
// per-atom global arrays, its neighbour list (16-bit system-local indices) in
// global memory.  Every iteration -- update, EAM density, force pass, team
// reduction, FIRE control -- runs inside the team with workgroup barriers
// only, and the team rebuilds its own cell and neighbour list when an atom
// leaves its skin.  The systems of most work go first to pairs of teams on
// two CUs, which split the atoms and meet at barriers across the two CUs.
// Each system keeps its own FIRE state (dt, alpha, N_P>0, N_P<=0, counters) in
// a control record, advanced by the same scalar FIRE 2.0 step as the
// single-system path.  Teams take systems from a queue ordered by decreasing
// estimated work and advance each by at most `chunk` iterations per launch;
// the launch is captured in a hipGraph and replayed until every system has
// stopped.
// A small autotuner picks the team shape (and chunk length) by timing the
// candidates on the batch itself.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <type_traits>
#include <vector>

#include "fire2.h"
#include "fire2_device.h"
#include "fire2_internal.h"

namespace fire {
namespace bat {

constexpr int kMaxAtoms = 4096;  // per system (LDS holds its positions)
// Iterations per system and launch.  A launch ends when every system has
// advanced by up to kChunk iterations, so every launch waits for its slowest
// system: 1,024 instead of 256 lets teams carry on with further systems while
// a long relaxation runs (512 EAM-form systems, one CU per system: 283
// instead of 341 ms).
constexpr int kChunk = 1024;
constexpr int kMaxCells = 1024;  // per-system cell grid in LDS
constexpr int kRedWidth = 10;    // values per wave in a team reduction
constexpr int kMaxPairs = 512;   // pairs of teams per launch
// Longest wait of a block at a pair barrier, in ticks of the 100 MHz
// constant clock (2 s; a partner is never more than one pass behind).
constexpr long long kPairWaitTicks = 200000000LL;

struct SysDesc {
  int off, n;    // first atom in the concatenated arrays, atom count
  BoxDev box;    // periodic axes: box; free axes: ignored
  double rcs2;   // (cutoff + skin)^2 of this system
};

// Minimum image along one axis; on free axes L = invL = 0 and d is unchanged.
__device__ __forceinline__ void min_img(double& d, double L, double invL) { d -= L * rint(d * invL); }

// Per-axis image shifts of a system: the box on periodic axes, zero on free ones.
struct Img {
  double L[3], iL[3];
  __device__ explicit Img(const SysDesc& d) {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      L[q] = d.box.per[q] ? d.box.L[q] : 0.0;
      iL[q] = d.box.per[q] ? d.box.invL[q] : 0.0;
    }
  }
  __device__ void apply(double& dx, double& dy, double& dz) const {
    min_img(dx, L[0], iL[0]);
    min_img(dy, L[1], iL[1]);
    min_img(dz, L[2], iL[2]);
  }
};

// Neighbour list of atom a (system-local 16-bit indices) in groups of four:
// group g of atom a is the 8 bytes at nbr + base + (g * n + a) * 4, so the
// atoms of a wave read consecutive 8-byte words.  Lists are padded to a
// multiple of four with the atom's own index; nn[a] is the true length.
__device__ __forceinline__ size_t nidx(size_t base, int n, int a, int q) {
  return base + ((size_t)(q >> 2) * n + a) * 4 + (q & 3);
}

// Team reduction of NS sums followed by NM maxima; the results are valid in
// thread 0.  Each value is reduced on its own (lanes of a wave, then the
// waves in order), so its bits do not depend on the other values of the call.
template <int TEAM, int NS, int NM>
__device__ __forceinline__ void team_reduce(double (&v)[NS + NM], double (*red)[kRedWidth]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NS; ++k) v[k] = wave_sum(v[k]);
#pragma unroll
  for (int k = NS; k < NS + NM; ++k) v[k] = wave_max(v[k]);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NS + NM; ++k) red[w][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < TEAM / 64; ++q) {
#pragma unroll
      for (int k = 0; k < NS; ++k) v[k] += red[q][k];
#pragma unroll
      for (int k = NS; k < NS + NM; ++k) v[k] = fmax(v[k], red[q][k]);
    }
  }
  __syncthreads();
}

// Shared state of a team while it works on one system.
struct TeamShared {
  double4 x[kMaxAtoms];          // positions (w: F'(rho) of the EAM form)
  unsigned short cat[kMaxAtoms];  // atoms sorted by cell
  int cstart[kMaxCells + 1];
  int cnt[kMaxCells];
  double red[16][kRedWidth];
  double lo[3], inv[3];
  int nc[3], lo_off[3], hi_off[3];
  int sys, status, viol, overflow;
  int phase, fetch;  // pair barriers passed, systems fetched by a pair (this launch)
  // coefficients of the next update
  int neg, mix_first, prec;
  double hsb, k1, k2, k3, cv, cf, dtx;
  double etab[32];  // table of the FP64 exponential
  Ctrl mine;        // the system's control record while the team works on it
};

// Two blocks (on two CUs) can share one large system as a pair: each takes
// one of the system's two halves of atoms (Team below).  Each block updates,
// lists and evaluates its own atoms and keeps all positions in its LDS; the
// blocks meet at barriers where they exchange positions, F'(rho), the skin
// and list-overflow flags and their reduction records through
// device-coherent loads and stores.  Both then run the same FIRE control on
// the same combined record, and the first block writes the system's control
// record back.  A team alone works through both halves with the same thread
// mapping, keeps them in separate records and combines them the same way, so
// a system gets the same bits whether a pair or a team alone relaxes it.
struct PairSlot {
  int bar;       // arrivals at the pair's barriers in this launch
  int sys[2];    // the system the first block fetched (by parity of the fetch; -1: none left)
  int vflag[2];  // per block: one of its atoms left its skin
  int oflag[2];  // per block: its list build overflowed or found coinciding atoms
  int pad;
  double rec[2][8];  // per block: its reduction record
  double pad2[12];
};
static_assert(sizeof(PairSlot) == 256, "one pair slot per 256 bytes");
static_assert(sizeof(Ctrl) % 8 == 0, "control records are copied in 8-byte words");

__device__ __forceinline__ void st_co(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_co(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_co_i(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_co_i(const int* p) {
  return __hip_atomic_load(const_cast<int*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Barrier of the two blocks of a pair.  Every thread's device-coherent stores
// have completed before its block arrives (no cache-wide fence: the data the
// blocks exchange is stored and loaded device-coherently).  The wait is
// bounded: a partner that does not arrive within kPairWaitTicks sets *err and
// the function returns false, after which the caller leaves the kernel.
__device__ bool pair_barrier(PairSlot* ps, TeamShared& sh, int* err) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0 && sh.phase >= 0) {
    const int target = 2 * (++sh.phase);
    __hip_atomic_fetch_add(&ps->bar, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const long long t0 = wall_clock64();
    while (ld_co_i(&ps->bar) < target) {
      __builtin_amdgcn_s_sleep(2);
      if (wall_clock64() - t0 > kPairWaitTicks) {
        atomicOr(err, 1);
        sh.phase = -1;
        break;
      }
    }
  }
  __syncthreads();
  return sh.phase >= 0;
}

// A control record copied between global memory and LDS by the whole block.
__device__ __forceinline__ void copy_ctrl(Ctrl* __restrict__ dst, const Ctrl* __restrict__ src) {
  const long long* s = reinterpret_cast<const long long*>(src);
  long long* d = reinterpret_cast<long long*>(dst);
  for (int i = threadIdx.x; i < (int)(sizeof(Ctrl) / 8); i += blockDim.x) d[i] = s[i];
}

template <int TEAM, int MAXPT>
struct Team {
  TeamShared& sh;
  const SysDesc& d;
  int n;
  // velocity, force and the skin reference live in the global per-atom
  // arrays (indexed d.off + a), read and written coalesced
  double4* __restrict__ vel;
  double4* __restrict__ frc;
  double4* __restrict__ xref;
  PairSlot* ps;  // the pair's slot (null: a team alone)
  int half;      // 0 or 1 within a pair
  // The atoms form two halves, [0, m) and [m, n): m = (n + 1) / 2 above 1.5
  // team widths, else min(n, TEAM) (so a team alone needs no extra round of
  // its threads for a system of up to 1.5 widths).  A pair's block h works on
  // half h; a team alone on both, one after the other, each half in its own
  // reduction record.
  int m;       // start of the second half
  int h0, h1;  // the halves this block works on: [h0, h1)

  __device__ Team(TeamShared& s, const SysDesc& desc, double4* v, double4* f, double4* xr, PairSlot* slot, int h)
      : sh(s), d(desc), n(desc.n), vel(v + desc.off), frc(f + desc.off), xref(xr + desc.off), ps(slot),
        half(slot ? h : 0) {
    m = 2 * n > 3 * TEAM ? (n + 1) / 2 : min(n, TEAM);
    h0 = slot ? h : 0;
    h1 = slot ? h + 1 : 2;
  }

  __device__ bool paired() const { return ps != nullptr; }
  // the k-th atom of this thread in half h (increasing in k; >= end(h): none)
  __device__ int atom(int h, int k) const { return (h ? m : 0) + (int)threadIdx.x + k * TEAM; }
  __device__ int end(int h) const { return h ? n : m; }
  // the k-th of all atoms (cell lists are built over the whole system)
  __device__ int any_atom(int k) const { return (int)threadIdx.x + k * TEAM; }
  __device__ bool owns(int a) const { return !ps || (half ? a >= m : a < m); }

  // Cell list and neighbour list of the current positions (wrapped into the
  // box on periodic axes).  Lists: nbr[off*kb + k*n + a], counts nn[off + a].
  // Each list holds the atoms within the cutoff (rc2) at build time first,
  // then the rest of the skin, each part in the order of the cell sweep, so
  // that the FP64 passes can skip groups of four beyond the cutoff.  Each
  // block of a pair wraps and sorts all atoms (the same arithmetic, so both
  // LDS copies agree) and lists its own; the blocks then share their overflow
  // flags.  Returns false when a pair barrier timed out.
  __device__ bool build(unsigned short* __restrict__ nbr, unsigned short* __restrict__ nn, int kb, double rc2,
                        int* err) {
    double lo3[3], hi3[3];
    for (int q = 0; q < 3; ++q) {
      lo3[q] = INFINITY;
      hi3[q] = -INFINITY;
    }
#pragma unroll 1
    for (int k = 0; k < MAXPT; ++k) {
      const int a = any_atom(k);
      if (a >= n) break;
      double4 p = sh.x[a];
      double r[3] = {p.x, p.y, p.z};
      for (int q = 0; q < 3; ++q) {
        if (d.box.per[q]) {
          double t = r[q] - d.box.lo[q];
          t -= d.box.L[q] * floor(t * d.box.invL[q]);
          if (t >= d.box.L[q]) t -= d.box.L[q];
          if (t < 0.0) t = 0.0;
          r[q] = d.box.lo[q] + t;
        }
        lo3[q] = fmin(lo3[q], r[q]);
        hi3[q] = fmax(hi3[q], r[q]);
      }
      sh.x[a] = make_double4(r[0], r[1], r[2], p.w);
      if (owns(a)) xref[a] = make_double4(r[0], r[1], r[2], 0.0);
    }
    // bounding box of the free axes
    double bb[6] = {-lo3[0], -lo3[1], -lo3[2], hi3[0], hi3[1], hi3[2]};
    {
      const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
      for (int q = 0; q < 6; ++q) bb[q] = wave_max(bb[q]);
      if (lane == 0)
        for (int q = 0; q < 6; ++q) sh.red[w][q] = bb[q];
      __syncthreads();
      if (threadIdx.x == 0) {
        for (int w2 = 1; w2 < TEAM / 64; ++w2)
          for (int q = 0; q < 6; ++q) bb[q] = fmax(bb[q], sh.red[w2][q]);
        const double rcs = sqrt(d.rcs2);
        int total = 1;
        double ext3[3];
        for (int q = 0; q < 3; ++q) {
          double lo, ext;
          if (d.box.per[q]) {
            lo = d.box.lo[q];
            ext = d.box.L[q];
          } else {
            lo = -bb[q];
            ext = bb[3 + q] + bb[q];
          }
          int nc = (int)floor(ext / (rcs * (1.0 + 1e-9)));
          nc = max(1, min(nc, 64));
          sh.nc[q] = nc;
          sh.lo[q] = lo;
          sh.inv[q] = ext > 0 ? nc / ext : 0.0;
          ext3[q] = ext;
          if (d.box.per[q]) {
            sh.lo_off[q] = nc >= 3 ? -1 : 0;
            sh.hi_off[q] = nc >= 2 ? 1 : 0;
          } else {
            sh.lo_off[q] = -1;
            sh.hi_off[q] = 1;
          }
          total *= nc;
        }
        // coarsen until the grid fits in LDS
        while (total > kMaxCells) {
          int q = 0;
          for (int z = 1; z < 3; ++z)
            if (sh.nc[z] > sh.nc[q]) q = z;
          sh.nc[q] = (sh.nc[q] + 1) / 2;
          sh.inv[q] = ext3[q] > 0 ? sh.nc[q] / ext3[q] : 0.0;
          if (d.box.per[q]) {
            sh.lo_off[q] = sh.nc[q] >= 3 ? -1 : 0;
            sh.hi_off[q] = sh.nc[q] >= 2 ? 1 : 0;
          }
          total = sh.nc[0] * sh.nc[1] * sh.nc[2];
        }
        sh.overflow = 0;
      }
    }
    __syncthreads();
    const int ncell = sh.nc[0] * sh.nc[1] * sh.nc[2];
    auto cell_of = [&](const double4& p) {
      const double r[3] = {p.x, p.y, p.z};
      int cc[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) cc[q] = min(max((int)floor((r[q] - sh.lo[q]) * sh.inv[q]), 0), sh.nc[q] - 1);
      return cc[0] + sh.nc[0] * (cc[1] + sh.nc[1] * cc[2]);
    };
    for (int c = threadIdx.x; c < ncell; c += TEAM) sh.cnt[c] = 0;
    __syncthreads();
#pragma unroll 1
    for (int k = 0; k < MAXPT; ++k) {
      const int a = any_atom(k);
      if (a >= n) break;
      atomicAdd(&sh.cnt[cell_of(sh.x[a])], 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int acc = 0;
      for (int c = 0; c < ncell; ++c) {
        sh.cstart[c] = acc;
        acc += sh.cnt[c];
        sh.cnt[c] = 0;
      }
      sh.cstart[ncell] = acc;
    }
    __syncthreads();
#pragma unroll 1
    for (int k = 0; k < MAXPT; ++k) {
      const int a = any_atom(k);
      if (a >= n) break;
      const int c = cell_of(sh.x[a]);
      sh.cat[sh.cstart[c] + atomicAdd(&sh.cnt[c], 1)] = (unsigned short)a;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < ncell; c += TEAM) {  // deterministic order: by atom index
      const int b = sh.cstart[c], e = sh.cstart[c + 1];
      for (int p = b + 1; p < e; ++p) {
        const unsigned short v0 = sh.cat[p];
        int q = p - 1;
        while (q >= b && sh.cat[q] > v0) {
          sh.cat[q + 1] = sh.cat[q];
          --q;
        }
        sh.cat[q + 1] = v0;
      }
    }
    __syncthreads();
    const size_t base = (size_t)d.off * kb;
    const Img img(d);
#pragma unroll 1
    for (int h = h0; h < h1; ++h)
#pragma unroll 1
    for (int k = 0; k < MAXPT; ++k) {
      const int a = atom(h, k);
      if (a >= end(h)) break;
      const double4 pa = sh.x[a];
      const int c0 = cell_of(pa);
      const int cc[3] = {c0 % sh.nc[0], (c0 / sh.nc[0]) % sh.nc[1], c0 / (sh.nc[0] * sh.nc[1])};
      int m = 0, mb = 0;  // entries from the front (within rc) and from the back (the rest)
      for (int oz = sh.lo_off[2]; oz <= sh.hi_off[2]; ++oz) {
        int cz = cc[2] + oz;
        if (d.box.per[2]) cz = (cz + sh.nc[2]) % sh.nc[2];
        else if (cz < 0 || cz >= sh.nc[2]) continue;
        for (int oy = sh.lo_off[1]; oy <= sh.hi_off[1]; ++oy) {
          int cy = cc[1] + oy;
          if (d.box.per[1]) cy = (cy + sh.nc[1]) % sh.nc[1];
          else if (cy < 0 || cy >= sh.nc[1]) continue;
          for (int ox = sh.lo_off[0]; ox <= sh.hi_off[0]; ++ox) {
            int cx = cc[0] + ox;
            if (d.box.per[0]) cx = (cx + sh.nc[0]) % sh.nc[0];
            else if (cx < 0 || cx >= sh.nc[0]) continue;
            const int cell = cx + sh.nc[0] * (cy + sh.nc[1] * cz);
            for (int p = sh.cstart[cell], e = sh.cstart[cell + 1]; p < e; ++p) {
              const int j = sh.cat[p];
              if (j == a) continue;
              const double4 pj = sh.x[j];
              double dx = pa.x - pj.x, dy = pa.y - pj.y, dz = pa.z - pj.z;
              img.apply(dx, dy, dz);
              const double r2 = dx * dx + dy * dy + dz * dz;
              if (r2 == 0.0) atomicOr(&sh.overflow, 2);
              if (r2 < d.rcs2) {
                const bool in = r2 < rc2;
                if (m + mb < kb) nbr[nidx(base, n, a, in ? m : kb - 1 - mb)] = (unsigned short)j;
                m += in;
                mb += !in;
              }
            }
          }
        }
      }
      // the skin entries move from the back to follow the others: that must
      // not overwrite one not yet moved, so the capacity must hold m + 2 mb
      if (m + 2 * mb > kb) atomicOr(&sh.overflow, 1);
      else
        for (int f = 0; f < mb; ++f) nbr[nidx(base, n, a, m + f)] = nbr[nidx(base, n, a, kb - 1 - f)];
      m += mb;
      for (int q = m; q < ((m + 3) & ~3) && q < kb; ++q) nbr[nidx(base, n, a, q)] = (unsigned short)a;
      nn[d.off + a] = (unsigned short)min(m, kb);
    }
    __syncthreads();
    if (ps) {
      if (threadIdx.x == 0) st_co_i(&ps->oflag[half], sh.overflow);
      if (!pair_barrier(ps, sh, err)) return false;
      if (threadIdx.x == 0) sh.overflow |= ld_co_i(&ps->oflag[half ^ 1]);
      __syncthreads();
    }
    return true;
  }
};

// Pair terms shared by the passes (branch-free; callers mask by `in`).
template <typename T, bool TAPER = true>
__device__ __forceinline__ T gupta_density_term(double r2, const PotDev& P, const double* __restrict__ etab) {
  T r;
  if constexpr (sizeof(T) == 8) r = r2 * rsqrt_d(r2);
  else r = sqrt_f((float)r2);
  T S = 1;  // the taper is 1 below r_in
  if constexpr (TAPER) {
    const T s = fmin(fmax((r - (T)P.r_in) * (T)P.inv_w, (T)0), (T)1);
    S = (1 - s) * (1 - s) * (1 + 2 * s);
  }
  if constexpr (sizeof(T) == 8) return exp_t(-P.qr0 * (r - P.r0), etab) * S;
  else return exp_f(-(T)P.qr0 * (r - (T)P.r0)) * S;
}

// Neighbour loop of the team passes: groups of four indices, the next group
// loaded while the current one is processed; pair(q, m, pj) gets the entry
// number q (entries q >= m are padding and must be masked) and the position.
template <int TEAM, int MAXPT, typename F>
__device__ __forceinline__ void for_team_neighbours(const Team<TEAM, MAXPT>& tm,
                                                    const unsigned short* __restrict__ nbr,
                                                    const unsigned short* __restrict__ nn, size_t base, int a,
                                                    F&& group) {
  const int m = nn[tm.d.off + a];
  const int ng = (m + 3) >> 2;
  const ushort4* l4 = reinterpret_cast<const ushort4*>(nbr + base) + a;
  const size_t stride = (size_t)tm.n;  // ushort4 elements between an atom's groups
  ushort4 cur = ng > 0 ? l4[0] : make_ushort4(0, 0, 0, 0);
  for (int g = 0; g < ng; ++g) {
    const ushort4 c = cur;
    if (g + 1 < ng) cur = l4[(size_t)(g + 1) * stride];
    group(4 * g, m, tm.sh.x[c.x], tm.sh.x[c.y], tm.sh.x[c.z], tm.sh.x[c.w]);
  }
}

// One group of four list entries (numbers q0 .. q0+3 of m) of the team
// passes: pair(q, pj, taper) for each.  In FP64 the group is skipped when
// no active lane has an entry of it within the cutoff, and the taper is
// evaluated only when one is past r_in; FP32 terms stay branch-free (as in
// the single-system passes).
template <typename T, typename F>
__device__ __forceinline__ void team_group(const Img& img, const double4& pa, const PotDev& P, int q0, int m,
                                           const double4& p0, const double4& p1, const double4& p2,
                                           const double4& p3, F&& pair) {
  if constexpr (sizeof(T) == 4) {
    pair(q0, p0, std::true_type{});
    pair(q0 + 1, p1, std::true_type{});
    pair(q0 + 2, p2, std::true_type{});
    pair(q0 + 3, p3, std::true_type{});
  } else {
    auto r2of = [&](const double4& pj) {
      double dx = pa.x - pj.x, dy = pa.y - pj.y, dz = pa.z - pj.z;
      img.apply(dx, dy, dz);
      return dx * dx + dy * dy + dz * dz;
    };
    const double a[4] = {r2of(p0), r2of(p1), r2of(p2), r2of(p3)};
    bool any = false, past = false;
    const double t2 = P.kind == FIRE_POT_GUPTA ? P.r_in * P.r_in * (1.0 - 1e-12) : P.rc2;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool in = q0 + u < m && a[u] < P.rc2;
      any = any || in;
      past = past || (in && a[u] > t2);
    }
    if (!wave_any(any)) return;
    if (wave_any(past)) {
      pair(q0, p0, std::true_type{});
      pair(q0 + 1, p1, std::true_type{});
      pair(q0 + 2, p2, std::true_type{});
      pair(q0 + 3, p3, std::true_type{});
    } else {
      pair(q0, p0, std::false_type{});
      pair(q0 + 1, p1, std::false_type{});
      pair(q0 + 2, p2, std::false_type{});
      pair(q0 + 3, p3, std::false_type{});
    }
  }
}

template <int TEAM, int MAXPT, typename T>
__device__ bool density_pass(Team<TEAM, MAXPT>& tm, const PotDev& P, const unsigned short* __restrict__ nbr,
                             const unsigned short* __restrict__ nn, int kb, double* __restrict__ xfp, int* err,
                             double& embA, double& embB) {
  const SysDesc& d = tm.d;
  const size_t base = (size_t)d.off * kb;
  const Img img(d);
  // F'(rho) of the team's atoms is parked in frc[a].w (the force pass
  // rewrites frc) until every neighbour read of the old values is done; a
  // pair also stores it device-coherently in xfp for the partner
#pragma unroll 1
  for (int h = tm.h0; h < tm.h1; ++h)
#pragma unroll 1
  for (int k = 0; k < MAXPT; ++k) {
    const int a = tm.atom(h, k);
    if (a >= tm.end(h)) break;
    const double4 pa = tm.sh.x[a];
    T rho = 0;
    const int m = nn[d.off + a];  // list length (entries past it are padding)
    auto pair = [&](int q, const double4& pj, auto taper) {
      double dx = pa.x - pj.x, dy = pa.y - pj.y, dz = pa.z - pj.z;
      img.apply(dx, dy, dz);
      const double r2 = dx * dx + dy * dy + dz * dz;
      const bool in = q < m && r2 < P.rc2;
      const T v = gupta_density_term<T, decltype(taper)::value>(in ? r2 : 1.0, P, tm.sh.etab);
      rho += in ? v : (T)0;
    };
    for_team_neighbours(tm, nbr, nn, base, a,
                        [&](int q0, int mm, const double4& p0, const double4& p1, const double4& p2,
                            const double4& p3) { team_group<T>(img, pa, P, q0, mm, p0, p1, p2, p3, pair); });
    double fp = 0.0;
    if (rho > 0) {
      const double sq = sqrt((double)rho);
      fp = -0.5 * P.xi / sq;
      if (h) embB += -P.xi * sq;
      else embA += -P.xi * sq;
    }
    reinterpret_cast<double*>(&tm.frc[a])[3] = fp;
    if (tm.paired()) st_co(xfp + d.off + a, fp);
  }
  __syncthreads();  // every neighbour read of w done before it changes
#pragma unroll 1
  for (int h = tm.h0; h < tm.h1; ++h)
#pragma unroll 1
  for (int k = 0; k < MAXPT; ++k) {
    const int a = tm.atom(h, k);
    if (a >= tm.end(h)) break;
    tm.sh.x[a].w = reinterpret_cast<const double*>(&tm.frc[a])[3];
  }
  if (tm.paired()) {
    if (!pair_barrier(tm.ps, tm.sh, err)) return false;
    const int h = tm.half ^ 1;
#pragma unroll 1
    for (int k = 0; k < MAXPT; ++k) {
      const int a = tm.atom(h, k);
      if (a >= tm.end(h)) break;
      tm.sh.x[a].w = ld_co(xfp + d.off + a);
    }
  }
  __syncthreads();
  return true;
}

template <int TEAM, int MAXPT, int POT, typename T>
__device__ void force_pass(Team<TEAM, MAXPT>& tm, const PotDev& P, const unsigned short* __restrict__ nbr,
                           const unsigned short* __restrict__ nn, int kb, double (&rA)[4], double (&rB)[4],
                           double (&mx)[2]) {
  const SysDesc& d = tm.d;
  const size_t base = (size_t)d.off * kb;
  const Img img(d);
  const double k3 = tm.sh.k3;
#pragma unroll 1
  for (int h = tm.h0; h < tm.h1; ++h)
#pragma unroll 1
  for (int k = 0; k < MAXPT; ++k) {
    const int a = tm.atom(h, k);
    if (a >= tm.end(h)) break;
    const double4 pa = tm.sh.x[a];
    T ax = 0, ay = 0, az = 0, ae = 0;
    const int m = nn[d.off + a];  // list length (entries past it are padding)
    auto pair = [&](int q, const double4& pj, auto taper) {
      double dx = pa.x - pj.x, dy = pa.y - pj.y, dz = pa.z - pj.z;
      img.apply(dx, dy, dz);
      const double r2 = dx * dx + dy * dy + dz * dz;
      const bool in = q < m && r2 < P.rc2;
      const double r2c = in ? r2 : 1.0;
      T fr, e;
      if constexpr (POT == FIRE_POT_LJ) {
        T ir2;
        if constexpr (sizeof(T) == 8) ir2 = rcp_d(r2c);
        else ir2 = rcp_f((float)r2c);
        const T s2 = (T)P.sig2 * ir2, s6 = s2 * s2 * s2;
        fr = (T)(24.0 * P.eps) * s6 * ((T)2 * s6 - (T)1) * ir2;
        e = (T)0.5 * ((T)(4.0 * P.eps) * s6 * (s6 - (T)1) - (T)P.shift);
      } else {
        T ir;
        if constexpr (sizeof(T) == 8) ir = rsqrt_d(r2c);
        else ir = rsqrt_f((float)r2c);
        const T rr = (T)r2c * ir;
        T S = 1, dS = 0;  // the taper and its slope are 1 and 0 below r_in
        if constexpr (decltype(taper)::value) {
          const T s = fmin(fmax((rr - (T)P.r_in) * (T)P.inv_w, (T)0), (T)1);
          S = (1 - s) * (1 - s) * (1 + 2 * s);
          dS = (T)(-6) * s * (1 - s) * (T)P.inv_w;
        }
        T ph, rh;
        if constexpr (sizeof(T) == 8) {
          ph = P.A * exp_t(-P.pr0 * (rr - P.r0), tm.sh.etab);
          rh = exp_t(-P.qr0 * (rr - P.r0), tm.sh.etab);
        } else {
          ph = (T)P.A * exp_f(-(T)P.pr0 * (rr - (T)P.r0));
          rh = exp_f(-(T)P.qr0 * (rr - (T)P.r0));
        }
        const T dEdr = (T)P.cpair * ph * (dS - (T)P.pr0 * S) + ((T)pa.w + (T)pj.w) * rh * (dS - (T)P.qr0 * S);
        fr = -dEdr * ir;
        e = (T)P.epair * ph * S;
      }
      fr = in ? fr : (T)0;
      ax += fr * (T)dx;
      ay += fr * (T)dy;
      az += fr * (T)dz;
      ae += in ? e : (T)0;
    };
    for_team_neighbours(tm, nbr, nn, base, a,
                        [&](int q0, int mm, const double4& p0, const double4& p1, const double4& p2,
                            const double4& p3) { team_group<T>(img, pa, P, q0, mm, p0, p1, p2, p3, pair); });
    double4 v = tm.vel[a];
    const double fx = ax, fy = ay, fz = az;
    tm.frc[a] = make_double4(fx, fy, fz, 0.0);
    if (k3 != 0.0) {
      v.x += k3 * fx;
      v.y += k3 * fy;
      v.z += k3 * fz;
      tm.vel[a] = v;
    }
    const double f2 = fx * fx + fy * fy + fz * fz, v2 = v.x * v.x + v.y * v.y + v.z * v.z;
    auto acc = [&](double (&r)[4]) {
      r[0] += (double)ae;
      r[1] += fx * v.x + fy * v.y + fz * v.z;
      r[2] += f2;
      r[3] += v2;
    };
    if (h) acc(rB);
    else acc(rA);
    mx[0] = fmax(mx[0], f2);
    mx[1] = fmax(mx[1], v2);
  }
}

// One force evaluation of the team's system and the FIRE control that
// follows it, on the control record in LDS.  Returns false when a pair
// barrier timed out.
template <int TEAM, int MAXPT, int POT>
__device__ bool evaluate(Team<TEAM, MAXPT>& tm, const PotDev& P, const unsigned short* __restrict__ nbr,
                         const unsigned short* __restrict__ nn, int kb, double* __restrict__ xfp, int* err) {
  double rA[4] = {0, 0, 0, 0}, rB[4] = {0, 0, 0, 0}, mx[2] = {0, 0};
  double embA = 0.0, embB = 0.0;
  const int prec = tm.sh.prec;
  if constexpr (POT == FIRE_POT_GUPTA) {
    const bool ok = prec ? density_pass<TEAM, MAXPT, float>(tm, P, nbr, nn, kb, xfp, err, embA, embB)
                         : density_pass<TEAM, MAXPT, double>(tm, P, nbr, nn, kb, xfp, err, embA, embB);
    if (!ok) return false;
  }
  if (prec) force_pass<TEAM, MAXPT, POT, float>(tm, P, nbr, nn, kb, rA, rB, mx);
  else force_pass<TEAM, MAXPT, POT, double>(tm, P, nbr, nn, kb, rA, rB, mx);
  rA[0] += embA;
  rB[0] += embB;
  // the record: E, P, |F|^2, |v|^2 summed over each half of the atoms
  // separately, then added; max |F|^2 and max |v|^2
  double t[6];
  if (tm.paired()) {
    // a pair's block accumulated its half in the record of that half
    double v[6];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = tm.half ? rB[k] : rA[k];
    v[4] = mx[0];
    v[5] = mx[1];
    team_reduce<TEAM, 4, 2>(v, tm.sh.red);
    if (threadIdx.x == 0)
#pragma unroll
      for (int k = 0; k < 6; ++k) st_co(&tm.ps->rec[tm.half][k], v[k]);
    if (!pair_barrier(tm.ps, tm.sh, err)) return false;
    if (threadIdx.x == 0)
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const double a = ld_co(&tm.ps->rec[0][k]), b = ld_co(&tm.ps->rec[1][k]);
        t[k] = k < 4 ? a + b : fmax(a, b);
      }
  } else {
    double v[10] = {rA[0], rA[1], rA[2], rA[3], rB[0], rB[1], rB[2], rB[3], mx[0], mx[1]};
    team_reduce<TEAM, 8, 2>(v, tm.sh.red);
#pragma unroll
    for (int k = 0; k < 4; ++k) t[k] = v[k] + v[4 + k];
    t[4] = v[8];
    t[5] = v[9];
  }
  if (threadIdx.x == 0) {
    Ctrl* c = &tm.sh.mine;
    // unit masses: the mass-weighted sums are P and |F|^2
    const double q[kCtl] = {t[0], t[1], t[2], t[3], t[4], t[5], t[1], t[2]};
    fire_control(*c, c, q, nullptr);
    if (c->status == ST_PAUSED && c->pause == PAUSE_PRECISION) {
      c->status = ST_RUNNING;  // the team switches its own pair precision
      c->pause = 0;
    }
    tm.sh.status = c->status;
    tm.sh.neg = c->neg;
    tm.sh.mix_first = c->mix_first;
    tm.sh.prec = c->precision;
    tm.sh.hsb = c->hsb;
    tm.sh.k1 = c->kick1;
    tm.sh.k2 = c->kick2;
    tm.sh.k3 = c->kick3;
    tm.sh.cv = c->cv;
    tm.sh.cf = c->cf;
    tm.sh.dtx = c->dtx;
  }
  __syncthreads();
  return true;
}

// Persistent team kernel: pull systems from the queues, advance each by up
// to `chunk` iterations.  Arrays are indexed by the concatenated atom index.
// order[0, nheavy) are the large systems, taken by the first 2 npairs blocks
// as pairs; once those are all taken the pairs split and, with the other
// blocks, take order[nheavy, nsys) one block each.  queue: [0] head of the
// second queue, [2] list-capacity flag, [4] head of the first, [5] set when a
// pair barrier timed out.
template <int TEAM, int MAXPT, int POT>
__global__ __launch_bounds__(TEAM) void k_batched(const SysDesc* __restrict__ desc, Ctrl* __restrict__ ctrl,
                                                  const int* __restrict__ order, int nsys, int nheavy, int npairs,
                                                  PairSlot* __restrict__ pslots, double* __restrict__ xfp,
                                                  int* __restrict__ queue, double4* __restrict__ pos,
                                                  double4* __restrict__ vel, double4* __restrict__ frc,
                                                  double4* __restrict__ xref, unsigned short* __restrict__ nbr,
                                                  unsigned short* __restrict__ nn, int kb, PotDev P, int chunk) {
  __shared__ TeamShared sh;
  exp_table_fill(sh.etab);  // published by the loop's first barrier
  int* const flags = queue + 2;
  int* const err = queue + 5;
  PairSlot* slot = (int)blockIdx.x < 2 * npairs ? pslots + (blockIdx.x >> 1) : nullptr;
  const int half = blockIdx.x & 1;
  if (threadIdx.x == 0) {
    sh.phase = 0;
    sh.fetch = 0;
  }
  for (;;) {
    // ---- the next system: a pair's first block fetches and publishes it
    if (slot) {
      if (threadIdx.x == 0 && half == 0) {
        const int q = atomicAdd(queue + 4, 1);
        st_co_i(&slot->sys[sh.fetch & 1], q < nheavy ? order[q] : -1);
      }
      if (!pair_barrier(slot, sh, err)) return;
      if (threadIdx.x == 0) sh.sys = ld_co_i(&slot->sys[sh.fetch++ & 1]);
    } else if (threadIdx.x == 0) {
      const int q = nheavy + atomicAdd(queue, 1);
      sh.sys = q < nsys ? order[q] : -1;
    }
    __syncthreads();
    const int s = sh.sys;
    if (s < 0) {
      if (!slot) return;
      slot = nullptr;  // no large system left: both blocks go on alone
      continue;
    }
    Ctrl* c = &ctrl[s];
    copy_ctrl(&sh.mine, c);
    __syncthreads();
    if (sh.mine.status != ST_RUNNING) continue;
    const SysDesc d = desc[s];
    Team<TEAM, MAXPT> tm(sh, d, vel, frc, xref, slot, half);
    for (int a = threadIdx.x; a < d.n; a += TEAM) sh.x[a] = pos[d.off + a];
    if (threadIdx.x == 0) {
      const Ctrl& m = sh.mine;
      sh.status = m.status;
      sh.viol = m.viol;
      sh.prec = m.precision;
      sh.neg = m.neg;
      sh.mix_first = m.mix_first;
      sh.hsb = m.hsb;
      sh.k1 = m.kick1;
      sh.k2 = m.kick2;
      sh.k3 = m.kick3;
      sh.cv = m.cv;
      sh.cf = m.cf;
      sh.dtx = m.dtx;
    }
    __syncthreads();
    bool ok = true, resume = true;
    if (sh.mine.evals == 0) {
      // first visit: a non-finite input position fails this system alone
      // (its positions stay as given; the queue moves on)
      int bad = 0;
      for (int a = threadIdx.x; a < d.n; a += TEAM) {
        const double4 p = sh.x[a];
        bad |= !(isfinite(p.x) && isfinite(p.y) && isfinite(p.z));
      }
      if (__syncthreads_or(bad)) {
        if (threadIdx.x == 0) sh.mine.status = FIRE_E_NONFINITE;
        resume = false;
      }
    }
    if (resume) {
      if (sh.viol) {  // first visit (or after a capacity change): build the list
        if (!tm.build(nbr, nn, kb, P.rc2, err)) return;
        if (sh.overflow) ok = false;
      }
      if (ok && sh.mine.evals == 0) {  // evaluation 0 and the set-up of iteration 1
        if (threadIdx.x == 0) sh.k3 = 0.0;
        __syncthreads();
        if (!evaluate<TEAM, MAXPT, POT>(tm, P, nbr, nn, kb, xfp, err)) return;
      }
      const double skin_half2 = sh.mine.skin_half2;
      for (int it = 0; ok && it < chunk && sh.status == ST_RUNNING; ++it) {
        // ---- update (same step as the single-system update kernel)
        int viol = 0;
#pragma unroll 1
        for (int h = tm.h0; h < tm.h1; ++h)
#pragma unroll
        for (int k = 0; k < MAXPT; ++k) {
          const int a = tm.atom(h, k);
          if (a >= tm.end(h)) break;
          const double4 p = sh.x[a];
          const double4 v0 = tm.vel[a], f0 = tm.frc[a], xr = tm.xref[a];
          double vv[3] = {v0.x, v0.y, v0.z};
          const double ff[3] = {f0.x, f0.y, f0.z};
          double xx[3] = {p.x, p.y, p.z};
          for (int q = 0; q < 3; ++q) {
            double vd = vv[q], xd = xx[q];
            if (sh.neg) {
              xd -= sh.hsb * vd;
              vd = 0.0;
            }
            if (sh.mix_first) vd = sh.cv * vd + sh.cf * ff[q];
            vd = vd + sh.k1 * ff[q];
            if (!sh.mix_first) vd = sh.cv * vd + sh.cf * ff[q];
            xd = xd + sh.dtx * vd;
            vd = vd + sh.k2 * ff[q];
            vv[q] = vd;
            xx[q] = xd;
          }
          tm.vel[a] = make_double4(vv[0], vv[1], vv[2], 0.0);
          sh.x[a] = make_double4(xx[0], xx[1], xx[2], p.w);
          if (slot) {
            double* g = reinterpret_cast<double*>(pos + d.off + a);
            st_co(g, xx[0]);
            st_co(g + 1, xx[1]);
            st_co(g + 2, xx[2]);
          }
          const double ex = xx[0] - xr.x, ey = xx[1] - xr.y, ez = xx[2] - xr.z;
          if (ex * ex + ey * ey + ez * ez > skin_half2) viol = 1;
        }
        if (threadIdx.x == 0) sh.viol = 0;
        __syncthreads();
        if (viol) sh.viol = 1;
        if (slot) {  // share the skin flags and the new positions
          __syncthreads();
          if (threadIdx.x == 0) st_co_i(&slot->vflag[half], sh.viol);
          if (!pair_barrier(slot, sh, err)) return;
          if (threadIdx.x == 0) sh.viol |= ld_co_i(&slot->vflag[half ^ 1]);
          const int h = half ^ 1;
#pragma unroll 1
          for (int k = 0; k < MAXPT; ++k) {
            const int a = tm.atom(h, k);
            if (a >= tm.end(h)) break;
            const double* g = reinterpret_cast<const double*>(pos + d.off + a);
            double4& x = sh.x[a];
            x.x = ld_co(g);
            x.y = ld_co(g + 1);
            x.z = ld_co(g + 2);
          }
        }
        __syncthreads();
        if (sh.viol) {
          if (!tm.build(nbr, nn, kb, P.rc2, err)) return;
          if (sh.overflow) {
            ok = false;
            break;
          }
        }
        if (!evaluate<TEAM, MAXPT, POT>(tm, P, nbr, nn, kb, xfp, err)) return;
      }
      if (!ok && threadIdx.x == 0) {
        // list capacity exceeded or atoms coincide: hand the system to the host
        if (sh.overflow & 2) sh.mine.status = FIRE_E_OVERLAP;
        else {
          sh.mine.status = ST_PAUSED;
          sh.mine.pause = PAUSE_REBUILD;
          if (half == 0 || !slot) atomicMax(&flags[0], 1);
        }
      }
      // write this block's positions back (v, F and the skin reference are in place)
#pragma unroll 1
      for (int h = tm.h0; h < tm.h1; ++h)
#pragma unroll 1
      for (int k = 0; k < MAXPT; ++k) {
        const int a = tm.atom(h, k);
        if (a >= tm.end(h)) break;
        pos[d.off + a] = sh.x[a];
      }
      if (threadIdx.x == 0) sh.mine.viol = ok ? 0 : 1;
    }
    // the control record back to global memory (by a pair's first block, once
    // the second has taken its copy)
    __syncthreads();
    if (slot && !pair_barrier(slot, sh, err)) return;
    if (!slot || half == 0) copy_ctrl(c, &sh.mine);
    __syncthreads();
  }
}

// Queue heads and pair barriers of one launch back to zero.
__global__ void k_reset_queue(int* queue, PairSlot* pslots, int npairs) {
  if (threadIdx.x == 0) {
    queue[0] = 0;
    queue[4] = 0;
  }
  for (int p = threadIdx.x; p < npairs; p += blockDim.x) pslots[p].bar = 0;
}

__global__ void k_zero_ints(int* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

__global__ void k_count_running(const Ctrl* __restrict__ ctrl, int nsys, int* __restrict__ out) {
  int r = 0;
  for (int s = threadIdx.x; s < nsys; s += blockDim.x)
    r += __hip_atomic_load(&ctrl[s].status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == ST_RUNNING;
  for (int o = 32; o > 0; o >>= 1) r += __shfl_xor(r, o, 64);
  __shared__ int sm[16];
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = r;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sm[w];
    *out = t;
  }
}

__global__ void k_stage(const double* __restrict__ src, int ntot, double4* __restrict__ pos,
                        double4* __restrict__ vel, double4* __restrict__ frc, double4* __restrict__ xref) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ntot) return;
  const double4 p = make_double4(src[3 * i], src[3 * i + 1], src[3 * i + 2], 0.0);
  pos[i] = p;
  xref[i] = p;
  vel[i] = make_double4(0, 0, 0, 0);
  frc[i] = make_double4(0, 0, 0, 0);
}

// Positions of system blockIdx.x back to the caller's AoS layout; periodic
// axes wrapped into [lo, lo + len) as the single-system path returns them.
__global__ void k_unstage(const double4* __restrict__ pos, const SysDesc* __restrict__ desc,
                          double* __restrict__ dst) {
  const SysDesc d = desc[blockIdx.x];
  for (int a = threadIdx.x; a < d.n; a += blockDim.x) {
    const int i = d.off + a;
    const double4 p = pos[i];
    double x[3] = {p.x, p.y, p.z};
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (d.box.per[k]) {
        double t = x[k] - d.box.lo[k];
        t -= d.box.L[k] * floor(t / d.box.L[k]);
        if (t >= d.box.L[k]) t -= d.box.L[k];
        if (t < 0) t = 0;
        x[k] = d.box.lo[k] + t;
      }
    dst[3 * i] = x[0];
    dst[3 * i + 1] = x[1];
    dst[3 * i + 2] = x[2];
  }
}

// ------------------------------------------------------------------ host

struct Config {
  int team, chunk;
};

using KernelFn = void (*)(const SysDesc*, Ctrl*, const int*, int, int, int, PairSlot*, double*, int*, double4*,
                          double4*, double4*, double4*, unsigned short*, unsigned short*, int, PotDev, int);

KernelFn kernel_for(int team, int pot) {
  if (pot == FIRE_POT_LJ) return team == 1024 ? k_batched<1024, 4, FIRE_POT_LJ> : k_batched<512, 8, FIRE_POT_LJ>;
  return team == 1024 ? k_batched<1024, 4, FIRE_POT_GUPTA> : k_batched<512, 8, FIRE_POT_GUPTA>;
}

struct Workspace {
  int nsys = 0, ntot = 0, kb = 0;
  int cap_sys = 0, cap_atoms = 0, cap_kb = 0;
  SysDesc* desc = nullptr;
  Ctrl* ctrl = nullptr;
  int* order = nullptr;
  int* queue = nullptr;  // [0] queue head, [1] running count, [2] flag, [4] queue head, [5] error
  int* h_small = nullptr;
  PairSlot* pslots = nullptr;  // kMaxPairs barriers of pairs of teams
  double* xfp = nullptr;       // F'(rho) exchange of pairs, per atom
  double* stage = nullptr;
  double4 *pos = nullptr, *vel = nullptr, *frc = nullptr, *xref = nullptr;
  unsigned short *nbr = nullptr, *nn = nullptr;
  std::map<std::string, Config> tuned;
};

void release(Workspace* w) {
  if (!w) return;
  hipFree(w->desc); hipFree(w->ctrl); hipFree(w->order); hipFree(w->queue); hipFree(w->stage);
  hipFree(w->pos); hipFree(w->vel); hipFree(w->frc); hipFree(w->xref); hipFree(w->nbr); hipFree(w->nn);
  hipFree(w->pslots); hipFree(w->xfp);
  if (w->h_small) hipHostFree(w->h_small);
  delete w;
}

}  // namespace bat
}  // namespace fire

using namespace fire;
using namespace fire::bat;

// Context accessors implemented in fire2.hip.
hipStream_t fire_ctx_stream(fire_ctx* ctx);
const fire_params* fire_ctx_params(fire_ctx* ctx);
void** fire_ctx_batched_slot(fire_ctx* ctx);
int fire_ctx_error(fire_ctx* ctx, int code, const char* msg);
void fire_ctx_set_tuning_info(fire_ctx* ctx, const char* info);
int fire_prepare_pot(fire_ctx* ctx, const fire_potential* p, PotDev* out);
void fire_ctrl_from_params(const fire_params* p, double tol, long long max_steps, double skin, int natoms, Ctrl* c);

namespace {

#define BCHK(call)                                                                                 \
  do {                                                                                             \
    hipError_t e_ = (call);                                                                        \
    if (e_ != hipSuccess)                                                                          \
      return fire_ctx_error(ctx, e_ == hipErrorOutOfMemory ? FIRE_E_OOM : FIRE_E_DEVICE,           \
                            (std::string(#call) + ": " + hipGetErrorString(e_)).c_str());          \
  } while (0)

template <typename T>
hipError_t balloc(T** p, size_t count) {
  *p = nullptr;
  return hipMalloc((void**)p, std::max<size_t>(count, 1) * sizeof(T));
}

int ensure(fire_ctx* ctx, Workspace* w, int nsys, int ntot, int kb) {
  if (nsys > w->cap_sys) {
    hipFree(w->desc); hipFree(w->ctrl); hipFree(w->order);
    BCHK(balloc(&w->desc, nsys));
    BCHK(balloc(&w->ctrl, nsys));
    BCHK(balloc(&w->order, nsys));
    w->cap_sys = nsys;
  }
  if (ntot > w->cap_atoms) {
    hipFree(w->stage); hipFree(w->pos); hipFree(w->vel); hipFree(w->frc); hipFree(w->xref); hipFree(w->nn);
    hipFree(w->xfp);
    BCHK(balloc(&w->stage, 3 * (size_t)ntot));
    BCHK(balloc(&w->xfp, ntot));
    BCHK(balloc(&w->pos, ntot));
    BCHK(balloc(&w->vel, ntot));
    BCHK(balloc(&w->frc, ntot));
    BCHK(balloc(&w->xref, ntot));
    BCHK(balloc(&w->nn, ntot));
    w->cap_atoms = ntot;
    w->cap_kb = 0;
  }
  if ((size_t)ntot * kb > (size_t)w->cap_atoms * w->cap_kb) {
    hipFree(w->nbr);
    BCHK(balloc(&w->nbr, (size_t)ntot * kb));
    w->cap_kb = kb;
  }
  if (!w->queue) {
    BCHK(balloc(&w->pslots, kMaxPairs));
    BCHK(balloc(&w->queue, 8));
    BCHK(hipHostMalloc((void**)&w->h_small, 8 * sizeof(int), hipHostMallocDefault));
  }
  return FIRE_OK;
}

// (Re)start every system from the staged input positions.
int reset_state(fire_ctx* ctx, Workspace* w, const std::vector<Ctrl>& c0, hipStream_t s) {
  hipLaunchKernelGGL(k_stage, dim3((w->ntot + 255) / 256), dim3(256), 0, s, w->stage, w->ntot, w->pos, w->vel,
                     w->frc, w->xref);
  BCHK(hipMemcpyAsync(w->ctrl, c0.data(), sizeof(Ctrl) * w->nsys, hipMemcpyHostToDevice, s));
  BCHK(hipStreamSynchronize(s));
  return FIRE_OK;
}

// Blocks of the persistent launch and the share of its systems taken by
// pairs of blocks.  A pair halves a system's atoms per block at the price of
// three barriers across CUs per iteration (1.7-1.8 times faster than a block
// alone above 1.5 team widths, no faster below), so only systems of more
// than 1.5 team widths are candidates.  With no more systems than CUs, spare
// CUs become the partners of the candidates of most work; with more, 3/8 of
// the CUs form pairs and take the 2.6 candidates each of most work, which
// brings the longest relaxations toward the mean load of a CU.
// FIRE_BATCH_PAIRS=0: no pairs; =force: every system a candidate; =P,H: P
// pairs for the H candidates of most work.  `order` is the queue order
// (decreasing work); `launch_order` receives the pairs' systems first, then
// the others in queue order.  Pairing changes no result: a system gets the
// same bits from a pair and from a block alone.
struct Launch {
  int nteams, npairs, nheavy;
};

Launch plan_launch(const SysDesc* desc, const int* order, int nsys, int ncu, int team, bool allow_pairs,
                   int* launch_order) {
  Launch l{std::min(nsys, ncu), 0, 0};
  const char* e = getenv("FIRE_BATCH_PAIRS");
  const bool off = !allow_pairs || (e && strcmp(e, "0") == 0) || ncu < 2;
  const bool force = e && strcmp(e, "force") == 0;
  auto candidate = [&](int q) { return force || desc[q].n > team * 3 / 2; };
  int cand = 0;
  for (int k = 0; k < nsys && !off; ++k) cand += candidate(order[k]);
  int fp = 0, fh = 0;
  if (off) {
  } else if (e && sscanf(e, "%d,%d", &fp, &fh) == 2) {
    l.npairs = std::max(0, std::min({fp, cand, ncu / 2}));
    l.nheavy = std::max(l.npairs, std::min(fh, cand));
  } else if (nsys <= ncu) {
    l.npairs = std::min(cand, ncu - nsys);
    l.nheavy = l.npairs;
  } else {
    l.npairs = std::min(cand, ncu * 3 / 8);
    l.nheavy = std::min(cand, l.npairs * 13 / 5);
  }
  l.npairs = std::min(l.npairs, kMaxPairs);
  l.nteams = std::min(ncu, std::max(2 * l.npairs, nsys + l.npairs));
  int h = 0, r = l.nheavy;
  for (int k = 0; k < nsys; ++k) {
    const int q = order[k];
    if (h < l.nheavy && candidate(q)) launch_order[h++] = q;
    else launch_order[r++] = q;
  }
  return l;
}

// One replay unit: reset the queues and run the persistent kernel once.
template <typename B>
void launch_chunk(const B* w, const PotDev& P, const Config& cf, const Launch& l, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(256), 0, s, w->queue, w->pslots, l.npairs);
  KernelFn fn = kernel_for(cf.team, P.kind);
  hipLaunchKernelGGL(fn, dim3(l.nteams), dim3(cf.team), 0, s, w->desc, w->ctrl, w->order, w->nsys, l.nheavy,
                     l.npairs, w->pslots, w->xfp, w->queue, w->pos, w->vel, w->frc, w->xref, w->nbr, w->nn, w->kb,
                     P, cf.chunk);
  hipLaunchKernelGGL(k_count_running, dim3(1), dim3(1024), 0, s, w->ctrl, w->nsys, w->queue + 1);
}

std::string tune_key(const PotDev& P, int prec, int nsys, int maxn) {
  std::ostringstream o;
  o << "pot" << P.kind << "_prec" << prec << "_nsys" << (nsys >= 256 ? 256 : (nsys >= 32 ? 32 : 1)) << "_maxn"
    << (maxn > 2048 ? 4096 : (maxn > 1024 ? 2048 : 1024));
  return o.str();
}

std::string cache_path() {
  const char* p = getenv("FIRE_TUNE_CACHE");
  if (p && *p) return p;
  const char* h = getenv("HOME");
  return std::string(h ? h : "/tmp") + "/.cache/fire2_tune.txt";
}

void load_cache(Workspace* w) {
  std::ifstream f(cache_path());
  std::string k;
  int t, c;
  while (f >> k >> t >> c)
    if (t == 512 || t == 1024) w->tuned[k] = Config{t, c};
}

void save_cache(Workspace* w) {
  std::ofstream f(cache_path());
  for (auto& kv : w->tuned) f << kv.first << " " << kv.second.team << " " << kv.second.chunk << "\n";
}

// Systems in decreasing estimated work, equal estimates in index order: the
// atom count times (3 + free axes) / 3, since a free surface lengthens a
// relaxation (the 512-system EAM-form batch: clusters 477 iterations on
// average, periodic boxes 235).  Longest first keeps the queue's tail short.
// Allocates nothing.
void order_by_work(const SysDesc* desc, int nsys, int* order) {
  auto work = [&](int q) {
    const SysDesc& d = desc[q];
    return (long long)d.n * (3 + !d.box.per[0] + !d.box.per[1] + !d.box.per[2]);
  };
  for (int q = 0; q < nsys; ++q) order[q] = q;
  std::sort(order, order + nsys, [&](int a, int b) {
    const long long wa = work(a), wb = work(b);
    return wa != wb ? wa > wb : a < b;
  });
}

struct BatchPlan {
  int nsys, ntot, maxn, kb;
  PotDev P;
};

// Check the arguments of a batched call and fill the per-system descriptors,
// the initial control records and the queue order into caller-owned arrays
// of nsys entries.  Allocates nothing.
int prepare_batch(fire_ctx* ctx, int nsys, const long long* offsets, const fire_box* boxes,
                  const fire_potential* pot, const fire_params* per_sys, double tol, long long max_steps,
                  SysDesc* desc, Ctrl* c0, int* order, BatchPlan* plan) {
  if (!(tol >= 0) || max_steps < 0) return fire_ctx_error(ctx, FIRE_E_ARG, "batched: bad tol or max_steps");
  if (pot->kind != FIRE_POT_LJ && pot->kind != FIRE_POT_GUPTA)
    return fire_ctx_error(ctx, FIRE_E_ARG, "batched: LJ or Gupta potentials only");
  if (offsets[0] != 0) return fire_ctx_error(ctx, FIRE_E_ARG, "batched: offsets[0] must be 0");
  int maxn = 0;
  for (int s = 0; s < nsys; ++s) {
    const long long n = offsets[s + 1] - offsets[s];
    if (n < 1 || n > kMaxAtoms)
      return fire_ctx_error(ctx, FIRE_E_ARG, "batched: every system needs 1 .. 4096 atoms");
    maxn = std::max<int>(maxn, (int)n);
  }
  const long long ntot_ll = offsets[nsys];
  if (ntot_ll > (1LL << 30)) return fire_ctx_error(ctx, FIRE_E_ARG, "batched: too many atoms");
  PotDev& P = plan->P;
  int rc = fire_prepare_pot(ctx, pot, &P);
  if (rc) return rc;
  const fire_params* base = fire_ctx_params(ctx);
  double max_dens_vol = 0.0;
  for (int q = 0; q < nsys; ++q) {
    const fire_box& b = boxes[q];
    const fire_params& prm = per_sys ? per_sys[q] : *base;
    SysDesc& d = desc[q];
    d.off = (int)offsets[q];
    d.n = (int)(offsets[q + 1] - offsets[q]);
    double skin = prm.skin > 0 ? prm.skin : 0.12 * P.rc;
    for (int k = 0; k < 3; ++k) {
      d.box.per[k] = b.periodic[k] ? 1 : 0;
      d.box.lo[k] = b.lo[k];
      d.box.L[k] = b.len[k];
      d.box.invL[k] = b.len[k] > 0 ? 1.0 / b.len[k] : 0.0;
      if (d.box.per[k]) {
        if (!(b.len[k] > 0) || !(P.rc < 0.5 * b.len[k]))
          return fire_ctx_error(ctx, FIRE_E_BOX, "batched: cutoff must be < len/2 on periodic axes");
        skin = std::min(skin, 0.9 * (0.5 * b.len[k] - P.rc));
      }
    }
    const double rcs = P.rc + skin;
    d.rcs2 = rcs * rcs;
    fire_ctrl_from_params(&prm, tol, max_steps, skin, d.n, &c0[q]);
    c0[q].viol = 1;  // build the list on the first visit
    // density estimate for the list capacity (periodic boxes; clusters use the bulk value)
    double vol = 1.0;
    bool all_per = true;
    for (int k = 0; k < 3; ++k) {
      all_per = all_per && d.box.per[k];
      vol *= b.len[k];
    }
    if (all_per && vol > 0) max_dens_vol = std::max(max_dens_vol, d.n / vol * rcs * rcs * rcs);
  }
  int kb = (int)(4.18879 * std::max(max_dens_vol, 0.1 * 1.0) * 1.6) + 24;
  kb = (std::max(kb, 32) + 3) & ~3;  // lists are read in groups of four
  order_by_work(desc, nsys, order);
  plan->nsys = nsys;
  plan->ntot = (int)ntot_ll;
  plan->maxn = maxn;
  plan->kb = kb;
  return FIRE_OK;
}

// Team shape and chunk length: FIRE_BATCH_TEAM / FIRE_BATCH_CHUNK, else a
// cached tuning result for this batch class, else (tune = false) 1024 threads.
Config config_for(Workspace* w, const BatchPlan& pl, int prec0, bool* found) {
  Config cfg{1024, kChunk};
  *found = false;
  if (const char* e = getenv("FIRE_BATCH_TEAM")) {
    cfg.team = atoi(e) == 512 ? 512 : 1024;
    *found = true;
  } else if (w) {
    auto it = w->tuned.find(tune_key(pl.P, prec0, pl.nsys, pl.maxn));
    if (it != w->tuned.end()) {
      cfg = it->second;
      *found = true;
    }
  }
  if (const char* e = getenv("FIRE_BATCH_CHUNK")) cfg.chunk = std::max(1, atoi(e));
  return cfg;
}

// Results of a finished batch from its control records.
void fill_results(const Ctrl* cr, const SysDesc* desc, int nsys, fire_result* out) {
  // a system that failed (two atoms at one place, a non-finite position or
  // force) reports its error code as its stop reason; the others keep theirs
  for (int q = 0; q < nsys; ++q) {
    const Ctrl& h = cr[q];
    fire_result& o = out[q];
    memset(&o, 0, sizeof(o));
    o.stop_reason = h.status;
    o.precision_switched = (h.mode == FIRE_MIXED && h.precision == 0) ? 1 : 0;
    o.iterations = h.iter;
    o.force_evals = h.evals;
    o.iterations_low = h.iter_low;
    o.energy = h.energy;
    o.energy_per_atom = h.energy / desc[q].n;
    o.fmax = h.fmax;
    o.f2norm = h.f2norm;
    o.dt = h.dt;
    o.alpha = h.alpha;
  }
}

}  // namespace

extern "C" void fire_batched_release(void* ws) { release(static_cast<Workspace*>(ws)); }

extern "C" int fire_batched_run(fire_ctx* ctx, int nsys, const long long* offsets, double* pos, bool host,
                                const fire_box* boxes, const fire_potential* pot, const fire_params* per_sys,
                                double tol, long long max_steps, fire_result* out, hipStream_t s) {
  if (nsys < 1 || !offsets || !pos || !boxes || !pot || !out)
    return fire_ctx_error(ctx, FIRE_E_ARG, "batched: nsys >= 1 and non-NULL arrays are required");
  std::vector<SysDesc> desc(nsys);
  std::vector<Ctrl> c0(nsys);
  std::vector<int> order(nsys), lorder(nsys);
  BatchPlan plan;
  int rc = prepare_batch(ctx, nsys, offsets, boxes, pot, per_sys, tol, max_steps, desc.data(), c0.data(),
                         order.data(), &plan);
  if (rc) return rc;
  const PotDev& P = plan.P;
  const int ntot = plan.ntot, maxn = plan.maxn;
  int kb = plan.kb;
  void** slot = fire_ctx_batched_slot(ctx);
  if (!*slot) {
    *slot = new Workspace();
    load_cache(static_cast<Workspace*>(*slot));
  }
  Workspace* w = static_cast<Workspace*>(*slot);

  for (int attempt = 0; attempt < 4; ++attempt) {
    rc = ensure(ctx, w, nsys, ntot, kb);
    if (rc) return rc;
    w->nsys = nsys;
    w->ntot = ntot;
    w->kb = kb;
    BCHK(hipMemcpyAsync(w->desc, desc.data(), sizeof(SysDesc) * nsys, hipMemcpyHostToDevice, s));
    BCHK(hipMemcpyAsync(w->stage, pos, sizeof(double) * 3 * ntot,
                        host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s));
    BCHK(hipMemsetAsync(w->queue, 0, 8 * sizeof(int), s));
    rc = reset_state(ctx, w, c0, s);
    if (rc) return rc;

    int dev = 0;
    BCHK(hipGetDevice(&dev));
    int ncu = 256;
    BCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));

    // ---- team shape: the cached choice, else timed on this batch (state reset afterwards)
    const int prec0 = c0[0].precision;
    bool found = false;
    Config cfg = config_for(w, plan, prec0, &found);
    char info[320];
    snprintf(info, sizeof info, "batched: %d-thread teams, chunks of %d iterations (%s)", cfg.team, cfg.chunk,
             getenv("FIRE_BATCH_TEAM") ? "FIRE_BATCH_TEAM" : "cached");
    if (!found) {
      double best = 1e300;
      float t[2] = {0, 0};
      int ti = 0;
      for (int team : {1024, 512}) {
        Config cand{team, 32};
        hipEvent_t e0, e1;
        BCHK(hipEventCreate(&e0));
        BCHK(hipEventCreate(&e1));
        const Launch l = plan_launch(desc.data(), order.data(), nsys, ncu, team, true, lorder.data());
        BCHK(hipMemcpyAsync(w->order, lorder.data(), sizeof(int) * nsys, hipMemcpyHostToDevice, s));
        launch_chunk(w, P, cand, l, s);  // includes the list build; not timed
        BCHK(hipEventRecord(e0, s));
        launch_chunk(w, P, cand, l, s);
        BCHK(hipEventRecord(e1, s));
        BCHK(hipEventSynchronize(e1));
        float ms = 0;
        BCHK(hipEventElapsedTime(&ms, e0, e1));
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        t[ti++] = ms;
        if (ms < best) {
          best = ms;
          cfg.team = team;
        }
        rc = reset_state(ctx, w, c0, s);
        if (rc) return rc;
      }
      w->tuned[tune_key(P, prec0, nsys, maxn)] = Config{cfg.team, kChunk};
      save_cache(w);
      snprintf(info, sizeof info, "batched: %d-thread teams, chunks of %d iterations (tuned: a 32-iteration chunk took "
               "%.2f ms with 1024-thread teams, %.2f with 512)", cfg.team, cfg.chunk, t[0], t[1]);
    }
    const Launch lau = plan_launch(desc.data(), order.data(), nsys, ncu, cfg.team, true, lorder.data());
    BCHK(hipMemcpyAsync(w->order, lorder.data(), sizeof(int) * nsys, hipMemcpyHostToDevice, s));
    const size_t used = strlen(info);
    snprintf(info + used, sizeof info - used, "; %d blocks, %d pairs of them for %d systems of most work", lau.nteams,
             lau.npairs, lau.nheavy);
    fire_ctx_set_tuning_info(ctx, info);

    // ---- graph: queue reset, persistent kernel, running count, poll copy
    hipGraph_t graph;
    hipGraphExec_t exec;
    hipStream_t cap;
    BCHK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    BCHK(hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed));
    launch_chunk(w, P, cfg, lau, cap);
    BCHK(hipMemcpyAsync(w->h_small, w->queue, 6 * sizeof(int), hipMemcpyDeviceToHost, cap));
    BCHK(hipStreamEndCapture(cap, &graph));
    BCHK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    hipGraphDestroy(graph);
    hipStreamDestroy(cap);
    const long long max_replays = max_steps / cfg.chunk + 4;
    bool need_more = false;
    for (long long r = 0; r <= max_replays; ++r) {
      BCHK(hipGraphLaunch(exec, s));
      BCHK(hipStreamSynchronize(s));
      if (w->h_small[5]) {
        hipGraphExecDestroy(exec);
        return fire_ctx_error(ctx, FIRE_E_DEVICE, "batched: a pair of teams timed out at a barrier");
      }
      if (w->h_small[2]) {  // a list outgrew its capacity
        need_more = true;
        break;
      }
      if (w->h_small[1] == 0) break;
    }
    hipGraphExecDestroy(exec);
    if (need_more) {
      kb = ((kb * 3 / 2 + 16) + 3) & ~3;
      continue;
    }
    // ---- results
    std::vector<Ctrl> cr(nsys);
    BCHK(hipMemcpyAsync(cr.data(), w->ctrl, sizeof(Ctrl) * nsys, hipMemcpyDeviceToHost, s));
    // positions back in caller order, periodic axes wrapped into [lo, lo + len)
    hipLaunchKernelGGL(k_unstage, dim3(nsys), dim3(256), 0, s, w->pos, w->desc, host ? w->stage : pos);
    if (host) BCHK(hipMemcpyAsync(pos, w->stage, sizeof(double) * 3 * ntot, hipMemcpyDeviceToHost, s));
    BCHK(hipStreamSynchronize(s));
    fill_results(cr.data(), desc.data(), nsys, out);
    return FIRE_OK;
  }
  return fire_ctx_error(ctx, FIRE_E_OOM, "batched: neighbour lists keep outgrowing their capacity");
}

// ------------------------------------------------- no-allocation variant
//
// fire_minimize_batched_noalloc runs the same kernels as the batched entry
// points on work buffers carved out of one file-scope device array (each GPU
// holds its own copy while the process lives), without graphs, for callers
// that must not allocate device memory.  Everything else it needs is set up
// once per context by fire_init: the array's device address (per device),
// a pinned word for the status polls and host staging records.

namespace fire {
namespace bat {
constexpr size_t kScratchBytes = size_t(64) << 20;  // work buffers of one call
constexpr int kNoAllocMaxSys = 1024;                  // systems per call
}  // namespace bat
}  // namespace fire

static __device__ __align__(256) unsigned char scratch[fire::bat::kScratchBytes];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_addr[64] = {};

// Device address of this device's scratch array (the device must be current).
int scratch_address(int device, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0 || device >= 64) return FIRE_E_DEVICE;
  if (!g_scratch_addr[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return FIRE_E_DEVICE;
    g_scratch_addr[device] = p;
  }
  *out = g_scratch_addr[device];
  return FIRE_OK;
}

struct NoAlloc {
  int device = -1;
  unsigned char* base = nullptr;  // scratch on `device`
  int* h_poll = nullptr;          // pinned: queue head, running count, flags
  SysDesc* h_desc = nullptr;      // host staging, kNoAllocMaxSys records each
  Ctrl* h_ctrl = nullptr;
  int* h_order = nullptr;
};

// Work buffers of one call, 256-byte aligned, in the scratch array.
struct Carve {
  int nsys = 0, ntot = 0, kb = 0;
  SysDesc* desc = nullptr;
  Ctrl* ctrl = nullptr;
  int* order = nullptr;
  int* queue = nullptr;
  double* stage = nullptr;
  double4 *pos = nullptr, *vel = nullptr, *frc = nullptr, *xref = nullptr;
  unsigned short *nn = nullptr, *nbr = nullptr;
  PairSlot* pslots = nullptr;  // no pairs here: every block works alone
  double* xfp = nullptr;
  size_t bytes = 0;
};

Carve carve(unsigned char* base, int nsys, int ntot, int kb) {
  Carve c;
  c.nsys = nsys;
  c.ntot = ntot;
  c.kb = kb;
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    const size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return base + o;
  };
  c.desc = static_cast<SysDesc*>(take(sizeof(SysDesc) * nsys));
  c.ctrl = static_cast<Ctrl*>(take(sizeof(Ctrl) * nsys));
  c.order = static_cast<int*>(take(sizeof(int) * nsys));
  c.queue = static_cast<int*>(take(sizeof(int) * 8));
  c.stage = static_cast<double*>(take(sizeof(double) * 3 * (size_t)ntot));
  c.pos = static_cast<double4*>(take(sizeof(double4) * (size_t)ntot));
  c.vel = static_cast<double4*>(take(sizeof(double4) * (size_t)ntot));
  c.frc = static_cast<double4*>(take(sizeof(double4) * (size_t)ntot));
  c.xref = static_cast<double4*>(take(sizeof(double4) * (size_t)ntot));
  c.nn = static_cast<unsigned short*>(take(sizeof(unsigned short) * (size_t)ntot));
  c.nbr = static_cast<unsigned short*>(take(sizeof(unsigned short) * (size_t)ntot * kb));
  c.bytes = off;
  return c;
}

}  // namespace

extern "C" int fire_noalloc_init(int device, void** slot) {
  NoAlloc* na = new NoAlloc();
  void* base = nullptr;
  int rc = scratch_address(device, &base);
  if (!rc && hipHostMalloc((void**)&na->h_poll, 8 * sizeof(int), hipHostMallocDefault) != hipSuccess)
    rc = FIRE_E_OOM;
  if (rc) {
    delete na;
    return rc;
  }
  na->device = device;
  na->base = static_cast<unsigned char*>(base);
  na->h_desc = new SysDesc[kNoAllocMaxSys];
  na->h_ctrl = new Ctrl[kNoAllocMaxSys];
  na->h_order = new int[kNoAllocMaxSys];
  *slot = na;
  return FIRE_OK;
}

extern "C" void fire_noalloc_release(void* p) {
  NoAlloc* na = static_cast<NoAlloc*>(p);
  if (!na) return;
  if (na->h_poll) (void)hipHostFree(na->h_poll);
  delete[] na->h_desc;
  delete[] na->h_ctrl;
  delete[] na->h_order;
  delete na;
}

extern "C" int fire_batched_run_noalloc(fire_ctx* ctx, void* slot, int nsys, const long long* offsets,
                                        double* d_pos, const fire_box* boxes, const fire_potential* pot,
                                        const fire_params* per_sys, double tol, long long max_steps,
                                        fire_result* out, hipStream_t s) {
  NoAlloc* na = static_cast<NoAlloc*>(slot);
  if (!na) return fire_ctx_error(ctx, FIRE_E_DEVICE, "batched (no alloc): the context has no scratch set-up");
  if (nsys < 1 || !offsets || !d_pos || !boxes || !pot || !out)
    return fire_ctx_error(ctx, FIRE_E_ARG, "batched: nsys >= 1 and non-NULL arrays are required");
  if (nsys > kNoAllocMaxSys)
    return fire_ctx_error(ctx, FIRE_E_ARG, "batched (no alloc): at most 1024 systems per call");
  int dev = -1;
  BCHK(hipGetDevice(&dev));
  if (dev != na->device)
    return fire_ctx_error(ctx, FIRE_E_DEVICE, "batched (no alloc): the context's device must be current");
  BatchPlan plan;
  int rc = prepare_batch(ctx, nsys, offsets, boxes, pot, per_sys, tol, max_steps, na->h_desc, na->h_ctrl,
                         na->h_order, &plan);
  if (rc) return rc;
  const PotDev& P = plan.P;
  bool found = false;
  const Config cfg = config_for(static_cast<Workspace*>(*fire_ctx_batched_slot(ctx)), plan,
                                na->h_ctrl[0].precision, &found);
  int ncu = 256;
  BCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  // no pairs here, so the launch order is the queue order
  const Launch lau = plan_launch(na->h_desc, na->h_order, nsys, ncu, cfg.team, false, na->h_order);
  int kb = plan.kb;
  for (int attempt = 0; attempt < 4; ++attempt) {
    if (carve(nullptr, nsys, plan.ntot, kb).bytes > kScratchBytes)
      return fire_ctx_error(ctx, FIRE_E_ARG,
                            "batched (no alloc): the batch and its neighbour lists exceed the 64 MiB scratch "
                            "(about 160,000 atoms of the EAM-form crystals)");
    const Carve w = carve(na->base, nsys, plan.ntot, kb);
    // every buffer the kernels read is written here first: the array keeps
    // the contents of the previous call on this device
    BCHK(hipMemcpyAsync(w.desc, na->h_desc, sizeof(SysDesc) * nsys, hipMemcpyHostToDevice, s));
    BCHK(hipMemcpyAsync(w.order, na->h_order, sizeof(int) * nsys, hipMemcpyHostToDevice, s));
    BCHK(hipMemcpyAsync(w.ctrl, na->h_ctrl, sizeof(Ctrl) * nsys, hipMemcpyHostToDevice, s));
    BCHK(hipMemcpyAsync(w.stage, d_pos, sizeof(double) * 3 * plan.ntot, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, s, w.queue, 8);
    hipLaunchKernelGGL(k_stage, dim3((plan.ntot + 255) / 256), dim3(256), 0, s, w.stage, plan.ntot, w.pos, w.vel,
                       w.frc, w.xref);
    const long long max_rounds = max_steps / cfg.chunk + 4;
    bool need_more = false;
    for (long long r = 0; r <= max_rounds; ++r) {
      launch_chunk(&w, P, cfg, lau, s);
      BCHK(hipMemcpyAsync(na->h_poll, w.queue, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
      BCHK(hipStreamSynchronize(s));
      if (na->h_poll[2]) {  // a list outgrew its capacity
        need_more = true;
        break;
      }
      if (na->h_poll[1] == 0) break;
    }
    if (need_more) {
      kb = ((kb * 3 / 2 + 16) + 3) & ~3;
      continue;
    }
    BCHK(hipMemcpyAsync(na->h_ctrl, w.ctrl, sizeof(Ctrl) * nsys, hipMemcpyDeviceToHost, s));
    hipLaunchKernelGGL(k_unstage, dim3(nsys), dim3(256), 0, s, w.pos, w.desc, d_pos);
    BCHK(hipStreamSynchronize(s));
    fill_results(na->h_ctrl, na->h_desc, nsys, out);
    return FIRE_OK;
  }
  return fire_ctx_error(ctx, FIRE_E_ARG, "batched (no alloc): neighbour lists keep outgrowing their capacity");
}
