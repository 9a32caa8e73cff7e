// fire2.hip -- single-system FIRE 2.0 hot path for MI355X (gfx950) and the C ABI.
//
// Per iteration (one force evaluation, the paper's unit of cost):
//   k_update   FIRE 2.0 velocity/position step (Algorithm 2 branch outcome,
//              half-step-back, semi-implicit Euler kick + mixing + drift of
//              Algorithm 4; Algorithms 3/6 as options)
//   k_*_density / k_*_force
//              pair terms over a cell-sorted full neighbour list; the force
//              epilogue reduces E, P = F.v, |F|^2, |v|^2, max |F_i|^2,
//              max |v_i|^2 per block (wave64 shuffles -> LDS)
//   (last block of the force pass) fixed-order second reduction stage and
//              the scalar FIRE 2.0 logic (counters, dt/alpha, stop tests,
//              mixing coefficients)
// K iterations are captured in a hipGraph and replayed; every kernel exits at
// once when the control record says the run is stopped or paused, and the
// host only polls a 32-byte status word between replays.
//
// Layout in HBM, sorted by cell: pos double4 (x, y, z, w = F'(rho) for the
// EAM form), v and F as three FP64 planes, atom_id (sorted slot -> caller
// index), neighbour list int32 column-major [k][slot].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <type_traits>
#include <vector>

#include "fire2.h"
#include "fire2_internal.h"
#include "fire2_device.h"

namespace fire {

// ------------------------------------------------------------------ helpers

// Block-level reduction of NS sums followed by NM maxima; result valid in
// the first wave (thread 0 among them).  Each wave reduces by lane moves,
// then the first wave reduces the per-wave results the same way.  The order
// is fixed by the thread layout, so results are reproducible run to run.
// MAXB: the largest block size of the caller (its LDS scratch is sized for
// it; kernels at the LDS limit keep the default).
template <int NS, int NM, int MAXB = kBlock>
__device__ __forceinline__ void block_reduce(double (&v)[NS + NM]) {
  __shared__ double red[NS + NM][MAXB / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < NS; ++k) v[k] = wave_sum(v[k]);
#pragma unroll
  for (int k = NS; k < NS + NM; ++k) v[k] = wave_max(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NS + NM; ++k) red[k][w] = v[k];
  }
  __syncthreads();
  if (w == 0) {
    const bool has = lane < nw;
#pragma unroll
    for (int k = 0; k < NS; ++k) v[k] = wave_sum(has ? red[k][lane % (MAXB / 64)] : 0.0);
#pragma unroll
    for (int k = NS; k < NS + NM; ++k) v[k] = wave_max(has ? red[k][lane % (MAXB / 64)] : -INFINITY);
  }
}

// Blocks are dealt round-robin to the 8 XCDs; remap so that each XCD works
// on one contiguous run of (spatially sorted) atoms and its L2 holds their
// neighbours.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int x = b & 7, idx = b >> 3, per = nb >> 3, rem = nb & 7;
  return x * per + min(x, rem) + idx;
}

__device__ __forceinline__ bool ctrl_running(const Ctrl* c) {
  return __builtin_nontemporal_load(&c->status) == ST_RUNNING;
}

// ----------------------------------------------------------- stage in/out

// Caller AoS positions -> slot order (identity), zero v and F.
__global__ void k_stage_in(const double* __restrict__ src, int n, int ncap, double4* __restrict__ pos,
                           double* __restrict__ vel, double* __restrict__ frc, int* __restrict__ id,
                           int* __restrict__ flags) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double x = src[3 * i], y = src[3 * i + 1], z = src[3 * i + 2];
  if (!isfinite(x) || !isfinite(y) || !isfinite(z)) atomicOr(flags, ERR_NONFINITE);
  pos[i] = make_double4(x, y, z, 0.0);
  vel[i] = vel[ncap + i] = vel[2 * ncap + i] = 0.0;
  frc[i] = frc[ncap + i] = frc[2 * ncap + i] = 0.0;
  id[i] = i;
}

// Caller-order masses and freeze bits (either may be NULL) -> 1/m and 3-bit
// masks in caller order; a mass that is not positive and finite sets
// kBadMass in flags[0].
constexpr int kBadMass = 16;
__global__ void k_props_in(const double* __restrict__ mass, const unsigned char* __restrict__ frozen, int n,
                           double* __restrict__ minv, unsigned char* __restrict__ fm, int* __restrict__ flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (mass) {
    const double m = mass[i];
    if (!(m > 0.0) || !isfinite(m)) atomicOr(flags, kBadMass);
    minv[i] = 1.0 / m;
  }
  if (frozen) fm[i] = frozen[i] & 7;
}

// The properties in slot order: real slot s holds caller atom id[s].
__global__ void k_props_gather(int n, const int* __restrict__ id, const double* __restrict__ minv,
                               const unsigned char* __restrict__ fm, double* __restrict__ sinv,
                               unsigned char* __restrict__ fmask) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int a = id[s];
  if (minv) sinv[s] = minv[a];
  if (fm) fmask[s] = fm[a];
}

__global__ void k_set_pos(double4* __restrict__ pos, int slot, double v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) pos[slot] = make_double4(v, v, v, 0.0);
}

// Sorted-order vector (3 planes) from a caller-order AoS vector.
__global__ void k_gather_vec(const double* __restrict__ src, int n, int ncap, const int* __restrict__ id,
                             double* __restrict__ dst) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  int a = id[s];
  dst[s] = src[3 * a];
  dst[ncap + s] = src[3 * a + 1];
  dst[2 * ncap + s] = src[3 * a + 2];
}

__global__ void k_scatter_vec(const double* __restrict__ src, int n, int ncap, const int* __restrict__ id,
                              double* __restrict__ dst) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  int a = id[s];
  dst[3 * a] = src[s];
  dst[3 * a + 1] = src[ncap + s];
  dst[3 * a + 2] = src[2 * ncap + s];
}

__global__ void k_stage_out_pos(const double4* __restrict__ pos, int n, const int* __restrict__ id, BoxDev box,
                                double* __restrict__ dst) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  double4 p = pos[s];
  double r[3] = {p.x, p.y, p.z};
#pragma unroll
  for (int d = 0; d < 3; ++d)
    if (box.per[d]) {
      double t = r[d] - box.lo[d];
      t -= box.L[d] * floor(t * box.invL[d]);
      if (t >= box.L[d]) t -= box.L[d];
      if (t < 0.0) t = 0.0;
      r[d] = box.lo[d] + t;
    }
  int a = id[s];
  dst[3 * a] = r[0];
  dst[3 * a + 1] = r[1];
  dst[3 * a + 2] = r[2];
}

// ------------------------------------------------------- cell-list build
//
// Periodic images are explicit: at every list build each atom within rcs of a
// periodic face gets ghost copies (shifted by the box length) in an extra
// layer of cells outside the box, so pair loops never take a minimum image.
// All atoms (real and ghost) are counting-sorted by cell; cells inside the box
// are numbered first (along a Hilbert curve), so real atoms occupy slots [0, n) and
// ghosts follow.  The update and density kernels refresh each atom's ghosts.

struct Grid {
  int n[3];              // cells per axis, including one ghost layer on each side of periodic axes
  int ncell;
  double lo[3], inv[3];  // origin of the (extended) grid and 1 / cell edge
  int in_lo[3], in_hi[3];  // cell coordinates inside the box (real atoms)
};

// Shift of a ghost: two bits per axis (1: +L, 2: -L).
__device__ __forceinline__ double ghost_shift(int code, int d, const BoxDev& b) {
  const int c = (code >> (2 * d)) & 3;
  return c == 1 ? b.L[d] : (c == 2 ? -b.L[d] : 0.0);
}

// Bounding box partials (min x,y,z then max x,y,z) per block.
__global__ void k_bbox(const double4* __restrict__ pos, int n, double* __restrict__ part) {
  __shared__ double sm[6][kBlock];
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  double v[6];
  if (i < n) {
    double4 p = pos[i];
    v[0] = v[3] = p.x;
    v[1] = v[4] = p.y;
    v[2] = v[5] = p.z;
  } else {
    v[0] = v[1] = v[2] = INFINITY;
    v[3] = v[4] = v[5] = -INFINITY;
  }
  for (int k = 0; k < 6; ++k) sm[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      for (int k = 0; k < 3; ++k) sm[k][threadIdx.x] = fmin(sm[k][threadIdx.x], sm[k][threadIdx.x + s]);
      for (int k = 3; k < 6; ++k) sm[k][threadIdx.x] = fmax(sm[k][threadIdx.x], sm[k][threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 6; ++k) part[6 * blockIdx.x + k] = sm[k][0];
}

__device__ __forceinline__ int cell_coord(double x, const Grid& g, int d) {
  int c = (int)floor((x - g.lo[d]) * g.inv[d]);
  return min(max(c, 0), g.n[d] - 1);
}

// Cell of a real atom: always inside the box (rounding at a face cannot push
// it into a ghost layer).
__device__ __forceinline__ int real_cell_coord(double x, const Grid& g, int d) {
  int c = (int)floor((x - g.lo[d]) * g.inv[d]);
  return min(max(c, g.in_lo[d]), g.in_hi[d]);
}

// Cell of a ghost: in the ghost layer on every shifted axis, inside the box
// on the others.
__device__ __forceinline__ int ghost_cell_coord(double x, int code, const Grid& g, int d) {
  const int c = (code >> (2 * d)) & 3;
  if (c == 1) return g.n[d] - 1;
  if (c == 2) return 0;
  return real_cell_coord(x, g, d);
}

// Wrap the real atoms into the box on periodic axes and count their ghosts:
// an atom within rcs of the low face has an image at +L, within rcs of the
// high face one at -L; every non-empty combination over axes is one ghost.
__global__ void k_ghost_count(double4* __restrict__ pos, int n, BoxDev box, double rcs, int* __restrict__ gcount) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double4 p = pos[i];
  double r[3] = {p.x, p.y, p.z};
  int choices = 1;
#pragma unroll
  for (int d = 0; d < 3; ++d)
    if (box.per[d]) {
      double t = r[d] - box.lo[d];
      t -= box.L[d] * floor(t * box.invL[d]);
      if (t >= box.L[d]) t -= box.L[d];
      if (t < 0.0) t = 0.0;
      r[d] = box.lo[d] + t;
      if (t < rcs || t >= box.L[d] - rcs) choices *= 2;
    }
  pos[i] = make_double4(r[0], r[1], r[2], p.w);
  gcount[i] = choices - 1;
}

// Ghost positions (slots n + goff[i] ...) with their source slot and shift
// code; ghosts numbered gmax or above (beyond the slot capacity) are not
// written: the host, which learns the count at the end of the build, then
// grows the capacity and builds again.
__global__ void k_ghost_fill(double4* __restrict__ pos, int n, BoxDev box, double rcs, const int* __restrict__ goff,
                             int* __restrict__ gsrc, int* __restrict__ gcode, int gmax) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double4 p = pos[i];
  const double r[3] = {p.x, p.y, p.z};
  int opt[3] = {0, 0, 0};  // shift code per axis, 0 if none
#pragma unroll
  for (int d = 0; d < 3; ++d)
    if (box.per[d]) {
      const double t = r[d] - box.lo[d];
      if (t < rcs) opt[d] = 1;
      else if (t >= box.L[d] - rcs) opt[d] = 2;
    }
  int k = 0;
  for (int m = 1; m < 8; ++m) {
    if (((m & 1) && !opt[0]) || ((m & 2) && !opt[1]) || ((m & 4) && !opt[2])) continue;
    const int code = ((m & 1) ? opt[0] : 0) | (((m & 2) ? opt[1] : 0) << 2) | (((m & 4) ? opt[2] : 0) << 4);
    const int g = goff[i] + k++;
    if (g >= gmax) continue;
    pos[n + g] = make_double4(r[0] + ghost_shift(code, 0, box), r[1] + ghost_shift(code, 1, box),
                              r[2] + ghost_shift(code, 2, box), p.w);
    gsrc[g] = i;
    gcode[g] = code;
  }
}

// Slots of the current build: the real atoms and the ghosts counted on the
// device (goff[n]), at most gmax of them.  The kernels of a rebuild read the
// count here, so the host need not wait for it before launching them.
__device__ __forceinline__ int slot_count(int n, const int* __restrict__ gtot, int gmax) {
  return n + min(*gtot, gmax);
}

// counter[c] += 1 for every active lane, with one atomic per distinct c in
// the wave (slots follow the cells of the last build, so a wave's lanes share
// few cells); returns each lane's place among the additions to its counter,
// as atomicAdd would (in lane order within the wave).
__device__ __forceinline__ int wave_add_one(int* __restrict__ counter, int c) {
  const int lane = threadIdx.x & 63;
  for (;;) {
    const int cl = __builtin_amdgcn_readfirstlane(c);
    const unsigned long long peers = __builtin_amdgcn_ballot_w64(c == cl);
    if (c == cl) {
      const int leader = __builtin_ffsll((long long)peers) - 1;
      int base = 0;
      if (lane == leader) base = atomicAdd(&counter[cl], __popcll(peers));
      base = __shfl(base, leader, 64);
      return base + __popcll(peers & ((1ull << lane) - 1));
    }
  }
}

// Cell of every slot (real and ghost) and per-cell counts.  Ordering key
// inside a cell: caller index times 64, plus the ghost's shift code.
__global__ void k_cell_count(const double4* __restrict__ pos, int n, const int* __restrict__ gtot, int gmax, Grid g,
                             const int* __restrict__ cell_rank, const int* __restrict__ id,
                             const int* __restrict__ gsrc, const int* __restrict__ gcode,
                             int* __restrict__ cell_of, long long* __restrict__ key, int* __restrict__ count) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= slot_count(n, gtot, gmax)) return;
  const double4 p = pos[i];
  int cc[3];
  if (i < n) {
    cc[0] = real_cell_coord(p.x, g, 0);
    cc[1] = real_cell_coord(p.y, g, 1);
    cc[2] = real_cell_coord(p.z, g, 2);
  } else {
    const int code = gcode[i - n];
    cc[0] = ghost_cell_coord(p.x, code, g, 0);
    cc[1] = ghost_cell_coord(p.y, code, g, 1);
    cc[2] = ghost_cell_coord(p.z, code, g, 2);
  }
  const int c = cell_rank[cc[0] + g.n[0] * (cc[1] + g.n[1] * cc[2])];
  cell_of[i] = c;
  // unique per slot: a ghost's shift code (1..63) follows its source's index
  key[i] = i < n ? 64LL * id[i] : 64LL * id[gsrc[i - n]] + gcode[i - n];
  wave_add_one(count, c);
}

// Exclusive prefix sum start[0..m] of count[0..m) (start[m] = total) in three
// launches: per-chunk totals, a scan of the totals, and per-chunk scans with
// the chunk's offset.  A chunk is 4096 counts: 1024 threads x 4 consecutive.
constexpr int kScanThreads = 1024;
constexpr int kScanChunk = 4 * kScanThreads;

// Inclusive scan over the block (blockDim.x = kScanThreads); *total = sum.
__device__ __forceinline__ int block_scan_incl(int v, int* total) {
  __shared__ int wsum[kScanThreads / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(v, o, 64);
    if (lane >= o) v += y;
  }
  if (lane == 63) wsum[w] = v;
  __syncthreads();
  int off = 0, tot = 0;
  for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
    off += q < w ? wsum[q] : 0;
    tot += wsum[q];
  }
  __syncthreads();
  *total = tot;
  return off + v;
}

__device__ __forceinline__ int4 load_counts(const int* __restrict__ count, int m, int i) {
  if (i + 3 < m) return *reinterpret_cast<const int4*>(count + i);
  return make_int4(i < m ? count[i] : 0, i + 1 < m ? count[i + 1] : 0, i + 2 < m ? count[i + 2] : 0,
                   i + 3 < m ? count[i + 3] : 0);
}

__global__ __launch_bounds__(kScanThreads) void k_scan_part(const int* __restrict__ count, int m,
                                                            int* __restrict__ part) {
  const int i = blockIdx.x * kScanChunk + 4 * threadIdx.x;
  const int4 c = load_counts(count, m, i);
  int tot;
  block_scan_incl(c.x + c.y + c.z + c.w, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// One block: exclusive scan of part[0..np) in place, part[np] = total, and
// start[m] = total.
__global__ __launch_bounds__(kScanThreads) void k_scan_top(int* __restrict__ part, int np, int* __restrict__ start,
                                                           int m) {
  int carry = 0;
  for (int base = 0; base < np; base += kScanThreads) {
    const int q = base + threadIdx.x;
    const int v = q < np ? part[q] : 0;
    int tot;
    const int inc = block_scan_incl(v, &tot);
    if (q < np) part[q] = carry + inc - v;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    part[np] = carry;
    start[m] = carry;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const int* __restrict__ count, int m,
                                                             const int* __restrict__ part,
                                                             int* __restrict__ start) {
  const int i = blockIdx.x * kScanChunk + 4 * threadIdx.x;
  const int4 c = load_counts(count, m, i);
  const int t = c.x + c.y + c.z + c.w;
  int tot;
  const int e = part[blockIdx.x] + block_scan_incl(t, &tot) - t;
  if (i < m) start[i] = e;
  if (i + 1 < m) start[i + 1] = e + c.x;
  if (i + 2 < m) start[i + 2] = e + c.x + c.y;
  if (i + 3 < m) start[i + 3] = e + c.x + c.y + c.z;
}

__global__ void k_cell_fill(const int* __restrict__ cell_of, int n, const int* __restrict__ gtot, int gmax,
                            const int* __restrict__ start, int* __restrict__ cursor, int* __restrict__ order) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= slot_count(n, gtot, gmax)) return;
  const int c = cell_of[i];
  order[start[c] + wave_add_one(cursor, c)] = i;  // any order: k_cell_rank sorts each cell
}

// Deterministic order inside each cell: by key.  One thread per slot ranks
// its atom among the cell's members.
__global__ void k_cell_rank(const int* __restrict__ cell_of, const int* __restrict__ start,
                            const int* __restrict__ bucket, int n, const int* __restrict__ gtot, int gmax,
                            const long long* __restrict__ key, int* __restrict__ order) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= slot_count(n, gtot, gmax)) return;
  const int a = bucket[s], c = cell_of[a];
  const long long k = key[a];
  const int b = start[c], e = start[c + 1];
  int rank = 0;
  for (int t = b; t < e; ++t) rank += key[bucket[t]] < k;
  order[b + rank] = a;
}

// Gather every slot into its sorted place.  Real atoms (old slots < n) land
// in new slots < n and carry v, F, id; ghosts carry their source and shift.
__global__ void k_permute(const int* __restrict__ order, int n, const int* __restrict__ gtot, int gmax, int ncap,
                          const double4* __restrict__ pos,
                          const double* __restrict__ vel, const double* __restrict__ frc,
                          const int* __restrict__ id, const int* __restrict__ cell_of,
                          const int* __restrict__ gsrc, const int* __restrict__ gcode,
                          double4* __restrict__ pos2, double* __restrict__ vel2, double* __restrict__ frc2,
                          int* __restrict__ id2, int* __restrict__ srank, int* __restrict__ new_of_old,
                          int* __restrict__ gsrc2, int* __restrict__ gcode2) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= slot_count(n, gtot, gmax)) return;
  const int o = order[s];
  pos2[s] = pos[o];
  srank[s] = cell_of[o];
  if (s < n) {
    id2[s] = id[o];
    new_of_old[o] = s;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      vel2[d * ncap + s] = vel[d * ncap + o];
      frc2[d * ncap + s] = frc[d * ncap + o];
    }
  } else {
    gsrc2[s - n] = gsrc[o - n];  // still an old real slot; mapped by k_ghost_link
    gcode2[s - n] = gcode[o - n];
  }
}

// Copy the sorted slots back into the arrays the captured graphs read (their
// addresses must not change), and record the build positions for the skin
// test: one launch over max(nt, n) slots instead of one copy per array.
__global__ void k_commit(int n, const int* __restrict__ gtot, int gmax, int ncap, const double4* __restrict__ pos2,
                         const int* __restrict__ gsrc2, const int* __restrict__ gcode2,
                         const int* __restrict__ id2, const double* __restrict__ vel2,
                         const double* __restrict__ frc2, double4* __restrict__ pos, int* __restrict__ gsrc,
                         int* __restrict__ gcode, int* __restrict__ id, double* __restrict__ vel,
                         double* __restrict__ frc, double4* __restrict__ xref) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int nt = slot_count(n, gtot, gmax), ng = nt - n;
  if (s < nt) pos[s] = pos2[s];
  if (s < ng) {
    gsrc[s] = gsrc2[s];
    gcode[s] = gcode2[s];
  }
  if (s < n) {
    xref[s] = pos2[s];
    id[s] = id2[s];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      vel[d * ncap + s] = vel2[d * ncap + s];
      frc[d * ncap + s] = frc2[d * ncap + s];
    }
  }
}

// Link ghosts to the new slots of their sources: real_of[] (slot -> real
// slot, identity for real atoms) and the per-atom ghost lists (at most 7).
__global__ void k_ghost_link(int n, const int* __restrict__ gtot, int gmax, const int* __restrict__ new_of_old,
                             int* __restrict__ gsrc, int* __restrict__ real_of, int* __restrict__ gcnt,
                             int* __restrict__ glist) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n) real_of[s] = s;
  if (s >= slot_count(n, gtot, gmax) - n) return;
  const int src = new_of_old[gsrc[s]];
  gsrc[s] = src;
  real_of[n + s] = src;
  const int k = atomicAdd(&gcnt[src], 1);
  glist[8 * src + k] = n + s;
}

__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// Dynamic LDS of the kernels that size it at launch.
extern __shared__ __align__(16) unsigned char dyn_lds[];

// Neighbour k of lane `lane` of wave w: groups of four consecutive neighbours
// of one atom are adjacent, so a lane fetches a group with one vector load and
// a wave's group loads are contiguous.
__device__ __forceinline__ size_t lidx(int w, int k, int lane, int kcap) {
  return (((size_t)w * (kcap >> 2) + (k >> 2)) * 64 + lane) * 4 + (k & 3);
}

// FP32 copy of the slot positions relative to the grid origin, for the
// neighbour search's distance tests.
__global__ __launch_bounds__(kBlock) void k_pos_f32(const double4* __restrict__ pos, int n,
                                                    const int* __restrict__ gtot, int gmax, Grid g,
                                                    float4* __restrict__ posf) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < slot_count(n, gtot, gmax)) {
    const double4 p = pos[j];
    posf[j] = make_float4((float)(p.x - g.lo[0]), (float)(p.y - g.lo[1]), (float)(p.z - g.lo[2]), 0.0f);
  }
}

// Full neighbour list of every real atom: all slots (real or ghost) within
// rcs, in ascending slot order, stored per wave of 64 atoms at
// lidx(w, k, lane).  Each wave's lists are padded to a common length (a
// multiple of 4, kept in wcnt[w]) with a dummy slot far outside the system,
// so the force loops run a wave-uniform trip count and the padding fails
// every cutoff test.  The grid covers every wave of the allocation.
// The distance tests run in FP32 on posf against rcs2f, the square of rcs
// widened by the FP32 rounding bound of the coordinates (set by the host):
// every slot within rcs is in the list, and a few just beyond it may be,
// which the passes treat like any entry beyond the cutoff (zero terms).
// Half the bytes per candidate of FP64 positions, and half the loads.
// flags[0] |= overlap (positions equal in FP64), flags[1] = max count.
__global__ __launch_bounds__(kBlock) void k_nbr_build(const double4* __restrict__ pos,
                                                      const float4* __restrict__ posf, int n, Grid g,
                                                      const int* __restrict__ cell_rank,
                                                      const int* __restrict__ start, float rcs2f, float split2f,
                                                      float cut2f, int kcap, int dummy, int* __restrict__ nbr,
                                                      int* __restrict__ wcnt, int* __restrict__ flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int w = i >> 6, lane = threadIdx.x & 63;
  // Three classes of entries by their distance at build time: near
  // (r^2 < split2f), middle (split2f <= r^2 < cut2f) and far.  Near entries
  // fill the list from the front, the others from the back (middle ones
  // stored as -(j + 1)); each class stays in slot order.
  int cn = 0, cb = 0;
  bool overlap = false;
  if (i < n) {
    const double4 pi = pos[i];
    const float4 pf = posf[i];
    const int c[3] = {real_cell_coord(pi.x, g, 0), real_cell_coord(pi.y, g, 1), real_cell_coord(pi.z, g, 2)};
    // stencil cells in ascending rank, so each list comes out sorted by slot:
    // lanes of a wave then read nearby (or identical) neighbours at each step.
    // Sorted by a bitonic network over 32 entries (cells outside the grid
    // and the padding hold INT_MAX and sort last): every register index is
    // static.  An insertion sort indexes the array by a per-lane position,
    // which compiles to a compare-and-select over all entries per access and
    // cost several times the candidate tests themselves.
    int cells[32];
    int nc = 0;
#pragma unroll
    for (int o = 0; o < 32; ++o) {
      int r = INT_MAX;
      if (o < 27) {
        const int cx = c[0] + o % 3 - 1, cy = c[1] + (o / 3) % 3 - 1, cz = c[2] + o / 9 - 1;
        if (cx >= 0 && cx < g.n[0] && cy >= 0 && cy < g.n[1] && cz >= 0 && cz < g.n[2]) {
          r = cell_rank[cx + g.n[0] * (cy + g.n[1] * cz)];
          ++nc;
        }
      }
      cells[o] = r;
    }
#pragma unroll
    for (int k = 2; k <= 32; k <<= 1)
#pragma unroll
      for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
        for (int a = 0; a < 32; ++a) {
          const int b = a ^ j;
          if (b > a) {
            const int lo = min(cells[a], cells[b]), hi = max(cells[a], cells[b]);
            const bool up = (a & k) == 0;
            cells[a] = up ? lo : hi;
            cells[b] = up ? hi : lo;
          }
        }
    // this lane's list: entry k at lb[(k / 4) * 256 + k % 4] (lidx)
    int* const lb = nbr + (size_t)w * (kcap >> 2) * 256 + lane * 4;
    for (int q = 0; q < nc; ++q) {
      const int cell = cells[q];
      // candidates in groups of 8: all loads issued before the tests, so
      // their latencies overlap; entries are appended in slot order
      constexpr int kG = 8;
      for (int j0 = start[cell], e = start[cell + 1]; j0 < e; j0 += kG) {
        float4 pj[kG];
#pragma unroll
        for (int u = 0; u < kG; ++u) pj[u] = posf[min(j0 + u, e - 1)];
        // the tests as masks rather than branches (the exec-mask bookkeeping
        // of nested divergent branches had cost more than the tests)
#pragma unroll
        for (int u = 0; u < kG; ++u) {
          const int j = j0 + u;
          const float dx = pf.x - pj[u].x, dy = pf.y - pj[u].y, dz = pf.z - pj[u].z;
          const float r2 = dx * dx + dy * dy + dz * dz;
          const bool cand = j < e && j != i;
          if (cand && r2 == 0.0f) {  // equal in FP32: compare the FP64 positions
            const double4 q = pos[j];
            if (q.x == pi.x && q.y == pi.y && q.z == pi.z) overlap = true;
          }
          const bool acc = cand && r2 < rcs2f;
          const bool near = r2 < split2f, mid = !near && r2 < cut2f;
          const int k = near ? cn : kcap - 1 - cb;
          if (acc && cn + cb < kcap) lb[((k >> 2) << 8) + (k & 3)] = mid ? -(j + 1) : j;
          cn += acc && near;
          cb += acc && !near;
        }
      }
    }
  }
  // Final layout of each list: near, middle, then far entries, then padding
  // to the wave's longest list (a multiple of four).  Groups of four past
  // every lane's near + middle count hold far entries or padding only, so a
  // pass can skip such a group with one wave-uniform test when no lane of it
  // is within the cutoff.  The moves from the back must not overwrite an
  // entry not yet moved: that needs cn + 2 cb <= kcap, which the reported
  // size includes (a larger capacity and another build otherwise).
  const int m = wave_max_i(cn + 2 * cb);
  int kw = 0;
  if (m <= kcap) {
    int q = cn;
    for (int pass = 0; pass < 2; ++pass)  // middle entries, then far ones
      for (int f = 0; f < cb; ++f) {
        const int v = nbr[lidx(w, kcap - 1 - f, lane, kcap)];
        if ((v < 0) == (pass == 0)) nbr[lidx(w, q++, lane, kcap)] = v < 0 ? -v - 1 : v;
      }
    kw = (wave_max_i(q) + 3) & ~3;
    for (int k = q; k < kw; ++k) nbr[lidx(w, k, lane, kcap)] = dummy;
  }
  if (lane == 0) {
    wcnt[w] = kw;
    atomicMax(&flags[1], m);
  }
  if (overlap) atomicOr(&flags[0], ERR_OVERLAP);
}

// Candidates of tile b (the TILE slots of block b): the stencil cells of the
// tile's cells, sorted by rank and made unique, with the offsets of their atom
// runs (hoff, hoff[nu] = number of candidate atoms).  Returns nu, or -1 if
// the tile has more than kCandMax / 27 distinct cells.
constexpr int kCandMax = 4096;
template <int TILE>
__device__ int tile_candidates(const int* __restrict__ srank, const int* __restrict__ start,
                               const int* __restrict__ rank_cell, const int* __restrict__ cell_rank, int n,
                               const Grid& g, int* cand, int* hoff, int* dcell, int* s_shared) {
  const int b = blockIdx.x, t = threadIdx.x;
  const int s0 = b * TILE, s1 = min(s0 + TILE, n);
  int tot;
  {
    const int sl = s0 + t;
    const int f = (sl < s1 && (t == 0 || srank[sl] != srank[sl - 1])) ? 1 : 0;
    const int p = block_scan_incl(f, &tot) - f;
    if (f) dcell[p] = srank[sl];
  }
  __syncthreads();
  const int nd = tot;
  if (nd * 27 > kCandMax) return -1;
  const int ncand = nd * 27;
  int P = 1;
  while (P < ncand) P <<= 1;
  for (int q = t; q < P; q += blockDim.x) {
    int v = INT_MAX;
    if (q < ncand) {
      const int lin = rank_cell[dcell[q / 27]], o = q % 27;
      const int c3[3] = {lin % g.n[0] + o % 3 - 1, (lin / g.n[0]) % g.n[1] + (o / 3) % 3 - 1,
                         lin / (g.n[0] * g.n[1]) + o / 9 - 1};
      bool ok = true;
      for (int d = 0; d < 3; ++d)
        if (c3[d] < 0 || c3[d] >= g.n[d]) ok = false;
      if (ok) v = cell_rank[c3[0] + g.n[0] * (c3[1] + g.n[1] * c3[2])];
    }
    cand[q] = v;
  }
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1)  // bitonic sort of cand[0..P)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int q = t; q < P; q += blockDim.x) {
        const int p = q ^ j;
        if (p > q) {
          const int a = cand[q], c = cand[p];
          const bool up = (q & k) == 0;
          if ((a > c) == up) {
            cand[q] = c;
            cand[p] = a;
          }
        }
      }
      __syncthreads();
    }
  // unique cells and their run offsets; thread t owns kPer consecutive entries
  constexpr int kPer = kCandMax / TILE;
  int r[kPer], nu_t = 0, len_t = 0;
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int q = kPer * t + u;
    r[u] = (q < P && cand[q] != INT_MAX && (q == 0 || cand[q] != cand[q - 1])) ? cand[q] : -1;
    if (r[u] >= 0) {
      ++nu_t;
      len_t += start[r[u] + 1] - start[r[u]];
    }
  }
  int tu, tl;
  int pu = block_scan_incl(nu_t, &tu) - nu_t;
  int pl = block_scan_incl(len_t, &tl) - len_t;
  __syncthreads();  // all of cand[] read before it is compacted
#pragma unroll
  for (int u = 0; u < kPer; ++u)
    if (r[u] >= 0) {
      cand[pu] = r[u];
      hoff[pu] = pl;
      ++pu;
      pl += start[r[u] + 1] - start[r[u]];
    }
  if (t == 0) {
    hoff[tu] = tl;
    *s_shared = tu;
  }
  __syncthreads();
  return *s_shared;
}

// Per-tile halo for the LDS-staged passes.  Tile b is the TILE slots of block
// b (one thread per slot).  Its halo is the set of atoms that occur in the tile's neighbour lists:
// every list entry marks its candidate (tile_candidates) in a bitmap, and the
// marked candidates, in candidate order, are the halo.  The kernel writes the
// halo's slot list (hslot, at most hcap entries), its size (tile_h), and
// rewrites the tile's lists as 16-bit halo indices (nbr16; padding -> index H,
// an LDS slot set to a far position).  A halo that does not fit sets
// flags[3] bit 4; flags[2] = max H.
constexpr int kHaloCandMax = 16384;   // candidate atoms of one tile (bitmap bits)
template <int TILE>
__global__ __launch_bounds__(TILE) void k_tile_halo(const int* __restrict__ srank, const int* __restrict__ start,
                                                      const int* __restrict__ rank_cell,
                                                      const int* __restrict__ cell_rank, int n, Grid g,
                                                      const int* __restrict__ nbr, const int* __restrict__ wcnt,
                                                      int kcap, int hcap, int dummy, int* __restrict__ tile_h,
                                                      int* __restrict__ hslot, int* __restrict__ hsrc,
                                                      const int* __restrict__ real_of,
                                                      unsigned short* __restrict__ nbr16, int* __restrict__ flags) {
  __shared__ int cand[kCandMax];
  __shared__ int hoff[kCandMax + 1];
  __shared__ int dcell[TILE];
  __shared__ unsigned int used[kHaloCandMax / 32];
  __shared__ int wpre[kHaloCandMax / 32];
  __shared__ int s_nu;
  const int b = blockIdx.x, t = threadIdx.x;
  const int nu = tile_candidates<TILE>(srank, start, rank_cell, cell_rank, n, g, cand, hoff, dcell, &s_nu);
  int* cslot = cand;  // below, cand[h] is replaced by the first slot of run h (runs ascend in slot order)
  if (nu < 0 || hoff[nu] > kHaloCandMax) {
    if (t == 0) {
      tile_h[b] = -1;
      atomicOr(&flags[3], 4);
    }
    return;
  }
  const int Hc = hoff[nu];
  const int nwords = (Hc + 31) >> 5;
  for (int q = t; q < nwords; q += blockDim.x) used[q] = 0u;
  for (int h = t; h < nu; h += blockDim.x) cslot[h] = start[cand[h]];
  __syncthreads();
  // Searches by binary lifting: a trip count that is the same for every lane
  // (log2 of the block-uniform run count), so the four searches of a list
  // group interleave their LDS reads instead of waiting on each other.
  int top = 1;
  while (2 * top <= nu) top *= 2;
  // pass 1: candidate index of every list entry, marked in the bitmap and
  // kept in nbr16 until the halo numbering is known (padding: 0xFFFF).
  // Lists are read a group of four at a time (one 16-byte load per lane,
  // the next group in flight while this one is searched).
  const int i = b * TILE + t;
  const int w = i >> 6, lane = t & 63;
  const int kw = wcnt[w];  // a multiple of 4
  auto group = [&](int k) { return *reinterpret_cast<const int4*>(nbr + lidx(w, k, lane, kcap)); };
  int4 next = kw > 0 ? group(0) : make_int4(0, 0, 0, 0);
  for (int k = 0; k < kw; k += 4) {
    const int4 g4 = next;
    if (k + 4 < kw) next = group(k + 4);
    const int jv[4] = {g4.x, g4.y, g4.z, g4.w};
    // for each entry the last run h with cslot[h] <= j (h = 0 if none); the
    // four searches step together, so their LDS reads are in flight at once
    // (padding entries search too and are ignored)
    int hv[4] = {0, 0, 0, 0};
    for (int step = top; step > 0; step >>= 1)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int c = hv[u] + step;
        if (c < nu && cslot[min(c, nu - 1)] <= jv[u]) hv[u] = c;
      }
    int qv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = jv[u];
      int q = 0xFFFF;
      if (j != dummy) {
        const int h = hv[u];
        q = hoff[h] + (j - cslot[h]);
        if (j < cslot[h] || q >= hoff[h + 1]) {  // not among the candidates: cannot happen for valid lists
          atomicOr(&flags[3], 4);
          q = 0;
        }
        atomicOr(&used[q >> 5], 1u << (q & 31));
      }
      qv[u] = q;
    }
    *reinterpret_cast<ushort4*>(nbr16 + lidx(w, k, lane, kcap)) =
        make_ushort4((unsigned short)qv[0], (unsigned short)qv[1], (unsigned short)qv[2], (unsigned short)qv[3]);
  }
  __syncthreads();
  // halo index of the first marked candidate of each bitmap word
  int tot = 0;
  for (int base = 0; base < nwords; base += TILE) {
    const int q = base + t;
    const int pc = q < nwords ? __popc(used[q]) : 0;
    int part;
    const int ex = block_scan_incl(pc, &part) - pc;
    if (q < nwords) wpre[q] = tot + ex;
    tot += part;
  }
  __syncthreads();
  const int H = tot;
  if (H + 1 > hcap) {
    if (t == 0) {
      tile_h[b] = -1;
      atomicOr(&flags[3], 4);
      atomicMax(&flags[2], H);
    }
    return;
  }
  auto halo_index = [&](int q) { return wpre[q >> 5] + __popc(used[q >> 5] & ((1u << (q & 31)) - 1u)); };
  int* hs = hslot + (size_t)b * hcap;
  int* hr = hsrc + (size_t)b * hcap;
  for (int q = t; q < Hc; q += blockDim.x) {
    if (!(used[q >> 5] & (1u << (q & 31)))) continue;
    int h = 0;  // last run h with hoff[h] <= q
    for (int step = top; step > 0; step >>= 1)
      if (h + step < nu && hoff[h + step] <= q) h += step;
    const int j = cslot[h] + (q - hoff[h]);
    hs[halo_index(q)] = j;
    hr[halo_index(q)] = real_of[j];
  }
  // pass 2: candidate index -> halo index, a group of four per load and store
  auto group16 = [&](int k) { return *reinterpret_cast<const ushort4*>(nbr16 + lidx(w, k, lane, kcap)); };
  ushort4 next16 = kw > 0 ? group16(0) : make_ushort4(0, 0, 0, 0);
  for (int k = 0; k < kw; k += 4) {
    const ushort4 g4 = next16;
    if (k + 4 < kw) next16 = group16(k + 4);
    auto remap = [&](int q) { return (unsigned short)(q == 0xFFFF ? H : halo_index(q)); };
    *reinterpret_cast<ushort4*>(nbr16 + lidx(w, k, lane, kcap)) =
        make_ushort4(remap(g4.x), remap(g4.y), remap(g4.z), remap(g4.w));
  }
  if (t == 0) {
    tile_h[b] = H;
    atomicMax(&flags[2], H);
  }
}

// ----------------------------------------------------------- FIRE update

// One integration step of every atom with the coefficients the control
// prepared:
//   P <= 0 (neg):  x -= hsb v;  v = 0                      (Algorithm 2)
//   mix_first:     v = cv v + cf F                         (Algorithm 1)
//   v += kick1 F;  [v = cv v + cf F];  x += dtx v;  v += kick2 F
// semi-implicit Euler: kick1 = dt/m, kick2 = 0 (Algorithm 4); explicit Euler:
// kick1 = 0, kick2 = dt/m (Algorithm 3); velocity Verlet: kick1 = dt/2m and
// the second half kick in the force epilogue (Algorithm 6).
// An atom farther than skin/2 from its position at the last list build sets
// ctrl->viol; the next force pass then hands control to the host for a
// rebuild.
// Per-atom properties of a minimisation, in slot order (either may be NULL):
// sinv = 1 / m_i (mass relative to the one f2a implies) scales the atom's
// kicks; bit d of fmask holds component d of the atom fixed (its force is
// zeroed in the force epilogue, so v and x never change there).
struct Props {
  const double* sinv;
  const unsigned char* fmask;
};

// Coefficients of the pending update, as the control left them.
struct UpdCoef {
  int neg, mix_first;
  double hsb, k1, k2, cv, cf, dtx;
};
__device__ __forceinline__ UpdCoef load_coef(const Ctrl* __restrict__ c) {
  return UpdCoef{c->neg, c->mix_first, c->hsb, c->kick1, c->kick2, c->cv, c->cf, c->dtx};
}
// One atom's update (x, v in place) from its force f; s = 1/m_i scales the
// kicks (1 without masses: then k1 s = k1 exactly).  Every caller -- the
// update kernel, and the passes that apply the update while staging their
// halo -- runs this same arithmetic, so an atom gets the same bits wherever it
// is updated.
// fire_vel: everything before the drift (half step back and zeroing on
// P <= 0, kick, mixing); fire_drift: the drift with step dtx and the explicit
// Euler kick after it.  fire_step = both with dtx = dt.
__device__ __forceinline__ void fire_vel(const UpdCoef& u, double (&x)[3], double (&v)[3], const double (&f)[3],
                                         double s) {
  const double k1 = u.k1 * s;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double vd = v[d], xd = x[d];
    if (u.neg) {
      xd -= u.hsb * vd;
      vd = 0.0;
    }
    if (u.mix_first) vd = u.cv * vd + u.cf * f[d];
    vd = vd + k1 * f[d];
    if (!u.mix_first) vd = u.cv * vd + u.cf * f[d];
    v[d] = vd;
    x[d] = xd;
  }
}
__device__ __forceinline__ void fire_drift(const UpdCoef& u, double dtx, double (&x)[3], double (&v)[3],
                                           const double (&f)[3], double s) {
  const double k2 = u.k2 * s;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    x[d] = x[d] + dtx * v[d];
    v[d] = v[d] + k2 * f[d];
  }
}
__device__ __forceinline__ void fire_step(const UpdCoef& u, double (&x)[3], double (&v)[3], const double (&f)[3],
                                          double s) {
  fire_vel(u, x, v, f, s);
  fire_drift(u, u.dtx, x, v, f, s);
}

__global__ __launch_bounds__(kBlock) void k_update(double4* __restrict__ pos, double* __restrict__ vel,
                                                   const double* __restrict__ frc,
                                                   const double4* __restrict__ xref, const int* __restrict__ gcnt,
                                                   const int* __restrict__ glist, const int* __restrict__ gcode,
                                                   BoxDev box, int n, int ncap, Ctrl* __restrict__ ctrl,
                                                   Props pr) {
  // same block -> atoms map as the force passes, so each XCD updates the
  // atoms whose forces it just wrote (they are in its L2)
  const int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // the atom's own data does not depend on the control record: load it
  // first, so its latency overlaps the wait for the record
  const double4 p = pos[i];
  double v[3] = {vel[i], vel[ncap + i], vel[2 * ncap + i]};
  const double f[3] = {frc[i], frc[ncap + i], frc[2 * ncap + i]};
  const double4 r = xref[i];
  const int gc = gcnt[i];
  const double sc = pr.sinv ? pr.sinv[i] : 1.0;
  if (!ctrl_running(ctrl)) return;
  const UpdCoef u = load_coef(ctrl);
  double x[3] = {p.x, p.y, p.z};
  fire_step(u, x, v, f, sc);
  pos[i] = make_double4(x[0], x[1], x[2], p.w);
  vel[i] = v[0];
  vel[ncap + i] = v[1];
  vel[2 * ncap + i] = v[2];
  for (int k = 0; k < gc; ++k) {  // periodic images move along
    const int g = glist[8 * i + k], code = gcode[g - n];
    pos[g] = make_double4(x[0] + ghost_shift(code, 0, box), x[1] + ghost_shift(code, 1, box),
                          x[2] + ghost_shift(code, 2, box), p.w);
  }
  const double ex = x[0] - r.x, ey = x[1] - r.y, ez = x[2] - r.z;
  if (ex * ex + ey * ey + ez * ez > ctrl->skin_half2) atomicOr(&ctrl->viol, 1);
}

// The update with a displacement cap (dmax > 0) in two launches: k_update_vel
// applies everything before the drift and reduces max_i |v_i|^2; its last
// block sets the drift step dtx = min(dt, dmax / max|v|).  k_update_drift then
// moves the atoms (and their periodic images) by dtx v and tests the skin.
__global__ __launch_bounds__(kBlock) void k_update_vel(double4* __restrict__ pos, double* __restrict__ vel,
                                                       const double* __restrict__ frc, int n, int ncap,
                                                       double* __restrict__ part, Ctrl* __restrict__ ctrl,
                                                       Props pr) {
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int i = b * blockDim.x + threadIdx.x;
  if (!ctrl_running(ctrl)) return;  // uniform: the status does not change during this kernel
  const UpdCoef u = load_coef(ctrl);
  double r[1] = {0.0};
  if (i < n) {
    const double4 p = pos[i];
    double x[3] = {p.x, p.y, p.z};
    double v[3] = {vel[i], vel[ncap + i], vel[2 * ncap + i]};
    const double f[3] = {frc[i], frc[ncap + i], frc[2 * ncap + i]};
    fire_vel(u, x, v, f, pr.sinv ? pr.sinv[i] : 1.0);
    pos[i] = make_double4(x[0], x[1], x[2], p.w);
    vel[i] = v[0];
    vel[ncap + i] = v[1];
    vel[2 * ncap + i] = v[2];
    r[0] = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  }
  block_reduce<0, 1>(r);
  __shared__ int is_last;
  if (threadIdx.x == 0) {
    __hip_atomic_store(part + (size_t)kRed * b, r[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_s_waitcnt(0);
    const unsigned int t = __hip_atomic_fetch_add(&ctrl->ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    is_last = (t == gridDim.x - 1);
  }
  __syncthreads();
  if (!is_last) return;
  double q[1] = {0.0};
  for (int k = threadIdx.x; k < (int)gridDim.x; k += blockDim.x)
    q[0] = fmax(q[0], __hip_atomic_load(part + (size_t)kRed * k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  block_reduce<0, 1>(q);
  if (threadIdx.x == 0) {
    ctrl->ticket = 0;
    const double vmax = sqrt(q[0]), dt = u.dtx;
    ctrl->dtx = vmax * dt > ctrl->dmax ? ctrl->dmax / vmax : dt;
  }
}

__global__ __launch_bounds__(kBlock) void k_update_drift(double4* __restrict__ pos, double* __restrict__ vel,
                                                         const double* __restrict__ frc,
                                                         const double4* __restrict__ xref,
                                                         const int* __restrict__ gcnt, const int* __restrict__ glist,
                                                         const int* __restrict__ gcode, BoxDev box, int n, int ncap,
                                                         Ctrl* __restrict__ ctrl, Props pr) {
  const int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double4 p = pos[i];
  double v[3] = {vel[i], vel[ncap + i], vel[2 * ncap + i]};
  const double f[3] = {frc[i], frc[ncap + i], frc[2 * ncap + i]};
  const double4 r = xref[i];
  const int gc = gcnt[i];
  const double sc = pr.sinv ? pr.sinv[i] : 1.0;
  if (!ctrl_running(ctrl)) return;
  const UpdCoef u = load_coef(ctrl);
  double x[3] = {p.x, p.y, p.z};
  fire_drift(u, u.dtx, x, v, f, sc);
  pos[i] = make_double4(x[0], x[1], x[2], p.w);
  vel[i] = v[0];
  vel[ncap + i] = v[1];
  vel[2 * ncap + i] = v[2];
  for (int k = 0; k < gc; ++k) {
    const int g = glist[8 * i + k], code = gcode[g - n];
    pos[g] = make_double4(x[0] + ghost_shift(code, 0, box), x[1] + ghost_shift(code, 1, box),
                          x[2] + ghost_shift(code, 2, box), p.w);
  }
  const double ex = x[0] - r.x, ey = x[1] - r.y, ez = x[2] - r.z;
  if (ex * ex + ey * ey + ez * ez > ctrl->skin_half2) atomicOr(&ctrl->viol, 1);
}

// The loop that folds the update into the next pass leaves the state in
// either set (ctrl->cur).  These two kernels make the primary set current and
// complete: the second set's real atoms are copied over if it holds the state,
// then every periodic image is rebuilt from its source (that loop does not
// keep the images of the LJ pass up to date).
__global__ __launch_bounds__(kBlock) void k_state_home(int n, int ncap, const double4* __restrict__ pos2,
                                                       const double* __restrict__ vel2,
                                                       const double* __restrict__ frc2, double4* __restrict__ pos,
                                                       double* __restrict__ vel, double* __restrict__ frc,
                                                       const Ctrl* __restrict__ ctrl) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || ctrl->cur == 0) return;
  pos[i] = pos2[i];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    vel[d * ncap + i] = vel2[d * ncap + i];
    frc[d * ncap + i] = frc2[d * ncap + i];
  }
}

__global__ __launch_bounds__(kBlock) void k_ghost_refresh(int n, int ng, double4* __restrict__ pos,
                                                          const int* __restrict__ real_of,
                                                          const int* __restrict__ gcode, BoxDev box,
                                                          Ctrl* __restrict__ ctrl) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g == 0) ctrl->cur = 0;
  if (g >= ng) return;
  const double4 p = pos[real_of[n + g]];
  const int code = gcode[g];
  pos[n + g] = make_double4(p.x + ghost_shift(code, 0, box), p.y + ghost_shift(code, 1, box),
                            p.z + ghost_shift(code, 2, box), p.w);
}

// Entry gate of the force-evaluation kernels: run only while the FIRE loop is
// running and the list is valid; the first block that sees a skin violation
// hands control to the host.
// A pass that applies the update itself (UPD) sets the skin flag while it
// runs: it checks the status only, and its last block acts on the flag.
template <bool UPD = false>
__device__ __forceinline__ bool pass_gate(Ctrl* c) {
  const int st = __hip_atomic_load(&c->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (st != ST_RUNNING) return false;
  if constexpr (UPD) return true;
  if (__hip_atomic_load(&c->viol, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      c->pause |= PAUSE_REBUILD;
      __hip_atomic_store(&c->status, ST_PAUSED, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return false;
  }
  return true;
}

__device__ __forceinline__ double ld_cohere(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// What the epilogue needs of atom i besides its force: the velocity, 1/m
// (1 without masses) and the freeze mask.  Loaded when the pass starts (or
// carried from the update the pass applies), so the epilogue at the end of a
// block's life waits on no memory round trip.
struct EpiIn {
  double v[3];
  double sc;
  int mask;
};
__device__ __forceinline__ EpiIn epi_props(int i, bool valid, const Props& pr) {
  EpiIn a{{0.0, 0.0, 0.0}, 1.0, 0};
  if (valid) {
    if (pr.sinv) a.sc = pr.sinv[i];
    if (pr.fmask) a.mask = pr.fmask[i];
  }
  return a;
}
__device__ __forceinline__ EpiIn epi_load(int i, bool valid, const double* __restrict__ vel, int ncap,
                                          const Props& pr) {
  EpiIn a = epi_props(i, valid, pr);
  if (valid)
#pragma unroll
    for (int d = 0; d < 3; ++d) a.v[d] = vel[d * ncap + i];
  return a;
}

// Force-pass epilogue of one atom: zero the frozen components, store F,
// apply the velocity-Verlet second half kick, fold E, P, |F|^2, |v|^2,
// max |F_i|^2, max |v_i|^2 (and, with masses, sum s v.F and sum s^2 F^2)
// into the block's reduction record; the last block to finish reduces all
// records in fixed order (second stage) and runs the FIRE control.
template <int MAXB = kBlock>
__device__ __forceinline__ void force_epilogue(int i, bool valid, double fx, double fy, double fz, double e,
                                               const EpiIn& in, double* __restrict__ frc, double* __restrict__ vel,
                                               int ncap,
                                               double* __restrict__ part, double emb,
                                               int rec, Ctrl* __restrict__ ctrl, double* __restrict__ trace,
                                               const Props& pr, bool check_viol = false) {
  double r[6] = {0, 0, 0, 0, 0, 0};
  double rm[2] = {0, 0};
  if (valid) {
    if (in.mask & 1) fx = 0.0;
    if (in.mask & 2) fy = 0.0;
    if (in.mask & 4) fz = 0.0;
    frc[i] = fx;
    frc[ncap + i] = fy;
    frc[2 * ncap + i] = fz;
    double vx = in.v[0], vy = in.v[1], vz = in.v[2];
    const double sc = in.sc;
    const double kick3 = ctrl->kick3 * sc;
    if (kick3 != 0.0) {
      vx += kick3 * fx;
      vy += kick3 * fy;
      vz += kick3 * fz;
      vel[i] = vx;
      vel[ncap + i] = vy;
      vel[2 * ncap + i] = vz;
    }
    const double f2 = fx * fx + fy * fy + fz * fz, v2 = vx * vx + vy * vy + vz * vz;
    r[0] = e;
    r[1] = fx * vx + fy * vy + fz * vz;
    r[2] = f2;
    r[3] = v2;
    r[4] = f2;
    r[5] = v2;
    rm[0] = sc * r[1];
    rm[1] = (sc * sc) * f2;
  }
  // every memory operation of this thread (the skin flag's atomic among them)
  // has completed before the block's ticket is taken
  __builtin_amdgcn_s_waitcnt(0);
  block_reduce<4, 2, MAXB>(r);
  if (pr.sinv) block_reduce<2, 0, MAXB>(rm);  // uniform over the block
  __shared__ int is_last;
  if (threadIdx.x == 0) {
    // The partial record is the only data the last block reads: it is stored
    // with device-coherent atomic stores, which complete (the wait) before the
    // ticket is incremented; the last block reads the records, and the skin
    // flag, with device-coherent loads.  No cache-wide fence is needed, which
    // matters: such a fence writes back and invalidates the XCD's whole L2
    // under every other block still running there.  Later kernels see the
    // rest of this pass's output through the kernel boundary.
    // Records are stored field by field (field k of block b at k * grid + b),
    // so the last block's lanes read consecutive words.
    const double vals[kCtl] = {r[0] + emb, r[1], r[2], r[3], r[4], r[5], rm[0], rm[1]};
    const int nv = pr.sinv ? kCtl : 6;
    for (int k = 0; k < nv; ++k)
      __hip_atomic_store(part + (size_t)k * gridDim.x + rec, vals[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_s_waitcnt(0);
    const unsigned int t = __hip_atomic_fetch_add(&ctrl->ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    is_last = (t == gridDim.x - 1);
  }
  __syncthreads();
  if (!is_last) return;
  // Second stage: each lane reads up to four records per round with all
  // their loads in flight at once (one memory round trip per round), then the
  // lanes reduce.  Up to 256 records one wave does it alone (no LDS, no
  // barrier); beyond that the whole block reads and reduces.  Either order
  // is fixed for a given grid.  Without masses the mass-weighted sums are P
  // and |F|^2 exactly and are not read.
  const int nb = (int)gridDim.x;
  const bool one_wave = nb <= 4 * 64;
  if (one_wave && threadIdx.x >= 64) return;
  const int lanes = one_wave ? 64 : (int)blockDim.x;
  const int nv = pr.sinv ? kCtl : 6;
  // The control record and the skin flag, read once, in flight with the
  // records: nothing writes the record during the pass but this thread below,
  // and every block set the flag (device-scope atomic, completed) before
  // taking its ticket.
  Ctrl snap;
  int viol = 0;
  if (threadIdx.x == 0) {
    snap = *ctrl;
    if (check_viol) viol = __hip_atomic_load(&ctrl->viol, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  double q[6] = {0, 0, 0, 0, 0, 0};
  double qm[2] = {0, 0};
  for (int b0 = 0; b0 < nb; b0 += 4 * lanes) {
    double t[4][kCtl];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int b = b0 + u * lanes + (int)threadIdx.x;
#pragma unroll
      for (int k = 0; k < kCtl; ++k) t[u][k] = (b < nb && k < nv) ? ld_cohere(part + (size_t)k * nb + b) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      q[0] += t[u][R_E];
      q[1] += t[u][R_P];
      q[2] += t[u][R_F2];
      q[3] += t[u][R_V2];
      q[4] = fmax(q[4], t[u][R_FMAX2]);
      q[5] = fmax(q[5], t[u][R_VMAX2]);
      qm[0] += t[u][R_SVF];
      qm[1] += t[u][R_SFF];
    }
  }
  if (one_wave) {
#pragma unroll
    for (int k = 0; k < 4; ++k) q[k] = wave_sum(q[k]);
    q[4] = wave_max(q[4]);
    q[5] = wave_max(q[5]);
    if (pr.sinv) {
      qm[0] = wave_sum(qm[0]);
      qm[1] = wave_sum(qm[1]);
    }
  } else {
    block_reduce<4, 2, MAXB>(q);
    if (pr.sinv) block_reduce<2, 0, MAXB>(qm);
  }
  if (!pr.sinv) {
    qm[0] = q[R_P];
    qm[1] = q[R_F2];
  }
  if (threadIdx.x == 0) {
    const double qc[kCtl] = {q[0], q[1], q[2], q[3], q[4], q[5], qm[0], qm[1]};
    ctrl->ticket = 0;
    if (viol) {
      // the update applied in this pass moved an atom past its skin: these
      // forces used a stale list; hand over for a rebuild, FIRE state unchanged
      ctrl->pause = snap.pause | PAUSE_REBUILD;
      __hip_atomic_store(&ctrl->status, ST_PAUSED, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      snap.ticket = 0;
      fire_control(snap, ctrl, qc, trace);
    }
  }
}

// ------------------------------------------------------------ pair kernels

// Tile data of the LDS-staged passes.
struct Tiles {
  const int* tile_h;           // halo size per tile
  const int* hslot;            // halo slot lists, hcap per tile
  const int* hsrc;             // the real atom behind each halo slot (itself, or an image's source)
  const unsigned short* nbr16; // neighbour lists as halo indices
  int hcap;
};


// Position of the list padding slot: far outside any system, finite in FP32.
constexpr double kFar = 1.0e20;

// A tile's halo in LDS, S = H + 1 entries (entry H is the far padding atom):
// (x, y) pairs in the first 2S doubles, then z in [2S, 3S) or, with F'(rho)
// (the EAM force pass), (z, F'(rho)) pairs in [2S, 4S).  A neighbour costs
// one 16-byte read and one 8- or 16-byte read (against three or four 8-byte
// reads of separate arrays, the same bytes: LJ and EAM-form relaxations
// 1-2 % faster).
struct Halo {
  const double* a;
  int S;
};

// Copy tile b's halo into LDS; W: also F'(rho) (pos.w).  Four entries per
// thread and round, so their loads are in flight together.
template <bool W>
__device__ __forceinline__ Halo stage_halo(const double4* __restrict__ pos, const Tiles& tl, int b) {
  double* h = reinterpret_cast<double*>(dyn_lds);
  const int H = tl.tile_h[b];
  const int S = H + 1;
  const int* hs = tl.hslot + (size_t)b * tl.hcap;
  const int step = blockDim.x;
  for (int q0 = threadIdx.x; q0 < H; q0 += 4 * step) {
    int idx[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) idx[u] = (q0 + u * step < H) ? hs[q0 + u * step] : -1;
    double4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (idx[u] >= 0) v[u] = pos[idx[u]];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (idx[u] >= 0) {
        const int q = q0 + u * step;
        reinterpret_cast<double2*>(h)[q] = make_double2(v[u].x, v[u].y);
        if constexpr (W) reinterpret_cast<double2*>(h)[S + q] = make_double2(v[u].z, v[u].w);
        else h[2 * S + q] = v[u].z;
      }
  }
  if (threadIdx.x == 0) {
    reinterpret_cast<double2*>(h)[H] = make_double2(kFar, kFar);
    if constexpr (W) reinterpret_cast<double2*>(h)[S + H] = make_double2(kFar, 0.0);
    else h[2 * S + H] = kFar;
  }
  __syncthreads();
  return Halo{h, S};
}

// Neighbour loop shared by the pair kernels: one lane per atom, wave-uniform
// trip count, four neighbours per step (handed to group() together, so their
// terms interleave and a wave-uniform test can skip all four at once),
// software-pipelined: index groups are
// fetched two steps ahead (one 8- or 16-byte load per lane), and for global
// gathers the positions one step ahead.  Neighbouring lanes hold neighbouring
// atoms, so at each step they gather nearby (often identical) neighbours.
// LDS: positions from the tile's halo in LDS by 16-bit index (W: with
// F'(rho) in .w); otherwise gathered from global memory by slot index.
template <bool LDS, bool W, typename F>
__device__ __forceinline__ void for_neighbours(const double4* __restrict__ pos, const Halo& halo,
                                               const int* __restrict__ nbr, const Tiles& tl,
                                               const int* __restrict__ wcnt, int kcap, int i, F&& group) {
  const int w = i >> 6, lane = threadIdx.x & 63;
  const int ng = __builtin_amdgcn_readfirstlane(wcnt[w]) >> 2;
  const size_t base = (size_t)w * (kcap >> 2) * 64 + lane;
  if constexpr (LDS) {
    const ushort4* l4 = reinterpret_cast<const ushort4*>(tl.nbr16) + base;
    const double2* hxy = reinterpret_cast<const double2*>(halo.a);
    const double* hz = halo.a + 2 * halo.S;
    auto at = [&](int c) {
      const double2 xy = hxy[c];
      if constexpr (W) {
        const double2 zw = hxy[halo.S + c];
        return make_double4(xy.x, xy.y, zw.x, zw.y);
      } else {
        return make_double4(xy.x, xy.y, hz[c], 0.0);
      }
    };
    ushort4 a = make_ushort4(0, 0, 0, 0), b = a;
    if (ng > 0) a = l4[0];
    if (ng > 1) b = l4[64];
    for (int g = 0; g < ng; ++g) {
      const ushort4 c = a;
      a = b;
      if (g + 2 < ng) b = l4[(size_t)(g + 2) * 64];
      group(at(c.x), at(c.y), at(c.z), at(c.w));
    }
  } else {
    const int4* l4 = reinterpret_cast<const int4*>(nbr) + base;
    int4 a = make_int4(0, 0, 0, 0), b = a;
    double4 q0{}, q1{}, q2{}, q3{};
    if (ng > 0) {
      a = l4[0];
      q0 = pos[a.x];
      q1 = pos[a.y];
      q2 = pos[a.z];
      q3 = pos[a.w];
    }
    if (ng > 1) a = l4[64];
    if (ng > 2) b = l4[128];
    for (int g = 0; g < ng; ++g) {
      const double4 p0 = q0, p1 = q1, p2 = q2, p3 = q3;
      if (g + 1 < ng) {
        q0 = pos[a.x];
        q1 = pos[a.y];
        q2 = pos[a.z];
        q3 = pos[a.w];
      }
      a = b;
      if (g + 3 < ng) b = l4[(size_t)(g + 3) * 64];
      group(p0, p1, p2, p3);
    }
  }
}

// One set of per-atom state: positions (slots, with periodic images),
// velocities and forces (3 planes of ncap).  The LDS-staged loop keeps two
// sets and alternates between them: a pass that applies the update reads one
// and writes the other.
struct StateBuf {
  double4* pos;
  double* vel;
  double* frc;
};

// What a pass that applies the pending update needs besides the state.
struct UpdArgs {
  StateBuf src, dst;
  int dst_index;                  // 1 if dst is the second set
  const int* real_of;             // slot -> source real slot
  const int* gcode;               // image shift codes of the periodic images
  const int* gcnt;                // images per real atom
  const int* glist;               // their slots
  const double4* xref;            // positions at the last list build
  const double* sinv;             // 1 / m per real slot, or NULL
  BoxDev box;
};

// Tile b's halo with the pending update applied on the fly: each halo atom
// (an image through its source and shift) is advanced from `src` by
// fire_step, exactly as its owner advances it.
__device__ __forceinline__ Halo stage_halo_updated(const UpdArgs& ua, const UpdCoef& u, const Tiles& tl, int b,
                                                   int n, int ncap) {
  double* h = reinterpret_cast<double*>(dyn_lds);
  const int H = tl.tile_h[b];
  const int S = H + 1;
  const int* hs = tl.hslot + (size_t)b * tl.hcap;
  const int* hr = tl.hsrc + (size_t)b * tl.hcap;
  const int step = blockDim.x;
  for (int q0 = threadIdx.x; q0 < H; q0 += 2 * step) {  // two entries in flight
    int j[2], r[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int q = q0 + e * step;
      j[e] = q < H ? hs[q] : -1;
      r[e] = q < H ? hr[q] : 0;
    }
    double x[2][3], v[2][3], f[2][3], sc[2];
    int code[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      if (j[e] < 0) continue;
      const double4 p = ua.src.pos[r[e]];
      x[e][0] = p.x;
      x[e][1] = p.y;
      x[e][2] = p.z;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        v[e][d] = ua.src.vel[d * ncap + r[e]];
        f[e][d] = ua.src.frc[d * ncap + r[e]];
      }
      code[e] = j[e] >= n ? ua.gcode[j[e] - n] : 0;
      sc[e] = ua.sinv ? ua.sinv[r[e]] : 1.0;
    }
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      if (j[e] < 0) continue;
      fire_step(u, x[e], v[e], f[e], sc[e]);
      const int q = q0 + e * step;
      reinterpret_cast<double2*>(h)[q] =
          make_double2(x[e][0] + ghost_shift(code[e], 0, ua.box), x[e][1] + ghost_shift(code[e], 1, ua.box));
      h[2 * S + q] = x[e][2] + ghost_shift(code[e], 2, ua.box);
    }
  }
  if (threadIdx.x == 0) {
    reinterpret_cast<double2*>(h)[H] = make_double2(kFar, kFar);
    h[2 * S + H] = kFar;
  }
  __syncthreads();
  return Halo{h, S};
}

// The pending update of a pass's own atom i (< n): new position (returned,
// w as in src) and velocity written to dst (and kept in ep for the
// epilogue; ep.sc must hold the atom's 1/m), skin test against the build
// positions.
__device__ __forceinline__ double4 own_update(const UpdArgs& ua, const UpdCoef& u, int i, int ncap, Ctrl* ctrl,
                                              EpiIn& ep) {
  const double4 p = ua.src.pos[i];
  double x[3] = {p.x, p.y, p.z};
  double v[3] = {ua.src.vel[i], ua.src.vel[ncap + i], ua.src.vel[2 * ncap + i]};
  const double f[3] = {ua.src.frc[i], ua.src.frc[ncap + i], ua.src.frc[2 * ncap + i]};
  fire_step(u, x, v, f, ep.sc);
  ua.dst.vel[i] = v[0];
  ua.dst.vel[ncap + i] = v[1];
  ua.dst.vel[2 * ncap + i] = v[2];
#pragma unroll
  for (int d = 0; d < 3; ++d) ep.v[d] = v[d];
  const double4 xr = ua.xref[i];
  const double ex = x[0] - xr.x, ey = x[1] - xr.y, ez = x[2] - xr.z;
  if (ex * ex + ey * ey + ez * ez > ctrl->skin_half2) atomicOr(&ctrl->viol, 1);
  return make_double4(x[0], x[1], x[2], p.w);
}

__device__ __forceinline__ double sep2(const double4& a, const double4& b) {
  const double dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
  return dx * dx + dy * dy + dz * dz;
}

// One group of four neighbours of the EAM-form passes.  Nothing is added
// when no lane has one of them within the cutoff (the far entries of the
// lists and their padding); the taper is evaluated only when some lane has
// one of them past r_in (in range), which in a relaxed crystal is a few
// groups per list: pair(p, taper) with taper a compile-time bool.  The
// taper threshold is widened by 1e-12 relative so that rounding of r never
// skips it where it differs from 1.
template <typename T, typename F>
__device__ __forceinline__ void group_terms(const double4& pi, const double4& p0, const double4& p1,
                                            const double4& p2, const double4& p3, const PotDev& pot, F&& pair) {
  if constexpr (sizeof(T) == 4) {
    // FP32 terms: branch-free (measured faster there; their arithmetic per
    // entry is short enough that the tests do not pay)
    pair(p0, std::true_type{});
    pair(p1, std::true_type{});
    pair(p2, std::true_type{});
    pair(p3, std::true_type{});
    return;
  }
  const double a0 = sep2(pi, p0), a1 = sep2(pi, p1), a2 = sep2(pi, p2), a3 = sep2(pi, p3);
  if (!wave_any(a0 < pot.rc2 || a1 < pot.rc2 || a2 < pot.rc2 || a3 < pot.rc2)) return;
  const double t2 = pot.r_in * pot.r_in * (1.0 - 1e-12);
  auto past = [&](double a) { return a < pot.rc2 && a > t2; };
  if (wave_any(past(a0) || past(a1) || past(a2) || past(a3))) {
    pair(p0, std::true_type{});
    pair(p1, std::true_type{});
    pair(p2, std::true_type{});
    pair(p3, std::true_type{});
  } else {
    pair(p0, std::false_type{});
    pair(p1, std::false_type{});
    pair(p2, std::false_type{});
    pair(p3, std::false_type{});
  }
}

// Energy-shifted LJ.  Separations and the r^2 < rc^2 test in FP64; the pair
// terms and per-atom accumulation in T (double, or float for the mixed path).
// WE: accumulate the energy (the FIRE logic itself needs only forces).
// UPD: the pass first applies the pending update (halo atoms on the fly in
// LDS, own atoms written to ua.dst) and reads and writes ua's state sets
// instead of pos / frc / vel; requires LDS.
template <typename T, bool LDS, bool WE, bool UPD>
__device__ __forceinline__ void lj_force_pass(const double4* __restrict__ pos, const int* __restrict__ nbr, Tiles tl,
                                              const int* __restrict__ wcnt, int n, int kcap, int ncap, PotDev pot,
                                              double* __restrict__ frc, double* __restrict__ vel,
                                              double* __restrict__ part, Ctrl* __restrict__ ctrl,
                                              double* __restrict__ trace, const UpdArgs& ua, const Props& pr) {
  static_assert(!UPD || LDS, "the update is applied while staging the LDS halo");
  if (!pass_gate<UPD>(ctrl)) return;
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int i = b * blockDim.x + threadIdx.x;
  const bool valid = i < n;
  T ax = 0, ay = 0, az = 0, ae = 0;
  Halo halo{nullptr, 0};
  double4 pi;
  EpiIn ep;
  if constexpr (UPD) {
    const UpdCoef u = load_coef(ctrl);
    ep = epi_props(i, valid, pr);
    if (valid) {
      pi = own_update(ua, u, i, ncap, ctrl, ep);
      ua.dst.pos[i] = pi;
    } else {
      pi = ua.src.pos[i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) ctrl->cur = ua.dst_index;
    halo = stage_halo_updated(ua, u, tl, b, n, ncap);
    frc = ua.dst.frc;
    vel = ua.dst.vel;
  } else {
    ep = epi_load(i, valid, vel, ncap, pr);
    if constexpr (LDS) halo = stage_halo<false>(pos, tl, b);
    pi = pos[i];
  }
  const T eps24 = (T)(24.0 * pot.eps), eps4 = (T)(4.0 * pot.eps), sig2 = (T)pot.sig2, sh = (T)pot.shift;
  auto pair = [&](const double4& pj) {
    const double dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
    const double r2 = dx * dx + dy * dy + dz * dz;
    // branch-free within the wave: out-of-range lanes (including the far
    // padding) evaluate at r = 1 and get a zero weight
    const bool in = r2 < pot.rc2;
    T ir2;
    if constexpr (sizeof(T) == 8) ir2 = rcp_d(in ? r2 : 1.0);
    else ir2 = rcp_f(in ? (float)r2 : 1.0f);
    const T s2 = sig2 * ir2, s6 = s2 * s2 * s2;
    const T fr = in ? eps24 * s6 * ((T)2 * s6 - (T)1) * ir2 : (T)0;
    ax += fr * (T)dx;
    ay += fr * (T)dy;
    az += fr * (T)dz;
    if constexpr (WE) ae += in ? (T)0.5 * (eps4 * s6 * (s6 - (T)1) - sh) : (T)0;
  };
  for_neighbours<LDS, false>(pos, halo, nbr, tl, wcnt, kcap, i,
                             [&](const double4& p0, const double4& p1, const double4& p2, const double4& p3) {
                               pair(p0);
                               pair(p1);
                               pair(p2);
                               pair(p3);
                             });
  force_epilogue<kMaxTile>(i, valid, (double)ax, (double)ay, (double)az, (double)ae, ep, frc, vel, ncap, part, 0.0,
                           b, ctrl, trace, pr, UPD);
}

template <typename T, bool LDS, bool WE, bool UPD = false>
__global__ __launch_bounds__(kMaxTile) void k_lj_force(const double4* __restrict__ pos, const int* __restrict__ nbr,
                                                     Tiles tl, const int* __restrict__ wcnt, int n, int kcap,
                                                     int ncap, PotDev pot, double* __restrict__ frc,
                                                     double* __restrict__ vel, double* __restrict__ part,
                                                     Ctrl* __restrict__ ctrl, double* __restrict__ trace,
                                                     UpdArgs ua, Props pr) {
  lj_force_pass<T, LDS, WE, UPD>(pos, nbr, tl, wcnt, n, kcap, ncap, pot, frc, vel, part, ctrl, trace, ua, pr);
}

// The same pass compiled for four waves per SIMD (at most 128 VGPRs, a few
// spills outside the pair loop), so that two 512-atom tile blocks share a CU
// when there are more tiles than CUs (1,043,333 atoms: 179 against 231 us per
// pass).  With one tile per CU at most (the 130,417-atom box) k_lj_force,
// which keeps every value in registers, is a little faster (28.1 against
// 28.4 us).
template <typename T, bool LDS, bool WE, bool UPD = false>
__global__ __launch_bounds__(kMaxTile, 4) void k_lj_force_two_per_cu(
    const double4* __restrict__ pos, const int* __restrict__ nbr, Tiles tl, const int* __restrict__ wcnt, int n,
    int kcap, int ncap, PotDev pot, double* __restrict__ frc, double* __restrict__ vel, double* __restrict__ part,
    Ctrl* __restrict__ ctrl, double* __restrict__ trace, UpdArgs ua, Props pr) {
  lj_force_pass<T, LDS, WE, UPD>(pos, nbr, tl, wcnt, n, kcap, ncap, pot, frc, vel, part, ctrl, trace, ua, pr);
}

// Gupta density pass: rho_i = sum_j exp(-2q (r/r0 - 1)) S(r); stores
// F'(rho_i) = -xi / (2 sqrt(rho_i)) in pos[i].w and sums F(rho_i) per block.
// UPD: the pass first applies the pending update (as in k_lj_force) and
// writes the new positions, with F'(rho) in .w, of its atoms and their
// periodic images to ua.dst.pos; requires LDS.
template <typename T, bool LDS, bool UPD = false, int TILE = kBlock>
__global__ __launch_bounds__(TILE) void k_gupta_density(double4* __restrict__ pos, const int* __restrict__ nbr,
                                                          Tiles tl, const int* __restrict__ wcnt, int n, int kcap,
                                                          int ncap, PotDev pot, const int* __restrict__ gcnt,
                                                          const int* __restrict__ glist,
                                                          double* __restrict__ part_emb, Ctrl* __restrict__ ctrl,
                                                          UpdArgs ua) {
  static_assert(!UPD || LDS, "the update is applied while staging the LDS halo");
  if (!pass_gate<UPD>(ctrl)) return;
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int i = b * blockDim.x + threadIdx.x;
  double emb = 0.0;
  Halo halo{nullptr, 0};
  double4 pi;
  if constexpr (UPD) {
    const UpdCoef u = load_coef(ctrl);
    EpiIn ep{{0.0, 0.0, 0.0}, (ua.sinv && i < n) ? ua.sinv[i] : 1.0, 0};
    pi = i < n ? own_update(ua, u, i, ncap, ctrl, ep) : ua.src.pos[i];
    if (blockIdx.x == 0 && threadIdx.x == 0) ctrl->cur = ua.dst_index;
    halo = stage_halo_updated(ua, u, tl, b, n, ncap);
    pos = ua.dst.pos;
  } else {
    if constexpr (LDS) halo = stage_halo<false>(pos, tl, b);
    pi = pos[i];
  }
  const T qr0 = (T)pot.qr0, r0 = (T)pot.r0, r_in = (T)pot.r_in, inv_w = (T)pot.inv_w;
  T rho = 0;
  auto pair = [&](const double4& pj, auto taper) {
    const double r2 = sep2(pi, pj);
    const bool in = r2 < pot.rc2;
    T r;
    if constexpr (sizeof(T) == 8) {
      const double r2c = in ? r2 : 1.0;
      r = r2c * rsqrt_d(r2c);
    } else {
      r = sqrt_f(in ? (float)r2 : 1.0f);
    }
    T S = 1;  // the taper is 1 below r_in
    if constexpr (decltype(taper)::value) {
      const T s = fmin(fmax((r - r_in) * inv_w, (T)0), (T)1);
      S = (1 - s) * (1 - s) * (1 + 2 * s);
    }
    T e;
    if constexpr (sizeof(T) == 8) e = exp_d(-qr0 * (r - r0));
    else e = exp_f(-qr0 * (r - r0));
    rho += in ? e * S : (T)0;
  };
  for_neighbours<LDS, false>(pos, halo, nbr, tl, wcnt, kcap, i,
                             [&](const double4& p0, const double4& p1, const double4& p2, const double4& p3) {
                               group_terms<T>(pi, p0, p1, p2, p3, pot, pair);
                             });
  if (i < n) {
    double fp = 0.0;
    if (rho > 0) {
      const double sq = sqrt((double)rho);
      fp = -0.5 * pot.xi / sq;
      emb = -pot.xi * sq;
    }
    if constexpr (UPD) {  // new position and its images, with F'(rho)
      pos[i] = make_double4(pi.x, pi.y, pi.z, fp);
      for (int k = 0, gc = gcnt[i]; k < gc; ++k) {
        const int g = glist[8 * i + k], code = ua.gcode[g - n];
        pos[g] = make_double4(pi.x + ghost_shift(code, 0, ua.box), pi.y + ghost_shift(code, 1, ua.box),
                              pi.z + ghost_shift(code, 2, ua.box), fp);
      }
    } else {
      pos[i].w = fp;
      for (int k = 0, gc = gcnt[i]; k < gc; ++k) pos[glist[8 * i + k]].w = fp;
    }
  }
  double r[1] = {emb};
  block_reduce<1, 0, TILE>(r);
  if (threadIdx.x == 0) part_emb[b] = r[0];
}

// Gupta force pass: F_i = -sum_j [c phi_t'(r) + (F'_i + F'_j) rho_t'(r)] d/r,
// e_i = w_e sum_j phi_t(r).  512-atom tiles run two blocks per CU (their LDS
// reservation is sized for that), which needs four waves per SIMD: at most
// 128 VGPRs per lane.
template <typename T, bool LDS, bool WE, int TILE = kBlock>
__global__ __launch_bounds__(TILE, LDS && TILE >= 512 ? 4 : 1) void k_gupta_force(const double4* __restrict__ pos, const int* __restrict__ nbr,
                                                        Tiles tl, const int* __restrict__ wcnt, int n, int kcap,
                                                        int ncap, PotDev pot, double* __restrict__ frc,
                                                        double* __restrict__ vel, double* __restrict__ part,
                                                        const double* __restrict__ part_emb,
                                                        Ctrl* __restrict__ ctrl, double* __restrict__ trace,
                                                        Props pr) {
  if (!pass_gate(ctrl)) return;
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int i = b * blockDim.x + threadIdx.x;
  const bool valid = i < n;
  const EpiIn ep = epi_load(i, valid, vel, ncap, pr);
  const double emb = threadIdx.x == 0 ? part_emb[b] : 0.0;  // the block's sum of F(rho), from the density pass
  const Halo halo = LDS ? stage_halo<true>(pos, tl, b) : Halo{nullptr, 0};
  T ax = 0, ay = 0, az = 0, ae = 0;
  const double4 pi = pos[i];
  const T A = (T)pot.A, pr0 = (T)pot.pr0, qr0 = (T)pot.qr0, r0 = (T)pot.r0, r_in = (T)pot.r_in,
          inv_w = (T)pot.inv_w, cpair = (T)pot.cpair, epair = (T)pot.epair, fpi = (T)pi.w;
  auto pair = [&](const double4& pj, auto taper) {
    const double dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
    const double r2 = dx * dx + dy * dy + dz * dz;
    const bool in = r2 < pot.rc2;
    const double r2c = in ? r2 : 1.0;
    T ir;
    if constexpr (sizeof(T) == 8) ir = rsqrt_d(r2c);
    else ir = rsqrt_f((float)r2c);
    const T r = (T)r2c * ir;
    T S = 1, dS = 0;  // the taper and its slope are 1 and 0 below r_in
    if constexpr (decltype(taper)::value) {
      const T s = fmin(fmax((r - r_in) * inv_w, (T)0), (T)1);
      S = (1 - s) * (1 - s) * (1 + 2 * s);
      dS = (T)(-6) * s * (1 - s) * inv_w;
    }
    T ph, rh;
    if constexpr (sizeof(T) == 8) {
      ph = A * exp_d(-pr0 * (r - r0));
      rh = exp_d(-qr0 * (r - r0));
    } else {
      ph = A * exp_f(-pr0 * (r - r0));
      rh = exp_f(-qr0 * (r - r0));
    }
    const T dph = ph * (dS - pr0 * S);
    const T drh = rh * (dS - qr0 * S);
    const T fpj = in ? (T)pj.w : (T)0;
    const T dEdr = cpair * dph + (fpi + fpj) * drh;
    const T fr = in ? -dEdr * ir : (T)0;
    ax += fr * (T)dx;
    ay += fr * (T)dy;
    az += fr * (T)dz;
    if constexpr (WE) ae += in ? epair * ph * S : (T)0;
  };
  for_neighbours<LDS, true>(pos, halo, nbr, tl, wcnt, kcap, i,
                            [&](const double4& p0, const double4& p1, const double4& p2, const double4& p3) {
                              group_terms<T>(pi, p0, p1, p2, p3, pot, pair);
                            });
  force_epilogue<TILE>(i, valid, (double)ax, (double)ay, (double)az, (double)ae, ep, frc, vel, ncap, part, emb, b,
                 ctrl, trace, pr);
}

// Quadratic test well E = 1/2 sum k_d x_d^2 (no pairs).
__global__ __launch_bounds__(kBlock) void k_harmonic_force(const double4* __restrict__ pos, int n, int ncap,
                                                           PotDev pot, double* __restrict__ frc,
                                                           double* __restrict__ vel, double* __restrict__ part,
                                                           Ctrl* __restrict__ ctrl, double* __restrict__ trace,
                                                           Props pr) {
  if (!pass_gate(ctrl)) return;
  const int b = blockIdx.x;
  const int i = b * blockDim.x + threadIdx.x;
  const bool valid = i < n;
  double fx = 0, fy = 0, fz = 0, e = 0;
  if (valid) {
    double4 p = pos[i];
    fx = -pot.k[0] * p.x;
    fy = -pot.k[1] * p.y;
    fz = -pot.k[2] * p.z;
    e = 0.5 * (pot.k[0] * p.x * p.x + pot.k[1] * p.y * p.y + pot.k[2] * p.z * p.z);
  }
  force_epilogue(i, valid, fx, fy, fz, e, epi_load(i, valid, vel, ncap, pr), frc, vel, ncap, part, 0.0, b, ctrl,
                 trace, pr);
}

// Neighbour indices of atom i one at a time (dummy padding included; callers
// reject it by the cutoff test before touching per-atom arrays).
template <typename F>
__device__ __forceinline__ void for_neighbour_index(const int* __restrict__ nbr, const int* __restrict__ wcnt,
                                                    int kcap, int i, F&& fn) {
  const int w = i >> 6, lane = threadIdx.x & 63;
  const int kw = wcnt[w];
  for (int k = 0; k < kw; ++k) fn(nbr[lidx(w, k, lane, kcap)]);
}

// -------------------------------------------------- Stillinger-Weber (FP64)
//
// Two passes per evaluation.  k_sw_short compacts each real atom's in-range
// neighbours (r < a sigma) from the skin list into a short list of 64-byte
// records {x_j - x_i, 1/r ; g(r), g'(r), real atom of j} and sums the atom's
// pair terms.  k_sw_force then gathers every three-body term that contains x_i:
// the triplets centred at i, from i's own list, and the triplets centred at
// each neighbour m with i as one end, from m's list (a periodic image reads
// its source's list: relative vectors are the same).  No atomics: every
// atom sums its own force in a fixed order.

// (s/r)^p: integer exponents up to 16 by repeated squaring (the published Si
// set has p = 4, q = 0), others through pow.
__device__ __forceinline__ double sw_pow(double x, double p) {
  const int k = (int)p;
  if ((double)k == p && k >= 0 && k <= 16) {
    double r = 1.0, b = x;
    for (int m = k; m; m >>= 1) {
      if (m & 1) r *= b;
      b *= b;
    }
    return r;
  }
  return pow(x, p);
}

__device__ __forceinline__ void sw_record(double4* __restrict__ rec, double dx, double dy, double dz, double ir,
                                          double g, double g1, int j) {
  rec[0] = make_double4(dx, dy, dz, ir);
  rec[1] = make_double4(g, g1, (double)j, 0.0);
}

// G lanes per atom: lane g takes candidates g, g + G, ...; a wave ballot
// gives each in-range candidate its record slot in list order of the rounds
// (a wave's groups are atoms of one list wave, so every lane runs the same
// number of rounds).  The group's partial pair sums are combined by a fixed
// butterfly.
template <int G>
__global__ __launch_bounds__(kBlock) void k_sw_short(const double4* __restrict__ pos, const int* __restrict__ nbr,
                                                     const int* __restrict__ wcnt, const int* __restrict__ real_of,
                                                     int n, int kcap, PotDev pot,
                                                     double4* __restrict__ sw_nb, int* __restrict__ sw_cnt,
                                                     double4* __restrict__ sw_fe, Ctrl* __restrict__ ctrl) {
  static_assert(G > 0 && 64 % G == 0, "a group must divide the wave");
  if (!pass_gate(ctrl)) return;
  constexpr int kAtoms = kBlock / G;
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int i = b * kAtoms + (int)threadIdx.x / G, g = threadIdx.x % G;
  const int lane = threadIdx.x & 63;
  const unsigned long long group = ((1ull << G) - 1) << (lane & ~(G - 1));
  const bool valid = i < n;
  const int w = i >> 6, l = i & 63;
  const int kw = wcnt[w];
  const double4 pi = pos[valid ? i : 0];
  double4* rec = sw_nb + 2 * (size_t)i * kcap;
  double fx = 0.0, fy = 0.0, fz = 0.0, e = 0.0;
  int c = 0;
  for (int k0 = 0; k0 < kw; k0 += G) {
    const int k = k0 + g;
    bool in = false;
    int j = 0, rj = 0;
    double dx = 0.0, dy = 0.0, dz = 0.0, r2 = 0.0;
    if (valid && k < kw) {
      j = nbr[lidx(w, k, l, kcap)];
      const double4 pj = pos[j];
      rj = real_of[j];  // gathered beside the position; the force pass needs the real atom only
      dx = pj.x - pi.x;
      dy = pj.y - pi.y;
      dz = pj.z - pi.z;
      r2 = dx * dx + dy * dy + dz * dz;
      in = r2 < pot.rc2;
    }
    const unsigned long long mine = __ballot(in) & group;
    if (in) {
      const double r = sqrt(r2), ir = 1.0 / r, t = 1.0 / (r - pot.sw_as);
      const double gg = exp(pot.sw_gs * t), g1 = -pot.sw_gs * t * t * gg;
      // pair term and its derivative along r
      const double sr = pot.sw_s * ir;
      const double bp = pot.sw_B * sw_pow(sr, pot.sw_p), bq = sw_pow(sr, pot.sw_q);
      const double poly = bp - bq, dpoly = (-pot.sw_p * bp + pot.sw_q * bq) * ir;
      const double ex = exp(pot.sw_s * t), dex = -pot.sw_s * t * t * ex;
      const double f1 = pot.sw_Aeps * (dpoly * ex + poly * dex);
      e += 0.5 * pot.sw_Aeps * poly * ex;
      fx += f1 * dx * ir;
      fy += f1 * dy * ir;
      fz += f1 * dz * ir;
      sw_record(rec + 2 * (c + __popcll(mine & ((1ull << lane) - 1))), dx, dy, dz, ir, gg, g1, rj);
    }
    c += __popcll(mine);
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) {
    fx += __shfl_xor(fx, o, 64);
    fy += __shfl_xor(fy, o, 64);
    fz += __shfl_xor(fz, o, 64);
    e += __shfl_xor(e, o, 64);
  }
  if (valid && g == 0) {
    sw_cnt[i] = c;
    sw_fe[i] = make_double4(fx, fy, fz, e);
  }
}

// Gradient of the triplet term (centre c, ends a, b) with respect to the
// end vector u = x_a - x_c, given w = x_b - x_c; returns h.  When both is
// set, adds dh/du + dh/dw into acc, else subtracts dh/du.
template <bool BOTH>
__device__ __forceinline__ double sw_triplet(const PotDev& pot, const double (&u)[3], double iru, double gu,
                                             double gu1, const double (&w)[3], double irw, double gw, double gw1,
                                             double (&acc)[3]) {
  const double c = (u[0] * w[0] + u[1] * w[1] + u[2] * w[2]) * iru * irw;
  const double t = c + 1.0 / 3.0;
  const double a2 = 2.0 * pot.sw_leps * t * gu * gw;  // dh/dcos
  const double bu = pot.sw_leps * t * t * gu1 * gw * iru;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double dcu = w[d] * iru * irw - c * u[d] * iru * iru;
    const double dhu = a2 * dcu + bu * u[d];
    if constexpr (BOTH) {
      const double dcw = u[d] * iru * irw - c * w[d] * irw * irw;
      const double dhw = a2 * dcw + pot.sw_leps * t * t * gu * gw1 * irw * w[d];
      acc[d] += dhu + dhw;
    } else {
      acc[d] -= dhu;
    }
  }
  return pot.sw_leps * t * t * gu * gw;
}

// G lanes per atom: lane g takes the atom's short-list entries a = g, g + G, ...
// (the triplets centred at i with a as the first end, and those centred at
// neighbour a with i as an end); the group's sums are combined by a fixed
// butterfly and the first lane runs the epilogue.
template <int G>
__global__ __launch_bounds__(kBlock) void k_sw_force(const double4* __restrict__ sw_nb, const int* __restrict__ sw_cnt,
                                                     const double4* __restrict__ sw_fe, int n, int kcap, int ncap,
                                                     PotDev pot, double* __restrict__ frc, double* __restrict__ vel,
                                                     double* __restrict__ part, Ctrl* __restrict__ ctrl,
                                                     double* __restrict__ trace, Props pr) {
  static_assert(G > 0 && 64 % G == 0, "a group must divide the wave");
  if (!pass_gate(ctrl)) return;
  constexpr int kAtoms = kBlock / G;
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int i = b * kAtoms + (int)threadIdx.x / G, g = threadIdx.x % G;
  const bool valid = i < n;
  const bool lead = valid && g == 0;
  // the lead lane's epilogue inputs and pair-term sums, loaded up front
  const EpiIn ep = epi_load(i, lead, vel, ncap, pr);
  const double4 fe = lead ? sw_fe[i] : make_double4(0.0, 0.0, 0.0, 0.0);
  double f[3] = {0, 0, 0}, e = 0.0;
  if (valid) {
    // Records are read in batches of kB, issued together: a batch of a
    // neighbour's list is loaded beside its count (bounded by the list
    // capacity, not the count), so each lane waits for two round trips, not
    // one per record.  Only the arithmetic is limited to the live entries.
    constexpr int kB = 4;
    const int ci = sw_cnt[i];
    const double4* li = sw_nb + 2 * (size_t)i * kcap;
    for (int a = g; a < ci; a += G) {
      const double4 ra = li[2 * a], sa = li[2 * a + 1];
      const double u[3] = {ra.x, ra.y, ra.z};
      const int m = (int)sa.z;  // neighbour a's real atom (a periodic image reads its source's list)
      const double4* lm = sw_nb + 2 * (size_t)m * kcap;
      const double v[3] = {-ra.x, -ra.y, -ra.z};  // x_i - x_m
      double4 rk[kB], sk[kB];
#pragma unroll
      for (int q = 0; q < kB; ++q)
        if (q < kcap) {
          rk[q] = lm[2 * q];
          sk[q] = lm[2 * q + 1];
        }
      const int cm = sw_cnt[m];
      // triplets centred at i: (a, c) with c > a
      for (int c0 = a + 1; c0 < ci; c0 += kB) {
        double4 rc[kB], sc[kB];
#pragma unroll
        for (int q = 0; q < kB; ++q)
          if (c0 + q < ci) {
            rc[q] = li[2 * (c0 + q)];
            sc[q] = li[2 * (c0 + q) + 1];
          }
#pragma unroll
        for (int q = 0; q < kB; ++q)
          if (c0 + q < ci) {
            const double w[3] = {rc[q].x, rc[q].y, rc[q].z};
            e += sw_triplet<true>(pot, u, ra.w, sa.x, sa.y, w, rc[q].w, sc[q].x, sc[q].y, f);
          }
      }
      // triplets centred at m with i as one end
      for (int k0 = 0; k0 < cm; k0 += kB) {
        if (k0 > 0) {
#pragma unroll
          for (int q = 0; q < kB; ++q)
            if (k0 + q < cm) {
              rk[q] = lm[2 * (k0 + q)];
              sk[q] = lm[2 * (k0 + q) + 1];
            }
        }
#pragma unroll
        for (int q = 0; q < kB; ++q)
          if (k0 + q < cm && (int)sk[q].z != i) {
            const double w[3] = {rk[q].x, rk[q].y, rk[q].z};
            sw_triplet<false>(pot, v, ra.w, sa.x, sa.y, w, rk[q].w, sk[q].x, sk[q].y, f);
          }
      }
    }
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) {
    f[0] += __shfl_xor(f[0], o, 64);
    f[1] += __shfl_xor(f[1], o, 64);
    f[2] += __shfl_xor(f[2], o, 64);
    e += __shfl_xor(e, o, 64);
  }
  if (lead) {
    f[0] += fe.x;
    f[1] += fe.y;
    f[2] += fe.z;
    e += fe.w;
  }
  force_epilogue(i, lead, f[0], f[1], f[2], e, ep, frc, vel, ncap, part, 0.0, b, ctrl, trace, pr);
}

// ------------------------------------------------------- Hessian * u (FP64)

// Gupta HVP prologue: rho_i, F'_i, F''_i and s_i = sum_j rho'(r) dh.(u_i - u_j).
// Per-atom vectors are indexed by real slot (real_of maps ghosts to sources).
__global__ __launch_bounds__(kBlock) void k_gupta_hvp_pre(const double4* __restrict__ pos,
                                                          const int* __restrict__ nbr, const int* __restrict__ wcnt,
                                                          const int* __restrict__ real_of, int n, int kcap, int ncap,
                                                          PotDev pot, const double* __restrict__ u,
                                                          double* __restrict__ aux) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double4 pi = pos[i];
  const double ui[3] = {u[i], u[ncap + i], u[2 * ncap + i]};
  double rho = 0.0, s = 0.0;
  for_neighbour_index(nbr, wcnt, kcap, i, [&](int j) {
    const double4 pj = pos[j];
    const double dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 < pot.rc2) {
      j = real_of[j];
      const double r = sqrt(r2), ir = 1.0 / r;
      const double t = fmin(fmax((r - pot.r_in) * pot.inv_w, 0.0), 1.0);
      const double S = (1 - t) * (1 - t) * (1 + 2 * t), dS = -6.0 * t * (1 - t) * pot.inv_w;
      const double rh = exp(-pot.qr0 * (r - pot.r0));
      rho += rh * S;
      const double drh = rh * (dS - pot.qr0 * S);
      const double w = (dx * (ui[0] - u[j]) + dy * (ui[1] - u[ncap + j]) + dz * (ui[2] - u[2 * ncap + j])) * ir;
      s += drh * w;
    }
  });
  double f1 = 0.0, f2 = 0.0;
  if (rho > 0.0) {
    const double sq = sqrt(rho);
    f1 = -0.5 * pot.xi / sq;
    f2 = 0.25 * pot.xi / (rho * sq);
  }
  aux[i] = f1;
  aux[ncap + i] = f2;
  aux[2 * ncap + i] = s;
}

// Hu_i = sum_j [B(g1, g2) w + (F''_i s_i + F''_j s_j) rho' dh], w = u_i - u_j,
// with B(g1, g2) w = g2 (dh.w) dh + (g1 / r)(w - (dh.w) dh).
__global__ __launch_bounds__(kBlock) void k_hvp(const double4* __restrict__ pos, const int* __restrict__ nbr,
                                                const int* __restrict__ wcnt, const int* __restrict__ real_of, int n,
                                                int kcap, int ncap, PotDev pot, const double* __restrict__ u,
                                                const double* __restrict__ aux, double* __restrict__ hu) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double ui[3] = {u[i], u[ncap + i], u[2 * ncap + i]};
  if (pot.kind == FIRE_POT_HARMONIC) {
    for (int d = 0; d < 3; ++d) hu[d * ncap + i] = pot.k[d] * ui[d];
    return;
  }
  const double4 pi = pos[i];
  double acc[3] = {0, 0, 0};
  const bool gupta = pot.kind == FIRE_POT_GUPTA;
  const double f1i = gupta ? aux[i] : 0.0, f2i = gupta ? aux[ncap + i] : 0.0, si = gupta ? aux[2 * ncap + i] : 0.0;
  for_neighbour_index(nbr, wcnt, kcap, i, [&](int j) {
    const double4 pj = pos[j];
    const double d[3] = {pi.x - pj.x, pi.y - pj.y, pi.z - pj.z};
    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (!(r2 < pot.rc2)) return;
    j = real_of[j];
    const double r = sqrt(r2), ir = 1.0 / r;
    const double w[3] = {ui[0] - u[j], ui[1] - u[ncap + j], ui[2] - u[2 * ncap + j]};
    const double dw = (d[0] * w[0] + d[1] * w[1] + d[2] * w[2]) * ir;  // dh.w
    double g1, g2, extra = 0.0;
    if (!gupta) {
      const double s2 = pot.sig2 / r2, s6 = s2 * s2 * s2, s12 = s6 * s6;
      g1 = 4.0 * pot.eps * (-12.0 * s12 + 6.0 * s6) * ir;
      g2 = 4.0 * pot.eps * (156.0 * s12 - 42.0 * s6) / r2;
    } else {
      const double t = fmin(fmax((r - pot.r_in) * pot.inv_w, 0.0), 1.0);
      const bool in_taper = t > 0.0 && t < 1.0;
      const double S = (1 - t) * (1 - t) * (1 + 2 * t), dS = -6.0 * t * (1 - t) * pot.inv_w;
      const double d2S = in_taper ? -6.0 * (1 - 2 * t) * pot.inv_w * pot.inv_w : 0.0;
      const double ph = pot.A * exp(-pot.pr0 * (r - pot.r0)), rh = exp(-pot.qr0 * (r - pot.r0));
      const double dph = ph * (dS - pot.pr0 * S), d2ph = ph * (pot.pr0 * pot.pr0 * S - 2.0 * pot.pr0 * dS + d2S);
      const double drh = rh * (dS - pot.qr0 * S), d2rh = rh * (pot.qr0 * pot.qr0 * S - 2.0 * pot.qr0 * dS + d2S);
      const double f1 = f1i + aux[j];
      g1 = pot.cpair * dph + f1 * drh;
      g2 = pot.cpair * d2ph + f1 * d2rh;
      extra = (f2i * si + aux[ncap + j] * aux[2 * ncap + j]) * drh;
    }
    for (int q = 0; q < 3; ++q) {
      const double dh = d[q] * ir;
      acc[q] += g2 * dw * dh + g1 * ir * (w[q] - dw * dh) + extra * dh;
    }
  });
  hu[i] = acc[0];
  hu[ncap + i] = acc[1];
  hu[2 * ncap + i] = acc[2];
}

// ------------------------------------------------ vector kernels (Lanczos)

// Per-block partial dot products of two 3-plane vectors (fixed order).
__global__ __launch_bounds__(kBlock) void k_dot(const double* __restrict__ a, const double* __restrict__ b, int n,
                                                int ncap, double* __restrict__ part) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double r[1] = {0.0};
  if (i < n) r[0] = a[i] * b[i] + a[ncap + i] * b[ncap + i] + a[2 * ncap + i] * b[2 * ncap + i];
  block_reduce<1, 0>(r);
  if (threadIdx.x == 0) part[blockIdx.x] = r[0];
}

// Sum of per-block partials into out[slot] (one block, fixed order).
__global__ __launch_bounds__(kBlock) void k_sum_parts(const double* __restrict__ part, int m, double* __restrict__ out) {
  double r[1] = {0.0};
  for (int q = threadIdx.x; q < m; q += blockDim.x) r[0] += part[q];
  block_reduce<1, 0>(r);
  if (threadIdx.x == 0) *out = r[0];
}

// y = a * y + b * x (3 planes), coefficients read from device scalars
// (ca, cb may be NULL -> 1) times host factors.
__global__ __launch_bounds__(kBlock) void k_axpby(double* __restrict__ y, const double* __restrict__ x, int n,
                                                  int ncap, double fa, double fb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int d = 0; d < 3; ++d) y[d * ncap + i] = fa * y[d * ncap + i] + fb * x[d * ncap + i];
}

// Per-block partial sums of each plane (for removing the mean translation).
__global__ __launch_bounds__(kBlock) void k_plane_sums(const double* __restrict__ a, int n, int ncap,
                                                       double* __restrict__ part) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double r[3] = {0, 0, 0};
  if (i < n) {
    r[0] = a[i];
    r[1] = a[ncap + i];
    r[2] = a[2 * ncap + i];
  }
  block_reduce<3, 0>(r);
  if (threadIdx.x == 0)
    for (int d = 0; d < 3; ++d) part[3 * blockIdx.x + d] = r[d];
}

__global__ __launch_bounds__(kBlock) void k_sub_plane(double* __restrict__ a, int n, int ncap, double mx, double my,
                                                      double mz) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  a[i] -= mx;
  a[ncap + i] -= my;
  a[2 * ncap + i] -= mz;
}

}  // namespace fire

// =================================================================== host

using namespace fire;

namespace {

const char* hip_err_str(hipError_t e) { return hipGetErrorString(e); }

template <typename T>
hipError_t dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc((void**)p, count * sizeof(T));
}

inline int nblocks(long long n, int b = kBlock) { return (int)((n + b - 1) / b); }

}  // namespace

struct fire_ctx {
  int device = 0;
  hipStream_t stream = nullptr;      // default work stream
  hipStream_t cap_stream = nullptr;  // graph capture stream
  fire_params params{};
  std::string err;

  // ---- single-system workspace
  int n = 0, ncap = 0;        // real atoms and capacity (multiple of the block size)
  int ng = 0, tcap = 0;       // ghosts; slot capacity (real + ghost + padding slot tcap - 1)
  // slots; pos2 / vel2 / frc2 are the permutation scratch of a rebuild and,
  // between rebuilds, the second state set of the loop that folds the update
  // into the next pass (ctrl->cur says which set is current)
  double4 *pos = nullptr, *pos2 = nullptr;
  float4* posf = nullptr;  // FP32 copy of the slot positions for the neighbour search
  double *vel = nullptr, *vel2 = nullptr, *frc = nullptr, *frc2 = nullptr;
  int *id = nullptr, *id2 = nullptr, *cell_of = nullptr, *order = nullptr;
  long long* key = nullptr;                  // in-cell ordering key per slot
  int *gcount = nullptr, *goff = nullptr;    // ghosts per real atom (pre-sort) and offsets
  int *gsrc = nullptr, *gcode = nullptr, *gsrc2 = nullptr, *gcode2 = nullptr;  // per ghost
  int *gcnt = nullptr, *glist = nullptr;     // ghosts of each real slot (at most 7)
  int *new_of_old = nullptr, *real_of = nullptr;
  double* stage = nullptr;  // AoS staging [ncap][3]
  int ccap = 0;
  int *cell_count = nullptr, *cell_start = nullptr, *cell_cursor = nullptr;
  int kcap = 0;
  int *nbr = nullptr, *wcnt = nullptr;  // list [wave][k][lane], padded length per wave
  double4* xref = nullptr;                // positions at the last list build
  int* bucket = nullptr;                  // cell-bucketed slots before ranking
  int* srank = nullptr;                   // cell rank of each slot
  int *cell_rank = nullptr, *rank_cell = nullptr;  // linear cell <-> rank along the Hilbert curve
  int rank_dims[3] = {0, 0, 0}, rank_per = -1;
  // LDS-staged tiles
  int* tile_h = nullptr;
  int* hslot = nullptr;
  int* hsrc = nullptr;
  unsigned short* nbr16 = nullptr;
  int hcap = 0;
  bool use_lds = false;
  size_t lds_atoms = 0, lds_limit = 0;  // halo capacity per tile block; byte limit per block
  bool lds_default = true;              // no explicit limit: the LJ pass's 512-atom tiles get kLdsLj
  size_t lds_cap = 0;                   // the device's LDS per block, less a margin for static LDS
  int ncu = 256;                        // compute units of the device
  size_t lds_boost = 0;                 // default reservation raised for halos that outgrew it (per call)
  int tile = kBlock;                    // atoms per tile of the current lists' halos
  double *part = nullptr, *part_emb = nullptr, *bbox_part = nullptr;
  // per-atom properties of the running minimisation: 1/m and freeze bits in
  // caller order (minv_atom, fmask_atom) and in slot order (sinv, fmask),
  // regathered after every rebuild; used only while with_mass / with_frozen
  double *minv_atom = nullptr, *sinv = nullptr;
  unsigned char *fmask_atom = nullptr, *fmask = nullptr;
  bool with_mass = false, with_frozen = false;
  // Stillinger-Weber short lists: kcap records of 2 double4 per real slot,
  // their counts, and each atom's pair force and energy
  double4 *sw_nb = nullptr, *sw_fe = nullptr;
  int* sw_cnt = nullptr;
  size_t sw_cap = 0;
  double* aux = nullptr;  // HVP / Lanczos planes
  int aux_planes = 0;
  Ctrl* ctrl = nullptr;
  int* flags = nullptr;       // device: [0] error bits, [1] max neighbour count
  int* scan_part = nullptr;   // chunk totals of the prefix sums
  int scan_cap = 0;
  int* h_flags = nullptr;     // pinned; [4]: the ghost count read with the list flags
  bool ghosts_known = false;  // a build finished: ng holds its ghost count
  Ctrl* h_ctrl = nullptr;     // pinned
  unsigned long long* h_poll = nullptr;  // pinned, coherent: status | pause << 32, written by k_poll
  unsigned long long* d_poll = nullptr;  // its device address
  double* h_zero = nullptr;   // pinned scalar for small uploads
  double* trace = nullptr;
  long long trace_cap = 0;
  hipEvent_t ev[2] = {nullptr, nullptr};

  // current system description
  BoxDev box{};
  PotDev pot{};
  Grid grid{};
  double rcs = 0.0, skin = 0.0;
  bool have_list = false;
  // speed-only choices of the single-system path (see tune_single)
  bool list_classes = false;
  int eam_layout = -1;  // EAM-form tiles: -1 by size; 0: 256 atoms, three blocks per CU; 1: 256, two; 2: 512 atoms
  bool tune_loaded = false;
  std::map<std::string, int> tuned;
  std::string tuning_info = "none";

  // captured iteration graphs: [precision]
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  int graph_k = 0;
  long long graph_key[2] = {-1, -1};
  long long layout_version = 0;

  // batched workspace and the no-allocation set-up are owned by batched.hip
  void* batched = nullptr;
  void* noalloc = nullptr;
};

extern "C" void fire_batched_release(void* ws);
extern "C" __attribute__((visibility("hidden"))) int fire_noalloc_init(int device, void** slot);
extern "C" __attribute__((visibility("hidden"))) void fire_noalloc_release(void* p);
extern "C" __attribute__((visibility("hidden"))) int fire_batched_run_noalloc(
    fire_ctx* ctx, void* slot, int nsys, const long long* offsets, double* d_pos, const fire_box* boxes,
    const fire_potential* pot, const fire_params* per_sys, double tol, long long max_steps, fire_result* out,
    hipStream_t s);
extern "C" __attribute__((visibility("hidden"))) int fire_batched_run(fire_ctx* ctx, int nsys, const long long* offsets, double* pos, bool host,
                                const fire_box* boxes, const fire_potential* pot, const fire_params* per_sys,
                                double tol, long long max_steps, fire_result* out, hipStream_t s);

namespace {

int set_err(fire_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(call)                                                                               \
  do {                                                                                             \
    hipError_t e_ = (call);                                                                        \
    if (e_ != hipSuccess)                                                                          \
      return set_err(ctx, e_ == hipErrorOutOfMemory ? FIRE_E_OOM : FIRE_E_DEVICE,                 \
                     std::string(#call) + ": " + hip_err_str(e_));                                 \
  } while (0)

void free_slots(fire_ctx* c) {
  hipFree(c->pos); hipFree(c->pos2); hipFree(c->cell_of); hipFree(c->order); hipFree(c->bucket);
  hipFree(c->srank); hipFree(c->key); hipFree(c->real_of); hipFree(c->gsrc); hipFree(c->gcode);
  hipFree(c->gsrc2); hipFree(c->gcode2); hipFree(c->posf);
  c->pos = c->pos2 = nullptr;
  c->posf = nullptr;
  c->cell_of = c->order = c->bucket = c->srank = c->real_of = nullptr;
  c->gsrc = c->gcode = c->gsrc2 = c->gcode2 = nullptr;
  c->key = nullptr;
  c->tcap = 0;
}

void free_single(fire_ctx* c) {
  free_slots(c);
  hipFree(c->vel); hipFree(c->vel2); hipFree(c->frc); hipFree(c->frc2);
  hipFree(c->id); hipFree(c->id2); hipFree(c->stage);
  hipFree(c->part); hipFree(c->part_emb); hipFree(c->bbox_part);
  hipFree(c->xref); hipFree(c->wcnt); hipFree(c->tile_h); hipFree(c->hslot); hipFree(c->hsrc); hipFree(c->nbr16);
  hipFree(c->gcount); hipFree(c->goff); hipFree(c->gcnt); hipFree(c->glist); hipFree(c->new_of_old);
  hipFree(c->minv_atom); hipFree(c->sinv); hipFree(c->fmask_atom); hipFree(c->fmask);
  hipFree(c->sw_nb); hipFree(c->sw_fe); hipFree(c->sw_cnt);
  c->sw_nb = c->sw_fe = nullptr;
  c->sw_cnt = nullptr;
  c->sw_cap = 0;
  c->minv_atom = c->sinv = nullptr;
  c->fmask_atom = c->fmask = nullptr;
  c->with_mass = c->with_frozen = false;
  c->vel = c->vel2 = c->frc = c->frc2 = nullptr;
  c->id = c->id2 = nullptr;
  c->stage = c->part = c->part_emb = c->bbox_part = nullptr;
  c->xref = nullptr;
  c->wcnt = c->tile_h = c->hslot = c->hsrc = nullptr;
  c->nbr16 = nullptr;
  c->gcount = c->goff = c->gcnt = c->glist = c->new_of_old = nullptr;
  c->use_lds = false;
  c->ncap = 0;
}

void drop_graphs(fire_ctx* c) {
  for (int p = 0; p < 2; ++p) {
    if (c->gexec[p]) hipGraphExecDestroy(c->gexec[p]);
    c->gexec[p] = nullptr;
    c->graph_key[p] = -1;
  }
}

// Slot arrays (real atoms, their ghosts, and the padding slot tcap - 1).
// The positions of the first `keep` slots survive a reallocation.
int ensure_slots(fire_ctx* ctx, int nt, int keep = 0) {
  if (nt + 1 <= ctx->tcap) return FIRE_OK;
  drop_graphs(ctx);
  const int cap = std::max(nt + 1 + nt / 8, ctx->ncap + 1);
  double4* np = nullptr;
  HIPCHK(dalloc(&np, cap));
  if (keep > 0 && ctx->pos) {
    HIPCHK(hipMemcpyAsync(np, ctx->pos, sizeof(double4) * keep, hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
  }
  free_slots(ctx);
  ctx->pos = np;
  HIPCHK(dalloc(&ctx->pos2, cap));
  HIPCHK(dalloc(&ctx->cell_of, cap));
  HIPCHK(dalloc(&ctx->order, cap));
  HIPCHK(dalloc(&ctx->bucket, cap));
  HIPCHK(dalloc(&ctx->srank, cap));
  HIPCHK(dalloc(&ctx->key, cap));
  HIPCHK(dalloc(&ctx->real_of, cap));
  HIPCHK(dalloc(&ctx->gsrc, cap));
  HIPCHK(dalloc(&ctx->gcode, cap));
  HIPCHK(dalloc(&ctx->gsrc2, cap));
  HIPCHK(dalloc(&ctx->gcode2, cap));
  HIPCHK(dalloc(&ctx->posf, cap));
  ctx->tcap = cap;
  ctx->layout_version++;
  return FIRE_OK;
}

// Real-atom arrays.  Capacity is a multiple of the largest tile, so every
// launch over ceil(n/256) blocks, or ceil(n/512) tiles, stays inside them.
int ensure_atoms(fire_ctx* ctx, int n) {
  if (n <= ctx->ncap) return FIRE_OK;
  drop_graphs(ctx);
  free_single(ctx);
  const int cap = ((std::max(n, 64) + kMaxTile - 1) / kMaxTile) * kMaxTile;
  const int nb = cap / kBlock;
  HIPCHK(dalloc(&ctx->xref, cap));
  HIPCHK(dalloc(&ctx->vel, 3 * (size_t)cap));
  HIPCHK(dalloc(&ctx->vel2, 3 * (size_t)cap));
  HIPCHK(dalloc(&ctx->frc, 3 * (size_t)cap));
  HIPCHK(dalloc(&ctx->frc2, 3 * (size_t)cap));
  HIPCHK(dalloc(&ctx->id, cap));
  HIPCHK(dalloc(&ctx->id2, cap));
  HIPCHK(dalloc(&ctx->gcount, cap));
  HIPCHK(dalloc(&ctx->goff, cap + 1));
  HIPCHK(dalloc(&ctx->gcnt, cap));
  HIPCHK(dalloc(&ctx->glist, 8 * (size_t)cap));
  HIPCHK(dalloc(&ctx->new_of_old, cap));
  HIPCHK(dalloc(&ctx->wcnt, cap / 64));
  HIPCHK(dalloc(&ctx->tile_h, nb));
  HIPCHK(dalloc(&ctx->stage, 3 * (size_t)cap));
  HIPCHK(dalloc(&ctx->part, (size_t)kRed * (cap / kPartAtoms)));
  HIPCHK(dalloc(&ctx->part_emb, nb));
  HIPCHK(dalloc(&ctx->bbox_part, 6 * (size_t)nb));
  HIPCHK(hipMemset(ctx->wcnt, 0, sizeof(int) * (cap / 64)));
  HIPCHK(hipMemset(ctx->gcnt, 0, sizeof(int) * cap));
  ctx->ncap = cap;
  ctx->layout_version++;
  if (ctx->kcap) {  // the neighbour lists are sized by ncap
    hipFree(ctx->nbr);
    ctx->nbr = nullptr;
    ctx->kcap = 0;
  }
  if (ctx->aux_planes) {
    hipFree(ctx->aux);
    ctx->aux = nullptr;
    ctx->aux_planes = 0;
  }
  return ensure_slots(ctx, n + n / 2 + 64);
}

int ensure_aux(fire_ctx* ctx, int planes) {
  if (planes <= ctx->aux_planes) return FIRE_OK;
  hipFree(ctx->aux);
  ctx->aux = nullptr;
  HIPCHK(dalloc(&ctx->aux, (size_t)planes * ctx->ncap));
  ctx->aux_planes = planes;
  return FIRE_OK;
}

int prepare_pot(fire_ctx* ctx, const fire_potential* p, PotDev& d) {
  if (!p) return set_err(ctx, FIRE_E_ARG, "potential is required");
  if (p->kind != FIRE_POT_LJ && p->kind != FIRE_POT_GUPTA && p->kind != FIRE_POT_HARMONIC && p->kind != FIRE_POT_SW)
    return set_err(ctx, FIRE_E_ARG, "unknown potential kind");
  d = PotDev{};
  d.kind = p->kind;
  d.conv = p->convention;
  if (p->kind == FIRE_POT_LJ) {
    if (!(p->rc > 0) || !(p->sigma > 0)) return set_err(ctx, FIRE_E_ARG, "LJ needs rc > 0 and sigma > 0");
    d.rc = p->rc;
    d.eps = p->eps;
    d.sig2 = p->sigma * p->sigma;
    double s6 = std::pow(p->sigma / p->rc, 6.0);
    d.shift = 4.0 * p->eps * (s6 * s6 - s6);
  } else if (p->kind == FIRE_POT_GUPTA) {
    if (!(p->r_out > p->r_in) || !(p->r0 > 0))
      return set_err(ctx, FIRE_E_ARG, "Gupta needs r_out > r_in and r0 > 0");
    if (p->convention != FIRE_GUPTA_RGL && p->convention != FIRE_GUPTA_HALF)
      return set_err(ctx, FIRE_E_ARG, "unknown Gupta convention");
    d.rc = p->r_out;
    d.A = p->A;
    d.pr0 = p->p / p->r0;
    d.qr0 = 2.0 * p->q / p->r0;
    d.xi = p->xi;
    d.r0 = p->r0;
    d.r_in = p->r_in;
    d.inv_w = 1.0 / (p->r_out - p->r_in);
    d.cpair = p->convention == FIRE_GUPTA_RGL ? 2.0 : 1.0;
    d.epair = p->convention == FIRE_GUPTA_RGL ? 1.0 : 0.5;
  } else if (p->kind == FIRE_POT_SW) {
    if (!(p->sigma > 0) || !(p->sw_a > 0) || !std::isfinite(p->sigma * p->sw_a))
      return set_err(ctx, FIRE_E_ARG, "SW needs sigma > 0 and a > 0");
    d.rc = p->sw_a * p->sigma;
    d.sw_s = p->sigma;
    d.sw_as = p->sw_a * p->sigma;
    d.sw_Aeps = p->A * p->eps;
    d.sw_B = p->sw_B;
    d.sw_p = p->p;
    d.sw_q = p->q;
    d.sw_leps = p->sw_lambda * p->eps;
    d.sw_gs = p->sw_gamma * p->sigma;
  } else {
    for (int k = 0; k < 3; ++k) d.k[k] = p->k[k];
  }
  d.rc2 = d.rc * d.rc;
  return FIRE_OK;
}

int prepare_system(fire_ctx* ctx, const fire_box* b, const fire_potential* p) {
  if (!b || !p) return set_err(ctx, FIRE_E_ARG, "box and potential are required");
  int rc = prepare_pot(ctx, p, ctx->pot);
  if (rc) return rc;
  const PotDev& d = ctx->pot;
  BoxDev& bx = ctx->box;
  double skin = ctx->params.skin > 0 ? ctx->params.skin : 0.12 * d.rc;
  for (int k = 0; k < 3; ++k) {
    bx.per[k] = b->periodic[k] ? 1 : 0;
    bx.lo[k] = b->lo[k];
    bx.L[k] = b->len[k];
    bx.invL[k] = b->len[k] > 0 ? 1.0 / b->len[k] : 0.0;
    if (bx.per[k]) {
      if (!(b->len[k] > 0) || !std::isfinite(b->len[k])) return set_err(ctx, FIRE_E_BOX, "periodic length must be > 0");
      if (p->kind != FIRE_POT_HARMONIC) {
        if (!(d.rc < 0.5 * b->len[k]))
          return set_err(ctx, FIRE_E_BOX, "cutoff must be < len/2 on periodic axes (minimum image)");
        skin = std::min(skin, 0.9 * (0.5 * b->len[k] - d.rc));
      }
    }
  }
  if (p->kind == FIRE_POT_HARMONIC) skin = 0.0;
  ctx->skin = skin;
  ctx->rcs = d.rc + skin;
  ctx->lds_boost = 0;
  return FIRE_OK;
}

// Cell grid: edge >= rcs; on periodic axes the box plus one ghost layer on
// each side, on free axes the bounding box of the atoms.  Cells inside the
// box get the first ranks (Hilbert order), the ghost layers the rest, so a
// sort by rank puts real atoms before ghosts.
// start[0..m] = exclusive prefix sum of count[0..m), start[m] = total.
int launch_scan(fire_ctx* ctx, hipStream_t s, const int* count, int m, int* start) {
  const int np = std::max(1, (m + kScanChunk - 1) / kScanChunk);
  if (np + 1 > ctx->scan_cap) {
    hipFree(ctx->scan_part);
    ctx->scan_part = nullptr;
    HIPCHK(dalloc(&ctx->scan_part, (size_t)np + 1));
    ctx->scan_cap = np + 1;
  }
  hipLaunchKernelGGL(k_scan_part, dim3(np), dim3(kScanThreads), 0, s, count, m, ctx->scan_part);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, s, ctx->scan_part, np, start, m);
  hipLaunchKernelGGL(k_scan_apply, dim3(np), dim3(kScanThreads), 0, s, count, m, ctx->scan_part, start);
  return FIRE_OK;
}

int make_grid(fire_ctx* ctx, int n) {
  Grid& g = ctx->grid;
  double bmin[3] = {0, 0, 0}, bmax[3] = {0, 0, 0};
  bool any_free = !(ctx->box.per[0] && ctx->box.per[1] && ctx->box.per[2]);
  if (any_free) {
    int nb = nblocks(n);
    hipLaunchKernelGGL(k_bbox, dim3(nb), dim3(kBlock), 0, ctx->stream, ctx->pos, n, ctx->bbox_part);
    std::vector<double> h(6 * (size_t)nb);
    HIPCHK(hipMemcpyAsync(h.data(), ctx->bbox_part, h.size() * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (int k = 0; k < 3; ++k) {
      bmin[k] = INFINITY;
      bmax[k] = -INFINITY;
    }
    for (int q = 0; q < nb; ++q)
      for (int k = 0; k < 3; ++k) {
        bmin[k] = std::min(bmin[k], h[6 * q + k]);
        bmax[k] = std::max(bmax[k], h[6 * q + 3 + k]);
      }
  }
  const double rcs = ctx->rcs;
  long long ncell = 1;
  int in_lo[3], in_hi[3];
  for (int k = 0; k < 3; ++k) {
    double lo, ext;
    if (ctx->box.per[k]) {
      lo = ctx->box.lo[k];
      ext = ctx->box.L[k];
    } else {
      lo = bmin[k];
      ext = bmax[k] - bmin[k];
    }
    // cell edge strictly above rcs, so rounding at a cell face never
    // separates a pair inside the cutoff by more than one cell
    int nc = rcs > 0 ? (int)std::floor(ext / (rcs * (1.0 + 1e-9))) : 1;
    nc = std::max(1, std::min(nc, 1000));
    // a count just above a power of two (17, 33, 34, ...) leaves the curve's
    // whole cube inside the box with a shell of one or two cells around it,
    // which the curve crosses in thin runs: tiles there are slabs with large
    // halos (the 130,417-atom LJ box at 17 cells: the largest halo 3,939
    // atoms, against 2,474 at 16).  Fewer, larger cells cost up to 1/16 more
    // edge, about 20 % more candidates in the neighbour search.
    int p2 = 1;
    while (2 * p2 <= nc) p2 *= 2;
    if (p2 >= 8 && 16 * nc <= 17 * p2) nc = p2;
    const double inv = ext > 0 ? nc / ext : 0.0;
    if (ctx->box.per[k]) {
      g.n[k] = nc + 2;
      g.lo[k] = lo - ext / nc;
      in_lo[k] = 1;
      in_hi[k] = nc;
    } else {
      g.n[k] = nc;
      g.lo[k] = lo;
      in_lo[k] = 0;
      in_hi[k] = nc - 1;
    }
    g.inv[k] = inv;
    g.in_lo[k] = in_lo[k];
    g.in_hi[k] = in_hi[k];
    ncell *= g.n[k];
  }
  if (ncell > (1LL << 26)) return set_err(ctx, FIRE_E_ARG, "cell grid too large");
  g.ncell = (int)ncell;
  if (g.ncell + 1 > ctx->ccap) {
    hipFree(ctx->cell_count);
    hipFree(ctx->cell_start);
    hipFree(ctx->cell_cursor);
    hipFree(ctx->cell_rank);
    hipFree(ctx->rank_cell);
    int cap = g.ncell + 1;
    HIPCHK(dalloc(&ctx->cell_count, cap));
    HIPCHK(dalloc(&ctx->cell_start, cap));
    HIPCHK(dalloc(&ctx->cell_cursor, cap));
    HIPCHK(dalloc(&ctx->cell_rank, cap));
    HIPCHK(dalloc(&ctx->rank_cell, cap));
    ctx->ccap = cap;
    ctx->rank_dims[0] = 0;
  }
  const int per_code = ctx->box.per[0] | (ctx->box.per[1] << 1) | (ctx->box.per[2] << 2);
  if (ctx->rank_dims[0] != g.n[0] || ctx->rank_dims[1] != g.n[1] || ctx->rank_dims[2] != g.n[2] ||
      ctx->rank_per != per_code) {
    // Cells are ranked along a 3-D Hilbert curve (inside the box first, then
    // the periodic-image layers): consecutive ranks are face neighbours, so
    // every run of 256 or 512 slots -- a tile of the LDS-staged passes --
    // stays compact in space and its halo small.  A Morton order jumps across the
    // box at power-of-two boundaries, and a tile straddling a jump needs a
    // halo for two separate pieces.  The inside cells are indexed from 0, so
    // the largest power-of-two cube of the curve lies wholly inside the box
    // and the curve leaves it less often.  Index by Skilling's transpose
    // method (Programming the Hilbert curve, AIP Conf. Proc. 707, 2004).
    int bits = 1;
    while ((1 << bits) < std::max(g.n[0], std::max(g.n[1], g.n[2]))) ++bits;
    auto hilbert = [bits](const int (&cc)[3]) {
      unsigned x[3] = {(unsigned)cc[0], (unsigned)cc[1], (unsigned)cc[2]};
      const unsigned top = 1u << (bits - 1);
      for (unsigned q = top; q > 1; q >>= 1) {  // undo the excess work of the reflections
        const unsigned p = q - 1;
        for (int i = 0; i < 3; ++i) {
          if (x[i] & q) {
            x[0] ^= p;
          } else {
            const unsigned t = (x[0] ^ x[i]) & p;
            x[0] ^= t;
            x[i] ^= t;
          }
        }
      }
      for (int i = 1; i < 3; ++i) x[i] ^= x[i - 1];  // Gray code
      unsigned t = 0;
      for (unsigned q = top; q > 1; q >>= 1)
        if (x[2] & q) t ^= q - 1;
      for (int i = 0; i < 3; ++i) x[i] ^= t;
      unsigned long long h = 0;  // interleave, most significant level first
      for (int b = bits - 1; b >= 0; --b)
        for (int i = 0; i < 3; ++i) h = (h << 1) | ((x[i] >> b) & 1u);
      return h;
    };
    std::vector<std::pair<unsigned long long, int>> key(g.ncell);
    for (int c = 0; c < g.ncell; ++c) {
      const int cc[3] = {c % g.n[0], (c / g.n[0]) % g.n[1], c / (g.n[0] * g.n[1])};
      bool inside = true;
      for (int k = 0; k < 3; ++k) inside = inside && cc[k] >= in_lo[k] && cc[k] <= in_hi[k];
      int ci[3] = {cc[0], cc[1], cc[2]};
      if (inside)
        for (int k = 0; k < 3; ++k) ci[k] -= in_lo[k];
      key[c] = {(inside ? 0ULL : (1ULL << 40)) | hilbert(ci), c};
    }
    std::sort(key.begin(), key.end());
    std::vector<int> rank(g.ncell), cell(g.ncell);
    for (int r = 0; r < g.ncell; ++r) {
      cell[r] = key[r].second;
      rank[key[r].second] = r;
    }
    HIPCHK(hipMemcpy(ctx->cell_rank, rank.data(), sizeof(int) * g.ncell, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->rank_cell, cell.data(), sizeof(int) * g.ncell, hipMemcpyHostToDevice));
    for (int k = 0; k < 3; ++k) ctx->rank_dims[k] = g.n[k];
    ctx->rank_per = per_code;
  }
  return FIRE_OK;
}

int read_flags(fire_ctx* ctx) {
  HIPCHK(hipMemcpyAsync(ctx->h_flags, ctx->flags, 4 * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return FIRE_OK;
}

// LDS bytes per halo atom of the largest staged pass: x, y, z, plus F'(rho)
// for the EAM force pass.
size_t halo_bytes_per_atom(const fire_ctx* ctx) { return ctx->pot.kind == FIRE_POT_GUPTA ? 32 : 24; }

// Tiles of the LDS-staged passes.  The LJ pass takes 512 atoms per tile: its
// halo grows less than the tile (1.6 against 2 times), so fewer halo atoms
// are staged per atom, and its one pass per evaluation runs 29.1 instead of
// 30.3 us per launch on the 130,417-atom box.  78 KB of LDS per 512-atom
// tile block (LJ halos up to 3,328 atoms, EAM-form ones up to 2,496; the
// 130,417-atom LJ box's largest is 2,670) keeps two blocks, with their static
// LDS, within a CU's 160 KB.
//
// The EAM form has three layouts.  256-atom tiles reserve 52 KB (three
// force-pass blocks per CU) or 56 KB (two; the density pass keeps three);
// 512-atom tiles reserve 78 KB, two blocks per CU, whose force pass is held
// to 128 VGPRs so that both fit (at 129, as compiled without that bound,
// only one did).  Once every CU gets a 512-atom tile, those are fastest:
// they stage fewer halo atoms per atom, and at two blocks per CU the
// 253,440-atom bulk's 495 tiles run in one round where 990 256-atom tiles
// take 1.3 rounds of three per CU (81.1 against 86.7 us per FP64
// evaluation; 2,037,760-atom slab, FP32: 472 against 638 us with two
// 256-atom blocks per CU).  Smaller systems keep 256-atom tiles, which
// spread over more CUs.  That size rule is the default; the single-system
// tuner times all three.
constexpr size_t kLdsLj = 78 * 1024;
constexpr size_t kLdsEamLarge = 56 * 1024;

int eam_layout(const fire_ctx* ctx) {
  return ctx->eam_layout >= 0 ? ctx->eam_layout : ((long long)ctx->n >= (long long)ctx->ncu * kMaxTile ? 2 : 0);
}

int tile_atoms(const fire_ctx* ctx) {
  if (ctx->pot.kind == FIRE_POT_LJ) return kMaxTile;
  if (ctx->pot.kind == FIRE_POT_GUPTA && eam_layout(ctx) == 2) return kMaxTile;
  return kBlock;
}

size_t lds_budget(const fire_ctx* ctx, int tile) {
  if (!ctx->lds_default) return ctx->lds_limit;
  size_t d = ctx->lds_limit;
  if (tile == kMaxTile) d = std::min(kLdsLj, ctx->lds_cap);
  else if (ctx->pot.kind == FIRE_POT_GUPTA && eam_layout(ctx) == 1) d = std::min(kLdsEamLarge, ctx->lds_cap);
  return std::max(d, std::min(ctx->lds_boost, ctx->lds_cap));
}

// Neighbour lists (and, with the LDS budget, tile halos) of the current
// slots; one flag read for both kernels.  Grows the list capacity until every
// list fits.
int build_lists(fire_ctx* ctx) {
  hipStream_t s = ctx->stream;
  const int n = ctx->n, dummy = ctx->tcap - 1;
  const int tile = tile_atoms(ctx), nt = nblocks(n, tile);
  // FP32 distance tests: coordinates relative to the grid origin lie within
  // the grid's extent E, so each is off by at most E 2^-24 and a separation
  // by twice that per axis; widen rcs by the resulting bound (and r^2 by the
  // rounding of its own evaluation) so that no pair within rcs is missed
  double ext = 0.0;
  for (int k = 0; k < 3; ++k)
    if (ctx->grid.inv[k] > 0) ext = std::max(ext, ctx->grid.n[k] / ctx->grid.inv[k]);
  const double widen = 4.0 * std::sqrt(3.0) * ext * std::ldexp(1.0, -24);
  const float rcs2f = (float)((ctx->rcs + widen) * (ctx->rcs + widen) * (1.0 + std::ldexp(1.0, -20)));
  // Order of each list (speed only: every entry is tested against the
  // cutoff at every evaluation).  One class in slot order, or (EAM form, when
  // the tuner picks it) entries closer than the start of the taper at build
  // time, then those within the cutoff, then the rest of the skin, so that
  // the FP64 passes skip the taper in most groups and whole groups beyond
  // the cutoff, at the price of neighbouring lanes reading less related
  // neighbours at each step.
  const bool classes = ctx->pot.kind == FIRE_POT_GUPTA && ctx->list_classes;
  const float split2f = classes ? (float)(ctx->pot.r_in * ctx->pot.r_in) : rcs2f;
  const float cut2f = classes ? (float)ctx->pot.rc2 : rcs2f;
  hipLaunchKernelGGL(k_pos_f32, dim3(nblocks(ctx->tcap)), dim3(kBlock), 0, s, ctx->pos, n, ctx->goff + n,
                     ctx->tcap - 1 - n, ctx->grid, ctx->posf);
  const bool was = ctx->use_lds;
  const size_t limit = lds_budget(ctx, tile);
  // no LDS tiles for the three-body potential (its force pass reads the
  // neighbours' short lists, not their positions)
  const int hcap = ctx->pot.kind == FIRE_POT_SW || ctx->lds_limit == 0
                       ? 0
                       : (int)std::min<size_t>(limit / halo_bytes_per_atom(ctx), 65535);
  for (int attempt = 0; attempt < 6; ++attempt) {
    if (!ctx->nbr16) HIPCHK(dalloc(&ctx->nbr16, (size_t)ctx->kcap * ctx->ncap));
    if (hcap >= 64 && (!ctx->hslot || ctx->hcap != hcap || ctx->tile != tile)) {
      hipFree(ctx->hslot);
      hipFree(ctx->hsrc);
      ctx->hslot = ctx->hsrc = nullptr;
      HIPCHK(dalloc(&ctx->hslot, (size_t)hcap * (ctx->ncap / tile)));
      HIPCHK(dalloc(&ctx->hsrc, (size_t)hcap * (ctx->ncap / tile)));
      ctx->hcap = hcap;
      ctx->tile = tile;
      ctx->layout_version++;
    }
    HIPCHK(hipMemsetAsync(ctx->flags, 0, 4 * sizeof(int), s));
    hipLaunchKernelGGL(k_nbr_build, dim3(ctx->ncap / kBlock), dim3(kBlock), 0, s, ctx->pos, ctx->posf, n, ctx->grid,
                       ctx->cell_rank, ctx->cell_start, rcs2f, split2f, cut2f, ctx->kcap, dummy, ctx->nbr,
                       ctx->wcnt, ctx->flags);
    if (hcap >= 64) {
      if (tile == kMaxTile)
        hipLaunchKernelGGL(k_tile_halo<kMaxTile>, dim3(nt), dim3(kMaxTile), 0, s, ctx->srank, ctx->cell_start,
                           ctx->rank_cell, ctx->cell_rank, n, ctx->grid, ctx->nbr, ctx->wcnt, ctx->kcap, hcap, dummy,
                           ctx->tile_h, ctx->hslot, ctx->hsrc, ctx->real_of, ctx->nbr16, ctx->flags);
      else
        hipLaunchKernelGGL(k_tile_halo<kBlock>, dim3(nt), dim3(kBlock), 0, s, ctx->srank, ctx->cell_start,
                           ctx->rank_cell, ctx->cell_rank, n, ctx->grid, ctx->nbr, ctx->wcnt, ctx->kcap, hcap, dummy,
                           ctx->tile_h, ctx->hslot, ctx->hsrc, ctx->real_of, ctx->nbr16, ctx->flags);
    }
    HIPCHK(hipMemcpyAsync(ctx->h_flags + 4, ctx->goff + n, sizeof(int), hipMemcpyDeviceToHost, s));
    int rc = read_flags(ctx);
    if (rc) return rc;
    if (ctx->h_flags[0] & ERR_OVERLAP) return set_err(ctx, FIRE_E_OVERLAP, "two atoms coincide");
    if (ctx->h_flags[1] <= ctx->kcap) break;
    if (attempt == 5) return set_err(ctx, FIRE_E_OOM, "neighbour lists keep outgrowing their capacity");
    const int kmax = ctx->h_flags[1];
    hipFree(ctx->nbr);
    ctx->nbr = nullptr;
    ctx->kcap = ((kmax + kmax / 8 + 8) + 3) & ~3;
    HIPCHK(dalloc(&ctx->nbr, (size_t)ctx->kcap * ctx->ncap));
    hipFree(ctx->nbr16);
    ctx->nbr16 = nullptr;
    ctx->layout_version++;
  }
  // a tile's halo outgrew the default reservation: reserve room for the
  // largest halo and an eighth more (1 KB steps) while that fits a block's
  // LDS, and build again, instead of falling back to global gathers (fewer
  // tile blocks per CU cost far less).  The reservation only grows, so this
  // ends.
  if (hcap >= 64 && (ctx->h_flags[3] & 4) && ctx->lds_default) {
    const size_t atoms = (size_t)ctx->h_flags[2] + 1;
    const size_t need = ((atoms + atoms / 8) * halo_bytes_per_atom(ctx) + 1023) & ~(size_t)1023;
    if (need > limit && need <= ctx->lds_cap && need > ctx->lds_boost) {
      ctx->lds_boost = need;
      return build_lists(ctx);
    }
  }
  ctx->use_lds = false;
  if (hcap >= 64 && !(ctx->h_flags[3] & 4)) {
    // every tile block reserves the full halo capacity: the captured graphs
    // then survive rebuilds (a reservation sized to the largest halo changed
    // with it and forced a new capture), and three 256-atom (two 512-atom)
    // tile blocks still fit a CU
    const size_t rounded = (size_t)hcap;
    if (getenv("FIRE_DEBUG"))
      fprintf(stderr, "[fire] rebuild: n %d, kcap %d, max halo %d atoms, LDS for %zu atoms per tile block\n", n,
              ctx->kcap, ctx->h_flags[2], rounded);
    if (rounded != ctx->lds_atoms) {
      ctx->lds_atoms = rounded;
      ctx->layout_version++;
    }
    ctx->use_lds = true;
  }
  if (ctx->use_lds != was) ctx->layout_version++;  // captured graphs name the pass variant
  return FIRE_OK;
}

// Sort atoms by cell (stable: by caller index inside a cell), regenerate the
// periodic images and build the neighbour list of the current positions;
// positions on periodic axes are wrapped into the box.  Records the build
// positions for the skin test.
Props props_of(const fire_ctx* ctx) {
  return Props{ctx->with_mass ? ctx->sinv : nullptr, ctx->with_frozen ? ctx->fmask : nullptr};
}

// Slot-order properties after the atoms were (re)sorted.
void gather_props(fire_ctx* ctx, hipStream_t s) {
  if (!ctx->with_mass && !ctx->with_frozen) return;
  hipLaunchKernelGGL(k_props_gather, dim3(nblocks(ctx->n)), dim3(kBlock), 0, s, ctx->n, ctx->id,
                     ctx->with_mass ? ctx->minv_atom : nullptr, ctx->with_frozen ? ctx->fmask_atom : nullptr,
                     ctx->sinv, ctx->fmask);
}

int rebuild(fire_ctx* ctx) {
  const int n = ctx->n;
  hipStream_t s = ctx->stream;
  if (ctx->pot.kind == FIRE_POT_HARMONIC) {  // no pairs, no list
    HIPCHK(hipMemcpyAsync(ctx->xref, ctx->pos, sizeof(double4) * n, hipMemcpyDeviceToDevice, s));
    ctx->ng = 0;
    ctx->have_list = true;
    gather_props(ctx, s);
    return FIRE_OK;
  }
  const int nb = nblocks(n);
  // ---- periodic images.  Their number is counted on the device (goff[n]);
  // the kernels below read it there.  After a first build, while the slot
  // capacity holds the last count and a quarter more, the host launches the
  // whole rebuild without waiting for the count, and checks it with the
  // list flags at the end (a count beyond the capacity: larger arrays and
  // the build again, waiting this time).
  hipLaunchKernelGGL(k_ghost_count, dim3(nb), dim3(kBlock), 0, s, ctx->pos, n, ctx->box, ctx->rcs, ctx->gcount);
  int rc = launch_scan(ctx, s, ctx->gcount, n, ctx->goff);
  if (rc) return rc;
  const bool ahead = ctx->ghosts_known && ctx->tcap - 1 - n >= ctx->ng + std::max(ctx->ng / 4, 256);
  int ng_est = ctx->ng;  // the count, or (launching ahead) the last one
  if (!ahead) {
    HIPCHK(hipMemcpyAsync(ctx->h_flags, ctx->goff + n, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    ng_est = ctx->h_flags[0];
    rc = ensure_slots(ctx, n + ng_est, n);
    if (rc) return rc;
  }
  const int gmax = ctx->tcap - 1 - n;  // ghost slots before the dummy slot
  const int* gtot = ctx->goff + n;
  hipLaunchKernelGGL(k_ghost_fill, dim3(nb), dim3(kBlock), 0, s, ctx->pos, n, ctx->box, ctx->rcs, ctx->goff,
                     ctx->gsrc, ctx->gcode, gmax);
  // ---- cell sort of all slots
  rc = make_grid(ctx, n);
  if (rc) return rc;
  const Grid& g = ctx->grid;
  HIPCHK(hipMemsetAsync(ctx->cell_count, 0, sizeof(int) * (g.ncell + 1), s));
  HIPCHK(hipMemsetAsync(ctx->cell_cursor, 0, sizeof(int) * (g.ncell + 1), s));
  HIPCHK(hipMemsetAsync(ctx->gcnt, 0, sizeof(int) * ctx->ncap, s));
  const int nbt = nblocks(ctx->tcap);
  hipLaunchKernelGGL(k_cell_count, dim3(nbt), dim3(kBlock), 0, s, ctx->pos, n, gtot, gmax, g, ctx->cell_rank,
                     ctx->id, ctx->gsrc, ctx->gcode, ctx->cell_of, ctx->key, ctx->cell_count);
  rc = launch_scan(ctx, s, ctx->cell_count, g.ncell, ctx->cell_start);
  if (rc) return rc;
  hipLaunchKernelGGL(k_cell_fill, dim3(nbt), dim3(kBlock), 0, s, ctx->cell_of, n, gtot, gmax, ctx->cell_start,
                     ctx->cell_cursor, ctx->bucket);
  hipLaunchKernelGGL(k_cell_rank, dim3(nbt), dim3(kBlock), 0, s, ctx->cell_of, ctx->cell_start, ctx->bucket, n, gtot,
                     gmax, ctx->key, ctx->order);
  hipLaunchKernelGGL(k_permute, dim3(nbt), dim3(kBlock), 0, s, ctx->order, n, gtot, gmax, ctx->ncap, ctx->pos,
                     ctx->vel, ctx->frc, ctx->id, ctx->cell_of, ctx->gsrc, ctx->gcode, ctx->pos2, ctx->vel2, ctx->frc2,
                     ctx->id2, ctx->srank, ctx->new_of_old, ctx->gsrc2, ctx->gcode2);
  hipLaunchKernelGGL(k_ghost_link, dim3(nblocks(std::max(n, gmax))), dim3(kBlock), 0, s, n, gtot, gmax,
                     ctx->new_of_old, ctx->gsrc2, ctx->real_of, ctx->gcnt, ctx->glist);
  // copy back (not swap): captured graphs hold these buffers' addresses
  hipLaunchKernelGGL(k_commit, dim3(nbt), dim3(kBlock), 0, s, n, gtot, gmax, ctx->ncap, ctx->pos2, ctx->gsrc2,
                     ctx->gcode2, ctx->id2, ctx->vel2, ctx->frc2, ctx->pos, ctx->gsrc, ctx->gcode, ctx->id, ctx->vel,
                     ctx->frc, ctx->xref);
  const int dummy = ctx->tcap - 1;
  hipLaunchKernelGGL(k_set_pos, dim3(1), dim3(64), 0, s, ctx->pos, dummy, kFar);
  // ---- neighbour lists
  const double rcs2 = ctx->rcs * ctx->rcs;
  if (ctx->kcap == 0) {
    // first guess from the mean density; a larger count triggers one more pass
    double vol = 1.0;
    for (int k = 0; k < 3; ++k) vol *= (ctx->box.per[k] ? g.n[k] - 2 : g.n[k]) / std::max(g.inv[k], 1e-300);
    const double dens = n / std::max(vol, 1e-300);
    const int guess = (int)(1.4 * dens * 4.18879 * rcs2 * ctx->rcs) + 16;
    ctx->kcap = std::min((guess + 3) & ~3, std::max(4, ((n + ng_est + 3) & ~3)));
    HIPCHK(dalloc(&ctx->nbr, (size_t)ctx->kcap * ctx->ncap));
    ctx->layout_version++;
  }
  rc = build_lists(ctx);
  if (ahead && (rc || ctx->h_flags[4] > gmax)) {
    // more ghosts than the slots held (or a failure that might follow from
    // that): the build again, waiting for the count
    if (getenv("FIRE_DEBUG"))
      fprintf(stderr, "[fire] rebuild: %d ghosts beyond the %d ghost slots of a build launched ahead; again\n",
              ctx->h_flags[4], gmax);
    ctx->ghosts_known = false;
    return rebuild(ctx);
  }
  if (rc) return rc;
  ctx->ng = ctx->h_flags[4];
  ctx->ghosts_known = true;
  if (ctx->pot.kind == FIRE_POT_SW) {
    const size_t need = (size_t)ctx->kcap * ctx->ncap;
    if (need > ctx->sw_cap) {
      hipFree(ctx->sw_nb);
      hipFree(ctx->sw_fe);
      hipFree(ctx->sw_cnt);
      ctx->sw_nb = ctx->sw_fe = nullptr;
      ctx->sw_cnt = nullptr;
      ctx->sw_cap = 0;
      HIPCHK(dalloc(&ctx->sw_nb, 2 * need));
      HIPCHK(dalloc(&ctx->sw_fe, (size_t)ctx->ncap));
      HIPCHK(dalloc(&ctx->sw_cnt, (size_t)ctx->ncap));
      ctx->sw_cap = need;
      ctx->layout_version++;
    }
  }
  ctx->have_list = true;
  gather_props(ctx, s);
  return FIRE_OK;
}

StateBuf state_set(fire_ctx* ctx, int k) {
  return k ? StateBuf{ctx->pos2, ctx->vel2, ctx->frc2} : StateBuf{ctx->pos, ctx->vel, ctx->frc};
}

UpdArgs upd_args(fire_ctx* ctx, int parity) {
  UpdArgs u;
  u.src = state_set(ctx, parity);
  u.dst = state_set(ctx, parity ^ 1);
  u.dst_index = parity ^ 1;
  u.real_of = ctx->real_of;
  u.gcode = ctx->gcode;
  u.gcnt = ctx->gcnt;
  u.glist = ctx->glist;
  u.xref = ctx->xref;
  u.sinv = props_of(ctx).sinv;
  u.box = ctx->box;
  return u;
}

// The passes of one force evaluation.  parity < 0: on the primary state set;
// parity 0 / 1: the first pass also applies the pending update, reading set
// `parity` and writing the other (LDS-staged passes only).
template <typename T, bool LDS, bool WE>
void launch_pair_passes(fire_ctx* ctx, hipStream_t s, int parity) {
  // the pair passes run on their tiles' blocks also with global gathers, so
  // both forms reduce over the same atom groups and give the same bits
  const int tile = tile_atoms(ctx);
  const int n = ctx->n, nt = nblocks(n, tile), kc = ctx->kcap, nc = ctx->ncap;
  const PotDev& P = ctx->pot;
  const Tiles tl{ctx->tile_h, ctx->hslot, ctx->hsrc, ctx->nbr16, ctx->hcap};
  const size_t sm = LDS ? ctx->lds_atoms * 24 : 0;     // x, y, z
  const size_t smw = LDS ? ctx->lds_atoms * 32 : 0;    // x, y, z, F'(rho)
  const UpdArgs ua = upd_args(ctx, parity < 0 ? 0 : parity);
  const Props pr = props_of(ctx);
  if constexpr (LDS) {
    if (parity >= 0) {
      const StateBuf d = ua.dst;
      if (P.kind == FIRE_POT_LJ) {
        if (nt > ctx->ncu)
          hipLaunchKernelGGL((k_lj_force_two_per_cu<T, true, WE, true>), dim3(nt), dim3(tile), sm, s, ua.src.pos, ctx->nbr,
                             tl, ctx->wcnt, n, kc, nc, P, d.frc, d.vel, ctx->part, ctx->ctrl, ctx->trace, ua, pr);
        else
          hipLaunchKernelGGL((k_lj_force<T, true, WE, true>), dim3(nt), dim3(tile), sm, s, ua.src.pos, ctx->nbr, tl,
                             ctx->wcnt, n, kc, nc, P, d.frc, d.vel, ctx->part, ctx->ctrl, ctx->trace, ua, pr);
      } else if (tile == kMaxTile) {
        hipLaunchKernelGGL((k_gupta_density<T, true, true, kMaxTile>), dim3(nt), dim3(tile), sm, s, ua.src.pos,
                           ctx->nbr, tl, ctx->wcnt, n, kc, nc, P, ctx->gcnt, ctx->glist, ctx->part_emb, ctx->ctrl, ua);
        hipLaunchKernelGGL((k_gupta_force<T, true, WE, kMaxTile>), dim3(nt), dim3(tile), smw, s, d.pos, ctx->nbr, tl,
                           ctx->wcnt, n, kc, nc, P, d.frc, d.vel, ctx->part, ctx->part_emb, ctx->ctrl, ctx->trace,
                           pr);
      } else {
        hipLaunchKernelGGL((k_gupta_density<T, true, true>), dim3(nt), dim3(tile), sm, s, ua.src.pos, ctx->nbr,
                           tl, ctx->wcnt, n, kc, nc, P, ctx->gcnt, ctx->glist, ctx->part_emb, ctx->ctrl, ua);
        hipLaunchKernelGGL((k_gupta_force<T, true, WE>), dim3(nt), dim3(tile), smw, s, d.pos, ctx->nbr, tl,
                           ctx->wcnt, n, kc, nc, P, d.frc, d.vel, ctx->part, ctx->part_emb, ctx->ctrl, ctx->trace,
                           pr);
      }
      return;
    }
  }
  if (P.kind == FIRE_POT_LJ) {
    bool two_per_cu = false;
    if constexpr (LDS) two_per_cu = nt > ctx->ncu;
    if (two_per_cu)
      hipLaunchKernelGGL((k_lj_force_two_per_cu<T, true, WE>), dim3(nt), dim3(tile), sm, s, ctx->pos, ctx->nbr, tl,
                         ctx->wcnt, n, kc, nc, P, ctx->frc, ctx->vel, ctx->part, ctx->ctrl, ctx->trace, ua, pr);
    else
      hipLaunchKernelGGL((k_lj_force<T, LDS, WE>), dim3(nt), dim3(tile), sm, s, ctx->pos, ctx->nbr, tl, ctx->wcnt, n,
                         kc, nc, P, ctx->frc, ctx->vel, ctx->part, ctx->ctrl, ctx->trace, ua, pr);
  } else if (tile == kMaxTile) {
    hipLaunchKernelGGL((k_gupta_density<T, LDS, false, kMaxTile>), dim3(nt), dim3(tile), sm, s, ctx->pos, ctx->nbr,
                       tl, ctx->wcnt, n, kc, nc, P, ctx->gcnt, ctx->glist, ctx->part_emb, ctx->ctrl, ua);
    hipLaunchKernelGGL((k_gupta_force<T, LDS, WE, kMaxTile>), dim3(nt), dim3(tile), smw, s, ctx->pos, ctx->nbr, tl,
                       ctx->wcnt, n, kc, nc, P, ctx->frc, ctx->vel, ctx->part, ctx->part_emb, ctx->ctrl,
                       ctx->trace, pr);
  } else {
    hipLaunchKernelGGL((k_gupta_density<T, LDS>), dim3(nt), dim3(tile), sm, s, ctx->pos, ctx->nbr, tl,
                       ctx->wcnt, n, kc, nc, P, ctx->gcnt, ctx->glist, ctx->part_emb, ctx->ctrl, ua);
    hipLaunchKernelGGL((k_gupta_force<T, LDS, WE>), dim3(nt), dim3(tile), smw, s, ctx->pos, ctx->nbr, tl,
                       ctx->wcnt, n, kc, nc, P, ctx->frc, ctx->vel, ctx->part, ctx->part_emb, ctx->ctrl,
                       ctx->trace, pr);
  }
}

// Lanes per atom of the two Stillinger-Weber passes (the force pass's grid,
// n / (kBlock / kSwForceLanes) blocks, must fit the partial records).
constexpr int kSwShortLanes = 8, kSwForceLanes = 4;
static_assert(kBlock / kSwForceLanes >= kPartAtoms, "partial records are sized for this grid");

void launch_sw(fire_ctx* ctx, hipStream_t s) {
  const int n = ctx->n;
  hipLaunchKernelGGL(k_sw_short<kSwShortLanes>, dim3(nblocks(n, kBlock / kSwShortLanes)), dim3(kBlock), 0, s,
                     ctx->pos, ctx->nbr, ctx->wcnt, ctx->real_of, n, ctx->kcap, ctx->pot, ctx->sw_nb, ctx->sw_cnt,
                     ctx->sw_fe, ctx->ctrl);
  hipLaunchKernelGGL(k_sw_force<kSwForceLanes>, dim3(nblocks(n, kBlock / kSwForceLanes)), dim3(kBlock), 0, s,
                     ctx->sw_nb, ctx->sw_cnt, ctx->sw_fe, n, ctx->kcap, ctx->ncap, ctx->pot, ctx->frc,
                     ctx->vel, ctx->part, ctx->ctrl, ctx->trace, props_of(ctx));
}

template <bool WE>
void launch_pairs(fire_ctx* ctx, hipStream_t s, int prec, int parity) {
  if (ctx->pot.kind == FIRE_POT_SW) {  // FP64, global gathers, energy always summed
    launch_sw(ctx, s);
    return;
  }
  if (ctx->use_lds) {
    if (prec) launch_pair_passes<float, true, WE>(ctx, s, parity);
    else launch_pair_passes<double, true, WE>(ctx, s, parity);
  } else {
    if (prec) launch_pair_passes<float, false, WE>(ctx, s, -1);
    else launch_pair_passes<double, false, WE>(ctx, s, -1);
  }
}

// One force evaluation (passes + fused reductions and control) enqueued on
// stream s.  prec: 0 FP64 pair terms, 1 FP32.  with_e: also accumulate the
// energy (the FIRE steps themselves only need forces and P).
void launch_forces(fire_ctx* ctx, hipStream_t s, int prec, bool with_e = true) {
  if (ctx->pot.kind == FIRE_POT_HARMONIC) {
    hipLaunchKernelGGL(k_harmonic_force, dim3(nblocks(ctx->n)), dim3(kBlock), 0, s, ctx->pos, ctx->n, ctx->ncap,
                       ctx->pot, ctx->frc, ctx->vel, ctx->part, ctx->ctrl, ctx->trace, props_of(ctx));
    return;
  }
  if (with_e) launch_pairs<true>(ctx, s, prec, -1);
  else launch_pairs<false>(ctx, s, prec, -1);
}

// Whether the loop folds the update into the next pass: LDS-staged passes,
// pair potentials, and no velocity-Verlet half kick in the force epilogue
// (that kick would have to be undone when a rebuild discards the pass).
bool fold_update(const fire_ctx* ctx) {
  return ctx->use_lds && ctx->pot.kind != FIRE_POT_HARMONIC && ctx->params.integrator != FIRE_INT_VERLET &&
         !(ctx->params.dmax > 0);
}

// Primary state set current and its periodic images consistent (see
// k_state_home); no host synchronisation.
void materialize(fire_ctx* ctx, hipStream_t s) {
  const int n = ctx->n;
  hipLaunchKernelGGL(k_state_home, dim3(nblocks(n)), dim3(kBlock), 0, s, n, ctx->ncap, ctx->pos2, ctx->vel2,
                     ctx->frc2, ctx->pos, ctx->vel, ctx->frc, ctx->ctrl);
  hipLaunchKernelGGL(k_ghost_refresh, dim3(nblocks(std::max(ctx->ng, 1))), dim3(kBlock), 0, s, n, ctx->ng, ctx->pos,
                     ctx->real_of, ctx->gcode, ctx->box, ctx->ctrl);
}

void launch_update(fire_ctx* ctx, hipStream_t s) {
  if (ctx->params.dmax > 0) {  // the drift step depends on every atom's new velocity
    hipLaunchKernelGGL(k_update_vel, dim3(nblocks(ctx->n)), dim3(kBlock), 0, s, ctx->pos, ctx->vel, ctx->frc,
                       ctx->n, ctx->ncap, ctx->part, ctx->ctrl, props_of(ctx));
    hipLaunchKernelGGL(k_update_drift, dim3(nblocks(ctx->n)), dim3(kBlock), 0, s, ctx->pos, ctx->vel, ctx->frc,
                       ctx->xref, ctx->gcnt, ctx->glist, ctx->gcode, ctx->box, ctx->n, ctx->ncap, ctx->ctrl,
                       props_of(ctx));
    return;
  }
  hipLaunchKernelGGL(k_update, dim3(nblocks(ctx->n)), dim3(kBlock), 0, s, ctx->pos, ctx->vel, ctx->frc, ctx->xref,
                     ctx->gcnt, ctx->glist, ctx->gcode, ctx->box, ctx->n, ctx->ncap, ctx->ctrl, props_of(ctx));
}

// One FIRE iteration; energies only when a trace is recorded.
// parity: the state set the iteration starts from (iterations alternate).
// Status and pause bits of the loop, written to coherent host memory at the
// end of every graph replay: the host polls the word after the replay's event
// instead of enqueueing a device-to-host copy between replays.
__global__ void k_poll(const Ctrl* __restrict__ ctrl, unsigned long long* __restrict__ poll) {
  if (threadIdx.x == 0) {
    const unsigned st = (unsigned)__hip_atomic_load(&ctrl->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned pa = (unsigned)__hip_atomic_load(&ctrl->pause, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(poll, (unsigned long long)st | ((unsigned long long)pa << 32), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

void launch_iteration(fire_ctx* ctx, hipStream_t s, int prec, int parity) {
  if (fold_update(ctx)) {
    if (ctx->trace) launch_pairs<true>(ctx, s, prec, parity);
    else launch_pairs<false>(ctx, s, prec, parity);
    return;
  }
  launch_update(ctx, s);
  launch_forces(ctx, s, prec, ctx->trace != nullptr);
}

int graph_for(fire_ctx* ctx, int prec, hipGraphExec_t* out) {
  const long long key = (ctx->layout_version * 1000003LL + (long long)ctx->n * 7 + ctx->graph_k) * 4 +
                        (ctx->with_mass ? 1 : 0) + (ctx->with_frozen ? 2 : 0);
  if (ctx->gexec[prec] && ctx->graph_key[prec] == key && ctx->trace == nullptr) {
    *out = ctx->gexec[prec];
    return FIRE_OK;
  }
  if (ctx->gexec[prec]) hipGraphExecDestroy(ctx->gexec[prec]);
  ctx->gexec[prec] = nullptr;
  hipGraph_t g;
  HIPCHK(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeRelaxed));
  for (int k = 0; k < ctx->graph_k; ++k) launch_iteration(ctx, ctx->cap_stream, prec, k & 1);  // graph_k is even
  hipLaunchKernelGGL(k_poll, dim3(1), dim3(64), 0, ctx->cap_stream, ctx->ctrl, ctx->d_poll);
  HIPCHK(hipStreamEndCapture(ctx->cap_stream, &g));
  if (getenv("FIRE_DEBUG")) {  // dynamic LDS of the captured kernel nodes
    size_t nn = 0;
    hipGraphGetNodes(g, nullptr, &nn);
    std::vector<hipGraphNode_t> nodes(nn);
    hipGraphGetNodes(g, nodes.data(), &nn);
    size_t lo = SIZE_MAX, hi = 0, nk = 0;
    for (auto nd : nodes) {
      hipGraphNodeType ty;
      if (hipGraphNodeGetType(nd, &ty) != hipSuccess || ty != hipGraphNodeTypeKernel) continue;
      hipKernelNodeParams kp{};
      if (hipGraphKernelNodeGetParams(nd, &kp) != hipSuccess) continue;
      lo = std::min<size_t>(lo, kp.sharedMemBytes);
      hi = std::max<size_t>(hi, kp.sharedMemBytes);
      ++nk;
    }
    fprintf(stderr, "[fire] graph: %zu kernel nodes, dynamic LDS %zu..%zu B (use_lds %d, halo capacity %zu atoms)\n",
            nk, lo, hi, (int)ctx->use_lds, ctx->lds_atoms);
  }
  hipError_t e = hipGraphInstantiate(&ctx->gexec[prec], g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e != hipSuccess) return set_err(ctx, FIRE_E_DEVICE, std::string("hipGraphInstantiate: ") + hip_err_str(e));
  ctx->graph_key[prec] = ctx->trace ? -1 : key;
  *out = ctx->gexec[prec];
  return FIRE_OK;
}

int stage_in(fire_ctx* ctx, long long n, const double* src, bool host, hipStream_t s) {
  if (n <= 0 || n > (1LL << 30)) return set_err(ctx, FIRE_E_ARG, "n must be in 1 .. 2^30");
  if (!src) return set_err(ctx, FIRE_E_ARG, "positions are NULL");
  int rc = ensure_atoms(ctx, (int)n);
  if (rc) return rc;
  ctx->n = (int)n;
  const double* d = src;
  if (host) {
    for (long long i = 0; i < 3 * n; ++i)
      if (!std::isfinite(src[i])) return set_err(ctx, FIRE_E_NONFINITE, "non-finite input position");
    HIPCHK(hipMemcpyAsync(ctx->stage, src, sizeof(double) * 3 * n, hipMemcpyHostToDevice, s));
    d = ctx->stage;
  }
  HIPCHK(hipMemsetAsync(ctx->flags, 0, 2 * sizeof(int), s));
  hipLaunchKernelGGL(k_stage_in, dim3(nblocks(n)), dim3(kBlock), 0, s, d, (int)n, ctx->ncap, ctx->pos, ctx->vel,
                     ctx->frc, ctx->id, ctx->flags);
  if (!host) {
    rc = read_flags(ctx);
    if (rc) return rc;
    if (ctx->h_flags[0] & ERR_NONFINITE) return set_err(ctx, FIRE_E_NONFINITE, "non-finite input position");
  }
  return FIRE_OK;
}

// Per-atom masses and freeze bits of a minimisation (after stage_in): into
// the caller-order device arrays, validated, and switched on for the run.
// Host arrays are first copied into the slot-order buffers, which the first
// rebuild overwrites.
int setup_props(fire_ctx* ctx, const fire_atoms* a, bool host, hipStream_t s) {
  ctx->with_mass = ctx->with_frozen = false;
  if (!a || (!a->mass && !a->frozen)) return FIRE_OK;
  const int n = ctx->n, cap = ctx->ncap;
  const double* m = a->mass;
  const unsigned char* fz = a->frozen;
  if (m && !ctx->sinv) {
    HIPCHK(dalloc(&ctx->minv_atom, cap));
    HIPCHK(dalloc(&ctx->sinv, cap));
  }
  if (fz && !ctx->fmask) {
    HIPCHK(dalloc(&ctx->fmask_atom, cap));
    HIPCHK(dalloc(&ctx->fmask, cap));
  }
  if (host) {
    if (m) {
      for (int i = 0; i < n; ++i)
        if (!(m[i] > 0.0) || !std::isfinite(m[i])) return set_err(ctx, FIRE_E_ARG, "masses must be positive and finite");
      HIPCHK(hipMemcpyAsync(ctx->sinv, m, sizeof(double) * n, hipMemcpyHostToDevice, s));
      m = ctx->sinv;
    }
    if (fz) {
      HIPCHK(hipMemcpyAsync(ctx->fmask, fz, n, hipMemcpyHostToDevice, s));
      fz = ctx->fmask;
    }
  }
  HIPCHK(hipMemsetAsync(ctx->flags, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_props_in, dim3(nblocks(n)), dim3(kBlock), 0, s, m, fz, n, ctx->minv_atom, ctx->fmask_atom,
                     ctx->flags);
  int rc = read_flags(ctx);
  if (rc) return rc;
  if (ctx->h_flags[0] & kBadMass) return set_err(ctx, FIRE_E_ARG, "masses must be positive and finite");
  ctx->with_mass = m != nullptr;
  ctx->with_frozen = fz != nullptr;
  return FIRE_OK;
}

void ctrl_from_params(const fire_params& p, double tol, long long max_steps, double skin_half2, int natoms,
                      Ctrl& c) {
  memset(&c, 0, sizeof(c));
  c.status = ST_RUNNING;
  c.precision = p.precision == FIRE_FP64 ? 0 : 1;
  c.dt_start = p.dt_start;
  c.dtmax = p.tmax * p.dt_start;
  c.dtmin = p.tmin * p.dt_start;
  c.dtgrow = p.dtgrow;
  c.dtshrink = p.dtshrink;
  c.alpha0 = p.alpha0;
  c.alphashrink = p.alphashrink;
  c.f2a = p.f2a;
  c.tol = tol;
  c.switch_tol = p.mixed_switch > 0 ? p.mixed_switch : 100.0 * tol;
  c.skin_half2 = skin_half2;
  c.max_steps = max_steps;
  c.delaystep = p.delaystep;
  c.vdfmax = p.vdfmax;
  c.halfstepback = p.halfstepback;
  c.initialdelay = p.initialdelay;
  c.integrator = p.integrator;
  c.criterion = p.criterion;
  c.variant = p.variant;
  c.mode = p.precision;
  c.natoms = natoms;
  c.dt = p.dt_start;
  c.alpha = p.alpha0;
}

void ctrl_defaults(fire_ctx* ctx, Ctrl& c, double tol, long long max_steps, int eval_only) {
  const fire_params& p = ctx->params;
  memset(&c, 0, sizeof(c));
  c.status = ST_RUNNING;
  // the three-body path has FP64 terms only
  c.precision = (p.precision == FIRE_FP64 || ctx->pot.kind == FIRE_POT_SW) ? 0 : 1;
  c.dt_start = p.dt_start;
  c.dtmax = p.tmax * p.dt_start;
  c.dtmin = p.tmin * p.dt_start;
  c.dtgrow = p.dtgrow;
  c.dtshrink = p.dtshrink;
  c.alpha0 = p.alpha0;
  c.alphashrink = p.alphashrink;
  c.f2a = p.f2a;
  c.tol = tol;
  c.switch_tol = p.mixed_switch > 0 ? p.mixed_switch : 100.0 * tol;
  c.skin_half2 = ctx->pot.kind == FIRE_POT_HARMONIC ? 1e300 : 0.25 * ctx->skin * ctx->skin;
  c.dmax = p.dmax;
  c.eval_only = eval_only;
  c.max_steps = max_steps;
  c.delaystep = p.delaystep;
  c.vdfmax = p.vdfmax;
  c.halfstepback = p.halfstepback;
  c.initialdelay = p.initialdelay;
  c.integrator = p.integrator;
  c.criterion = p.criterion;
  c.variant = p.variant;
  c.mode = ctx->pot.kind == FIRE_POT_SW ? FIRE_FP64 : p.precision;
  c.natoms = ctx->n;
  c.dt = p.dt_start;
  c.alpha = p.alpha0;
  c.trace_cap = ctx->trace_cap;
}

int check_status_error(fire_ctx* ctx, int st) {
  if (st == FIRE_E_OVERLAP) return set_err(ctx, FIRE_E_OVERLAP, "two atoms coincide");
  if (st == FIRE_E_NONFINITE) return set_err(ctx, FIRE_E_NONFINITE, "non-finite energy or force");
  if (st < 0) return set_err(ctx, st, "device error");
  return FIRE_OK;
}

// Evaluate E and F at the staged positions (list rebuilt); precision per params.
int evaluate(fire_ctx* ctx, hipStream_t s) {
  int rc = rebuild(ctx);
  if (rc) return rc;
  ctrl_defaults(ctx, *ctx->h_ctrl, 0.0, 0, 1);
  HIPCHK(hipMemcpyAsync(ctx->ctrl, ctx->h_ctrl, sizeof(Ctrl), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  launch_forces(ctx, s, ctx->params.precision == FIRE_FP64 ? 0 : 1);
  return FIRE_OK;
}

// Resume the device FIRE loop: status running, no pause, no skin violation.
int resume(fire_ctx* ctx, hipStream_t s) {
  int* up = ctx->h_flags + 4;
  up[0] = ST_RUNNING;
  up[1] = 0;
  *ctx->h_zero = 0.0;
  HIPCHK(hipMemcpyAsync(ctx->ctrl, up, 2 * sizeof(int), hipMemcpyHostToDevice, s));
  // stream order puts the next launches after these copies; the pinned
  // sources hold the same constants on every call, so no wait is needed
  HIPCHK(hipMemcpyAsync(&ctx->ctrl->viol, ctx->h_zero, sizeof(int), hipMemcpyHostToDevice, s));
  return FIRE_OK;
}

// Average time of one force evaluation of the current system and lists, as
// inside the loop (see fire_repeat_forces_dev), in milliseconds.
int time_evaluation(fire_ctx* ctx, hipStream_t s, int prec, int reps, float* ms) {
  ctrl_defaults(ctx, *ctx->h_ctrl, 0.0, 0, 1);
  HIPCHK(hipMemcpyAsync(ctx->ctrl, ctx->h_ctrl, sizeof(Ctrl), hipMemcpyHostToDevice, s));
  auto one = [&]() {
    if (fold_update(ctx)) launch_pairs<false>(ctx, s, prec, 0);
    else launch_forces(ctx, s, prec, false);
  };
  one();
  one();
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, s));
  for (int r = 0; r < reps; ++r) one();
  HIPCHK(hipEventRecord(e1, s));
  HIPCHK(hipEventSynchronize(e1));
  HIPCHK(hipEventElapsedTime(ms, e0, e1));
  *ms /= reps;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (fold_update(ctx))  // the passes wrote the second state set and its index
    hipLaunchKernelGGL(k_ghost_refresh, dim3(1), dim3(kBlock), 0, s, ctx->n, 0, ctx->pos, ctx->real_of, ctx->gcode,
                       ctx->box, ctx->ctrl);
  return FIRE_OK;
}

std::string tune_cache_path() {
  const char* p = getenv("FIRE_TUNE_CACHE");
  if (p && *p) return std::string(p) + ".single";
  const char* h = getenv("HOME");
  return std::string(h ? h : "/tmp") + "/.cache/fire2_tune_single.txt";
}

// The single-system autotuner.  Some choices change speed only; the first
// minimisation of a class of systems (potential, starting pair precision,
// size in powers of two, periodic axes) times one force evaluation of its
// start positions under each candidate, keeps the fastest, and records it in
// the context and in a cache file that later processes read
// ($FIRE_TUNE_CACHE.single, default ~/.cache/fire2_tune_single.txt).  The
// choices are those of the EAM form: the list order (one class in slot
// order, or three distance classes) and the tile layout (256-atom tiles at
// three or two blocks per CU, or 512-atom tiles).  FIRE_LIST_CLASSES=0|1 and
// FIRE_EAM_LAYOUT=0|1|2 fix either; the size rule then gives the layout
// unless it is fixed too.  Small systems keep one class and the size rule
// without timing.  The start lists are rebuilt with the choice before the
// run begins.
int tune_single(fire_ctx* ctx, hipStream_t s) {
  if (ctx->pot.kind != FIRE_POT_GUPTA) return FIRE_OK;
  const char* ec = getenv("FIRE_LIST_CLASSES");
  const char* el = getenv("FIRE_EAM_LAYOUT");
  const int fixed_layout = el ? std::min(2, std::max(0, atoi(el))) : -1;
  auto describe = [](bool cls, int layout) {
    static const char* kLayout[3] = {"256-atom tiles, three blocks per CU", "256-atom tiles, two blocks per CU",
                                     "512-atom tiles"};
    return std::string("list order ") + (cls ? "classes" : "slot") + ", " +
           (layout < 0 ? std::string("tiles by the size rule") : std::string(kLayout[layout]));
  };
  bool cls = ctx->list_classes;
  int layout = ctx->eam_layout;
  if (ec || ctx->n < 16384) {
    cls = ec ? ec[0] == '1' : false;
    layout = fixed_layout;
    ctx->tuning_info = describe(cls, layout) + (ec ? " (FIRE_LIST_CLASSES)" : " (small system, not tuned)");
  } else {
    const int prec = ctx->params.precision == FIRE_FP64 ? 0 : 1;
    int lg = 0;
    while ((1 << (lg + 1)) <= ctx->n) ++lg;
    char key[96];
    snprintf(key, sizeof key, "eam_prec%d_n2e%d_per%d%d%d_layout%d", prec, lg, ctx->box.per[0], ctx->box.per[1],
             ctx->box.per[2], fixed_layout);
    if (!ctx->tune_loaded) {
      ctx->tune_loaded = true;
      FILE* f = fopen(tune_cache_path().c_str(), "r");
      if (f) {
        char k[96];
        int v;
        while (fscanf(f, "%95s %d", k, &v) == 2) ctx->tuned[k] = v;
        fclose(f);
      }
    }
    auto it = ctx->tuned.find(key);
    const bool cached = it != ctx->tuned.end();
    int choice;  // bit 0: distance classes; bits 1-2: the layout
    if (cached) {
      choice = it->second;
      ctx->tuning_info = describe(choice & 1, choice >> 1) + " (cached for " + key + ")";
    } else {
      std::string times;
      float best = 0.0f;
      choice = -1;
      for (int lay = 0; lay < 3; ++lay) {
        if (fixed_layout >= 0 && lay != fixed_layout) continue;
        for (int c = 0; c < 2; ++c) {
          ctx->list_classes = c != 0;
          ctx->eam_layout = lay;
          int rc = rebuild(ctx);
          if (rc) return rc;
          float t = 0.0f;
          rc = time_evaluation(ctx, s, prec, 6, &t);
          if (rc) return rc;
          static const char* kShort[3] = {"256x3", "256x2", "512"};
          char one[64];
          snprintf(one, sizeof one, "%s%s/%s %.1f", times.empty() ? "" : ", ", c ? "classes" : "slot", kShort[lay],
                   1e3 * t);
          times += one;
          if (choice < 0 || t < best) {
            best = t;
            choice = c | (lay << 1);
          }
        }
      }
      ctx->tuned[key] = choice;
      ctx->tuning_info = describe(choice & 1, choice >> 1) + " (tuned for " + key + ": " + times +
                         " us per evaluation; tile atoms x blocks per CU)";
      FILE* f = fopen(tune_cache_path().c_str(), "w");
      if (f) {
        for (auto& kv : ctx->tuned) fprintf(f, "%s %d\n", kv.first.c_str(), kv.second);
        fclose(f);
      }
    }
    cls = (choice & 1) != 0;
    layout = choice >> 1;
    if (!cached) {  // the timing runs left the last candidate's lists
      ctx->list_classes = cls;
      ctx->eam_layout = layout;
      return rebuild(ctx);
    }
  }
  if (cls != ctx->list_classes || layout != ctx->eam_layout) {
    ctx->list_classes = cls;
    ctx->eam_layout = layout;
    return rebuild(ctx);
  }
  return FIRE_OK;
}

int minimize_impl(fire_ctx* ctx, hipStream_t s, double tol, long long max_steps, fire_result* out) {
  if (max_steps < 0) return set_err(ctx, FIRE_E_ARG, "max_steps must be >= 0");
  int rc = rebuild(ctx);
  if (rc) return rc;
  rc = tune_single(ctx, s);
  if (rc) return rc;
  long long rebuilds = 1;
  ctrl_defaults(ctx, *ctx->h_ctrl, tol, max_steps, 0);
  int prec = ctx->h_ctrl->precision;
  // the pinned record is not written again before the copy back at the end
  HIPCHK(hipMemcpyAsync(ctx->ctrl, ctx->h_ctrl, sizeof(Ctrl), hipMemcpyHostToDevice, s));
  launch_forces(ctx, s, prec);  // evaluation 0 and the set-up of iteration 1
  // graph length: short for small systems (launch-bound), longer for large ones
  ctx->graph_k = ctx->n < 20000 ? 32 : 16;
  if (const char* e = getenv("FIRE_GRAPH_K")) ctx->graph_k = std::max(2, atoi(e) & ~1);  // even
  for (;;) {
    // two replays in flight; after the older one's event, read the status
    // word that the last node of a replay writes to host memory (the older
    // replay's, or the newer one's if that has finished too: either way the
    // state the stream is in once the host's next work runs)
    hipGraphExec_t g;
    rc = graph_for(ctx, prec, &g);
    if (rc) return rc;
    HIPCHK(hipGraphLaunch(g, s));
    HIPCHK(hipEventRecord(ctx->ev[0], s));
    int cur = 0;
    unsigned long long word = 0;
    for (;;) {
      HIPCHK(hipGraphLaunch(g, s));
      HIPCHK(hipEventRecord(ctx->ev[cur ^ 1], s));
      HIPCHK(hipEventSynchronize(ctx->ev[cur]));
      word = __atomic_load_n(ctx->h_poll, __ATOMIC_ACQUIRE);
      if ((int)(unsigned)word != ST_RUNNING) break;
      cur ^= 1;
    }
    materialize(ctx, s);
    // the replay seen ended stopped or paused, so every later kernel exits at
    // its gate and the status stays as read (no wait here; the next host read
    // of device data synchronises)
    const int status = (int)(unsigned)word;
    const int pause = (int)(unsigned)(word >> 32);
    if (status != ST_PAUSED) break;
    if (pause & PAUSE_PRECISION) {  // before the next update: switch pair precision
      prec = 0;
      rc = resume(ctx, s);
      if (rc) return rc;
    }
    if (pause & PAUSE_REBUILD) {  // after an update: new list, then this iteration's forces
      rc = rebuild(ctx);
      if (rc) return rc;
      ++rebuilds;
      rc = resume(ctx, s);
      if (rc) return rc;
      launch_forces(ctx, s, prec);
    }
  }
  HIPCHK(hipMemcpyAsync(ctx->h_ctrl, ctx->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  Ctrl h = *ctx->h_ctrl;
  rc = check_status_error(ctx, h.status);
  if (rc) return rc;
  if (!ctx->trace) {
    // the loop skips the energy; evaluate it once at the final positions with
    // the run's last pair precision (forces and norms come out identical)
    Ctrl& e = *ctx->h_ctrl;
    e.status = ST_RUNNING;
    e.pause = 0;
    e.viol = 0;
    e.eval_only = 1;
    e.kick3 = 0.0;
    e.ticket = 0;
    HIPCHK(hipMemcpyAsync(ctx->ctrl, &e, sizeof(Ctrl), hipMemcpyHostToDevice, s));
    launch_forces(ctx, s, h.precision, true);
    HIPCHK(hipMemcpyAsync(ctx->h_ctrl, ctx->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    rc = check_status_error(ctx, ctx->h_ctrl->status);
    if (rc) return rc;
    h.energy = ctx->h_ctrl->energy;
  }
  if (out) {
    memset(out, 0, sizeof(*out));
    out->stop_reason = h.status;
    out->precision_switched = (h.mode == FIRE_MIXED && h.precision == 0) ? 1 : 0;
    out->iterations = h.iter;
    out->force_evals = h.evals;
    out->iterations_low = h.iter_low;
    out->rebuilds = rebuilds;
    out->energy = h.energy;
    out->energy_per_atom = h.energy / ctx->n;
    out->fmax = h.fmax;
    out->f2norm = h.f2norm;
    out->dt = h.dt;
    out->alpha = h.alpha;
  }
  return FIRE_OK;
}

int check_ctx(fire_ctx* ctx) {
  if (!ctx) return FIRE_E_ARG;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return set_err(ctx, FIRE_E_DEVICE, std::string("hipSetDevice: ") + hip_err_str(e));
  return FIRE_OK;
}

// Device-pointer calls enqueue on the caller's stream as given (NULL is the
// legacy default stream, as everywhere in HIP).
hipStream_t pick_stream(fire_ctx* ctx, void* stream) {
  (void)ctx;
  return (hipStream_t)stream;
}

int validate_params(const fire_params* p) {
  if (!(p->dt_start > 0) || !(p->tmax > 0) || !(p->tmin >= 0) || !(p->dtgrow >= 1) || !(p->dtshrink > 0) ||
      !(p->dtshrink <= 1) || !(p->alpha0 >= 0) || !(p->alpha0 <= 1) || !(p->alphashrink > 0) ||
      !(p->alphashrink <= 1) || !(p->f2a > 0) || p->delaystep < 0 || p->vdfmax < 0)
    return FIRE_E_ARG;
  if (p->integrator < 0 || p->integrator > 2 || p->criterion < 0 || p->criterion > 1 || p->variant < 0 ||
      p->variant > 1 || p->precision < 0 || p->precision > 2)
    return FIRE_E_ARG;
  if (!(p->dmax >= 0) || !std::isfinite(p->dmax)) return FIRE_E_ARG;
  return FIRE_OK;
}

// ---- Lanczos helpers (vectors are 3 planes of ncap doubles in sorted order)

int dev_dot(fire_ctx* ctx, hipStream_t s, const double* a, const double* b, double* out_host) {
  const int n = ctx->n, nb = nblocks(n);
  hipLaunchKernelGGL(k_dot, dim3(nb), dim3(kBlock), 0, s, a, b, n, ctx->ncap, ctx->part);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(kBlock), 0, s, ctx->part, nb, ctx->part_emb);
  HIPCHK(hipMemcpyAsync(out_host, ctx->part_emb, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return FIRE_OK;
}

int dev_remove_mean(fire_ctx* ctx, hipStream_t s, double* a) {
  const int n = ctx->n, nb = nblocks(n);
  hipLaunchKernelGGL(k_plane_sums, dim3(nb), dim3(kBlock), 0, s, a, n, ctx->ncap, ctx->bbox_part);
  std::vector<double> h(3 * (size_t)nb);
  HIPCHK(hipMemcpyAsync(h.data(), ctx->bbox_part, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  double m[3] = {0, 0, 0};
  for (int q = 0; q < nb; ++q)
    for (int d = 0; d < 3; ++d) m[d] += h[3 * q + d];
  hipLaunchKernelGGL(k_sub_plane, dim3(nb), dim3(kBlock), 0, s, a, n, ctx->ncap, m[0] / n, m[1] / n, m[2] / n);
  return FIRE_OK;
}

// hu = H u for sorted-order planes u (list and positions current).
void launch_hvp(fire_ctx* ctx, hipStream_t s, const double* u, double* hu, double* pre) {
  const int n = ctx->n, nb = nblocks(n);
  if (ctx->pot.kind == FIRE_POT_GUPTA)
    hipLaunchKernelGGL(k_gupta_hvp_pre, dim3(nb), dim3(kBlock), 0, s, ctx->pos, ctx->nbr, ctx->wcnt, ctx->real_of, n,
                       ctx->kcap, ctx->ncap, ctx->pot, u, pre);
  hipLaunchKernelGGL(k_hvp, dim3(nb), dim3(kBlock), 0, s, ctx->pos, ctx->nbr, ctx->wcnt, ctx->real_of, n, ctx->kcap,
                     ctx->ncap, ctx->pot, u, (const double*)pre, hu);
}

// Smallest eigenvalue of the symmetric tridiagonal matrix (a diagonal, b off-diagonal) by Sturm bisection.
double tridiag_min_eig(const std::vector<double>& a, const std::vector<double>& b) {
  const int k = (int)a.size();
  double lo = INFINITY, hi = -INFINITY;
  for (int i = 0; i < k; ++i) {
    double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i < k - 1 ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  auto count_below = [&](double x) {
    int cnt = 0;
    double q = 1.0;
    for (int i = 0; i < k; ++i) {
      double bb = i > 0 ? b[i - 1] * b[i - 1] : 0.0;
      q = a[i] - x - (i > 0 ? bb / q : 0.0);
      if (q == 0.0) q = -1e-300;
      if (q < 0) ++cnt;
    }
    return cnt;
  };
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (count_below(mid) >= 1) hi = mid;
    else lo = mid;
  }
  return 0.5 * (lo + hi);
}

// Last component of the unit eigenvector of the symmetric tridiagonal T
// (diagonal a, off-diagonal b) for its eigenvalue lam, by inverse iteration:
// solves (T - sigma) x = y with sigma just below lam, Gaussian elimination
// with partial pivoting on the band.
double tridiag_last_component(const std::vector<double>& a, const std::vector<double>& b, double lam) {
  const int k = (int)a.size();
  if (k == 1) return 1.0;
  double scale = 0.0;
  for (int i = 0; i < k; ++i) scale = std::max(scale, std::fabs(a[i]) + (i < k - 1 ? std::fabs(b[i]) : 0.0));
  const double sigma = lam - 1e-10 * std::max(scale, 1e-300);
  std::vector<double> y(k, 1.0), x(k);
  for (int it = 0; it < 4; ++it) {
    // rows: d[i] on the diagonal, u1[i], u2[i] above it, l[i] below it
    std::vector<double> d(k), u1(k, 0.0), u2(k, 0.0), l(k, 0.0), r = y;
    for (int i = 0; i < k; ++i) {
      d[i] = a[i] - sigma;
      if (i < k - 1) u1[i] = b[i];
      if (i > 0) l[i] = b[i - 1];
    }
    for (int i = 0; i < k - 1; ++i) {
      if (std::fabs(l[i + 1]) > std::fabs(d[i])) {  // swap rows i and i + 1
        std::swap(d[i], l[i + 1]);
        std::swap(u1[i], d[i + 1]);
        std::swap(u2[i], u1[i + 1]);
        std::swap(r[i], r[i + 1]);
      }
      const double m = d[i] != 0.0 ? l[i + 1] / d[i] : 0.0;
      d[i + 1] -= m * u1[i];
      u1[i + 1] -= m * u2[i];
      r[i + 1] -= m * r[i];
    }
    for (int i = k - 1; i >= 0; --i) {
      double t = r[i];
      if (i + 1 < k) t -= u1[i] * x[i + 1];
      if (i + 2 < k) t -= u2[i] * x[i + 2];
      x[i] = t / (d[i] != 0.0 ? d[i] : 1e-300);
    }
    double nrm = 0.0;
    for (int i = 0; i < k; ++i) nrm += x[i] * x[i];
    nrm = std::sqrt(nrm);
    for (int i = 0; i < k; ++i) y[i] = x[i] / nrm;
  }
  return y[k - 1];
}

}  // namespace

// Accessors for the batched path (batched.hip).
hipStream_t fire_ctx_stream(fire_ctx* ctx) { return ctx->stream; }
const fire_params* fire_ctx_params(fire_ctx* ctx) { return &ctx->params; }
void** fire_ctx_batched_slot(fire_ctx* ctx) { return &ctx->batched; }
int fire_ctx_error(fire_ctx* ctx, int code, const char* msg) { return set_err(ctx, code, msg); }
void fire_ctx_set_tuning_info(fire_ctx* ctx, const char* info) { ctx->tuning_info = info; }
int fire_prepare_pot(fire_ctx* ctx, const fire_potential* p, PotDev* out) { return prepare_pot(ctx, p, *out); }
void fire_ctrl_from_params(const fire_params* p, double tol, long long max_steps, double skin, int natoms, Ctrl* c) {
  ctrl_from_params(*p, tol, max_steps, 0.25 * skin * skin, natoms, *c);
}

// =================================================================== C ABI

extern "C" {

void fire_params_default(fire_params* p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->dt_start = 1.0;
  p->tmax = 10.0;
  p->tmin = 0.02;
  p->dtgrow = 1.1;
  p->dtshrink = 0.5;
  p->alpha0 = 0.25;
  p->alphashrink = 0.99;
  p->f2a = 1.0;
  p->delaystep = 20;
  p->vdfmax = 2000;
  p->halfstepback = 1;
  p->initialdelay = 1;
  p->integrator = FIRE_INT_EULER_IMPLICIT;
  p->criterion = FIRE_CRIT_FMAX;
  p->variant = FIRE_VARIANT_FIRE2;
  p->precision = FIRE_FP64;
  p->mixed_switch = 0.0;
  p->skin = 0.0;
  p->dmax = 0.0;
}

const char* fire_stop_name(int r) {
  switch (r) {
    case FIRE_STOP_CONVERGED: return "converged";
    case FIRE_STOP_MAX_STEPS: return "max_steps";
    case FIRE_STOP_MAXVDOTF: return "maxvdotf";
    case FIRE_E_NONFINITE: return "nonfinite";
    case FIRE_E_OVERLAP: return "overlap";
    default: return "unknown";
  }
}

const char* fire_last_error(const fire_ctx* ctx) { return ctx ? ctx->err.c_str() : "no context"; }

const char* fire_tuning_info(const fire_ctx* ctx) { return ctx ? ctx->tuning_info.c_str() : "no context"; }

int fire_init(fire_ctx** out, int device, const fire_params* params) {
  if (!out) return FIRE_E_ARG;
  *out = nullptr;
  if (params && validate_params(params)) return FIRE_E_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return FIRE_E_DEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return FIRE_E_DEVICE;
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return FIRE_E_DEVICE;
  fire_ctx* ctx = new fire_ctx();
  ctx->device = device;
  ctx->ncu = std::max(1, prop.multiProcessorCount);
  if (params) ctx->params = *params;
  else fire_params_default(&ctx->params);
  int rc = FIRE_OK;
  auto init = [&]() -> int {
    HIPCHK(hipSetDevice(device));
    HIPCHK(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
    HIPCHK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    HIPCHK(hipMalloc((void**)&ctx->ctrl, sizeof(Ctrl)));
    HIPCHK(hipMalloc((void**)&ctx->flags, 8 * sizeof(int)));
    HIPCHK(hipHostMalloc((void**)&ctx->h_flags, 8 * sizeof(int), hipHostMallocDefault));
    // LDS-staged pair passes with at most 52 KB per 256-atom tile block
    // (three blocks per CU) and 78 KB per 512-atom LJ tile block (two);
    // FIRE_LDS=0: global gathers only; FIRE_LDS=<bytes>: that limit for both
    {
      const char* e = getenv("FIRE_LDS");
      const long v = e ? atol(e) : 1;
      const size_t cap = prop.sharedMemPerBlock > 4096 ? prop.sharedMemPerBlock - 4096 : 0;
      ctx->lds_limit = v <= 0 ? 0 : std::min<size_t>(cap, v == 1 ? 52 * 1024 : (size_t)v);
      ctx->lds_default = v == 1;
      ctx->lds_cap = cap;
    }
    HIPCHK(hipHostMalloc((void**)&ctx->h_ctrl, sizeof(Ctrl), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&ctx->h_poll, sizeof(unsigned long long), hipHostMallocCoherent));
    HIPCHK(hipHostGetDevicePointer((void**)&ctx->d_poll, ctx->h_poll, 0));
    HIPCHK(hipHostMalloc((void**)&ctx->h_zero, sizeof(double), hipHostMallocDefault));
    HIPCHK(hipEventCreateWithFlags(&ctx->ev[0], hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&ctx->ev[1], hipEventDisableTiming));
    // the scratch array of fire_minimize_batched_noalloc on this device
    const int na = fire_noalloc_init(device, &ctx->noalloc);
    if (na) return set_err(ctx, na, "no-allocation scratch set-up failed");
    return FIRE_OK;
  };
  rc = init();
  if (rc) {
    fire_finalize(ctx);
    return rc;
  }
  *out = ctx;
  return FIRE_OK;
}

void fire_finalize(fire_ctx* ctx) {
  if (!ctx) return;
  hipSetDevice(ctx->device);
  if (ctx->stream) hipStreamSynchronize(ctx->stream);
  drop_graphs(ctx);
  free_single(ctx);
  hipFree(ctx->nbr);
  hipFree(ctx->wcnt);
  hipFree(ctx->cell_count);
  hipFree(ctx->cell_start);
  hipFree(ctx->cell_cursor);
  hipFree(ctx->cell_rank);
  hipFree(ctx->rank_cell);
  hipFree(ctx->aux);
  hipFree(ctx->ctrl);
  hipFree(ctx->flags);
  hipFree(ctx->scan_part);
  hipFree(ctx->trace);
  if (ctx->h_flags) hipHostFree(ctx->h_flags);
  if (ctx->h_ctrl) hipHostFree(ctx->h_ctrl);
  if (ctx->h_poll) hipHostFree(ctx->h_poll);
  if (ctx->h_zero) hipHostFree(ctx->h_zero);
  for (int k = 0; k < 2; ++k)
    if (ctx->ev[k]) hipEventDestroy(ctx->ev[k]);
  fire_batched_release(ctx->batched);
  fire_noalloc_release(ctx->noalloc);
  if (ctx->stream) hipStreamDestroy(ctx->stream);
  if (ctx->cap_stream) hipStreamDestroy(ctx->cap_stream);
  delete ctx;
}

int fire_set_params(fire_ctx* ctx, const fire_params* p) {
  if (!ctx || !p) return FIRE_E_ARG;
  if (validate_params(p)) return set_err(ctx, FIRE_E_ARG, "invalid FIRE parameters");
  ctx->params = *p;
  drop_graphs(ctx);  // the captured loop depends on the integrator
  return FIRE_OK;
}

int fire_get_params(const fire_ctx* ctx, fire_params* p) {
  if (!ctx || !p) return FIRE_E_ARG;
  *p = ctx->params;
  return FIRE_OK;
}

static int energy_forces_common(fire_ctx* ctx, long long n, const double* pos, bool host, const fire_box* box,
                                const fire_potential* pot, double* energy, double* forces, hipStream_t s) {
  int rc = prepare_system(ctx, box, pot);
  if (rc) return rc;
  hipStream_t saved = ctx->stream;
  ctx->stream = s;
  rc = stage_in(ctx, n, pos, host, s);
  if (!rc) rc = evaluate(ctx, s);
  ctx->stream = saved;
  if (rc) return rc;
  if (host) {
    HIPCHK(hipMemcpyAsync(ctx->h_ctrl, ctx->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    if (forces) {
      hipLaunchKernelGGL(k_scatter_vec, dim3(nblocks(n)), dim3(kBlock), 0, s, ctx->frc, (int)n, ctx->ncap, ctx->id,
                         ctx->stage);
      HIPCHK(hipMemcpyAsync(forces, ctx->stage, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    rc = check_status_error(ctx, ctx->h_ctrl->status);
    if (rc) return rc;
    if (energy) *energy = ctx->h_ctrl->energy;
  } else {
    if (forces)
      hipLaunchKernelGGL(k_scatter_vec, dim3(nblocks(n)), dim3(kBlock), 0, s, ctx->frc, (int)n, ctx->ncap, ctx->id,
                         forces);
    if (energy) HIPCHK(hipMemcpyAsync(energy, &ctx->ctrl->energy, sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  return FIRE_OK;
}

int fire_energy_forces(fire_ctx* ctx, long long n, const double* pos, const fire_box* box, const fire_potential* pot,
                       double* energy, double* forces) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  return energy_forces_common(ctx, n, pos, true, box, pot, energy, forces, ctx->stream);
}

int fire_energy_forces_dev(fire_ctx* ctx, long long n, const double* d_pos, const fire_box* box,
                           const fire_potential* pot, double* d_energy, double* d_forces, void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  return energy_forces_common(ctx, n, d_pos, false, box, pot, d_energy, d_forces, pick_stream(ctx, stream));
}

static int minimize_common(fire_ctx* ctx, long long n, double* pos, bool host, const fire_box* box,
                           const fire_potential* pot, double tol, long long max_steps, fire_result* out,
                           double* trace_host, hipStream_t s, const fire_atoms* atoms = nullptr) {
  if (!(tol >= 0)) return set_err(ctx, FIRE_E_ARG, "tol must be >= 0");
  int rc = prepare_system(ctx, box, pot);
  if (rc) return rc;
  hipStream_t saved = ctx->stream;
  ctx->stream = s;
  rc = stage_in(ctx, n, pos, host, s);
  if (!rc) rc = setup_props(ctx, atoms, host, s);
  if (!rc && trace_host) {
    hipFree(ctx->trace);
    ctx->trace = nullptr;
    ctx->trace_cap = max_steps + 1;
    hipError_t e = dalloc(&ctx->trace, (size_t)FIRE_TRACE_COLS * (max_steps + 1));
    if (e != hipSuccess) rc = set_err(ctx, FIRE_E_OOM, "trace allocation");
  }
  if (!rc) rc = minimize_impl(ctx, s, tol, max_steps, out);
  if (!rc) {
    double* dst = host ? ctx->stage : pos;
    hipLaunchKernelGGL(k_stage_out_pos, dim3(nblocks(n)), dim3(kBlock), 0, s, ctx->pos, (int)n, ctx->id, ctx->box,
                       dst);
    if (host) {
      hipError_t e = hipMemcpyAsync(pos, ctx->stage, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, s);
      if (e != hipSuccess) rc = set_err(ctx, FIRE_E_DEVICE, hip_err_str(e));
    }
    if (!rc && trace_host && out) {
      hipError_t e = hipMemcpyAsync(trace_host, ctx->trace,
                                    sizeof(double) * FIRE_TRACE_COLS * (size_t)(out->iterations + 1),
                                    hipMemcpyDeviceToHost, s);
      if (e != hipSuccess) rc = set_err(ctx, FIRE_E_DEVICE, hip_err_str(e));
    }
    hipError_t e = hipStreamSynchronize(s);
    if (!rc && e != hipSuccess) rc = set_err(ctx, FIRE_E_DEVICE, hip_err_str(e));
  }
  if (trace_host) {
    hipFree(ctx->trace);
    ctx->trace = nullptr;
    ctx->trace_cap = 0;
    drop_graphs(ctx);
  }
  ctx->with_mass = ctx->with_frozen = false;
  ctx->stream = saved;
  return rc;
}

int fire_minimize(fire_ctx* ctx, long long n, double* pos, const fire_box* box, const fire_potential* pot, double tol,
                  long long max_steps, fire_result* out) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  return minimize_common(ctx, n, pos, true, box, pot, tol, max_steps, out, nullptr, ctx->stream);
}

int fire_minimize_traced(fire_ctx* ctx, long long n, double* pos, const fire_box* box, const fire_potential* pot,
                         double tol, long long max_steps, fire_result* out, double* trace) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!trace || !out) return set_err(ctx, FIRE_E_ARG, "trace and out are required");
  return minimize_common(ctx, n, pos, true, box, pot, tol, max_steps, out, trace, ctx->stream);
}

int fire_minimize_dev(fire_ctx* ctx, long long n, double* d_pos, const fire_box* box, const fire_potential* pot,
                      double tol, long long max_steps, fire_result* out, void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  return minimize_common(ctx, n, d_pos, false, box, pot, tol, max_steps, out, nullptr, pick_stream(ctx, stream));
}

int fire_minimize_ex(fire_ctx* ctx, long long n, double* pos, const fire_box* box, const fire_potential* pot,
                     const fire_atoms* atoms, double tol, long long max_steps, fire_result* out, double* trace) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (trace && !out) return set_err(ctx, FIRE_E_ARG, "a trace requires out");
  return minimize_common(ctx, n, pos, true, box, pot, tol, max_steps, out, trace, ctx->stream, atoms);
}

int fire_minimize_ex_dev(fire_ctx* ctx, long long n, double* d_pos, const fire_box* box, const fire_potential* pot,
                         const fire_atoms* d_atoms, double tol, long long max_steps, fire_result* out,
                         void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  return minimize_common(ctx, n, d_pos, false, box, pot, tol, max_steps, out, nullptr, pick_stream(ctx, stream),
                         d_atoms);
}

static int hvp_common(fire_ctx* ctx, long long n, const double* pos, const double* u, bool host, const fire_box* box,
                      const fire_potential* pot, double* hu, hipStream_t s) {
  if (!u || !hu) return set_err(ctx, FIRE_E_ARG, "u and hu are required");
  int rc = prepare_system(ctx, box, pot);
  if (rc) return rc;
  if (ctx->pot.kind == FIRE_POT_SW) return set_err(ctx, FIRE_E_ARG, "no Hessian product for the SW potential");
  hipStream_t saved = ctx->stream;
  ctx->stream = s;
  rc = stage_in(ctx, n, pos, host, s);
  if (!rc) rc = rebuild(ctx);
  if (!rc) rc = ensure_aux(ctx, 9);
  if (!rc) {
    const double* usrc = u;
    if (host) {
      hipError_t e = hipMemcpyAsync(ctx->stage, u, sizeof(double) * 3 * n, hipMemcpyHostToDevice, s);
      if (e != hipSuccess) rc = set_err(ctx, FIRE_E_DEVICE, hip_err_str(e));
      usrc = ctx->stage;
    }
    double* us = ctx->aux;
    double* hs = ctx->aux + 3 * (size_t)ctx->ncap;
    double* pre = ctx->aux + 6 * (size_t)ctx->ncap;
    if (!rc) {
      hipLaunchKernelGGL(k_gather_vec, dim3(nblocks(n)), dim3(kBlock), 0, s, usrc, (int)n, ctx->ncap, ctx->id, us);
      launch_hvp(ctx, s, us, hs, pre);
      double* dst = host ? ctx->stage : hu;
      hipLaunchKernelGGL(k_scatter_vec, dim3(nblocks(n)), dim3(kBlock), 0, s, hs, (int)n, ctx->ncap, ctx->id, dst);
      if (host) {
        hipError_t e = hipMemcpyAsync(hu, ctx->stage, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) rc = set_err(ctx, FIRE_E_DEVICE, hip_err_str(e));
        e = hipStreamSynchronize(s);
        if (!rc && e != hipSuccess) rc = set_err(ctx, FIRE_E_DEVICE, hip_err_str(e));
      }
    }
  }
  ctx->stream = saved;
  return rc;
}

int fire_hvp(fire_ctx* ctx, long long n, const double* pos, const double* u, const fire_box* box,
             const fire_potential* pot, double* hu) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  return hvp_common(ctx, n, pos, u, true, box, pot, hu, ctx->stream);
}

int fire_hvp_dev(fire_ctx* ctx, long long n, const double* d_pos, const double* d_u, const fire_box* box,
                 const fire_potential* pot, double* d_hu, void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  return hvp_common(ctx, n, d_pos, d_u, false, box, pot, d_hu, pick_stream(ctx, stream));
}

int fire_lowest_curvature(fire_ctx* ctx, long long n, const double* pos, const fire_box* box,
                          const fire_potential* pot, const double* u0, int k, double* lambda_min,
                          double* residual) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!lambda_min || k < 1 || k > 500) return set_err(ctx, FIRE_E_ARG, "need lambda_min and 1 <= k <= 500");
  rc = prepare_system(ctx, box, pot);
  if (rc) return rc;
  if (ctx->pot.kind == FIRE_POT_SW) return set_err(ctx, FIRE_E_ARG, "no Hessian product for the SW potential");
  hipStream_t s = ctx->stream;
  rc = stage_in(ctx, n, pos, true, s);
  if (rc) return rc;
  rc = rebuild(ctx);
  if (rc) return rc;
  // planes: k+1 Lanczos vectors (3 each) + w (3) + hvp prologue (3)
  const int nv = k + 1;
  rc = ensure_aux(ctx, 3 * nv + 6);
  if (rc) return rc;
  const size_t pl = 3 * (size_t)ctx->ncap;
  double* V = ctx->aux;
  double* w = ctx->aux + nv * pl;
  double* pre = w + pl;
  std::vector<double> start(3 * (size_t)n);
  if (u0) {
    memcpy(start.data(), u0, sizeof(double) * 3 * n);
  } else {
    unsigned long long x = 0x9E3779B97F4A7C15ULL;  // splitmix64 stream, deterministic start vector
    for (size_t i = 0; i < start.size(); ++i) {
      x += 0x9E3779B97F4A7C15ULL;
      unsigned long long z = x;
      z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
      z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
      z ^= z >> 31;
      start[i] = (double)(z >> 11) * (1.0 / 9007199254740992.0) - 0.5;
    }
  }
  HIPCHK(hipMemcpyAsync(ctx->stage, start.data(), sizeof(double) * 3 * n, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_gather_vec, dim3(nblocks(n)), dim3(kBlock), 0, s, ctx->stage, (int)n, ctx->ncap, ctx->id, V);
  // rigid translations are zero modes of every pair potential: keep them out
  const bool project = ctx->pot.kind != FIRE_POT_HARMONIC;
  if (project) {
    rc = dev_remove_mean(ctx, s, V);
    if (rc) return rc;
  }
  double nrm2;
  rc = dev_dot(ctx, s, V, V, &nrm2);
  if (rc) return rc;
  if (!(nrm2 > 0)) return set_err(ctx, FIRE_E_ARG, "start vector has no component off translations");
  const int nb = nblocks(n);
  hipLaunchKernelGGL(k_axpby, dim3(nb), dim3(kBlock), 0, s, V, V, (int)n, ctx->ncap, 1.0 / std::sqrt(nrm2), 0.0);
  std::vector<double> a, b;
  double beta_last = 0.0;
  for (int j = 0; j < k; ++j) {
    double* vj = V + j * pl;
    launch_hvp(ctx, s, vj, w, pre);
    rc = dev_remove_mean(ctx, s, w);
    if (rc) return rc;
    // full re-orthogonalisation against all previous vectors (twice)
    double aj = 0.0;
    for (int pass = 0; pass < 2; ++pass)
      for (int q = 0; q <= j; ++q) {
        double h;
        rc = dev_dot(ctx, s, V + q * pl, w, &h);
        if (rc) return rc;
        if (q == j) aj += h;
        hipLaunchKernelGGL(k_axpby, dim3(nb), dim3(kBlock), 0, s, w, V + q * pl, (int)n, ctx->ncap, 1.0, -h);
      }
    a.push_back(aj);
    double bb;
    rc = dev_dot(ctx, s, w, w, &bb);
    if (rc) return rc;
    double bj = std::sqrt(std::max(bb, 0.0));
    beta_last = bj;
    if (j == k - 1 || bj < 1e-12 * std::fabs(aj)) break;
    b.push_back(bj);
    HIPCHK(hipMemcpyAsync(V + (j + 1) * pl, w, sizeof(double) * pl, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_axpby, dim3(nb), dim3(kBlock), 0, s, V + (j + 1) * pl, V, (int)n, ctx->ncap, 1.0 / bj, 0.0);
  }
  b.resize(a.size() > 0 ? a.size() - 1 : 0);
  *lambda_min = tridiag_min_eig(a, b);
  // |H z - theta z| of the Ritz vector z = V y is beta_k |y_k|
  if (residual) *residual = beta_last * std::fabs(tridiag_last_component(a, b, *lambda_min));
  return FIRE_OK;
}

int fire_repeat_forces_dev(fire_ctx* ctx, int reps, void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  if (!ctx->have_list || ctx->n <= 0 || reps < 0) return set_err(ctx, FIRE_E_ARG, "no evaluated system");
  hipStream_t s = pick_stream(ctx, stream);
  // a running control record with no Verlet half kick, so the passes recompute
  // forces and reductions only
  ctrl_defaults(ctx, *ctx->h_ctrl, 0.0, 0, 1);
  HIPCHK(hipMemcpyAsync(ctx->ctrl, ctx->h_ctrl, sizeof(Ctrl), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  const int prec = ctx->params.precision == FIRE_FP64 ? 0 : 1;
  if (fold_update(ctx)) {
    // the loop's pass: the (here zero) pending update applied while staging,
    // from the primary set into the second one, which is scratch outside the
    // loop; every repeat reads the same primary set
    for (int r = 0; r < reps; ++r) launch_pairs<false>(ctx, s, prec, 0);
    hipLaunchKernelGGL(k_ghost_refresh, dim3(1), dim3(kBlock), 0, s, ctx->n, 0, ctx->pos, ctx->real_of, ctx->gcode,
                       ctx->box, ctx->ctrl);  // ng = 0: only resets ctrl->cur
  } else {
    for (int r = 0; r < reps; ++r) launch_forces(ctx, s, prec, false);
  }
  return FIRE_OK;
}

// The batched form has no displacement cap.
static int batched_no_dmax(fire_ctx* ctx, int nsys, const fire_params* per_sys) {
  bool any = ctx->params.dmax > 0;
  for (int s = 0; per_sys && s < nsys && !any; ++s) any = per_sys[s].dmax > 0;
  return any ? set_err(ctx, FIRE_E_ARG, "batched: dmax is not available") : FIRE_OK;
}

int fire_minimize_batched(fire_ctx* ctx, int nsys, const long long* offsets, double* pos, const fire_box* boxes,
                          const fire_potential* pot, const fire_params* per_sys, double tol, long long max_steps,
                          fire_result* out) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  rc = batched_no_dmax(ctx, nsys, per_sys);
  if (rc) return rc;
  return fire_batched_run(ctx, nsys, offsets, pos, true, boxes, pot, per_sys, tol, max_steps, out, ctx->stream);
}

int fire_minimize_batched_dev(fire_ctx* ctx, int nsys, const long long* offsets, double* d_pos,
                              const fire_box* boxes, const fire_potential* pot, const fire_params* per_sys,
                              double tol, long long max_steps, fire_result* out, void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  rc = batched_no_dmax(ctx, nsys, per_sys);
  if (rc) return rc;
  return fire_batched_run(ctx, nsys, offsets, d_pos, false, boxes, pot, per_sys, tol, max_steps, out,
                          pick_stream(ctx, stream));
}

int fire_minimize_batched_noalloc(fire_ctx* ctx, int nsys, const long long* offsets, double* d_pos,
                                  const fire_box* boxes, const fire_potential* pot, const fire_params* per_sys,
                                  double tol, long long max_steps, fire_result* out, void* stream) {
  int rc = check_ctx(ctx);
  if (rc) return rc;
  rc = batched_no_dmax(ctx, nsys, per_sys);
  if (rc) return rc;
  return fire_batched_run_noalloc(ctx, ctx->noalloc, nsys, offsets, d_pos, boxes, pot, per_sys, tol, max_steps,
                                  out, pick_stream(ctx, stream));
}

}  // extern "C"
