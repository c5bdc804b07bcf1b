// Charge and current deposit: rho^n at x^n, J^{n+1/2} at x^{n+1/2} (velocity
// v^{n+1/2}) and rho^{n+1} at x^{n+1}, linear shapes, every azimuthal mode.
//
// Work decomposition (no global atomics anywhere):
//   * particles are sorted by the cell of x^{n+1}; the cells are cut into
//     TZ x TR tiles and each particle belongs to exactly one tile;
//   * a tile's particles touch the nodes of its cells plus a halo of H cells
//     (x^n, x^{n+1/2} lie within dt c of x^{n+1}, dt <= H dz and H dr), so
//     a workgroup accumulates a (TZ + 2H + 1) x (TR + 2H + 1) node block in
//     LDS (FP64: on gfx950 an FP64 LDS atomic is ~20x cheaper than an FP32
//     one) and writes it to an FP32 scratch slot;
//   * dense tiles (beam cores and compressed plasma, more than tile_max
//     particles) are cut into chunks of `chunk` particles, each its own
//     workgroup and slot; the device builds this work list (k_tile_plan) from
//     the sorted offsets, and k_chunk_reduce sums a tile's chunk slots into
//     its first one;
//   * k_deposit_combine sums, node by node, the slots of the tiles covering
//     the node and writes the grid.
// Within a workgroup every lane takes runs of at most kRun particles of one
// cell.  Particles of one cell share their four nodes, so a lane sums the node
// contributions of each of the three positions in registers and issues the
// LDS atomics only when that position's cell changes; for x^{n+1} that is at
// most once per run, for all lanes together.  Beam cores with thousands of
// particles per cell cost one flush per run rather than one atomic per
// particle.  Waves whose particles are all at rest skip the current and reuse
// the x^{n+1} shape for rho^n.
//
// Immobile background: the ion deposit of each tile is kept as an FP64 block
// (built once at set-up by this same kernel) and added to both densities in
// the LDS block of the tile's first work item before the FP32 rounding, so
// the rounding acts on the net charge, not on two order-one densities that
// nearly cancel.
#include <type_traits>

#include "common.h"
#include "launch.h"

namespace pic {

constexpr int kChunkMin = 2048;  // smallest chunk of a dense tile (sizes the work list)
constexpr int kChunkMax = 8192;  // largest chunk (keeps a work item's run table in 16 bits)
constexpr int kTZ = 32;          // tile rows (z)
constexpr int kRun = 8;          // particles of one cell per lane per run

__device__ __forceinline__ size_t dfidx(int c, int m, int M, int nr, int nz) {
  return ((size_t)c * M + m) * (size_t)nr * nz;
}

template <int TR, int H>
struct Blk {
  static constexpr int BZ = kTZ + 2 * H + 1;   // nodes J0 - H .. J0 + TZ + H
  static constexpr int BR = TR + 2 * H + 1;    // nodes C0 - 1 - H .. C0 + TR - 1 + H
  static constexpr int NODES = BZ * BR;
};

struct TileGeom {
  int ntz, ntr, ntiles;
  int tile_max;   // a tile with more particles than this is cut into chunks
  int chunk;      // particles per chunk of a dense tile
};

// ---------------------------------------------------------------------------
// planning: particles per tile -> chunks -> work list
// ---------------------------------------------------------------------------
template <int TR>
__global__ __launch_bounds__(256) void k_tile_totals(const int* __restrict__ offset, Grid g, TileGeom tg,
                                                     int* __restrict__ nchunk) {
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (t >= tg.ntiles) return;
  const int J0 = (t % tg.ntz) * kTZ, C0 = (t / tg.ntz) * TR;
  const int C1 = min(C0 + TR, g.ncol);
  int s = 0;
  if (lane < kTZ) {
    const int j = J0 + lane;
    s = offset[j * g.ncol + C1] - offset[j * g.ncol + C0];
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) nchunk[t] = s > tg.tile_max ? (s + tg.chunk - 1) / tg.chunk : 1;
}

// Exclusive scans over the tiles (wave scans, then the wave totals): the
// chunk counts give chunk_start[0..ntiles] (chunk_start[ntiles] = work
// items), the tiles cut into more than one chunk are listed in ascending order
// in dense[0..ndense), with ndense stored in dense[ntiles].
__global__ __launch_bounds__(1024) void k_tile_plan(const int* __restrict__ nchunk, int ntiles,
                                                   int* __restrict__ chunk_start, int* __restrict__ dense) {
  __shared__ int wsum[2][16];
  __shared__ int carry[2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) carry[0] = carry[1] = 0;
  __syncthreads();
  for (int b0 = 0; b0 < ntiles; b0 += 1024) {
    const int i = b0 + threadIdx.x;
    const int v = i < ntiles ? nchunk[i] : 0;
    const int f = v > 1 ? 1 : 0;
    int a = v, d = f;   // inclusive scans within the wave
    for (int off = 1; off < 64; off <<= 1) {
      const int ua = __shfl_up(a, off, 64), ud = __shfl_up(d, off, 64);
      if (lane >= off) {
        a += ua;
        d += ud;
      }
    }
    if (lane == 63) {
      wsum[0][wave] = a;
      wsum[1][wave] = d;
    }
    __syncthreads();
    int pa = carry[0], pd = carry[1];
    for (int w = 0; w < wave; ++w) {
      pa += wsum[0][w];
      pd += wsum[1][w];
    }
    if (i < ntiles) {
      chunk_start[i] = pa + a - v;
      if (f) dense[pd + d - 1] = i;
    }
    __syncthreads();   // carry and wsum are read by every thread before they change
    if (threadIdx.x == 1023) {
      carry[0] = pa + a;
      carry[1] = pd + d;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    chunk_start[ntiles] = carry[0];
    dense[ntiles] = carry[1];
  }
}

// ---------------------------------------------------------------------------
// Compact value layout of a block (FP64 in LDS, FP32 in the scratch slot),
// [value][node]: mode 0 holds J+ (re, im), Jz, rho^n, rho^{n+1} (the mode-0
// densities and J_z are real, J-,0 = conj(J+,0) is rebuilt by the combine);
// each mode m >= 1 holds J+, J-, Jz, rho^n, rho^{n+1}, complex.
template <int M>
struct Vals {
  static constexpr int N = 5 + 10 * (M - 1);
};
__device__ __forceinline__ constexpr int vbase(int m) { return m == 0 ? 0 : 5 + 10 * (m - 1); }

// ---------------------------------------------------------------------------
// per-position values and their place in the block: each value k has a
// compile-time offset (value index times the block's node count) and the
// parity of its Hankel order (sign of the ghost node across the axis).
// ---------------------------------------------------------------------------
template <int M, int NODES>
struct RhoSet {
  static constexpr int K = 1 + 2 * (M - 1);
  static __device__ __forceinline__ constexpr int mode(int k) { return k == 0 ? 0 : 1 + (k - 1) / 2; }
  static __device__ __forceinline__ constexpr int part(int k) { return k == 0 ? 0 : (k - 1) & 1; }
  static __device__ __forceinline__ constexpr int parity(int k) { return mode(k) & 1; }
  // slot 3: rho^n, slot 4: rho^{n+1}
  static __device__ __forceinline__ constexpr int off(int slot, int k) {
    return (k == 0 ? slot : vbase(mode(k)) + (slot == 3 ? 6 : 8) + part(k)) * NODES;
  }
  static __device__ __forceinline__ void values(float qw, float2 e, float (&v)[K]) {
    v[0] = qw;
    float2 em = e;
#pragma unroll
    for (int m = 1; m < M; ++m) {
      v[1 + 2 * (m - 1)] = qw * em.x;
      v[2 + 2 * (m - 1)] = qw * em.y;
      em = cmul(em, e);
    }
  }
};

template <int M, int NODES>
struct JSet {
  static constexpr int K = 3 + 6 * (M - 1);
  // k < 3: J+,0 (re, im), Jz,0 (re); then per mode m >= 1: J+ (re, im), J- (re, im), Jz (re, im)
  static __device__ __forceinline__ constexpr int mode(int k) { return k < 3 ? 0 : 1 + (k - 3) / 6; }
  static __device__ __forceinline__ constexpr int slot(int k) { return k < 3 ? (k < 2 ? 0 : 2) : ((k - 3) % 6) / 2; }
  static __device__ __forceinline__ constexpr int part(int k) { return k < 3 ? (k < 2 ? k : 0) : (k - 3) & 1; }
  static __device__ __forceinline__ constexpr int parity(int k) {
    return slot(k) == 2 ? (mode(k) & 1) : ((mode(k) + 1) & 1);
  }
  static __device__ __forceinline__ constexpr int off(int k) {
    return (k < 3 ? k : vbase(mode(k)) + (k - 3) % 6) * NODES;
  }
  static __device__ __forceinline__ void values(float qw, float vx, float vy, float vz, float2 e, float (&v)[K]) {
    // J+ = qw (vx - i vy)/2 e^{i(m+1)theta}; J- = qw (vx + i vy)/2 e^{i(m-1)theta}; Jz = qw vz e^{i m theta}
    const float2 ap = make_float2(0.5f * qw * vx, -0.5f * qw * vy);
    const float2 am = make_float2(0.5f * qw * vx, 0.5f * qw * vy);
    const float az = qw * vz;
    const float2 p1 = cmul(ap, e);
    v[0] = p1.x;
    v[1] = p1.y;
    v[2] = az;
    float2 em = e;
#pragma unroll
    for (int m = 1; m < M; ++m) {
      const float2 jp = cmul(ap, cmul(em, e));
      const float2 jm = cmul(am, cmul(em, cconj(e)));
      const int b = 3 + 6 * (m - 1);
      v[b + 0] = jp.x;
      v[b + 1] = jp.y;
      v[b + 2] = jm.x;
      v[b + 3] = jm.y;
      v[b + 4] = az * em.x;
      v[b + 5] = az * em.y;
      em = cmul(em, e);
    }
  }
};

// local node coordinates of one position inside the tile block, with the
// radial multipliers (ghost fold for the a-node, 0 for nodes outside the box
// or, for corrupted positions, outside the block)
template <int TR, int H>
struct Local {
  int na, nb;             // block node index of (ia, j0) and (ib, j0); +1 in z is the next node
  float sa_even, sa_odd, sb;
};

template <int TR, int H>
__device__ __forceinline__ Local<TR, H> localize(const ShapePos& s, const Grid& g, int J0, int C0) {
  using B = Blk<TR, H>;
  Local<TR, H> L;
  int bz = s.j0 - (J0 - H);
  if (bz < 0) bz += g.nz;
  if (bz >= g.nz) bz -= g.nz;
  const bool zok = bz >= 0 && bz + 1 < B::BZ;
  const bool ghost = s.i0 == -1;
  const int ia = ghost ? 0 : s.i0, ib = s.i0 + 1;
  const int ra = ia - (C0 - 1 - H), rb = ib - (C0 - 1 - H);
  const bool aok = zok && ia >= 0 && ia < g.nr && ra >= 0 && ra < B::BR;
  const bool bok = zok && ib < g.nr && rb >= 0 && rb < B::BR;
  L.na = aok ? ra * B::BZ + bz : 0;
  L.nb = bok ? rb * B::BZ + bz : 0;
  L.sa_even = aok ? 1.f : 0.f;
  L.sa_odd = aok ? (ghost ? -1.f : 1.f) : 0.f;
  L.sb = bok ? 1.f : 0.f;
  return L;
}

__device__ __forceinline__ uint32_t pos_key(const ShapePos& s, int nr) {
  const int ic = (s.i0 > nr ? nr : s.i0) + 1;
  return (uint32_t)s.j0 * 2048u + (uint32_t)ic;
}

// Cubic B-spline shape (an option): the four nodes -1 .. 2 of each axis around
// the cell start, weights of the fourfold convolution of the unit box.
__device__ __forceinline__ void cubic_weights(float f, float (&w)[4]) {
  const float g = 1.f - f;
  w[0] = g * g * g * (1.f / 6.f);
  w[1] = (4.f - 6.f * f * f + 3.f * f * f * f) * (1.f / 6.f);
  w[2] = (4.f - 6.f * g * g + 3.f * g * g * g) * (1.f / 6.f);
  w[3] = f * f * f * (1.f / 6.f);
}

// One particle's K values on its 16 cubic nodes, straight into the FP64 block
// (no register runs: sixteen nodes per value would not fit).  Ghost nodes
// -1, -2 across the axis stand for nodes 0, 1 with the factor (-1)^nu of each
// value's Hankel order; nodes at i >= nr are dropped; rows outside the block
// (corrupted positions only) are skipped.
template <int TR, int H, int K, class Set, class OffFn>
__device__ __forceinline__ void cubic_deposit(double* __restrict__ lds, const float (&v)[K], const ShapePos& s,
                                              const Grid& g, int J0, int C0, OffFn off) {
  using B = Blk<TR, H>;
  float wz[4], wr[4];
  cubic_weights(s.fz, wz);
  cubic_weights(s.fr, wr);
  int bz0 = s.j0 - 1 - (J0 - H);
  if (bz0 < 0) bz0 += g.nz;
  if (bz0 >= g.nz) bz0 -= g.nz;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    int i = s.i0 - 1 + a;
    const bool ghost = i < 0;
    if (ghost) i = -1 - i;
    const int br = i - (C0 - 1 - H);
    if (i >= g.nr || br < 0 || br >= B::BR) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int bz = bz0 + b;
      if (bz < 0 || bz >= B::BZ) continue;
      const int node = br * B::BZ + bz;
      const float w = wr[a] * wz[b];
#pragma unroll
      for (int k = 0; k < K; ++k)
        atomicAdd(lds + off(k) + node, (double)((ghost && Set::parity(k) ? -w : w) * v[k]));
    }
  }
}

// Cubic shapes: the particles of one run share the cell of x^{n+1}, hence the
// 4 x 4 nodes of their rho^{n+1} stencil; a lane sums the 16 node weights
// times the K values in registers and adds them to the block once per run
// (cubic_deposit's node mapping, the ghost sign applied at the flush).
template <int K>
struct CubAcc {
  uint32_t key;
  float a[16 * K];
};

struct NoCubAcc {   // linear shapes: no cubic accumulator
  uint32_t key = kInvalidKey;
};

template <int K>
__device__ __forceinline__ void cub_reset(CubAcc<K>& A, uint32_t key) {
  A.key = key;
#pragma unroll
  for (int i = 0; i < 16 * K; ++i) A.a[i] = 0.f;
}

template <int K>
__device__ __forceinline__ void cub_add(CubAcc<K>& A, const float (&v)[K], float fz, float fr) {
  float wz[4], wr[4];
  cubic_weights(fz, wz);
  cubic_weights(fr, wr);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const float w = wr[a] * wz[b];
#pragma unroll
      for (int k = 0; k < K; ++k) A.a[(4 * a + b) * K + k] = fmaf(w, v[k], A.a[(4 * a + b) * K + k]);
    }
}

template <int TR, int H, int K, class Set, class OffFn>
__device__ __forceinline__ void cub_flush(double* __restrict__ lds, const CubAcc<K>& A, const Grid& g, int J0,
                                          int C0, OffFn off) {
  using B = Blk<TR, H>;
  const int j0 = (int)(A.key >> 11), i0 = (int)(A.key & 2047u) - 1;
  int bz0 = j0 - 1 - (J0 - H);
  if (bz0 < 0) bz0 += g.nz;
  if (bz0 >= g.nz) bz0 -= g.nz;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    int i = i0 - 1 + a;
    const bool ghost = i < 0;
    if (ghost) i = -1 - i;
    const int br = i - (C0 - 1 - H);
    if (i >= g.nr || br < 0 || br >= B::BR) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int bz = bz0 + b;
      if (bz < 0 || bz >= B::BZ) continue;
      const int node = br * B::BZ + bz;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const float x = A.a[(4 * a + b) * K + k];
        atomicAdd(lds + off(k) + node, (double)(ghost && Set::parity(k) ? -x : x));
      }
    }
  }
}

// Register accumulator of one position kind: the cell key it belongs to and
// the K values times the four node weights (ia,j0), (ia,j0+1), (ib,j0),
// (ib,j0+1).  A run adds at most a few particles before it is flushed into
// the FP64 block.
template <int K>
struct Acc {
  uint32_t key;
  float a[4 * K];
};

template <int K>
__device__ __forceinline__ void acc_reset(Acc<K>& A, uint32_t key) {
  A.key = key;
#pragma unroll
  for (int i = 0; i < 4 * K; ++i) A.a[i] = 0.f;
}

template <int K>
__device__ __forceinline__ void acc_add(Acc<K>& A, const float (&v)[K], float fz, float fr) {
  const float w0 = (1.f - fz) * (1.f - fr), w1 = fz * (1.f - fr), w2 = (1.f - fz) * fr, w3 = fz * fr;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    A.a[4 * k + 0] += w0 * v[k];
    A.a[4 * k + 1] += w1 * v[k];
    A.a[4 * k + 2] += w2 * v[k];
    A.a[4 * k + 3] += w3 * v[k];
  }
}

// LDS atomics (FP64) of one accumulator at the nodes of its cell key
template <int TR, int H, int K, class Set, class OffFn>
__device__ __forceinline__ void acc_flush(double* __restrict__ lds, const Acc<K>& A, const Grid& g, int J0, int C0,
                                          OffFn off) {
  ShapePos s;
  s.j0 = (int)(A.key >> 11);
  s.i0 = (int)(A.key & 2047u) - 1;
  const Local<TR, H> L = localize<TR, H>(s, g, J0, C0);
  if (L.sb != 0.f) {
    double* pb = lds + L.nb;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int o = off(k);
      atomicAdd(pb + o, (double)A.a[4 * k + 2]);
      atomicAdd(pb + o + 1, (double)A.a[4 * k + 3]);
    }
  }
  if (L.sa_even != 0.f) {
    double* pa = lds + L.na;
    const float sg = L.sa_odd;   // -1 on the ghost node across the axis (odd Hankel orders)
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int o = off(k);
      atomicAdd(pa + o, (double)(Set::parity(k) ? sg * A.a[4 * k + 0] : A.a[4 * k + 0]));
      atomicAdd(pa + o + 1, (double)(Set::parity(k) ? sg * A.a[4 * k + 1] : A.a[4 * k + 1]));
    }
  }
}

// one position of one particle: flush the accumulator if the cell changed,
// then add the node contributions.  The restart after a flush is folded into
// the accumulation (old sums times 0 or 1): with no branch rewriting the
// accumulators, the compiler keeps them in one register set instead of copying
// them around the particle loop.
template <int TR, int H, int K, class Set, class OffFn>
__device__ __forceinline__ void acc_step(double* __restrict__ lds, Acc<K>& A, uint32_t key, const float (&v)[K],
                                         const ShapePos& s, const Grid& g, int J0, int C0, OffFn off) {
  const bool change = key != A.key;
  if (change && A.key != kInvalidKey) acc_flush<TR, H, K, Set>(lds, A, g, J0, C0, off);
  const float keep = change ? 0.f : 1.f;
  A.key = key;
  const float fz = s.fz, fr = s.fr;
  const float w0 = (1.f - fz) * (1.f - fr), w1 = fz * (1.f - fr), w2 = (1.f - fz) * fr, w3 = fz * fr;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    A.a[4 * k + 0] = fmaf(w0, v[k], A.a[4 * k + 0] * keep);
    A.a[4 * k + 1] = fmaf(w1, v[k], A.a[4 * k + 1] * keep);
    A.a[4 * k + 2] = fmaf(w2, v[k], A.a[4 * k + 2] * keep);
    A.a[4 * k + 3] = fmaf(w3, v[k], A.a[4 * k + 3] * keep);
  }
}

// Two accumulators for one position kind (the current J^{n+1/2}): the
// particles of one x^{n+1} cell have their x^{n+1/2} in at most a few cells
// (the run's cell and a neighbour the faster particles crossed from), so a
// particle goes to the slot holding its cell and a flush happens only when a
// third cell appears (then the slot not hit last is flushed and reused).
// Each slot adds w times the values with w = 0 or 1, so both slots stay in
// one register set without branches.
template <int K>
struct Acc2 {
  Acc<K> a, b;
  bool last_b;   // the last particle went to slot b
};

template <int TR, int H, int K, class Set, class OffFn>
__device__ __forceinline__ void acc2_step(double* __restrict__ lds, Acc2<K>& A, uint32_t key, const float (&v)[K],
                                          const ShapePos& s, const Grid& g, int J0, int C0, OffFn off) {
  const bool hit_a = key == A.a.key, hit_b = key == A.b.key;
  if (!hit_a && !hit_b) {
    // a third cell: flush the slot not hit last and give it this cell
    Acc<K>& victim = A.last_b ? A.a : A.b;
    if (victim.key != kInvalidKey) acc_flush<TR, H, K, Set>(lds, victim, g, J0, C0, off);
    acc_reset(victim, key);
  }
  const bool to_b = key == A.b.key;
  A.last_b = to_b;
  const float fb = to_b ? 1.f : 0.f, fa = 1.f - fb;
  const float fz = s.fz, fr = s.fr;
  const float w0 = (1.f - fz) * (1.f - fr), w1 = fz * (1.f - fr), w2 = (1.f - fz) * fr, w3 = fz * fr;
  const float a0 = fa * w0, a1 = fa * w1, a2 = fa * w2, a3 = fa * w3;
  const float b0 = fb * w0, b1 = fb * w1, b2 = fb * w2, b3 = fb * w3;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    A.a.a[4 * k + 0] = fmaf(a0, v[k], A.a.a[4 * k + 0]);
    A.a.a[4 * k + 1] = fmaf(a1, v[k], A.a.a[4 * k + 1]);
    A.a.a[4 * k + 2] = fmaf(a2, v[k], A.a.a[4 * k + 2]);
    A.a.a[4 * k + 3] = fmaf(a3, v[k], A.a.a[4 * k + 3]);
    A.b.a[4 * k + 0] = fmaf(b0, v[k], A.b.a[4 * k + 0]);
    A.b.a[4 * k + 1] = fmaf(b1, v[k], A.b.a[4 * k + 1]);
    A.b.a[4 * k + 2] = fmaf(b2, v[k], A.b.a[4 * k + 2]);
    A.b.a[4 * k + 3] = fmaf(b3, v[k], A.b.a[4 * k + 3]);
  }
}

// one particle's deposit inputs
struct PLoad {
  double x = 0.0, y = 0.0, z = 0.0, uz = 0.0;
  float ux = 0.f, uy = 0.f, w = 0.f;
  __device__ __forceinline__ void load(const Parts& p, int i) {
    x = p.x[i];
    y = p.y[i];
    z = p.z[i];
    uz = p.uz[i];
    ux = p.ux[i];
    uy = p.uy[i];
    w = p.w[i];
  }
};

// number of rho values per node (mode 0 real, complex from mode 1 on)
template <int M>
struct RhoVals {
  static constexpr int N = 1 + 2 * (M - 1);
};

// What a launch of the tile kernel deposits:
//   kDepFull   rho^n, J^{n+1/2} and rho^{n+1} of every work item;
//   kDepCarry  J^{n+1/2} and rho^{n+1} only: rho^n is the previous step's
//              rho^{n+1} carried over (the same particles at the same
//              positions), re-deposited only in the edge tiles (kDepEdgeRho);
//   kDepEdgeRho rho^n of the two tile rows at the ends of the window along z
//              (one workgroup per tile, all its particles), written into the
//              rho^n part of the tile's first slot after kDepCarry: these
//              hold the nodes the window move changes (particles that left
//              behind the window, the column injected at the head);
//   kDepIon    set-up of the immobile background: FP64 rho^{n+1} blocks.
enum DepMode { kDepFull = 0, kDepCarry = 1, kDepEdgeRho = 2, kDepIon = 3 };

// Otherwise the first work item of each tile adds the tile's FP64 background
// block `ionblk` (when given) to the densities it deposits.
template <int TR, int H, int M, int MODE, int SHAPE>
__global__ __launch_bounds__(256) void k_deposit(Parts p, const int* __restrict__ offset,
                                                 const int* __restrict__ nchunk, const int* __restrict__ chunk_start,
                                                 float* __restrict__ scratch, const double* __restrict__ ionblk, Grid g,
                                                 TileGeom tg, DevState* st) {
  using B = Blk<TR, H>;
  using RS = RhoSet<M, B::NODES>;
  using JS = JSet<M, B::NODES>;
  constexpr bool kRhoN = MODE == kDepFull || MODE == kDepEdgeRho || MODE == kDepIon;
  constexpr bool kRho1J = MODE != kDepEdgeRho;
  extern __shared__ double lds[];
  constexpr int nacc = Vals<M>::N * B::NODES;
  constexpr int kCells = kTZ * TR;   // cells (key columns x rows) of a tile
  __shared__ int rowstart[kTZ];      // sorted index of each tile row's first particle
  __shared__ int rowpref[kTZ + 1];   // tile-local index of each row's first particle
  __shared__ uint16_t runpref[kCells + 1];   // runs of <= kRun particles before each cell
  __shared__ int wsum[4];
  __shared__ int s_tile;
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  if (MODE != kDepIon && MODE != kDepEdgeRho && b == 0 && tid == 0) {
    st->n_part = st->n_live;
    if (chunk_start[tg.ntiles] > (int)gridDim.x) st->overflow = 2;   // work list larger than the launch
  }
  if (MODE == kDepEdgeRho) {
    // edge tiles: tz = 0 and tz = ntz - 1 of every radial tile column
    if (tid == 0) s_tile = (b >> 1) * tg.ntz + ((b & 1) ? tg.ntz - 1 : 0);
  } else {
    if (b >= chunk_start[tg.ntiles]) return;   // uniform per workgroup
    if (tid == 0) {
      int lo = 0, hi = tg.ntiles;   // chunk_start[lo] <= b < chunk_start[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (chunk_start[mid] <= b) lo = mid;
        else hi = mid;
      }
      s_tile = lo;
    }
  }
  for (int e = tid; e < nacc; e += blockDim.x) lds[e] = 0.0;
  __syncthreads();
  const int t = s_tile;
  const int chunk = MODE == kDepEdgeRho ? 0 : b - chunk_start[t];
  const int J0 = (t % tg.ntz) * kTZ, C0 = (t / tg.ntz) * TR;
  const int C1 = min(C0 + TR, g.ncol);
  if (tid < kTZ) {
    const int j = J0 + tid;
    const int a = offset[j * g.ncol + C0];
    rowstart[tid] = a;
    rowpref[tid + 1] = offset[j * g.ncol + C1] - a;
  }
  __syncthreads();
  if (tid == 0) {
    rowpref[0] = 0;
    for (int r = 1; r <= kTZ; ++r) rowpref[r] += rowpref[r - 1];
  }
  __syncthreads();
  const int total = rowpref[kTZ];
  const double zmin = st->zmin;
  const double dt = g.dt;
  // Particle range of this work item: one chunk of a dense tile, or the whole
  // tile.  The edge pass takes its whole tile in pieces of one chunk.
  const int npiece = MODE == kDepEdgeRho ? max(1, (total + tg.chunk - 1) / tg.chunk) : 1;
  int f0 = 0, f1 = total;
  if (MODE != kDepEdgeRho && nchunk[t] != 1) {
    f0 = chunk * tg.chunk;
    f1 = min(total, f0 + tg.chunk);
  }
  Acc<RS::K> An, A1;
  Acc2<JS::K> AJ;
  std::conditional_t<SHAPE == 3, CubAcc<RS::K>, NoCubAcc> Cb;   // cubic shapes: rho^{n+1} of the run
  if constexpr (SHAPE == 3) cub_reset(Cb, kInvalidKey);
  acc_reset(An, kInvalidKey);
  acc_reset(A1, kInvalidKey);
  acc_reset(AJ.a, kInvalidKey);
  acc_reset(AJ.b, kInvalidKey);
  AJ.last_b = true;
  for (int piece = 0; piece < npiece; ++piece) {
    if (MODE == kDepEdgeRho) {
      f0 = piece * tg.chunk;
      f1 = min(total, f0 + tg.chunk);
    }
    // Runs: every cell's particles (clipped to [f0, f1)) are cut into runs of
    // at most kRun, so a run never leaves its cell of x^{n+1}; runpref is the
    // exclusive prefix of the run counts over the tile's cells.
    auto cell_range = [&](int c, int& lo, int& hi) {
      const int row = c / TR, col = c % TR;
      lo = hi = 0;
      if (C0 + col < C1) {
        const int* o = offset + (J0 + row) * g.ncol + C0 + col;
        lo = max(f0, rowpref[row] + (o[0] - rowstart[row]));
        hi = min(f1, rowpref[row] + (o[1] - rowstart[row]));
      }
    };
    __syncthreads();   // the previous piece's table is no longer read
    {
      static_assert(kCells % 256 == 0 && kCells <= 512, "tile cells per thread");
      constexpr int per = kCells / 256;
      int nrun[per], tot = 0;
#pragma unroll
      for (int q = 0; q < per; ++q) {
        int lo, hi;
        cell_range(tid * per + q, lo, hi);
        nrun[q] = hi > lo ? (hi - lo + kRun - 1) / kRun : 0;
        tot += nrun[q];
      }
      // block-wide exclusive scan of the per-thread totals
      const int lane = tid & 63, wave = tid >> 6;
      int inc = tot;
      for (int d = 1; d < 64; d <<= 1) {
        const int u = __shfl_up(inc, d, 64);
        if (lane >= d) inc += u;
      }
      if (lane == 63) wsum[wave] = inc;
      __syncthreads();
      int excl = inc - tot;
      for (int w = 0; w < wave; ++w) excl += wsum[w];
#pragma unroll
      for (int q = 0; q < per; ++q) {
        runpref[tid * per + q] = (uint16_t)excl;
        excl += nrun[q];
      }
      if (tid == 255) runpref[kCells] = (uint16_t)excl;
      __syncthreads();
    }
    const int nruns = runpref[kCells];
    // Round r0: thread tid takes run r0 + tid.  All lanes start their runs
    // together, so the rho^{n+1} accumulator (whose cell is the run's cell)
    // flushes at most once per round; J keeps two cells (the cells its
    // half-step positions fall in) and flushes one only when a third appears;
    // rho^n flushes when its cell changes.  A lane keeps its accumulators
    // across rounds (a beam cell with thousands of particles gives one lane
    // consecutive runs of one cell).
    for (int r0 = 0; r0 < nruns; r0 += 256) {
      const int r = r0 + tid;
      int len = 0, idx0 = 0;
      uint32_t rkey = SHAPE == 3 ? Cb.key : A1.key;
      if (r < nruns) {
        int lo = 0, hi = kCells;   // runpref[lo] <= r < runpref[hi]
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if ((int)runpref[mid] <= r) lo = mid;
          else hi = mid;
        }
        int a, e;
        cell_range(lo, a, e);
        const int start = a + (r - (int)runpref[lo]) * kRun;
        len = min(kRun, e - start);
        const int row = lo / TR, col = lo % TR;
        idx0 = rowstart[row] + (start - rowpref[row]);
        rkey = (uint32_t)(J0 + row) * 2048u + (uint32_t)(C0 + col);
      }
      if constexpr (SHAPE == 3) {
        if (kRho1J && rkey != Cb.key) {
          if (Cb.key != kInvalidKey)
            cub_flush<TR, H, RS::K, RS>(lds, Cb, g, J0, C0, [](int k) { return RS::off(4, k); });
          cub_reset(Cb, rkey);
        }
      } else if (kRho1J && rkey != A1.key) {
        if (A1.key != kInvalidKey)
          acc_flush<TR, H, RS::K, RS>(lds, A1, g, J0, C0, [](int k) { return RS::off(4, k); });
        acc_reset(A1, rkey);
      }
      // particle data of the next iteration is loaded before the current one
      // is processed, so its latency overlaps the arithmetic
      PLoad nx;
      if (len > 0) nx.load(p, idx0);
      for (int it = 0; it < kRun; ++it) {
        const bool valid = it < len;
        const PLoad cur = nx;
        if (it + 1 < len) nx.load(p, idx0 + it + 1);
        double x = 0.0, y = 0.0, z = zmin;
        float ux = 0.f, uy = 0.f, uz = 0.f, qw = 0.f;
        if (valid) {
          x = cur.x;
          y = cur.y;
          z = cur.z;
          ux = cur.ux;
          uy = cur.uy;
          uz = (float)cur.uz;
          qw = cur.w;
        }
        const bool cold = __ballot(valid && (ux != 0.f || uy != 0.f || uz != 0.f)) == 0;
        const float ginv = 1.f / sqrtf(1.f + ux * ux + uy * uy + uz * uz);
        const float vx = ux * ginv, vy = uy * ginv, vz = uz * ginv;
        if constexpr (SHAPE == 3) {
          // cubic shapes: every position of the particle straight into the block
          if (valid) {
            if (kRho1J) {
              const ShapePos s = shape_at(x, y, z, zmin, g);
              float v[RS::K];
              RS::values(qw, s.eith, v);
              // the run's cell fixes the stencil, except in the last key
              // column, which also holds particles beyond the last node
              if ((Cb.key & 2047u) < (uint32_t)g.nr) cub_add(Cb, v, s.fz, s.fr);
              else cubic_deposit<TR, H, RS::K, RS>(lds, v, s, g, J0, C0, [](int k) { return RS::off(4, k); });
              const ShapePos sh = shape_at(x - 0.5 * dt * (double)vx, y - 0.5 * dt * (double)vy,
                                           z - 0.5 * dt * (double)vz, zmin, g);
              float vj[JS::K];
              JS::values(qw, vx, vy, vz, sh.eith, vj);
              cubic_deposit<TR, H, JS::K, JS>(lds, vj, sh, g, J0, C0, [](int k) { return JS::off(k); });
            }
            if (kRhoN) {
              const ShapePos s0 = shape_at(x - dt * (double)vx, y - dt * (double)vy, z - dt * (double)vz, zmin, g);
              float v[RS::K];
              RS::values(qw, s0.eith, v);
              cubic_deposit<TR, H, RS::K, RS>(lds, v, s0, g, J0, C0, [](int k) { return RS::off(3, k); });
            }
          }
          continue;
        }
        // rho^{n+1} at x^{n+1}, in the run's cell (particles beyond the last
        // radial node share the last key column and deposit nothing); rho^n
        // too when the whole wave is at rest
        if (kRho1J || cold) {
          const ShapePos s = shape_at(x, y, z, zmin, g);
          const uint32_t key = pos_key(s, g.nr);
          float v[RS::K];
          RS::values(valid && s.i0 < g.nr ? qw : 0.f, s.eith, v);
          if (kRho1J) acc_add(A1, v, s.fz, s.fr);
          if (cold) {
            if (kRhoN) {
              const uint32_t key0 = valid ? key : An.key;
              acc_step<TR, H, RS::K, RS>(lds, An, key0, v, s, g, J0, C0, [](int k) { return RS::off(3, k); });
            }
            continue;
          }
        }
        // J^{n+1/2} at x^{n+1/2} = x^{n+1} - dt v / 2
        if (kRho1J) {
          const ShapePos s = shape_at(x - 0.5 * dt * (double)vx, y - 0.5 * dt * (double)vy,
                                      z - 0.5 * dt * (double)vz, zmin, g);
          const uint32_t key = valid ? pos_key(s, g.nr) : (AJ.last_b ? AJ.b.key : AJ.a.key);
          float v[JS::K];
          JS::values(valid ? qw : 0.f, vx, vy, vz, s.eith, v);
          acc2_step<TR, H, JS::K, JS>(lds, AJ, key, v, s, g, J0, C0, [](int k) { return JS::off(k); });
        }
        // rho^n at x^n = x^{n+1} - dt v
        if (kRhoN) {
          const ShapePos s = shape_at(x - dt * (double)vx, y - dt * (double)vy, z - dt * (double)vz, zmin, g);
          const uint32_t key = valid ? pos_key(s, g.nr) : An.key;
          float v[RS::K];
          RS::values(valid ? qw : 0.f, s.eith, v);
          acc_step<TR, H, RS::K, RS>(lds, An, key, v, s, g, J0, C0, [](int k) { return RS::off(3, k); });
        }
      }
    }
  }   // pieces
  if (kRho1J) {
    if constexpr (SHAPE == 3) {
      if (Cb.key != kInvalidKey) cub_flush<TR, H, RS::K, RS>(lds, Cb, g, J0, C0, [](int k) { return RS::off(4, k); });
    }
    if (A1.key != kInvalidKey) acc_flush<TR, H, RS::K, RS>(lds, A1, g, J0, C0, [](int k) { return RS::off(4, k); });
    if (AJ.a.key != kInvalidKey) acc_flush<TR, H, JS::K, JS>(lds, AJ.a, g, J0, C0, [](int k) { return JS::off(k); });
    if (AJ.b.key != kInvalidKey) acc_flush<TR, H, JS::K, JS>(lds, AJ.b, g, J0, C0, [](int k) { return JS::off(k); });
  }
  if (kRhoN && An.key != kInvalidKey) acc_flush<TR, H, RS::K, RS>(lds, An, g, J0, C0, [](int k) { return RS::off(3, k); });
  __syncthreads();
  constexpr int nr_vals = RhoVals<M>::N;
  if (MODE == kDepIon) {
    double* dst = reinterpret_cast<double*>(scratch) + (size_t)b * nr_vals * B::NODES;
    for (int e = tid; e < nr_vals * B::NODES; e += blockDim.x) {
      const int k = e / B::NODES, node = e % B::NODES;
      dst[e] = lds[RS::off(4, k) + node];
    }
    return;
  }
  if (ionblk && chunk == 0) {
    // the tile's background, once per tile, in FP64, into the densities this
    // launch deposits
    const double* src = ionblk + (size_t)t * nr_vals * B::NODES;
    for (int e = tid; e < nr_vals * B::NODES; e += blockDim.x) {
      const int k = e / B::NODES, node = e % B::NODES;
      const double v = src[e];
      if (kRhoN) lds[RS::off(3, k) + node] += v;
      if (kRho1J) lds[RS::off(4, k) + node] += v;
    }
    __syncthreads();
  }
  if (MODE == kDepEdgeRho) {
    // only the rho^n part of the tile's first slot (the rest is the carry launch's)
    float* dst = scratch + (size_t)chunk_start[t] * nacc;
    for (int e = tid; e < nr_vals * B::NODES; e += blockDim.x) {
      const int k = e / B::NODES, node = e % B::NODES;
      dst[RS::off(3, k) + node] = (float)lds[RS::off(3, k) + node];
    }
    return;
  }
  float* dst = scratch + (size_t)b * nacc;
  for (int e = tid; e < nacc; e += blockDim.x) dst[e] = (float)lds[e];
}

// ---------------------------------------------------------------------------
// Steady-state deposit (J^{n+1/2} and rho^{n+1}; rho^n carried over), linear
// shapes: four lanes per run of at most kRun particles of one cell, lane q
// taking particles q and q + 4 of it.  The runs of a round are consecutive in
// memory, so a wavefront's loads stay within a few lines.  A lane sums its
// particles' node contributions in registers, node-major (slot s of K values:
// node s ^ q of the cell), and the four lanes then sum over the group by a
// reduce-scatter (two exchange steps, each halving what a lane keeps), after
// which lane q holds every value of node q and issues their FP64 LDS atomics
// at offsets known at compile time.
//   * rho^{n+1}: every particle of a run is in the run's cell;
//   * J^{n+1/2}: particles whose half-step cell is the run's cell join its
//     sums; of the others, those in the cell of the group's first such
//     particle are summed into a second set; any further cell deposits
//     particle by particle.
// ---------------------------------------------------------------------------
constexpr int kLPR = 4;              // lanes per run: one per node of the cell
constexpr int kPPL = kRun / kLPR;    // particles per lane and run

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}

// one exchange step over the first N entries: the lane keeps the lower half
// and adds the partner's upper half to it
template <int N, int CTRL, int CAP>
__device__ __forceinline__ void rs_step(float (&a)[CAP]) {
#pragma unroll
  for (int i = 0; i < N / 2; ++i) a[i] += dpp_mov<CTRL>(a[N / 2 + i]);
}

// Sum over the four lanes of a group of node-major entries (four nodes of K
// values) that lane q keeps in slots rotated by q: slot s holds node s ^ q.
// Step one (partner q ^ 2): slots 0, 1 of lane q and slots 2, 3 of its
// partner hold the same two nodes, q and q ^ 1; step two (partner q ^ 1): slot
// 0 of lane q and slot 1 of its partner hold node q.  No step depends on the
// lane, and lane q ends with the sums of node q in a[0 .. K).
template <int N>
__device__ __forceinline__ void reduce_scatter4(float (&a)[N]) {
  static_assert(N % 4 == 0 && kLPR == 4, "four lanes per run, one node per lane");
  rs_step<N, 0x4E>(a);       // partner q ^ 2
  rs_step<N / 2, 0xB1>(a);   // partner q ^ 1
}

// the four node weights of a position in lane q's rotated slots: slot s gets
// the weight of node s ^ q (bit 0 of a node: z + 1, bit 1: the outer radial node)
__device__ __forceinline__ void rotated_weights(float fz, float fr, int q, float scale, float (&w)[4]) {
  const float z0 = (q & 1) ? fz : 1.f - fz, z1 = (q & 1) ? 1.f - fz : fz;
  const float r0 = (q & 2) ? fr : 1.f - fr, r1 = (q & 2) ? 1.f - fr : fr;
  w[0] = scale * z0 * r0;
  w[1] = scale * z1 * r0;
  w[2] = scale * z0 * r1;
  w[3] = scale * z1 * r1;
}

// The position kinds of the lane-group kernel.  kDepCarry: rho^{n+1} at
// x^{n+1} (always the run's cell) and the split set J^{n+1/2} at x^{n+1/2};
// kDepEdgeRho: only the split set rho^n at x^n.
template <int M, int NODES, int MODE>
struct LaneSets {
  using RS = RhoSet<M, NODES>;
  using JS = JSet<M, NODES>;
  static constexpr bool kEdge = MODE == kDepEdgeRho;
  static constexpr int KR = kEdge ? 0 : RS::K;   // values that always go to the run's cell
  static constexpr int KS = kEdge ? RS::K : JS::K;   // values of the split set
  static __device__ __forceinline__ constexpr int split_off(int k) { return kEdge ? RS::off(3, k) : JS::off(k); }
  static __device__ __forceinline__ constexpr int split_parity(int k) {
    return kEdge ? RS::parity(k) : JS::parity(k);
  }
};

// FP64 LDS atomics of node q of the cell `key` (q = 0, 1: the inner radial
// node at j0, j0 + 1; q = 2, 3: the outer one) from lane q's reduced values
// a[0 .. KN): the values that always go to the run's cell first when
// kAlways, then those of the split set.
template <int TR, int H, int M, int MODE, bool kAlways, int N>
__device__ __forceinline__ void flush_node(double* __restrict__ lds, const float (&a)[N], uint32_t key,
                                          const Grid& g, int J0, int C0, int q) {
  using B = Blk<TR, H>;
  using RS = RhoSet<M, B::NODES>;
  using LS = LaneSets<M, B::NODES, MODE>;
  constexpr int NR = kAlways ? LS::KR : 0;
  constexpr int KN = NR + LS::KS;
  static_assert(N == 4 * KN, "node-major entries");
  ShapePos s;
  s.j0 = (int)(key >> 11);
  s.i0 = (int)(key & 2047u) - 1;
  const Local<TR, H> L = localize<TR, H>(s, g, J0, C0);
  const bool outer = q >= 2;
  if ((outer ? L.sb : L.sa_even) == 0.f) return;
  double* __restrict__ base = lds + (outer ? L.nb : L.na) + (q & 1);
  const float sg = outer ? 1.f : L.sa_odd;   // -1 on the ghost node across the axis (odd Hankel orders)
#pragma unroll
  for (int k = 0; k < KN; ++k) {
    const bool always = k < NR;
    const int off = always ? RS::off(4, k) : LS::split_off(k - NR);
    const bool par = always ? RS::parity(k) : LS::split_parity(k - NR);
    atomicAdd(base + off, (double)(par ? sg * a[k] : a[k]));
  }
}

// what a particle keeps of its split-set position for the second cell and
// the particle-by-particle atomics
template <int K>
struct LaneSplit {
  float fz, fr;            // position within its cell
  uint32_t key;            // its cell key
  float v[K];
};

// One pass of the lane-group deposit over the particles of a tile.
// kDepCarry: J^{n+1/2} and rho^{n+1} of the work item's particles [f0, f1);
// kDepEdgeRho: rho^n of all the tile's particles, in pieces of one chunk.
// Sums into the FP64 block `lds`; the tile's row table is already in LDS.
template <int TR, int H, int M, int MODE, int NT>
__device__ __forceinline__ void lane_pass(const Parts& p, const int* __restrict__ offset, const Grid& g,
                                          const TileGeom& tg, double* __restrict__ lds, const int* rowstart,
                                          const int* rowpref, uint16_t* runpref, int* cfirst, int* ccount,
                                          int* wsum, int J0, int C0, int C1, int f0, int f1, int total,
                                          double zmin) {
  using B = Blk<TR, H>;
  using RS = RhoSet<M, B::NODES>;
  using JS = JSet<M, B::NODES>;
  using LS = LaneSets<M, B::NODES, MODE>;
  static_assert(MODE == kDepCarry || MODE == kDepEdgeRho, "steady-state modes");
  constexpr bool kEdge = LS::kEdge;
  constexpr int kCells = kTZ * TR;
  constexpr int kGroups = NT / kLPR;          // runs per round
  constexpr int KA = LS::KR + LS::KS;         // values per node, run cell
  constexpr int KB = LS::KS;                  // values per node, second cell
  constexpr uint32_t kGroupMask = (1u << kLPR) - 1u;
  const int tid = threadIdx.x;
  const double dt = g.dt;
  const int q = tid & (kLPR - 1);
  const int lane = tid & 63, gbase = lane & ~(kLPR - 1);
  const int npiece = kEdge ? max(1, (total + tg.chunk - 1) / tg.chunk) : 1;
  for (int piece = 0; piece < npiece; ++piece) {
    if (kEdge) {
      f0 = piece * tg.chunk;
      f1 = min(total, f0 + tg.chunk);
    }
    __syncthreads();   // the previous piece's table is no longer read
    {
      // cells of the piece, their runs of at most kRun, and the exclusive
      // prefix of the run counts
      static_assert(kCells % NT == 0 || NT % kCells == 0, "tile cells per thread");
      constexpr int per = kCells >= NT ? kCells / NT : 1;
      int nrun[per], tot = 0;
#pragma unroll
      for (int qq = 0; qq < per; ++qq) {
        const int c = tid * per + qq;
        nrun[qq] = 0;
        if (c < kCells) {
          const int row = c / TR, col = c % TR;
          int lo = 0, hi = 0;
          if (C0 + col < C1) {
            const int* o = offset + (J0 + row) * g.ncol + C0 + col;
            lo = max(f0, rowpref[row] + (o[0] - rowstart[row]));
            hi = min(f1, rowpref[row] + (o[1] - rowstart[row]));
          }
          const int n = hi > lo ? hi - lo : 0;
          cfirst[c] = rowstart[row] + (lo - rowpref[row]);
          ccount[c] = n;
          nrun[qq] = (n + kRun - 1) / kRun;
        }
        tot += nrun[qq];
      }
      const int wave = tid >> 6;
      int inc = tot;
      for (int d = 1; d < 64; d <<= 1) {
        const int u = __shfl_up(inc, d, 64);
        if (lane >= d) inc += u;
      }
      if (lane == 63) wsum[wave] = inc;
      __syncthreads();
      int excl = inc - tot;
      for (int w = 0; w < wave; ++w) excl += wsum[w];
#pragma unroll
      for (int qq = 0; qq < per; ++qq) {
        if (tid * per + qq < kCells) runpref[tid * per + qq] = (uint16_t)excl;
        excl += nrun[qq];
      }
      if (tid == NT - 1) runpref[kCells] = (uint16_t)excl;
      __syncthreads();
    }
    const int nruns = runpref[kCells];
    // lane q of the group taking run r: the sorted index of its first
    // particle (q of the run; the others follow kLPR apart), how many of its
    // kPPL particles exist, and the run's cell key (kInvalidKey past the last
    // run)
    auto slot_of = [&](int r, int& idx, int& cnt, uint32_t& key) {
      idx = 0;
      cnt = 0;
      key = kInvalidKey;
      if (r >= nruns) return;
      int lo = 0, hi = kCells;   // runpref[lo] <= r < runpref[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((int)runpref[mid] <= r) lo = mid;
        else hi = mid;
      }
      const int k = (r - (int)runpref[lo]) * kRun + q;
      const int left = ccount[lo] - k;   // particles of the cell from this lane's first on
      cnt = left <= 0 ? 0 : min(kPPL, (left + kLPR - 1) / kLPR);
      idx = cfirst[lo] + k;
      key = (uint32_t)(J0 + lo / TR) * 2048u + (uint32_t)(C0 + lo % TR);
    };
    int nidx, ncnt;
    uint32_t nkey;
    slot_of(tid / kLPR, nidx, ncnt, nkey);
    PLoad nx[kPPL];
#pragma unroll
    for (int h = 0; h < kPPL; ++h)
      if (h < ncnt) nx[h].load(p, nidx + h * kLPR);
    for (int r0 = 0; r0 < nruns; r0 += kGroups) {
      const int cnt = ncnt;
      const uint32_t rkey = nkey;
      PLoad cur[kPPL];
#pragma unroll
      for (int h = 0; h < kPPL; ++h) cur[h] = nx[h];
      if (r0 + kGroups < nruns) {
        slot_of(r0 + kGroups + tid / kLPR, nidx, ncnt, nkey);
#pragma unroll
        for (int h = 0; h < kPPL; ++h)
          if (h < ncnt) nx[h].load(p, nidx + h * kLPR);
      }
      // the run's cell: the values that always go there (rho^{n+1}) and the
      // split-set values of the particles whose position is in it, summed in
      // registers over the lane's particles
      float X[4 * KA];
#pragma unroll
      for (int e = 0; e < 4 * KA; ++e) X[e] = 0.f;
      LaneSplit<LS::KS> P[kPPL];
      bool inA[kPPL];
      uint32_t outA[kPPL];
#pragma unroll
      for (int h = 0; h < kPPL; ++h) {
        const bool valid = h < cnt;
        double x = 0.0, y = 0.0, z = zmin;
        float ux = 0.f, uy = 0.f, uz = 0.f, qw = 0.f;
        if (valid) {
          x = cur[h].x;
          y = cur[h].y;
          z = cur[h].z;
          ux = cur[h].ux;
          uy = cur[h].uy;
          uz = (float)cur[h].uz;
          qw = cur[h].w;
        }
        const float ginv = 1.f / sqrtf(1.f + ux * ux + uy * uy + uz * uz);
        const float vx = ux * ginv, vy = uy * ginv, vz = uz * ginv;
        ShapePos sp;
        if constexpr (kEdge) {
          // rho^n at x^n = x^{n+1} - dt v
          sp = shape_at(x - dt * (double)vx, y - dt * (double)vy, z - dt * (double)vz, zmin, g);
          RS::values(qw, sp.eith, P[h].v);
        } else {
          // rho^{n+1} at x^{n+1}, in the run's cell (particles beyond the
          // last radial node share the last key column and deposit nothing)
          const ShapePos s = shape_at(x, y, z, zmin, g);
          float vr[RS::K];
          RS::values(valid && s.i0 < g.nr ? qw : 0.f, s.eith, vr);
          float rz[4];
          rotated_weights(s.fz, s.fr, q, 1.f, rz);
#pragma unroll
          for (int k = 0; k < RS::K; ++k)
#pragma unroll
            for (int n = 0; n < 4; ++n) X[n * KA + k] = fmaf(rz[n], vr[k], X[n * KA + k]);
          // J^{n+1/2} at x^{n+1/2} = x^{n+1} - dt v / 2
          sp = shape_at(x - 0.5 * dt * (double)vx, y - 0.5 * dt * (double)vy, z - 0.5 * dt * (double)vz, zmin, g);
          JS::values(qw, vx, vy, vz, sp.eith, P[h].v);
        }
        P[h].fz = sp.fz;
        P[h].fr = sp.fr;
        P[h].key = pos_key(sp, g.nr);
        inA[h] = !valid || P[h].key == rkey;
        outA[h] = (uint32_t)(__ballot(!inA[h]) >> gbase) & kGroupMask;
        float wz[4];
        rotated_weights(sp.fz, sp.fr, q, inA[h] ? 1.f : 0.f, wz);
#pragma unroll
        for (int k = 0; k < LS::KS; ++k)
#pragma unroll
          for (int n = 0; n < 4; ++n) X[n * KA + LS::KR + k] = fmaf(wz[n], P[h].v[k], X[n * KA + LS::KR + k]);
      }
      reduce_scatter4(X);
      if (rkey != kInvalidKey) flush_node<TR, H, M, MODE, true>(lds, X, rkey, g, J0, C0, q);
      // the group's second cell: that of its first particle outside the
      // run's cell, in lane order, then particle order
      uint32_t any = 0;
#pragma unroll
      for (int h = 0; h < kPPL; ++h) any |= outA[h];
      const int first = any ? __ffs(any) - 1 : 0;
      uint32_t kB = kInvalidKey;
      {
        bool taken = false;
#pragma unroll
        for (int h = 0; h < kPPL; ++h) {
          const uint32_t kk = (uint32_t)__shfl((int)P[h].key, gbase + first, 64);
          if (!taken && ((outA[h] >> first) & 1u)) {
            kB = kk;
            taken = true;
          }
        }
      }
      bool inB[kPPL];
      bool anyB = false;
#pragma unroll
      for (int h = 0; h < kPPL; ++h) {
        inB[h] = !inA[h] && P[h].key == kB;
        anyB = anyB || inB[h];
        if (!inA[h] && !inB[h]) {
          // a third cell in the group: this particle's own atomics
          Acc<LS::KS> R;
          R.key = P[h].key;
          const float fz = P[h].fz, fr = P[h].fr;
          const float wz[4] = {(1.f - fz) * (1.f - fr), fz * (1.f - fr), (1.f - fz) * fr, fz * fr};
#pragma unroll
          for (int k = 0; k < LS::KS; ++k)
#pragma unroll
            for (int n = 0; n < 4; ++n) R.a[4 * k + n] = wz[n] * P[h].v[k];
          if constexpr (kEdge)
            acc_flush<TR, H, LS::KS, RS>(lds, R, g, J0, C0, [](int k) { return RS::off(3, k); });
          else
            acc_flush<TR, H, LS::KS, JS>(lds, R, g, J0, C0, [](int k) { return JS::off(k); });
        }
      }
      const uint64_t bmask = __ballot(anyB);
      if (bmask) {   // uniform over the wavefront
        float Y[4 * KB];
#pragma unroll
        for (int e = 0; e < 4 * KB; ++e) Y[e] = 0.f;
#pragma unroll
        for (int h = 0; h < kPPL; ++h) {
          float wz[4];
          rotated_weights(P[h].fz, P[h].fr, q, inB[h] ? 1.f : 0.f, wz);
#pragma unroll
          for (int k = 0; k < KB; ++k)
#pragma unroll
            for (int n = 0; n < 4; ++n) Y[n * KB + k] = fmaf(wz[n], P[h].v[k], Y[n * KB + k]);
        }
        reduce_scatter4(Y);
        if ((bmask >> gbase) & kGroupMask) flush_node<TR, H, M, MODE, false>(lds, Y, kB, g, J0, C0, q);
      }
    }
  }   // pieces
}

// The steady-state deposit, one workgroup per work item (NT threads): the
// pass of kDepCarry over the item's particles, written as the item's whole
// slot.  With `edge_rows` (the window moved), the first work item of each tile
// of the two tile rows at the window ends also takes the kDepEdgeRho pass over
// all of its tile's particles (rho^n where particles left and the new column
// entered); those items get the first workgroups of the launch, so that their
// longer work overlaps the others instead of ending the launch.
template <int TR, int H, int M, int NT>
__global__ __launch_bounds__(NT) void k_deposit_lanes(Parts p, const int* __restrict__ offset,
                                                      const int* __restrict__ nchunk,
                                                      const int* __restrict__ chunk_start,
                                                      float* __restrict__ scratch, const double* __restrict__ ionblk,
                                                      Grid g, TileGeom tg, DevState* st, int edge_rows) {
  using B = Blk<TR, H>;
  using RS = RhoSet<M, B::NODES>;
  extern __shared__ double lds[];
  constexpr int nacc = Vals<M>::N * B::NODES;
  constexpr int kCells = kTZ * TR;
  constexpr int kWaves = NT / 64;
  __shared__ int rowstart[kTZ];
  __shared__ int rowpref[kTZ + 1];
  __shared__ uint16_t runpref[kCells + 1];
  __shared__ int cfirst[kCells];   // sorted index of each cell's first particle (clipped to the piece)
  __shared__ int ccount[kCells];   // its particles in the piece
  __shared__ int wsum[kWaves];
  __shared__ int s_tile, s_item, s_edge;
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  if (b == 0 && tid == 0) {
    st->n_part = st->n_live;
    if (chunk_start[tg.ntiles] > (int)gridDim.x) st->overflow = 2;   // work list larger than the launch
  }
  const int items = chunk_start[tg.ntiles];
  if (b >= items) return;   // uniform per workgroup
  if (tid == 0) {
    // edge tiles in ascending order: tz = 0 and tz = ntz - 1 of every radial
    // tile column (one tile per column when ntz = 1)
    const int per_col = tg.ntz > 1 ? 2 : 1;
    const int n_edge = edge_rows ? per_col * tg.ntr : 0;
    auto edge_tile = [&](int e) { return (e / per_col) * tg.ntz + ((e % per_col) ? tg.ntz - 1 : 0); };
    int item, edge = 0;
    if (b < n_edge) {
      item = chunk_start[edge_tile(b)];
      edge = 1;
    } else {
      // the (b - n_edge)-th item that is not an edge tile's first: skip the k
      // edge items E_j with E_j - j <= b - n_edge (E_j - j ascends with j)
      const int pos = b - n_edge;
      int lo = 0, hi = n_edge;   // count of j with E_j - j <= pos
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (chunk_start[edge_tile(mid)] - mid <= pos) lo = mid + 1;
        else hi = mid;
      }
      item = pos + lo;
    }
    int lo = 0, hi = tg.ntiles;   // chunk_start[lo] <= item < chunk_start[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (chunk_start[mid] <= item) lo = mid;
      else hi = mid;
    }
    s_tile = lo;
    s_item = item;
    s_edge = edge;
  }
  __syncthreads();
  const int item = s_item;
  // a work list larger than the launch (flagged above) has items without a
  // slot: those are left out rather than written past the scratch slots
  if (item >= (int)gridDim.x) return;   // uniform per workgroup
  for (int e = tid; e < nacc; e += NT) lds[e] = 0.0;
  __syncthreads();
  const int t = s_tile;
  const bool edge = s_edge != 0;
  const int chunk = item - chunk_start[t];
  const int J0 = (t % tg.ntz) * kTZ, C0 = (t / tg.ntz) * TR;
  const int C1 = min(C0 + TR, g.ncol);
  if (tid < kTZ) {
    const int j = J0 + tid;
    const int a = offset[j * g.ncol + C0];
    rowstart[tid] = a;
    rowpref[tid + 1] = offset[j * g.ncol + C1] - a;
  }
  __syncthreads();
  if (tid == 0) {
    rowpref[0] = 0;
    for (int r = 1; r <= kTZ; ++r) rowpref[r] += rowpref[r - 1];
  }
  __syncthreads();
  const int total = rowpref[kTZ];
  const double zmin = st->zmin;
  int f0 = 0, f1 = total;
  if (nchunk[t] != 1) {
    f0 = chunk * tg.chunk;
    f1 = min(total, f0 + tg.chunk);
  }
  lane_pass<TR, H, M, kDepCarry, NT>(p, offset, g, tg, lds, rowstart, rowpref, runpref, cfirst, ccount, wsum, J0,
                                     C0, C1, f0, f1, total, zmin);
  if (edge)   // uniform per workgroup
    lane_pass<TR, H, M, kDepEdgeRho, NT>(p, offset, g, tg, lds, rowstart, rowpref, runpref, cfirst, ccount, wsum,
                                         J0, C0, C1, 0, total, total, zmin);
  __syncthreads();
  constexpr int nr_vals = RhoVals<M>::N;
  if (ionblk && chunk == 0) {
    // the tile's background, once per tile, in FP64, into rho^{n+1} (and into
    // rho^n where this item deposits it)
    const double* src = ionblk + (size_t)t * nr_vals * B::NODES;
    for (int e = tid; e < nr_vals * B::NODES; e += NT) {
      const int k = e / B::NODES, node = e % B::NODES;
      lds[RS::off(4, k) + node] += src[e];
      if (edge) lds[RS::off(3, k) + node] += src[e];
    }
    __syncthreads();
  }
  float* dst = scratch + (size_t)item * nacc;
  for (int e = tid; e < nacc; e += NT) dst[e] = (float)lds[e];
}

// Set-up of the background blocks: the FP64 rho slots of a tile's work items
// (the chunks of a dense tile) are summed into the tile's block.
template <int TR, int H, int M>
__global__ __launch_bounds__(256) void k_ion_reduce(const int* __restrict__ nchunk, const int* __restrict__ chunk_start,
                                                    const double* __restrict__ slots, double* __restrict__ ionblk,
                                                    int ntiles) {
  constexpr int n = RhoVals<M>::N * Blk<TR, H>::NODES;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)ntiles * n) return;
  const int t = (int)(i / n), e = (int)(i % n);
  const double* base = slots + (size_t)chunk_start[t] * n + e;
  double a = 0.0;
  for (int c = 0; c < nchunk[t]; ++c) a += base[(size_t)c * n];
  ionblk[i] = a;
}

// rho^n of a step that follows a deposit: the previous rho^{n+1} (same
// particles, same positions), moved one node toward the tail when the window
// moved in between (the grid node j is then the old node j + 1); the edge
// columns are overwritten by the edge-tile deposit.
__global__ __launch_bounds__(256) void k_rho_carry(float2* __restrict__ real, int M, int nr, int nz, int shift) {
  const int64_t plane = (int64_t)nr * nz;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)M * plane) return;
  const int64_t m = i / plane, node = i % plane;
  const int r = (int)(node / nz), j = (int)(node % nz);
  int js = j + shift;
  if (js >= nz) js -= nz;
  const float2* src = real + ((size_t)(kCompJ + 4) * M + m) * plane + (size_t)r * nz;
  float2* dst = real + ((size_t)(kCompJ + 3) * M + m) * plane + (size_t)r * nz;
  dst[j] = src[js];
}

// Chunks of a dense tile: their blocks are summed into the tile's first slot.
// Work items are (dense tile, 256-element block) pairs taken from the dense
// list in a grid-stride loop, so a launch of fixed size covers any number of
// dense tiles and the sparse tiles cost nothing.
template <int TR, int H, int M>
__global__ __launch_bounds__(256) void k_chunk_reduce(const int* __restrict__ nchunk, const int* __restrict__ dense,
                                                      const int* __restrict__ chunk_start, float* __restrict__ scratch,
                                                      int ntiles) {
  using B = Blk<TR, H>;
  constexpr int nacc = Vals<M>::N * B::NODES;
  constexpr int neb = (nacc + 255) / 256;
  const int items = dense[ntiles] * neb;
  for (int item = blockIdx.x; item < items; item += gridDim.x) {
    const int t = dense[item / neb];
    const int e = (item % neb) * 256 + threadIdx.x;
    if (e >= nacc) continue;
    const int nch = nchunk[t];
    float* base = scratch + (size_t)chunk_start[t] * nacc + e;
    // eight chunks in flight per batch (a beam-core tile has about twelve)
    float a[8] = {base[0], 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int c = 1;
    for (; c + 7 < nch; c += 8) {
#pragma unroll
      for (int q = 0; q < 8; ++q) a[q] += base[(size_t)(c + q) * nacc];
    }
    for (; c < nch; ++c) a[0] += base[(size_t)c * nacc];
    base[0] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  }
}

// Node-parallel sum of the tile blocks covering the node, then: J-,0 =
// conj(J+,0), division by the ring volume 2 pi r_i dr dz (the immobile
// background is already in the blocks).
// rho_n_cols: 0 writes rho^n everywhere; 1 only in the kEdgeCols columns at
// each end of the window along z (the carried values stay elsewhere); 2 nowhere.
constexpr int kEdgeColsTail = 2, kEdgeColsHead = 3;   // columns 0..1 and nz-3..nz-1
template <int TR, int H, int M>
__global__ __launch_bounds__(256) void k_deposit_combine(const int* __restrict__ chunk_start,
                                                         const float* __restrict__ scratch,
                                                         float2* __restrict__ real, Grid g, TileGeom tg,
                                                         int rho_n_cols) {
  using B = Blk<TR, H>;
  constexpr int NV = Vals<M>::N;
  constexpr int nacc = NV * B::NODES;
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int nz = g.nz, nr = g.nr;
  if (node >= (int64_t)nr * nz) return;
  const int i = (int)(node / nz), j = (int)(node % nz);
  // covering tiles (at most two along z times two along r):
  // bz = j - (J0 - H) mod nz in [0, BZ); br = i - (C0 - 1 - H) in [0, BR)
  int tq[4] = {0, 0, 0, 0}, toff[4] = {0, 0, 0, 0}, nt = 0;   // the centre tile always covers the node
  const int tz0 = j / kTZ;
  const int tr0 = (i + 1) / TR;
  for (int dtz = -1; dtz <= 1; ++dtz) {
    int tz = tz0 + dtz;
    if (tz < 0) tz += tg.ntz;
    if (tz >= tg.ntz) tz -= tg.ntz;
    if (dtz != 0 && tz == tz0) continue;
    if (dtz == 1 && tg.ntz == 2) continue;   // the two neighbours coincide
    int bz = j - (tz * kTZ - H);
    if (bz < 0) bz += nz;
    if (bz >= nz) bz -= nz;
    if (bz >= B::BZ) continue;
    for (int dtr = -1; dtr <= 1; ++dtr) {
      const int tr = tr0 + dtr;
      if (tr < 0 || tr >= tg.ntr) continue;
      const int br = i - (tr * TR - 1 - H);
      if (br < 0 || br >= B::BR) continue;
      if (nt < 4) {
        tq[nt] = tr * tg.ntz + tz;
        toff[nt] = br * B::BZ + bz;
        ++nt;
      }
    }
  }
  // every load in flight at once; a slot no lane of the wavefront needs (the
  // second r tile away from tile edges) is skipped by the whole wavefront
  int cs[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) cs[q] = chunk_start[tq[q < nt ? q : 0]];
  float x[4][NV];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
#pragma unroll
    for (int v = 0; v < NV; ++v) x[q][v] = 0.f;
    if (q < nt) {
      const float* qp = scratch + (size_t)cs[q] * nacc + toff[q];
#pragma unroll
      for (int v = 0; v < NV; ++v) x[q][v] = qp[v * B::NODES];
    }
  }
  float acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.f;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float wq = q < nt ? 1.f : 0.f;
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = fmaf(wq, x[q][v], acc[v]);
  }
  const float inv_v = (float)(1.0 / (2.0 * M_PI * g.dr * g.dr * g.dz * (i + 0.5)));
  // slot order of the grid: J+, J-, Jz, rho^n, rho^{n+1}
  float2 out[5][M];
  out[0][0] = make_float2(acc[0], acc[1]);
  out[1][0] = make_float2(acc[0], -acc[1]);
  out[2][0] = make_float2(acc[2], 0.f);
  out[3][0] = make_float2(acc[3], 0.f);
  out[4][0] = make_float2(acc[4], 0.f);
#pragma unroll
  for (int m = 1; m < M; ++m) {
    const int b0 = vbase(m);
#pragma unroll
    for (int sl = 0; sl < 5; ++sl) out[sl][m] = make_float2(acc[b0 + 2 * sl], acc[b0 + 2 * sl + 1]);
  }
  const bool write_rho_n =
      rho_n_cols == 0 || (rho_n_cols == 1 && (j < kEdgeColsTail || j >= nz - kEdgeColsHead));
#pragma unroll
  for (int sl = 0; sl < 5; ++sl)
#pragma unroll
    for (int m = 0; m < M; ++m) {
      if (sl == 3 && !write_rho_n) continue;
      real[dfidx(kCompJ + sl, m, M, nr, nz) + node] = cscale(out[sl][m], inv_v);
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
DepositShape deposit_shape(int nz, int nr, int nmodes, int halo, int64_t cap) {
  DepositShape d;
  d.TZ = kTZ;
  d.TR = nmodes <= 1 ? 16 : 8;
  d.halo = halo;
  d.ntz = nz / d.TZ;
  d.ntr = (nr + 1 + d.TR - 1) / d.TR;   // key columns 0..nr
  d.ntiles = d.ntz * d.ntr;
  d.max_items = d.ntiles + (int)((cap + kChunkMin - 1) / kChunkMin);
  d.chunk = 4096;
  d.tile_max = 3 * d.chunk;
  const int bz = d.TZ + 2 * halo + 1, br = d.TR + 2 * halo + 1;
  const int nv = 5 + 10 * (nmodes - 1);
  d.acc_floats2 = ((size_t)nv * bz * br + 1) / 2;     // FP32 scratch slot per work item
  d.lds_bytes = (size_t)nv * bz * br * sizeof(double);
  d.ion_doubles = (size_t)(2 * nmodes - 1) * bz * br;   // FP64 background block per tile
  return d;
}

template <class K>
static bool set_lds_limit(K kernel, size_t bytes) {
  return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) ==
         hipSuccess;
}

template <int TR, int H, int M, int SHAPE>
static void launch_dep(const Parts& p, const int* offset, int* nchunk, int* chunk_start, float2* scratch,
                       float2* real, const double* ionblk, double* ionblk_out, const Grid& g, const DepositShape& d,
                       DevState* st, int stages, int rho_mode, hipStream_t s) {
  TileGeom tg{d.ntz, d.ntr, d.ntiles, d.tile_max, d.chunk};
  const size_t lds = (size_t)Vals<M>::N * Blk<TR, H>::NODES * sizeof(double);
  if (stages & kDepPlan) {
    hipLaunchKernelGGL((k_tile_totals<TR>), dim3((d.ntiles + 3) / 4), dim3(256), 0, s, offset, g, tg, nchunk);
    hipLaunchKernelGGL(k_tile_plan, dim3(1), dim3(1024), 0, s, nchunk, d.ntiles, chunk_start, nchunk + d.ntiles);
    if (rho_mode != kRhoDeposit) {
      const int64_t n = (int64_t)g.nmodes * g.nr * g.nz;
      hipLaunchKernelGGL(k_rho_carry, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, real, g.nmodes, g.nr, g.nz,
                         rho_mode == kRhoCarryShift ? 1 : 0);
    }
  }
  if (ionblk_out) {   // set-up: FP64 background blocks instead of the grid
    if (!(stages & kDepTiles)) return;
    static bool attr_ion = false;
    if (!attr_ion) {
      if (!set_lds_limit(k_deposit<TR, H, M, kDepIon, SHAPE>, lds)) return;   // error stays pending for the caller's check
      attr_ion = true;
    }
    hipLaunchKernelGGL((k_deposit<TR, H, M, kDepIon, SHAPE>), dim3(d.max_items), dim3(256), lds, s, p, offset, nchunk,
                       chunk_start, (float*)scratch, (const double*)nullptr, g, tg, st);
    const int64_t n = (int64_t)d.ntiles * RhoVals<M>::N * Blk<TR, H>::NODES;
    hipLaunchKernelGGL((k_ion_reduce<TR, H, M>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, nchunk,
                       chunk_start, (const double*)scratch, ionblk_out, d.ntiles);
    return;
  }
  if (stages & kDepTiles) {
    static bool attr_set[3] = {false, false, false};   // dynamic LDS above the default limit
    if (!attr_set[0]) {
      if (!set_lds_limit(k_deposit<TR, H, M, kDepFull, SHAPE>, lds) || !set_lds_limit(k_deposit<TR, H, M, kDepCarry, SHAPE>, lds) ||
          !set_lds_limit(k_deposit<TR, H, M, kDepEdgeRho, SHAPE>, lds))
        return;
      attr_set[0] = true;
    }
    if (rho_mode == kRhoDeposit) {
      hipLaunchKernelGGL((k_deposit<TR, H, M, kDepFull, SHAPE>), dim3(d.max_items), dim3(256), lds, s, p, offset, nchunk,
                         chunk_start, (float*)scratch, ionblk, g, tg, st);
    } else {
      if constexpr (SHAPE == 1 && M <= 4) {
        static bool attr_lanes = false;
        if (!attr_lanes) {
          if (!set_lds_limit(k_deposit_lanes<TR, H, M, 256>, lds)) return;
          attr_lanes = true;
        }
        hipLaunchKernelGGL((k_deposit_lanes<TR, H, M, 256>), dim3(d.max_items), dim3(256), lds, s, p, offset,
                           nchunk, chunk_start, (float*)scratch, ionblk, g, tg, st,
                           rho_mode == kRhoCarryShift ? 1 : 0);
      } else {
        hipLaunchKernelGGL((k_deposit<TR, H, M, kDepCarry, SHAPE>), dim3(d.max_items), dim3(256), lds, s, p, offset,
                           nchunk, chunk_start, (float*)scratch, ionblk, g, tg, st);
        if (rho_mode == kRhoCarryShift)
          hipLaunchKernelGGL((k_deposit<TR, H, M, kDepEdgeRho, SHAPE>), dim3(2 * d.ntr), dim3(256), lds, s, p, offset,
                             nchunk, chunk_start, (float*)scratch, ionblk, g, tg, st);
      }
    }
  }
  if (stages & kDepCombine) {
    constexpr int nacc = Vals<M>::N * Blk<TR, H>::NODES;
    const int items = d.ntiles * ((nacc + 255) / 256);
    hipLaunchKernelGGL((k_chunk_reduce<TR, H, M>), dim3(items < 1024 ? items : 1024), dim3(256), 0, s, nchunk,
                       nchunk + d.ntiles, chunk_start, (float*)scratch, d.ntiles);
    const int64_t nodes = (int64_t)g.nr * g.nz;
    const int cols = rho_mode == kRhoDeposit ? 0 : rho_mode == kRhoCarryShift ? 1 : 2;
    hipLaunchKernelGGL((k_deposit_combine<TR, H, M>), dim3((unsigned)((nodes + 255) / 256)), dim3(256), 0, s,
                       chunk_start, (const float*)scratch, real, g, tg, cols);
  }
}

template <int H, int SHAPE>
static void launch_dep_h(const Parts& p, const int* offset, int* nchunk, int* chunk_start, float2* scratch,
                         float2* real, const double* ionblk, double* ionblk_out, const Grid& g, const DepositShape& d,
                         DevState* st, int stages, int rho_mode, hipStream_t s) {
  switch (g.nmodes) {
    case 1: launch_dep<16, H, 1, SHAPE>(p, offset, nchunk, chunk_start, scratch, real, ionblk, ionblk_out, g, d, st, stages, rho_mode, s); break;
    case 2: launch_dep<8, H, 2, SHAPE>(p, offset, nchunk, chunk_start, scratch, real, ionblk, ionblk_out, g, d, st, stages, rho_mode, s); break;
    case 3: launch_dep<8, H, 3, SHAPE>(p, offset, nchunk, chunk_start, scratch, real, ionblk, ionblk_out, g, d, st, stages, rho_mode, s); break;
    default: launch_dep<8, H, 4, SHAPE>(p, offset, nchunk, chunk_start, scratch, real, ionblk, ionblk_out, g, d, st, stages, rho_mode, s); break;
  }
}

void launch_deposit(const Parts& p, const int* offset, const DepositShape& d, int* nchunk, int* chunk_start,
                    float2* scratch, float2* real, const double* ionblk, double* ionblk_out, const Grid& g,
                    DevState* st, int stages, int rho_mode, hipStream_t s) {
  // the block halo: cells a particle moves per step (1 or 2), one more for cubic shapes
  if (g.shape == 3) {
    if (d.halo == 2) launch_dep_h<2, 3>(p, offset, nchunk, chunk_start, scratch, real, ionblk, ionblk_out, g, d, st, stages, rho_mode, s);
    else launch_dep_h<3, 3>(p, offset, nchunk, chunk_start, scratch, real, ionblk, ionblk_out, g, d, st, stages, rho_mode, s);
  } else {
    if (d.halo == 1) launch_dep_h<1, 1>(p, offset, nchunk, chunk_start, scratch, real, ionblk, ionblk_out, g, d, st, stages, rho_mode, s);
    else launch_dep_h<2, 1>(p, offset, nchunk, chunk_start, scratch, real, ionblk, ionblk_out, g, d, st, stages, rho_mode, s);
  }
}

}  // namespace pic
