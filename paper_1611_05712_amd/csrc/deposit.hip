// Charge and current deposit: rho^n at x^n, J^{n+1/2} at x^{n+1/2} (velocity
// v^{n+1/2}) and rho^{n+1} at x^{n+1}, linear shapes, every azimuthal mode.
//
// Work decomposition (no global atomics anywhere):
//   * particles are sorted by the cell of x^{n+1}; the cells are cut into
//     TZ x TR tiles and each particle belongs to exactly one tile;
//   * a tile's particles touch the nodes of its cells plus a halo of H cells
//     (x^n, x^{n+1/2} lie within dt c of x^{n+1}, dt <= H dz and H dr), so
//     a workgroup accumulates a (TZ + 2H + 1) x (TR + 2H + 1) node block in LDS
//     and writes it to a scratch slot;
//   * dense tiles (beam cores hold thousands of particles per cell) are cut
//     into chunks of at most kChunk particles, each with its own slot; the
//     device builds this work list (k_tile_plan) from the sorted offsets;
//   * k_deposit_combine sums, node by node, the slots of every block covering
//     the node and writes the grid.
// Within a wavefront consecutive lanes hold consecutive (cell-sorted)
// particles.  For each of the three positions, lanes sharing a cell form
// runs; the node contributions are summed along each run with DPP row shifts
// (runs are cut at 16-lane row boundaries) and only the run head issues the
// LDS atomics.  Waves whose particles are all at rest deposit rho once (it is
// rho^n and rho^{n+1}) and no current.
#include "common.h"
#include "launch.h"

namespace pic {

constexpr int kChunk = 16384;   // max particles per workgroup
constexpr int kTZ = 32;

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
  if (lane == 0) nchunk[t] = s > 0 ? (s + kChunk - 1) / kChunk : 1;
}

// exclusive scan of chunk counts: chunk_start[0..ntiles], chunk_start[ntiles] = work items
__global__ __launch_bounds__(1024) void k_tile_plan(const int* __restrict__ nchunk, int ntiles,
                                                   int* __restrict__ chunk_start) {
  __shared__ int sh[1024];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int b0 = 0; b0 < ntiles; b0 += 1024) {
    int i = b0 + threadIdx.x;
    int v = i < ntiles ? nchunk[i] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      int u = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
      __syncthreads();
      sh[threadIdx.x] += u;
      __syncthreads();
    }
    if (i < ntiles) chunk_start[i] = carry + sh[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry += sh[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) chunk_start[ntiles] = carry;
}

// ---------------------------------------------------------------------------
// run reduction along DPP rows
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ float row_shl(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

struct RunMask {
  int dist;              // lanes after this one in its run (within the row)
  bool head;
  bool s1, s2, s4, s8;   // wave-uniform: some run needs this step
};

__device__ __forceinline__ RunMask run_mask(uint32_t key) {
  const int lane = threadIdx.x & 63;
  const uint32_t prev = __shfl_up(key, 1, 64);
  const bool head = ((lane & 15) == 0) || (prev != key);
  const uint64_t heads = __ballot(head);
  const uint64_t after = (lane == 63) ? 0ull : (heads & ~((2ull << lane) - 1ull));
  const int next = after ? (__ffsll((long long)after) - 1) : 64;
  RunMask rm;
  rm.head = head;
  rm.dist = next - lane - 1;
  rm.s1 = __ballot(rm.dist >= 1) != 0;
  rm.s2 = __ballot(rm.dist >= 2) != 0;
  rm.s4 = __ballot(rm.dist >= 4) != 0;
  rm.s8 = __ballot(rm.dist >= 8) != 0;
  return rm;
}

// r[i] <- sum of r[i] over lanes l .. l + dist (one wave-uniform branch per
// step; the n independent shifts of a step interleave)
template <int N>
__device__ __forceinline__ void run_reduce(float (&r)[N], const RunMask& rm) {
  if (rm.s1) {
    const bool c = rm.dist >= 1;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const float t = row_shl<0x101>(r[i]);
      r[i] += c ? t : 0.f;
    }
  }
  if (rm.s2) {
    const bool c = rm.dist >= 2;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const float t = row_shl<0x102>(r[i]);
      r[i] += c ? t : 0.f;
    }
  }
  if (rm.s4) {
    const bool c = rm.dist >= 4;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const float t = row_shl<0x104>(r[i]);
      r[i] += c ? t : 0.f;
    }
  }
  if (rm.s8) {
    const bool c = rm.dist >= 8;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const float t = row_shl<0x108>(r[i]);
      r[i] += c ? t : 0.f;
    }
  }
}

// ---------------------------------------------------------------------------
// per-position values and their place in the LDS block.  Block layout:
// [slot][m][br][bz] complex (slot 0 J+, 1 J-, 2 Jz, 3 rho^n, 4 rho^{n+1});
// the mode-0 density and J_z are real, J-,0 = conj(J+,0) is rebuilt by the
// combine.  Each value k has a compile-time float offset and the parity of
// its Hankel order (sign of the ghost node across the axis).
// ---------------------------------------------------------------------------
template <int M, int NODES>
struct RhoSet {
  static constexpr int K = 1 + 2 * (M - 1);
  static __device__ __forceinline__ constexpr int mode(int k) { return k == 0 ? 0 : 1 + (k - 1) / 2; }
  static __device__ __forceinline__ constexpr int part(int k) { return k == 0 ? 0 : (k - 1) & 1; }
  static __device__ __forceinline__ constexpr int parity(int k) { return mode(k) & 1; }
  static __device__ __forceinline__ constexpr int off(int slot, int k) {
    return 2 * (slot * M + mode(k)) * NODES + part(k);
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
    return 2 * (slot(k) * M + mode(k)) * NODES + part(k);
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

// products with the four node weights, run reduction, head flush
template <int K, class Set, class OffFn>
__device__ __forceinline__ void deposit_set(float* __restrict__ lds, const float (&v)[K], bool valid, const RunMask& rm,
                                            const ShapePos& s, int na, int nb, float sa_even, float sa_odd,
                                            float sb, OffFn off) {
  const float fz = s.fz, fr = s.fr;
  const float w0 = (1.f - fz) * (1.f - fr), w1 = fz * (1.f - fr), w2 = (1.f - fz) * fr, w3 = fz * fr;
  float r[4 * K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const float vk = valid ? v[k] : 0.f;
    r[4 * k + 0] = w0 * vk;   // (ia, j0)
    r[4 * k + 1] = w1 * vk;   // (ia, j0 + 1)
    r[4 * k + 2] = w2 * vk;   // (ib, j0)
    r[4 * k + 3] = w3 * vk;   // (ib, j0 + 1)
  }
  run_reduce<4 * K>(r, rm);
  if (rm.head && valid) {
    float* pa = lds + 2 * na;
    float* pb = lds + 2 * nb;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const float sa = Set::parity(k) ? sa_odd : sa_even;
      const int o = off(k);
      atomicAdd(pa + o, sa * r[4 * k + 0]);
      atomicAdd(pa + o + 2, sa * r[4 * k + 1]);
      atomicAdd(pb + o, sb * r[4 * k + 2]);
      atomicAdd(pb + o + 2, sb * r[4 * k + 3]);
    }
  }
}

__device__ __forceinline__ uint32_t pos_key(const ShapePos& s, int nr) {
  const int ic = (s.i0 > nr ? nr : s.i0) + 1;
  return (uint32_t)s.j0 * 2048u + (uint32_t)ic;
}

template <int TR, int H, int M>
__global__ __launch_bounds__(256) void k_deposit(Parts p, const int* __restrict__ offset,
                                                 const int* __restrict__ nchunk, const int* __restrict__ chunk_start,
                                                 float2* __restrict__ scratch, Grid g, TileGeom tg, DevState* st) {
  using B = Blk<TR, H>;
  using RS = RhoSet<M, B::NODES>;
  using JS = JSet<M, B::NODES>;
  extern __shared__ float2 lds_blk[];
  __shared__ int rowstart[kTZ];
  __shared__ int rowpref[kTZ + 1];
  __shared__ int s_tile;
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  if (b == 0 && tid == 0) {
    st->n_part = st->n_live;
    if (chunk_start[tg.ntiles] > (int)gridDim.x) st->overflow = 2;   // work list larger than the launch
  }
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
  constexpr int nacc = 5 * M * B::NODES;
  for (int e = tid; e < nacc; e += blockDim.x) lds_blk[e] = make_float2(0.f, 0.f);
  __syncthreads();
  const int t = s_tile;
  const int chunk = b - chunk_start[t];
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
  const int f0 = chunk * kChunk;
  const int f1 = min(total, f0 + kChunk);
  float* lds = (float*)lds_blk;
  const double zmin = st->zmin;
  const double dt = g.dt;
  const int lane = tid & 63, wave = tid >> 6;
  for (int base = f0 + wave * 64; base < f1; base += 256) {
    const int f = base + lane;
    const bool valid = f < f1;
    double x = 0.0, y = 0.0, z = zmin;
    float ux = 0.f, uy = 0.f, uz = 0.f, qw = 0.f;
    if (valid) {
      int lo = 0, hi = kTZ;   // rowpref[lo] <= f < rowpref[hi]
#pragma unroll
      for (int it = 0; it < 5; ++it) {
        const int mid = (lo + hi) >> 1;
        if (rowpref[mid] <= f) lo = mid;
        else hi = mid;
      }
      const int idx = rowstart[lo] + (f - rowpref[lo]);
      x = p.x[idx];
      y = p.y[idx];
      z = p.z[idx];
      ux = p.ux[idx];
      uy = p.uy[idx];
      uz = p.uz[idx];
      qw = p.w[idx];
    }
    const bool cold = __ballot(valid && (ux != 0.f || uy != 0.f || uz != 0.f)) == 0;
    const float ginv = 1.f / sqrtf(1.f + ux * ux + uy * uy + uz * uz);
    const float vx = ux * ginv, vy = uy * ginv, vz = uz * ginv;
    // rho^{n+1} at x^{n+1} (also rho^n when the whole wave is at rest)
    {
      const ShapePos s = shape_at(x, y, z, zmin, g);
      const RunMask rm = run_mask(valid ? pos_key(s, g.nr) : kInvalidKey);
      const Local<TR, H> L = localize<TR, H>(s, g, J0, C0);
      float v[RS::K];
      RS::values(qw, s.eith, v);
      deposit_set<RS::K, RS>(lds, v, valid, rm, s, L.na, L.nb, L.sa_even, L.sa_odd, L.sb,
                             [](int k) { return RS::off(4, k); });
      if (cold) {
        deposit_set<RS::K, RS>(lds, v, valid, rm, s, L.na, L.nb, L.sa_even, L.sa_odd, L.sb,
                               [](int k) { return RS::off(3, k); });
        continue;
      }
    }
    // J^{n+1/2} at x^{n+1/2} = x^{n+1} - dt v / 2
    {
      const ShapePos s = shape_at(x - 0.5 * dt * (double)vx, y - 0.5 * dt * (double)vy,
                                  z - 0.5 * dt * (double)vz, zmin, g);
      const RunMask rm = run_mask(valid ? pos_key(s, g.nr) : kInvalidKey);
      const Local<TR, H> L = localize<TR, H>(s, g, J0, C0);
      float v[JS::K];
      JS::values(qw, vx, vy, vz, s.eith, v);
      deposit_set<JS::K, JS>(lds, v, valid, rm, s, L.na, L.nb, L.sa_even, L.sa_odd, L.sb,
                             [](int k) { return JS::off(k); });
    }
    // rho^n at x^n = x^{n+1} - dt v
    {
      const ShapePos s = shape_at(x - dt * (double)vx, y - dt * (double)vy, z - dt * (double)vz, zmin, g);
      const RunMask rm = run_mask(valid ? pos_key(s, g.nr) : kInvalidKey);
      const Local<TR, H> L = localize<TR, H>(s, g, J0, C0);
      float v[RS::K];
      RS::values(qw, s.eith, v);
      deposit_set<RS::K, RS>(lds, v, valid, rm, s, L.na, L.nb, L.sa_even, L.sa_odd, L.sb,
                             [](int k) { return RS::off(3, k); });
    }
  }
  __syncthreads();
  float2* dst = scratch + (size_t)b * nacc;
  for (int e = tid; e < nacc; e += blockDim.x) dst[e] = lds_blk[e];
}

// Node-parallel sum of every block slot covering the node, then: J-,0 =
// conj(J+,0), division by the ring volume 2 pi r_i dr dz, immobile background
// added to both densities.
template <int TR, int H, int M>
__global__ __launch_bounds__(256) void k_deposit_combine(const int* __restrict__ nchunk,
                                                         const int* __restrict__ chunk_start,
                                                         const float2* __restrict__ scratch,
                                                         float2* __restrict__ real, const float2* __restrict__ bg,
                                                         Grid g, TileGeom tg) {
  using B = Blk<TR, H>;
  constexpr int nacc = 5 * M * B::NODES;
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int nz = g.nz, nr = g.nr;
  if (node >= (int64_t)nr * nz) return;
  const int i = (int)(node / nz), j = (int)(node % nz);
  float2 acc[5][M];
#pragma unroll
  for (int sl = 0; sl < 5; ++sl)
#pragma unroll
    for (int m = 0; m < M; ++m) acc[sl][m] = make_float2(0.f, 0.f);
  // covering tiles: bz = j - (J0 - H) mod nz in [0, BZ); br = i - (C0 - 1 - H) in [0, BR)
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
      const int t = tr * tg.ntz + tz;
      const int nch = nchunk[t];
      const float2* blk = scratch + (size_t)chunk_start[t] * nacc + br * B::BZ + bz;
      for (int c = 0; c < nch; ++c) {
        const float2* q = blk + (size_t)c * nacc;
#pragma unroll
        for (int sl = 0; sl < 5; ++sl)
#pragma unroll
          for (int m = 0; m < M; ++m) acc[sl][m] = cadd(acc[sl][m], q[(sl * M + m) * B::NODES]);
      }
    }
  }
  acc[1][0] = cconj(acc[0][0]);
  const float inv_v = (float)(1.0 / (2.0 * M_PI * g.dr * g.dr * g.dz * (i + 0.5)));
#pragma unroll
  for (int sl = 0; sl < 5; ++sl)
#pragma unroll
    for (int m = 0; m < M; ++m) {
      float2 v = cscale(acc[sl][m], inv_v);
      if (bg && sl >= 3) v = cadd(v, bg[(size_t)m * nr * nz + node]);
      real[dfidx(kCompJ + sl, m, M, nr, nz) + node] = v;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
DepositShape deposit_shape(int nz, int nr, int nmodes, int halo, int64_t cap) {
  DepositShape d;
  d.TZ = kTZ;
  d.TR = nmodes <= 2 ? 16 : 8;
  d.halo = halo;
  d.ntz = nz / d.TZ;
  d.ntr = (nr + 1 + d.TR - 1) / d.TR;   // key columns 0..nr
  d.ntiles = d.ntz * d.ntr;
  d.max_items = d.ntiles + (int)((cap + kChunk - 1) / kChunk);
  const int bz = d.TZ + 2 * halo + 1, br = d.TR + 2 * halo + 1;
  d.acc_floats2 = (size_t)5 * nmodes * bz * br;
  return d;
}

template <int TR, int H, int M>
static void launch_dep(const Parts& p, const int* offset, int* nchunk, int* chunk_start, float2* scratch,
                       float2* real, const float2* bg, const Grid& g, const DepositShape& d, DevState* st,
                       hipStream_t s) {
  TileGeom tg{d.ntz, d.ntr, d.ntiles};
  const size_t lds = (size_t)5 * M * Blk<TR, H>::NODES * sizeof(float2);
  hipLaunchKernelGGL((k_tile_totals<TR>), dim3((d.ntiles + 3) / 4), dim3(256), 0, s, offset, g, tg, nchunk);
  hipLaunchKernelGGL(k_tile_plan, dim3(1), dim3(1024), 0, s, nchunk, d.ntiles, chunk_start);
  hipLaunchKernelGGL((k_deposit<TR, H, M>), dim3(d.max_items), dim3(256), lds, s, p, offset, nchunk, chunk_start,
                     scratch, g, tg, st);
  const int64_t nodes = (int64_t)g.nr * g.nz;
  hipLaunchKernelGGL((k_deposit_combine<TR, H, M>), dim3((unsigned)((nodes + 255) / 256)), dim3(256), 0, s, nchunk,
                     chunk_start, scratch, real, bg, g, tg);
}

template <int H>
static void launch_dep_h(const Parts& p, const int* offset, int* nchunk, int* chunk_start, float2* scratch,
                         float2* real, const float2* bg, const Grid& g, const DepositShape& d, DevState* st,
                         hipStream_t s) {
  switch (g.nmodes) {
    case 1: launch_dep<16, H, 1>(p, offset, nchunk, chunk_start, scratch, real, bg, g, d, st, s); break;
    case 2: launch_dep<16, H, 2>(p, offset, nchunk, chunk_start, scratch, real, bg, g, d, st, s); break;
    case 3: launch_dep<8, H, 3>(p, offset, nchunk, chunk_start, scratch, real, bg, g, d, st, s); break;
    default: launch_dep<8, H, 4>(p, offset, nchunk, chunk_start, scratch, real, bg, g, d, st, s); break;
  }
}

void launch_deposit(const Parts& p, const int* offset, const DepositShape& d, int* nchunk, int* chunk_start,
                    float2* scratch, float2* real, const float2* bg, const Grid& g, DevState* st, hipStream_t s) {
  if (d.halo == 1) launch_dep_h<1>(p, offset, nchunk, chunk_start, scratch, real, bg, g, d, st, s);
  else launch_dep_h<2>(p, offset, nchunk, chunk_start, scratch, real, bg, g, d, st, s);
}

}  // namespace pic
