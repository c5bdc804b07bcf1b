// Particle kernels: gather + Boris push, cell sort, tile deposit, injection.
//
// Shapes are linear in z (periodic) and r.  A particle below the first radial
// node shares weight with a ghost node at r = -dr/2, i.e. node 0 seen across
// the axis, where a component of Hankel order nu takes the factor (-1)^nu.
// Nodes at i >= nr are outside the box.  Mode-m densities carry the phase
// exp(i m theta) and are divided by the ring volume 2 pi r_i dr dz.
#include "common.h"
#include "launch.h"

namespace pic {

__device__ __forceinline__ size_t fidx(int c, int m, int M, int nr, int nz) {
  return ((size_t)c * M + m) * (size_t)nr * nz;
}

// --------------------------------------------------------------------------
// wavefront helpers: runs of equal keys in consecutive lanes
// --------------------------------------------------------------------------
struct RunInfo {
  bool head;
  int len;        // valid on heads
  int head_lane;  // lane of this lane's run head
};

__device__ __forceinline__ RunInfo wave_runs(uint32_t k) {
  const int lane = threadIdx.x & 63;
  uint32_t prev = __shfl_up(k, 1, 64);
  bool head = (lane == 0) || (prev != k);
  uint64_t heads = __ballot(head);
  RunInfo ri;
  ri.head = head;
  uint64_t after = heads & ~((2ull << lane) - 1ull);
  if (lane == 63) after = 0;
  int next = after ? (__ffsll((long long)after) - 1) : 64;
  ri.len = next - lane;
  uint64_t upto = heads & ((lane == 63) ? ~0ull : ((2ull << lane) - 1ull));
  ri.head_lane = 63 - __clzll((long long)upto);
  return ri;
}

// histogram increment with one atomic per distinct key of the wavefront
__device__ __forceinline__ void wave_count(uint32_t k, int* __restrict__ count) {
  const int lane = threadIdx.x & 63;
  bool todo = k != kInvalidKey;
  uint64_t pending = __ballot(todo);
  while (pending) {
    const int leader = __ffsll((long long)pending) - 1;
    const uint32_t kl = __shfl(k, leader, 64);
    const bool mine = todo && k == kl;
    const uint64_t mask = __ballot(mine);
    if (lane == leader) atomicAdd(&count[kl], __popcll(mask));
    todo = todo && !mine;
    pending &= ~mask;
  }
}

// --------------------------------------------------------------------------
// field gather.  The gather reads a node-interleaved copy of the real-space
// E, B: record (i, j) holds what the Cartesian field at a particle needs, so a
// particle's four nodes are two contiguous segments [(ia, j0), (ia, j0+1)] and
// [(ib, j0), (ib, j0+1)].  Mode 0 is real (F_+,0 = conj F_-,0, F_z,0 real):
// its part is E-, B- and the real parts of Ez, Bz (4 float2 with one of
// padding); every mode m >= 1 adds E+, E-, Ez, B+, B-, Bz.  kRecF2(M) = 6M - 2
// float2 per record, an even count, so records stay 16-byte aligned.
// --------------------------------------------------------------------------
// A workgroup packs 256 consecutive nodes: the 6M planes are read coalesced
// into the node records in LDS, which are then written out as one contiguous
// block with 16-byte stores (the records of a node are 6M float2, an even
// count, and the block starts at a multiple of 256 records).
__host__ __device__ constexpr int rec_f2(int M) { return 6 * M - 2; }

__global__ __launch_bounds__(256) void k_pack_gather(const float2* __restrict__ real, float2* __restrict__ gf, int nr,
                                                     int nz, int M) {
  extern __shared__ float4 rec4[];  // [256][6M - 2] float2, 16-byte aligned
  float2* rec = reinterpret_cast<float2*>(rec4);
  const int64_t n = (int64_t)nr * nz;
  const int64_t node0 = (int64_t)blockIdx.x * 256;
  const int64_t node = node0 + threadIdx.x;
  const int w = rec_f2(M);
  if (node < n) {
    float2* r = rec + threadIdx.x * w;
    r[0] = real[fidx(1, 0, M, nr, nz) + node];   // E-,0
    r[1] = real[fidx(4, 0, M, nr, nz) + node];   // B-,0
    r[2] = make_float2(real[fidx(2, 0, M, nr, nz) + node].x, real[fidx(5, 0, M, nr, nz) + node].x);
    r[3] = make_float2(0.f, 0.f);
    for (int m = 1; m < M; ++m)
#pragma unroll
      for (int c = 0; c < 6; ++c) r[4 + 6 * (m - 1) + c] = real[fidx(c, m, M, nr, nz) + node];
  }
  __syncthreads();
  const int64_t nodes = n - node0 < 256 ? n - node0 : 256;
  const int nq = (int)(nodes * w / 2);   // float4 count of the block
  float4* dst = reinterpret_cast<float4*>(gf + node0 * w);
  for (int q = threadIdx.x; q < nq; q += 256) dst[q] = rec4[q];
}

template <int M>
struct Gathered {
  float2 f[M][6];   // E+, E-, Ez, B+, B-, Bz per mode
};

// record (i, j) of the node-interleaved copy in HBM
template <int M>
struct GlobalRecs {
  const float4* __restrict__ gf4;
  int nz;
  __device__ __forceinline__ const float4* operator()(int i, int j) const {
    return gf4 + ((size_t)i * nz + j) * (rec_f2(M) / 2);
  }
};

template <int M>
__device__ __forceinline__ void gather_node(Gathered<M>& acc, const float4* rec, float w_even, float w_odd) {
  {
    // mode 0: E-, B- (Hankel order -1: odd), real Ez, Bz (order 0: even)
    const float4 a = rec[0], b = rec[1];
    acc.f[0][1].x += w_odd * a.x;
    acc.f[0][1].y += w_odd * a.y;
    acc.f[0][4].x += w_odd * a.z;
    acc.f[0][4].y += w_odd * a.w;
    acc.f[0][2].x += w_even * b.x;
    acc.f[0][5].x += w_even * b.y;
  }
#pragma unroll
  for (int q = 0; q < 3 * (M - 1); ++q) {
    const float4 v = rec[2 + q];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = 2 * q + h;
      const int m = 1 + e / 6, c = e % 6;
      // Hankel order: m+1 (E+, B+), m-1 (E-, B-), m (Ez, Bz)
      const bool odd = (c % 3 == 2) ? (m & 1) : ((m + 1) & 1);
      const float w = odd ? w_odd : w_even;
      const float re = h ? v.z : v.x, im = h ? v.w : v.y;
      acc.f[m][c].x += w * re;
      acc.f[m][c].y += w * im;
    }
  }
}

// F_z = sum_{m=-M..M} F_{z,m} e^{-i m theta};
// F_x + i F_y = 2 [ sum_{m>=0} F_{-,m} e^{-i(m-1) theta} + sum_{m>=1} conj(F_{+,m}) e^{i(m+1) theta} ]
template <int M>
__device__ __forceinline__ void cartesian(const Gathered<M>& a, int cb, float2 e, float& fx, float& fy, float& fz) {
  float2 xy = cscale(cmul(a.f[0][cb + 1], e), 2.f);
  float zz = a.f[0][cb + 2].x;
  float2 em = e;
#pragma unroll
  for (int m = 1; m < M; ++m) {
    zz += 2.f * cmul(a.f[m][cb + 2], cconj(em)).x;
    float2 t1 = cmul(a.f[m][cb + 1], cmul(cconj(em), e));
    float2 t2 = cmul(cconj(a.f[m][cb + 0]), cmul(em, e));
    xy = cadd(xy, cscale(cadd(t1, t2), 2.f));
    em = cmul(em, e);
  }
  fx = xy.x;
  fy = xy.y;
  fz = zz;
}

template <int M, class Recs>
__device__ __forceinline__ void gather_eb(const Recs& rec, const ShapePos& s, const Grid& g, float& Ex, float& Ey,
                                          float& Ez, float& Bx, float& By, float& Bz) {
  Gathered<M> a;
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int c = 0; c < 6; ++c) a.f[m][c] = make_float2(0.f, 0.f);
  const int ja = s.j0, jb = (s.j0 + 1 == g.nz) ? 0 : s.j0 + 1;
  const float wza = 1.f - s.fz, wzb = s.fz;
  const float wra = 1.f - s.fr, wrb = s.fr;
  const int ia = s.i0, ib = s.i0 + 1;
  if (ia == -1) {              // ghost across the axis: node 0 with (-1)^nu
    gather_node<M>(a, rec(0, ja), wra * wza, -wra * wza);
    gather_node<M>(a, rec(0, jb), wra * wzb, -wra * wzb);
  } else if (ia >= 0 && ia < g.nr) {
    gather_node<M>(a, rec(ia, ja), wra * wza, wra * wza);
    gather_node<M>(a, rec(ia, jb), wra * wzb, wra * wzb);
  }
  if (ib >= 0 && ib < g.nr) {
    gather_node<M>(a, rec(ib, ja), wrb * wza, wrb * wza);
    gather_node<M>(a, rec(ib, jb), wrb * wzb, wrb * wzb);
  }
  cartesian<M>(a, 0, s.eith, Ex, Ey, Ez);
  cartesian<M>(a, 3, s.eith, Bx, By, Bz);
}

// Cubic B-spline gather (an option): the 4 x 4 nodes -1 .. 2 around the
// cell start along z (periodic) and r; ghost nodes -1, -2 across the axis
// read nodes 0, 1 with the factor (-1)^nu; nodes at i >= nr are outside.
__device__ __forceinline__ void cubic_wts(float f, float (&w)[4]) {
  const float g = 1.f - f;
  w[0] = g * g * g * (1.f / 6.f);
  w[1] = (4.f - 6.f * f * f + 3.f * f * f * f) * (1.f / 6.f);
  w[2] = (4.f - 6.f * g * g + 3.f * g * g * g) * (1.f / 6.f);
  w[3] = f * f * f * (1.f / 6.f);
}

template <int M, class Recs>
__device__ __forceinline__ void gather_eb_cubic(const Recs& rec, const ShapePos& s, const Grid& g, float& Ex,
                                                float& Ey, float& Ez, float& Bx, float& By, float& Bz) {
  Gathered<M> a;
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int c = 0; c < 6; ++c) a.f[m][c] = make_float2(0.f, 0.f);
  float wz[4], wr[4];
  cubic_wts(s.fz, wz);
  cubic_wts(s.fr, wr);
  for (int q = 0; q < 4; ++q) {
    int i = s.i0 - 1 + q;
    const bool ghost = i < 0;
    if (ghost) i = -1 - i;
    if (i >= g.nr) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int j = (s.j0 - 1 + b) & (g.nz - 1);   // nz is a power of two
      const float w = wr[q] * wz[b];
      gather_node<M>(a, rec(i, j), w, ghost ? -w : w);
    }
  }
  cartesian<M>(a, 0, s.eith, Ex, Ey, Ez);
  cartesian<M>(a, 3, s.eith, Bx, By, Bz);
}

// --------------------------------------------------------------------------
// gather + Boris push + move + new cell key + key histogram, one particle per
// thread.  Measured at 2048 x 256: one particle per thread beats two, three or
// four with all their loads issued first (fewer VGPRs, more wavefronts).
// --------------------------------------------------------------------------
struct PushRec {
  double x, y, z, uz;
  float ux, uy;
  uint8_t sp;
};

// Boris rotation (J. P. Boris, 1970) and move; returns the new cell key.  The
// transverse momenta and all increments are FP32; u_z accumulates its
// increments in FP64.
__device__ __forceinline__ uint32_t boris_move(PushRec& r, float qm, float Ex, float Ey, float Ez, float Bx, float By,
                                               float Bz, const Grid& g, double zmin) {
  float eps = qm * (float)g.dt * 0.5f;
  float umx = r.ux + eps * Ex, umy = r.uy + eps * Ey;
  double umz = r.uz + (double)(eps * Ez);
  float fmz = (float)umz;
  const float igm = rsqrtf(1.f + umx * umx + umy * umy + fmz * fmz);   // 1 / gamma at u^-
  float tx = eps * Bx * igm, ty = eps * By * igm, tz = eps * Bz * igm;
  float sfac = 2.f / (1.f + tx * tx + ty * ty + tz * tz);
  float sx = sfac * tx, sy = sfac * ty, sz = sfac * tz;
  float dpz = umx * ty - umy * tx;
  float upx = umx + (umy * tz - fmz * ty);
  float upy = umy + (fmz * tx - umx * tz);
  float upz = (float)(umz + (double)dpz);
  float uqx = umx + (upy * sz - upz * sy);
  float uqy = umy + (upz * sx - upx * sz);
  r.ux = uqx + eps * Ex;
  r.uy = uqy + eps * Ey;
  r.uz = umz + (double)(upx * sy - upy * sx) + (double)(eps * Ez);
  double ginv = rsqrt_f64(1.0 + (double)r.ux * r.ux + (double)r.uy * r.uy + r.uz * r.uz);
  r.x += g.dt * ((double)r.ux * ginv);
  r.y += g.dt * ((double)r.uy * ginv);
  r.z += g.dt * (r.uz * ginv);
  return cell_key(shape_at(r.x, r.y, r.z, zmin, g), g);
}

// Field records a workgroup may stage in LDS.  Sorted by cell, the 256
// particles of a workgroup usually sit in a few cells of one z column: their
// nodes form a small box of records, which the workgroup copies into LDS with
// coalesced loads once, and every particle then reads its records from LDS
// instead of through L1 (the records, read with 16-byte loads by every
// particle, dominate the gather's cost).  A workgroup whose box is larger (a
// column boundary inside it, a scrambled or sparse region) reads the records
// from the HBM copy.
constexpr int kStageRecs = 128;

template <int M, int SHAPE>
__global__ __launch_bounds__(256) void k_gather_push(Parts p, const float2* __restrict__ gf, Grid g, SpeciesConst sc,
                                                     const DevState* __restrict__ st, uint32_t* __restrict__ key,
                                                     int* __restrict__ count) {
  constexpr int R4 = rec_f2(M) / 2;   // float4 per record
  __shared__ float4 stage[kStageRecs * R4];
  __shared__ int wbox[4][4];
  const int n = st->n_part;
  // XCD-aware order: the hardware deals workgroups round-robin over the 8
  // XCDs; each XCD gets one contiguous range of the active blocks, so the
  // field nodes shared by neighbouring particles stay in one L2
  const int nact = (n + 255) / 256;
  const int bx = blockIdx.x;
  if (bx >= nact) return;
  const int q8 = nact >> 3, r8 = nact & 7, x8 = bx & 7;
  const int lb = x8 * q8 + min(x8, r8) + (bx >> 3);
  const int tid = threadIdx.x;
  const int i = lb * 256 + tid;
  const double zmin = st->zmin;
  const bool kill = g.moving_window && st->n_shift > 0;
  const GlobalRecs<M> grec{reinterpret_cast<const float4*>(gf), g.nz};
  PushRec r;
  bool live = false;
  uint32_t k = kInvalidKey;
  if (i < n) {
    r.x = p.x[i];
    r.y = p.y[i];
    r.z = p.z[i];
    r.uz = p.uz[i];
    r.ux = p.ux[i];
    r.uy = p.uy[i];
    r.sp = p.sp[i];
    live = !(kill && r.z < zmin);
    if (!live) k = (uint32_t)g.ncells;
  }
  ShapePos s;
  if (live) s = shape_at(r.x, r.y, r.z, zmin, g);
  float Ex = 0.f, Ey = 0.f, Ez = 0.f, Bx = 0.f, By = 0.f, Bz = 0.f;
  {
    // box of the records the workgroup reads, over its particles: linear
    // shapes rows max(i0, 0) .. min(i0 + 1, nr - 1) (the ghost row -1 reads
    // row 0), columns j0 .. j0 + 1; cubic shapes rows max(i0 - 1, 0) ..
    // min(i0 + 2, nr - 1) (ghost rows -1, -2 read rows 0, 1), columns
    // j0 - 1 .. j0 + 2.  A box that wraps around z is not staged.
    constexpr int kLo = SHAPE == 3 ? 1 : 0, kHi = SHAPE == 3 ? 2 : 1;
    int ilo = INT_MAX, ihi = INT_MIN, jlo = INT_MAX, jhi = INT_MIN;
    if (live) {
      const int a = s.i0 - kLo < 0 ? 0 : s.i0 - kLo;
      const int b = s.i0 + kHi < g.nr ? s.i0 + kHi : g.nr - 1;
      if (a <= b) {
        ilo = a;
        ihi = b;
        jlo = s.j0 - kLo;
        jhi = s.j0 + kHi;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      ilo = min(ilo, __shfl_xor(ilo, off, 64));
      ihi = max(ihi, __shfl_xor(ihi, off, 64));
      jlo = min(jlo, __shfl_xor(jlo, off, 64));
      jhi = max(jhi, __shfl_xor(jhi, off, 64));
    }
    const int wv = tid >> 6;
    if ((tid & 63) == 0) {
      wbox[wv][0] = ilo;
      wbox[wv][1] = ihi;
      wbox[wv][2] = jlo;
      wbox[wv][3] = jhi;
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      ilo = min(ilo, wbox[v][0]);
      ihi = max(ihi, wbox[v][1]);
      jlo = min(jlo, wbox[v][2]);
      jhi = max(jhi, wbox[v][3]);
    }
    const bool any = ilo <= ihi;   // some thread reads a record
    const int ni = any ? ihi - ilo + 1 : 0, nj = any ? jhi - jlo + 1 : 0;
    const bool staged = any && jlo >= 0 && jhi < g.nz && ni * nj <= kStageRecs;   // uniform over the workgroup
    if (staged) {
      const int total = ni * nj * R4;
      for (int q = tid; q < total; q += 256) {
        const int rec = q / R4, part = q - rec * R4;
        const int ii = rec / nj, jj = rec - ii * nj;
        stage[q] = grec(ilo + ii, jlo + jj)[part];
      }
      __syncthreads();
      const float4* st4 = stage;
      const auto lrec = [=](int ii, int jj) { return st4 + ((ii - ilo) * nj + (jj - jlo)) * R4; };
      if (live) {
        if constexpr (SHAPE == 3) gather_eb_cubic<M>(lrec, s, g, Ex, Ey, Ez, Bx, By, Bz);
        else gather_eb<M>(lrec, s, g, Ex, Ey, Ez, Bx, By, Bz);
      }
    } else if (live) {
      if constexpr (SHAPE == 3) gather_eb_cubic<M>(grec, s, g, Ex, Ey, Ez, Bx, By, Bz);
      else gather_eb<M>(grec, s, g, Ex, Ey, Ez, Bx, By, Bz);
    }
  }
  if (live) k = boris_move(r, sc.qm[r.sp], Ex, Ey, Ez, Bx, By, Bz, g, zmin);
  if (i < n) {
    if (k != (uint32_t)g.ncells) {
      p.x[i] = r.x;
      p.y[i] = r.y;
      p.z[i] = r.z;
      p.uz[i] = r.uz;
      p.ux[i] = r.ux;
      p.uy[i] = r.uy;
    }
    key[i] = k;
  }
  wave_count(k, count);
}

// key + histogram of the current positions (no push): background deposit at setup
__global__ __launch_bounds__(256) void k_keys(Parts p, Grid g, const DevState* __restrict__ st,
                                              uint32_t* __restrict__ key, int* __restrict__ count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = st->n_part;
  uint32_t k = kInvalidKey;
  if (i < n) {
    k = cell_key(shape_at(p.x[i], p.y[i], p.z[i], st->zmin, g), g);
    key[i] = k;
  }
  wave_count(k, count);
}

// --------------------------------------------------------------------------
// exclusive scan of the ncells + 1 bucket counts in 2 passes: block totals,
// then every block adds up the totals of the blocks before it (a few hundred
// to two thousand values) and scans its own counts
// --------------------------------------------------------------------------
constexpr int kScanPerThread = 8;
constexpr int kScanBlock = 256 * kScanPerThread;

// wavefront scans (shuffles) and the four wavefront totals through LDS
__device__ __forceinline__ int block_exclusive_scan(int v, int* sh, int& total) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int inc = v;
  for (int d = 1; d < 64; d <<= 1) {
    const int u = __shfl_up(inc, d, 64);
    if (lane >= d) inc += u;
  }
  if (lane == 63) sh[w] = inc;
  __syncthreads();
  int pre = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) pre += i < w ? sh[i] : 0;
  total = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return pre + inc - v;
}

typedef int intx4 __attribute__((ext_vector_type(4)));

// a thread's kScanPerThread consecutive counts (zero past n); the arrays start
// 256-byte aligned, so a full group is two aligned 16-byte loads
__device__ __forceinline__ void load_counts(const int* __restrict__ c, int base, int n, int (&v)[kScanPerThread]) {
  static_assert(kScanPerThread == 8, "two 16-byte vectors per thread");
  if (base + 8 <= n) {
    const intx4 a = *reinterpret_cast<const intx4*>(c + base);
    const intx4 b = *reinterpret_cast<const intx4*>(c + base + 4);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      v[e] = a[e];
      v[e + 4] = b[e];
    }
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = base + e < n ? c[base + e] : 0;
  }
}

__global__ __launch_bounds__(256) void k_scan_blocks(const int* __restrict__ count, int n, int* __restrict__ bsum) {
  __shared__ int sh[4];
  const int base = blockIdx.x * kScanBlock + threadIdx.x * kScanPerThread;
  int v[kScanPerThread];
  load_counts(count, base, n, v);
  int s = 0;
#pragma unroll
  for (int e = 0; e < kScanPerThread; ++e) s += v[e];
  int total;
  block_exclusive_scan(s, sh, total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// writes offset[0..n] (offset[n] = total), cursor = offset, count = 0;
// n_live = offset[ncells] (everything except the removed bucket)
__global__ __launch_bounds__(256) void k_scan_apply(int* __restrict__ count, int n, const int* __restrict__ bsum,
                                                    int* __restrict__ offset, int* __restrict__ cursor,
                                                    int ncells, DevState* st) {
  __shared__ int sh[4];
  __shared__ int wpart[4];
  // this block's offset: the totals of the blocks before it
  int pre = 0;
  for (int i = threadIdx.x; i < (int)blockIdx.x; i += 256) pre += bsum[i];
  for (int off = 32; off > 0; off >>= 1) pre += __shfl_xor(pre, off, 64);
  if ((threadIdx.x & 63) == 0) wpart[threadIdx.x >> 6] = pre;
  const int base = blockIdx.x * kScanBlock + threadIdx.x * kScanPerThread;
  int v[kScanPerThread];
  load_counts(count, base, n, v);
  int s = 0;
#pragma unroll
  for (int e = 0; e < kScanPerThread; ++e) s += v[e];
  int total;
  int ex = block_exclusive_scan(s, sh, total);   // its barriers also publish wpart
  ex += wpart[0] + wpart[1] + wpart[2] + wpart[3];
  int o[kScanPerThread];
#pragma unroll
  for (int e = 0; e < kScanPerThread; ++e) {
    o[e] = ex;
    ex += v[e];
  }
  if (base + 8 <= n) {
    const intx4 a = {o[0], o[1], o[2], o[3]}, b = {o[4], o[5], o[6], o[7]}, z = {0, 0, 0, 0};
    *reinterpret_cast<intx4*>(offset + base) = a;
    *reinterpret_cast<intx4*>(offset + base + 4) = b;
    *reinterpret_cast<intx4*>(cursor + base) = a;
    *reinterpret_cast<intx4*>(cursor + base + 4) = b;
    *reinterpret_cast<intx4*>(count + base) = z;
    *reinterpret_cast<intx4*>(count + base + 4) = z;
  } else {
#pragma unroll
    for (int e = 0; e < kScanPerThread; ++e)
      if (base + e < n) {
        offset[base + e] = o[e];
        cursor[base + e] = o[e];
        count[base + e] = 0;
      }
  }
#pragma unroll
  for (int e = 0; e < kScanPerThread; ++e) {
    const int idx = base + e;
    if (idx == ncells) st->n_live = o[e];
    if (idx == n - 1) offset[n] = o[e] + v[e];
  }
}

// --------------------------------------------------------------------------
// scatter into cell order (removed particles dropped).  Block-level
// multisplit: every run of equal keys in a block reserves one contiguous range
// of its cell with a single atomic, and thread t writes the t-th particle of
// the block in key order, so particles bound for one cell leave as one
// contiguous run even when the wake has scrambled the input order.
//
// The input is the previous step's sorted order pushed by at most a cell (a
// window move lowers every key alike), so most blocks arrive with ascending
// keys: such a block reserves its runs while its particle records are still in
// flight and writes them from registers.  Any other block sorts its 256 keys
// (bitonic network on key then original index, so the order is stable; in
// registers, with LDS only for the stages whose partners sit in another
// wavefront) and stages its records in LDS.
// --------------------------------------------------------------------------
struct PartRec {
  double x, y, z, uz;
  float ux, uy, w;
  uint32_t sp;
};

__device__ __forceinline__ uint32_t scatter_key(const uint32_t* __restrict__ key, int i, int n, int ncells) {
  const uint32_t k = (i >= 0 && i < n) ? key[i] : kInvalidKey;
  return k >= (uint32_t)ncells ? kInvalidKey : k;   // removed or past the end
}

// run head of every thread of the block from the per-thread "first of a run"
// flags: the nearest head at or below tid.  wlast[w] is the last head of
// wavefront w (-1 if none); thread 0 is always a head.
__device__ __forceinline__ int run_head(bool first, int* wlast) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint64_t heads = __ballot(first);
  if (lane == 0) wlast[w] = heads ? (w << 6) + 63 - __clzll((long long)heads) : -1;
  __syncthreads();
  const uint64_t upto = heads & ((lane == 63) ? ~0ull : ((2ull << lane) - 1ull));
  if (upto) return (w << 6) + 63 - __clzll((long long)upto);
  int h = -1;
  for (int v = 0; v < w; ++v) h = wlast[v] > h ? wlast[v] : h;
  return h;
}

struct ScatterLds {
  uint64_t sk[256];     // (key << 32) | local index
  PartRec rec[256];
  int base_of[256];     // destination of the run headed at t
  int wlast[4];
};

__device__ __forceinline__ void write_rec(const Parts& dst, int d, double x, double y, double z, double uz, float ux,
                                          float uy, float w, uint32_t sp) {
  dst.x[d] = x;
  dst.y[d] = y;
  dst.z[d] = z;
  dst.ux[d] = ux;
  dst.uy[d] = uy;
  dst.uz[d] = uz;
  dst.w[d] = w;
  dst.sp[d] = (uint8_t)sp;
}

// Thread tid of the block holds the record of key k (k_prev, k_next: the keys
// of the neighbouring input positions; kInvalidKey drops a particle).  Every
// thread of the block calls this.  The record travels as scalars: held in a
// struct, the two write-outs below are merged over a pointer that is either
// the registers' stack copy or LDS, and the copy lands in scratch memory.
__device__ __forceinline__ void scatter_block(ScatterLds& L, uint32_t k, uint32_t k_prev, uint32_t k_next, double x,
                                              double y, double z, double uz, float ux, float uy, float w, uint32_t sp,
                                              const Parts& dst, int* __restrict__ cursor) {
  const int tid = threadIdx.x;
  const bool ascending = __syncthreads_and(tid == 255 || k <= k_next);
  if (ascending) {
    const int h = run_head(tid == 0 || k_prev != k, L.wlast);
    const bool last = tid == 255 || k_next != k;
    if (last && k != kInvalidKey) L.base_of[h] = atomicAdd(&cursor[k], tid - h + 1);
    __syncthreads();
    if (k != kInvalidKey) write_rec(dst, L.base_of[h] + (tid - h), x, y, z, uz, ux, uy, w, sp);
    return;
  }
  if (k != kInvalidKey) {
    PartRec& q = L.rec[tid];
    q.x = x;
    q.y = y;
    q.z = z;
    q.uz = uz;
    q.ux = ux;
    q.uy = uy;
    q.w = w;
    q.sp = sp;
  }
  uint64_t e = ((uint64_t)k << 32) | (uint32_t)tid;
  // partners within a wavefront exchange through __shfl_xor, the three stages
  // with stride >= 64 through LDS
  for (int size = 2; size <= 256; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      uint64_t other;
      if (stride >= 64) {
        L.sk[tid] = e;
        __syncthreads();
        other = L.sk[tid ^ stride];
        __syncthreads();
      } else {
        const uint32_t lo = __shfl_xor((uint32_t)e, stride, 64);
        const uint32_t hi = __shfl_xor((uint32_t)(e >> 32), stride, 64);
        other = ((uint64_t)hi << 32) | lo;
      }
      const bool keep_min = ((tid & stride) == 0) == ((tid & size) == 0);
      e = keep_min ? (other < e ? other : e) : (other > e ? other : e);
    }
  }
  L.sk[tid] = e;
  __syncthreads();
  const uint32_t mk = (uint32_t)(e >> 32);
  const bool first = (tid == 0) || ((uint32_t)(L.sk[tid - 1] >> 32) != mk);
  const bool last = (tid == 255) || ((uint32_t)(L.sk[tid + 1] >> 32) != mk);
  const int h = run_head(first, L.wlast);
  if (last && mk != kInvalidKey) L.base_of[h] = atomicAdd(&cursor[mk], tid - h + 1);
  __syncthreads();
  if (mk != kInvalidKey) {
    const PartRec& q = L.rec[(uint32_t)e];
    write_rec(dst, L.base_of[h] + (tid - h), q.x, q.y, q.z, q.uz, q.ux, q.uy, q.w, q.sp);
  }
}

// the copy into cell order of the pushed particles
__global__ __launch_bounds__(256) void k_scatter(Parts src, Parts dst, const uint32_t* __restrict__ key,
                                                 int* __restrict__ cursor, const DevState* __restrict__ st,
                                                 int ncells) {
  __shared__ ScatterLds L;
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int n = st->n_part;
  const uint32_t k = scatter_key(key, i, n, ncells);
  const uint32_t k_prev = scatter_key(key, i - 1, n, ncells);
  const uint32_t k_next = scatter_key(key, i + 1, n, ncells);
  double x = 0.0, y = 0.0, z = 0.0, uz = 0.0;
  float ux = 0.f, uy = 0.f, w = 0.f;
  uint32_t sp = 0;
  if (i < n) {   // requested before the reservation; a removed particle's record goes unused
    x = src.x[i];
    y = src.y[i];
    z = src.z[i];
    ux = src.ux[i];
    uy = src.uy[i];
    uz = src.uz[i];
    w = src.w[i];
    sp = src.sp[i];
  }
  scatter_block(L, k, k_prev, k_next, x, y, z, uz, ux, uy, w, sp, dst, cursor);
}

// --------------------------------------------------------------------------
// head injection after a window move: one cold lattice column per injecting
// species, appended behind the sorted particles
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_inject(Parts p, DevState* st, Grid g, InjectTable tab, int cap) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int base = st->n_live;
  if (t == 0) {
    int want = base + tab.total;
    st->n_part = want <= cap ? want : cap;
    if (want > cap) st->overflow = 1;
  }
  if (t >= tab.total) return;
  int sidx = 0;
  while (sidx + 1 < tab.ns && t >= tab.start[sidx + 1]) ++sidx;
  int loc = t - tab.start[sidx];
  const int pz = tab.ppc_z[sidx], pr = tab.ppc_r[sidx], pt = tab.ppc_t[sidx];
  int l = loc % pt;
  loc /= pt;
  int b = loc % pr;
  loc /= pr;
  int a = loc % pz;
  int i = loc / pz;
  double zmin = st->zmin;
  double z = zmin + ((double)(g.nz - 1) + (a + 0.5) / pz) * g.dz;
  double r = ((double)i + (b + 0.5) / pr) * g.dr;
  double th = 2.0 * M_PI * l / pt;
  double w = tab.density[sidx] * r * (g.dr / pr) * (g.dz / pz) * (2.0 * M_PI / pt);
  float wf = (float)w;
  int d = base + t;
  if (d >= cap) return;
  p.x[d] = r * cos(th);
  p.y[d] = r * sin(th);
  p.z[d] = z;
  p.ux[d] = 0.f;
  p.uy[d] = 0.f;
  p.uz[d] = 0.0;
  p.w[d] = (float)(tab.q[sidx] * (double)wf);
  p.sp[d] = (uint8_t)tab.sp[sidx];
}

// z-uniformity check of the real-space background rho (all modes): out[0] =
// max |rho(i,j) - rho(i,0)|, out[1] = max |rho| (float bits as uint max)
__global__ void k_uniform_check(const float2* __restrict__ rho, int rows, int nz, unsigned int* out) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * nz) return;
  int row = idx / nz;
  float2 v = rho[idx], v0 = rho[(size_t)row * nz];
  float d = fmaxf(fabsf(v.x - v0.x), fabsf(v.y - v0.y));
  float a = fmaxf(fabsf(v.x), fabsf(v.y));
  atomicMax(&out[0], __float_as_uint(d));
  atomicMax(&out[1], __float_as_uint(a));
}

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------
static inline int nblk(int64_t n, int b) { return (int)((n + b - 1) / b); }

void launch_gather_push(const Parts& p, const float2* gf, const Grid& g, const SpeciesConst& sc,
                        const DevState* st, uint32_t* key, int* count, int cap, hipStream_t s) {
  dim3 grid(nblk(cap, 256));
  if (g.shape == 3) {
    switch (g.nmodes) {
      case 1: hipLaunchKernelGGL((k_gather_push<1, 3>), grid, dim3(256), 0, s, p, gf, g, sc, st, key, count); break;
      case 2: hipLaunchKernelGGL((k_gather_push<2, 3>), grid, dim3(256), 0, s, p, gf, g, sc, st, key, count); break;
      case 3: hipLaunchKernelGGL((k_gather_push<3, 3>), grid, dim3(256), 0, s, p, gf, g, sc, st, key, count); break;
      default: hipLaunchKernelGGL((k_gather_push<4, 3>), grid, dim3(256), 0, s, p, gf, g, sc, st, key, count); break;
    }
    return;
  }
  switch (g.nmodes) {
    case 1: hipLaunchKernelGGL((k_gather_push<1, 1>), grid, dim3(256), 0, s, p, gf, g, sc, st, key, count); break;
    case 2: hipLaunchKernelGGL((k_gather_push<2, 1>), grid, dim3(256), 0, s, p, gf, g, sc, st, key, count); break;
    case 3: hipLaunchKernelGGL((k_gather_push<3, 1>), grid, dim3(256), 0, s, p, gf, g, sc, st, key, count); break;
    default: hipLaunchKernelGGL((k_gather_push<4, 1>), grid, dim3(256), 0, s, p, gf, g, sc, st, key, count); break;
  }
}
void launch_pack_gather(const float2* real, float2* gf, int nr, int nz, int M, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_gather, dim3(nblk((int64_t)nr * nz, 256)), dim3(256),
                     (size_t)256 * rec_f2(M) * sizeof(float2), s, real, gf, nr, nz, M);
}
void launch_keys(const Parts& p, const Grid& g, const DevState* st, uint32_t* key, int* count, int cap,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_keys, dim3(nblk(cap, 256)), dim3(256), 0, s, p, g, st, key, count);
}
int scan_scratch_ints(int n) { return nblk(n, kScanBlock) + 1; }
void launch_scan(int* count, int n, int* bsum, int* offset, int* cursor, int ncells, DevState* st, hipStream_t s) {
  int nb = nblk(n, kScanBlock);
  hipLaunchKernelGGL(k_scan_blocks, dim3(nb), dim3(256), 0, s, count, n, bsum);
  hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(256), 0, s, count, n, bsum, offset, cursor, ncells, st);
}
void launch_scatter(const Parts& src, const Parts& dst, const uint32_t* key, int* cursor, const DevState* st,
                    int ncells, int cap, hipStream_t s) {
  hipLaunchKernelGGL(k_scatter, dim3(nblk(cap, 256)), dim3(256), 0, s, src, dst, key, cursor, st, ncells);
}

void launch_inject(const Parts& p, DevState* st, const Grid& g, const InjectTable& tab, int cap, hipStream_t s) {
  hipLaunchKernelGGL(k_inject, dim3(nblk(tab.total > 0 ? tab.total : 1, 256)), dim3(256), 0, s, p, st, g, tab,
                     cap);
}
void launch_uniform_check(const float2* rho, int rows, int nz, unsigned int* out, hipStream_t s) {
  hipLaunchKernelGGL(k_uniform_check, dim3(nblk((int64_t)rows * nz, 256)), dim3(256), 0, s, rho, rows, nz, out);
}

}  // namespace pic
