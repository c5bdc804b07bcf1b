// Charge and current deposit: rho^n at x^n, J^{n+1/2} at x^{n+1/2} (velocity
// v^{n+1/2}) and rho^{n+1} at x^{n+1}, linear shapes, every azimuthal mode.
//
// Work decomposition (no global atomics anywhere):
//   * the (z, r) node grid is cut into TZ x TR tiles; a tile depends on the
//     particles whose x^{n+1} cell lies within a halo of (hz, hr) cells around
//     it (x^n and x^{n+1/2} are at most dt c away), read as contiguous ranges
//     of the cell-sorted particle arrays;
//   * k_tile_totals / k_tile_plan count those particles per tile and cut each
//     tile's list into chunks of at most kChunk particles (dense beam cores
//     hold thousands of particles per cell, the plasma sixteen), giving a
//     device-side work list;
//   * k_deposit processes one (tile, chunk) per workgroup, accumulating in
//     LDS; a single-chunk tile writes its nodes directly, a split tile writes
//     a partial tile that k_deposit_combine sums node by node.
// Within a wavefront consecutive lanes hold consecutive (cell-sorted)
// particles.  For each of the three positions, lanes sharing a cell form
// runs; the node contributions are summed along each run with DPP row shifts
// (runs are cut at 16-lane row boundaries) and only the run head issues the
// LDS atomics, so a cell holding a thousand particles costs a few atomics per
// row instead of a 64-way conflict per particle.
#include "common.h"
#include "launch.h"

namespace pic {

constexpr int kChunk = 16384;   // max particles per workgroup

__device__ __forceinline__ size_t dfidx(int c, int m, int M, int nr, int nz) {
  return ((size_t)c * M + m) * (size_t)nr * nz;
}

// ---------------------------------------------------------------------------
// planning
// ---------------------------------------------------------------------------
struct TileGeom {
  int TZ, TR, ntz, ntr, hz, hr;
};

__device__ __forceinline__ void tile_rows(const TileGeom& tg, const Grid& g, int t, int& J0, int& I0, int& nrow,
                                          int& jstart, int& clo, int& chi) {
  const int tz = t % tg.ntz, tr = t / tg.ntz;
  J0 = tz * tg.TZ;
  I0 = tr * tg.TR;
  nrow = tg.TZ + 2 * tg.hz + 1;
  jstart = J0 - tg.hz - 1;
  if (nrow >= g.nz) {
    nrow = g.nz;
    jstart = 0;
  }
  clo = I0 - tg.hr;                 // key column = i0 + 1 >= I0 - hr
  chi = I0 + tg.TR + tg.hr;         // i0 <= I0 + TR - 1 + hr
  if (clo < 0) clo = 0;
  if (chi > g.nr) chi = g.nr;
}

__device__ __forceinline__ int wrap_row(int j, int nz) {
  j %= nz;
  return j < 0 ? j + nz : j;
}

// one wavefront per tile: particles in the tile's cell window
__global__ __launch_bounds__(256) void k_tile_totals(const int* __restrict__ offset, Grid g, TileGeom tg, int ntiles,
                                                     int* __restrict__ nchunk) {
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (t >= ntiles) return;
  int J0, I0, nrow, jstart, clo, chi;
  tile_rows(tg, g, t, J0, I0, nrow, jstart, clo, chi);
  int s = 0;
  for (int r = lane; r < nrow; r += 64) {
    int jj = wrap_row(jstart + r, g.nz);
    s += offset[jj * g.ncol + chi + 1] - offset[jj * g.ncol + clo];
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

// lanes l .. l + dist of a run -> value at l (meaningful on run heads)
struct RunMask {
  int dist;        // lanes after this one in its run (within the row)
  bool head;
  bool s1, s2, s4, s8;  // wave-uniform: some run needs this step
};

__device__ __forceinline__ RunMask run_mask(uint32_t key) {
  const int lane = threadIdx.x & 63;
  uint32_t prev = __shfl_up(key, 1, 64);
  bool head = ((lane & 15) == 0) || (prev != key);
  uint64_t heads = __ballot(head);
  uint64_t after = (lane == 63) ? 0ull : (heads & ~((2ull << lane) - 1ull));
  int next = after ? (__ffsll((long long)after) - 1) : 64;
  RunMask rm;
  rm.head = head;
  rm.dist = next - lane - 1;
  rm.s1 = __ballot(rm.dist >= 1) != 0;
  rm.s2 = __ballot(rm.dist >= 2) != 0;
  rm.s4 = __ballot(rm.dist >= 4) != 0;
  rm.s8 = __ballot(rm.dist >= 8) != 0;
  return rm;
}

__device__ __forceinline__ float run_sum(float v, const RunMask& rm) {
  if (rm.s1) {
    float t = row_shl<0x101>(v);
    v += rm.dist >= 1 ? t : 0.f;
  }
  if (rm.s2) {
    float t = row_shl<0x102>(v);
    v += rm.dist >= 2 ? t : 0.f;
  }
  if (rm.s4) {
    float t = row_shl<0x104>(v);
    v += rm.dist >= 4 ? t : 0.f;
  }
  if (rm.s8) {
    float t = row_shl<0x108>(v);
    v += rm.dist >= 8 ? t : 0.f;
  }
  return v;
}

// ---------------------------------------------------------------------------
// per-position values.  Each entry: LDS slot (0 J+, 1 J-, 2 Jz, 3 rho^n,
// 4 rho^{n+1}), mode, real/imaginary part, parity of the Hankel order.
// Mode 0 of rho and Jz is real; J-,0 = conj(J+,0) is rebuilt at write-out.
// ---------------------------------------------------------------------------
template <int M>
struct RhoVals {
  static constexpr int K = 1 + 2 * (M - 1);
  float v[K];
  __device__ __forceinline__ void set(float qw, float2 e) {
    v[0] = qw;
    float2 em = e;
#pragma unroll
    for (int m = 1; m < M; ++m) {
      v[1 + 2 * (m - 1)] = qw * em.x;
      v[2 + 2 * (m - 1)] = qw * em.y;
      em = cmul(em, e);
    }
  }
  static __device__ __forceinline__ void meta(int k, int& mode, int& part, int& parity) {
    mode = k == 0 ? 0 : 1 + (k - 1) / 2;
    part = k == 0 ? 0 : (k - 1) & 1;
    parity = mode & 1;
  }
};

template <int M>
struct JVals {
  static constexpr int K = 3 + 6 * (M - 1);
  float v[K];
  __device__ __forceinline__ void set(float qw, float vx, float vy, float vz, float2 e) {
    // J+ = qw (vx - i vy)/2 e^{i(m+1)theta}; J- = qw (vx + i vy)/2 e^{i(m-1)theta}; Jz = qw vz e^{i m theta}
    const float2 ap = make_float2(0.5f * qw * vx, -0.5f * qw * vy);
    const float2 am = make_float2(0.5f * qw * vx, 0.5f * qw * vy);
    const float az = qw * vz;
    float2 p1 = cmul(ap, e);
    v[0] = p1.x;
    v[1] = p1.y;
    v[2] = az;
    float2 em = e;   // e^{i m theta}
#pragma unroll
    for (int m = 1; m < M; ++m) {
      float2 jp = cmul(ap, cmul(em, e));
      float2 jm = cmul(am, cmul(em, cconj(e)));
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
  // slot, mode, part, parity of the Hankel order
  static __device__ __forceinline__ void meta(int k, int& slot, int& mode, int& part, int& parity) {
    if (k < 3) {
      mode = 0;
      slot = k < 2 ? 0 : 2;
      part = k < 2 ? k : 0;
      parity = k < 2 ? 1 : 0;
      return;
    }
    const int q = (k - 3) % 6;
    mode = 1 + (k - 3) / 6;
    slot = q / 2;
    part = q & 1;
    parity = (slot == 2) ? (mode & 1) : ((mode + 1) & 1);
  }
};

template <int TZ, int TR>
struct Acc {
  float* a;   // [5][M][TR][TZ] float2 viewed as floats
  int J0, I0, M, nz, nr;
  __device__ __forceinline__ void add(int slot, int m, int part, int i, int j, float v) {
    int ir = i - I0;
    int jz = j - J0;
    if (jz < 0) jz += nz;
    if ((unsigned)ir >= (unsigned)TR || (unsigned)jz >= (unsigned)TZ) return;
    atomicAdd(a + 2 * ((((size_t)slot * M + m) * TR + ir) * TZ + jz) + part, v);
  }
};

// Sums a position's node contributions along the lane runs and lets run
// heads add them to the tile.  `s` must be the same for every lane of a run
// (runs are built from the cell key of this position).
template <int TZ, int TR, int K, class Meta>
__device__ __forceinline__ void flush_position(Acc<TZ, TR>& acc, const ShapePos& s, bool valid, const float (&v)[K],
                                               const RunMask& rm, const Grid& g, Meta meta) {
  const float wza = 1.f - s.fz, wzb = s.fz;
  const float wra = 1.f - s.fr, wrb = s.fr;
  const float w[4] = {wza * wra, wza * wrb, wzb * wra, wzb * wrb};   // (ja,ia) (ja,ib) (jb,ia) (jb,ib)
  float r[4][K];
#pragma unroll
  for (int n = 0; n < 4; ++n)
#pragma unroll
    for (int k = 0; k < K; ++k) r[n][k] = run_sum(valid ? w[n] * v[k] : 0.f, rm);
  if (!(rm.head && valid)) return;
  const int ja = s.j0, jb = (s.j0 + 1 == g.nz) ? 0 : s.j0 + 1;
  const bool ghost = (s.i0 == -1);
  const int ia = ghost ? 0 : s.i0, ib = s.i0 + 1;
  const bool a_ok = ia >= 0 && ia < g.nr;
  const bool b_ok = ib >= 0 && ib < g.nr;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    int slot, mode, part, parity;
    meta(k, slot, mode, part, parity);
    const float sa = (ghost && parity) ? -1.f : 1.f;
    if (a_ok) {
      acc.add(slot, mode, part, ia, ja, sa * r[0][k]);
      acc.add(slot, mode, part, ia, jb, sa * r[2][k]);
    }
    if (b_ok) {
      acc.add(slot, mode, part, ib, ja, r[1][k]);
      acc.add(slot, mode, part, ib, jb, r[3][k]);
    }
  }
}

// injective on the cells that can touch the grid (radial cells beyond the box
// share one key: none of their nodes exists)
__device__ __forceinline__ uint32_t pos_key(const ShapePos& s, int nr) {
  const int ic = (s.i0 > nr ? nr : s.i0) + 1;
  return (uint32_t)s.j0 * 2048u + (uint32_t)ic;
}

// rho^n, J, rho^{n+1} of every mode, value layout of the tile accumulator ->
// real-space grid (J-,0 = conj(J+,0); divide by the ring volume; add the
// immobile background to both densities)
template <int TZ, int TR>
__device__ __forceinline__ void finalize_tile(const float2* acc, float2* __restrict__ real, const float2* __restrict__ bg,
                                              const Grid& g, int J0, int I0) {
  const int M = g.nmodes, nr = g.nr, nz = g.nz;
  const int n = 5 * M * TR * TZ;
  const double vol0 = 2.0 * M_PI * g.dr * g.dr * g.dz;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int jz = e % TZ;
    int t = e / TZ;
    const int ir = t % TR;
    t /= TR;
    const int m = t % M;
    const int slot = t / M;
    const int i = I0 + ir;
    if (i >= nr) continue;
    float2 v = acc[e];
    if (slot == 1 && m == 0) v = cconj(acc[(((size_t)0 * M + 0) * TR + ir) * TZ + jz]);
    const float inv_v = (float)(1.0 / (vol0 * (i + 0.5)));
    v = cscale(v, inv_v);
    if (bg && slot >= 3) v = cadd(v, bg[((size_t)m * nr + i) * nz + J0 + jz]);
    real[dfidx(kCompJ + slot, m, M, nr, nz) + (size_t)i * nz + J0 + jz] = v;
  }
}

template <int TZ, int TR, int M>
__global__ __launch_bounds__(256) void k_deposit(Parts p, const int* __restrict__ offset,
                                                 const int* __restrict__ nchunk, const int* __restrict__ chunk_start,
                                                 float2* __restrict__ partial, float2* __restrict__ real,
                                                 const float2* __restrict__ bg, Grid g, TileGeom tg, int ntiles,
                                                 DevState* st) {
  extern __shared__ float2 lds_acc[];
  __shared__ int rowstart[160];
  __shared__ int rowpref[161];
  __shared__ int s_tile;
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  if (b == 0 && tid == 0) {
    st->n_part = st->n_live;
    if (chunk_start[ntiles] > (int)gridDim.x) st->overflow = 2;   // work list larger than the launch
  }
  if (b >= chunk_start[ntiles]) return;   // uniform per workgroup
  if (tid == 0) {
    int lo = 0, hi = ntiles;   // chunk_start[lo] <= b < chunk_start[hi]
    while (hi - lo > 1) {
      int mid = (lo + hi) >> 1;
      if (chunk_start[mid] <= b) lo = mid;
      else hi = mid;
    }
    s_tile = lo;
  }
  const int nacc = 5 * M * TR * TZ;
  for (int e = tid; e < nacc; e += blockDim.x) lds_acc[e] = make_float2(0.f, 0.f);
  __syncthreads();
  const int t = s_tile;
  const int chunk = b - chunk_start[t];
  const int nch = nchunk[t];
  int J0, I0, nrow, jstart, clo, chi;
  tile_rows(tg, g, t, J0, I0, nrow, jstart, clo, chi);
  if (tid < nrow) {
    int jj = wrap_row(jstart + tid, g.nz);
    int a = offset[jj * g.ncol + clo];
    rowstart[tid] = a;
    rowpref[tid + 1] = offset[jj * g.ncol + chi + 1] - a;
  }
  __syncthreads();
  if (tid == 0) {
    rowpref[0] = 0;
    for (int r = 1; r <= nrow; ++r) rowpref[r] += rowpref[r - 1];
  }
  __syncthreads();
  const int total = rowpref[nrow];
  const int f0 = chunk * kChunk;
  const int f1 = min(total, f0 + kChunk);
  Acc<TZ, TR> acc{(float*)lds_acc, J0, I0, M, g.nz, g.nr};
  const double zmin = st->zmin;
  const double dt = g.dt;
  const int lane = tid & 63, wave = tid >> 6;
  for (int base = f0 + wave * 64; base < f1; base += 256) {
    const int f = base + lane;
    const bool valid = f < f1;
    double x = 0.0, y = 0.0, z = zmin;
    float ux = 0.f, uy = 0.f, uz = 0.f, qw = 0.f;
    if (valid) {
      int lo = 0, hi = nrow;   // rowpref[lo] <= f < rowpref[hi]
      while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
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
    const float ginv = 1.f / sqrtf(1.f + ux * ux + uy * uy + uz * uz);
    const float vx = ux * ginv, vy = uy * ginv, vz = uz * ginv;
    // rho^{n+1} at x^{n+1}
    {
      ShapePos s = shape_at(x, y, z, zmin, g);
      RunMask rm = run_mask(valid ? pos_key(s, g.nr) : kInvalidKey);
      RhoVals<M> rv;
      rv.set(qw, s.eith);
      flush_position<TZ, TR, RhoVals<M>::K>(acc, s, valid, rv.v, rm, g,
                                            [](int k, int& slot, int& mode, int& part, int& parity) {
                                              slot = 4;
                                              RhoVals<M>::meta(k, mode, part, parity);
                                            });
    }
    // J^{n+1/2} at x^{n+1/2} = x^{n+1} - dt v / 2
    {
      ShapePos s = shape_at(x - 0.5 * dt * (double)vx, y - 0.5 * dt * (double)vy, z - 0.5 * dt * (double)vz,
                            zmin, g);
      RunMask rm = run_mask(valid ? pos_key(s, g.nr) : kInvalidKey);
      JVals<M> jv;
      jv.set(qw, vx, vy, vz, s.eith);
      flush_position<TZ, TR, JVals<M>::K>(acc, s, valid, jv.v, rm, g,
                                          [](int k, int& slot, int& mode, int& part, int& parity) {
                                            JVals<M>::meta(k, slot, mode, part, parity);
                                          });
    }
    // rho^n at x^n = x^{n+1} - dt v
    {
      ShapePos s = shape_at(x - dt * (double)vx, y - dt * (double)vy, z - dt * (double)vz, zmin, g);
      RunMask rm = run_mask(valid ? pos_key(s, g.nr) : kInvalidKey);
      RhoVals<M> rv;
      rv.set(qw, s.eith);
      flush_position<TZ, TR, RhoVals<M>::K>(acc, s, valid, rv.v, rm, g,
                                            [](int k, int& slot, int& mode, int& part, int& parity) {
                                              slot = 3;
                                              RhoVals<M>::meta(k, mode, part, parity);
                                            });
    }
  }
  __syncthreads();
  if (nch == 1) {
    finalize_tile<TZ, TR>(lds_acc, real, bg, g, J0, I0);
  } else {
    float2* dst = partial + (size_t)b * nacc;
    for (int e = tid; e < nacc; e += blockDim.x) dst[e] = lds_acc[e];
  }
}

// sums the partial tiles of split tiles and writes them
template <int TZ, int TR, int M>
__global__ __launch_bounds__(256) void k_deposit_combine(const int* __restrict__ nchunk,
                                                         const int* __restrict__ chunk_start,
                                                         const float2* __restrict__ partial,
                                                         float2* __restrict__ real, const float2* __restrict__ bg,
                                                         Grid g, TileGeom tg) {
  extern __shared__ float2 lds_acc[];
  const int t = blockIdx.x;
  const int nch = nchunk[t];
  if (nch == 1) return;
  const int nacc = 5 * M * TR * TZ;
  const float2* src = partial + (size_t)chunk_start[t] * nacc;
  for (int e = threadIdx.x; e < nacc; e += blockDim.x) {
    float2 s = make_float2(0.f, 0.f);
    for (int c = 0; c < nch; ++c) s = cadd(s, src[(size_t)c * nacc + e]);
    lds_acc[e] = s;
  }
  __syncthreads();
  const int J0 = (t % tg.ntz) * TZ, I0 = (t / tg.ntz) * TR;
  finalize_tile<TZ, TR>(lds_acc, real, bg, g, J0, I0);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
DepositShape deposit_shape(int nz, int nr, int nmodes, int hz, int hr, int64_t cap) {
  DepositShape d;
  d.TZ = 32;
  d.TR = nmodes <= 2 ? 16 : 8;
  d.ntz = nz / d.TZ;
  d.ntr = (nr + d.TR - 1) / d.TR;
  d.ntiles = d.ntz * d.ntr;
  // a cell lies in the windows (tile + halo) of at most mz x mr tiles
  const int64_t mz = (d.TZ + 2 * hz + 1 + d.TZ - 1) / d.TZ;
  const int64_t mr = (d.TR + 2 * hr + 1 + d.TR - 1) / d.TR;
  d.max_items = d.ntiles + (int)((mz * mr * cap + kChunk - 1) / kChunk);
  d.acc_floats2 = (size_t)5 * nmodes * d.TR * d.TZ;
  d.hz = hz;
  d.hr = hr;
  return d;
}

template <int TR, int M>
static void launch_dep(const Parts& p, const int* offset, int* nchunk, int* chunk_start, float2* partial,
                       float2* real, const float2* bg, const Grid& g, const DepositShape& d, DevState* st,
                       hipStream_t s) {
  TileGeom tg{d.TZ, d.TR, d.ntz, d.ntr, d.hz, d.hr};
  size_t lds = d.acc_floats2 * sizeof(float2);
  hipLaunchKernelGGL(k_tile_totals, dim3((d.ntiles + 3) / 4), dim3(256), 0, s, offset, g, tg, d.ntiles, nchunk);
  hipLaunchKernelGGL(k_tile_plan, dim3(1), dim3(1024), 0, s, nchunk, d.ntiles, chunk_start);
  hipLaunchKernelGGL((k_deposit<32, TR, M>), dim3(d.max_items), dim3(256), lds, s, p, offset, nchunk, chunk_start,
                     partial, real, bg, g, tg, d.ntiles, st);
  hipLaunchKernelGGL((k_deposit_combine<32, TR, M>), dim3(d.ntiles), dim3(256), lds, s, nchunk, chunk_start,
                     partial, real, bg, g, tg);
}

void launch_deposit(const Parts& p, const int* offset, const DepositShape& d, int* nchunk, int* chunk_start,
                    float2* partial, float2* real, const float2* bg, const Grid& g, DevState* st, hipStream_t s) {
  switch (g.nmodes) {
    case 1: launch_dep<16, 1>(p, offset, nchunk, chunk_start, partial, real, bg, g, d, st, s); break;
    case 2: launch_dep<16, 2>(p, offset, nchunk, chunk_start, partial, real, bg, g, d, st, s); break;
    case 3: launch_dep<8, 3>(p, offset, nchunk, chunk_start, partial, real, bg, g, d, st, s); break;
    default: launch_dep<8, 4>(p, offset, nchunk, chunk_start, partial, real, bg, g, d, st, s); break;
  }
}

}  // namespace pic
