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

// --------------------------------------------------------------------------
// field gather (Cartesian E, B at one position)
// --------------------------------------------------------------------------
struct Weights {
  int ja, jb;        // z nodes
  int ia, ib;        // radial nodes (ia clamped to 0 for the ghost)
  float wza, wzb;
  float wra_even, wra_odd, wrb;   // radial weights incl. fold sign / out-of-box zeroing
};

__device__ __forceinline__ Weights make_weights(const ShapePos& s, const Grid& g) {
  Weights w;
  w.ja = s.j0;
  w.jb = (s.j0 + 1 == g.nz) ? 0 : s.j0 + 1;
  w.wza = 1.f - s.fz;
  w.wzb = s.fz;
  float wa = 1.f - s.fr, wb = s.fr;
  int ia = s.i0, ib = s.i0 + 1;
  if (ia == -1) {
    w.ia = 0;
    w.wra_even = wa;
    w.wra_odd = -wa;
  } else if (ia >= g.nr || ia < -1) {
    w.ia = 0;
    w.wra_even = w.wra_odd = 0.f;
  } else {
    w.ia = ia;
    w.wra_even = w.wra_odd = wa;
  }
  if (ib >= g.nr || ib < 0) {
    w.ib = 0;
    w.wrb = 0.f;
  } else {
    w.ib = ib;
    w.wrb = wb;
  }
  return w;
}

__device__ __forceinline__ float2 interp(const float2* __restrict__ f, const Weights& w, bool odd, int nz) {
  float wra = odd ? w.wra_odd : w.wra_even;
  const float2* ra = f + (size_t)w.ia * nz;
  const float2* rb = f + (size_t)w.ib * nz;
  float2 a0 = ra[w.ja], a1 = ra[w.jb], b0 = rb[w.ja], b1 = rb[w.jb];
  float2 r;
  r.x = wra * (w.wza * a0.x + w.wzb * a1.x) + w.wrb * (w.wza * b0.x + w.wzb * b1.x);
  r.y = wra * (w.wza * a0.y + w.wzb * a1.y) + w.wrb * (w.wza * b0.y + w.wzb * b1.y);
  return r;
}

// F_z = sum_{m=-M..M} F_{z,m} e^{-i m theta};
// F_x + i F_y = 2 [ sum_{m>=0} F_{-,m} e^{-i(m-1) theta} + sum_{m>=1} conj(F_{+,m}) e^{i(m+1) theta} ]
__device__ __forceinline__ void gather_cart(const float2* __restrict__ real, int cbase, const ShapePos& s,
                                            const Weights& w, const Grid& g, float& fx, float& fy, float& fz) {
  const int M = g.nmodes, nr = g.nr, nz = g.nz;
  float2 xy = make_float2(0.f, 0.f);
  float zz = 0.f;
  float2 e = s.eith;                       // e^{i theta}
  float2 em = make_float2(1.f, 0.f);       // e^{i m theta}
  for (int m = 0; m < M; ++m) {
    bool odd_m = m & 1;
    float2 fzm = interp(real + fidx(cbase + 2, m, M, nr, nz), w, odd_m, nz);
    float2 fmm = interp(real + fidx(cbase + 1, m, M, nr, nz), w, !odd_m, nz);
    if (m == 0) {
      zz += fzm.x;
      xy = cadd(xy, cscale(cmul(fmm, e), 2.f));
    } else {
      float2 fpm = interp(real + fidx(cbase + 0, m, M, nr, nz), w, !odd_m, nz);
      zz += 2.f * cmul(fzm, cconj(em)).x;
      // e^{-i(m-1) theta} = conj(e^{i m theta}) e^{i theta}
      float2 t1 = cmul(fmm, cmul(cconj(em), e));
      float2 t2 = cmul(cconj(fpm), cmul(em, e));
      xy = cadd(xy, cscale(cadd(t1, t2), 2.f));
    }
    em = cmul(em, e);
  }
  fx = xy.x;
  fy = xy.y;
  fz = zz;
}

// --------------------------------------------------------------------------
// gather + Boris push + move + new cell key + key histogram
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gather_push(Parts p, const float2* __restrict__ real, Grid g,
                                                     SpeciesConst sc, const DevState* __restrict__ st,
                                                     uint32_t* __restrict__ key, int* __restrict__ count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = st->n_part;
  const double zmin = st->zmin;
  const bool kill = g.moving_window && st->n_shift > 0;
  uint32_t k = kInvalidKey;
  if (i < n) {
    double z = p.z[i];
    if (kill && z < zmin) {
      k = (uint32_t)g.ncells;
    } else {
      double x = p.x[i], y = p.y[i];
      float ux = p.ux[i], uy = p.uy[i], uz = p.uz[i];
      float qm = sc.qm[p.sp[i]];
      ShapePos s = shape_at(x, y, z, zmin, g);
      Weights w = make_weights(s, g);
      float Ex, Ey, Ez, Bx, By, Bz;
      gather_cart(real, 0, s, w, g, Ex, Ey, Ez);
      gather_cart(real, 3, s, w, g, Bx, By, Bz);
      // Boris rotation (J. P. Boris, 1970)
      float eps = qm * (float)g.dt * 0.5f;
      float umx = ux + eps * Ex, umy = uy + eps * Ey, umz = uz + eps * Ez;
      float gm = sqrtf(1.f + umx * umx + umy * umy + umz * umz);
      float tx = eps * Bx / gm, ty = eps * By / gm, tz = eps * Bz / gm;
      float sfac = 2.f / (1.f + tx * tx + ty * ty + tz * tz);
      float sx = sfac * tx, sy = sfac * ty, sz = sfac * tz;
      float upx = umx + (umy * tz - umz * ty);
      float upy = umy + (umz * tx - umx * tz);
      float upz = umz + (umx * ty - umy * tx);
      float uqx = umx + (upy * sz - upz * sy);
      float uqy = umy + (upz * sx - upx * sz);
      float uqz = umz + (upx * sy - upy * sx);
      ux = uqx + eps * Ex;
      uy = uqy + eps * Ey;
      uz = uqz + eps * Ez;
      float ginv = 1.f / sqrtf(1.f + ux * ux + uy * uy + uz * uz);
      x += g.dt * (double)(ux * ginv);
      y += g.dt * (double)(uy * ginv);
      z += g.dt * (double)(uz * ginv);
      p.x[i] = x;
      p.y[i] = y;
      p.z[i] = z;
      p.ux[i] = ux;
      p.uy[i] = uy;
      p.uz[i] = uz;
      k = cell_key(shape_at(x, y, z, zmin, g), g);
    }
    key[i] = k;
  }
  RunInfo ri = wave_runs(k);
  if (ri.head && k != kInvalidKey) atomicAdd(&count[k], ri.len);
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
  RunInfo ri = wave_runs(k);
  if (ri.head && k != kInvalidKey) atomicAdd(&count[k], ri.len);
}

// --------------------------------------------------------------------------
// exclusive scan of the ncells + 1 bucket counts (3 passes)
// --------------------------------------------------------------------------
constexpr int kScanPerThread = 8;
constexpr int kScanBlock = 256 * kScanPerThread;

__device__ __forceinline__ int block_exclusive_scan(int v, int* sh, int& total) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    int t = tid >= off ? sh[tid - off] : 0;
    __syncthreads();
    sh[tid] += t;
    __syncthreads();
  }
  total = sh[255];
  int ex = sh[tid] - v;
  __syncthreads();
  return ex;
}

__global__ __launch_bounds__(256) void k_scan_blocks(const int* __restrict__ count, int n, int* __restrict__ bsum) {
  __shared__ int sh[256];
  const int base = blockIdx.x * kScanBlock + threadIdx.x * kScanPerThread;
  int s = 0;
  for (int e = 0; e < kScanPerThread; ++e)
    if (base + e < n) s += count[base + e];
  int total;
  block_exclusive_scan(s, sh, total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(256) void k_scan_bsum(int* bsum, int nb) {
  __shared__ int sh[256];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int b0 = 0; b0 < nb; b0 += 256) {
    int i = b0 + threadIdx.x;
    int v = i < nb ? bsum[i] : 0;
    int total;
    int ex = block_exclusive_scan(v, sh, total);
    if (i < nb) bsum[i] = ex + carry;
    __syncthreads();
    if (threadIdx.x == 0) carry += total;
    __syncthreads();
  }
}

// writes offset[0..n] (offset[n] = total), cursor = offset, count = 0;
// n_live = offset[ncells] (everything except the removed bucket)
__global__ __launch_bounds__(256) void k_scan_apply(int* __restrict__ count, int n, const int* __restrict__ bsum,
                                                    int* __restrict__ offset, int* __restrict__ cursor,
                                                    int ncells, DevState* st) {
  __shared__ int sh[256];
  const int base = blockIdx.x * kScanBlock + threadIdx.x * kScanPerThread;
  int v[kScanPerThread];
  int s = 0;
  for (int e = 0; e < kScanPerThread; ++e) {
    v[e] = (base + e < n) ? count[base + e] : 0;
    s += v[e];
  }
  int total;
  int ex = block_exclusive_scan(s, sh, total) + bsum[blockIdx.x];
  for (int e = 0; e < kScanPerThread; ++e) {
    int idx = base + e;
    if (idx < n) {
      offset[idx] = ex;
      cursor[idx] = ex;
      count[idx] = 0;
      if (idx == ncells) st->n_live = ex;
      if (idx == n - 1) offset[n] = ex + v[e];
    }
    ex += v[e];
  }
}

// --------------------------------------------------------------------------
// scatter into cell order (removed particles dropped)
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_scatter(Parts src, Parts dst, const uint32_t* __restrict__ key,
                                                 int* __restrict__ cursor, const DevState* __restrict__ st,
                                                 int ncells) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = st->n_part;
  uint32_t k = (i < n) ? key[i] : kInvalidKey;
  if (k == (uint32_t)ncells) k = kInvalidKey;   // removed
  RunInfo ri = wave_runs(k);
  int base = 0;
  if (ri.head && k != kInvalidKey) base = atomicAdd(&cursor[k], ri.len);
  const int lane = threadIdx.x & 63;
  base = __shfl(base, ri.head_lane, 64);
  if (k != kInvalidKey) {
    int d = base + (lane - ri.head_lane);
    dst.x[d] = src.x[i];
    dst.y[d] = src.y[i];
    dst.z[d] = src.z[i];
    dst.ux[d] = src.ux[i];
    dst.uy[d] = src.uy[i];
    dst.uz[d] = src.uz[i];
    dst.w[d] = src.w[i];
    dst.sp[d] = src.sp[i];
  }
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
  p.uz[d] = 0.f;
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

void launch_gather_push(const Parts& p, const float2* real, const Grid& g, const SpeciesConst& sc,
                        const DevState* st, uint32_t* key, int* count, int cap, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_push, dim3(nblk(cap, 256)), dim3(256), 0, s, p, real, g, sc, st, key, count);
}
void launch_keys(const Parts& p, const Grid& g, const DevState* st, uint32_t* key, int* count, int cap,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_keys, dim3(nblk(cap, 256)), dim3(256), 0, s, p, g, st, key, count);
}
int scan_scratch_ints(int n) { return nblk(n, kScanBlock) + 1; }
void launch_scan(int* count, int n, int* bsum, int* offset, int* cursor, int ncells, DevState* st, hipStream_t s) {
  int nb = nblk(n, kScanBlock);
  hipLaunchKernelGGL(k_scan_blocks, dim3(nb), dim3(256), 0, s, count, n, bsum);
  hipLaunchKernelGGL(k_scan_bsum, dim3(1), dim3(256), 0, s, bsum, nb);
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
