// Discrete Hankel transform as a batched dense product on the matrix cores.
//
// For one (mode, component) the radial transform is Y = A X with A an n x n
// real matrix (backward: B_nu[i][k] = J_nu(k_k r_i); forward: F_nu, the
// pseudo-inverse of B_nu built once at set-up from an FP64 Jacobi SVD)
// and X the [n][nz] complex field seen as an n x 2nz real matrix, so the
// contraction runs on MFMA with the complex interleave untouched.
//
// Tiling (64-wide wavefronts): a workgroup of 4 waves computes a
// (32*BM) x (128*BN) output tile; each wave owns (32*BM) x (32*BN) as BM x BN
// blocks of the 32x32 MFMA accumulator.  K is staged through LDS in chunks of
// 16 with double buffering (register prefetch of the next chunk while the
// current one feeds the MFMAs).  A is stored transposed (at[k][m]) so both
// operand tiles are loaded as contiguous rows.
//
// FP32 path: v_mfma_f32_32x32x2_f32.  Split paths: every operand is split
// x = hi + lo (bfloat16, or float16 with lo scaled by 2^11) when it is read
// from LDS; hi*hi + (hi*lo + lo*hi) go through v_mfma_f32_32x32x16_{bf16,f16}
// with FP32 accumulation (the lo*lo term is dropped).
#include <cmath>

#include "common.h"
#include "launch.h"

namespace pic {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const floatx4* gcfloat4_p;

constexpr int KT = 16;

// Operand chunks move as 16-byte vectors (global loads into registers, LDS
// stores): against one float per load, 0.54 -> 0.69 of the matrix-core peak
// for 256 x 256 by 256 x 4096 products (12 of them, 128 x 128 tiles).  Rows of
// A^T and X start at multiples of 4 floats (n and ncols are multiples of 32
// and 128), so every vector is aligned when the matrices are.
template <int BM, int BN>
struct GemmTile {
  static constexpr int MT = 32 * BM;
  static constexpr int NT = 128 * BN;
  static constexpr int A_ELEMS = KT * MT;       // floats per A chunk
  static constexpr int B_ELEMS = KT * NT;
  static constexpr int A_VECS = A_ELEMS / 4;    // 16-byte vectors per chunk
  static constexpr int B_VECS = B_ELEMS / 4;
  static constexpr int A_PER_THR = (A_VECS + 255) / 256;
  static constexpr int B_PER_THR = (B_VECS + 255) / 256;
};

template <int BM, int BN>
__device__ __forceinline__ void load_chunk(gcfloat_p __restrict__ at, gcfloat_p __restrict__ x, int n, int ncols,
                                           int m0, int n0, int k0, floatx4* ra, floatx4* rb) {
  using T = GemmTile<BM, BN>;
  const int tid = threadIdx.x;
#pragma unroll
  for (int e = 0; e < T::A_PER_THR; ++e) {
    const int idx = tid + e * 256;
    if (T::A_VECS % 256 == 0 || idx < T::A_VECS) {
      const int kk = idx / (T::MT / 4), mm = 4 * (idx % (T::MT / 4));
      ra[e] = *(gcfloat4_p)(at + (size_t)(k0 + kk) * n + m0 + mm);
    }
  }
#pragma unroll
  for (int e = 0; e < T::B_PER_THR; ++e) {
    const int idx = tid + e * 256;
    const int kk = idx / (T::NT / 4), nn = 4 * (idx % (T::NT / 4));
    rb[e] = *(gcfloat4_p)(x + (size_t)(k0 + kk) * ncols + n0 + nn);
  }
}

// Output tile of this workgroup.  Workgroups are dealt round-robin to the
// 8 XCDs (each with its own L2); when the column tiles come in multiples of 8,
// the k-th workgroup of XCD x takes row tile k mod R of column tile
// 8 (k div R) + x, so all R row tiles of one column block (which read the same
// operand columns) run back to back on one XCD.  A bijection of the grid.
__device__ __forceinline__ void gemm_tile_of(int& rt, int& ct) {
  const int ncx = gridDim.x, nry = gridDim.y;
  if ((ncx & 7) != 0) {
    rt = blockIdx.y;
    ct = blockIdx.x;
    return;
  }
  const int lin = blockIdx.y * ncx + blockIdx.x;
  const int k = lin >> 3;
  rt = k % nry;
  ct = (k / nry) * 8 + (lin & 7);
}

template <int BM, int BN>
__device__ __forceinline__ void store_chunk(float* As, float* Bs, const floatx4* ra, const floatx4* rb) {
  using T = GemmTile<BM, BN>;
  const int tid = threadIdx.x;
#pragma unroll
  for (int e = 0; e < T::A_PER_THR; ++e) {
    const int idx = tid + e * 256;
    if (T::A_VECS % 256 == 0 || idx < T::A_VECS) reinterpret_cast<floatx4*>(As)[idx] = ra[e];
  }
#pragma unroll
  for (int e = 0; e < T::B_PER_THR; ++e) reinterpret_cast<floatx4*>(Bs)[tid + e * 256] = rb[e];
}

template <int BM, int BN>
__device__ __forceinline__ void store_out(gfloat_p __restrict__ y, int ncols, int m0, int n0, const floatx16 (&acc)[BM][BN]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j) {
      const int col = n0 + wave * 32 * BN + j * 32 + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = m0 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        y[(size_t)row * ncols + col] = acc[i][j][r];
      }
    }
}

// ---------------------------------------------------------------------------
// FP32
// ---------------------------------------------------------------------------
template <int BM, int BN>
__global__ __launch_bounds__(256) void k_gemm_f32(const float* const* __restrict__ AT, const float* const* __restrict__ X,
                                                  float* const* __restrict__ Y, int n, int ncols) {
  using T = GemmTile<BM, BN>;
  __shared__ __attribute__((aligned(16))) float As[2][T::A_ELEMS];
  __shared__ __attribute__((aligned(16))) float Bs[2][T::B_ELEMS];
  gcfloat_p at = (gcfloat_p)AT[blockIdx.z];
  gcfloat_p x = (gcfloat_p)X[blockIdx.z];
  gfloat_p y = (gfloat_p)Y[blockIdx.z];
  int rt, ct;
  gemm_tile_of(rt, ct);
  const int m0 = rt * T::MT, n0 = ct * T::NT;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  floatx16 acc[BM][BN];
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
  floatx4 ra[T::A_PER_THR], rb[T::B_PER_THR];
  load_chunk<BM, BN>(at, x, n, ncols, m0, n0, 0, ra, rb);
  store_chunk<BM, BN>(As[0], Bs[0], ra, rb);
  __syncthreads();
  const int nk = n / KT;
  for (int kc = 0; kc < nk; ++kc) {
    const int cur = kc & 1;
    if (kc + 1 < nk) load_chunk<BM, BN>(at, x, n, ncols, m0, n0, (kc + 1) * KT, ra, rb);
    const float* as = As[cur];
    const float* bs = Bs[cur];
#pragma unroll
    for (int kk = 0; kk < KT; kk += 2) {
      const int kr = kk + (lane >> 5);
      float a[BM], b[BN];
#pragma unroll
      for (int i = 0; i < BM; ++i) a[i] = as[kr * T::MT + i * 32 + (lane & 31)];
#pragma unroll
      for (int j = 0; j < BN; ++j) b[j] = bs[kr * T::NT + wave * 32 * BN + j * 32 + (lane & 31)];
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (kc + 1 < nk) store_chunk<BM, BN>(As[cur ^ 1], Bs[cur ^ 1], ra, rb);
    __syncthreads();
  }
  store_out<BM, BN>(y, ncols, m0, n0, acc);
}

// ---------------------------------------------------------------------------
// split hi + lo (bf16 or f16)
// ---------------------------------------------------------------------------
template <bool F16>
struct Split;

template <>
struct Split<false> {
  typedef bf16x8 vec;
  static constexpr float kLoScale = 1.f;
  static __device__ __forceinline__ void split8(const float* v, vec& hi, vec& lo) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      __bf16 h = (__bf16)v[e];
      hi[e] = h;
      lo[e] = (__bf16)(v[e] - (float)h);
    }
  }
};

template <>
struct Split<true> {
  typedef halfx8 vec;
  static constexpr float kLoScale = 2048.f;
  static __device__ __forceinline__ void split8(const float* v, vec& hi, vec& lo) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      _Float16 h = (_Float16)v[e];
      hi[e] = h;
      lo[e] = (_Float16)((v[e] - (float)h) * kLoScale);
    }
  }
};

template <bool F16>
__device__ __forceinline__ floatx16 mfma16(typename Split<F16>::vec a, typename Split<F16>::vec b, floatx16 c) {
  if constexpr (F16) return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  else return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

template <int BM, int BN, bool F16>
__global__ __launch_bounds__(256) void k_gemm_split(const float* const* __restrict__ AT, const float* const* __restrict__ X,
                                                    float* const* __restrict__ Y, int n, int ncols,
                                                    int* __restrict__ nonfinite) {
  using T = GemmTile<BM, BN>;
  using S = Split<F16>;
  __shared__ __attribute__((aligned(16))) float As[2][T::A_ELEMS];
  __shared__ __attribute__((aligned(16))) float Bs[2][T::B_ELEMS];
  gcfloat_p at = (gcfloat_p)AT[blockIdx.z];
  gcfloat_p x = (gcfloat_p)X[blockIdx.z];
  gfloat_p y = (gfloat_p)Y[blockIdx.z];
  int rt, ct;
  gemm_tile_of(rt, ct);
  const int m0 = rt * T::MT, n0 = ct * T::NT;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  floatx16 acc[BM][BN], acl[BM][BN];
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        acc[i][j][r] = 0.f;
        acl[i][j][r] = 0.f;
      }
  floatx4 ra[T::A_PER_THR], rb[T::B_PER_THR];
  load_chunk<BM, BN>(at, x, n, ncols, m0, n0, 0, ra, rb);
  store_chunk<BM, BN>(As[0], Bs[0], ra, rb);
  __syncthreads();
  const int nk = n / KT;
  for (int kc = 0; kc < nk; ++kc) {
    const int cur = kc & 1;
    if (kc + 1 < nk) load_chunk<BM, BN>(at, x, n, ncols, m0, n0, (kc + 1) * KT, ra, rb);
    const float* as = As[cur];
    const float* bs = Bs[cur];
    // one 32x32x16 step covers the whole chunk: lane holds k = 8*(lane/32) + 0..7
    const int kb = 8 * (lane >> 5);
    typename S::vec ah[BM], al[BM], bh[BN], bl[BN];
#pragma unroll
    for (int i = 0; i < BM; ++i) {
      float v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = as[(kb + e) * T::MT + i * 32 + (lane & 31)];
      S::split8(v, ah[i], al[i]);
    }
#pragma unroll
    for (int j = 0; j < BN; ++j) {
      float v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = bs[(kb + e) * T::NT + wave * 32 * BN + j * 32 + (lane & 31)];
      S::split8(v, bh[j], bl[j]);
    }
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int j = 0; j < BN; ++j) {
        acc[i][j] = mfma16<F16>(ah[i], bh[j], acc[i][j]);
        acl[i][j] = mfma16<F16>(ah[i], bl[j], acl[i][j]);
        acl[i][j] = mfma16<F16>(al[i], bh[j], acl[i][j]);
      }
    if (kc + 1 < nk) store_chunk<BM, BN>(As[cur ^ 1], Bs[cur ^ 1], ra, rb);
    __syncthreads();
  }
  const float inv = 1.f / S::kLoScale;
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] += acl[i][j][r] * inv;
  if (nonfinite) {
    // an operand beyond the halves' range (FP16: 65504) gives inf or NaN;
    // flag it for the caller's next synchronizing call
    bool bad = false;
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int j = 0; j < BN; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) bad = bad || !isfinite(acc[i][j][r]);
    if (__ballot(bad) != 0 && lane == 0) atomicOr(nonfinite, 1);
  }
  store_out<BM, BN>(y, ncols, m0, n0, acc);
}

// ---------------------------------------------------------------------------
// launcher: picks the tile from n (rows) and ncols
// ---------------------------------------------------------------------------
template <int BM, int BN>
static void launch_tile(const float* const* at, const float* const* x, float* const* y, int batch, int n, int ncols,
                        int prec, int* nonfinite, hipStream_t s) {
  using T = GemmTile<BM, BN>;
  dim3 grid(ncols / T::NT, n / T::MT, batch);
  if (prec == 0)
    hipLaunchKernelGGL((k_gemm_f32<BM, BN>), grid, dim3(256), 0, s, at, x, y, n, ncols);
  else if (prec == 1)
    hipLaunchKernelGGL((k_gemm_split<BM, BN, false>), grid, dim3(256), 0, s, at, x, y, n, ncols, nonfinite);
  else
    hipLaunchKernelGGL((k_gemm_split<BM, BN, true>), grid, dim3(256), 0, s, at, x, y, n, ncols, nonfinite);
}

// tile choice: rows per workgroup 32*BM with BM in {4, 2, 1} dividing n; BN = 1.
int gemm_tile_bm(int n, int pref_bm) {
  int bm = pref_bm;
  while (bm > 1 && (n % (32 * bm))) bm >>= 1;
  return bm;
}

// compute units of the current device (cached per device)
static int device_cus() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
    cached[dev] = v;
  }
  return cached[dev];
}

// Automatic tile (pref_bm = 0): the largest of 128, 64, 32 rows whose
// workgroups fill the compute units in nearly whole rounds (at least 90 % of
// the last round busy), else the one that wastes the least of its last round.
// At nr = 256, 2 nz = 4096: the 10 forward products take 64 rows (1280
// workgroups, 5 per unit; 128 rows would leave half of the third round idle),
// the 12 inverse ones 128 rows (768, 3 per unit).  The split products stop at
// 64 rows: their 128-row tile holds hi and lo accumulators in 256 registers
// per lane, one wavefront per SIMD.
int gemm_pick_bm(int n, int ncols, int batch, int pref_bm, int prec) {
  if (pref_bm > 0) return gemm_tile_bm(n, pref_bm);
  const double cus = device_cus();
  int best = 1;
  double best_eff = -1.0;
  for (int bm : {4, 2, 1}) {
    if (prec != 0 && bm > 2) continue;
    if (n % (32 * bm)) continue;
    const double rounds = (double)(ncols / 128) * (n / (32 * bm)) * batch / cus;
    const double eff = rounds / std::ceil(rounds);
    if (eff >= 0.9) return bm;
    if (eff > best_eff) {
      best_eff = eff;
      best = bm;
    }
  }
  return best;
}

void launch_dht_gemm(const float* const* at, const float* const* x, float* const* y, int batch, int n, int ncols,
                     int prec, int pref_bm, hipStream_t s, int* nonfinite) {
  const int bm = gemm_pick_bm(n, ncols, batch, pref_bm, prec);
  if (bm == 4) launch_tile<4, 1>(at, x, y, batch, n, ncols, prec, nonfinite, s);
  else if (bm == 2) launch_tile<2, 1>(at, x, y, batch, n, ncols, prec, nonfinite, s);
  else launch_tile<1, 1>(at, x, y, batch, n, ncols, prec, nonfinite, s);
}

}  // namespace pic
