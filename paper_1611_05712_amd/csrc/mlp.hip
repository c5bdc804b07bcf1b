// Surrogate network: forward, backward and Adam kernels of a small GELU
// multilayer perceptron, plus the C interface of include/mlp.h.
//
// Matrix products (forward layer, gradient of a layer's input, gradient of
// its weights), C(m, n) = sum_k A(m, k) B(k, n) with operands read through
// strides (the transposes of the backward pass cost nothing):
//   * both operands bfloat16 (the BF16 mode's hidden layers and gradients):
//     matrix cores, v_mfma_f32_32x32x16_bf16 with FP32 accumulation; each
//     wavefront computes one 32 x 32 output tile, four per workgroup;
//   * otherwise (FP32 mode, and the layer that reads the FP32 input
//     features): a 256-thread workgroup per 32 x 32 output tile staging
//     32-deep slices of both operands in LDS, each thread accumulating 2 x 2.
// The bias, GELU and GELU-derivative steps are fused into the epilogue.
#include <cmath>
#include <type_traits>
#include <vector>

#include "common.h"
#include "mlp.h"

namespace pic {
namespace {

constexpr size_t kMlpAlign = 256;

// bfloat16 <-> float32, round to nearest even (finite values)
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float ld(const float* p, size_t i) { return p[i]; }
__device__ __forceinline__ float ld(const uint16_t* p, size_t i) { return bf2f(p[i]); }
__device__ __forceinline__ void st(float* p, size_t i, float v) { p[i] = v; }
__device__ __forceinline__ void st(uint16_t* p, size_t i, float v) { p[i] = f2bf(v); }

// GELU, exact form z Phi(z), and its derivative Phi(z) + z phi(z)
__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float z) {
  return 0.5f * (1.f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

enum Epi {
  kEpiBiasGelu = 0,  // zout = acc + bias, out = gelu(zout)
  kEpiBias = 1,      // zout = acc + bias
  kEpiGeluGrad = 2,  // out = acc * gelu'(zin)
  kEpiStore = 3      // out = acc
};

// C(m, n) = sum_k A(m, k) B(k, n), A(m, k) = a[m sam + k sak], B(k, n) = b[k sbk + n sbn];
// row m of every output/epilogue array starts at m * ldo.
template <typename TA, typename TB, typename TO, int EPI>
__global__ __launch_bounds__(256) void k_mlp_gemm(const TA* __restrict__ a, int64_t sam, int64_t sak,
                                                  const TB* __restrict__ b, int64_t sbk, int64_t sbn, int M, int N,
                                                  int K, const float* __restrict__ bias,
                                                  const float* __restrict__ zin, float* __restrict__ zout,
                                                  TO* __restrict__ out, int64_t ldo) {
  __shared__ float As[32][33];   // [k][m]
  __shared__ float Bs[32][33];   // [k][n]
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int m0 = blockIdx.y * 32, n0 = blockIdx.x * 32;
  float acc00 = 0.f, acc01 = 0.f, acc10 = 0.f, acc11 = 0.f;
  for (int k0 = 0; k0 < K; k0 += 32) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int e = tid + 256 * j;
      // fastest-varying index along the operand's contiguous direction
      int kk, mm;
      if (sak == 1) { kk = e & 31; mm = e >> 5; } else { mm = e & 31; kk = e >> 5; }
      const int gm = m0 + mm, gk = k0 + kk;
      As[kk][mm] = (gm < M && gk < K) ? ld(a, (size_t)(gm * sam + gk * sak)) : 0.f;
      int kb, nn;
      if (sbn == 1) { nn = e & 31; kb = e >> 5; } else { kb = e & 31; nn = e >> 5; }
      const int gn = n0 + nn, gkb = k0 + kb;
      Bs[kb][nn] = (gn < N && gkb < K) ? ld(b, (size_t)(gkb * sbk + gn * sbn)) : 0.f;
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < 32; ++kk) {
      const float a0 = As[kk][2 * ty], a1 = As[kk][2 * ty + 1];
      const float b0 = Bs[kk][2 * tx], b1 = Bs[kk][2 * tx + 1];
      acc00 = fmaf(a0, b0, acc00);
      acc01 = fmaf(a0, b1, acc01);
      acc10 = fmaf(a1, b0, acc10);
      acc11 = fmaf(a1, b1, acc11);
    }
    __syncthreads();
  }
  const float acc[2][2] = {{acc00, acc01}, {acc10, acc11}};
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int m = m0 + 2 * ty + i;
    if (m >= M) continue;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + 2 * tx + j;
      if (n >= N) continue;
      const size_t o = (size_t)m * ldo + n;
      const float c = acc[i][j];
      if (EPI == kEpiBiasGelu) {
        const float z = c + bias[n];
        zout[o] = z;
        st(out, o, gelu(z));
      } else if (EPI == kEpiBias) {
        zout[o] = c + bias[n];
      } else if (EPI == kEpiGeluGrad) {
        st(out, o, c * gelu_d(zin[o]));
      } else {
        st(out, o, c);
      }
    }
  }
}

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// 8 consecutive-k bfloat16 values of an operand, zero outside [0, M) x [0, K)
__device__ __forceinline__ bf16x8 load8_bf16(const uint16_t* __restrict__ p, int64_t s_row, int64_t s_k, int row,
                                             int k0, int nrow, int nk) {
  bf16x8 v;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int k = k0 + e;
    const uint16_t h = (row < nrow && k < nk) ? p[(size_t)((int64_t)row * s_row + (int64_t)k * s_k)] : (uint16_t)0;
    v[e] = __builtin_bit_cast(__bf16, h);
  }
  return v;
}

// C(m, n) = sum_k A(m, k) B(k, n), A and B bfloat16, on the matrix cores.
// Lane l of a wavefront holds rows / columns (l & 31) and k = 8 (l >> 5) + 0..7
// of each 16-deep step; accumulator element r is row 8 (r >> 2) + 4 (l >> 5)
// + (r & 3), column (l & 31).
template <typename TO, int EPI>
__global__ __launch_bounds__(256) void k_mlp_gemm_mfma(const uint16_t* __restrict__ a, int64_t sam, int64_t sak,
                                                       const uint16_t* __restrict__ b, int64_t sbk, int64_t sbn, int M,
                                                       int N, int K, const float* __restrict__ bias,
                                                       const float* __restrict__ zin, float* __restrict__ zout,
                                                       TO* __restrict__ out, int64_t ldo) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m0 = blockIdx.y * 64 + (wave >> 1) * 32, n0 = blockIdx.x * 64 + (wave & 1) * 32;
  if (m0 >= M || n0 >= N) return;   // uniform per wavefront
  const int kb = 8 * (lane >> 5);
  floatx16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.f;
  for (int k0 = 0; k0 < K; k0 += 16) {
    const bf16x8 av = load8_bf16(a, sam, sak, m0 + (lane & 31), k0 + kb, M, K);
    const bf16x8 bv = load8_bf16(b, sbn, sbk, n0 + (lane & 31), k0 + kb, N, K);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
  }
  const int n = n0 + (lane & 31);
  if (n >= N) return;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int m = m0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    if (m >= M) continue;
    const size_t o = (size_t)m * ldo + n;
    const float c = acc[r];
    if (EPI == kEpiBiasGelu) {
      const float z = c + bias[n];
      zout[o] = z;
      st(out, o, gelu(z));
    } else if (EPI == kEpiBias) {
      zout[o] = c + bias[n];
    } else if (EPI == kEpiGeluGrad) {
      st(out, o, c * gelu_d(zin[o]));
    } else {
      st(out, o, c);
    }
  }
}

// out[n] = sum over rows m of g[m][n] (bias gradients); one thread per column
template <typename T>
__global__ void k_mlp_colsum(const T* __restrict__ g, int M, int N, float* __restrict__ out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int m = 0; m < M; ++m) s += ld(g, (size_t)m * N + n);
  out[n] = s;
}

// Mean squared error over rows x outputs; dz = dL/dy = 2 (y - t) / count.
// One workgroup, fixed summation order.
template <typename T>
__global__ __launch_bounds__(256) void k_mlp_mse(const float* __restrict__ y, const float* __restrict__ t, int count,
                                                 T* __restrict__ dz, float* __restrict__ loss) {
  __shared__ float part[256];
  const int tid = threadIdx.x;
  const float scale = 2.f / (float)count;
  float s = 0.f;
  for (int e = tid; e < count; e += 256) {
    const float d = y[e] - t[e];
    st(dz, (size_t)e, scale * d);
    s = fmaf(d, d, s);
  }
  part[tid] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) part[tid] += part[tid + o];
    __syncthreads();
  }
  if (tid == 0 && loss) loss[0] = part[0] / (float)count;
}

// Minibatch rows idx[0..batch) of the data set; an index outside [0, n_data)
// gives a zero row and raises *bad.
__global__ void k_mlp_gather(const float* __restrict__ x, const float* __restrict__ t, int n_data,
                             const int32_t* __restrict__ idx, int batch, int n_in, int n_out, float* __restrict__ xb,
                             float* __restrict__ tb, int* __restrict__ bad) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int w = n_in + n_out;
  if (e >= batch * w) return;
  const int row = e / w, c = e % w;
  const int r = idx[row];
  const bool ok = r >= 0 && r < n_data;
  if (!ok && c == 0) *bad = 1;
  if (c < n_in) xb[(size_t)row * n_in + c] = ok ? x[(size_t)r * n_in + c] : 0.f;
  else tb[(size_t)row * n_out + (c - n_in)] = ok ? t[(size_t)r * n_out + (c - n_in)] : 0.f;
}

// Adam with bias correction (bc1 = 1 - b1^t, bc2 = 1 - b2^t); refreshes the
// bfloat16 copy of the parameters when there is one.
__global__ void k_mlp_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                           float* __restrict__ v, uint16_t* __restrict__ pb, int64_t n, float lr, float b1, float b2,
                           float eps, float bc1, float bc2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  p[i] = pi;
  if (pb) pb[i] = f2bf(pi);
}

__global__ void k_mlp_to_bf16(const float* __restrict__ p, uint16_t* __restrict__ pb, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) pb[i] = f2bf(p[i]);
}

__global__ void k_mlp_fill(uint32_t* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

bool cfg_ok(const pic_mlp_config* c) {
  return c && c->n_in >= 1 && c->n_in <= 64 && c->hidden >= 1 && c->hidden <= 1024 && c->n_hidden_layers >= 1 &&
         c->n_hidden_layers <= 8 && c->n_out >= 1 && c->n_out <= 64 && (c->prec == PIC_MLP_FP32 || c->prec == PIC_MLP_BF16) &&
         c->max_batch >= 1 && c->max_batch <= 65536;
}

int n_layers(const pic_mlp_config* c) { return c->n_hidden_layers + 1; }
int layer_in(const pic_mlp_config* c, int l) { return l == 0 ? c->n_in : c->hidden; }
int layer_out(const pic_mlp_config* c, int l) { return l == n_layers(c) - 1 ? c->n_out : c->hidden; }

int64_t num_params(const pic_mlp_config* c) {
  int64_t n = 0;
  for (int l = 0; l < n_layers(c); ++l) n += (int64_t)layer_out(c, l) * (layer_in(c, l) + 1);
  return n;
}

struct MlpCarver {
  size_t off = 0;
  char* base = nullptr;
  template <class T>
  T* take(size_t count) {
    off = (off + kMlpAlign - 1) / kMlpAlign * kMlpAlign;
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

}  // namespace
}  // namespace pic

using namespace pic;

struct pic_mlp {
  pic_mlp_config cfg;
  hipStream_t stream = nullptr;
  int64_t np = 0, steps = 0;
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  uint16_t* pb = nullptr;   // bfloat16 copy of the parameters (BF16 mode)
  float *xb = nullptr, *tb = nullptr, *loss = nullptr;
  int* bad = nullptr;
  std::vector<float*> z;    // pre-activations of every layer [rows][out_l]
  std::vector<void*> act;   // hidden activations [rows][hidden] (float or bf16)
  void* dz[2] = {nullptr, nullptr};
  std::vector<int64_t> offw, offb;
};

namespace {

size_t carve_mlp(pic_mlp* x, char* base, const pic_mlp_config* c) {
  MlpCarver cv;
  cv.base = base;
  const int64_t np = num_params(c);
  const int L = n_layers(c);
  const size_t B = (size_t)c->max_batch;
  const int wmax = c->hidden > c->n_out ? c->hidden : c->n_out;
  float* p = cv.take<float>(np);
  float* g = cv.take<float>(np);
  float* m = cv.take<float>(np);
  float* v = cv.take<float>(np);
  uint16_t* pb = cv.take<uint16_t>(np);
  float* xb = cv.take<float>(B * c->n_in);
  float* tb = cv.take<float>(B * c->n_out);
  float* loss = cv.take<float>(64);
  int* bad = cv.take<int>(64);
  std::vector<float*> z(L);
  for (int l = 0; l < L; ++l) z[l] = cv.take<float>(B * layer_out(c, l));
  std::vector<void*> act(L - 1);
  for (int l = 0; l < L - 1; ++l) act[l] = cv.take<float>(B * c->hidden);
  void* d0 = cv.take<float>(B * wmax);
  void* d1 = cv.take<float>(B * wmax);
  if (x) {
    x->np = np;
    x->p = p;
    x->g = g;
    x->m = m;
    x->v = v;
    x->pb = pb;
    x->xb = xb;
    x->tb = tb;
    x->loss = loss;
    x->bad = bad;
    x->z = z;
    x->act = act;
    x->dz[0] = d0;
    x->dz[1] = d1;
    x->offw.resize(L);
    x->offb.resize(L);
    int64_t o = 0;
    for (int l = 0; l < L; ++l) {
      x->offw[l] = o;
      o += (int64_t)layer_out(c, l) * layer_in(c, l);
      x->offb[l] = o;
      o += layer_out(c, l);
    }
  }
  return cv.off + kMlpAlign;
}

template <typename TA, typename TB, typename TO, int EPI>
void gemm(hipStream_t s, const TA* a, int64_t sam, int64_t sak, const TB* b, int64_t sbk, int64_t sbn, int M, int N,
          int K, const float* bias, const float* zin, float* zout, TO* out, int64_t ldo) {
  if constexpr (std::is_same<TA, uint16_t>::value && std::is_same<TB, uint16_t>::value) {
    dim3 grid(nblk(N, 64), nblk(M, 64));
    hipLaunchKernelGGL((k_mlp_gemm_mfma<TO, EPI>), grid, dim3(256), 0, s, a, sam, sak, b, sbk, sbn, M, N, K, bias,
                       zin, zout, out, ldo);
  } else {
    dim3 grid(nblk(N, 32), nblk(M, 32));
    hipLaunchKernelGGL((k_mlp_gemm<TA, TB, TO, EPI>), grid, dim3(256), 0, s, a, sam, sak, b, sbk, sbn, M, N, K, bias,
                       zin, zout, out, ldo);
  }
}

// Forward pass over n rows of x (float32); returns the output array z[L-1].
template <typename T>
const float* forward_t(pic_mlp* x, const float* in, int n) {
  const pic_mlp_config& c = x->cfg;
  const int L = n_layers(&c);
  const T* W = std::is_same<T, float>::value ? (const T*)x->p : (const T*)x->pb;
  hipStream_t s = x->stream;
  for (int l = 0; l < L; ++l) {
    const int K = layer_in(&c, l), N = layer_out(&c, l);
    const float* bias = x->p + x->offb[l];
    const T* w = W + x->offw[l];
    // W_l is [N][K]: B(k, n) = W[n][k] -> sbk = 1, sbn = K
    if (l == 0) {
      if (L == 1)
        gemm<float, T, float, kEpiBias>(s, in, K, 1, w, 1, K, n, N, K, bias, nullptr, x->z[l], (float*)nullptr, N);
      else
        gemm<float, T, T, kEpiBiasGelu>(s, in, K, 1, w, 1, K, n, N, K, bias, nullptr, x->z[l], (T*)x->act[l], N);
    } else if (l < L - 1) {
      gemm<T, T, T, kEpiBiasGelu>(s, (const T*)x->act[l - 1], K, 1, w, 1, K, n, N, K, bias, nullptr, x->z[l],
                                  (T*)x->act[l], N);
    } else {
      gemm<T, T, float, kEpiBias>(s, (const T*)x->act[l - 1], K, 1, w, 1, K, n, N, K, bias, nullptr, x->z[l],
                                  (float*)nullptr, N);
    }
  }
  return x->z[L - 1];
}

// Loss and backward pass after forward_t over the same n rows; gradients to gp.
template <typename T>
void backward_t(pic_mlp* x, const float* in, const float* t, int n, float* gp, float* loss) {
  const pic_mlp_config& c = x->cfg;
  const int L = n_layers(&c);
  const T* W = std::is_same<T, float>::value ? (const T*)x->p : (const T*)x->pb;
  hipStream_t s = x->stream;
  int cur = 0;
  hipLaunchKernelGGL(k_mlp_mse<T>, dim3(1), dim3(256), 0, s, x->z[L - 1], t, n * c.n_out, (T*)x->dz[cur], loss);
  for (int l = L - 1; l >= 0; --l) {
    const int K = layer_in(&c, l), N = layer_out(&c, l);
    const T* d = (const T*)x->dz[cur];
    // dW_l[N][K] = sum_rows dz[row][N] a_{l-1}[row][K]
    if (l == 0)
      gemm<T, float, float, kEpiStore>(s, d, 1, N, in, K, 1, N, K, n, nullptr, nullptr, nullptr, gp + x->offw[l], K);
    else
      gemm<T, T, float, kEpiStore>(s, d, 1, N, (const T*)x->act[l - 1], K, 1, N, K, n, nullptr, nullptr, nullptr,
                                   gp + x->offw[l], K);
    hipLaunchKernelGGL(k_mlp_colsum<T>, dim3(nblk(N, 128)), dim3(128), 0, s, d, n, N, gp + x->offb[l]);
    if (l > 0) {
      // dz_{l-1}[row][K] = (sum_n dz[row][n] W_l[n][K]) gelu'(z_{l-1}[row][K])
      gemm<T, T, T, kEpiGeluGrad>(s, d, N, 1, W + x->offw[l], K, 1, n, K, N, nullptr, x->z[l - 1], nullptr,
                                  (T*)x->dz[cur ^ 1], K);
      cur ^= 1;
    }
  }
}

int ck(hipError_t e) { return e == hipSuccess ? PIC_OK : PIC_EHIP; }
int last() { return ck(hipGetLastError()); }

int sync_net(pic_mlp* x) {
  int rc = ck(hipStreamSynchronize(x->stream));
  if (rc) return rc;
  int bad = 0;
  rc = ck(hipMemcpy(&bad, x->bad, sizeof(int), hipMemcpyDeviceToHost));
  if (rc) return rc;
  return bad ? PIC_EINVAL : PIC_OK;
}

}  // namespace

extern "C" {

int pic_mlp_num_params(const pic_mlp_config* cfg, int64_t* n) {
  if (!cfg_ok(cfg) || !n) return PIC_EINVAL;
  *n = num_params(cfg);
  return PIC_OK;
}

int pic_mlp_workspace_bytes(const pic_mlp_config* cfg, size_t* bytes) {
  if (!cfg_ok(cfg) || !bytes) return PIC_EINVAL;
  *bytes = carve_mlp(nullptr, nullptr, cfg);
  return PIC_OK;
}

int pic_mlp_init(const pic_mlp_config* cfg, const float* params, void* workspace, size_t bytes, void* hip_stream,
                 pic_mlp** out) {
  if (!cfg_ok(cfg) || !params || !workspace || !out) return PIC_EINVAL;
  *out = nullptr;
  if (bytes < carve_mlp(nullptr, nullptr, cfg)) return PIC_ENOSPC;
  pic_mlp* x = new pic_mlp();
  x->cfg = *cfg;
  x->stream = (hipStream_t)hip_stream;
  char* base = (char*)(((uintptr_t)workspace + kMlpAlign - 1) / kMlpAlign * kMlpAlign);
  carve_mlp(x, base, cfg);
  hipStream_t s = x->stream;
  int rc = ck(hipMemcpyAsync(x->p, params, (size_t)x->np * sizeof(float), hipMemcpyHostToDevice, s));
  if (!rc) {
    hipLaunchKernelGGL(k_mlp_fill, dim3(nblk(x->np, 256)), dim3(256), 0, s, (uint32_t*)x->m, x->np);
    hipLaunchKernelGGL(k_mlp_fill, dim3(nblk(x->np, 256)), dim3(256), 0, s, (uint32_t*)x->v, x->np);
    hipLaunchKernelGGL(k_mlp_fill, dim3(1), dim3(64), 0, s, (uint32_t*)x->bad, (int64_t)64);
    hipLaunchKernelGGL(k_mlp_to_bf16, dim3(nblk(x->np, 256)), dim3(256), 0, s, x->p, x->pb, x->np);
    rc = last();
  }
  if (!rc) rc = sync_net(x);
  if (rc) {
    delete x;
    return rc;
  }
  *out = x;
  return PIC_OK;
}

int pic_mlp_forward(pic_mlp* x, const float* in, int32_t n, float* y) {
  if (!x || n < 0 || n > x->cfg.max_batch || (n > 0 && (!in || !y))) return PIC_EINVAL;
  if (n == 0) return PIC_OK;
  const float* z = x->cfg.prec == PIC_MLP_BF16 ? forward_t<uint16_t>(x, in, n) : forward_t<float>(x, in, n);
  int rc = ck(hipMemcpyAsync(y, z, (size_t)n * x->cfg.n_out * sizeof(float), hipMemcpyDeviceToDevice, x->stream));
  return rc ? rc : last();
}

int pic_mlp_loss_grad(pic_mlp* x, const float* in, const float* t, int32_t n, float* grad, float* loss) {
  if (!x || !in || !t || !grad || !loss || n < 1 || n > x->cfg.max_batch) return PIC_EINVAL;
  if (x->cfg.prec == PIC_MLP_BF16) {
    forward_t<uint16_t>(x, in, n);
    backward_t<uint16_t>(x, in, t, n, grad, loss);
  } else {
    forward_t<float>(x, in, n);
    backward_t<float>(x, in, t, n, grad, loss);
  }
  return last();
}

int pic_mlp_train(pic_mlp* x, const float* in, const float* t, int32_t n_data, const int32_t* idx, int32_t batch,
                  int32_t steps, const pic_adam* opt, float* loss) {
  if (!x || !in || !t || !idx || !opt || n_data < 1 || batch < 1 || batch > x->cfg.max_batch || steps < 0)
    return PIC_EINVAL;
  if (!(opt->lr > 0.f) || !(opt->beta1 >= 0.f && opt->beta1 < 1.f) || !(opt->beta2 >= 0.f && opt->beta2 < 1.f) ||
      !(opt->eps > 0.f))
    return PIC_EINVAL;
  hipStream_t s = x->stream;
  const pic_mlp_config& c = x->cfg;
  const bool bf = c.prec == PIC_MLP_BF16;
  for (int32_t k = 0; k < steps; ++k) {
    const int w = c.n_in + c.n_out;
    hipLaunchKernelGGL(k_mlp_gather, dim3(nblk((int64_t)batch * w, 256)), dim3(256), 0, s, in, t, n_data,
                       idx + (size_t)k * batch, batch, c.n_in, c.n_out, x->xb, x->tb, x->bad);
    float* lk = loss ? loss + k : x->loss;
    if (bf) {
      forward_t<uint16_t>(x, x->xb, batch);
      backward_t<uint16_t>(x, x->xb, x->tb, batch, x->g, lk);
    } else {
      forward_t<float>(x, x->xb, batch);
      backward_t<float>(x, x->xb, x->tb, batch, x->g, lk);
    }
    x->steps += 1;
    const double st = (double)x->steps;
    const float bc1 = (float)(1.0 - pow((double)opt->beta1, st));
    const float bc2 = (float)(1.0 - pow((double)opt->beta2, st));
    hipLaunchKernelGGL(k_mlp_adam, dim3(nblk(x->np, 256)), dim3(256), 0, s, x->p, x->g, x->m, x->v,
                       bf ? x->pb : nullptr, x->np, opt->lr, opt->beta1, opt->beta2, opt->eps, bc1, bc2);
  }
  return last();
}

int pic_mlp_get_params(pic_mlp* x, float* params) {
  if (!x || !params) return PIC_EINVAL;
  int rc = sync_net(x);
  if (rc) return rc;
  return ck(hipMemcpy(params, x->p, (size_t)x->np * sizeof(float), hipMemcpyDeviceToHost));
}

int pic_mlp_set_params(pic_mlp* x, const float* params) {
  if (!x || !params) return PIC_EINVAL;
  int rc = ck(hipMemcpyAsync(x->p, params, (size_t)x->np * sizeof(float), hipMemcpyHostToDevice, x->stream));
  if (rc) return rc;
  hipLaunchKernelGGL(k_mlp_to_bf16, dim3(nblk(x->np, 256)), dim3(256), 0, x->stream, x->p, x->pb, x->np);
  rc = last();
  return rc ? rc : sync_net(x);
}

int pic_mlp_steps(pic_mlp* x, int64_t* steps) {
  if (!x || !steps) return PIC_EINVAL;
  *steps = x->steps;
  return PIC_OK;
}

int pic_mlp_sync(pic_mlp* x) {
  if (!x) return PIC_EINVAL;
  return sync_net(x);
}

int pic_mlp_free(pic_mlp* x) {
  if (!x) return PIC_EINVAL;
  int rc = ck(hipStreamSynchronize(x->stream));
  delete x;
  return rc;
}

}  // extern "C"
