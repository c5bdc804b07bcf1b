// Beam diagnostics: weighted moments accumulated in FP64 with fixed-shape
// block reductions (deterministic for a given particle order), slice energy
// spread with per-slice FP64 sums.
#include "common.h"
#include "launch.h"

namespace pic {


__device__ __forceinline__ bool diag_alive(const Parts& p, int i, int species, const DiagSel& sel) {
  if (p.sp[i] != species) return false;
  if (sel.kill && p.z[i] < sel.zmin) return false;
  return true;
}

template <int K>
__device__ __forceinline__ void block_reduce_store(double (&v)[K], double* out) {
  __shared__ double sh[256];
  for (int c = 0; c < K; ++c) {
    sh[threadIdx.x] = v[c];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[(size_t)blockIdx.x * K + c] = sh[0];
    __syncthreads();
  }
}

// pass 1: count, sum w, w x, w y, w z, w ux, w uy, w gamma, non-finite count
__global__ __launch_bounds__(256) void k_diag_pass1(Parts p, const DevState* st, DiagSel sel, double* partial) {
  double v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  const int n = st->n_part;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    if (!diag_alive(p, i, sel.species, sel)) continue;
    double x = p.x[i], y = p.y[i], z = p.z[i];
    double ux = p.ux[i], uy = p.uy[i], uz = p.uz[i];
    double w = (double)p.w[i] * sel.inv_q;
    bool fin = isfinite(x) && isfinite(y) && isfinite(z) && isfinite(ux) && isfinite(uy) && isfinite(uz);
    if (!fin) {
      v[8] += 1.0;
      continue;
    }
    double g = sqrt(1.0 + ux * ux + uy * uy + uz * uz);
    v[0] += 1.0;
    v[1] += w;
    v[2] += w * x;
    v[3] += w * y;
    v[4] += w * z;
    v[5] += w * ux;
    v[6] += w * uy;
    v[7] += w * g;
  }
  block_reduce_store<9>(v, partial);
}

// pass 2: central moments w dx^2, w dux^2, w dx dux, w dy^2, w duy^2, w dy duy, w dg^2, w dz^2
__global__ __launch_bounds__(256) void k_diag_pass2(Parts p, const DevState* st, DiagSel sel, DiagMeans mu,
                                                    double* partial) {
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int n = st->n_part;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    if (!diag_alive(p, i, sel.species, sel)) continue;
    double ux = p.ux[i], uy = p.uy[i], uz = p.uz[i];
    double w = (double)p.w[i] * sel.inv_q;
    double g = sqrt(1.0 + ux * ux + uy * uy + uz * uz);
    if (!isfinite(g) || !isfinite(p.x[i]) || !isfinite(p.y[i]) || !isfinite(p.z[i])) continue;
    double dx = p.x[i] - mu.x, dy = p.y[i] - mu.y, dz = p.z[i] - mu.z;
    double dux = ux - mu.ux, duy = uy - mu.uy, dg = g - mu.g;
    v[0] += w * dx * dx;
    v[1] += w * dux * dux;
    v[2] += w * dx * dux;
    v[3] += w * dy * dy;
    v[4] += w * duy * duy;
    v[5] += w * dy * duy;
    v[6] += w * dg * dg;
    v[7] += w * dz * dz;
  }
  block_reduce_store<8>(v, partial);
}

// column sums of partial[nb][K] -> out[K]
__global__ __launch_bounds__(256) void k_diag_reduce(const double* partial, int nb, int K, double* out) {
  __shared__ double sh[256];
  for (int c = 0; c < K; ++c) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) s += partial[(size_t)b * K + c];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = sh[0];
    __syncthreads();
  }
}

// slices: index floor((z - <z>)/L) + h for |z - <z>| <= n_sigma sigma_z
__device__ __forceinline__ int slice_of(double z, const DiagMeans& mu) {
  double xi = z - mu.z;
  if (!(fabs(xi) <= mu.zcut)) return -1;
  long long s = (long long)floor(xi / mu.slice_len) + mu.half;
  if (s < 0 || s >= 2 * mu.half) return -1;
  return (int)s;
}

// slice sums: [s][0] count, [s][1] sum w, [s][2] sum w gamma
__global__ __launch_bounds__(256) void k_diag_slice1(Parts p, const DevState* st, DiagSel sel, DiagMeans mu,
                                                     double* acc) {
  const int n = st->n_part;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    if (!diag_alive(p, i, sel.species, sel)) continue;
    int s = slice_of(p.z[i], mu);
    if (s < 0) continue;
    double ux = p.ux[i], uy = p.uy[i], uz = p.uz[i];
    double g = sqrt(1.0 + ux * ux + uy * uy + uz * uz);
    if (!isfinite(g)) continue;
    double w = (double)p.w[i] * sel.inv_q;
    atomicAdd(&acc[3 * s + 0], 1.0);
    atomicAdd(&acc[3 * s + 1], w);
    atomicAdd(&acc[3 * s + 2], w * g);
  }
}

// per-slice sum w (gamma - <gamma>_s)^2 -> var[s]
__global__ __launch_bounds__(256) void k_diag_slice2(Parts p, const DevState* st, DiagSel sel, DiagMeans mu,
                                                     const double* acc, double* var) {
  const int n = st->n_part;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    if (!diag_alive(p, i, sel.species, sel)) continue;
    int s = slice_of(p.z[i], mu);
    if (s < 0) continue;
    double ux = p.ux[i], uy = p.uy[i], uz = p.uz[i];
    double g = sqrt(1.0 + ux * ux + uy * uy + uz * uz);
    if (!isfinite(g)) continue;
    double w = (double)p.w[i] * sel.inv_q;
    double gm = acc[3 * s + 2] / acc[3 * s + 1];
    atomicAdd(&var[s], w * (g - gm) * (g - gm));
  }
}

// compacted copy of one species (for pic_get_particles), structure of arrays
__global__ __launch_bounds__(256) void k_collect(Parts p, const DevState* st, DiagSel sel, int64_t cap, Parts out,
                                                 int* counter) {
  const int n = st->n_part;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (!diag_alive(p, i, sel.species, sel)) return;
  int d = atomicAdd(counter, 1);
  if (d >= cap) return;
  out.x[d] = p.x[i];
  out.y[d] = p.y[i];
  out.z[d] = p.z[i];
  out.ux[d] = p.ux[i];
  out.uy[d] = p.uy[i];
  out.uz[d] = p.uz[i];
  out.w[d] = (float)((double)p.w[i] * sel.inv_q);
}

__global__ __launch_bounds__(256) void k_count_alive(Parts p, const DevState* st, DiagSel sel, int* counter) {
  __shared__ int wsum[4];
  const int n = st->n_part;
  int c = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    c += !(sel.kill && p.z[i] < sel.zmin);
  for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(counter, wsum[0] + wsum[1] + wsum[2] + wsum[3]);
}

void launch_diag_pass1(const Parts& p, const DevState* st, const DiagSel& sel, double* partial, double* out,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_diag_pass1, dim3(kDiagBlocks), dim3(256), 0, s, p, st, sel, partial);
  hipLaunchKernelGGL(k_diag_reduce, dim3(1), dim3(256), 0, s, partial, kDiagBlocks, 9, out);
}
void launch_diag_pass2(const Parts& p, const DevState* st, const DiagSel& sel, const DiagMeans& mu, double* partial,
                       double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_pass2, dim3(kDiagBlocks), dim3(256), 0, s, p, st, sel, mu, partial);
  hipLaunchKernelGGL(k_diag_reduce, dim3(1), dim3(256), 0, s, partial, kDiagBlocks, 8, out);
}
void launch_diag_slices(const Parts& p, const DevState* st, const DiagSel& sel, const DiagMeans& mu, double* acc,
                        double* var, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_slice1, dim3(kDiagBlocks), dim3(256), 0, s, p, st, sel, mu, acc);
  hipLaunchKernelGGL(k_diag_slice2, dim3(kDiagBlocks), dim3(256), 0, s, p, st, sel, mu, acc, var);
}
int diag_partial_doubles() { return kDiagPartialDoubles; }
void launch_collect(const Parts& p, const DevState* st, const DiagSel& sel, int64_t cap, const Parts& out,
                    int* counter, int nmax, hipStream_t s) {
  hipLaunchKernelGGL(k_collect, dim3((nmax + 255) / 256), dim3(256), 0, s, p, st, sel, cap, out, counter);
}
void launch_count_alive(const Parts& p, const DevState* st, const DiagSel& sel, int* counter, int nmax,
                        hipStream_t s) {
  int nb = (nmax + 255) / 256;
  if (nb > 1024) nb = 1024;
  hipLaunchKernelGGL(k_count_alive, dim3(nb), dim3(256), 0, s, p, st, sel, counter);
}

}  // namespace pic
