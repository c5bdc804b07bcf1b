// Batched complex FFT along z (the contiguous axis), Stockham autosort in LDS.
//
// One row of nz complex values lives in one LDS buffer, overwritten in place
// by every pass; the first radix pass reads straight from global memory and
// the last one writes straight to global memory, both coalesced (consecutive
// butterflies touch consecutive addresses).  Radix-8 passes, plus one radix-2
// or radix-4 pass for log2(nz) mod 3 (2048 points: four passes).  Twiddles
// come from an FP64-built float32 table of exp(-2 pi i t / nz).
//
// The inverse transform can fuse the moving-window shift: output sample j is
// written to column j - 1, column nz - 1 is zeroed and sample 0 (the column
// that leaves the window) is saved to `tail`.
#include "common.h"
#include "launch.h"

namespace pic {

template <int R, bool INV>
__device__ __forceinline__ void dft_small(float2* v);

// radix 8: two radix-4 DFTs of the even and odd samples, odd ones rotated by
// W8^k = exp(-/+ i pi k / 4), then one radix-2 stage
template <bool INV>
__device__ __forceinline__ void dft8(float2* v) {
  float2 e[4] = {v[0], v[2], v[4], v[6]};
  float2 o[4] = {v[1], v[3], v[5], v[7]};
  dft_small<4, INV>(e);
  dft_small<4, INV>(o);
  const float h = 0.70710678118654752f;
  const float sg = INV ? 1.f : -1.f;
  o[1] = cmul(o[1], make_float2(h, sg * h));
  o[2] = cmuli(cscale(o[2], sg));
  o[3] = cmul(o[3], make_float2(-h, sg * h));
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = cadd(e[k], o[k]);
    v[k + 4] = csub(e[k], o[k]);
  }
}

template <int R, bool INV>
__device__ __forceinline__ void dft_small(float2* v) {
  if constexpr (R == 8) {
    dft8<INV>(v);
  } else if constexpr (R == 2) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else {
    // radix 4: X1 = (v0 - v2) -/+ i (v1 - v3) for the forward/inverse sign
    float2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    float2 a2 = cadd(v[1], v[3]), d = csub(v[1], v[3]);
    float2 a3 = INV ? cmuli(d) : cmuli(cscale(d, -1.f));
    v[0] = cadd(a0, a2);
    v[1] = cadd(a1, a3);
    v[2] = csub(a0, a2);
    v[3] = csub(a1, a3);
  }
}

struct FftOut {
  bool shift;     // inverse + moving window
  float scale;
  float2* tail;   // per-row saved column 0 (when shift)
  int64_t row;
};

// Twiddles of one radix-8 pass for this thread's butterflies:
// w[jj][r-1] = exp(-2 pi i r k / (8 Ns)), k = j mod Ns (conjugated by the caller
// for the inverse); from the FP64-built table, or computed in FP64 without one.
template <int JJ>
__device__ __forceinline__ void load_tw8(const float2* __restrict__ tw, int N, int Ns, int t, int tpr,
                                         float2 (&w)[JJ][7]) {
  const int NR = N / 8;
  const int step = N / (Ns * 8);
#pragma unroll
  for (int jj = 0; jj < JJ; ++jj) {
    const int j = t + jj * tpr;
    const int k = j & (Ns - 1);
#pragma unroll
    for (int r = 1; r < 8; ++r) {
      float2 v = make_float2(1.f, 0.f);
      if (j < NR) {
        if (tw) {
          v = tw[r * k * step];
        } else {
          double sn, cs;
          sincospi(-2.0 * (double)(r * k * step) / (double)N, &sn, &cs);
          v = make_float2((float)cs, (float)sn);
        }
      }
      w[jj][r - 1] = v;
    }
  }
}

// Butterflies of one radix-R Stockham pass (Ns: size of the sub-transforms
// already done) from src into registers: v[jj R + r] of butterfly
// j = t + jj tpr.  Twiddles apply for Ns > 1 (radix-8 passes only).
template <int R, bool INV, int VPT, int JJ8>
__device__ __forceinline__ void pass_compute(const float2* src, int N, int Ns, int t, int tpr,
                                             const float2 (&w)[JJ8][7], float2 (&v)[VPT],
                                             const float2* minus = nullptr) {
  const int NR = N / R;
  constexpr int JJ = VPT / R;
#pragma unroll
  for (int jj = 0; jj < JJ; ++jj) {
    const int j = t + jj * tpr;
    if (j < NR) {
      float2* u = v + jj * R;
#pragma unroll
      for (int r = 0; r < R; ++r) u[r] = src[j + r * NR];
      if (minus) {
#pragma unroll
        for (int r = 0; r < R; ++r) u[r] = csub(u[r], minus[j + r * NR]);
      }
      if constexpr (R == 8) {
        if (Ns > 1) {
#pragma unroll
          for (int r = 1; r < 8; ++r) {
            float2 ww = w[jj < JJ8 ? jj : 0][r - 1];
            if (INV) ww.y = -ww.y;
            u[r] = cmul(u[r], ww);
          }
        }
      }
      dft_small<R, INV>(u);
    }
  }
}

// Results of the pass to their Stockham places: into the row buffer, or, for
// the last pass, scaled into global memory (with the fused window shift).
template <int R, bool LAST, int VPT>
__device__ __forceinline__ void pass_store(float2* dst, int N, int Ns, int t, int tpr, const FftOut& o,
                                           const float2 (&v)[VPT]) {
  const int NR = N / R;
  constexpr int JJ = VPT / R;
#pragma unroll
  for (int jj = 0; jj < JJ; ++jj) {
    const int j = t + jj * tpr;
    if (j < NR) {
      const int k = j & (Ns - 1);
      const int idxD = (j / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int d = idxD + r * Ns;
        const float2 x = v[jj * R + r];
        if (LAST) {
          float2 val = cscale(x, o.scale);
          if (o.shift) {
            if (d == 0) {
              if (o.tail) o.tail[o.row] = val;
              dst[N - 1] = make_float2(0.f, 0.f);
            } else {
              dst[d - 1] = val;
            }
          } else {
            dst[d] = val;
          }
        } else {
          dst[d] = x;
        }
      }
    }
  }
}

template <bool INV, int R0, int VPT>
__device__ __forceinline__ void first_pass(const float2* gin, const float2* gminus, float2* buf, float2* gout, int N,
                                           int t, int tpr, bool active, bool last, const FftOut& o,
                                           const float2 (&w)[VPT / 8][7], float2 (&v)[VPT]) {
  if (active) {
    pass_compute<R0, INV, VPT, VPT / 8>(gin, N, 1, t, tpr, w, v, gminus);
    if (last) pass_store<R0, true, VPT>(gout, N, 1, t, tpr, o, v);
    else pass_store<R0, false, VPT>(buf, N, 1, t, tpr, o, v);
  }
}

// One row of N points per tpr threads, one LDS buffer per row: every pass
// after the first reads its inputs into registers, waits for the whole
// workgroup, then writes its outputs in place (16 KB of LDS per 2048-point
// row).  The twiddles of pass p + 1 are requested before pass p starts, so
// their latency hides behind that pass.  VPT: complex values per thread and
// pass (8 up to 2048 points, 16 at 4096).  Rows [diff_lo, diff_hi) transform
// the difference in[row + diff_off] - in[row] instead of in[row].
template <bool INV, int VPT>
__global__ __launch_bounds__(256) void k_fft(const float2* __restrict__ in, float2* __restrict__ out,
                                             const float2* __restrict__ tw, int N, int logN, int rows_per_wg,
                                             int64_t rows, int shift, float2* tail, int64_t diff_lo,
                                             int64_t diff_hi, int64_t diff_off) {
  constexpr int JJ8 = VPT / 8;
  extern __shared__ float2 lds[];
  const int tpr = blockDim.x / rows_per_wg;
  const int rloc = threadIdx.x / tpr;
  const int t = threadIdx.x % tpr;
  const int64_t row = (int64_t)blockIdx.x * rows_per_wg + rloc;
  const bool active = row < rows;
  float2* buf = lds + (size_t)rloc * N;
  const float2* gin = in + row * N;
  const float2* gminus = nullptr;
  if (row >= diff_lo && row < diff_hi) {
    gminus = gin;
    gin = in + (row + diff_off) * N;
  }
  float2* gout = out + row * N;
  FftOut o;
  o.shift = INV && shift;
  o.scale = INV ? 1.f / (float)N : 1.f;
  o.tail = tail;
  o.row = row;
  // pass plan: one radix-2 or radix-4 pass for log2(N) mod 3, then radix-8 passes
  const int rem = logN % 3;
  const int npass = logN / 3 + (rem ? 1 : 0);
  const int R0 = rem == 1 ? 2 : (rem == 2 ? 4 : 8);
  float2 w[JJ8][7];
  float2 v[VPT];
  if (npass > 1 && active) load_tw8<JJ8>(tw, N, R0, t, tpr, w);
  {
    const bool last = npass == 1;
    if (R0 == 2) first_pass<INV, 2, VPT>(gin, gminus, buf, gout, N, t, tpr, active, last, o, w, v);
    else if (R0 == 4) first_pass<INV, 4, VPT>(gin, gminus, buf, gout, N, t, tpr, active, last, o, w, v);
    else first_pass<INV, 8, VPT>(gin, gminus, buf, gout, N, t, tpr, active, last, o, w, v);
  }
  __syncthreads();
  int Ns = R0;
  for (int p = 1; p < npass; ++p) {
    const bool last = p == npass - 1;
    if (active) pass_compute<8, INV, VPT, JJ8>(buf, N, Ns, t, tpr, w, v);
    if (!last && active) load_tw8<JJ8>(tw, N, Ns * 8, t, tpr, w);
    if (!last) __syncthreads();   // in place: every read of this pass before its writes
    if (active) {
      if (last) pass_store<8, true, VPT>(gout, N, Ns, t, tpr, o, v);
      else pass_store<8, false, VPT>(buf, N, Ns, t, tpr, o, v);
    }
    if (!last) __syncthreads();
    Ns *= 8;
  }
}

static int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

void fft_config(int nz, int& rows_per_wg, size_t& lds) {
  int tpr = nz / 4 < 256 ? nz / 4 : 256;
  if (tpr < 1) tpr = 1;
  rows_per_wg = 256 / tpr;
  lds = (size_t)rows_per_wg * nz * sizeof(float2);
}

template <bool INV>
static void launch_fft_dir(const float2* in, float2* out, const float2* tw, int nz, int64_t rows, bool shift,
                           float2* tail, int64_t diff_lo, int64_t diff_hi, int64_t diff_off, hipStream_t s) {
  int rpw;
  size_t lds;
  fft_config(nz, rpw, lds);
  const int64_t nb = (rows + rpw - 1) / rpw;
  const int logN = ilog2(nz);
  if (nz > 2048)
    hipLaunchKernelGGL((k_fft<INV, 16>), dim3((unsigned)nb), dim3(256), lds, s, in, out, tw, nz, logN, rpw, rows,
                       shift ? 1 : 0, tail, diff_lo, diff_hi, diff_off);
  else
    hipLaunchKernelGGL((k_fft<INV, 8>), dim3((unsigned)nb), dim3(256), lds, s, in, out, tw, nz, logN, rpw, rows,
                       shift ? 1 : 0, tail, diff_lo, diff_hi, diff_off);
}

void launch_fft(const float2* in, float2* out, const float2* tw, int nz, int64_t rows, bool inverse, bool shift,
                float2* tail, hipStream_t s, int64_t diff_lo, int64_t diff_hi, int64_t diff_off) {
  if (inverse) launch_fft_dir<true>(in, out, tw, nz, rows, shift, tail, 0, 0, 0, s);
  else launch_fft_dir<false>(in, out, tw, nz, rows, false, tail, diff_lo, diff_hi, diff_off, s);
}

}  // namespace pic
