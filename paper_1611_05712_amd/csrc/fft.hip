// Batched complex FFT along z (the contiguous axis), Stockham autosort in LDS.
//
// One row of nz complex values lives in LDS (ping-pong buffers); the first
// radix pass reads straight from global memory and the last one writes
// straight to global memory, both coalesced (consecutive butterflies touch
// consecutive addresses).  Radix-8 passes, plus one radix-2 or radix-4 pass
// for log2(nz) mod 3 (2048 points: four passes).  Twiddles come from an FP64-built float32 table of
// exp(-2 pi i t / nz).
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

template <int R, bool INV, bool LAST>
__device__ __forceinline__ void fft_pass(const float2* src, float2* dst, const float2* __restrict__ tw, int N, int Ns,
                                         int t, int tpr, const FftOut& o) {
  const int NR = N / R;
  for (int j = t; j < NR; j += tpr) {
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = src[j + r * NR];
    const int k = j & (Ns - 1);
    if (Ns > 1) {
      const int step = N / (Ns * R);
#pragma unroll
      for (int r = 1; r < R; ++r) {
        float2 w;
        if (tw) {
          w = tw[r * k * step];
        } else {
          double sn, cs;
          sincospi(-2.0 * (double)(r * k * step) / (double)N, &sn, &cs);
          w = make_float2((float)cs, (float)sn);
        }
        if (INV) w.y = -w.y;
        v[r] = cmul(v[r], w);
      }
    }
    dft_small<R, INV>(v);
    const int idxD = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      int d = idxD + r * Ns;
      if (LAST) {
        float2 val = cscale(v[r], o.scale);
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
        dst[d] = v[r];
      }
    }
  }
}

template <bool INV>
__global__ __launch_bounds__(256) void k_fft(const float2* __restrict__ in, float2* __restrict__ out,
                                             const float2* __restrict__ tw, int N, int logN, int rows_per_wg,
                                             int64_t rows, int shift, float2* tail) {
  extern __shared__ float2 lds[];
  const int tpr = blockDim.x / rows_per_wg;
  const int rloc = threadIdx.x / tpr;
  const int t = threadIdx.x % tpr;
  const int64_t row = (int64_t)blockIdx.x * rows_per_wg + rloc;
  const bool active = row < rows;
  float2* b0 = lds + (size_t)rloc * 2 * N;
  float2* b1 = b0 + N;
  const float2* gin = in + row * N;
  float2* gout = out + row * N;
  FftOut o;
  o.shift = INV && shift;
  o.scale = INV ? 1.f / (float)N : 1.f;
  o.tail = tail;
  o.row = row;
  // pass plan: one radix-2 or radix-4 pass for log2(N) mod 3, then radix-8 passes
  const int rem = logN % 3;
  const int n8 = logN / 3;
  const int npass = n8 + (rem ? 1 : 0);
  int Ns = 1;
  int pass = 0;
  const float2* src = gin;
  float2* cur = b0;
  float2* other = b1;
  if (rem) {
    const bool last = (pass == npass - 1);
    if (active) {
      if (rem == 1) {
        if (last) fft_pass<2, INV, true>(src, gout, tw, N, Ns, t, tpr, o);
        else fft_pass<2, INV, false>(src, cur, tw, N, Ns, t, tpr, o);
      } else {
        if (last) fft_pass<4, INV, true>(src, gout, tw, N, Ns, t, tpr, o);
        else fft_pass<4, INV, false>(src, cur, tw, N, Ns, t, tpr, o);
      }
    }
    __syncthreads();
    Ns *= (rem == 1) ? 2 : 4;
    ++pass;
    src = cur;
    float2* tmp = cur;
    cur = other;
    other = tmp;
  }
  for (int q = 0; q < n8; ++q) {
    const bool last = (pass == npass - 1);
    if (active) {
      if (last) fft_pass<8, INV, true>(src, gout, tw, N, Ns, t, tpr, o);
      else fft_pass<8, INV, false>(src, cur, tw, N, Ns, t, tpr, o);
    }
    __syncthreads();
    Ns *= 8;
    ++pass;
    src = cur;
    float2* tmp = cur;
    cur = other;
    other = tmp;
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
  lds = (size_t)rows_per_wg * 2 * nz * sizeof(float2);
}

void launch_fft(const float2* in, float2* out, const float2* tw, int nz, int64_t rows, bool inverse, bool shift,
                float2* tail, hipStream_t s) {
  int rpw;
  size_t lds;
  fft_config(nz, rpw, lds);
  int64_t nb = (rows + rpw - 1) / rpw;
  int logN = ilog2(nz);
  if (inverse)
    hipLaunchKernelGGL(k_fft<true>, dim3((unsigned)nb), dim3(256), lds, s, in, out, tw, nz, logN, rpw, rows,
                       shift ? 1 : 0, tail);
  else
    hipLaunchKernelGGL(k_fft<false>, dim3((unsigned)nb), dim3(256), lds, s, in, out, tw, nz, logN, rpw, rows, 0,
                       tail);
}

}  // namespace pic
