// Shared device-side definitions of the gfx950 PIC library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

constexpr int kMaxModes = 4;
constexpr int kMaxSpecies = 16;
constexpr int kNumComp = 11;           // E+,E-,Ez,B+,B-,Bz,J+,J-,Jz,rho^n,rho^{n+1}
constexpr int kCompJ = 6;              // first source component
constexpr int kNumSrc = 5;             // J+,J-,Jz,rho^n,rho^{n+1}
constexpr int kCompRho0 = 9;           // rho^n (spectral slot: rho^{n+1} - rho^n)
constexpr uint32_t kInvalidKey = 0xFFFFFFFFu;
// The forward discrete Hankel transform is the pseudo-inverse of the Bessel
// synthesis matrix: singular values below this fraction of the largest are
// dropped (near-null directions are projected out, not amplified).
constexpr double kPinvRcond = 1e-4;

// Device-resident mutable state: kernels read and update it so that a step
// can be captured once and replayed without host-side argument changes.
struct DevState {
  double zmin;          // window position (node j = 0)
  int64_t n_shift;      // completed window moves
  int32_t n_part;       // particles in the current buffer, [0, n_part)
  int32_t n_live;       // particles kept by the last sort (sorted prefix)
  int32_t pending_shift;// spectral E, B still need the last window move applied
  int32_t overflow;     // capacity exceeded at an injection
  int32_t nonfinite;    // a split-precision Hankel product produced inf/NaN
  int32_t pad;
};

// Grid constants passed by value to kernels.
struct Grid {
  int nz, nr, nmodes;
  int ncol;             // key columns per z row: nr + 1 (lower node i0 = -1 .. nr - 1)
  int ncells;           // nz * ncol; key value ncells marks a removed particle
  double dz, dr, dt;
  double inv_dz, inv_dr;
  double zmin0;
  int moving_window;
  int shape;            // particle shape order: 1 linear, 3 cubic B-spline
};

// Particle storage (structure of arrays); w holds the signed charge weight q*w.
// Positions and the longitudinal momentum are FP64: a beam at gamma ~ 1e3
// moves u_z by far less than one FP32 ulp per step, and its slice energy
// spread is a few ulp of gamma in FP32.
struct Parts {
  double *x, *y, *z, *uz;
  float *ux, *uy, *w;
  uint8_t* sp;
};

struct SpeciesConst {
  float qm[kMaxSpecies];   // q / m
};

// Global-address-space pointers.  A pointer read from a device-side table is
// generic (flat): accesses through it are flat instructions, which count
// against the LDS wait counter too, so every LDS wait also waits for them.
// Converted to these types, the accesses are global ones.
typedef __attribute__((address_space(1))) const float* gcfloat_p;
typedef __attribute__((address_space(1))) float* gfloat_p;

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// i * a
__device__ __forceinline__ float2 cmuli(float2 a) { return make_float2(-a.y, a.x); }

// Linear-shape bookkeeping of one position: lower z node j0 (wrapped into
// [0, nz)), fraction fz; lower radial node i0 (may be -1: the ghost node across
// the axis), fraction fr; exp(i theta).
struct ShapePos {
  int j0, i0;
  float fz, fr;
  float2 eith;
};

// 1/sqrt(a) for a > 0 to FP64 accuracy: float32 estimate + two Newton steps
__device__ __forceinline__ double rsqrt_f64(double a) {
  double y = (double)rsqrtf((float)a);
  y = y * (1.5 - 0.5 * a * y * y);
  y = y * (1.5 - 0.5 * a * y * y);
  return y;
}

__device__ __forceinline__ ShapePos shape_at(double x, double y, double z, double zmin, const Grid& g) {
  ShapePos s;
  double sz = (z - zmin) * g.inv_dz;
  sz = fmin(fmax(sz, -1e9), 1e9);
  double fj = floor(sz);
  s.fz = (float)(sz - fj);
  s.j0 = (int)((long long)fj & (long long)(g.nz - 1));   // nz is a power of two: periodic wrap
  double r2 = x * x + y * y;
  double ir = r2 > 1e-30 ? rsqrt_f64(r2) : 0.0;
  double r = r2 * ir;
  double sr = r * g.inv_dr - 0.5;
  sr = fmin(sr, (double)(1 << 30));
  double fi = floor(sr);
  s.fr = (float)(sr - fi);
  s.i0 = (int)fi;
  s.eith = r2 > 1e-30 ? make_float2((float)(x * ir), (float)(y * ir)) : make_float2(1.f, 0.f);
  return s;
}

// Sort key of a position: (z row, lower radial node + 1), radial index clamped
// into [0, nr] (particles beyond the last node touch nothing).
__device__ __forceinline__ uint32_t cell_key(const ShapePos& s, const Grid& g) {
  int ic = s.i0 + 1;
  if (ic > g.nr) ic = g.nr;
  if (ic < 0) ic = 0;
  return (uint32_t)(s.j0 * g.ncol + ic);
}

}  // namespace pic

// Host-side launchers implemented in the kernel translation units.
namespace pic {
struct Ctx;
}
