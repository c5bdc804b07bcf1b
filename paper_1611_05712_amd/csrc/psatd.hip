// Spectral step: pending window shift, current correction and the order-p
// PSATD update, fused per spectral cell (k_perp, k_z) and looped over modes.
//
// In plasma units (c = 1) the paper's Eqs. (1a)-(1b) with the quasi-cylindrical
// operators of Eqs. (2a)-(2b) read, with k = sqrt(k_perp^2 + [k_z]^2),
// C = cos(k dt), S = sin(k dt):
//   E' = C E + (S/k) curl B - (S/k) J
//        + grad[((S/(k dt) - 1) rho^{n+1} + (C - S/(k dt)) rho^n) / k^2]
//   B' = C B - (S/k) curl E + ((1 - C)/k^2) curl J
//   grad s    = (-k_perp s/2, +k_perp s/2, i [k_z] s)
//   curl V    = ([k_z] V+ - i k_perp Vz/2, -[k_z] V- - i k_perp Vz/2, i k_perp (V+ + V-))
//   div V     = k_perp (V+ - V-) + i [k_z] Vz
// Current correction: J += grad F, F = (div J + (rho^{n+1} - rho^n)/dt) / k^2.
// The coefficients are evaluated in FP64 (C, S, and the cancellation-prone
// 1 - C and C - S/(k dt) near k -> 0) and rounded once to float32.
//
// The rho^n slot holds d = rho^{n+1} - rho^n, transformed as such: F takes d
// directly, and the charge term is written
//   (S/(k dt) - 1) rho^{n+1} + (C - S/(k dt)) rho^n = (C - 1) rho^{n+1} - (C - S/(k dt)) d,
// so no difference of two separately rounded transforms enters the update.
//
// A moving window shifts the real-space fields one cell toward the tail and
// zeroes the head column.  On the spectral state that is
//   F <- exp(+i k_z dz) (F - F_nu c)
// with c the real-space column that left the window; it is applied here,
// before the update, so the spectral E, B never round-trip through real space.
#include "common.h"
#include "launch.h"

namespace pic {

struct Coef {
  float C, Sk, omc, r0, ik2;
};

__device__ __forceinline__ Coef make_coef(double kp, double kz, double dt) {
  double k2 = kp * kp + kz * kz;
  double k = sqrt(k2);
  double x = k * dt;
  double s, c;
  sincos(x, &s, &c);
  double sx = s / x;
  Coef o;
  o.C = (float)c;
  o.Sk = (float)(s / k);
  o.omc = (float)((1.0 - c) / k2);
  o.r0 = (float)((c - sx) / k2);
  o.ik2 = (float)(1.0 / k2);
  return o;
}

// One spectral cell (k_perp index, k_z index) per thread, every mode.  All
// loads of all modes are issued before any store (the stores could alias
// them as far as the compiler knows), and the FP64 coefficients are computed
// while they are in flight.
template <int M>
__global__ __launch_bounds__(256) void k_psatd(float2* __restrict__ spec, const double* __restrict__ kperp,
                                               const double* __restrict__ kzm, const float2* __restrict__ tw,
                                               const float2* __restrict__ tailhat, int nz, int nr, double dt,
                                               int apply_shift, int correct, const double* __restrict__ kz_grid,
                                               double dz, double dr, int filter) {
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= (int64_t)nr * nz) return;
  const int ik = (int)(cell / nz);
  const int iz = (int)(cell % nz);
  const size_t plane = (size_t)nr * nz;
  float2 E[M][3], B[M][3], J[M][3], r0[M], r1[M];
#pragma unroll
  for (int m = 0; m < M; ++m) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      E[m][c] = spec[((size_t)c * M + m) * plane + cell];
      B[m][c] = spec[((size_t)(3 + c) * M + m) * plane + cell];
      J[m][c] = spec[((size_t)(6 + c) * M + m) * plane + cell];
    }
    r0[m] = spec[((size_t)kCompRho0 * M + m) * plane + cell];      // rho^{n+1} - rho^n
    r1[m] = spec[((size_t)(kCompRho0 + 1) * M + m) * plane + cell];
  }
  float2 th[M][6];
  if (apply_shift) {
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
      for (int c = 0; c < 6; ++c) th[m][c] = tailhat[((size_t)c * M + m) * nr + ik];
  }
  const double kzd = kzm[iz];
  const float kz = (float)kzd;
  float2 ph = make_float2(1.f, 0.f);
  if (apply_shift) ph = cconj(tw[iz]);   // exp(+2 pi i iz / nz)
  const float idt = (float)(1.0 / dt);
  double kp_prev = -1.0;
  Coef co{};
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const double kpd = kperp[m * nr + ik];
    if (kpd != kp_prev) {
      co = make_coef(kpd, kzd, dt);
      kp_prev = kpd;
    }
    const float kp = (float)kpd;
    float2* f[kNumComp];
#pragma unroll
    for (int c = 0; c < kNumComp; ++c) f[c] = spec + ((size_t)c * M + m) * plane + cell;
    float2 Em[3], Bm[3], Jm[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Em[c] = E[m][c];
      Bm[c] = B[m][c];
      Jm[c] = J[m][c];
    }
    float2 dq = r0[m], q1 = r1[m];
    if (filter) {
      // `filter` binomial (1/4, 1/2, 1/4) passes along z and along r, in spectral form
      const double cz = cos(0.5 * kz_grid[iz] * dz), cr = cos(0.5 * kpd * dr);
      const double f1 = cz * cz * cr * cr;
      double fp = f1;
      for (int q = 1; q < filter; ++q) fp *= f1;
      const float fs = (float)fp;
#pragma unroll
      for (int c = 0; c < 3; ++c) Jm[c] = cscale(Jm[c], fs);
      dq = cscale(dq, fs);
      q1 = cscale(q1, fs);
    }
    if (apply_shift) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        Em[c] = cmul(ph, csub(Em[c], th[m][c]));
        Bm[c] = cmul(ph, csub(Bm[c], th[m][3 + c]));
      }
    }
    if (correct) {
      float2 dvj = cadd(cscale(csub(Jm[0], Jm[1]), kp), cmuli(cscale(Jm[2], kz)));
      float2 F = cscale(cadd(dvj, cscale(dq, idt)), co.ik2);
      Jm[0] = cadd(Jm[0], cscale(F, -0.5f * kp));
      Jm[1] = cadd(Jm[1], cscale(F, 0.5f * kp));
      Jm[2] = cadd(Jm[2], cmuli(cscale(F, kz)));
#pragma unroll
      for (int c = 0; c < 3; ++c) *f[6 + c] = Jm[c];
    }
    // curls
    float2 cB[3], cE[3], cJ[3];
    {
      const float hk = 0.5f * kp;
      cB[0] = csub(cscale(Bm[0], kz), cmuli(cscale(Bm[2], hk)));
      cB[1] = csub(cscale(Bm[1], -kz), cmuli(cscale(Bm[2], hk)));
      cB[2] = cmuli(cscale(cadd(Bm[0], Bm[1]), kp));
      cE[0] = csub(cscale(Em[0], kz), cmuli(cscale(Em[2], hk)));
      cE[1] = csub(cscale(Em[1], -kz), cmuli(cscale(Em[2], hk)));
      cE[2] = cmuli(cscale(cadd(Em[0], Em[1]), kp));
      cJ[0] = csub(cscale(Jm[0], kz), cmuli(cscale(Jm[2], hk)));
      cJ[1] = csub(cscale(Jm[1], -kz), cmuli(cscale(Jm[2], hk)));
      cJ[2] = cmuli(cscale(cadd(Jm[0], Jm[1]), kp));
    }
    const float2 gs = csub(cscale(q1, -co.omc), cscale(dq, co.r0));
    const float2 g[3] = {cscale(gs, -0.5f * kp), cscale(gs, 0.5f * kp), cmuli(cscale(gs, kz))};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float2 En = cadd(cadd(cscale(Em[c], co.C), cscale(csub(cB[c], Jm[c]), co.Sk)), g[c]);
      float2 Bn = cadd(csub(cscale(Bm[c], co.C), cscale(cE[c], co.Sk)), cscale(cJ[c], co.omc));
      *f[c] = En;
      *f[3 + c] = Bn;
    }
  }
}

// ---------------------------------------------------------------------------
// Galilean variant: the fields live in coordinates moving with the grid (one
// cell per step, v = dz / dt), where Maxwell's equations gain the advection
// term i w F, w = [k_z] v.  With J constant over the step in those
// coordinates the update is the exact solution, with theta2 = exp(i w dt),
//   X1 = int_0^dt exp(i w u) cos(k u) du,  X2 = int_0^dt exp(i w u) sin(k u) du,
//   phi = int_0^dt exp(i w u) du:
//   E' = theta2 C E + theta2 (S/k) curl B - X1 J
//        + grad[(X1/phi - 1) rho^{n+1} + theta2 (C - X1/phi) rho^n] / k^2
//   B' = theta2 C B - theta2 (S/k) curl E + (X2/k) curl J
// and the current correction enforces the moving-frame continuity
//   div J = (theta2 rho^n - rho^{n+1}) / phi.
// The deposit works on the grid of t^n; rho^{n+1} is moved onto the grid of
// t^{n+1} (exp(i k_z dz), the exact one-node shift of the periodic DFT) and J
// onto the grid of t^{n+1/2} (exp(i k_z dz / 2), taken as zero at the Nyquist
// wavenumber, where half a cell has no real reading).  With the rho^n slot
// holding d = rho^{n+1} - rho^n (both on the grid of t^n) and P = exp(i k_z dz):
//   rho^{n+1}' - theta2 rho^n = (P - theta2) rho^{n+1} + theta2 d
//   charge term numerator     = (r1 P + r0) rho^{n+1} - r0 d,
//   r1 = X1/phi - 1, r0 = theta2 (C - X1/phi).
// Every coefficient is built in FP64 and rounded once to complex float32.
struct GCoef {
  float2 cC, cS, X1, X2k, q1, qd, f1, fd, half;
  float ik2;
};

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zdiv(double2 a, double2 b) {
  const double d = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ __forceinline__ float2 zf(double2 a) { return make_float2((float)a.x, (float)a.y); }

// int_0^dt exp(i a u) du = dt exp(i a dt / 2) sinc(a dt / 2)
__device__ __forceinline__ double2 phase_integral(double a, double dt) {
  const double x = 0.5 * a * dt;
  double sn, cs;
  sincos(x, &sn, &cs);
  const double sc = fabs(x) < 1e-8 ? 1.0 - x * x / 6.0 : sn / x;
  return make_double2(dt * sc * cs, dt * sc * sn);
}

__device__ __forceinline__ GCoef make_gcoef(double kp, double kzm, double kz_dft, double dt, double dz,
                                            bool nyquist) {
  const double v = dz / dt;
  const double k2 = kp * kp + kzm * kzm, k = sqrt(k2);
  const double w = kzm * v;
  double s, c, sw, cw;
  sincos(k * dt, &s, &c);
  sincos(w * dt, &sw, &cw);
  const double2 th2 = make_double2(cw, sw);
  const double2 pp = phase_integral(w + k, dt), pm = phase_integral(w - k, dt), ph = phase_integral(w, dt);
  const double2 X1 = make_double2(0.5 * (pp.x + pm.x), 0.5 * (pp.y + pm.y));
  const double2 X2 = make_double2(0.5 * (pp.y - pm.y), -0.5 * (pp.x - pm.x));   // (pp - pm) / 2i
  const double2 x1p = zdiv(X1, ph);
  const double2 r1 = make_double2(x1p.x - 1.0, x1p.y);
  const double2 r0 = zmul(th2, make_double2(c - x1p.x, -x1p.y));
  double sp, cp, sh, ch;
  sincos(kz_dft * dz, &sp, &cp);
  sincos(0.5 * kz_dft * dz, &sh, &ch);
  const double2 P = make_double2(cp, sp);
  const double2 q1 = zmul(r1, P);
  GCoef o;
  o.cC = zf(make_double2(th2.x * c, th2.y * c));
  o.cS = zf(make_double2(th2.x * s / k, th2.y * s / k));
  o.X1 = zf(X1);
  o.X2k = zf(make_double2(X2.x / k, X2.y / k));
  o.q1 = zf(make_double2((q1.x + r0.x) / k2, (q1.y + r0.y) / k2));
  o.qd = zf(make_double2(-r0.x / k2, -r0.y / k2));
  o.f1 = zf(zdiv(make_double2(P.x - th2.x, P.y - th2.y), ph));
  o.fd = zf(zdiv(th2, ph));
  o.half = nyquist ? make_float2(0.f, 0.f) : make_float2((float)ch, (float)sh);
  o.ik2 = (float)(1.0 / k2);
  return o;
}

template <int M>
__global__ __launch_bounds__(256) void k_psatd_gal(float2* __restrict__ spec, const double* __restrict__ kperp,
                                                   const double* __restrict__ kzm, int nz, int nr, double dt,
                                                   int correct, const double* __restrict__ kz_grid, double dz,
                                                   double dr, int filter) {
  const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= (int64_t)nr * nz) return;
  const int ik = (int)(cell / nz);
  const int iz = (int)(cell % nz);
  const size_t plane = (size_t)nr * nz;
  float2 E[M][3], B[M][3], J[M][3], d0[M], r1[M];
#pragma unroll
  for (int m = 0; m < M; ++m) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      E[m][c] = spec[((size_t)c * M + m) * plane + cell];
      B[m][c] = spec[((size_t)(3 + c) * M + m) * plane + cell];
      J[m][c] = spec[((size_t)(6 + c) * M + m) * plane + cell];
    }
    d0[m] = spec[((size_t)kCompRho0 * M + m) * plane + cell];        // rho^{n+1} - rho^n
    r1[m] = spec[((size_t)(kCompRho0 + 1) * M + m) * plane + cell];
  }
  const double kzd = kzm[iz], kzt = kz_grid[iz];
  const float kz = (float)kzd;
  const bool nyquist = 2 * iz == nz;
  double kp_prev = -1.0;
  GCoef co{};
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const double kpd = kperp[m * nr + ik];
    if (kpd != kp_prev) {
      co = make_gcoef(kpd, kzd, kzt, dt, dz, nyquist);
      kp_prev = kpd;
    }
    const float kp = (float)kpd;
    float2* f[kNumComp];
#pragma unroll
    for (int c = 0; c < kNumComp; ++c) f[c] = spec + ((size_t)c * M + m) * plane + cell;
    float2 Em[3], Bm[3], Jm[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Em[c] = E[m][c];
      Bm[c] = B[m][c];
      Jm[c] = cmul(co.half, J[m][c]);   // onto the grid of t^{n+1/2}
    }
    float2 dq = d0[m], q1 = r1[m];
    if (filter) {
      const double cz = cos(0.5 * kzt * dz), cr = cos(0.5 * kpd * dr);
      const double f1 = cz * cz * cr * cr;
      double fp = f1;
      for (int q = 1; q < filter; ++q) fp *= f1;
      const float fs = (float)fp;
#pragma unroll
      for (int c = 0; c < 3; ++c) Jm[c] = cscale(Jm[c], fs);
      dq = cscale(dq, fs);
      q1 = cscale(q1, fs);
    }
    if (correct) {
      const float2 dvj = cadd(cscale(csub(Jm[0], Jm[1]), kp), cmuli(cscale(Jm[2], kz)));
      const float2 D = cadd(cmul(co.f1, q1), cmul(co.fd, dq));
      const float2 F = cscale(cadd(dvj, D), co.ik2);
      Jm[0] = cadd(Jm[0], cscale(F, -0.5f * kp));
      Jm[1] = cadd(Jm[1], cscale(F, 0.5f * kp));
      Jm[2] = cadd(Jm[2], cmuli(cscale(F, kz)));
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) *f[6 + c] = Jm[c];
    float2 cB[3], cE[3], cJ[3];
    {
      const float hk = 0.5f * kp;
      cB[0] = csub(cscale(Bm[0], kz), cmuli(cscale(Bm[2], hk)));
      cB[1] = csub(cscale(Bm[1], -kz), cmuli(cscale(Bm[2], hk)));
      cB[2] = cmuli(cscale(cadd(Bm[0], Bm[1]), kp));
      cE[0] = csub(cscale(Em[0], kz), cmuli(cscale(Em[2], hk)));
      cE[1] = csub(cscale(Em[1], -kz), cmuli(cscale(Em[2], hk)));
      cE[2] = cmuli(cscale(cadd(Em[0], Em[1]), kp));
      cJ[0] = csub(cscale(Jm[0], kz), cmuli(cscale(Jm[2], hk)));
      cJ[1] = csub(cscale(Jm[1], -kz), cmuli(cscale(Jm[2], hk)));
      cJ[2] = cmuli(cscale(cadd(Jm[0], Jm[1]), kp));
    }
    const float2 gs = cadd(cmul(co.q1, q1), cmul(co.qd, dq));   // already divided by k^2
    const float2 g[3] = {cscale(gs, -0.5f * kp), cscale(gs, 0.5f * kp), cmuli(cscale(gs, kz))};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float2 En = cadd(csub(cadd(cmul(co.cC, Em[c]), cmul(co.cS, cB[c])), cmul(co.X1, Jm[c])), g[c]);
      const float2 Bn = cadd(csub(cmul(co.cC, Bm[c]), cmul(co.cS, cE[c])), cmul(co.X2k, cJ[c]));
      *f[c] = En;
      *f[3 + c] = Bn;
    }
  }
}

// tailhat[c][m][k] = sum_r F_nu[k][r] tail[c][m][r]  (F stored transposed: ft[r][k]).
// Workgroup (row, 64-wide k block): 16 waves split the r sum (several loads in
// flight per wave), LDS reduction in a fixed order.  The first thread of the
// grid also advances the window state (one more move, z_min of node 0), which
// no other part of this launch reads.
__global__ __launch_bounds__(1024) void k_tail_transform(const float2* __restrict__ tail, float2* __restrict__ tailhat,
                                                         const float* const* __restrict__ ft_of_row, int nr,
                                                         DevState* __restrict__ st, double zmin0, double dz) {
  __shared__ float2 part[16][64];
  const int row = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int k = blockIdx.x * 64 + lane;
  if (st && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
    st->n_shift += 1;
    st->zmin = zmin0 + (double)st->n_shift * dz;
  }
  gcfloat_p ft = (gcfloat_p)ft_of_row[row];
  const float2* t = tail + (size_t)row * nr;
  float sx = 0.f, sy = 0.f;
  if (k < nr) {
#pragma unroll 8
    for (int r = wave; r < nr; r += 16) {
      const float a = ft[(size_t)r * nr + k];
      const float2 v = t[r];
      sx += a * v.x;
      sy += a * v.y;
    }
  }
  part[wave][lane] = make_float2(sx, sy);
  __syncthreads();
  if (wave == 0 && k < nr) {
    float2 acc = part[0][lane];
    for (int w = 1; w < 16; ++w) acc = cadd(acc, part[w][lane]);
    tailhat[(size_t)row * nr + k] = acc;
  }
}

// Own field of a cold beam moving rigidly along z with velocity beta (Lorentz
// factor gamma), added to the spectral E, B from the beam's rho in the
// rho^{n+1} slot: phi = rho / (k_perp^2 + [k_z]^2 / gamma^2), E = -grad phi
// with E_z scaled by 1 / gamma^2, B_+ = -i beta E_+, B_- = +i beta E_-.
// div E = k_perp (E_+ - E_-) + i [k_z] E_z = rho holds by construction.
__global__ __launch_bounds__(256) void k_beam_field(float2* __restrict__ spec, const double* __restrict__ kperp,
                                                    const double* __restrict__ kzm, int nz, int nr, int M,
                                                    double gamma, double beta) {
  const size_t plane = (size_t)nr * nz;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)M * plane) return;
  const int m = (int)(idx / plane);
  const size_t cell = idx % plane;
  const int ik = (int)(cell / nz), iz = (int)(cell % nz);
  const double kp = kperp[(size_t)m * nr + ik], kz = kzm[iz];
  const double ig2 = 1.0 / (gamma * gamma);
  const float2 rho = spec[((size_t)(kCompJ + 4) * M + m) * plane + cell];
  const double den = kp * kp + kz * kz * ig2;
  const double pr = rho.x / den, pi = rho.y / den;            // phi
  const double ep_r = 0.5 * kp * pr, ep_i = 0.5 * kp * pi;    // E_+ = k_perp phi / 2
  const double em_r = -ep_r, em_i = -ep_i;                    // E_- = -k_perp phi / 2
  const double ez_r = kz * pi * ig2, ez_i = -kz * pr * ig2;   // E_z = -i [k_z] phi / gamma^2
  float2* f[5];
#pragma unroll
  for (int c = 0; c < 5; ++c) f[c] = spec + ((size_t)c * M + m) * plane + cell;
  f[0]->x += (float)ep_r;
  f[0]->y += (float)ep_i;
  f[1]->x += (float)em_r;
  f[1]->y += (float)em_i;
  f[2]->x += (float)ez_r;
  f[2]->y += (float)ez_i;
  f[3]->x += (float)(beta * ep_i);                            // B_+ = -i beta E_+
  f[3]->y += (float)(-beta * ep_r);
  f[4]->x += (float)(-beta * em_i);                           // B_- = +i beta E_-
  f[4]->y += (float)(beta * em_r);
}

// Absorbing layers at both z ends: one thread per (row, damped column); the
// profile sin^2(pi s / (2 nd)) is evaluated in FP64 and rounded once.
__global__ __launch_bounds__(256) void k_damp(float2* __restrict__ f, int nz, int64_t rows, int nd) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int per = 2 * nd;
  if (i >= rows * per) return;
  const int64_t row = i / per;
  const int c = (int)(i % per);
  const int sdist = c < nd ? c : c - nd;
  const int col = c < nd ? c : nz - 1 - sdist;
  const double a = sinpi(0.5 * (double)sdist / (double)nd);
  const float w = (float)(a * a);
  float2 v = f[row * nz + col];
  f[row * nz + col] = make_float2(v.x * w, v.y * w);
}

void launch_damp(float2* f, int nz, int64_t rows, int nd, hipStream_t s) {
  const int64_t n = rows * 2 * nd;
  if (n == 0) return;
  hipLaunchKernelGGL(k_damp, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, f, nz, rows, nd);
}

void launch_beam_field(float2* spec, const double* kperp, const double* kzm, int nz, int nr, int M, double gamma,
                       double beta, hipStream_t s) {
  const size_t n = (size_t)M * nr * nz;
  hipLaunchKernelGGL(k_beam_field, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, spec, kperp, kzm, nz, nr, M,
                     gamma, beta);
}

template <int M>
static void launch_psatd_m(float2* spec, const double* kperp, const double* kzm, const float2* tw,
                           const float2* tailhat, int nz, int nr, double dt, bool apply_shift, bool correct,
                           const double* kz_grid, double dz, double dr, int filter, bool galilean, hipStream_t s) {
  const int64_t n = (int64_t)nr * nz;
  const dim3 grid((unsigned)((n + 255) / 256));
  if (galilean)
    hipLaunchKernelGGL((k_psatd_gal<M>), grid, dim3(256), 0, s, spec, kperp, kzm, nz, nr, dt, correct ? 1 : 0,
                       kz_grid, dz, dr, filter);
  else
    hipLaunchKernelGGL((k_psatd<M>), grid, dim3(256), 0, s, spec, kperp, kzm, tw, tailhat, nz, nr, dt,
                       apply_shift ? 1 : 0, correct ? 1 : 0, kz_grid, dz, dr, filter);
}

void launch_psatd(float2* spec, const double* kperp, const double* kzm, const float2* tw, const float2* tailhat,
                  int nz, int nr, int M, double dt, bool apply_shift, bool correct, const double* kz_grid, double dz,
                  double dr, int filter, bool galilean, hipStream_t s) {
  switch (M) {
    case 1: launch_psatd_m<1>(spec, kperp, kzm, tw, tailhat, nz, nr, dt, apply_shift, correct, kz_grid, dz, dr, filter, galilean, s); break;
    case 2: launch_psatd_m<2>(spec, kperp, kzm, tw, tailhat, nz, nr, dt, apply_shift, correct, kz_grid, dz, dr, filter, galilean, s); break;
    case 3: launch_psatd_m<3>(spec, kperp, kzm, tw, tailhat, nz, nr, dt, apply_shift, correct, kz_grid, dz, dr, filter, galilean, s); break;
    default: launch_psatd_m<4>(spec, kperp, kzm, tw, tailhat, nz, nr, dt, apply_shift, correct, kz_grid, dz, dr, filter, galilean, s); break;
  }
}

void launch_tail_transform(const float2* tail, float2* tailhat, const float* const* ft_of_row, int nr, int nrows,
                           DevState* st, double zmin0, double dz, hipStream_t s) {
  hipLaunchKernelGGL(k_tail_transform, dim3((nr + 63) / 64, nrows), dim3(1024), 0, s, tail, tailhat, ft_of_row, nr,
                     st, zmin0, dz);
}

}  // namespace pic
