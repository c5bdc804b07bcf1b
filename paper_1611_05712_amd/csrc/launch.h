// Host-side launchers of the kernel translation units (all asynchronous on
// the given stream).
#pragma once

#include "common.h"

namespace pic {

struct InjectTable {
  int ns;                    // injecting mobile species
  int total;                 // particles per window move (all species)
  int start[kMaxSpecies];    // first injected index of each species
  int ppc_z[kMaxSpecies], ppc_r[kMaxSpecies], ppc_t[kMaxSpecies];
  int sp[kMaxSpecies];       // species id stored per particle
  double q[kMaxSpecies], density[kMaxSpecies];
};

struct DiagSel {
  int species;
  int kill;
  double inv_q;
  double zmin;
};

struct DiagMeans {
  double x, y, z, ux, uy, g;
  double slice_len, zcut;
  int half;
};

// setup (FP64)
void launch_kz_table(double* kz, double* kzm, int nz, double dz, int order, hipStream_t st);
void launch_kperp(double* kperp, int nr, double R, int kind, int m, hipStream_t st);
void launch_bessel_matrix(double* B, const double* kperp, int nr, double dr, int nu, hipStream_t st);
void launch_jacobi_svd(const double* A, double* W, double* V, int count, int n, int* fail, hipStream_t st);
void launch_pinv_f32(const double* W, const double* V, float* out, int n, double rcond, hipStream_t st);
void launch_to_f32_transposed(const double* in, float* out, int n, hipStream_t st);
void launch_twiddles(float2* tw, int n, hipStream_t st);

// particles
void launch_gather_push(const Parts& p, const float2* gf, const Grid& g, const SpeciesConst& sc,
                        const DevState* st, uint32_t* key, int* count, int cap, hipStream_t s);
void launch_pack_gather(const float2* real, float2* gf, int nr, int nz, int M, hipStream_t s);
void launch_keys(const Parts& p, const Grid& g, const DevState* st, uint32_t* key, int* count, int cap,
                 hipStream_t s);
int scan_scratch_ints(int n);
void launch_scan(int* count, int n, int* bsum, int* offset, int* cursor, int ncells, DevState* st, hipStream_t s);
void launch_scatter(const Parts& src, const Parts& dst, const uint32_t* key, int* cursor, const DevState* st,
                    int ncells, int cap, hipStream_t s);
struct DepositShape {
  int TZ, TR, ntz, ntr, ntiles;
  int halo;             // cells a particle can move per step (1 or 2)
  int max_items;        // workgroups launched (upper bound of the work list)
  size_t acc_floats2;   // FP32 scratch slot per work item, in float2 units (values x block nodes)
  size_t lds_bytes;     // LDS of one workgroup: FP64 node block + particle staging
  int chunk;            // particles per chunk of a dense tile (2048 .. 8192, tunable)
  int tile_max;         // tiles above this many particles are chunked (3 x chunk)
  size_t ion_doubles;   // FP64 immobile-background block per tile (rho values x block nodes)
};
DepositShape deposit_shape(int nz, int nr, int nmodes, int halo, int64_t cap);
// stages of the deposit: work-list planning, tile accumulation, node combine.
// nchunk holds 2 ntiles + 1 ints: chunks per tile, then the list of tiles with
// more than one chunk and its length; chunk_start holds ntiles + 1.
constexpr int kDepPlan = 1, kDepTiles = 2, kDepCombine = 4, kDepAll = 7;
// ionblk: the per-tile FP64 background blocks added to both densities (null:
// none).  ionblk_out non-null: set-up pass that deposits the particles (the
// immobile background) into those blocks instead of the grid.
// rho_mode: how rho^n is formed.  kRhoDeposit: deposited at x^n like the
// other sources.  After a deposit of the same particles, rho^n is the previous
// rho^{n+1}: kRhoCarry copies it (window at rest), kRhoCarryShift copies it one
// node toward the tail (the window moved by one cell) and re-deposits rho^n in
// the edge tiles at both ends of the window, where particles left and the new
// head column entered.
constexpr int kRhoDeposit = 0, kRhoCarry = 1, kRhoCarryShift = 2;
void launch_deposit(const Parts& p, const int* offset, const DepositShape& d, int* nchunk, int* chunk_start,
                    float2* scratch, float2* real, const double* ionblk, double* ionblk_out, const Grid& g,
                    DevState* st, int stages, int rho_mode, hipStream_t s);
void launch_inject(const Parts& p, DevState* st, const Grid& g, const InjectTable& tab, int cap, hipStream_t s);
void launch_uniform_check(const float2* rho, int rows, int nz, unsigned int* out, hipStream_t s);

// fields
void fft_config(int nz, int& rows_per_wg, size_t& lds);
// Forward transforms of rows [diff_lo, diff_hi) take in[row + diff_off] - in[row]
// as their input (rho^{n+1} - rho^n without an intermediate array).
void launch_fft(const float2* in, float2* out, const float2* tw, int nz, int64_t rows, bool inverse, bool shift,
                float2* tail, hipStream_t s, int64_t diff_lo = 0, int64_t diff_hi = 0, int64_t diff_off = 0);
// Absorbing layers: columns [0, nd) and [nz - nd, nz) of `rows` real-space rows
// scaled by sin^2(pi s / (2 nd)), s the distance from the end column.
void launch_damp(float2* rows_base, int nz, int64_t rows, int nd, hipStream_t s);
int gemm_tile_bm(int n, int pref_bm);
// nonfinite (may be null): set to 1 when a split-precision product yields inf/NaN
void launch_dht_gemm(const float* const* at, const float* const* x, float* const* y, int batch, int n, int ncols,
                     int prec, int pref_bm, hipStream_t s, int* nonfinite = nullptr);
void launch_psatd(float2* spec, const double* kperp, const double* kzm, const float2* tw, const float2* tailhat,
                  int nz, int nr, int M, double dt, bool apply_shift, bool correct, const double* kz_grid, double dz,
                  double dr, int filter, bool galilean, hipStream_t s);
void launch_beam_field(float2* spec, const double* kperp, const double* kzm, int nz, int nr, int M, double gamma,
                       double beta, hipStream_t s);
// tail column transform; with st non-null also one window move of the device state
void launch_tail_transform(const float2* tail, float2* tailhat, const float* const* ft_of_row, int nr, int nrows,
                           DevState* st, double zmin0, double dz, hipStream_t s);

// diagnostics: kDiagBlocks workgroups each leave 9 partial sums
constexpr int kDiagBlocks = 512;
constexpr int kDiagPartialDoubles = kDiagBlocks * 9;
int diag_partial_doubles();
void launch_diag_pass1(const Parts& p, const DevState* st, const DiagSel& sel, double* partial, double* out,
                       hipStream_t s);
void launch_diag_pass2(const Parts& p, const DevState* st, const DiagSel& sel, const DiagMeans& mu, double* partial,
                       double* out, hipStream_t s);
void launch_diag_slices(const Parts& p, const DevState* st, const DiagSel& sel, const DiagMeans& mu, double* acc,
                        double* var, hipStream_t s);
void launch_collect(const Parts& p, const DevState* st, const DiagSel& sel, int64_t cap, const Parts& out,
                    int* counter, int nmax, hipStream_t s);
void launch_count_alive(const Parts& p, const DevState* st, const DiagSel& sel, int* counter, int nmax,
                        hipStream_t s);

// small utilities (api.hip)
void launch_fill_zero(void* p, size_t bytes, hipStream_t s);

}  // namespace pic
