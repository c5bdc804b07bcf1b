// C interface of the quasi-cylindrical order-p PSATD PIC cycle (see include/pic.h).
#include <math.h>
#include <stddef.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "pic.h"
#include "common.h"
#include "launch.h"

using namespace pic;

// records the first HIP error of a sequence into `rc`
#define PIC_CK(expr)                                          \
  do {                                                        \
    if ((expr) != hipSuccess && rc == PIC_OK) rc = PIC_EHIP; \
  } while (0)

namespace pic {

__global__ void k_fill_zero(uint32_t* p, size_t nwords) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < nwords; i += stride) p[i] = 0u;
}

void launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  size_t nw = (bytes + 3) / 4;
  if (nw == 0) return;
  size_t nb = (nw + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)nb), dim3(256), 0, s, (uint32_t*)p, nw);
}

__global__ void k_state_init(DevState* st, double zmin, int n_part) {
  st->zmin = zmin;
  st->n_shift = 0;
  st->n_part = n_part;
  st->n_live = n_part;
  st->pending_shift = 0;
  st->overflow = 0;
  st->nonfinite = 0;
}

__global__ void k_set_npart(DevState* st, int n) {
  st->n_part = n;
  st->n_live = n;
}

// F <- exp(+i k_z dz) (F - tailhat) on the spectral E, B of every mode
__global__ void k_apply_shift(float2* spec, const float2* tw, const float2* tailhat, int nz, int nr, int M) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t plane = (int64_t)nr * nz;
  if (idx >= 6 * M * plane) return;
  int64_t cm = idx / plane;           // c*M + m
  int64_t cell = idx % plane;
  int ik = (int)(cell / nz), iz = (int)(cell % nz);
  float2 ph = cconj(tw[iz]);
  spec[idx] = cmul(ph, csub(spec[idx], tailhat[cm * nr + ik]));
}

// out = a - b over n complex values (the spectral rho^n from the stored
// rho^{n+1} and rho^{n+1} - rho^n)
__global__ void k_csub(float2* out, const float2* a, const float2* b, int64_t n) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < n) out[idx] = csub(a[idx], b[idx]);
}

}  // namespace pic

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
struct SpeciesInfo {
  double q, m;
  int mobile, inject, ppc_z, ppc_r, ppc_t, diag;
  double density;
  int64_t n;
};

struct pic_ctx {
  pic_config cfg;
  hipStream_t stream;
  Grid g;
  int M, nz, nr;
  int64_t cap;
  int n_species;
  SpeciesInfo sp[kMaxSpecies];
  SpeciesConst sc;
  InjectTable inj;
  int hz, hr;
  int gemm_bm;
  DepositShape dep;
  // device
  DevState* st;
  Parts parts[2];
  int cur;
  uint32_t* key;
  int *count, *offset, *cursor, *bsum;
  int *dep_nchunk, *dep_start;
  float2* dep_partial;
  float2 *real, *spec, *tmp, *tail, *tailhat;
  float2* gfield;        // node-interleaved real-space E, B for the gather: [r][z][m][6]
  double* ionblk;        // FP64 immobile-background block of every deposit tile
  double *kz, *kzm, *kperp;
  float2* tw;
  float* mats;           // [m][order slot 0..2][dir 0 fwd / 1 bwd][nr][nr], transposed
  double* setup64;
  const float** ptr_tab; // device pointer tables (see init)
  double *diag_partial, *diag_out, *diag_slices;
  int* misc;             // [0] SVD unconverged, [1..2] uniform check, [3] counter
  double* static_scratch;// device address of the library's static diagnostics scratch on this context's GPU
  bool have_bg;
  bool rho_carry;        // the last deposit's rho^{n+1} is the next step's rho^n (shifted with the window)
  // host mirrors
  int phase;             // 0: expect gather_push, 1: expect deposit, 2: expect spectral_push
  bool eb_stale;
  bool spec_pending;
  uint32_t src_set[kMaxModes];
  int64_t steps;
  int64_t n_shift;
  // timing
  bool timing;
  std::vector<hipEvent_t> ev_pool;
  struct Rec { int phase; hipEvent_t a, b; };
  std::vector<Rec> recs;
  size_t ev_used;
  // pointer-table offsets (entries of ptr_tab)
  int pt_fwd_src, pt_fwd_eb, pt_inv_eb, pt_tail;
  // captured two-step graph and the launch parameters it was captured with
  hipGraphExec_t graph;
  bool graph_ok;
  int graph_bm, graph_chunk;
  bool graph_shift;
  int graph_cur;         // particle buffer the captured steps start from
};

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxSlices = 16384;

struct Carver {
  size_t off = 0;
  char* base = nullptr;
  template <class T>
  T* take(size_t count) {
    off = (off + kAlign - 1) / kAlign * kAlign;
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

int validate(const pic_config* c, const pic_species* s, int ns) {
  if (!c) return PIC_EINVAL;
  if (!is_pow2(c->nz) || c->nz < 64 || c->nz > 4096) return PIC_EINVAL;
  if (c->nr < 32 || c->nr > 1024 || (c->nr % 32)) return PIC_EINVAL;
  if (c->n_modes < 1 || c->n_modes > kMaxModes) return PIC_EINVAL;
  if (c->order < 0 || (c->order % 2) || c->order == 1) return PIC_EINVAL;
  if (!(c->dz > 0) || !(c->dr > 0) || !(c->dt > 0) || !isfinite(c->z_min)) return PIC_EINVAL;
  if (c->dt > 2.0 * c->dz || c->dt > 2.0 * c->dr) return PIC_EINVAL;   // deposit halo of <= 2 cells
  if (c->moving_window && fabs(c->dt - c->dz) > 1e-12 * c->dz) return PIC_EINVAL;
  if (c->kperp_grid < 0 || c->kperp_grid > 2) return PIC_EINVAL;
  if (c->hankel_prec < 0 || c->hankel_prec > 2) return PIC_EINVAL;
  if (c->filter < 0 || c->filter > 4) return PIC_EINVAL;
  if (c->damp_cells < 0 || c->damp_cells > c->nz / 4) return PIC_EINVAL;
  if (c->galilean != 0 && (c->galilean != 1 || !c->moving_window)) return PIC_EINVAL;
  if (c->shape_order != 0 && c->shape_order != 1 && c->shape_order != 3) return PIC_EINVAL;
  if (ns < 0 || ns > kMaxSpecies || (ns > 0 && !s)) return PIC_EINVAL;
  for (int i = 0; i < ns; ++i) {
    const pic_species& p = s[i];
    if (p.n < 0 || !(p.m > 0) || p.q == 0.0 || !isfinite(p.q)) return PIC_EINVAL;
    if (p.n > 0 && (!p.x || !p.y || !p.z || !p.w)) return PIC_EINVAL;
    if (p.n > 0 && p.mobile && (!p.ux || !p.uy || !p.uz)) return PIC_EINVAL;
    if (p.inject && (p.ppc_z < 1 || p.ppc_r < 1 || p.ppc_t < 1 || !(p.density > 0))) return PIC_EINVAL;
    if (p.self_field && !p.mobile) return PIC_EINVAL;
  }
  return PIC_OK;
}

struct Counts {
  int64_t mobile = 0, immobile = 0, inject_per_step = 0;
};

Counts count_species(const pic_config* c, const pic_species* s, int ns) {
  Counts k;
  for (int i = 0; i < ns; ++i) {
    if (s[i].mobile) k.mobile += s[i].n;
    else k.immobile += s[i].n;
    if (s[i].mobile && s[i].inject) k.inject_per_step += (int64_t)c->nr * s[i].ppc_z * s[i].ppc_r * s[i].ppc_t;
  }
  return k;
}

int64_t capacity_for(const pic_config* c, const pic_species* s, int ns, int64_t max_particles) {
  Counts k = count_species(c, s, ns);
  int64_t cap = max_particles > 0 ? max_particles : k.mobile + k.mobile / 8 + 2 * k.inject_per_step;
  cap = std::max(cap, k.mobile + k.inject_per_step);
  cap = std::max(cap, k.immobile);
  cap = std::max<int64_t>(cap, 256);
  return (cap + 255) / 256 * 256;
}

// Lays out (or measures) the workspace.
int halo_cells(double dt, double d) { return std::max(1, (int)ceil(dt / d - 1e-12)); }

// halo of the deposit's tile blocks: the cells a particle moves per step, plus
// one for the wider cubic shape
int deposit_halo(const pic_config* c) {
  return std::max(halo_cells(c->dt, c->dz), halo_cells(c->dt, c->dr)) + (c->shape_order == 3 ? 1 : 0);
}

size_t carve(pic_ctx* x, char* base, const pic_config* c, int64_t cap) {
  Carver cv;
  const DepositShape dep = deposit_shape(c->nz, c->nr, c->n_modes, deposit_halo(c), cap);
  cv.base = base;
  const int M = c->n_modes, nz = c->nz, nr = c->nr;
  const size_t plane = (size_t)nr * nz;
  const int ncells = nz * (nr + 1);
  DevState* st = cv.take<DevState>(1);
  Parts pp[2];
  for (int b = 0; b < 2; ++b) {
    pp[b].x = cv.take<double>(cap);
    pp[b].y = cv.take<double>(cap);
    pp[b].z = cv.take<double>(cap);
    pp[b].uz = cv.take<double>(cap);
    pp[b].ux = cv.take<float>(cap);
    pp[b].uy = cv.take<float>(cap);
    pp[b].w = cv.take<float>(cap);
    pp[b].sp = cv.take<uint8_t>(cap);
  }
  uint32_t* key = cv.take<uint32_t>(cap);
  int* count = cv.take<int>(ncells + 2);
  int* offset = cv.take<int>(ncells + 2);
  int* cursor = cv.take<int>(ncells + 2);
  int* bsum = cv.take<int>(scan_scratch_ints(ncells + 1));
  int* dep_nchunk = cv.take<int>(2 * (size_t)dep.ntiles + 1);   // chunk counts, then the dense-tile list
  int* dep_start = cv.take<int>(dep.ntiles + 1);
  float2* dep_partial = cv.take<float2>((size_t)dep.max_items * dep.acc_floats2);
  float2* real = cv.take<float2>(kNumComp * M * plane);
  float2* spec = cv.take<float2>(kNumComp * M * plane);
  float2* tmp = cv.take<float2>(kNumComp * M * plane);
  double* ionblk = cv.take<double>((size_t)dep.ntiles * dep.ion_doubles);
  float2* gfield = cv.take<float2>(6 * M * plane);
  float2* tail = cv.take<float2>(6 * M * nr);
  float2* tailhat = cv.take<float2>(6 * M * nr);
  double* kz = cv.take<double>(nz);
  double* kzm = cv.take<double>(nz);
  double* kperp = cv.take<double>(M * nr);
  float2* tw = cv.take<float2>(nz);
  float* mats = cv.take<float>((size_t)M * 6 * nr * nr);
  double* setup64 = cv.take<double>((size_t)9 * nr * nr);
  const float** ptr_tab = cv.take<const float*>((size_t)(3 * (5 + 6 + 6) + 6) * M);
  double* dpart = cv.take<double>(diag_partial_doubles());
  double* dout = cv.take<double>(32);
  double* dsl = cv.take<double>(4 * kMaxSlices);
  int* misc = cv.take<int>(16);
  if (x) {
    x->st = st;
    x->parts[0] = pp[0];
    x->parts[1] = pp[1];
    x->key = key;
    x->count = count;
    x->offset = offset;
    x->cursor = cursor;
    x->bsum = bsum;
    x->dep_nchunk = dep_nchunk;
    x->dep_start = dep_start;
    x->dep_partial = dep_partial;
    x->dep = dep;
    x->real = real;
    x->spec = spec;
    x->tmp = tmp;
    x->ionblk = ionblk;
    x->tail = tail;
    x->gfield = gfield;
    x->tailhat = tailhat;
    x->kz = kz;
    x->kzm = kzm;
    x->kperp = kperp;
    x->tw = tw;
    x->mats = mats;
    x->setup64 = setup64;
    x->ptr_tab = ptr_tab;
    x->diag_partial = dpart;
    x->diag_out = dout;
    x->diag_slices = dsl;
    x->misc = misc;
  }
  return cv.off + kAlign;
}

}  // namespace

// ---------------------------------------------------------------------------
// Static scratch of pic_diagnostics_slices_noalloc (for callers that cannot
// allocate): block partial sums, reduced moments and per-slice accumulators
// for at most kStaticSlices slices, 168 KB, one copy per GPU for the life of
// the process.  In host code `scratch` is a host-side stand-in for the array,
// not its device address: host code only ever uses the address that
// hipGetSymbolAddress returns for the current device.
// ---------------------------------------------------------------------------
namespace {
constexpr int kStaticSlices = 4096;
constexpr size_t kStaticScratchDoubles = (size_t)kDiagPartialDoubles + 32 + 4 * (size_t)kStaticSlices;
}  // namespace

static __device__ __align__(256) double scratch[kStaticScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices];   // per device, null until looked up

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
int static_scratch_for_current_device(double** out) {
  *out = nullptr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PIC_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return PIC_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PIC_EHIP;
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return PIC_OK;
}

inline size_t plane_of(const pic_ctx* x) { return (size_t)x->nr * x->nz; }
inline float2* fld(float2* base, const pic_ctx* x, int c, int m) {
  return base + ((size_t)c * x->M + m) * plane_of(x);
}
// matrix slot of Hankel order nu in mode m: nu = m - 1, m, m + 1 -> 0, 1, 2
inline float* mat(const pic_ctx* x, int m, int nu, int dir) {
  int slot = nu - (m - 1);
  return x->mats + ((size_t)(m * 3 + slot) * 2 + dir) * x->nr * x->nr;
}
inline int comp_nu(int c, int m) {
  // E+,E-,Ez,B+,B-,Bz,J+,J-,Jz,rho,rho
  static const int d[kNumComp] = {1, -1, 0, 1, -1, 0, 1, -1, 0, 0, 0};
  return m + d[c];
}

int hip_status(hipError_t e) { return e == hipSuccess ? PIC_OK : PIC_EHIP; }

int check_launch() {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? PIC_OK : PIC_EHIP;
}

static_assert(offsetof(DevState, nonfinite) == offsetof(DevState, overflow) + sizeof(int32_t),
              "sync reads both flags with one copy");

int sync(pic_ctx* x) {
  hipError_t e = hipStreamSynchronize(x->stream);
  if (e != hipSuccess) return PIC_EHIP;
  int rc = check_launch();
  if (rc) return rc;
  int flags[2] = {0, 0};   // overflow, nonfinite (adjacent in DevState)
  if (hipMemcpy(flags, &x->st->overflow, sizeof(flags), hipMemcpyDeviceToHost) != hipSuccess) return PIC_EHIP;
  if (flags[0]) return PIC_ENOSPC;    // particle capacity or deposit work list exceeded
  return flags[1] ? PIC_ENUMERIC : PIC_OK;   // a split-precision Hankel product overflowed
}

hipEvent_t take_event(pic_ctx* x) {
  if (x->ev_used == x->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    x->ev_pool.push_back(e);
  }
  return x->ev_pool[x->ev_used++];
}

// brackets the enclosed launches with events when timing is on
struct Phase {
  pic_ctx* x;
  int phase;
  hipEvent_t a = nullptr;
  Phase(pic_ctx* x_, int ph) : x(x_), phase(ph) {
    if (x->timing) {
      a = take_event(x);
      if (a) (void)hipEventRecord(a, x->stream);
    }
  }
  ~Phase() {
    if (x->timing && a) {
      hipEvent_t b = take_event(x);
      if (b) {
        (void)hipEventRecord(b, x->stream);
        x->recs.push_back({phase, a, b});
      }
    }
  }
};

// forward transform: real[c0 .. c0+nc) -> tmp (FFT) -> spec (DHT).  With the
// sources, the rho^n slot is transformed as rho^{n+1} - rho^n: the current
// correction and the PSATD charge terms need that difference, an order of
// magnitude below rho itself in a wake, and taking it before the transforms
// keeps their FP32 rounding relative to it rather than to rho.
void forward_transform(pic_ctx* x, float2* src_base, int c0, int nc, int pt_entry) {
  const int M = x->M;
  {
    Phase ph(x, PIC_T_FFT_FWD);
    const int64_t plane_rows = (int64_t)M * x->nr;
    const bool src = c0 == kCompJ;
    const int64_t lo = src ? (kCompRho0 - kCompJ) * plane_rows : 0;
    launch_fft(fld(src_base, x, c0, 0), fld(x->tmp, x, c0, 0), x->tw, x->nz, (int64_t)nc * plane_rows, false, false,
               nullptr, x->stream, lo, src ? lo + plane_rows : 0, plane_rows);
  }
  const float* const* tab = x->ptr_tab + pt_entry;
  int batch = nc * M;
  Phase ph(x, PIC_T_DHT_FWD);
  launch_dht_gemm(tab, tab + batch, (float* const*)(tab + 2 * batch), batch, x->nr, 2 * x->nz,
                  x->cfg.hankel_prec, x->gemm_bm, x->stream, &x->st->nonfinite);
}

}  // namespace

// ---------------------------------------------------------------------------
// interface
// ---------------------------------------------------------------------------
extern "C" {

const char* pic_strerror(int status) {
  switch (status) {
    case PIC_OK: return "ok";
    case PIC_EINVAL: return "invalid argument";
    case PIC_ENOSPC: return "workspace too small or particle capacity exceeded";
    case PIC_EHIP: return "HIP runtime error";
    case PIC_ESTATE: return "call out of order";
    case PIC_ENUMERIC: return "non-finite value detected";
    default: return "unknown status";
  }
}

int pic_workspace_bytes(const pic_config* cfg, const pic_species* species, int n_species, int64_t max_particles,
                        size_t* bytes) {
  if (!bytes) return PIC_EINVAL;
  int v = validate(cfg, species, n_species);
  if (v) return v;
  int64_t cap = capacity_for(cfg, species, n_species, max_particles);
  if (cap > (int64_t)INT32_MAX / 2) return PIC_EINVAL;
  *bytes = carve(nullptr, nullptr, cfg, cap);
  return PIC_OK;
}

int pic_init(const pic_config* cfg, const pic_species* species, int n_species, int64_t max_particles,
             void* workspace, size_t bytes, void* hip_stream, pic_ctx** out) {
  if (!out || !workspace) return PIC_EINVAL;
  *out = nullptr;
  int v = validate(cfg, species, n_species);
  if (v) return v;
  int64_t cap = capacity_for(cfg, species, n_species, max_particles);
  if (cap > (int64_t)INT32_MAX / 2) return PIC_EINVAL;
  size_t need = carve(nullptr, nullptr, cfg, cap);
  if (bytes < need) return PIC_ENOSPC;
  Counts cnt = count_species(cfg, species, n_species);
  if (cnt.mobile > cap) return PIC_ENOSPC;
  {
    // the deposit's FP64 tile block must fit one workgroup's LDS
    const DepositShape dep = deposit_shape(cfg->nz, cfg->nr, cfg->n_modes, deposit_halo(cfg), cap);
    int dev = 0, lds_max = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      return PIC_EHIP;
    if (dep.lds_bytes + 1024 > (size_t)lds_max) return PIC_EINVAL;
  }

  pic_ctx* x = new pic_ctx();   // value-initialized: every scalar member starts at zero
  x->cfg = *cfg;
  x->stream = (hipStream_t)hip_stream;
  // the static diagnostics scratch of this GPU (null if the lookup failed:
  // pic_diagnostics_slices_noalloc then reports PIC_EHIP, nothing else uses it)
  (void)static_scratch_for_current_device(&x->static_scratch);
  x->M = cfg->n_modes;
  x->nz = cfg->nz;
  x->nr = cfg->nr;
  x->cap = cap;
  x->n_species = n_species;
  char* base = (char*)(((uintptr_t)workspace + kAlign - 1) / kAlign * kAlign);
  carve(x, base, cfg, cap);
  Grid& g = x->g;
  g.nz = cfg->nz;
  g.nr = cfg->nr;
  g.nmodes = cfg->n_modes;
  g.ncol = cfg->nr + 1;
  g.ncells = cfg->nz * (cfg->nr + 1);
  g.dz = cfg->dz;
  g.dr = cfg->dr;
  g.dt = cfg->dt;
  g.inv_dz = 1.0 / cfg->dz;
  g.inv_dr = 1.0 / cfg->dr;
  g.zmin0 = cfg->z_min;
  g.moving_window = cfg->moving_window;
  g.shape = cfg->shape_order == 3 ? 3 : 1;
  x->hz = halo_cells(cfg->dt, cfg->dz);
  x->hr = halo_cells(cfg->dt, cfg->dr);
  x->gemm_bm = 0;   // automatic per product
  hipStream_t s = x->stream;
  const int M = x->M, nr = x->nr, nz = x->nz;
  const size_t plane = plane_of(x);

  // species tables
  x->inj.ns = 0;
  x->inj.total = 0;
  for (int i = 0; i < n_species; ++i) {
    const pic_species& p = species[i];
    SpeciesInfo& si = x->sp[i];
    si.q = p.q;
    si.m = p.m;
    si.mobile = p.mobile;
    si.inject = p.inject;
    si.ppc_z = p.ppc_z;
    si.ppc_r = p.ppc_r;
    si.ppc_t = p.ppc_t;
    si.diag = p.diag;
    si.density = p.density;
    si.n = p.n;
    x->sc.qm[i] = (float)(p.q / p.m);
    if (p.mobile && p.inject && cfg->moving_window) {
      int k = x->inj.ns++;
      x->inj.start[k] = x->inj.total;
      x->inj.ppc_z[k] = p.ppc_z;
      x->inj.ppc_r[k] = p.ppc_r;
      x->inj.ppc_t[k] = p.ppc_t;
      x->inj.sp[k] = i;
      x->inj.q[k] = p.q;
      x->inj.density[k] = p.density;
      x->inj.total += nr * p.ppc_z * p.ppc_r * p.ppc_t;
    }
  }

  int rc = PIC_OK;
  // -------- zero everything that is read before written
  launch_fill_zero(x->count, (size_t)(g.ncells + 2) * sizeof(int), s);
  launch_fill_zero(x->real, kNumComp * M * plane * sizeof(float2), s);
  launch_fill_zero(x->spec, kNumComp * M * plane * sizeof(float2), s);
  launch_fill_zero(x->ionblk, (size_t)x->dep.ntiles * x->dep.ion_doubles * sizeof(double), s);
  launch_fill_zero(x->gfield, 6 * M * plane * sizeof(float2), s);
  launch_fill_zero(x->tailhat, 6 * M * nr * sizeof(float2), s);
  launch_fill_zero(x->misc, 16 * sizeof(int), s);

  // -------- FP64 spectral setup
  launch_kz_table(x->kz, x->kzm, nz, cfg->dz, cfg->order, s);
  launch_twiddles(x->tw, nz, s);
  const double R = nr * cfg->dr;
  for (int m = 0; m < M; ++m) launch_kperp(x->kperp + (size_t)m * nr, nr, R, cfg->kperp_grid, m, s);
  for (int m = 0; m < M; ++m) {
    double* B = x->setup64;                        // 3 synthesis matrices
    double* W = x->setup64 + (size_t)3 * nr * nr;  // their Jacobi factors
    double* V = x->setup64 + (size_t)6 * nr * nr;
    for (int slot = 0; slot < 3; ++slot) {
      int nu = m - 1 + slot;
      launch_bessel_matrix(B + (size_t)slot * nr * nr, x->kperp + (size_t)m * nr, nr, cfg->dr, nu, s);
    }
    launch_jacobi_svd(B, W, V, 3, nr, x->misc + 0, s);
    for (int slot = 0; slot < 3; ++slot) {
      int nu = m - 1 + slot;
      launch_pinv_f32(W + (size_t)slot * nr * nr, V + (size_t)slot * nr * nr, mat(x, m, nu, 0), nr, kPinvRcond, s);
      launch_to_f32_transposed(B + (size_t)slot * nr * nr, mat(x, m, nu, 1), nr, s);
    }
  }
  // pointer tables for the batched products
  {
    std::vector<const float*> tab;
    auto add_batch = [&](int c0, int nc, int dir, float2* xin, float2* yout) {
      int start = (int)tab.size();
      std::vector<const float*> a, xs, ys;
      for (int c = c0; c < c0 + nc; ++c)
        for (int m = 0; m < M; ++m) {
          a.push_back(mat(x, m, comp_nu(c, m), dir));
          xs.push_back((const float*)fld(xin, x, c, m));
          ys.push_back((const float*)fld(yout, x, c, m));
        }
      tab.insert(tab.end(), a.begin(), a.end());
      tab.insert(tab.end(), xs.begin(), xs.end());
      tab.insert(tab.end(), ys.begin(), ys.end());
      return start;
    };
    x->pt_fwd_src = add_batch(kCompJ, kNumSrc, 0, x->tmp, x->spec);
    x->pt_fwd_eb = add_batch(0, 6, 0, x->tmp, x->spec);
    x->pt_inv_eb = add_batch(0, 6, 1, x->spec, x->tmp);
    // tail transform: F_nu of each E/B (c, m)
    x->pt_tail = (int)tab.size();
    for (int c = 0; c < 6; ++c)
      for (int m = 0; m < M; ++m) tab.push_back(mat(x, m, comp_nu(c, m), 0));
    PIC_CK(hipMemcpyAsync((void*)x->ptr_tab, tab.data(), tab.size() * sizeof(float*), hipMemcpyHostToDevice, s));
    PIC_CK(hipStreamSynchronize(s));
  }

  // -------- immobile background: sort + deposit, transform once
  x->have_bg = cnt.immobile > 0;
  x->cur = 0;
  if (x->have_bg) {
    Parts& P = x->parts[1];
    int64_t off = 0;
    for (int i = 0; i < n_species; ++i) {
      const pic_species& p = species[i];
      if (p.mobile || p.n == 0) continue;
      std::vector<float> qw(p.n);
      for (int64_t k = 0; k < p.n; ++k) qw[k] = (float)(p.q * (double)p.w[k]);
      PIC_CK(hipMemcpyAsync(P.x + off, p.x, p.n * sizeof(double), hipMemcpyHostToDevice, s));
      PIC_CK(hipMemcpyAsync(P.y + off, p.y, p.n * sizeof(double), hipMemcpyHostToDevice, s));
      PIC_CK(hipMemcpyAsync(P.z + off, p.z, p.n * sizeof(double), hipMemcpyHostToDevice, s));
      PIC_CK(hipMemcpyAsync(P.w + off, qw.data(), p.n * sizeof(float), hipMemcpyHostToDevice, s));
      PIC_CK(hipStreamSynchronize(s));
      off += p.n;
    }
    launch_fill_zero(P.ux, cap * sizeof(float), s);
    launch_fill_zero(P.uy, cap * sizeof(float), s);
    launch_fill_zero(P.uz, cap * sizeof(double), s);
    launch_fill_zero(P.sp, cap, s);
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(1), 0, s, x->st, cfg->z_min, (int)off);
    launch_keys(P, g, x->st, x->key, x->count, (int)cap, s);
    launch_scan(x->count, g.ncells + 1, x->bsum, x->offset, x->cursor, g.ncells, x->st, s);
    launch_scatter(P, x->parts[0], x->key, x->cursor, x->st, g.ncells, (int)cap, s);
    if (cfg->moving_window) {
      // the window moves over a background that must look the same from every
      // position: check its deposited density is uniform in z
      launch_deposit(x->parts[0], x->offset, x->dep, x->dep_nchunk, x->dep_start, x->dep_partial, x->real, nullptr,
                     nullptr, g, x->st, kDepAll, kRhoDeposit, s);
      launch_uniform_check(fld(x->real, x, kCompJ + 4, 0), M * nr, nz, (unsigned*)(x->misc + 1), s);
      launch_fill_zero(x->real, kNumComp * M * plane * sizeof(float2), s);
    }
    // keep the background as FP64 blocks of the deposit tiles: every deposit
    // adds them to its tile blocks before rounding to FP32
    launch_deposit(x->parts[0], x->offset, x->dep, x->dep_nchunk, x->dep_start, x->dep_partial, x->real, nullptr,
                   x->ionblk, g, x->st, kDepAll, kRhoDeposit, s);
  }

  // -------- own fields of the beams flagged self_field: each beam alone is
  // sorted and deposited, its rho transformed, and the field of that charge
  // moving rigidly at the beam's mean u_z added to the spectral E, B
  bool self_fields = false;
  for (int i = 0; i < n_species; ++i)
    self_fields = self_fields || (species[i].self_field && species[i].mobile && species[i].n > 0);
  if (self_fields) {
    Parts& P = x->parts[1];
    for (int i = 0; i < n_species; ++i) {
      const pic_species& p = species[i];
      if (!p.self_field || !p.mobile || p.n == 0) continue;
      double sw = 0.0, su = 0.0;
      std::vector<float> qw(p.n);
      for (int64_t k = 0; k < p.n; ++k) {
        sw += (double)p.w[k];
        su += (double)p.w[k] * (double)p.uz[k];
        qw[k] = (float)(p.q * (double)p.w[k]);
      }
      const double ubar = sw > 0.0 ? su / sw : 0.0;
      const double gam = sqrt(1.0 + ubar * ubar), beta = ubar / gam;
      PIC_CK(hipMemcpyAsync(P.x, p.x, p.n * sizeof(double), hipMemcpyHostToDevice, s));
      PIC_CK(hipMemcpyAsync(P.y, p.y, p.n * sizeof(double), hipMemcpyHostToDevice, s));
      PIC_CK(hipMemcpyAsync(P.z, p.z, p.n * sizeof(double), hipMemcpyHostToDevice, s));
      PIC_CK(hipMemcpyAsync(P.w, qw.data(), p.n * sizeof(float), hipMemcpyHostToDevice, s));
      PIC_CK(hipStreamSynchronize(s));
      launch_fill_zero(P.ux, cap * sizeof(float), s);
      launch_fill_zero(P.uy, cap * sizeof(float), s);
      launch_fill_zero(P.uz, cap * sizeof(double), s);
      launch_fill_zero(P.sp, cap, s);
      hipLaunchKernelGGL(k_state_init, dim3(1), dim3(1), 0, s, x->st, cfg->z_min, (int)p.n);
      launch_keys(P, g, x->st, x->key, x->count, (int)cap, s);
      launch_scan(x->count, g.ncells + 1, x->bsum, x->offset, x->cursor, g.ncells, x->st, s);
      launch_scatter(P, x->parts[0], x->key, x->cursor, x->st, g.ncells, (int)cap, s);
      launch_deposit(x->parts[0], x->offset, x->dep, x->dep_nchunk, x->dep_start, x->dep_partial, x->real, nullptr,
                     nullptr, g, x->st, kDepAll, kRhoDeposit, s);
      forward_transform(x, x->real, kCompJ, kNumSrc, x->pt_fwd_src);
      launch_beam_field(x->spec, x->kperp, x->kzm, nz, nr, M, gam, beta, s);
    }
    // real-space E, B and the gather copy of the initial fields
    const float* const* tab = x->ptr_tab + x->pt_inv_eb;
    launch_dht_gemm(tab, tab + 6 * M, (float* const*)(tab + 12 * M), 6 * M, nr, 2 * nz, cfg->hankel_prec,
                    x->gemm_bm, s);
    launch_fft(fld(x->tmp, x, 0, 0), fld(x->real, x, 0, 0), x->tw, nz, (int64_t)6 * M * nr, true, false, nullptr, s);
    launch_pack_gather(x->real, x->gfield, nr, nz, M, s);
    launch_fill_zero(fld(x->real, x, kCompJ, 0), (size_t)kNumSrc * M * plane * sizeof(float2), s);
    launch_fill_zero(fld(x->spec, x, kCompJ, 0), (size_t)kNumSrc * M * plane * sizeof(float2), s);
  }

  // -------- mobile particles
  {
    Parts& P = x->parts[0];
    int64_t off = 0;
    for (int i = 0; i < n_species; ++i) {
      const pic_species& p = species[i];
      if (!p.mobile || p.n == 0) continue;
      std::vector<float> qw(p.n);
      std::vector<double> uz(p.uz, p.uz + p.n);
      std::vector<uint8_t> id(p.n, (uint8_t)i);
      for (int64_t k = 0; k < p.n; ++k) qw[k] = (float)(p.q * (double)p.w[k]);
      PIC_CK(hipMemcpyAsync(P.x + off, p.x, p.n * sizeof(double), hipMemcpyHostToDevice, s));
      PIC_CK(hipMemcpyAsync(P.y + off, p.y, p.n * sizeof(double), hipMemcpyHostToDevice, s));
      PIC_CK(hipMemcpyAsync(P.z + off, p.z, p.n * sizeof(double), hipMemcpyHostToDevice, s));
      PIC_CK(hipMemcpyAsync(P.ux + off, p.ux, p.n * sizeof(float), hipMemcpyHostToDevice, s));
      PIC_CK(hipMemcpyAsync(P.uy + off, p.uy, p.n * sizeof(float), hipMemcpyHostToDevice, s));
      PIC_CK(hipMemcpyAsync(P.uz + off, uz.data(), p.n * sizeof(double), hipMemcpyHostToDevice, s));
      PIC_CK(hipMemcpyAsync(P.w + off, qw.data(), p.n * sizeof(float), hipMemcpyHostToDevice, s));
      PIC_CK(hipMemcpyAsync(P.sp + off, id.data(), p.n, hipMemcpyHostToDevice, s));
      PIC_CK(hipStreamSynchronize(s));
      off += p.n;
    }
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(1), 0, s, x->st, cfg->z_min, (int)off);
  }
  if (rc == PIC_OK) rc = sync(x);
  if (rc == PIC_OK) {
    int misc[3];
    PIC_CK(hipMemcpy(misc, x->misc, sizeof(misc), hipMemcpyDeviceToHost));
    if (misc[0]) rc = PIC_EINVAL;   // Jacobi SVD of a Hankel matrix did not converge
    if (x->have_bg && cfg->moving_window) {
      float dmax, amax;
      memcpy(&dmax, &misc[1], 4);
      memcpy(&amax, &misc[2], 4);
      if (dmax > 1e-5f * amax) rc = PIC_EINVAL;   // background not uniform in z
    }
  }
  if (rc != PIC_OK) {
    delete x;
    return rc;
  }
  x->phase = 0;
  x->eb_stale = false;
  x->spec_pending = false;
  x->steps = 0;
  x->n_shift = 0;
  *out = x;
  return PIC_OK;
}

int pic_gather_push(pic_ctx* x) {
  if (!x) return PIC_EINVAL;
  if (x->phase != 0) return PIC_ESTATE;
  {
    Phase ph(x, PIC_T_GATHER_PUSH);
    launch_gather_push(x->parts[x->cur], x->gfield, x->g, x->sc, x->st, x->key, x->count, (int)x->cap, x->stream);
  }
  x->phase = 1;
  return check_launch();
}

int pic_deposit(pic_ctx* x) {
  if (!x) return PIC_EINVAL;
  if (x->phase != 1) return PIC_ESTATE;
  const Grid& g = x->g;
  {
    Phase ph(x, PIC_T_SCAN);
    launch_scan(x->count, g.ncells + 1, x->bsum, x->offset, x->cursor, g.ncells, x->st, x->stream);
  }
  {
    Phase ph(x, PIC_T_SORT);
    launch_scatter(x->parts[x->cur], x->parts[x->cur ^ 1], x->key, x->cursor, x->st, g.ncells, (int)x->cap,
                   x->stream);
  }
  x->cur ^= 1;
  const double* ion = x->have_bg ? x->ionblk : nullptr;
  // rho^n: the same particles at the same positions as the last deposit's
  // rho^{n+1} when that deposit was this context's previous step
  const int rho_mode = !x->rho_carry ? kRhoDeposit : x->cfg.moving_window ? kRhoCarryShift : kRhoCarry;
  const int stage[3] = {kDepPlan, kDepTiles, kDepCombine};
  const int timer[3] = {PIC_T_DEP_PLAN, PIC_T_DEPOSIT, PIC_T_DEP_COMBINE};
  for (int k = 0; k < 3; ++k) {
    Phase ph(x, timer[k]);
    launch_deposit(x->parts[x->cur], x->offset, x->dep, x->dep_nchunk, x->dep_start, x->dep_partial, x->real, ion,
                   nullptr, g, x->st, stage[k], rho_mode, x->stream);
  }
  x->rho_carry = true;
  x->phase = 2;
  return check_launch();
}

int pic_spectral_push(pic_ctx* x) {
  if (!x) return PIC_EINVAL;
  bool sources_set = true;
  for (int m = 0; m < x->M; ++m) sources_set = sources_set && (x->src_set[m] == 0x1Fu);
  if (x->phase != 2 && !(x->phase == 0 && sources_set)) return PIC_ESTATE;
  if (x->phase == 0) x->rho_carry = false;   // sources given by the caller, not deposited
  hipStream_t s = x->stream;
  const int M = x->M, nr = x->nr, nz = x->nz;
  bool apply_shift = x->spec_pending;
  // with absorbing layers the damped real-space E, B are the state
  if (x->eb_stale || x->cfg.damp_cells > 0) {
    forward_transform(x, x->real, 0, 6, x->pt_fwd_eb);
    x->eb_stale = false;
    apply_shift = false;
  }
  forward_transform(x, x->real, kCompJ, kNumSrc, x->pt_fwd_src);
  {
    Phase ph(x, PIC_T_PSATD);
    launch_psatd(x->spec, x->kperp, x->kzm, x->tw, x->tailhat, nz, nr, M, x->cfg.dt, apply_shift,
                 x->cfg.current_correction != 0, x->kz, x->cfg.dz, x->cfg.dr, x->cfg.filter, x->cfg.galilean != 0, s);
  }
  x->spec_pending = false;
  {
    Phase ph(x, PIC_T_DHT_INV);
    const float* const* tab = x->ptr_tab + x->pt_inv_eb;
    int batch = 6 * M;
    launch_dht_gemm(tab, tab + batch, (float* const*)(tab + 2 * batch), batch, nr, 2 * nz, x->cfg.hankel_prec,
                    x->gemm_bm, s, &x->st->nonfinite);
  }
  const bool mw = x->cfg.moving_window != 0;
  // the Galilean update leaves E, B on the moved grid: no shift of their own
  const bool shift_fields = mw && !x->cfg.galilean;
  {
    Phase ph(x, PIC_T_FFT_INV);
    launch_fft(fld(x->tmp, x, 0, 0), fld(x->real, x, 0, 0), x->tw, nz, (int64_t)6 * M * nr, true, shift_fields,
               x->tail, s);
  }
  if (x->cfg.damp_cells > 0) {
    Phase ph(x, PIC_T_WINDOW);
    launch_damp(fld(x->real, x, 0, 0), nz, (int64_t)6 * M * nr, x->cfg.damp_cells, s);
  }
  {
    Phase ph(x, PIC_T_PACK);
    launch_pack_gather(x->real, x->gfield, nr, nz, M, s);
  }
  if (mw) {
    Phase ph(x, PIC_T_WINDOW);
    launch_tail_transform(x->tail, x->tailhat, x->ptr_tab + x->pt_tail, nr, 6 * M, x->st, x->cfg.z_min, x->cfg.dz, s);
    if (x->inj.total > 0) launch_inject(x->parts[x->cur], x->st, x->g, x->inj, (int)x->cap, s);
    x->spec_pending = shift_fields;
    x->n_shift += 1;
  }
  for (int m = 0; m < M; ++m) x->src_set[m] = 0;
  x->phase = 0;
  x->steps += 1;
  return check_launch();
}

int pic_step(pic_ctx* x, int n) {
  if (!x || n < 0) return PIC_EINVAL;
  for (int i = 0; i < n; ++i) {
    int rc = pic_gather_push(x);
    if (rc) return rc;
    rc = pic_deposit(x);
    if (rc) return rc;
    rc = pic_spectral_push(x);
    if (rc) return rc;
  }
  return PIC_OK;
}

int pic_sync(pic_ctx* x) {
  if (!x) return PIC_EINVAL;
  return sync(x);
}

int pic_num_particles(pic_ctx* x, int64_t* n) {
  if (!x || !n) return PIC_EINVAL;
  DiagSel sel{};
  sel.kill = (x->cfg.moving_window && x->n_shift > 0) ? 1 : 0;
  sel.zmin = x->cfg.z_min + (double)x->n_shift * x->cfg.dz;
  int* counter = x->misc + 3;
  launch_fill_zero(counter, sizeof(int), x->stream);
  launch_count_alive(x->parts[x->cur], x->st, sel, counter, (int)x->cap, x->stream);
  int rc = sync(x);
  if (rc) return rc;
  int v;
  if (hipMemcpy(&v, counter, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return PIC_EHIP;
  *n = v;
  return PIC_OK;
}

int pic_get_particles(pic_ctx* x, int species, int64_t cap, double* xyz, double* uvw, float* w, int64_t* n) {
  if (!x || !xyz || !uvw || !n || species < 0 || species >= x->n_species || cap < 0) return PIC_EINVAL;
  if (!x->sp[species].mobile) return PIC_EINVAL;
  int rc = sync(x);
  if (rc) return rc;
  // stage through the ping-pong buffer that is not in use
  const Parts& stage = x->parts[x->cur ^ 1];
  int64_t lim = std::min<int64_t>(cap, x->cap);
  DiagSel sel{};
  sel.species = species;
  sel.kill = (x->cfg.moving_window && x->n_shift > 0) ? 1 : 0;
  sel.zmin = x->cfg.z_min + (double)x->n_shift * x->cfg.dz;
  sel.inv_q = 1.0 / x->sp[species].q;
  int* counter = x->misc + 3;
  launch_fill_zero(counter, sizeof(int), x->stream);
  launch_collect(x->parts[x->cur], x->st, sel, lim, stage, counter, (int)x->cap, x->stream);
  rc = sync(x);
  if (rc) return rc;
  int cnt;
  if (hipMemcpy(&cnt, counter, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return PIC_EHIP;
  int64_t got = std::min<int64_t>(cnt, lim);
  std::vector<double> hx(got), hy(got), hz(got), hw(got);
  std::vector<float> hu(got), hv(got), hq(got);
  bool ok = hipMemcpy(hx.data(), stage.x, got * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess &&
            hipMemcpy(hy.data(), stage.y, got * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess &&
            hipMemcpy(hz.data(), stage.z, got * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess &&
            hipMemcpy(hu.data(), stage.ux, got * sizeof(float), hipMemcpyDeviceToHost) == hipSuccess &&
            hipMemcpy(hv.data(), stage.uy, got * sizeof(float), hipMemcpyDeviceToHost) == hipSuccess &&
            hipMemcpy(hw.data(), stage.uz, got * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess &&
            hipMemcpy(hq.data(), stage.w, got * sizeof(float), hipMemcpyDeviceToHost) == hipSuccess;
  if (!ok) return PIC_EHIP;
  for (int64_t k = 0; k < got; ++k) {
    xyz[3 * k] = hx[k];
    xyz[3 * k + 1] = hy[k];
    xyz[3 * k + 2] = hz[k];
    uvw[3 * k] = hu[k];
    uvw[3 * k + 1] = hv[k];
    uvw[3 * k + 2] = hw[k];
    if (w) w[k] = hq[k];
  }
  *n = got;
  if (cnt > lim) return PIC_ENOSPC;
  return PIC_OK;
}

int pic_get_field(pic_ctx* x, int mode, int comp, int spectral, void* host_dst) {
  if (!x || !host_dst || mode < 0 || mode >= x->M || comp < 0 || comp >= kNumComp) return PIC_EINVAL;
  if (spectral && comp < 6 && x->spec_pending) {
    int64_t n = (int64_t)6 * x->M * plane_of(x);
    hipLaunchKernelGGL(k_apply_shift, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, x->stream, x->spec, x->tw,
                       x->tailhat, x->nz, x->nr, x->M);
    x->spec_pending = false;
  }
  int rc = sync(x);
  if (rc) return rc;
  const float2* src = fld(spectral ? x->spec : x->real, x, comp, mode);
  if (spectral && comp == kCompRho0) {
    // the slot holds rho^{n+1} - rho^n; the transform buffer is free between steps
    float2* t = fld(x->tmp, x, kCompRho0, mode);
    const int64_t n = plane_of(x);
    hipLaunchKernelGGL(k_csub, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, x->stream, t,
                       fld(x->spec, x, kCompRho0 + 1, mode), src, n);
    rc = sync(x);
    if (rc) return rc;
    src = t;
  }
  if (hipMemcpy(host_dst, src, plane_of(x) * sizeof(float2), hipMemcpyDeviceToHost) != hipSuccess) return PIC_EHIP;
  return PIC_OK;
}

int pic_set_field(pic_ctx* x, int mode, int comp, const void* host_src) {
  if (!x || !host_src || mode < 0 || mode >= x->M || comp < 0 || comp >= kNumComp) return PIC_EINVAL;
  int rc = sync(x);
  if (rc) return rc;
  float2* dst = fld(x->real, x, comp, mode);
  if (hipMemcpy(dst, host_src, plane_of(x) * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess) return PIC_EHIP;
  if (comp < 6) {
    x->eb_stale = true;
    x->spec_pending = false;
    launch_pack_gather(x->real, x->gfield, x->nr, x->nz, x->M, x->stream);
    rc = sync(x);
    if (rc) return rc;
  } else {
    x->src_set[mode] |= 1u << (comp - kCompJ);
    x->rho_carry = false;   // the next deposit's rho^n comes from the particles again
  }
  return PIC_OK;
}

int pic_get_state(pic_ctx* x, double* z_min, int64_t* steps) {
  if (!x) return PIC_EINVAL;
  if (z_min) *z_min = x->cfg.z_min + (double)x->n_shift * x->cfg.dz;
  if (steps) *steps = x->steps;
  return PIC_OK;
}

namespace {
// Moments of one species (two passes) and, when `slice_sigma` is given, the
// weighted rms gamma of every slice (0 for a skipped slice).
// Device scratch of one diagnostics call: block partial sums, the reduced
// moments and per-slice accumulators (count, weight, weighted gamma; then the
// weighted squared deviation), room for max_slices slices.
struct DiagScratch {
  double* partial;
  double* out;
  double* slices;
  int max_slices;
  int too_many_slices;   // status returned when the slices exceed max_slices
};

DiagScratch workspace_diag_scratch(pic_ctx* x) {
  return DiagScratch{x->diag_partial, x->diag_out, x->diag_slices, kMaxSlices, PIC_EINVAL};
}

// Beam moments of one species and, with sigma_gamma/count (cap entries),
// the per-slice values; *n_total (if given) receives the slice count.  The
// per-slice sums are brought to the host a block at a time through a fixed
// stack buffer, so the call allocates nothing on the host either.
int diag_run(pic_ctx* x, const pic_diag_req* req, pic_diag_out* out, const DiagScratch& scr, double* slice_sigma,
             double* slice_count, int cap, int32_t* n_total) {
  if (!x || !req || !out) return PIC_EINVAL;
  if (req->species < 0 || req->species >= x->n_species || !x->sp[req->species].mobile) return PIC_EINVAL;
  if (!(req->slice_len > 0) || !(req->n_sigma > 0)) return PIC_EINVAL;
  memset(out, 0, sizeof(*out));
  if (n_total) *n_total = 0;
  hipStream_t s = x->stream;
  DiagSel sel{};
  sel.species = req->species;
  sel.kill = (x->cfg.moving_window && x->n_shift > 0) ? 1 : 0;
  sel.zmin = x->cfg.z_min + (double)x->n_shift * x->cfg.dz;
  sel.inv_q = 1.0 / x->sp[req->species].q;
  const Parts& P = x->parts[x->cur];
  launch_diag_pass1(P, x->st, sel, scr.partial, scr.out, s);
  int rc = sync(x);
  if (rc) return rc;
  double a[9];
  PIC_CK(hipMemcpy(a, scr.out, sizeof(a), hipMemcpyDeviceToHost));
  if (rc) return rc;
  out->n = (int64_t)a[0];
  out->nan_flag = a[8] > 0 ? 1 : 0;
  if (a[0] <= 0 || !(a[1] > 0)) return out->nan_flag ? PIC_ENUMERIC : PIC_OK;
  const double W = a[1];
  DiagMeans mu{};
  mu.x = a[2] / W;
  mu.y = a[3] / W;
  mu.z = a[4] / W;
  mu.ux = a[5] / W;
  mu.uy = a[6] / W;
  mu.g = a[7] / W;
  launch_diag_pass2(P, x->st, sel, mu, scr.partial, scr.out, s);
  rc = sync(x);
  if (rc) return rc;
  double b[8];
  PIC_CK(hipMemcpy(b, scr.out, sizeof(b), hipMemcpyDeviceToHost));
  if (rc) return rc;
  for (double& v : b) v /= W;
  out->eps_nx = sqrt(std::max(0.0, b[0] * b[1] - b[2] * b[2]));
  out->eps_ny = sqrt(std::max(0.0, b[3] * b[4] - b[5] * b[5]));
  out->mean_gamma = mu.g;
  out->sigma_gamma = sqrt(b[6]);
  out->z_mean = mu.z;
  out->sigma_z = sqrt(b[7]);
  if (out->sigma_z > 0) {
    mu.slice_len = req->slice_len;
    mu.zcut = req->n_sigma * out->sigma_z;
    const double h = ceil(mu.zcut / req->slice_len);
    if (h > scr.max_slices / 2) {
      if (n_total) *n_total = h < 1e9 ? (int32_t)(2 * h) : INT32_MAX;
      return scr.too_many_slices;
    }
    mu.half = (int)h;
    const int ns = 2 * mu.half;
    if (n_total) *n_total = ns;
    double* acc = scr.slices;
    double* var = scr.slices + 3 * (size_t)scr.max_slices;
    launch_fill_zero(acc, 3 * (size_t)ns * sizeof(double), s);
    launch_fill_zero(var, (size_t)ns * sizeof(double), s);
    launch_diag_slices(P, x->st, sel, mu, acc, var, s);
    rc = sync(x);
    if (rc) return rc;
    constexpr int kBlk = 256;
    double ha[3 * kBlk], hv[kBlk];
    double sum = 0;
    int kept = 0;
    for (int k0 = 0; k0 < ns; k0 += kBlk) {
      const int nb = std::min(kBlk, ns - k0);
      PIC_CK(hipMemcpy(ha, acc + 3 * (size_t)k0, 3 * (size_t)nb * sizeof(double), hipMemcpyDeviceToHost));
      PIC_CK(hipMemcpy(hv, var + k0, (size_t)nb * sizeof(double), hipMemcpyDeviceToHost));
      if (rc) return rc;
      for (int q = 0; q < nb; ++q) {
        const int k = k0 + q;
        const bool keep = !(ha[3 * q] < req->min_per_slice) && ha[3 * q + 1] > 0;
        const double sg = keep ? sqrt(hv[q] / ha[3 * q + 1]) : 0.0;
        if (k < cap) {
          if (slice_count) slice_count[k] = ha[3 * q];
          if (slice_sigma) slice_sigma[k] = sg;
        }
        if (keep) {
          sum += sg;
          ++kept;
        }
      }
    }
    out->n_slices = kept;
    out->mean_slice_sigma_gamma = kept ? sum / kept : 0.0;
  }
  return out->nan_flag ? PIC_ENUMERIC : PIC_OK;
}
}  // namespace

int pic_diagnostics(pic_ctx* x, const pic_diag_req* req, pic_diag_out* out) {
  if (!x) return PIC_EINVAL;
  return diag_run(x, req, out, workspace_diag_scratch(x), nullptr, nullptr, 0, nullptr);
}
int pic_diagnostics_slices(pic_ctx* x, const pic_diag_req* req, pic_diag_out* out, double* sigma_gamma,
                           double* count, int32_t cap, int32_t* n_total) {
  if (!x || !req || !out || !n_total || cap < 0 || (cap > 0 && (!sigma_gamma || !count))) return PIC_EINVAL;
  return diag_run(x, req, out, workspace_diag_scratch(x), sigma_gamma, count, cap, n_total);
}

int pic_diagnostics_slices_noalloc(pic_ctx* x, const pic_diag_req* req, pic_diag_out* out, double* sigma_gamma,
                                   double* count, int32_t cap, int32_t* n_total) {
  if (!x || !req || !out || !n_total || cap < 0 || (cap > 0 && (!sigma_gamma || !count))) return PIC_EINVAL;
  if (!x->static_scratch) return PIC_EHIP;
  double* base = x->static_scratch;
  const DiagScratch scr{base, base + kDiagPartialDoubles, base + kDiagPartialDoubles + 32, kStaticSlices,
                        PIC_ENOSPC};
  return diag_run(x, req, out, scr, sigma_gamma, count, cap, n_total);
}

int pic_free(pic_ctx* x) {
  if (!x) return PIC_EINVAL;
  int rc = sync(x);
  for (hipEvent_t e : x->ev_pool) (void)hipEventDestroy(e);
  if (x->graph_ok) (void)hipGraphExecDestroy(x->graph);
  delete x;
  return rc;
}

// ---------------------------------------------------------------------------
// tuning, graph replay, batches
// ---------------------------------------------------------------------------
int pic_get_tuning(pic_ctx* x, pic_tuning* t) {
  if (!x || !t) return PIC_EINVAL;
  t->gemm_tile_m = x->gemm_bm == 0 ? 0 : 32 * gemm_tile_bm(x->nr, x->gemm_bm);
  t->deposit_chunk = x->dep.chunk;
  return PIC_OK;
}

int pic_set_tuning(pic_ctx* x, const pic_tuning* t) {
  if (!x || !t) return PIC_EINVAL;
  if (t->gemm_tile_m != 0 && t->gemm_tile_m != 32 && t->gemm_tile_m != 64 && t->gemm_tile_m != 128)
    return PIC_EINVAL;
  if (t->deposit_chunk != 2048 && t->deposit_chunk != 4096 && t->deposit_chunk != 8192) return PIC_EINVAL;
  if (t->gemm_tile_m != 0 && (x->nr % t->gemm_tile_m) != 0) return PIC_EINVAL;
  x->gemm_bm = t->gemm_tile_m / 32;
  x->dep.chunk = t->deposit_chunk;
  x->dep.tile_max = 3 * t->deposit_chunk;
  return PIC_OK;
}

namespace {

// Captures two steps (the particle buffers ping-pong, so two steps return to
// the same launch arguments) into a graph.  The host mirrors advanced by the
// capture are restored: nothing ran.
int capture_graph(pic_ctx* x) {
  if (x->graph_ok) {
    // the previous graph's replays may still run on the stream: wait for
    // them before its executable (and the memory its launches use) is freed
    if (hipStreamSynchronize(x->stream) != hipSuccess) return PIC_EHIP;
    (void)hipGraphExecDestroy(x->graph);
    x->graph_ok = false;
  }
  const int cur = x->cur, phase = x->phase;
  const int64_t steps = x->steps, n_shift = x->n_shift;
  const bool spec_pending = x->spec_pending, eb_stale = x->eb_stale, rho_carry = x->rho_carry;
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(x->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return PIC_EHIP;
  int rc = pic_step(x, 2);
  hipError_t e = hipStreamEndCapture(x->stream, &g);
  x->cur = cur;
  x->phase = phase;
  x->steps = steps;
  x->n_shift = n_shift;
  x->spec_pending = spec_pending;
  x->eb_stale = eb_stale;
  x->rho_carry = rho_carry;
  if (rc != PIC_OK || e != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return rc != PIC_OK ? rc : PIC_EHIP;
  }
  e = hipGraphInstantiate(&x->graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return PIC_EHIP;
  x->graph_ok = true;
  x->graph_bm = x->gemm_bm;
  x->graph_chunk = x->dep.chunk;
  x->graph_shift = x->spec_pending;
  x->graph_cur = x->cur;
  return PIC_OK;
}

// Enqueues n steps as graph replays (an odd step runs eagerly).
int graph_steps(pic_ctx* x, int n) {
  if (x->phase != 0) return PIC_ESTATE;
  if (!x->stream || x->timing) return PIC_EINVAL;   // the legacy stream cannot be captured
  for (int m = 0; m < x->M; ++m)
    if (x->src_set[m]) return PIC_ESTATE;
  int rc = PIC_OK;
  // one eager step settles the one-time work (re-transform of set fields,
  // first window shift, kernel attributes, a rho^n that cannot be carried
  // over), so that every captured step is an ordinary one
  if (n > 0 && (x->steps == 0 || x->eb_stale || !x->rho_carry)) {
    rc = pic_step(x, 1);
    if (rc) return rc;
    --n;
  }
  if (n >= 2) {
    // the captured steps read the particle buffer that was current at the
    // capture: after an odd number of steps since, an odd remainder is taken
    // first (eagerly), else the graph is captured again
    const bool params = x->graph_ok && x->graph_bm == x->gemm_bm && x->graph_chunk == x->dep.chunk &&
                        x->graph_shift == x->spec_pending;
    if (params && x->cur != x->graph_cur && (n & 1)) {
      if ((rc = pic_step(x, 1)) != PIC_OK) return rc;
      --n;
    }
    if (!params || x->cur != x->graph_cur) {
      rc = capture_graph(x);
      if (rc) return rc;
    }
  }
  for (; n >= 2; n -= 2) {
    if (hipGraphLaunch(x->graph, x->stream) != hipSuccess) return PIC_EHIP;
    x->steps += 2;
    if (x->cfg.moving_window) x->n_shift += 2;
  }
  if (n == 1) rc = pic_step(x, 1);
  return rc;
}

}  // namespace

int pic_step_graph(pic_ctx* x, int n) {
  if (!x || n < 0) return PIC_EINVAL;
  return graph_steps(x, n);
}

}  // extern "C"

// A batch of independent contexts advanced by one graph: two steps of every
// context, each on its own stream, forked from and joined back into the
// batch's lead stream inside one capture, so a replay is one launch for the
// whole batch and the GPU overlaps the instances' kernels.
struct pic_batch {
  std::vector<pic_ctx*> ctx;
  hipStream_t lead = nullptr;
  hipEvent_t ev_lead = nullptr;          // lead stream -> context streams
  std::vector<hipEvent_t> ev_ctx;        // context streams -> lead stream
  hipGraphExec_t exec = nullptr;
  // launch parameters and current particle buffer of every context when the
  // graph was captured
  std::vector<int> bm, chunk, cur;
  std::vector<char> shift;
};

namespace {

struct HostMirror {
  int cur, phase;
  int64_t steps, n_shift;
  bool spec_pending, eb_stale, rho_carry;
};

HostMirror save_mirror(const pic_ctx* x) {
  return {x->cur, x->phase, x->steps, x->n_shift, x->spec_pending, x->eb_stale, x->rho_carry};
}

void restore_mirror(pic_ctx* x, const HostMirror& h) {
  x->cur = h.cur;
  x->phase = h.phase;
  x->steps = h.steps;
  x->n_shift = h.n_shift;
  x->spec_pending = h.spec_pending;
  x->eb_stale = h.eb_stale;
  x->rho_carry = h.rho_carry;
}

bool batch_params(const pic_batch* b) {
  if (!b->exec) return false;
  for (size_t i = 0; i < b->ctx.size(); ++i) {
    const pic_ctx* x = b->ctx[i];
    if (x->gemm_bm != b->bm[i] || x->dep.chunk != b->chunk[i] || (char)x->spec_pending != b->shift[i]) return false;
  }
  return true;
}

// 1: every context is on the particle buffer of the capture; -1: every one on
// the other buffer; 0: mixed
int batch_parity(const pic_batch* b) {
  int same = 0;
  for (size_t i = 0; i < b->ctx.size(); ++i) same += b->ctx[i]->cur == b->cur[i];
  return same == (int)b->ctx.size() ? 1 : same == 0 ? -1 : 0;
}

int batch_capture(pic_batch* b) {
  if (b->exec) {
    // wait for the previous graph's replays on the lead stream before its
    // executable is freed
    if (hipStreamSynchronize(b->lead) != hipSuccess) return PIC_EHIP;
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  // the events are recorded again inside the capture: first let the waits the
  // context streams still hold on their earlier records complete
  for (pic_ctx* x : b->ctx)
    if (hipStreamSynchronize(x->stream) != hipSuccess) return PIC_EHIP;
  const size_t n = b->ctx.size();
  std::vector<HostMirror> saved(n);
  for (size_t i = 0; i < n; ++i) saved[i] = save_mirror(b->ctx[i]);
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(b->lead, hipStreamCaptureModeThreadLocal) != hipSuccess) return PIC_EHIP;
  int rc = hipEventRecord(b->ev_lead, b->lead) == hipSuccess ? PIC_OK : PIC_EHIP;
  for (size_t i = 0; i < n && rc == PIC_OK; ++i) {
    pic_ctx* x = b->ctx[i];
    if (hipStreamWaitEvent(x->stream, b->ev_lead, 0) != hipSuccess) rc = PIC_EHIP;
    if (rc == PIC_OK) rc = pic_step(x, 2);
    if (rc == PIC_OK && (hipEventRecord(b->ev_ctx[i], x->stream) != hipSuccess ||
                         hipStreamWaitEvent(b->lead, b->ev_ctx[i], 0) != hipSuccess))
      rc = PIC_EHIP;
  }
  hipError_t e = hipStreamEndCapture(b->lead, &g);
  for (size_t i = 0; i < n; ++i) restore_mirror(b->ctx[i], saved[i]);
  if (rc != PIC_OK || e != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return rc != PIC_OK ? rc : PIC_EHIP;
  }
  e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    b->exec = nullptr;
    return PIC_EHIP;
  }
  for (size_t i = 0; i < n; ++i) {
    b->bm[i] = b->ctx[i]->gemm_bm;
    b->chunk[i] = b->ctx[i]->dep.chunk;
    b->shift[i] = (char)b->ctx[i]->spec_pending;
    b->cur[i] = b->ctx[i]->cur;
  }
  return PIC_OK;
}

}  // namespace

extern "C" {

int pic_batch_create(pic_ctx* const* ctxs, int n_ctx, pic_batch** out) {
  if (!out) return PIC_EINVAL;
  *out = nullptr;
  if (!ctxs || n_ctx < 1) return PIC_EINVAL;
  for (int c = 0; c < n_ctx; ++c) {
    if (!ctxs[c] || !ctxs[c]->stream) return PIC_EINVAL;
    for (int d = 0; d < c; ++d)
      if (ctxs[d] == ctxs[c]) return PIC_EINVAL;
  }
  pic_batch* b = new pic_batch;
  b->ctx.assign(ctxs, ctxs + n_ctx);
  b->bm.assign(n_ctx, 0);
  b->chunk.assign(n_ctx, 0);
  b->cur.assign(n_ctx, 0);
  b->shift.assign(n_ctx, 0);
  b->ev_ctx.assign(n_ctx, nullptr);
  bool ok = hipStreamCreateWithFlags(&b->lead, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&b->ev_lead, hipEventDisableTiming) == hipSuccess;
  for (int c = 0; c < n_ctx && ok; ++c)
    ok = hipEventCreateWithFlags(&b->ev_ctx[c], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    (void)pic_batch_free(b);
    return PIC_EHIP;
  }
  *out = b;
  return PIC_OK;
}

int pic_batch_run(pic_batch* b, int n) {
  if (!b || n < 0) return PIC_EINVAL;
  for (pic_ctx* x : b->ctx) {
    if (x->phase != 0) return PIC_ESTATE;
    if (x->timing) return PIC_EINVAL;
    for (int m = 0; m < x->M; ++m)
      if (x->src_set[m]) return PIC_ESTATE;
  }
  if (n == 0) return PIC_OK;
  int rc = PIC_OK;
  // one eager step of every context settles any one-time work (as in
  // pic_step_graph); the contexts stay in step with each other
  bool settle = false;
  for (pic_ctx* x : b->ctx) settle = settle || x->steps == 0 || x->eb_stale || !x->rho_carry;
  if (settle) {
    for (pic_ctx* x : b->ctx)
      if ((rc = pic_step(x, 1)) != PIC_OK) return rc;
    --n;
  }
  if (n >= 2) {
    // as in pic_step_graph: the graph reads the particle buffers current at
    // its capture
    const bool params = batch_params(b);
    if (params && batch_parity(b) == -1 && (n & 1)) {
      for (pic_ctx* x : b->ctx)
        if ((rc = pic_step(x, 1)) != PIC_OK) return rc;
      --n;
    }
    if ((!params || batch_parity(b) != 1) && (rc = batch_capture(b)) != PIC_OK) return rc;
    // the replays start after the work already queued on every context's
    // stream, and that stream's later work starts after the replays
    for (size_t i = 0; i < b->ctx.size(); ++i)
      if (hipEventRecord(b->ev_ctx[i], b->ctx[i]->stream) != hipSuccess ||
          hipStreamWaitEvent(b->lead, b->ev_ctx[i], 0) != hipSuccess)
        return PIC_EHIP;
    for (; n >= 2; n -= 2) {
      if (hipGraphLaunch(b->exec, b->lead) != hipSuccess) return PIC_EHIP;
      for (pic_ctx* x : b->ctx) {
        x->steps += 2;
        if (x->cfg.moving_window) x->n_shift += 2;
      }
    }
    if (hipEventRecord(b->ev_lead, b->lead) != hipSuccess) return PIC_EHIP;
    for (pic_ctx* x : b->ctx)
      if (hipStreamWaitEvent(x->stream, b->ev_lead, 0) != hipSuccess) return PIC_EHIP;
  }
  if (n == 1)
    for (pic_ctx* x : b->ctx)
      if ((rc = pic_step(x, 1)) != PIC_OK) return rc;
  return check_launch();
}

int pic_batch_free(pic_batch* b) {
  if (!b) return PIC_EINVAL;
  int rc = PIC_OK;
  if (b->lead && hipStreamSynchronize(b->lead) != hipSuccess) rc = PIC_EHIP;
  // every context's stream holds a wait on the lead event after the replays:
  // let those waits complete before the event and the lead stream they refer
  // to are destroyed
  for (pic_ctx* x : b->ctx)
    if (hipStreamSynchronize(x->stream) != hipSuccess) rc = PIC_EHIP;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->ev_lead) (void)hipEventDestroy(b->ev_lead);
  for (hipEvent_t e : b->ev_ctx)
    if (e) (void)hipEventDestroy(e);
  if (b->lead) (void)hipStreamDestroy(b->lead);
  delete b;
  return rc;
}

int pic_batch_step(pic_ctx* const* ctxs, int n_ctx, int n) {
  if (!ctxs || n_ctx < 0 || n < 0) return PIC_EINVAL;
  if (n_ctx == 0 || n == 0) {
    for (int c = 0; c < n_ctx; ++c)
      if (!ctxs[c]) return PIC_EINVAL;
    return PIC_OK;
  }
  pic_batch* b = nullptr;
  int rc = pic_batch_create(ctxs, n_ctx, &b);
  if (rc) return rc;
  rc = pic_batch_run(b, n);
  const int rc2 = pic_batch_free(b);
  return rc ? rc : rc2;
}

int pic_autotune(pic_ctx* x, int steps_per_trial, pic_tuning* best, double* best_ms) {
  if (!x || steps_per_trial < 2 || !best) return PIC_EINVAL;
  if (!x->stream || x->timing || x->phase != 0) return PIC_EINVAL;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return PIC_EHIP;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return PIC_EHIP;
  }
  pic_tuning cand[12];
  int nc = 0;
  for (int tm : {0, 64, 128, 32})
    for (int ch : {2048, 4096, 8192})
      if (tm == 0 || x->nr % tm == 0) cand[nc++] = pic_tuning{tm, ch};
  int rc = PIC_OK;
  double bms = 1e300;
  pic_tuning bt = cand[0];
  for (int i = 0; i < nc && rc == PIC_OK; ++i) {
    rc = pic_set_tuning(x, &cand[i]);
    if (rc == PIC_OK) rc = graph_steps(x, 2);   // capture with these parameters, untimed
    if (rc != PIC_OK) break;
    (void)hipEventRecord(a, x->stream);
    rc = graph_steps(x, steps_per_trial);
    (void)hipEventRecord(b, x->stream);
    if (rc != PIC_OK) break;
    if (hipEventSynchronize(b) != hipSuccess) {
      rc = PIC_EHIP;
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    if (ms < bms) {
      bms = ms;
      bt = cand[i];
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc == PIC_OK) rc = pic_set_tuning(x, &bt);
  if (rc == PIC_OK) rc = sync(x);
  *best = bt;
  if (best_ms) *best_ms = bms / steps_per_trial;
  return rc;
}

int pic_timing_enable(pic_ctx* x, int enable) {
  if (!x) return PIC_EINVAL;
  int rc = sync(x);
  x->recs.clear();
  x->ev_used = 0;
  x->timing = enable != 0;
  return rc;
}

int pic_timing_read(pic_ctx* x, int timer, double* total_ms, int64_t* launches) {
  if (!x || timer < 0 || timer >= PIC_T_N || !total_ms || !launches) return PIC_EINVAL;
  int rc = sync(x);
  if (rc) return rc;
  double t = 0.0;
  int64_t k = 0;
  for (const auto& r : x->recs) {
    if (r.phase != timer) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return PIC_EHIP;
    t += ms;
    ++k;
  }
  *total_ms = t;
  *launches = k;
  return PIC_OK;
}

int pic_fft_z(void* data, int64_t rows, int nz, int inverse, void* hip_stream) {
  if (!data || rows < 0 || !is_pow2(nz) || nz < 16 || nz > 4096) return PIC_EINVAL;
  if (rows == 0) return PIC_OK;
  launch_fft((float2*)data, (float2*)data, nullptr, nz, rows, inverse != 0, false, nullptr, (hipStream_t)hip_stream);
  return check_launch();
}

int pic_dht_gemm(const void* const* a_t, const void* const* xin, void* const* y, int batch, int n, int ncols, int prec,
                 void* hip_stream) {
  if (!a_t || !xin || !y || batch < 0 || n < 32 || (n % 32) || ncols < 128 || (ncols % 128) || prec < 0 || prec > 2)
    return PIC_EINVAL;
  if (batch == 0) return PIC_OK;
  launch_dht_gemm((const float* const*)a_t, (const float* const*)xin, (float* const*)y, batch, n, ncols, prec, 0,
                  (hipStream_t)hip_stream);
  return check_launch();
}

}  // extern "C"
