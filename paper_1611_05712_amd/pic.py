"""Thin Python binding of libpic.so (argument marshalling only).

Every step of the PIC cycle runs in the HIP library; PyTorch only provides
the device workspace and the stream.  Names mirror the C interface of
include/pic.h.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpic.so")

PIC_OK, PIC_EINVAL, PIC_ENOSPC, PIC_EHIP, PIC_ESTATE, PIC_ENUMERIC = 0, -1, -2, -3, -4, -5
KPERP_J0_ZEROS, KPERP_SINE, KPERP_JM_ZEROS = 0, 1, 2
H_FP32, H_BF16X3, H_FP16X3 = 0, 1, 2
COMP = {"E+": 0, "E-": 1, "Ez": 2, "B+": 3, "B-": 4, "Bz": 5, "J+": 6, "J-": 7, "Jz": 8,
        "rho_old": 9, "rho_new": 10}

EXPORTED = (
    "pic_workspace_bytes", "pic_init", "pic_gather_push", "pic_deposit", "pic_spectral_push",
    "pic_step", "pic_sync", "pic_diagnostics", "pic_get_field", "pic_set_field",
    "pic_num_particles", "pic_get_particles", "pic_get_state", "pic_free", "pic_strerror",
    "pic_fft_z", "pic_dht_gemm", "pic_timing_enable", "pic_timing_read",
    "pic_get_tuning", "pic_set_tuning", "pic_step_graph", "pic_batch_step", "pic_batch_create",
    "pic_batch_run", "pic_batch_free", "pic_autotune",
    "pic_diagnostics_slices", "pic_diagnostics_slices_noalloc",
    "pic_mlp_num_params", "pic_mlp_workspace_bytes", "pic_mlp_init", "pic_mlp_forward", "pic_mlp_loss_grad",
    "pic_mlp_train", "pic_mlp_get_params", "pic_mlp_set_params", "pic_mlp_steps", "pic_mlp_sync", "pic_mlp_free",
)
TIMERS = ("gather_push", "sort", "deposit", "fft_fwd", "dht_fwd", "psatd", "dht_inv", "fft_inv",
          "window", "scan", "dep_plan", "dep_combine", "pack")


class PicError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {_strerror(code)} ({code})")
        self.code = code


class pic_config(ctypes.Structure):
    _fields_ = [("nz", ctypes.c_int32), ("nr", ctypes.c_int32), ("n_modes", ctypes.c_int32),
                ("order", ctypes.c_int32), ("dz", ctypes.c_double), ("dr", ctypes.c_double),
                ("dt", ctypes.c_double), ("z_min", ctypes.c_double),
                ("moving_window", ctypes.c_int32), ("kperp_grid", ctypes.c_int32),
                ("hankel_prec", ctypes.c_int32), ("current_correction", ctypes.c_int32),
                ("filter", ctypes.c_int32), ("damp_cells", ctypes.c_int32), ("galilean", ctypes.c_int32),
                ("shape_order", ctypes.c_int32)]


class pic_tuning(ctypes.Structure):
    _fields_ = [("gemm_tile_m", ctypes.c_int32), ("deposit_chunk", ctypes.c_int32)]


_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)


class pic_species(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("q", ctypes.c_double), ("m", ctypes.c_double),
                ("mobile", ctypes.c_int32), ("inject", ctypes.c_int32),
                ("ppc_z", ctypes.c_int32), ("ppc_r", ctypes.c_int32), ("ppc_t", ctypes.c_int32),
                ("density", ctypes.c_double), ("diag", ctypes.c_int32), ("self_field", ctypes.c_int32),
                ("x", _dp), ("y", _dp), ("z", _dp), ("ux", _fp), ("uy", _fp), ("uz", _fp),
                ("w", _fp)]


class pic_diag_req(ctypes.Structure):
    _fields_ = [("species", ctypes.c_int32), ("slice_len", ctypes.c_double),
                ("n_sigma", ctypes.c_double), ("min_per_slice", ctypes.c_int32)]


class pic_diag_out(ctypes.Structure):
    _fields_ = [("eps_nx", ctypes.c_double), ("eps_ny", ctypes.c_double),
                ("mean_gamma", ctypes.c_double), ("sigma_gamma", ctypes.c_double),
                ("mean_slice_sigma_gamma", ctypes.c_double), ("z_mean", ctypes.c_double),
                ("sigma_z", ctypes.c_double), ("n", ctypes.c_int64),
                ("n_slices", ctypes.c_int32), ("nan_flag", ctypes.c_int32)]


class pic_mlp_config(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int32), ("hidden", ctypes.c_int32), ("n_hidden_layers", ctypes.c_int32),
                ("n_out", ctypes.c_int32), ("prec", ctypes.c_int32), ("max_batch", ctypes.c_int32)]


class pic_adam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libpic.so (torch must be importable: its HIP runtime is shared)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing "
                           "(run python -m paper_1611_05712_amd.build)")
    import torch  # noqa: F401  -- loads the HIP runtime the library links against
    L = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    L.pic_workspace_bytes.argtypes = [ctypes.POINTER(pic_config), ctypes.POINTER(pic_species), i32,
                                      i64, ctypes.POINTER(ctypes.c_size_t)]
    L.pic_init.argtypes = [ctypes.POINTER(pic_config), ctypes.POINTER(pic_species), i32, i64, vp,
                           ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    for name in ("pic_gather_push", "pic_deposit", "pic_spectral_push", "pic_sync", "pic_free"):
        getattr(L, name).argtypes = [vp]
    L.pic_step.argtypes = [vp, i32]
    L.pic_diagnostics.argtypes = [vp, ctypes.POINTER(pic_diag_req), ctypes.POINTER(pic_diag_out)]
    L.pic_diagnostics_slices_noalloc.argtypes = [vp, ctypes.POINTER(pic_diag_req), ctypes.POINTER(pic_diag_out),
                                                 _dp, _dp, i32, ctypes.POINTER(i32)]
    L.pic_diagnostics_slices.argtypes = [vp, ctypes.POINTER(pic_diag_req), ctypes.POINTER(pic_diag_out), _dp, _dp,
                                         i32, ctypes.POINTER(ctypes.c_int32)]
    L.pic_get_field.argtypes = [vp, i32, i32, i32, vp]
    L.pic_set_field.argtypes = [vp, i32, i32, vp]
    L.pic_num_particles.argtypes = [vp, ctypes.POINTER(i64)]
    L.pic_get_particles.argtypes = [vp, i32, i64, _dp, _dp, _fp, ctypes.POINTER(i64)]
    L.pic_get_state.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
    L.pic_strerror.argtypes = [i32]
    L.pic_strerror.restype = ctypes.c_char_p
    L.pic_fft_z.argtypes = [vp, i64, i32, i32, vp]
    L.pic_dht_gemm.argtypes = [vp, vp, vp, i32, i32, i32, i32, vp]
    L.pic_timing_enable.argtypes = [vp, i32]
    L.pic_timing_read.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
    L.pic_get_tuning.argtypes = [vp, ctypes.POINTER(pic_tuning)]
    L.pic_set_tuning.argtypes = [vp, ctypes.POINTER(pic_tuning)]
    L.pic_step_graph.argtypes = [vp, i32]
    L.pic_batch_step.argtypes = [ctypes.POINTER(vp), i32, i32]
    L.pic_batch_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(vp)]
    L.pic_batch_run.argtypes = [vp, i32]
    L.pic_batch_free.argtypes = [vp]
    L.pic_autotune.argtypes = [vp, i32, ctypes.POINTER(pic_tuning), ctypes.POINTER(ctypes.c_double)]
    cfgp = ctypes.POINTER(pic_mlp_config)
    L.pic_mlp_num_params.argtypes = [cfgp, ctypes.POINTER(i64)]
    L.pic_mlp_workspace_bytes.argtypes = [cfgp, ctypes.POINTER(ctypes.c_size_t)]
    L.pic_mlp_init.argtypes = [cfgp, _fp, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.pic_mlp_forward.argtypes = [vp, vp, i32, vp]
    L.pic_mlp_loss_grad.argtypes = [vp, vp, vp, i32, vp, vp]
    L.pic_mlp_train.argtypes = [vp, vp, vp, i32, vp, i32, i32, ctypes.POINTER(pic_adam), vp]
    L.pic_mlp_get_params.argtypes = [vp, _fp]
    L.pic_mlp_set_params.argtypes = [vp, _fp]
    L.pic_mlp_steps.argtypes = [vp, ctypes.POINTER(i64)]
    L.pic_mlp_sync.argtypes = [vp]
    L.pic_mlp_free.argtypes = [vp]
    for name in EXPORTED:
        if name != "pic_strerror":
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _strerror(code: int) -> str:
    try:
        return load().pic_strerror(code).decode()
    except Exception:
        return "error"


def _check(code: int, what: str):
    if code != PIC_OK:
        raise PicError(code, what)


def _stream_handle(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


# ---------------------------------------------------------------------------
class Simulation:
    """One quasi-cylindrical order-p PSATD PIC context on one GPU.

    `species` is a sequence of objects with the attributes of
    workloads.Species (name, q, m, mobile, x, y, z, ux, uy, uz, w, inject, ppc,
    density, diag)."""

    def __init__(self, nz, nr, n_modes, order, dz, dr, dt, z_min, species: Sequence,
                 moving_window=False, kperp_grid=KPERP_JM_ZEROS, hankel_prec=H_FP32,
                 current_correction=True, max_particles=0, device="cuda:0", stream=None, filter=0,
                 damp_cells=0, galilean=False, shape_order=1):
        import torch
        L = load()
        self._L = L
        self.device = torch.device(device)
        self.cfg = pic_config(nz, nr, n_modes, order, dz, dr, dt, z_min, int(bool(moving_window)),
                              kperp_grid, hankel_prec, int(bool(current_correction)), int(filter),
                              int(damp_cells), int(bool(galilean)), int(shape_order))
        self.nz, self.nr, self.n_modes = nz, nr, n_modes
        self.species_names = [s.name for s in species]
        self._keep = []
        arr = (pic_species * max(1, len(species)))()
        for k, s in enumerate(species):
            x = np.ascontiguousarray(s.x, np.float64)
            y = np.ascontiguousarray(s.y, np.float64)
            z = np.ascontiguousarray(s.z, np.float64)
            ux = np.ascontiguousarray(s.ux, np.float32)
            uy = np.ascontiguousarray(s.uy, np.float32)
            uz = np.ascontiguousarray(s.uz, np.float32)
            w = np.ascontiguousarray(s.w, np.float32)
            self._keep += [x, y, z, ux, uy, uz, w]
            ppc = tuple(getattr(s, "ppc", (1, 1, 1)))
            arr[k] = pic_species(
                x.shape[0], s.q, s.m, int(bool(s.mobile)), int(bool(getattr(s, "inject", False))),
                ppc[0], ppc[1], ppc[2], float(getattr(s, "density", 1.0)),
                int(bool(getattr(s, "diag", False))), int(bool(getattr(s, "self_field", False))),
                x.ctypes.data_as(_dp), y.ctypes.data_as(_dp), z.ctypes.data_as(_dp),
                ux.ctypes.data_as(_fp), uy.ctypes.data_as(_fp), uz.ctypes.data_as(_fp),
                w.ctypes.data_as(_fp))
        nbytes = ctypes.c_size_t()
        _check(L.pic_workspace_bytes(ctypes.byref(self.cfg), arr, len(species), max_particles,
                                     ctypes.byref(nbytes)), "pic_workspace_bytes")
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        # a stream of its own (default priority): graph capture needs a
        # non-null stream, and contexts of a batch overlap on separate streams
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self.workspace.record_stream(self.stream)
        ctx = ctypes.c_void_p()
        _check(L.pic_init(ctypes.byref(self.cfg), arr, len(species), max_particles,
                          ctypes.c_void_p(self.workspace.data_ptr()), nbytes.value,
                          ctypes.c_void_p(_stream_handle(self.stream)), ctypes.byref(ctx)),
               "pic_init")
        self._ctx = ctx
        self._keep = []   # host inputs are copied by pic_init

    @classmethod
    def from_workload(cls, wl, **kw):
        kw.setdefault("filter", getattr(wl, "filter", 0))
        kw.setdefault("damp_cells", getattr(wl, "damp_cells", 0))
        kw.setdefault("galilean", getattr(wl, "galilean", False))
        kw.setdefault("shape_order", getattr(wl, "shape_order", 1))
        return cls(wl.nz, wl.nr, wl.n_modes, wl.order, wl.dz, wl.dr, wl.dt, wl.zmin, wl.species,
                   moving_window=wl.moving_window, kperp_grid=wl.kperp_grid, **kw)

    # -- cycle -------------------------------------------------------------
    def gather_push(self):
        _check(self._L.pic_gather_push(self._ctx), "pic_gather_push")

    def deposit(self):
        _check(self._L.pic_deposit(self._ctx), "pic_deposit")

    def spectral_push(self):
        _check(self._L.pic_spectral_push(self._ctx), "pic_spectral_push")

    def step(self, n: int = 1):
        _check(self._L.pic_step(self._ctx, int(n)), "pic_step")

    def step_graph(self, n: int = 1):
        _check(self._L.pic_step_graph(self._ctx, int(n)), "pic_step_graph")

    def tuning(self) -> dict:
        t = pic_tuning()
        _check(self._L.pic_get_tuning(self._ctx, ctypes.byref(t)), "pic_get_tuning")
        return {"gemm_tile_m": t.gemm_tile_m, "deposit_chunk": t.deposit_chunk}

    def set_tuning(self, gemm_tile_m: int, deposit_chunk: int):
        t = pic_tuning(int(gemm_tile_m), int(deposit_chunk))
        _check(self._L.pic_set_tuning(self._ctx, ctypes.byref(t)), "pic_set_tuning")

    def autotune(self, steps_per_trial: int = 4):
        t = pic_tuning()
        ms = ctypes.c_double()
        _check(self._L.pic_autotune(self._ctx, int(steps_per_trial), ctypes.byref(t), ctypes.byref(ms)),
               "pic_autotune")
        return {"gemm_tile_m": t.gemm_tile_m, "deposit_chunk": t.deposit_chunk, "ms_per_step": ms.value}

    def sync(self):
        _check(self._L.pic_sync(self._ctx), "pic_sync")

    # -- access ------------------------------------------------------------
    def get_field(self, mode: int, comp, spectral: bool = False) -> np.ndarray:
        c = COMP[comp] if isinstance(comp, str) else int(comp)
        out = np.empty((self.nr, self.nz), np.complex64)
        _check(self._L.pic_get_field(self._ctx, mode, c, int(bool(spectral)),
                                     out.ctypes.data_as(ctypes.c_void_p)), "pic_get_field")
        return out

    def set_field(self, mode: int, comp, values: np.ndarray):
        c = COMP[comp] if isinstance(comp, str) else int(comp)
        v = np.ascontiguousarray(values, np.complex64)
        assert v.shape == (self.nr, self.nz)
        _check(self._L.pic_set_field(self._ctx, mode, c, v.ctypes.data_as(ctypes.c_void_p)),
               "pic_set_field")

    def num_particles(self) -> int:
        n = ctypes.c_int64()
        _check(self._L.pic_num_particles(self._ctx, ctypes.byref(n)), "pic_num_particles")
        return n.value

    def get_particles(self, species, cap: Optional[int] = None):
        k = self.species_names.index(species) if isinstance(species, str) else int(species)
        if cap is None:
            cap = self.num_particles()
        xyz = np.empty((cap, 3), np.float64)
        uvw = np.empty((cap, 3), np.float64)
        w = np.empty(cap, np.float32)
        n = ctypes.c_int64()
        _check(self._L.pic_get_particles(self._ctx, k, cap, xyz.ctypes.data_as(_dp),
                                         uvw.ctypes.data_as(_dp), w.ctypes.data_as(_fp),
                                         ctypes.byref(n)), "pic_get_particles")
        m = n.value
        return {"x": xyz[:m, 0], "y": xyz[:m, 1], "z": xyz[:m, 2], "ux": uvw[:m, 0],
                "uy": uvw[:m, 1], "uz": uvw[:m, 2], "w": w[:m]}

    def state(self):
        z = ctypes.c_double()
        s = ctypes.c_int64()
        _check(self._L.pic_get_state(self._ctx, ctypes.byref(z), ctypes.byref(s)), "pic_get_state")
        return z.value, s.value

    def diagnostics(self, species, slice_len: float, n_sigma: float = 3.0, min_per_slice: int = 10,
                    allow_nan: bool = False) -> dict:
        k = self.species_names.index(species) if isinstance(species, str) else int(species)
        req = pic_diag_req(k, slice_len, n_sigma, min_per_slice)
        out = pic_diag_out()
        rc = self._L.pic_diagnostics(self._ctx, ctypes.byref(req), ctypes.byref(out))
        if not (rc == PIC_OK or (allow_nan and rc == PIC_ENUMERIC)):
            _check(rc, "pic_diagnostics")
        return {f: getattr(out, f) for f, _ in pic_diag_out._fields_}

    def diagnostics_slices(self, species, slice_len: float, n_sigma: float = 3.0, min_per_slice: int = 10,
                           allow_nan: bool = False, noalloc: bool = False):
        """pic_diagnostics plus per-slice rms gamma and counts: returns
        (moments dict, sigma_gamma[n], count[n]); slice k covers
        xi in [(k - n/2) L, (k - n/2 + 1) L).  noalloc=True calls
        pic_diagnostics_slices_noalloc (static device scratch, at most 4096
        slices)."""
        name = "pic_diagnostics_slices_noalloc" if noalloc else "pic_diagnostics_slices"
        fn = getattr(self._L, name)
        k = self.species_names.index(species) if isinstance(species, str) else int(species)
        req = pic_diag_req(k, slice_len, n_sigma, min_per_slice)
        out = pic_diag_out()
        n = ctypes.c_int32()
        rc = fn(self._ctx, ctypes.byref(req), ctypes.byref(out), None, None, 0, ctypes.byref(n))
        if not (rc == PIC_OK or (allow_nan and rc == PIC_ENUMERIC)):
            _check(rc, name)
        sg = np.zeros(max(n.value, 1))
        cnt = np.zeros(max(n.value, 1))
        rc = fn(self._ctx, ctypes.byref(req), ctypes.byref(out), sg.ctypes.data_as(_dp), cnt.ctypes.data_as(_dp),
                n.value, ctypes.byref(n))
        if not (rc == PIC_OK or (allow_nan and rc == PIC_ENUMERIC)):
            _check(rc, name)
        return {f: getattr(out, f) for f, _ in pic_diag_out._fields_}, sg[:n.value], cnt[:n.value]

    def timing_enable(self, on: bool = True):
        _check(self._L.pic_timing_enable(self._ctx, int(bool(on))), "pic_timing_enable")

    def timing_read(self) -> dict:
        """{phase: (total_ms, launches)} since timing_enable."""
        out = {}
        for k, name in enumerate(TIMERS):
            t = ctypes.c_double()
            n = ctypes.c_int64()
            _check(self._L.pic_timing_read(self._ctx, k, ctypes.byref(t), ctypes.byref(n)),
                   "pic_timing_read")
            out[name] = (t.value, n.value)
        return out

    def close(self):
        if getattr(self, "_ctx", None):
            ctx, self._ctx = self._ctx, None
            _check(self._L.pic_free(ctx), "pic_free")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# kernel-level entry points
# ---------------------------------------------------------------------------
def batch_step(sims: Sequence["Simulation"], n: int):
    """n steps of every simulation as replays of one graph that holds two
    steps of all of them (pic_batch_step); returns once they are done."""
    if not sims:
        return
    L = load()
    arr = (ctypes.c_void_p * len(sims))(*[s._ctx for s in sims])
    _check(L.pic_batch_step(arr, len(sims), int(n)), "pic_batch_step")


class Batch:
    """Independent simulations advanced together by one captured graph
    (pic_batch_create / pic_batch_run / pic_batch_free); the simulations must
    stay open while the batch is."""

    def __init__(self, sims: Sequence["Simulation"]):
        self._L = load()
        self.sims = list(sims)
        arr = (ctypes.c_void_p * len(self.sims))(*[s._ctx for s in self.sims])
        h = ctypes.c_void_p()
        _check(self._L.pic_batch_create(arr, len(self.sims), ctypes.byref(h)), "pic_batch_create")
        self._h = h

    def run(self, n: int):
        """n steps of every simulation (asynchronous)."""
        _check(self._L.pic_batch_run(self._h, int(n)), "pic_batch_run")

    def close(self):
        if self._h:
            h, self._h = self._h, None
            _check(self._L.pic_batch_free(h), "pic_batch_free")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fft_z(t, inverse: bool = False, stream=None):
    """In-place batched FFT along the last axis of a complex64 CUDA tensor."""
    import torch
    assert t.dtype == torch.complex64 and t.is_cuda and t.is_contiguous()
    nz = t.shape[-1]
    rows = t.numel() // nz
    _check(load().pic_fft_z(ctypes.c_void_p(t.data_ptr()), rows, nz, int(bool(inverse)),
                            ctypes.c_void_p(_stream_handle(stream))), "pic_fft_z")
    return t


def dht_gemm(a_t: Sequence, x: Sequence, y: Sequence, prec: int = H_FP32, stream=None):
    """Batched Y_b = A_b X_b on the matrix cores.  a_t[b]: float32 (n, n) CUDA tensor
    holding A_b transposed; x[b], y[b]: float32 (n, ncols) CUDA tensors."""
    import torch
    b = len(a_t)
    n, ncols = x[0].shape
    dev = x[0].device
    ptrs = torch.tensor([[t.data_ptr() for t in a_t], [t.data_ptr() for t in x],
                         [t.data_ptr() for t in y]], dtype=torch.int64, device=dev)
    _check(load().pic_dht_gemm(ctypes.c_void_p(ptrs[0].data_ptr()), ctypes.c_void_p(ptrs[1].data_ptr()),
                               ctypes.c_void_p(ptrs[2].data_ptr()), b, n, ncols, prec,
                               ctypes.c_void_p(_stream_handle(stream))), "pic_dht_gemm")
    return y
