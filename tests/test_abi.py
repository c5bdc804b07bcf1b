"""CPU-side checks of the C interface: every declared symbol is exported by the
built library, and argument validation returns the documented codes without
touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1611_05712_amd import pic
from workloads import preset

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(pic_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pic.LIB_PATH):
        pytest.fail("libpic.so is not built (run python -m paper_1611_05712_amd.build)")
    return pic.load()


def test_header_declares_and_library_exports_every_entry_point(lib):
    names = _declared()
    assert "pic_init" in names and "pic_spectral_push" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(pic.EXPORTED)


def _cfg(**kw):
    base = dict(nz=64, nr=32, n_modes=2, order=8, dz=0.1, dr=0.1, dt=0.1, z_min=0.0,
                moving_window=1, kperp_grid=0, hankel_prec=0, current_correction=1)
    base.update(kw)
    return pic.pic_config(**base)


def _bytes(lib, cfg, species=None, n=0):
    out = ctypes.c_size_t()
    rc = lib.pic_workspace_bytes(ctypes.byref(cfg), species, n, 0, ctypes.byref(out))
    return rc, out.value


def test_workspace_bytes_valid_and_scaling(lib):
    rc, b1 = _bytes(lib, _cfg())
    assert rc == pic.PIC_OK and b1 > 0
    rc, b2 = _bytes(lib, _cfg(nz=128))
    assert rc == pic.PIC_OK and b2 > b1


@pytest.mark.parametrize("bad", [
    dict(nz=100), dict(nz=32), dict(nz=8192), dict(nr=48), dict(nr=16), dict(n_modes=0),
    dict(n_modes=5), dict(order=3), dict(order=-2), dict(dz=0.0), dict(dt=-1.0),
    dict(dt=0.05), dict(kperp_grid=7), dict(hankel_prec=3), dict(dr=float("nan")), dict(filter=5),
])
def test_invalid_configs_rejected(lib, bad):
    rc, _ = _bytes(lib, _cfg(**bad))
    assert rc == pic.PIC_EINVAL


def test_invalid_species_rejected(lib):
    arr = (pic.pic_species * 1)()
    arr[0] = pic.pic_species(10, 0.0, 1.0, 1, 0, 1, 1, 1, 1.0, 0, 0, None, None, None, None, None,
                             None, None)
    rc, _ = _bytes(lib, _cfg(), arr, 1)
    assert rc == pic.PIC_EINVAL           # zero charge
    arr[0].q = -1.0
    rc, _ = _bytes(lib, _cfg(), arr, 1)
    assert rc == pic.PIC_EINVAL           # null position arrays with n > 0
    arr[0].n = 0
    rc, _ = _bytes(lib, _cfg(), arr, 1)
    assert rc == pic.PIC_OK


def test_null_arguments(lib):
    cfg = _cfg()
    ctx = ctypes.c_void_p()
    assert lib.pic_init(ctypes.byref(cfg), None, 0, 0, None, 0, None, ctypes.byref(ctx)) == pic.PIC_EINVAL
    assert lib.pic_workspace_bytes(ctypes.byref(cfg), None, 0, 0, None) == pic.PIC_EINVAL
    for name in ("pic_gather_push", "pic_deposit", "pic_spectral_push", "pic_sync", "pic_free"):
        assert getattr(lib, name)(None) == pic.PIC_EINVAL
    assert lib.pic_step(None, 1) == pic.PIC_EINVAL
    assert lib.pic_fft_z(None, 1, 64, 0, None) == pic.PIC_EINVAL
    assert lib.pic_fft_z(ctypes.c_void_p(8), 1, 48, 0, None) == pic.PIC_EINVAL
    assert lib.pic_dht_gemm(None, None, None, 1, 64, 128, 0, None) == pic.PIC_EINVAL


def _mlp_cfg(**kw):
    base = dict(n_in=5, hidden=128, n_hidden_layers=4, n_out=2, prec=1, max_batch=256)
    base.update(kw)
    return pic.pic_mlp_config(**base)


def test_mlp_sizes_and_validation(lib):
    n = ctypes.c_int64()
    assert lib.pic_mlp_num_params(ctypes.byref(_mlp_cfg()), ctypes.byref(n)) == pic.PIC_OK
    assert n.value == 5 * 128 + 128 + 3 * (128 * 128 + 128) + 128 * 2 + 2
    b = ctypes.c_size_t()
    assert lib.pic_mlp_workspace_bytes(ctypes.byref(_mlp_cfg()), ctypes.byref(b)) == pic.PIC_OK
    assert b.value > 4 * 4 * n.value
    for bad in (dict(n_in=0), dict(hidden=2000), dict(n_hidden_layers=0), dict(n_out=65), dict(prec=2),
                dict(max_batch=0)):
        assert lib.pic_mlp_workspace_bytes(ctypes.byref(_mlp_cfg(**bad)), ctypes.byref(b)) == pic.PIC_EINVAL
    ctx = ctypes.c_void_p()
    assert lib.pic_mlp_init(ctypes.byref(_mlp_cfg()), None, None, 0, None, ctypes.byref(ctx)) == pic.PIC_EINVAL
    for name in ("pic_mlp_sync", "pic_mlp_free"):
        assert getattr(lib, name)(None) == pic.PIC_EINVAL
    assert lib.pic_mlp_forward(None, None, 1, None) == pic.PIC_EINVAL


def test_strerror_covers_codes(lib):
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.pic_strerror(code).decode() != "unknown status"
    assert lib.pic_strerror(-99).decode() == "unknown status"


def test_workload_presets_fit_the_interface(lib):
    for name in ("tiny", "small", "c0"):
        wl = preset(name)
        arr = (pic.pic_species * len(wl.species))()
        keep = []
        for k, s in enumerate(wl.species):
            a = [np.ascontiguousarray(getattr(s, f)) for f in ("x", "y", "z", "ux", "uy", "uz", "w")]
            keep += a
            arr[k] = pic.pic_species(s.n, s.q, s.m, int(s.mobile), int(s.inject), *s.ppc, s.density,
                                     int(s.diag), int(s.self_field), *[v.ctypes.data_as(pic._dp) for v in a[:3]],
                                     *[v.ctypes.data_as(pic._fp) for v in a[3:]])
        cfg = _cfg(nz=wl.nz, nr=wl.nr, order=wl.order, dz=wl.dz, dr=wl.dr, dt=wl.dt, z_min=wl.zmin,
                   moving_window=int(wl.moving_window))
        rc, b = _bytes(lib, cfg, arr, len(wl.species))
        assert rc == pic.PIC_OK and b > 0
