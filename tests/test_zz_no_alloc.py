"""pic_diagnostics_slices_noalloc (static device scratch, no allocation)
against pic_diagnostics_slices (workspace scratch) through the C interface:
two calls in a row, the second on a smaller input, plus the slice limit."""
import ctypes

import numpy as np
import pytest

from workloads import preset

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SLICE = 0.02975   # 0.5 um at n0 = 1e23 m^-3
KEYS = ("eps_nx", "eps_ny", "mean_gamma", "sigma_gamma", "mean_slice_sigma_gamma", "z_mean", "sigma_z")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _compare(sim, species, slice_len):
    ref, sg_ref, cnt_ref = sim.diagnostics_slices(species, slice_len)
    got, sg, cnt = sim.diagnostics_slices(species, slice_len, noalloc=True)
    assert got["n"] == ref["n"] and got["n_slices"] == ref["n_slices"] and got["nan_flag"] == 0
    for k in KEYS:
        # moments: same kernels and block partials; slice sums are FP64 atomics
        # whose order may differ between calls
        assert got[k] == pytest.approx(ref[k], rel=1e-9, abs=1e-300), k
    assert sg.size == sg_ref.size and sg.size > 2
    np.testing.assert_array_equal(cnt, cnt_ref)
    np.testing.assert_allclose(sg, sg_ref, rtol=1e-9, atol=0)
    return sg.size


def test_noalloc_diagnostics_match_the_workspace_ones_on_two_calls():
    from paper_1611_05712_amd import Simulation
    big = Simulation.from_workload(preset("small"))
    big.step(3)
    n1 = _compare(big, "drive", SLICE)
    # second call: a smaller input (a 64-particle bunch, fewer slices) on
    # another context of the same GPU, after the larger call filled more of
    # the shared array
    small = Simulation.from_workload(preset("tiny"))
    small.step(2)
    n2 = _compare(small, "bunch", 0.1)
    assert n2 < n1
    # and back on the first context with a coarser slicing
    _compare(big, "drive", 4 * SLICE)
    small.close()
    big.close()


def test_noalloc_diagnostics_reject_more_than_4096_slices():
    from paper_1611_05712_amd import Simulation, pic
    sim = Simulation.from_workload(preset("tiny"))
    k = sim.species_names.index("bunch")
    ref = sim.diagnostics("bunch", 0.1)
    req = pic.pic_diag_req(k, ref["sigma_z"] * 3.0 / 2500.0, 3.0, 10)   # 5000 slices
    out = pic.pic_diag_out()
    n = ctypes.c_int32()
    rc = sim._L.pic_diagnostics_slices_noalloc(sim._ctx, ctypes.byref(req), ctypes.byref(out), None, None, 0,
                                               ctypes.byref(n))
    assert rc == pic.PIC_ENOSPC
    assert n.value > 4096
    assert out.n == ref["n"] and out.sigma_z == pytest.approx(ref["sigma_z"], rel=1e-12)
    sim.close()
