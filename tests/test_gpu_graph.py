"""Graph replay, batches and tunables: the same cycle as eager stepping, to
rounding (LDS and global atomics make the summation order vary)."""
import numpy as np
import pytest

from workloads import preset

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

COMPS = ["E+", "E-", "Ez", "B+", "B-", "Bz"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _sim(wl, **kw):
    from paper_1611_05712_amd import Simulation
    return Simulation.from_workload(wl, **kw)


def _field_rel(a, b, modes=2):
    worst = 0.0
    for m in range(modes):
        for off in (0, 3):
            ga = np.stack([a.get_field(m, COMPS[off + c]) for c in range(3)])
            gb = np.stack([b.get_field(m, COMPS[off + c]) for c in range(3)])
            worst = max(worst, np.linalg.norm(ga - gb) / max(np.linalg.norm(gb), 1e-30))
    return worst


def _moments_close(a, b, name, rel=1e-6):
    da = a.diagnostics(name, slice_len=0.02975)
    db = b.diagnostics(name, slice_len=0.02975)
    for k in ("z_mean", "sigma_z", "mean_gamma", "eps_nx", "eps_ny", "sigma_gamma"):
        assert da[k] == pytest.approx(db[k], rel=rel, abs=1e-12), k


@pytest.mark.parametrize("n", [1, 2, 7])
def test_graph_steps_match_eager(n):
    wl = preset("small")
    a, b = _sim(wl), _sim(wl)
    a.step(n)
    b.step_graph(n)
    assert a.state() == b.state()
    assert a.num_particles() == b.num_particles()
    assert _field_rel(b, a) < 1e-5
    _moments_close(b, a, "drive")


@pytest.mark.parametrize("calls", [(3, 3, 4), (4, 3, 2, 5), (1, 2, 2, 3, 2)])
def test_graph_steps_across_calls_of_any_length(calls):
    """Graph stepping split into calls of odd and even length (the replays
    must start from the particle buffer they were captured with; the
    workload injects plasma at every window move, so a replay from the other
    buffer would lose a column): the same as eager steps."""
    wl = preset("small")
    a, b = _sim(wl), _sim(wl)
    a.step(sum(calls))
    for n in calls:
        b.step_graph(n)
    assert a.state() == b.state()
    assert a.num_particles() == b.num_particles()
    assert _field_rel(b, a) < 1e-5
    _moments_close(b, a, "drive")


@pytest.mark.parametrize("modes", [1, 3])
def test_graph_steps_match_eager_other_mode_counts(modes):
    import dataclasses
    wl = dataclasses.replace(preset("small"), n_modes=modes)
    a, b = _sim(wl), _sim(wl)
    a.step(3)
    b.step_graph(3)
    assert a.state() == b.state()
    assert a.num_particles() == b.num_particles()
    assert _field_rel(b, a, modes) < 1e-5
    _moments_close(b, a, "drive")


def test_graph_recaptures_after_tuning_change():
    wl = preset("small")
    a, b = _sim(wl), _sim(wl)
    a.step(6)
    b.step_graph(2)
    b.set_tuning(32, 2048)
    b.step_graph(2)
    b.set_tuning(32, 8192)
    b.step_graph(2)
    assert b.tuning() == {"gemm_tile_m": 32, "deposit_chunk": 8192}
    assert _field_rel(b, a) < 1e-5
    _moments_close(b, a, "drive")


def test_set_tuning_rejects_unsupported_values():
    from paper_1611_05712_amd import PicError
    sim = _sim(preset("tiny"))
    for tm, ch in ((48, 4096), (64, 3000), (32, 0)):
        with pytest.raises(PicError):
            sim.set_tuning(tm, ch)


def test_batch_matches_individual_runs():
    from paper_1611_05712_amd import batch_step
    wls = [preset("small"), preset("tiny"), preset("small", seed=3)]
    wls[2].order = 0                       # infinite order beside finite ones
    batch = [_sim(w) for w in wls]
    solo = [_sim(w) for w in wls]
    batch_step(batch, 5)
    for s in solo:
        s.step(5)
    for bs, ss, w in zip(batch, solo, wls):
        assert bs.state() == ss.state()
        assert _field_rel(bs, ss) < 1e-5
        name = "drive" if w.name != "tiny" else "bunch"
        _moments_close(bs, ss, name)


def test_batch_graph_over_several_runs_and_a_tuning_change():
    """One graph for three instances (two grids, a finite and the infinite
    order): runs of 4, then 3 (an odd step runs eagerly), a tuning change of
    one instance (the graph is captured again), then 2 more; every instance
    matches its own eager run."""
    from paper_1611_05712_amd import Batch
    wls = [preset("small"), preset("tiny"), preset("small", seed=3)]
    wls[2].order = 0
    sims = [_sim(w) for w in wls]
    solo = [_sim(w) for w in wls]
    b = Batch(sims)
    b.run(4)
    b.run(3)
    sims[0].set_tuning(32, 2048)
    b.run(2)
    b.close()
    for s in solo:
        s.step(9)
    for bs, ss, w in zip(sims, solo, wls):
        assert bs.state() == ss.state()
        assert _field_rel(bs, ss) < 1e-5
        name = "drive" if w.name != "tiny" else "bunch"
        _moments_close(bs, ss, name)


def test_batch_rejects_bad_contexts():
    from paper_1611_05712_amd import Batch, PicError
    s = _sim(preset("tiny"))
    with pytest.raises(PicError):
        Batch([s, s])
    with pytest.raises(PicError):
        Batch([])


def test_autotune_picks_a_supported_pair_and_keeps_results():
    wl = preset("small")
    a, b = _sim(wl), _sim(wl)
    best = b.autotune(steps_per_trial=2)
    assert best["gemm_tile_m"] in (0, 32, 64, 128) and best["deposit_chunk"] in (2048, 4096, 8192)
    assert best["ms_per_step"] > 0
    _, steps = b.state()
    a.step(steps)
    assert _field_rel(b, a) < 1e-5
    _moments_close(b, a, "drive")
