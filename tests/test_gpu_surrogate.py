"""The learned extension end to end: the order surrogate is trained on the
GPU (the library's forward, backward and Adam kernels) on the finite-order
error scan, and on held-out physical set-ups it is compared with the method
without it, the full order scan, which needs every order and the
infinite-order twin to find the lowest acceptable order."""
import os

import numpy as np
import pytest

from workloads import mlp_layer_sizes, mlp_init, minibatch_indices

pytestmark = pytest.mark.gpu

DATA = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1611_05712_amd",
                    "data", "ncr_scan_s1_t288.json")


def _split(scan):
    """Held-out physical set-ups: every fifth; the rest train (a quarter of them
    only as the early-stopping validation set)."""
    ids = sorted(t["tuple"] for t in scan["tuples"])
    held = set(ids[::5])
    return [i for i in ids if i not in held], sorted(held)


@pytest.fixture(scope="module")
def trained():
    from paper_1611_05712_amd import surrogate as S
    scan = S.load_scan(DATA)
    train_ids, held_ids = _split(scan)
    val_ids = train_ids[::4]
    fit_ids = [i for i in train_ids if i not in val_ids]
    X, T, _ = S.dataset(scan, fit_ids)
    Xval, Tval, _ = S.dataset(scan, val_ids)
    sur = S.OrderSurrogate(mlp_init(mlp_layer_sizes(), seed=0))
    idx = minibatch_indices(len(X), 256, S.MAX_STEPS, seed=1)
    losses, hist, best = sur.fit_early_stopping(X, T, Xval, Tval, idx)
    print(f"early stopping: best validation MSE {min(h[1] for h in hist):.4f} at step {best} of {S.MAX_STEPS}")
    yield S, scan, fit_ids, held_ids, sur, losses
    sur.close()


def test_training_converges(trained):
    S, scan, train_ids, held_ids, sur, losses = trained
    assert np.isfinite(losses).all()
    assert losses[-100:].mean() < 0.3 * losses[:20].mean()


def test_held_out_error_beats_the_data_mean(trained):
    # what the network knows beyond the average error of the scan: held-out
    # mean squared error of log10 |Err| against predicting the training mean
    S, scan, train_ids, held_ids, sur, _ = trained
    X, T, _ = S.dataset(scan, train_ids)
    Xv, Tv, _ = S.dataset(scan, held_ids)
    pred = sur.predict(Xv)
    mse_net = float(((pred - Tv) ** 2).mean())
    mse_mean = float(((Tv - T.mean(axis=0)) ** 2).mean())
    print(f"held-out MSE of log10|Err|: network {mse_net:.4f}, training mean {mse_mean:.4f}")
    assert mse_net < 0.8 * mse_mean


def test_order_choice_beats_the_methods_without_the_network(trained):
    # per held-out set-up the order is settled by the plain simulation (the
    # referee) starting from a pick and climbing one order at a time until the
    # errors pass; cost = the infinite-order twin (or, for a pick of infinity,
    # the production run itself) + every finite order simulated.  Against the
    # methods that use no network:
    #   the full scan          every order + twin: always exact, most runs;
    #   climb from p = 8       always exact (the lowest passing order), but
    #                          climbs through every rejected order;
    #   always infinity        one run, exact only where infinity is needed;
    #   majority order         the training set's most frequent answer.
    # The network must be more often exact than both constant pickers and
    # cheaper than both exact methods.
    S, scan, train_ids, held_ids, sur, _ = trained
    major = S.majority_order(scan, train_ids)
    res = S.compare_pickers(scan, held_ids, {
        "network": lambda t: sur.choose_order(S.tuple_params(t)),
        "infinite": lambda t: 0,
        "majority": lambda t: major,
        "climb": lambda t: S.ORDERS[0]})
    n = len(held_ids)
    for name, r in res.items():
        print(f"{name:9s} runs {r['runs']:4d}  exact {r['exact']:3d}/{n}  higher {r['over']:3d}")
    net = res["network"]
    assert net["exact"] > res["infinite"]["exact"]
    assert net["exact"] > res["majority"]["exact"]
    assert net["runs"] < res["climb"]["runs"]
    assert net["runs"] <= 0.5 * res["scan"]["runs"]
    # the referee keeps every accepted order within the threshold: never below the scan's answer
    assert net["exact"] + net["over"] == n


def test_plain_simulation_referees_a_held_out_pick(trained):
    # the referee itself, live: the surrogate's order for one held-out set-up is
    # run through the plain simulation against its infinite-order twin, and the
    # measured errors agree with the scan's record of the same runs
    from workloads import scan_instances
    S, scan, train_ids, held_ids, sur, _ = trained
    rec = {t["tuple"]: t for t in scan["tuples"]}[held_ids[0]]
    insts = [i for i in scan_instances(n_tuples=len(scan["tuples"]), seed=scan["seed"], extra=0)
             if i.tuple_index == rec["tuple"]]
    pick = sur.choose_order(S.tuple_params(rec)) or S.ORDERS[-1]
    referee = S.PlainReferee({i.order: i for i in insts}, scan["steps"])
    es, ee = referee(pick)
    want = rec["errors"][str(pick)]
    assert es == pytest.approx(want["err_sigma_gamma"], rel=0.05, abs=2e-3)
    assert ee == pytest.approx(want["err_eps"], rel=0.05, abs=2e-3)
    assert referee.runs == 2
