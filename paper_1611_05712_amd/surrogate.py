"""Order surrogate: a small network that predicts the finite-order error of a
run and picks the lowest acceptable stencil order.

The paper judges an order p by the witness errors against the infinite-order
twin, Err_sigma_gamma (Eq. (11)) and Err_eps (Eq. (12)), and reads off the
lowest order with both below 0.05 (Sec. "Accurate modeling of plasma
accelerators in finite order PSATD" and its parameter-scan figure).  Finding
that order by simulation means running the whole order scan.  Here a GELU
MLP (5 -> 4 x 128 -> 2, trained on the GPU by the library's own forward,
backward and Adam kernels) maps (2/p, k_p dz, k_p dr, gamma, witness charge)
to the two errors; the order it picks is then checked by the plain
simulation, which stays the referee: when the measured errors miss the
threshold the next order up is run, so the answer is never worse than the
scan's, only cheaper.
"""
from __future__ import annotations

import json
import math
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

from .mlp import MLP, MLP_BF16

ORDERS = (8, 16, 24, 32, 48, 64)     # finite orders of the scan; 0 = infinite
THRESHOLD = 0.05                     # the paper's accuracy criterion
TARGET_FLOOR = 1e-3                  # targets are log10(|Err| + floor)
MAX_STEPS = 1200                     # Adam steps of batch 256 (early stopping)
CHECK_EVERY = 25
LEARNING_RATE = 3e-4


def features(order: int, dz: float, dr: float, gamma: float, charge_pC: float) -> np.ndarray:
    """Network input: (2/p, k_p dz, k_p dr, ln gamma, charge) mapped affinely
    onto about [-1, 1] over the scan's ranges (2/p in [0, 1/4], k_p dz in
    [0.01, 0.05], k_p dr in [0.03, 0.08], gamma in [500, 4000], charge in
    [10, 100] pC)."""
    inv = 0.0 if order == 0 else 2.0 / order
    return np.array([inv / 0.125 - 1.0, (dz - 0.03) / 0.02, (dr - 0.055) / 0.025,
                     (math.log(gamma) - 7.2544) / 1.0397, (charge_pC - 55.0) / 45.0], dtype=np.float32)


def targets(err_sigma_gamma: float, err_eps: float) -> np.ndarray:
    return np.log10(np.abs([err_sigma_gamma, err_eps]) + TARGET_FLOOR).astype(np.float32)


def errors_from_targets(y) -> np.ndarray:
    return np.maximum(np.power(10.0, np.asarray(y, np.float64)) - TARGET_FLOOR, 0.0)


def load_scan(path: str) -> Dict[str, object]:
    with open(path) as f:
        return json.load(f)


def tuple_params(t: Dict[str, object]) -> Tuple[float, float, float, float]:
    return (t["dz"], t["dr"], t["gamma_w"], t["charge_w_pC"])


def dataset(scan: Dict[str, object], tuple_ids: Optional[Sequence[int]] = None):
    """(X [n][5], T [n][2], tuple id per row) of every finite-order run with
    finite errors."""
    X, T, ids = [], [], []
    for t in scan["tuples"]:
        if tuple_ids is not None and t["tuple"] not in tuple_ids:
            continue
        for p, e in t["errors"].items():
            es, ee = e["err_sigma_gamma"], e["err_eps"]
            if not (np.isfinite(es) and np.isfinite(ee)):
                continue
            X.append(features(int(p), *tuple_params(t)))
            T.append(targets(es, ee))
            ids.append(t["tuple"])
    return np.array(X, np.float32), np.array(T, np.float32), np.array(ids)


def required_order(t: Dict[str, object], threshold: float = THRESHOLD, orders=ORDERS) -> int:
    """The scan's answer: the lowest order whose measured errors are both
    below the threshold (0 = infinite order)."""
    for p in orders:
        e = t["errors"].get(str(p))
        if e and abs(e["err_sigma_gamma"]) < threshold and abs(e["err_eps"]) < threshold:
            return p
    return 0


class OrderSurrogate:
    def __init__(self, params: np.ndarray, prec: int = MLP_BF16, max_batch: int = 256, device="cuda:0"):
        self.net = MLP(params, 5, 128, 4, 2, prec=prec, max_batch=max_batch, device=device)

    def fit(self, X, T, idx, batch: int = 256, lr: float = LEARNING_RATE):
        """Adam over the minibatch order idx (len(idx) // batch steps); returns the losses."""
        return self.net.train(X, T, idx, batch, lr=lr).cpu().numpy()

    def fit_early_stopping(self, X, T, Xval, Tval, idx, batch: int = 256, lr: float = LEARNING_RATE,
                           check_every: int = CHECK_EVERY):
        """Adam over the minibatch order idx, checking the validation mean
        squared error every `check_every` steps and ending on the parameters
        of the best check (the scan's few hundred runs are easy to overfit).
        Returns (training losses, [(step, validation mse)], best step)."""
        steps = len(idx) // batch
        losses, hist = [], []
        best = (float("inf"), 0, self.net.params())
        for s0 in range(0, steps, check_every):
            n = min(check_every, steps - s0)
            losses.append(self.fit(X, T, idx[s0 * batch:(s0 + n) * batch], batch, lr))
            mse = float(((self.predict(Xval) - Tval) ** 2).mean())
            hist.append((s0 + n, mse))
            if mse < best[0]:
                best = (mse, s0 + n, self.net.params())
        self.net.set_params(best[2])
        return np.concatenate(losses) if losses else np.zeros(0), hist, best[1]

    def predict(self, X) -> np.ndarray:
        return self.net.forward(np.asarray(X, np.float32)).cpu().numpy()

    def predicted_errors(self, params: Tuple[float, float, float, float], orders=ORDERS) -> np.ndarray:
        X = np.stack([features(p, *params) for p in orders])
        return errors_from_targets(self.predict(X))

    def choose_order(self, params, threshold: float = THRESHOLD, orders=ORDERS) -> int:
        """Lowest order predicted to meet the threshold on both errors (0 = infinite)."""
        e = self.predicted_errors(params, orders)
        for p, (es, ee) in zip(orders, e):
            if es < threshold and ee < threshold:
                return p
        return 0

    def close(self):
        self.net.close()


def select_with_fallback(pick: int, referee: Callable[[int], Tuple[float, float]], threshold: float = THRESHOLD,
                         orders=ORDERS) -> Tuple[int, List[int]]:
    """Starting at the picked order, ask the referee (the plain simulation of that
    order against its infinite-order twin) and move one order up until both
    errors are below the threshold; infinite order is always acceptable.
    Returns the accepted order and the finite orders that were simulated."""
    ran: List[int] = []
    if pick == 0:
        return 0, ran
    for p in [q for q in orders if q >= pick]:
        ran.append(p)
        es, ee = referee(p)
        if abs(es) < threshold and abs(ee) < threshold:
            return p, ran
    return 0, ran


def settle_cost(ran: Sequence[int]) -> int:
    """Simulations needed to settle a set-up's order: the infinite-order run
    (the twin every finite order is judged against, or, when the pick is
    infinite, the production run itself) plus every finite order simulated."""
    return 1 + len(ran)


def majority_order(scan: Dict[str, object], tuple_ids: Sequence[int], orders=ORDERS) -> int:
    """The most frequent required order over the given set-ups (ties: the
    lower order); the no-network predictor that always picks it."""
    req = [required_order(t, orders=orders) for t in scan["tuples"] if t["tuple"] in set(tuple_ids)]
    counts = {p: req.count(p) for p in tuple(orders) + (0,)}
    rank = {p: i for i, p in enumerate(tuple(orders) + (0,))}
    return max(counts, key=lambda p: (counts[p], -rank[p]))


def compare_pickers(scan: Dict[str, object], held_ids: Sequence[int], pickers: Dict[str, Callable],
                    orders=ORDERS) -> Dict[str, Dict[str, int]]:
    """For each picker (set-up record -> order, 0 = infinite): over the held-out
    set-ups, the simulations needed with the referee's fallback (settle_cost),
    how often the accepted order is the scan's answer, and how often it is
    higher.  The scan itself needs every finite order plus the twin."""
    recs = {t["tuple"]: t for t in scan["tuples"]}
    rank = {p: i for i, p in enumerate(tuple(orders) + (0,))}
    out = {name: {"runs": 0, "exact": 0, "over": 0} for name in pickers}
    out["scan"] = {"runs": 0, "exact": 0, "over": 0}
    for k in held_ids:
        t = recs[k]
        want = required_order(t, orders=orders)
        out["scan"]["runs"] += len(orders) + 1
        out["scan"]["exact"] += 1
        for name, pick_fn in pickers.items():
            got, ran = select_with_fallback(pick_fn(t), table_referee(t), orders=orders)
            out[name]["runs"] += settle_cost(ran)
            out[name]["exact"] += int(got == want)
            out[name]["over"] += int(rank[got] > rank[want])
    return out


def table_referee(t: Dict[str, object]) -> Callable[[int], Tuple[float, float]]:
    """Referee from a scan record (the errors its plain simulations measured)."""
    def referee(p: int):
        e = t["errors"][str(p)]
        return e["err_sigma_gamma"], e["err_eps"]
    return referee


class PlainReferee:
    """Referee that runs the plain simulation: the infinite-order twin once, then
    each asked order, and measures Err_sigma_gamma and Err_eps of the witness."""

    def __init__(self, inst_by_order: Dict[int, object], steps: int, device="cuda:0"):
        from workloads import scan_workload
        from .pic import Simulation
        from .scan import witness_state
        self._mk = lambda inst: Simulation.from_workload(scan_workload(inst, steps), device=device)
        self._state = witness_state
        self.insts = inst_by_order
        self.steps = steps
        self.runs = 0
        self.ref = self._run(0)

    def _run(self, p: int):
        sim = self._mk(self.insts[p])
        sim.step_graph(self.steps)
        st = self._state(sim)
        sim.close()
        self.runs += 1
        return st

    def __call__(self, p: int):
        from .scan import err_sigma_gamma
        st = self._run(p)
        es = err_sigma_gamma(st["slice_sigma_gamma"], st["slice_count"], self.ref["slice_sigma_gamma"],
                             self.ref["slice_count"])
        ee = (st["eps_nx"] - self.ref["eps_nx"]) / self.ref["eps_nx"]
        return es, ee
