"""Learned warm start for a family of LPs that share A (the config-4 family).

Everything numerical runs in the library: target solves (the FP64 PDHG
solver), the network's forward and backward passes and Adam (BF16/FP32 MFMA
kernels), the trial runs of the judge.  This module only sequences those calls.

Protocol:
  1. solve every training instance with the FP64 solver to eps (targets);
  2. reference point = mean of the training solutions (and of c, b);
  3. train the network (residual on the reference point) with Adam;
  4. for a held-out instance: predict (x0, y0); judge the prediction, its
     primal part alone, its dual part alone and the cold start (0 clamped
     into X, 0 projected onto Y) by a short trial: one check block
     (check_period iterations) from each, scored by the fixed-point residual
     r(z) = ||z - T(z)||_P of App. B.2 at the block's last check (all trials
     start with the same primal weight, so the scores share one norm); the
     solve starts from the best-scoring point, and the trial iterations are
     counted in its total; if a warm run does not converge within its
     iteration cap, a cold run takes over.
"""
from __future__ import annotations

import time
from typing import List, Optional

import numpy as np

from . import CONVERGED, Problem, WarmStartNet, row_b

H = 128
F = 16


def n_params(layers: int) -> int:
    return 2 * F * H + layers * 2 * (2 * H * H) + 2 * H


def init_params(layers: int, seed: int = 0) -> np.ndarray:
    """He-normal matrices, zero output heads (so the untrained network returns
    the reference point exactly)."""
    rng = np.random.default_rng(seed)
    parts = [rng.standard_normal(F * H) * np.sqrt(2.0 / F),
             rng.standard_normal(F * H) * np.sqrt(2.0 / F)]
    for _ in range(layers):
        parts += [rng.standard_normal(2 * H * H) * np.sqrt(1.0 / (2 * H)),
                  rng.standard_normal(2 * H * H) * np.sqrt(1.0 / (2 * H))]
    parts += [np.zeros(H), np.zeros(H)]
    return np.concatenate(parts).astype(np.float32)


def solve_member(prob: Problem, inst, x0=None, y0=None) -> dict:
    prob.update_data(inst.c, inst.con_lo, inst.con_hi)
    t0 = time.perf_counter()
    r = prob.solve(x0, y0)
    r["wall"] = time.perf_counter() - t0
    return r


def family_targets(prob: Problem, instances, log=None) -> List[Optional[dict]]:
    """FP64 solutions of the instances (None for a member that did not
    converge, e.g. one made infeasible by the perturbation)."""
    out = []
    for i, inst in enumerate(instances):
        r = solve_member(prob, inst)
        out.append(dict(x=r["x"], y=r["y"], iters=r["iters"]) if r["status"] == CONVERGED else None)
        if log and (i + 1) % 16 == 0:
            log(f"targets {i + 1}/{len(instances)}")
    return out


def reference(instances, sols):
    ok = [(a, s) for a, s in zip(instances, sols) if s is not None]
    c_ref = np.mean([a.c for a, _ in ok], axis=0)
    b_ref = np.mean([row_b(a.con_lo, a.con_hi) for a, _ in ok], axis=0)
    x_ref = np.mean([s["x"] for _, s in ok], axis=0)
    y_ref = np.mean([s["y"] for _, s in ok], axis=0)
    return c_ref, b_ref, x_ref, y_ref


def train(net: WarmStartNet, instances, sols, epochs: int = 8, lr: float = 1e-3,
          seed: int = 0, log=None) -> list:
    rng = np.random.default_rng(seed)
    idx = [i for i, s in enumerate(sols) if s is not None]
    hist = []
    for ep in range(epochs):
        rng.shuffle(idx)
        tot = np.zeros(2)
        for i in idx:
            inst = instances[i]
            net.set_instance(inst.c, inst.con_lo, inst.con_hi)
            tot += net.backward(sols[i]["x"], sols[i]["y"])
            net.adam_step(lr)
        hist.append((tot / max(len(idx), 1)).tolist())
        if log:
            log(f"epoch {ep + 1}/{epochs}: mean loss (cols, rows) {hist[-1]}")
    return hist


def start_kkt(prob: Problem, x0=None, y0=None) -> float:
    """Relative KKT error of the start point the solver would use (x0, y0
    clamped into X and projected onto Y by dpdlp_init; None = cold start)."""
    prob.init(x0, y0)
    k = prob.kkt()
    return float(max(k[0], k[1], k[2]))


def trial_score(prob: Problem, x0=None, y0=None) -> tuple:
    """One check block from the start point: the fixed-point residual r of
    its last check (App. B.2) and that check's relative KKT error."""
    prob.init(x0, y0)
    prob.iterate(int(prob.params.check_period))
    last = prob.log()[-1]
    return float(last["r"]), float(max(last["r_primal"], last["r_dual"], last["r_gap"]))


def warm_solve(prob: Problem, inst, mode: str, net: Optional[WarmStartNet] = None,
               ref=None, warm_cap: Optional[int] = None) -> dict:
    """Solve one member from a cold, mean-reference or network start.

    Judge: the candidate starts (x0, y0), (x0, cold y), (cold x, y0) and the
    cold start each run one check block; the one with the smallest
    fixed-point residual at its end is solved from the start, so a
    prediction is used only where its trial beats the cold start's.  The
    trial iterations count in the total.  A warm run that does not converge
    within warm_cap iterations is followed by a cold run (both counted)."""
    prob.update_data(inst.c, inst.con_lo, inst.con_hi)
    t0 = time.perf_counter()
    x0 = y0 = None
    if mode == "gnn":
        net.set_instance(inst.c, inst.con_lo, inst.con_hi)
        x0, y0 = net.forward()
    elif mode == "mean":
        x0, y0 = ref[2], ref[3]
    total_iters = 0
    sw = sc = None
    choice = "cold"
    if x0 is not None:
        cands = {"cold": (None, None), "both": (x0, y0), "primal": (x0, None),
                 "dual": (None, y0)}
        scores = {}
        for k, v in cands.items():
            scores[k] = trial_score(prob, *v)[0]
            total_iters += int(prob.params.check_period)
        choice = min(scores, key=scores.get)
        sc = scores["cold"]
        sw = min(v for k, v in scores.items() if k != "cold")
        x0, y0 = cands[choice]
    fallback = choice == "cold" and mode != "cold"
    saved = prob.params.max_iters
    warm = x0 is not None or y0 is not None
    if warm and warm_cap:
        prob.set_params(max_iters=warm_cap)
    r = prob.solve(x0, y0)
    total_iters += r["iters"]
    log = prob.log()
    if r["status"] != CONVERGED and warm:
        prob.set_params(max_iters=saved)
        r = prob.solve()
        total_iters += r["iters"]
        log = prob.log()
        fallback = True
    prob.set_params(max_iters=saved)
    el = time.perf_counter() - t0
    return dict(mode=mode, iters=int(total_iters), seconds=el, status=int(r["status"]),
                fallback=fallback, choice=choice, judge_warm=sw, judge_cold=sc,
                obj=r["obj_primal"], kkt=max(r["r_primal"], r["r_dual"], r["r_gap"]),
                first_iter=first_reach(log, total_iters - int(r["iters"])))


def first_reach(log, offset: int, tols=(1e-4, 1e-6, 1e-8)) -> dict:
    """Iteration count (plus offset) at which the solve's checks first
    reached each tolerance, from its restart-decision log."""
    out = {}
    for tol in tols:
        out[f"{tol:g}"] = next((offset + int(e["t"]) + 1 for e in log
                                if max(e["r_primal"], e["r_dual"], e["r_gap"]) <= tol), None)
    return out
