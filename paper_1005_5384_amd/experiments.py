"""Experiments around the force path (the paper's Sec. 3 and its parameter
choices in Sec. 2): a sweep of the leaf and group capacities, including the
per-particle walk (groups of one particle); the force error against the
direct sum as a function of the opening angle and N on the Milky-Way-like
stand-in of the paper's galaxy model; and the boundary-centre opening test
against the centre-of-mass offset variant at equal error. Every
configuration prints one JSON line.

    python -m paper_1005_5384_amd.experiments sweep [--workload plummer1m]
    python -m paper_1005_5384_amd.experiments errors
    python -m paper_1005_5384_amd.experiments mac [--workload plummer1m]
    python -m paper_1005_5384_amd.experiments energy

Errors are |a - a_ref| / |a_ref| (Sec. 3.1) on 4096 seeded sampled particles,
a_ref from the library's compensated FP32 direct sum; percentiles are nearest
rank. Times are HIP-event times of whole force calls (walk, evaluation,
totals and diagnostics) with the tree resident on the device."""
from __future__ import annotations

import argparse
import json
import math
import sys

import numpy as np

from . import octgrav as og
from . import workloads as W

FLOP_PP, FLOP_PC = 38, 70


def nearest_rank(x: np.ndarray, q: float) -> float:
    """The ceil(q n)-th smallest value of x (q in (0, 1])."""
    s = np.sort(np.asarray(x, dtype=np.float64))
    return float(s[max(0, math.ceil(q * s.size) - 1)])


def _errors(acc, ref) -> dict:
    a = acc.double()
    r = ref.double()
    e = ((a - r).norm(dim=1) / r.norm(dim=1)).cpu().numpy()
    return {"p10": nearest_rank(e, 0.1), "median": nearest_rank(e, 0.5),
            "p90": nearest_rank(e, 0.9), "p99": nearest_rank(e, 0.99), "max": float(e.max())}


def _timed(T, theta, eps, steps):
    """Median ms of `steps` force calls, and the interaction counts of the last."""
    import torch
    acc = torch.empty((T.n, 3), dtype=torch.float32, device="cuda")
    pot = torch.empty(T.n, dtype=torch.float32, device="cuda")
    T.forces(theta, eps, acc=acc, pot=pot)
    ms = []
    for _ in range(steps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        T.forces(theta, eps, acc=acc, pot=pot)
        b.record()
        b.synchronize()
        ms.append(a.elapsed_time(b))
    return float(np.median(ms)), T.last_counts(), acc


def _row(T, n, theta, eps, steps, smp, ref):
    ms, c, acc = _timed(T, theta, eps, steps)
    flops = FLOP_PP * c["n_pp"] + FLOP_PC * c["n_pc"]
    return {"ms": ms, "particles_per_s": n / (ms * 1e-3), "tflops": flops / (ms * 1e-3) / 1e12,
            "pc_per_particle": c["n_pc"] / n, "pp_per_particle": c["n_pp"] / n,
            "err": _errors(acc[smp], ref)}


def leaf_group_sweep(workload="plummer1m", theta=0.5, leaves=(4, 8, 16, 32, 64),
                     groups=(1, 8, 16, 32, 64, 128, 256), steps=5, out=sys.stdout,
                     extra=((1, 1), (1, 64))):
    """Leaf capacity x group capacity at one opening angle, plus the `extra`
    (n_leaf, n_group) pairs. The paper's choices are n_leaf = 16 and groups of
    at most 64. A group is a maximal cell of at most n_group particles or a
    leaf, so n_leaf = n_group = 1 is the per-particle walk."""
    import torch
    w = W.WORKLOADS[workload]
    pos, m = W.make(workload)
    n, eps = pos.shape[0], w["eps"]
    smp = torch.as_tensor(W.sample_indices(n, 4096, 4096), device="cuda")
    ref = None
    rows = []
    for nl, ng in [(a, b) for a in leaves for b in groups] + list(extra):
        T = og.Tree(pos, m, nl, ng, device_build=True)
        if ref is None:
            ref, _ = T.direct(eps, smp)
        r = {"experiment": "leaf_group_sweep", "workload": workload, "n": n, "theta": theta,
             "eps": eps, "n_leaf": nl, "n_group": ng, "cells": T.stats["n_cells"],
             "groups": T.stats["n_groups"], "work_items": T.stats["n_work"],
             **_row(T, n, theta, eps, steps, smp, ref)}
        T.close()
        print(json.dumps(r), file=out, flush=True)
        rows.append(r)
    return rows


def error_curves(ns=(1 << 16, 1 << 18, 1 << 20, 1 << 22),
                 thetas=(0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9, 1.0), eps=1e-3, n_leaf=16,
                 n_group=64, seed=109, steps=3, out=sys.stdout):
    """Error percentiles and cost against theta for several N on the
    Milky-Way-like stand-in, and the fitted slope of log(median error)
    against log(theta) per N."""
    import torch
    rows = []
    for n in ns:
        pos, m = W.milky_way(n, seed)
        T = og.Tree(pos, m, n_leaf, n_group, device_build=True)
        smp = torch.as_tensor(W.sample_indices(n, 4096, 4096), device="cuda")
        ref, _ = T.direct(eps, smp)
        med = []
        for th in thetas:
            r = {"experiment": "error_curves", "workload": "milky_way", "n": n, "seed": seed,
                 "theta": th, "eps": eps, "n_leaf": n_leaf, "n_group": n_group,
                 **_row(T, n, th, eps, steps, smp, ref)}
            med.append(r["err"]["median"])
            print(json.dumps(r), file=out, flush=True)
            rows.append(r)
        k = [i for i, th in enumerate(thetas) if 0.3 <= th <= 0.8]
        slope = float(np.polyfit(np.log([thetas[i] for i in k]), np.log([med[i] for i in k]), 1)[0])
        s = {"experiment": "error_curves_slope", "n": n, "thetas": [thetas[i] for i in k],
             "median_error_slope": slope}
        print(json.dumps(s), file=out, flush=True)
        rows.append(s)
        T.close()
    return rows


def mac_variants(workload="plummer1m", targets=(2.5e-4, 5e-4, 1e-3), steps=5, out=sys.stdout):
    """The boundary-centre opening test against the centre-of-mass offset
    test at equal p99 error: theta bisected for each (the offset test within
    its range, theta <= 0.57), then both timed on the fused wave path (the
    offset test's path) so that only the criterion differs."""
    import torch
    from .learned import bisect
    w = W.WORKLOADS[workload]
    pos, m = W.make(workload)
    n, eps = pos.shape[0], w["eps"]
    T = og.Tree(pos, m, w["n_leaf"], 64, device_build=True)
    smp = torch.as_tensor(W.sample_indices(n, 4096, 4096), device="cuda")
    ref, _ = T.direct(eps, smp)

    def p99(theta, com):
        acc, _ = T.forces(theta, eps, with_pot=False, com=com)
        return _errors(acc[smp], ref)["p99"]

    rows = []
    for tgt in targets:
        r = {"experiment": "mac_variants", "workload": workload, "n": n, "target_p99": tgt}
        for name, com, hi in (("boundary", False, 1.0), ("com_offset", True, 0.57)):
            th, e = bisect(lambda x: p99(x, com), 0.1, hi, tgt, increasing=True)
            ms, c, _ = _timed_mac(T, th, eps, steps, com)
            r[name] = {"theta": th, "p99": e, "ms": ms, "pc_per_particle": c["n_pc"] / n,
                       "pp_per_particle": c["n_pp"] / n}
        r["offset_speedup"] = r["boundary"]["ms"] / r["com_offset"]["ms"]
        print(json.dumps(r), file=out, flush=True)
        rows.append(r)
    T.close()
    return rows


def _timed_mac(T, theta, eps, steps, com):
    import torch
    acc = torch.empty((T.n, 3), dtype=torch.float32, device="cuda")
    path = "fused_wave"
    T.forces(theta, eps, acc=acc, with_pot=False, com=com, path=path)
    ms = []
    for _ in range(steps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        T.forces(theta, eps, acc=acc, with_pot=False, com=com, path=path)
        b.record()
        b.synchronize()
        ms.append(a.elapsed_time(b))
    return float(np.median(ms)), T.last_counts(), acc


def energy_runs(n=1 << 20, thetas=(0.3, 0.5, 0.75), eps=1e-3, dt=1.0 / 256, steps=2048,
                every=256, seed=102, out=sys.stdout):
    """Energy conservation of the leapfrog with the tree rebuilt on the GPU
    every step (an equilibrium Plummer sphere): relative energy change and
    momentum drift every `every` steps, per opening angle."""
    pos, vel, m = W.plummer_with_velocities(n, seed)
    rows = []
    for th in thetas:
        S = og.Sim(pos, vel, m, 16, 64)
        S.run(th, eps, dt, 0)
        e0 = S.energy()
        for k in range(every, steps + 1, every):
            S.run(th, eps, dt, every)
            e = S.energy()
            r = {"experiment": "energy_runs", "n": n, "theta": th, "eps": eps, "dt": dt,
                 "step": k, "t": k * dt, "dE_over_E": (e["E"] - e0["E"]) / abs(e0["E"]),
                 "dP": float(np.linalg.norm(e["P"] - e0["P"])),
                 "virial_2K_over_W": 2 * e["K"] / abs(e["W"]),
                 "ms_per_step": S.timings()["step_ms"]}
            print(json.dumps(r), file=out, flush=True)
            rows.append(r)
        S.close()
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("what", choices=["sweep", "errors", "mac", "energy"])
    ap.add_argument("--workload", default="plummer1m")
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--steps", type=int, default=5)
    a = ap.parse_args(argv)
    if a.what == "sweep":
        leaf_group_sweep(a.workload, a.theta, steps=a.steps)
    elif a.what == "mac":
        mac_variants(a.workload, steps=a.steps)
    elif a.what == "energy":
        energy_runs()
    else:
        error_curves(steps=a.steps)


if __name__ == "__main__":
    main()
