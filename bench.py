"""Benchmark of the force path on one MI355X.

A step is one force evaluation of the whole hot path: count walk, offsets,
write walk, evaluation (p-c + p-p, compensated), unsort and the FP64
diagnostics, on the 2^20-particle Plummer sphere (theta = 0.5, eps = 1e-3,
n_leaf = 16, groups of <= 64) whose tree is already resident in HBM.
Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("particles/s and % FP32 VALU peak at N=2^20, learned vs θ-MAC at p99 err 1e-3")
PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector peak (spec sheet; reached only with packed FP32)
# Non-packed FP32 (the instructions the force kernels are built with): one
# wave64 FMA per SIMD per 4 cycles, 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP x 2.4 GHz.
PEAK_FP32_NONPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
FLOP_PP, FLOP_PC = 38, 70  # the paper's per-interaction convention (Sec. 3.3)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "walk_eval_kernel_plummer1m_theta0.5_traffic.md")
HWFLOPS_PROFILE = os.path.join(ROOT, "profiles", "walk_eval_kernel_plummer1m_theta0.5_hwflops.md")


def source_digest(files):
    """SHA-256 of the given sources with comments and blank lines removed (so
    that only code changes invalidate a recorded measurement)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in files:
        txt = open(os.path.join(ROOT, f)).read()
        txt = re.sub(r"//[^\n]*", "", txt) if not f.endswith(".py") else re.sub(r"#[^\n]*", "", txt)
        h.update("\n".join(l.rstrip() for l in txt.splitlines() if l.strip()).encode())
    return h.hexdigest()


def recorded(path, key):
    """A per-launch figure of the default kernel from a committed counter
    summary, if the kernel's code is still the one it was taken with."""
    import re
    try:
        txt = open(path).read()
        d = json.loads(re.search(r"```json\n(.*?)```", txt, re.S).group(1))
        return d[key] if source_digest(d["sources"]) == d["source_sha256"] else None
    except (OSError, AttributeError, KeyError, ValueError):
        return None


def recorded_traffic():
    """HBM bytes per launch (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy)."""
    return recorded(TRAFFIC_PROFILE, "traffic_bytes")


def valu_rate():
    """Measured issue rate of non-packed VALU instructions (the library's
    measurement program, run as a child process)."""
    import subprocess
    exe = os.path.join(ROOT, "paper_1005_5384_amd", "valu_rate")
    if not os.path.exists(exe):
        return None
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    return json.loads(r.stdout) if r.returncode == 0 else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(pos, m, w, gpu_acc, gpu_pot, plain=None, whole_limit=1 << 21, sweep=None,
                 lvt=None):
    """The oracle as it stands on the same workload: its own tree build, the
    same-tree walk and FP64 evaluation at theta = 0.5 of every group (the
    whole force call) up to `whole_limit` particles, above it of the groups
    that hold the 4096 sampled particles; the same sample on one core; and
    the FP64 direct sum for the sampled particles (the tree-error reference).
    With `sweep` (theta -> GPU outputs, compensated and plain), each angle's
    outputs are judged on the sampled groups against the same-tree oracle and
    on the sample against the FP64 direct sum; with `lvt` (the learned-vs-
    theta comparison's sampled accelerations), both operating points' p99 is
    judged against the FP64 direct sum."""
    import oracle
    cores = oracle.num_threads()
    n = pos.shape[0]
    t0 = time.perf_counter()
    O = oracle.Tree(pos, m, w["n_leaf"], 64)
    t_build = time.perf_counter() - t0
    tg = W_sample(n, w)
    ex = O.export()
    first = ex["topo"][ex["groups"], 2].astype(np.int64)
    rank = np.empty(n, np.int64)
    rank[ex["order"]] = np.arange(n)
    sel = np.unique(np.searchsorted(first, rank[tg], side="right") - 1).astype(np.int32)
    n_sel = int(ex["topo"][ex["groups"][sel], 3].sum())
    whole = n <= whole_limit
    t0 = time.perf_counter()
    ar, pr = O.forces(0.5, w["eps"]) if whole else O.forces(0.5, w["eps"], groups=sel)
    t_eval = time.perf_counter() - t0
    done = np.isfinite(pr)
    ea = oracle.rel_err(gpu_acc[done], ar[done])
    ep = oracle.rel_err(gpu_pot[done], pr[done])
    t0 = time.perf_counter()
    ad, _ = oracle.direct(pos, m, w["eps"], targets=tg)
    t_direct = time.perf_counter() - t0
    oracle.set_threads(1)
    t0 = time.perf_counter()
    O.forces(0.5, w["eps"], groups=sel)
    t_one = time.perf_counter() - t0
    oracle.set_threads(cores)
    judged = {}
    for th, r in (sweep or {}).items():
        sa, sp = O.forces(th, w["eps"], groups=sel)
        judged[th] = {"compensated_vs_same_tree_oracle": _errs((r["acc"], r["pot"]), sa, sp),
                      "plain_vs_same_tree_oracle": _errs((r["plain_acc"], r["plain_pot"]), sa, sp),
                      "vs_direct_fp64": oracle.err_summary(r["acc"][tg], ad),
                      "same_tree_sample": f"the {len(sel)} groups ({n_sel} particles) holding "
                                          f"the {len(tg)} sampled particles"}
    lvt_fp64 = None
    if lvt is not None:
        lvt_fp64 = {k: oracle.err_summary(v, ad) for k, v in lvt.items()}
    what = (f"the whole force call ({O.n_groups} groups)" if whole else
            f"the {len(sel)} groups ({n_sel} particles) holding the {len(tg)} sampled particles")
    return {
        "value": (n if whole else n_sel) / t_eval, "unit": "particles/s", "cores": cores,
        "kind": "oracle",
        "one_core": {"value": n_sel / t_one, "unit": "particles/s", "cores": 1,
                     "sample": f"the {len(sel)} groups ({n_sel} particles) holding the "
                               f"{len(tg)} sampled particles, same-tree walk + FP64 evaluation, "
                               f"{t_one:.2f} s"},
        "sample": (f"{w['gen']} n={n} at theta=0.5: same-tree FP64 walk + evaluation of {what}, "
                   f"{t_eval:.2f} s; oracle tree build {t_build:.2f} s; FP64 direct sum of the "
                   f"{len(tg)} sampled particles {t_direct:.2f} s"),
        "eval_s": t_eval,
        "gpu_vs_same_tree_oracle": {"acc_med": float(np.median(ea)), "acc_max": float(ea.max()),
                                    "pot_med": float(np.median(ep)), "pot_max": float(ep.max()),
                                    "particles": int(done.sum())},
        **({} if plain is None else {"gpu_plain_sum_vs_same_tree_oracle": _errs(plain, ar, pr)}),
        "gpu_vs_direct_fp64": oracle.err_summary(gpu_acc[tg], ad) | {"n": len(tg)},
        **({"theta_sweep": judged} if judged else {}),
        **({"learned_vs_theta_vs_direct_fp64": lvt_fp64} if lvt_fp64 else {}),
    }


def _errs(out, ar, pr):
    import oracle
    done = np.isfinite(pr)
    ea = oracle.rel_err(out[0][done], ar[done])
    ep = oracle.rel_err(out[1][done], pr[done])
    return {"acc_med": float(np.median(ea)), "acc_max": float(ea.max()),
            "pot_med": float(np.median(ep)), "pot_max": float(ep.max())}


def integration_rate(n, theta, eps, steps, dt=1.0 / 256):
    """Kick-drift-kick steps of an equilibrium Plummer sphere of n particles
    with the tree rebuilt on the GPU every step: the science rate (particles
    advanced per second) and the energy change over the timed steps."""
    from paper_1005_5384_amd import octgrav as og
    from paper_1005_5384_amd import workloads as W
    pos, vel, m = W.plummer_with_velocities(n, 102)
    S = og.Sim(pos, vel, m, 16, 64)
    S.run(theta, eps, dt, 1)  # first forces and one step
    e0 = S.energy()
    S.run(theta, eps, dt, steps)
    e1 = S.energy()
    t = S.timings()
    return {"workload": f"equilibrium Plummer sphere (Aarseth-Henon-Wielen velocities), n={n}",
            "theta": theta, "eps": eps, "dt": dt, "steps": steps,
            "ms_per_step": t["step_ms"], "tree_build_ms": t["build_ms"], "forces_ms": t["forces_ms"],
            "particles_per_s": n / (t["step_ms"] * 1e-3),
            "energy_rel_change": abs(e1["E"] - e0["E"]) / abs(e0["E"]),
            "virial_2K_over_W": 2 * e0["K"] / abs(e0["W"])}


def list_spread(T, theta, eps):
    """Spread of the theta walk's per-group list lengths |C_g|, |L_g| and
    source-particle counts n_pp(g) (the library's per-group counts of one
    force call; no list export), and of the algorithmic FLOPs per 32-target
    work item (the unit a wave takes from the work counter)."""
    T.forces(theta, eps)
    cnt = T.group_counts().astype(np.int64)
    n_c, n_l, n_pp = cnt[:, 0], cnt[:, 1], cnt[:, 2]
    ex = T.export()
    gsize = ex["topo"][ex["groups"], 3].astype(np.int64)
    items = (gsize + 31) // 32
    g = np.repeat(np.arange(gsize.size), items)
    k = np.arange(g.size) - np.repeat(np.cumsum(items) - items, items)
    tgt = np.minimum(32, gsize[g] - 32 * k)
    flops = tgt * (38.0 * n_pp[g] + 70.0 * n_c[g])
    q = lambda a: {"min": float(a.min()), "median": float(np.median(a)),
                   "p90": float(np.quantile(a, 0.9)), "p99": float(np.quantile(a, 0.99)),
                   "max": float(a.max()), "mean": float(a.mean())}
    return {"theta": theta, "groups": int(gsize.size), "group_size": q(gsize),
            "cell_list": q(n_c), "leaf_list": q(n_l), "pp_sources": q(n_pp),
            "work_items": int(g.size), "item_flops": q(flops),
            "item_max_over_mean": float(flops.max() / flops.mean())}


def W_sample(n, w):
    from paper_1005_5384_amd import workloads as W
    return W.sample_indices(n, w.get("sample", 4096), w.get("sample_seed", 4096))


def learned_vs_theta(T, w, steps, band=None, beta=30.0, target=1e-3, params=None,
                     band_rel=(-0.015, 0.25)):
    """The learned acceptance criterion against the opening angle at equal
    p99 relative force error (against the GPU direct sum on the 4096-particle
    sample): theta* by bisection, then tau_pair (budget = beta * tau_pair) by
    bisection in log tau, then both timed over `steps` force calls.  Returns
    the summary and the sampled accelerations of both operating points (for
    the FP64 judgement in the CPU-baseline leg).  The
    network decides in the band (theta* + a, theta* + b), band_rel = (a, b),
    or in the fixed `band` when one is given.
    The target is unreachable when the band's lower edge exceeds theta*
    (everything that edge accepts is accepted): `target_met` says whether the
    learned operating point met it."""
    import torch
    from paper_1005_5384_amd import learned as L
    from paper_1005_5384_amd import octgrav as og
    from paper_1005_5384_amd import workloads as W
    eps = w["eps"]
    smp = W.sample_indices(T.n, w.get("sample", 4096), w.get("sample_seed", 4096))
    ref, _ = T.direct(eps, smp)
    sm = torch.as_tensor(smp, device="cuda")
    acc = torch.empty((T.n, 3), dtype=torch.float32, device="cuda")

    def p99(theta):
        return L.p99_error(T, eps, sm, ref, theta)

    def timed(theta):
        T.forces(theta, eps, acc=acc, with_pot=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            T.forces(theta, eps, acc=acc, with_pot=False)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    def sampled(theta):
        a, _ = T.forces(theta, eps, with_pot=False)
        return a[sm].double().cpu().numpy()

    T.set_mac(None)
    th, e_th = L.bisect(p99, 0.3, 1.0, target, increasing=True)
    t_th = timed(th)
    c_th = T.last_counts()
    acc_th = sampled(th)
    log(f"bench: theta* {th:.4f} p99 {e_th:.3e} {t_th * 1e3:.3f} ms")
    if band is None:
        band = (min(1.0, max(0.0, th + band_rel[0])), min(1.0, th + band_rel[1]))
    net = og.Mlp(L.load_params() if params is None else L.load_params(params))

    def p99_tau(lt):
        T.set_mac(net, band[0], band[1], 10.0 ** lt, beta * 10.0 ** lt)
        return p99(th)
    lt, e_l = L.bisect(p99_tau, -6.0, -1.0, target, increasing=True)
    tau = 10.0 ** lt
    T.set_mac(net, band[0], band[1], tau, beta * tau)
    t_l = timed(th)
    c_l = T.last_counts()
    st = T.mac_stats()
    acc_l = sampled(th)
    T.set_mac(None)
    log(f"bench: learned tau {tau:.3e} p99 {e_l:.3e} {t_l * 1e3:.3f} ms")
    n = T.n
    return {
        "target_p99": target, "sample": len(smp), "reference": "GPU FP32-compensated direct sum",
        "theta": {"theta_star": th, "p99": e_th, "particles_per_s": n / t_th, "ms": t_th * 1e3,
                  "pc_per_particle": c_th["n_pc"] / n, "pp_per_particle": c_th["n_pp"] / n},
        "learned": {"theta_lo": band[0], "theta_hi": band[1], "tau_pair": tau,
                    "budget": beta * tau, "fallback_theta": th, "p99": e_l,
                    "particles_per_s": n / t_l, "ms": t_l * 1e3,
                    "pc_per_particle": c_l["n_pc"] / n, "pp_per_particle": c_l["n_pp"] / n,
                    "band_scored": st["band"], "groups_fell_back": st["fell_back"],
                    "groups": T.stats["n_groups"]},
        "speedup": t_th / t_l,
        "flop_ratio": ((FLOP_PC * c_th["n_pc"] + FLOP_PP * c_th["n_pp"])
                       / (FLOP_PC * c_l["n_pc"] + FLOP_PP * c_l["n_pp"])),
        "target_met": bool(e_l <= target),
    }, {"theta_star": acc_th, "learned": acc_l}


def theta_sweep(T, w, steps, thetas, path=None):
    """Every opening angle of the workload's set on the same tree: `steps`
    compensated force calls (host clock over the calls; the fused kernel's
    HIP-event phase for the roofline fraction) and `steps` with plain FP32
    accumulation.  Returns the per-angle summary and the host copies of the
    outputs (for the oracle's judgement in the CPU-baseline leg)."""
    import torch
    eps, n = w["eps"], T.n
    acc = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    pot = torch.empty(n, dtype=torch.float32, device="cuda")
    summary, outputs = {}, {}

    def run(theta, plain):
        for _ in range(2):
            T.forces(theta, eps, acc=acc, pot=pot, plain=plain, timed=True, path=path)
        torch.cuda.synchronize()
        ev = []
        t0 = time.perf_counter()
        for _ in range(steps):
            T.forces(theta, eps, acc=acc, pot=pot, plain=plain, timed=True, path=path)
            ev.append(T.last_timings()["eval"])
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps * 1e3, float(np.mean(ev))

    for th in thetas:
        ms, ev_ms = run(th, False)
        c = T.last_counts()
        a, p = acc.double().cpu().numpy(), pot.double().cpu().numpy()
        ms_p, ev_p = run(th, True)
        flops = FLOP_PP * c["n_pp"] + FLOP_PC * c["n_pc"]
        summary[th] = {"ms_per_call": ms, "particles_per_s": n / (ms * 1e-3),
                       "kernel_ms": ev_ms, "flops_per_launch": flops,
                       "frac": flops / (ev_ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS,
                       "frac_nonpacked": flops / (ev_ms * 1e-3) / 1e12 / PEAK_FP32_NONPACKED_TFLOPS,
                       "path_frac": flops / (ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS,
                       "interactions_per_particle": {"pc": c["n_pc"] / n, "pp": c["n_pp"] / n},
                       "plain_ms_per_call": ms_p, "plain_kernel_ms": ev_p}
        outputs[th] = {"acc": a, "pot": p, "plain_acc": acc.double().cpu().numpy(),
                       "plain_pot": pot.double().cpu().numpy()}
        log(f"bench: theta {th}: {ms:.3f} ms ({ev_ms:.3f} kernel, "
            f"{summary[th]['frac'] * 100:.1f} % of peak), plain {ms_p:.3f} ms")
    return summary, outputs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="plummer1m")
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--path", default=None, choices=["two_pass", "fused_block", "fused_wave"],
                    help="force one implementation path (default: the library's choice for theta)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-criterion vs theta comparison at equal p99 error")
    ap.add_argument("--mac", default="theta", choices=["theta", "learned"],
                    help="acceptance criterion of the timed steps")
    ap.add_argument("--tau", type=float, default=4.21e-4,
                    help="tau_pair of --mac learned (budget --beta x tau)")
    ap.add_argument("--band", type=float, nargs=2, default=None, metavar=("LO", "HI"),
                    help="opening angles bounding the learned criterion's band (--mac learned: "
                         "default 0.4 0.8; learned-vs-theta: default theta*-0.015, theta*+0.25)")
    ap.add_argument("--band-rel", type=float, nargs=2, default=(-0.015, 0.25), metavar=("A", "B"),
                    help="learned-vs-theta comparison: band (theta* + A, theta* + B) unless "
                         "--band is given")
    ap.add_argument("--beta", type=float, default=30.0,
                    help="group budget of the learned criterion in units of tau_pair")
    ap.add_argument("--params", default=None,
                    help="network parameters of the learned criterion (.npy, 5057 float32; "
                         "default: the shipped network)")
    ap.add_argument("--no-valu-rate", action="store_true",
                    help="skip the measurement of the non-packed VALU instruction rates")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the timing of the workload's other opening angles")
    ap.add_argument("--no-integration", action="store_true",
                    help="skip the leapfrog science-rate measurement")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="instead of the bench: time a plain device copy of this many bytes "
                         "(the reference for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the library "
              "drives one GPU per process; a multi-GPU run would shard the groups over a "
              "replicated tree)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1005_5384_amd import octgrav as og
    from paper_1005_5384_amd import workloads as W

    torch.cuda.set_device(0)
    if args.copy_bytes:
        nb = args.copy_bytes // 16 * 16
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(args.warmup):
            dst.copy_(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        print(json.dumps({"copy_bytes": nb, "ms": dt * 1e3, "read_plus_write_GBps": 2 * nb / dt / 1e9}))
        return
    w = W.WORKLOADS[args.workload]
    log(f"bench: generating {args.workload} n={w['n']}")
    pos, m = W.make(args.workload)
    n = pos.shape[0]
    # first use (library load, HIP context, allocator pools), then the timed build
    og.Tree(pos, m, w["n_leaf"], 64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    T = og.Tree(pos, m, w["n_leaf"], 64)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    log(f"bench: tree built+uploaded in {t_build:.3f} s: {T.stats}")
    # the same tree built on the GPU (bit-identical; timed, then released)
    og.Tree(pos[:1024], m[:1024], w["n_leaf"], 64, device_build=True)  # first-use setup
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Tdev = og.Tree(pos, m, w["n_leaf"], 64, device_build=True)
    torch.cuda.synchronize()
    t_dev_build = time.perf_counter() - t0
    del Tdev
    log(f"bench: device build {t_dev_build:.4f} s")
    acc = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    pot = torch.empty(n, dtype=torch.float32, device="cuda")
    theta, eps = args.theta, w["eps"]
    if args.mac == "learned":
        from paper_1005_5384_amd import learned as L
        net = og.Mlp(L.load_params() if args.params is None else L.load_params(args.params))
        band = tuple(args.band) if args.band else (0.4, 0.8)
        T.set_mac(net, band[0], band[1], args.tau, args.beta * args.tau)

    for _ in range(args.warmup):
        T.forces(theta, eps, acc=acc, pot=pot, timed=True, path=args.path)
    torch.cuda.synchronize()
    log("bench: warmup done")

    phases = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        T.forces(theta, eps, acc=acc, pot=pot, timed=True, path=args.path)
        phases.append(T.last_timings())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"bench: {args.steps} steps in {elapsed:.4f} s")

    counts = T.last_counts()
    flops = FLOP_PP * counts["n_pp"] + FLOP_PC * counts["n_pc"]
    ph = {k: float(np.mean([p[k] for p in phases])) for k in phases[0]}
    eval_s = ph["eval"] * 1e-3
    achieved = flops / eval_s / 1e12
    ms_step = elapsed / args.steps * 1e3
    path_tflops = flops / (ms_step * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": n * args.steps / elapsed,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "distribution": w["gen"], "theta": theta,
                   "eps": eps, "n_leaf": w["n_leaf"], "n_group": 64, "mac": args.mac,
                   "accumulation": "compensated",
                   "path": args.path or "default"},
        "roofline": {"bound": "alu",
                     "kernel": ("walk_eval_kernel: fused walk + evaluation, HIP-event phase on "
                                "the library's stream (two-pass path: eval_kernel)"),
                     "achieved": achieved,
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": (recorded_traffic() if (args.workload == "plummer1m" and theta == 0.5
                                                        and args.path is None and args.mac == "theta")
                                 else None),
                     "flops_per_launch": flops, "flop_convention": "38 per p-p, 70 per p-c",
                     "peak_nonpacked": PEAK_FP32_NONPACKED_TFLOPS,
                     "frac_nonpacked": achieved / PEAK_FP32_NONPACKED_TFLOPS},
        "hw_fp32": None,
        "path_frac_peak": path_tflops / PEAK_FP32_TFLOPS,
        "path_tflops": path_tflops,
        "interactions_per_s": (counts["n_pp"] + counts["n_pc"]) / (ms_step * 1e-3),
        "interactions": counts,
        "phases_ms": ph,
        "host_build_upload_s": t_build,
        "device_build_s": t_dev_build,
        # one force call from host particles: tree build (+ upload) and the call
        "end_to_end_ms": {"host_build": t_build * 1e3 + ms_step,
                          "device_build": t_dev_build * 1e3 + ms_step},
        "tree": T.stats,
    }
    default_kernel = (args.workload == "plummer1m" and theta == 0.5 and args.path is None
                      and args.mac == "theta")
    hw = recorded(HWFLOPS_PROFILE, "hw_fp32_flops_per_launch") if default_kernel else None
    if hw:
        # Hardware-counted FP32 operations of the same kernel (FMA = 2, one per
        # active lane) over this run's kernel time: the paper's convention
        # counts more per interaction than the instructions execute.
        out["hw_fp32"] = {"flops_per_launch": hw, "tflops": hw / eval_s / 1e12,
                          "frac": hw / eval_s / 1e12 / PEAK_FP32_TFLOPS,
                          "frac_nonpacked": hw / eval_s / 1e12 / PEAK_FP32_NONPACKED_TFLOPS,
                          "counters": "SQ_INSTS_VALU_FLOPS_FP32 + SQ_INSTS_VALU_FLOPS_FP32_TRANS"}
    if args.mac == "learned":
        out["config"].update({"tau_pair": args.tau, "theta_lo": band[0],
                              "theta_hi": band[1], "budget": args.beta * args.tau})
        out["mac_stats"] = T.mac_stats()
        T.set_mac(None)
    if args.mac == "theta":
        log("bench: list-length spread ...")
        out["list_spread"] = list_spread(T, theta, eps)
    if not args.no_integration and args.workload == "plummer1m":
        log("bench: leapfrog science rate ...")
        out["integration"] = integration_rate(n, theta, eps, args.steps)
    if not args.no_valu_rate:
        log("bench: VALU issue-rate probe ...")
        out["valu_rate"] = valu_rate()
    sweep_out = None
    if args.mac == "theta" and len(w.get("thetas", ())) > 1 and not args.no_sweep:
        log(f"bench: opening angles {w['thetas']} ...")
        out["theta_sweep"], sweep_out = theta_sweep(T, w, args.steps, w["thetas"], args.path)
    lvt_acc = None
    if not args.no_learned:
        log("bench: learned criterion vs theta at p99 1e-3 ...")
        out["learned_vs_theta"], lvt_acc = learned_vs_theta(
            T, w, args.steps, band=tuple(args.band) if args.band else None, beta=args.beta,
            params=args.params, band_rel=tuple(args.band_rel))
    # FP32 plain accumulation (no compensation) on the same call, for comparison
    plain = None
    if args.mac == "theta":
        pa = torch.empty_like(acc)
        pp = torch.empty_like(pot)
        T.forces(theta, eps, acc=pa, pot=pp, plain=True, path=args.path)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            T.forces(theta, eps, acc=pa, pot=pp, plain=True, path=args.path)
        torch.cuda.synchronize()
        out["plain_sum_ms_per_step"] = (time.perf_counter() - t0) / args.steps * 1e3
        plain = (pa.double().cpu().numpy(), pp.double().cpu().numpy())
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle) ...")
        a = acc.double().cpu().numpy()
        p = pot.double().cpu().numpy()
        out["cpu_baseline"] = cpu_baseline(pos, m, w, a, p, plain, sweep=sweep_out, lvt=lvt_acc)
        log("bench: cpu baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
