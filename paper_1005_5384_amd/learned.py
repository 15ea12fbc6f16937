"""Training and calibration of the learned acceptance criterion.

Everything numerical runs in the library's kernels: labels from the GPU
direct sum and the per-pair label kernel, training by the library's
forward / backward / Adam kernels.  This module only shuffles batches and
drives the loops.

    python -m paper_1005_5384_amd.learned train --out params.npy
"""
from __future__ import annotations

import argparse
import os
import time

import numpy as np

from . import octgrav as og
from . import workloads as W

THETA_LO, THETA_HI = 0.3, 1.0
PINBALL_TAU = 0.9
PARAMS_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data",
                           "learned_mac_params.npy")


def load_params(path: str = PARAMS_PATH) -> np.ndarray:
    """The trained network's 5057 FP32 parameters (written by `train`)."""
    P = np.load(path, allow_pickle=False)
    if P.dtype != np.float32 or P.shape != (og.N_PARAMS,):
        raise ValueError(f"{path}: expected {og.N_PARAMS} float32 parameters")
    return P


def collect(pos, mass, eps, n_leaf=16, n_group=64, stride=1, cap=1 << 23):
    """(features [k,12], targets log10(max(e, 1e-12)) [k]) of the band pairs
    of one particle set (torch CUDA tensors)."""
    import torch
    T = og.Tree(pos, mass, n_leaf, n_group)
    acc, _ = T.direct(eps)
    feat, lab, _, _ = T.mac_collect(eps, acc, THETA_LO, THETA_HI, stride=stride, cap=cap)
    y = torch.log10(torch.clamp(lab, min=1e-12))
    return feat.clone(), y.clone()


def init_params(seed: int) -> np.ndarray:
    """He-normal weights, zero biases, output bias at a typical log10 error."""
    rng = np.random.default_rng(seed)
    P = np.zeros(og.N_PARAMS, np.float32)
    P[0:768] = rng.normal(0, np.sqrt(2 / 12), 768)
    P[832:4928] = rng.normal(0, np.sqrt(2 / 64), 4096)
    P[4992:5056] = rng.normal(0, np.sqrt(1 / 64), 64)
    P[5056] = -4.0
    return P


# ------------------------------------------------------------------ checkpoints
#
# A training checkpoint is an .npz of plain arrays (no pickled objects):
# format version, FP32 master parameters, Adam moments, the Adam step count,
# the epochs done, the batch generator's state, the run's settings and a
# SHA-256 over all of them.  Loading checks the version, the shapes and the
# checksum; a resumed run continues exactly as the uninterrupted one.

CKPT_VERSION = 1
CKPT_KEYS = ("version", "params", "mom1", "mom2", "step", "epoch", "gen_state", "settings")


def _ckpt_digest(arrs) -> np.ndarray:
    import hashlib
    h = hashlib.sha256()
    for k in CKPT_KEYS:
        a = np.ascontiguousarray(arrs[k])
        h.update(k.encode())
        h.update(str(a.dtype).encode())
        h.update(np.asarray(a.shape, np.int64).tobytes())
        h.update(a.tobytes())
    return np.frombuffer(h.digest(), np.uint8).copy()


def pack_checkpoint(params, mom1, mom2, step, epoch, gen_state, settings) -> dict:
    """The arrays of a checkpoint (settings: [epochs, batch, lr, lr_final,
    tau, seed] as FP64)."""
    arrs = {
        "version": np.int64(CKPT_VERSION),
        "params": np.ascontiguousarray(params, np.float32),
        "mom1": np.ascontiguousarray(mom1, np.float32),
        "mom2": np.ascontiguousarray(mom2, np.float32),
        "step": np.int64(step),
        "epoch": np.int64(epoch),
        "gen_state": np.ascontiguousarray(gen_state, np.uint8),
        "settings": np.ascontiguousarray(settings, np.float64),
    }
    for k in ("params", "mom1", "mom2"):
        if arrs[k].shape != (og.N_PARAMS,):
            raise ValueError(f"checkpoint {k}: expected {og.N_PARAMS} values")
    arrs["sha256"] = _ckpt_digest(arrs)
    return arrs


def save_checkpoint(path, arrs) -> None:
    """Writes the checkpoint atomically (temporary file, then rename)."""
    tmp = path + ".tmp.npz"
    with open(tmp, "wb") as f:
        np.savez(f, **arrs)
    os.replace(tmp, path)


def load_checkpoint(path) -> dict:
    """Reads and verifies a checkpoint; ValueError if it is of another
    version, malformed or corrupted."""
    with np.load(path, allow_pickle=False) as z:
        missing = [k for k in CKPT_KEYS + ("sha256",) if k not in z.files]
        if missing:
            raise ValueError(f"{path}: not a training checkpoint (missing {missing})")
        arrs = {k: z[k] for k in CKPT_KEYS + ("sha256",)}
    if int(arrs["version"]) != CKPT_VERSION:
        raise ValueError(f"{path}: checkpoint version {int(arrs['version'])}, "
                         f"this code reads {CKPT_VERSION}")
    for k in ("params", "mom1", "mom2"):
        if arrs[k].dtype != np.float32 or arrs[k].shape != (og.N_PARAMS,):
            raise ValueError(f"{path}: {k} has the wrong type or shape")
    if not np.array_equal(arrs["sha256"], _ckpt_digest(arrs)):
        raise ValueError(f"{path}: checksum mismatch (corrupted checkpoint)")
    return arrs


def train(x, y, epochs=30, batch=4096, lr=1e-3, tau=PINBALL_TAU, seed=0, params=None,
          lr_final=1e-4, log=None, checkpoint=None, resume=None, stop_after=None):
    """Trains a network on (x, y) (CUDA tensors) with mini-batch Adam and a
    geometric learning-rate decay; returns the Mlp.  With `checkpoint`, the
    optimiser state is saved there after every epoch; with `resume`, training
    continues from that checkpoint (same data and settings required);
    `stop_after` ends the run after that many epochs in all."""
    import torch
    settings = np.array([epochs, batch, lr, lr_final, tau, seed], np.float64)
    m = og.Mlp(init_params(seed) if params is None else params)
    n = x.shape[0]
    gen = torch.Generator().manual_seed(seed)
    nb = max(1, n // batch)
    total = epochs * nb
    step, ep0 = 0, 0
    if resume is not None:
        ck = load_checkpoint(resume)
        if not np.array_equal(ck["settings"], settings):
            raise ValueError(f"{resume}: saved with other settings {ck['settings'].tolist()}")
        m.set_state(ck["params"], ck["mom1"], ck["mom2"])
        gen.set_state(torch.from_numpy(ck["gen_state"].copy()))
        step, ep0 = int(ck["step"]), int(ck["epoch"])
        if step != ep0 * nb:
            raise ValueError(f"{resume}: step {step} does not match {ep0} epochs of {nb} batches")
    last = epochs if stop_after is None else min(epochs, stop_after)
    for ep in range(ep0, last):
        perm = torch.randperm(n, generator=gen).cuda()
        run = 0.0
        for b in range(nb):
            idx = perm[b * batch:(b + 1) * batch]
            loss, _ = m.loss_grad(x[idx], y[idx], tau, want_grad=False)
            run += loss
            step += 1
            m.adam(step, lr=lr * (lr_final / lr) ** (step / total))
        if log:
            log(f"epoch {ep + 1}/{epochs} loss {run / nb:.5f}")
        if checkpoint is not None:
            m1, m2 = m.moments()
            save_checkpoint(checkpoint, pack_checkpoint(m.params(), m1, m2, step, ep + 1,
                                                        gen.get_state().numpy(), settings))
    return m


def merger_snapshots(n, seed, separation, impact, dt, every, count, theta, eps=W.TRAINING_EPS):
    """Positions and masses of a two-Plummer merger run on the GPU (the
    library's leapfrog, tree rebuilt every step): the initial conditions and
    then a snapshot every `every` steps, `count` in all."""
    pos, vel, m = W.plummer_pair_orbit(n, seed, separation, impact)
    S = og.Sim(pos, vel, m, 16, 64)
    S.run(theta, eps, dt, 0)
    out = [(pos, m)]
    for _ in range(1, count):
        S.run(theta, eps, dt, every)
        out.append((S.state()[0], m))
    S.close()
    return out


def training_data(stride=1, log=None, merger=False):
    """Band pairs of the static training sets and, with `merger`, of the
    merger run's snapshots."""
    import torch
    sets = [W.make_training(k) for k in range(len(W.TRAINING_SETS))]
    if merger:
        t0 = time.time()
        sets += merger_snapshots(**W.MERGER_SET)
        if log:
            log(f"merger run: {W.MERGER_SET['count']} snapshots in {time.time() - t0:.1f} s")
    xs, ys = [], []
    for k, (pos, mass) in enumerate(sets):
        t0 = time.time()
        x, y = collect(pos, mass, W.TRAINING_EPS, stride=stride)
        xs.append(x)
        ys.append(y)
        if log:
            log(f"set {k}: {x.shape[0]} pairs in {time.time() - t0:.1f} s")
    return torch.cat(xs), torch.cat(ys)


# ------------------------------------------------------------------ calibration

def p99_error(T, eps, sample, ref_acc, theta):
    """99th percentile of |a - a_ref| / |a_ref| over the sampled particles."""
    acc, _ = T.forces(theta, eps, with_pot=False)
    a = acc[sample].double()
    r = ref_acc.double()
    e = (a - r).norm(dim=1) / r.norm(dim=1)
    return float(np.quantile(e.cpu().numpy(), 0.99))


def bisect(f, lo, hi, target, increasing, iters=12, rtol=0.02):
    """x in [lo, hi] with f(x) ~ target (f monotone; `increasing` in x).
    Returns (x, f(x)) of the last point on the safe side of the target."""
    best = None
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        v = f(mid)
        if v <= target:
            best = (mid, v)
        if abs(v - target) <= rtol * target and v <= target:
            break
        if (v < target) == increasing:
            lo = mid
        else:
            hi = mid
    if best is None:
        x = lo if increasing else hi
        best = (x, f(x))
    return best


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    tr = sub.add_parser("train")
    tr.add_argument("--out", required=True)
    tr.add_argument("--epochs", type=int, default=30)
    tr.add_argument("--stride", type=int, default=1)
    tr.add_argument("--seed", type=int, default=0)
    tr.add_argument("--merger", action="store_true",
                    help="add the snapshots of a two-Plummer merger run to the static sets")
    tr.add_argument("--checkpoint", default=None,
                    help="save the optimiser state here after every epoch")
    tr.add_argument("--resume", default=None, help="continue from this checkpoint")
    a = ap.parse_args()
    if a.cmd == "train":
        x, y = training_data(a.stride, log=lambda s: print(s, flush=True), merger=a.merger)
        t0 = time.time()
        m = train(x, y, epochs=a.epochs, seed=a.seed, log=lambda s: print(s, flush=True),
                  checkpoint=a.checkpoint, resume=a.resume)
        print(f"trained on {x.shape[0]} pairs in {time.time() - t0:.1f} s", flush=True)
        np.save(a.out, m.params())


if __name__ == "__main__":
    main()
