"""TEST INFRASTRUCTURE ONLY: Python face of the FP64 CPU oracle.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It loads ``liboracle.so`` (built from ``oracle.cpp`` and
``oracle_mac.cpp`` by ``oracle/build_oracle.py``) and never touches the HIP
library under test.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# OCTGRAV_ORACLE_LIB selects another build of the same sources (the mutation
# tests load deliberately broken copies through it).
LIB_PATH = os.environ.get("OCTGRAV_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build_oracle
            build_oracle.build()
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.orc_direct.argtypes = [_f32p, _f32p, C.c_int64, C.c_float, vp, C.c_int64, _f64p, vp]
        L.orc_tree_build.restype = vp
        L.orc_tree_build.argtypes = [_f32p, _f32p, C.c_int64, C.c_int, C.c_int]
        L.orc_tree_free.argtypes = [vp]
        L.orc_tree_sizes.argtypes = [vp, _i64p]
        L.orc_tree_export.argtypes = [vp] + [vp] * 8
        L.orc_tree_cubes.argtypes = [vp, _f64p]
        L.orc_multipole_eval.argtypes = [_f32p, _f32p, C.c_int64, _f64p, C.c_float, C.c_int,
                                         _f64p]
        L.orc_mac_open.argtypes = [_f32p, _f32p, _f32p, C.c_float]
        for f in (L.orc_lists, L.orc_lists_brute):
            f.argtypes = [vp, C.c_float, vp, vp, vp, vp, vp, vp]
        L.orc_mac_open_com.argtypes = [_f32p, _f32p, _f32p, _f32p, C.c_float]
        L.orc_lists_com.argtypes = [vp, C.c_float, _f32p, C.c_int, vp, vp, vp, vp, vp, vp]
        L.orc_forces.argtypes = [vp, C.c_float, C.c_float, vp, C.c_int64, _f64p, vp]
        L.orc_counts.argtypes = [vp, C.c_float, _i64p]
        L.orc_leapfrog.argtypes = [_f64p, _f64p, _f64p, C.c_int64, C.c_double, C.c_double,
                                   C.c_int64, _f64p, _f64p, vp]
        L.orc_forces_lists.argtypes = [vp, C.c_float, _i64p, _i32p, _i64p, _i32p, vp, C.c_int64,
                                       _f64p, vp]
        L.orc_diagnostics.argtypes = [_f32p, _f64p, vp, C.c_int64, _f64p]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_mlp_params.restype = C.c_int
        L.orc_mac_features.argtypes = [vp, _i32p, _i32p, C.c_int64, _f32p]
        L.orc_mac_band.argtypes = [vp, C.c_float, C.c_float, vp, C.c_int64, vp, vp, C.c_int64,
                                   C.POINTER(C.c_int64)]
        L.orc_mac_labels.argtypes = [vp, _f64p, C.c_float, _i32p, _i32p, C.c_int64, _f64p]
        L.orc_mlp_forward.argtypes = [_f64p, _f32p, C.c_int64, C.c_int, _f64p]
        L.orc_mlp_loss_grad.argtypes = [_f64p, _f32p, _f64p, C.c_int64, C.c_double, C.c_int,
                                        C.POINTER(C.c_double), _f64p]
        L.orc_adam.argtypes = [_f64p, _f64p, _f64p, _f64p, C.c_int64, C.c_double, C.c_double,
                               C.c_double, C.c_double, C.c_int]
        L.orc_lists_learned.argtypes = [vp, C.c_float, C.c_float, C.c_float, C.c_float, C.c_float,
                                        vp, vp, vp, vp, C.c_int64, vp, vp, vp, vp,
                                        C.POINTER(C.c_int64), C.POINTER(C.c_int64), vp]
        L.orc_lists_groups.argtypes = [vp, C.c_float, vp, C.c_int64, vp, vp, vp, vp, vp, vp]
        L.orc_lists_learned_groups.argtypes = [vp, C.c_float, C.c_float, C.c_float, C.c_float,
                                               C.c_float, vp, vp, vp, vp, C.c_int64, vp,
                                               C.c_int64, vp, vp, vp, vp, C.POINTER(C.c_int64),
                                               C.POINTER(C.c_int64), vp]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _pos(pos):
    return np.ascontiguousarray(pos, dtype=np.float32).reshape(-1, 3)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_threads(k: int) -> None:
    """Threads of the oracle's parallel loops from now on."""
    lib().orc_set_threads(int(k))


def direct(pos, mass, eps, targets=None):
    """FP64 direct summation; returns (acc [nt,3], pot [nt]) for the targets."""
    pos = _pos(pos)
    mass = np.ascontiguousarray(mass, dtype=np.float32)
    n = pos.shape[0]
    tg = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = n if tg is None else tg.shape[0]
    acc = np.zeros((nt, 3))
    pot = np.zeros(nt)
    rc = lib().orc_direct(pos, mass, n, float(eps), _ptr(tg), nt, acc, _ptr(pot))
    assert rc == 0
    return acc, pot


def multipole_eval(pos, mass, target, eps, use_quad=True):
    """Field of a particle set's monopole(+quadrupole) at `target`: (acc[3], phi)."""
    out = np.zeros(4)
    lib().orc_multipole_eval(_pos(pos), np.ascontiguousarray(mass, dtype=np.float32),
                             _pos(pos).shape[0], np.asarray(target, np.float64), float(eps),
                             int(bool(use_quad)), out)
    return out[:3], out[3]


def log10_threshold(tau) -> float:
    """The FP32 threshold a network output is compared with under the learned
    test (accept iff output <= it): the FP64 log10 of the FP32 tau_pair,
    rounded once to FP32."""
    return float(np.float32(np.log10(np.float64(np.float32(tau)))))


def mac_open(gmin, gmax, geo, theta) -> bool:
    return bool(lib().orc_mac_open(np.asarray(gmin, np.float32), np.asarray(gmax, np.float32),
                                   np.asarray(geo, np.float32), float(theta)))


def mac_open_com(gmin, gmax, com, geo, theta) -> bool:
    """The centre-of-mass offset opening test of one cell for one group box."""
    f = lambda a: np.ascontiguousarray(a, np.float32)
    return bool(lib().orc_mac_open_com(f(gmin), f(gmax), f(com), f(geo), float(theta)))


class Tree:
    """The oracle's own octree (independent builder), with its FP64 moments."""

    def __init__(self, pos, mass, n_leaf=16, n_group=64):
        self.pos = _pos(pos)
        self.mass = np.ascontiguousarray(mass, dtype=np.float32)
        self.n = self.pos.shape[0]
        h = lib().orc_tree_build(self.pos, self.mass, self.n, int(n_leaf), int(n_group))
        if not h:
            raise ValueError("oracle tree build rejected its arguments")
        self._h = C.c_void_p(h)
        s = np.zeros(5, np.int64)
        lib().orc_tree_sizes(self._h, s)
        self.n_cells, self.n_leaves, self.n_groups, self.max_depth = (int(v) for v in s[1:])

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.orc_tree_free(self._h)
            self._h = None

    def export(self):
        nc, ng = self.n_cells, self.n_groups
        out = dict(order=np.zeros(self.n, np.int32), topo=np.zeros((nc, 4), np.int32),
                   geo=np.zeros((nc, 4), np.float32), mp=np.zeros((nc, 10)),
                   box=np.zeros((nc, 6)), depth=np.zeros(nc, np.int32),
                   groups=np.zeros(ng, np.int32), cube=np.zeros(4))
        lib().orc_tree_export(self._h, *(_ptr(out[k]) for k in
                                         ("order", "topo", "geo", "mp", "box", "depth", "groups",
                                          "cube")))
        return out

    def cubes(self):
        """[n_cells, 4]: octree cube corner xyz and side of every cell."""
        out = np.zeros((self.n_cells, 4))
        lib().orc_tree_cubes(self._h, out)
        return out

    def _lists(self, fn, theta, ng=None):
        ng = self.n_groups if ng is None else ng
        nc, nl = C.c_int64(), C.c_int64()
        if fn(self._h, float(theta), None, None, None, None, C.byref(nc), C.byref(nl)) != 0:
            raise ValueError("oracle lists rejected their arguments")
        c_off = np.zeros(ng + 1, np.int64)
        l_off = np.zeros(ng + 1, np.int64)
        c_ids = np.zeros(max(1, nc.value), np.int32)
        l_ids = np.zeros(max(1, nl.value), np.int32)
        fn(self._h, float(theta), _ptr(c_off), _ptr(c_ids), _ptr(l_off), _ptr(l_ids),
           C.byref(nc), C.byref(nl))
        return c_off, c_ids[:nc.value], l_off, l_ids[:nl.value]

    def lists(self, theta, groups=None):
        """(c_off, c_ids, l_off, l_ids): CSR lists per group from the stack walk
        (of the given group indices only, in that order, with `groups`)."""
        if groups is None:
            return self._lists(lib().orc_lists, theta)
        sel = np.ascontiguousarray(groups, np.int32)
        fn = lambda h, th, *a: lib().orc_lists_groups(h, th, _ptr(sel), sel.size, *a)
        return self._lists(fn, theta, sel.size)

    def lists_brute(self, theta):
        """The same lists from their walk-free characterisation (slow)."""
        return self._lists(lib().orc_lists_brute, theta)

    def lists_com(self, theta, com, brute=False):
        """Lists under the centre-of-mass offset test; com [n_cells, 3] is the
        FP32 centre of mass of every cell (the test's input)."""
        com = np.ascontiguousarray(com, np.float32).reshape(self.n_cells, 3)
        fn = lambda h, th, *a: lib().orc_lists_com(h, th, com, int(brute), *a)
        return self._lists(fn, theta)

    def counts(self, theta):
        """[n_groups, 3]: |C_g|, |L_g|, source particles in L_g."""
        out = np.zeros((self.n_groups, 3), np.int64)
        lib().orc_counts(self._h, float(theta), out)
        return out

    # ---- learned acceptance criterion (oracle_mac.cpp)
    def mac_features(self, g, c):
        g = np.ascontiguousarray(g, np.int32)
        c = np.ascontiguousarray(c, np.int32)
        out = np.zeros((g.shape[0], 12), np.float32)
        lib().orc_mac_features(self._h, g, c, g.shape[0], out)
        return out

    def mac_band(self, theta_lo=0.3, theta_hi=1.0, groups=None):
        """(group index, cell id) band candidates of the theta_lo walks."""
        sel = None if groups is None else np.ascontiguousarray(groups, np.int32)
        n = C.c_int64()
        lib().orc_mac_band(self._h, theta_lo, theta_hi, _ptr(sel), 0 if sel is None else sel.size,
                           None, None, 0, C.byref(n))
        g = np.zeros(max(1, n.value), np.int32)
        c = np.zeros(max(1, n.value), np.int32)
        lib().orc_mac_band(self._h, theta_lo, theta_hi, _ptr(sel), 0 if sel is None else sel.size,
                           _ptr(g), _ptr(c), n.value, C.byref(n))
        return g[:n.value], c[:n.value]

    def mac_labels(self, acc_direct, eps, g, c):
        g = np.ascontiguousarray(g, np.int32)
        c = np.ascontiguousarray(c, np.int32)
        out = np.zeros(g.shape[0])
        lib().orc_mac_labels(self._h, np.ascontiguousarray(acc_direct, np.float64), float(eps),
                             g, c, g.shape[0], out)
        return out

    def lists_learned(self, theta, theta_lo, theta_hi, log10_tau, budget, params=None,
                      replay=None, groups=None):
        """Lists under the learned criterion (network `params`, or a replay
        (g, c, score) table sorted by (g, c)); returns lists + fell_back
        (of the given group indices only, in that order, with `groups`)."""
        P = None if params is None else np.ascontiguousarray(params, np.float64)
        if replay is not None:
            rg, rc, rs = (np.ascontiguousarray(replay[0], np.int32),
                          np.ascontiguousarray(replay[1], np.int32),
                          np.ascontiguousarray(replay[2], np.float32))
            nr = rg.shape[0]
        else:
            rg = rc = rs = None
            nr = 0
        nc, nl = C.c_int64(), C.c_int64()
        args = (self._h, float(theta), float(theta_lo), float(theta_hi), float(log10_tau),
                float(budget), _ptr(P), _ptr(rg), _ptr(rc), _ptr(rs), nr)
        if groups is None:
            fn, ng = lib().orc_lists_learned, self.n_groups
        else:
            sel = np.ascontiguousarray(groups, np.int32)
            args = args + (_ptr(sel), sel.size)
            fn, ng = lib().orc_lists_learned_groups, sel.size
        rc_ = fn(*args, None, None, None, None, C.byref(nc), C.byref(nl), None)
        if rc_ == -2:
            raise ValueError("replay table misses a band candidate")
        if rc_ != 0:
            raise ValueError("oracle learned lists rejected their arguments")
        c_off = np.zeros(ng + 1, np.int64)
        l_off = np.zeros(ng + 1, np.int64)
        c_ids = np.zeros(max(1, nc.value), np.int32)
        l_ids = np.zeros(max(1, nl.value), np.int32)
        fb = np.zeros(ng, np.int32)
        fn(*args, _ptr(c_off), _ptr(c_ids), _ptr(l_off), _ptr(l_ids), C.byref(nc), C.byref(nl),
           _ptr(fb))
        return (c_off, c_ids[:nc.value], l_off, l_ids[:nl.value]), fb

    def forces(self, theta, eps, groups=None):
        """FP64 same-tree forces; (acc [n,3], pot [n]) by input index.  With
        `groups`, only those groups' particles are filled (others are NaN)."""
        acc = np.full((self.n, 3), np.nan)
        pot = np.full(self.n, np.nan)
        sel = None if groups is None else np.ascontiguousarray(groups, dtype=np.int32)
        rc = lib().orc_forces(self._h, float(theta), float(eps), _ptr(sel),
                              0 if sel is None else sel.shape[0], acc, _ptr(pot))
        assert rc == 0
        return acc, pot


def _forces_lists(self, lists, eps, groups=None):
    """FP64 forces from given CSR lists (c_off, c_ids, l_off, l_ids)."""
    c_off, c_ids, l_off, l_ids = (np.ascontiguousarray(lists[0], np.int64),
                                  np.ascontiguousarray(lists[1], np.int32),
                                  np.ascontiguousarray(lists[2], np.int64),
                                  np.ascontiguousarray(lists[3], np.int32))
    if c_ids.size == 0:
        c_ids = np.zeros(1, np.int32)
    if l_ids.size == 0:
        l_ids = np.zeros(1, np.int32)
    acc = np.full((self.n, 3), np.nan)
    pot = np.full(self.n, np.nan)
    sel = None if groups is None else np.ascontiguousarray(groups, dtype=np.int32)
    rc = lib().orc_forces_lists(self._h, float(eps), c_off, c_ids, l_off, l_ids, _ptr(sel),
                                0 if sel is None else sel.shape[0], acc, _ptr(pot))
    assert rc == 0
    return acc, pot


Tree.forces_lists = _forces_lists


def leapfrog(pos, vel, mass, eps, dt, steps):
    """FP64 kick-drift-kick leapfrog with direct-sum forces: (pos, vel,
    energies [steps + 1, 2] = (K, W))."""
    pos = np.ascontiguousarray(pos, np.float64).reshape(-1, 3)
    vel = np.ascontiguousarray(vel, np.float64).reshape(-1, 3)
    mass = np.ascontiguousarray(mass, np.float64)
    n = pos.shape[0]
    po, vo = np.zeros_like(pos), np.zeros_like(vel)
    en = np.zeros((steps + 1, 2))
    assert lib().orc_leapfrog(pos, vel, mass, n, float(eps), float(dt), int(steps), po, vo,
                              _ptr(en)) == 0
    return po, vo, en


def mlp_params() -> int:
    return int(lib().orc_mlp_params())


def mlp_forward(params, x, round_bf16=True):
    x = np.ascontiguousarray(x, np.float32).reshape(-1, 12)
    y = np.zeros(x.shape[0])
    lib().orc_mlp_forward(np.ascontiguousarray(params, np.float64), x, x.shape[0],
                          int(bool(round_bf16)), y)
    return y


def mlp_loss_grad(params, x, target, tau=0.9, round_bf16=True):
    x = np.ascontiguousarray(x, np.float32).reshape(-1, 12)
    g = np.zeros(mlp_params())
    loss = C.c_double()
    lib().orc_mlp_loss_grad(np.ascontiguousarray(params, np.float64), x,
                            np.ascontiguousarray(target, np.float64), x.shape[0], float(tau),
                            int(bool(round_bf16)), C.byref(loss), g)
    return loss.value, g


def adam_step(params, m, v, grad, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam step on float64 arrays (step counted from 1)."""
    lib().orc_adam(params, m, v, np.ascontiguousarray(grad, np.float64), params.shape[0],
                   lr, b1, b2, eps, int(step))


def diagnostics(mass, acc, pot):
    """FP64 (sum m a [3], 1/2 sum m phi)."""
    mass = np.ascontiguousarray(mass, dtype=np.float32)
    acc = np.ascontiguousarray(acc, dtype=np.float64)
    p = None if pot is None else np.ascontiguousarray(pot, dtype=np.float64)
    out = np.zeros(4)
    lib().orc_diagnostics(mass, acc, _ptr(p), mass.shape[0], out)
    return out[:3], out[3]


def rel_err(a, a_ref):
    """Per-particle relative error |a - a_ref| / |a_ref| (Sec. 3.1)."""
    a = np.asarray(a, np.float64)
    a_ref = np.asarray(a_ref, np.float64)
    if a.ndim == 2:
        return np.linalg.norm(a - a_ref, axis=1) / np.linalg.norm(a_ref, axis=1)
    return np.abs(a - a_ref) / np.abs(a_ref)


def percentile_nr(x, q):
    """Nearest-rank percentile: the ceil(q*n)-th smallest value (q in (0,1])."""
    x = np.sort(np.asarray(x).ravel())
    k = max(1, int(np.ceil(q * x.size - 1e-12)))
    return float(x[k - 1])


def err_summary(a, a_ref):
    e = rel_err(a, a_ref)
    return dict(p50=percentile_nr(e, 0.5), p90=percentile_nr(e, 0.9),
                p99=percentile_nr(e, 0.99), max=float(e.max()))
