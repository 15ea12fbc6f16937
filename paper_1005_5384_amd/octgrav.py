"""Thin Python binding of the C ABI in include/octgrav.h (ctypes).

Argument marshalling only: every step of the force computation runs in the
HIP library.  PyTorch provides device memory and the stream.  Loading fails
loudly when the built library is missing; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# OCTGRAV_LIB selects another build of the same sources (the sanitizer build
# that the CPU checks of the host code load).
LIB_PATH = os.environ.get("OCTGRAV_LIB") or os.path.join(HERE, "libocgrav.so")

OK, EINVAL, ENOMEM, EHIP, ECAPACITY = 0, -1, -2, -3, -4
BUILD_HOST_ONLY = 1
BUILD_DEVICE = 2
PLAIN_SUM = 1
TIMED = 2
TWO_PASS = 4
FUSED_BLOCK = 8
FUSED_WAVE = 16
MAC_COM = 32  # centre-of-mass offset opening test (fused wave path, theta <= 0.57)
PATHS = {None: 0, "two_pass": TWO_PASS, "fused_block": FUSED_BLOCK, "fused_wave": FUSED_WAVE}

_lib = None


class OctgravError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"octgrav error {code}: {msg}")
        self.code = code


class Stats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("n", "n_cells", "n_leaves", "n_groups", "max_depth",
                                         "max_level_cells", "n_work", "n_leaf", "n_group")]


class TreeView(C.Structure):
    _fields_ = [("perm", C.c_void_p), ("topo", C.c_void_p), ("geo", C.c_void_p),
                ("mp", C.c_void_p), ("mp64", C.c_void_p), ("box", C.c_void_p),
                ("depth", C.c_void_p), ("groups", C.c_void_p), ("cube", C.c_void_p)]


EXPORTED = ["octgrav_build_tree", "octgrav_build_tree_ex", "octgrav_forces", "octgrav_forces_ex",
            "octgrav_forces_noalloc",
            "octgrav_free", "octgrav_last_error", "octgrav_set_stream", "octgrav_tree_stats",
            "octgrav_export_tree", "octgrav_lists", "octgrav_lists_ex", "octgrav_lists_select",
            "octgrav_diagnostics",
            "octgrav_last_counts", "octgrav_group_counts", "octgrav_direct", "octgrav_mac_collect",
            "octgrav_last_timings", "octgrav_mlp_create", "octgrav_mlp_free",
            "octgrav_mlp_set_stream", "octgrav_mlp_set_params", "octgrav_mlp_get_params",
            "octgrav_mlp_get_moments", "octgrav_mlp_set_state",
            "octgrav_mlp_forward", "octgrav_mlp_loss_grad", "octgrav_mlp_adam", "octgrav_set_mac",
            "octgrav_mac_stats", "octgrav_mac_trace", "octgrav_mac_trace_select", "octgrav_sim_create", "octgrav_sim_free",
            "octgrav_sim_set_stream", "octgrav_sim_run", "octgrav_sim_energy", "octgrav_sim_state",
            "octgrav_sim_timings"]

N_PARAMS = 12 * 64 + 64 + 64 * 64 + 64 + 64 + 1  # 5057


def lib():
    """The loaded libocgrav.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        # torch ships its own HIP runtime under the same soname; loading torch
        # first makes this library bind to that one runtime, so torch's
        # streams and allocations are valid handles here.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, i64, i32, f32 = C.c_void_p, C.c_int64, C.c_int32, C.c_float
        L.octgrav_build_tree.restype = vp
        L.octgrav_build_tree.argtypes = [vp, vp, i64, i32]
        L.octgrav_build_tree_ex.restype = vp
        L.octgrav_build_tree_ex.argtypes = [vp, vp, i64, i32, i32, C.c_uint32]
        L.octgrav_forces.argtypes = [vp, f32, f32, vp, vp]
        L.octgrav_forces_ex.argtypes = [vp, f32, f32, vp, vp, C.c_uint32]
        L.octgrav_forces_noalloc.argtypes = [vp, f32, f32, vp, vp]
        L.octgrav_free.argtypes = [vp]
        L.octgrav_free.restype = None
        L.octgrav_last_error.restype = C.c_char_p
        L.octgrav_set_stream.argtypes = [vp, vp]
        L.octgrav_tree_stats.argtypes = [vp, C.POINTER(Stats)]
        L.octgrav_export_tree.argtypes = [vp, C.POINTER(TreeView)]
        L.octgrav_lists.argtypes = [vp, f32, vp, vp, vp, vp, C.POINTER(i64), C.POINTER(i64)]
        L.octgrav_lists_ex.argtypes = [vp, f32, C.c_uint32, vp, vp, vp, vp, C.POINTER(i64),
                                       C.POINTER(i64)]
        L.octgrav_lists_select.argtypes = [vp, f32, C.c_uint32, vp, i64, vp, vp, vp, vp,
                                           C.POINTER(i64), C.POINTER(i64)]
        L.octgrav_diagnostics.argtypes = [vp, vp, vp]
        L.octgrav_last_counts.argtypes = [vp, vp]
        L.octgrav_group_counts.argtypes = [vp, vp]
        L.octgrav_last_timings.argtypes = [vp, vp]
        L.octgrav_direct.argtypes = [vp, f32, vp, i64, vp, vp]
        L.octgrav_mac_collect.argtypes = [vp, f32, f32, f32, vp, i32, vp, vp, vp, vp, i64,
                                          C.POINTER(i64)]
        L.octgrav_mlp_create.restype = vp
        L.octgrav_mlp_create.argtypes = [vp]
        L.octgrav_mlp_free.argtypes = [vp]
        L.octgrav_mlp_free.restype = None
        L.octgrav_mlp_set_stream.argtypes = [vp, vp]
        L.octgrav_mlp_set_params.argtypes = [vp, vp]
        L.octgrav_mlp_get_params.argtypes = [vp, vp]
        L.octgrav_mlp_get_moments.argtypes = [vp, vp, vp]
        L.octgrav_mlp_set_state.argtypes = [vp, vp, vp, vp]
        L.octgrav_mlp_forward.argtypes = [vp, vp, i64, vp]
        L.octgrav_mlp_loss_grad.argtypes = [vp, vp, vp, i64, f32, vp, vp]
        L.octgrav_mlp_adam.argtypes = [vp, f32, f32, f32, f32, i32]
        L.octgrav_set_mac.argtypes = [vp, vp, f32, f32, f32, f32]
        L.octgrav_mac_stats.argtypes = [vp, vp]
        L.octgrav_mac_trace.argtypes = [vp, f32, vp, vp, vp, i64, C.POINTER(i64), vp]
        L.octgrav_mac_trace_select.argtypes = [vp, f32, vp, i64, vp, vp, vp, i64, C.POINTER(i64),
                                               vp]
        L.octgrav_sim_create.restype = vp
        L.octgrav_sim_create.argtypes = [vp, vp, vp, i64, i32, i32]
        L.octgrav_sim_free.argtypes = [vp]
        L.octgrav_sim_free.restype = None
        L.octgrav_sim_set_stream.argtypes = [vp, vp]
        L.octgrav_sim_run.argtypes = [vp, f32, f32, f32, i32]
        L.octgrav_sim_energy.argtypes = [vp, vp]
        L.octgrav_sim_state.argtypes = [vp, vp, vp, vp]
        L.octgrav_sim_timings.argtypes = [vp, vp]
        _lib = L
    return _lib


def last_error() -> str:
    return lib().octgrav_last_error().decode()


def _check(rc):
    if rc != OK:
        raise OctgravError(rc, last_error())


def _ptr(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


class Tree:
    """A built tree (host FP64 build + device upload) and its force calls."""

    def __init__(self, pos, mass, n_leaf=16, n_group=64, host_only=False, device_build=False):
        pos = np.ascontiguousarray(pos, dtype=np.float32).reshape(-1, 3)
        mass = np.ascontiguousarray(mass, dtype=np.float32).reshape(-1)
        self.n = pos.shape[0]
        if mass.shape[0] != self.n:
            raise ValueError("pos and mass disagree on n")
        flags = (BUILD_HOST_ONLY if host_only else 0) | (BUILD_DEVICE if device_build else 0)
        h = lib().octgrav_build_tree_ex(_ptr(pos), _ptr(mass), self.n, int(n_leaf), int(n_group),
                                        flags)
        if not h:
            raise OctgravError(EINVAL, last_error())
        self._h = C.c_void_p(h)
        s = Stats()
        _check(lib().octgrav_tree_stats(self._h, C.byref(s)))
        self.stats = {k: int(getattr(s, k)) for k, _ in Stats._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.octgrav_free(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def _bind_stream(self):
        import torch
        _check(lib().octgrav_set_stream(self._h, C.c_void_p(torch.cuda.current_stream().cuda_stream)))

    def forces(self, theta, eps, acc=None, pot=None, plain=False, timed=False, with_pot=True,
               two_pass=False, path=None, com=False):
        """(acc [n,3], pot [n]) as float32 torch tensors on the current device;
        com=True selects the centre-of-mass offset opening test."""
        import torch
        if acc is None:
            acc = torch.empty((self.n, 3), dtype=torch.float32, device="cuda")
        if pot is None and with_pot:
            pot = torch.empty(self.n, dtype=torch.float32, device="cuda")
        for t in (acc, pot):
            if t is not None and (t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous()):
                raise ValueError("acc/pot must be contiguous float32 CUDA tensors")
        if acc.numel() != 3 * self.n or (pot is not None and pot.numel() != self.n):
            raise ValueError("acc must hold n*3 and pot n elements")
        self._bind_stream()
        flags = (PLAIN_SUM if plain else 0) | (TIMED if timed else 0) | (TWO_PASS if two_pass else 0)
        flags |= PATHS[path] | (MAC_COM if com else 0)
        _check(lib().octgrav_forces_ex(self._h, float(theta), float(eps), C.c_void_p(acc.data_ptr()),
                                       None if pot is None else C.c_void_p(pot.data_ptr()), flags))
        return acc, pot

    def forces_noalloc(self, theta, eps, acc, pot=None):
        """octgrav_forces_noalloc into the caller's acc [n,3] (and pot [n], or
        None): contiguous float32 CUDA tensors; the call allocates nothing."""
        import torch
        for t in (acc, pot):
            if t is not None and (t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous()):
                raise ValueError("acc/pot must be contiguous float32 CUDA tensors")
        if acc.numel() != 3 * self.n or (pot is not None and pot.numel() != self.n):
            raise ValueError("acc must hold n*3 and pot n elements")
        self._bind_stream()
        _check(lib().octgrav_forces_noalloc(self._h, float(theta), float(eps),
                                            C.c_void_p(acc.data_ptr()),
                                            None if pot is None else C.c_void_p(pot.data_ptr())))
        return acc, pot

    def lists(self, theta, two_pass=False, path=None, com=False, groups=None):
        """(c_off, c_ids, l_off, l_ids) numpy CSR lists built by the GPU walk of
        the selected path (default: the force path's default for theta) and
        opening test (com=True: the centre-of-mass offset test); with `groups`
        (group indices), only those groups' lists, in that order."""
        self._bind_stream()
        fl = (TWO_PASS if two_pass else 0) | PATHS[path] | (MAC_COM if com else 0)
        nc, nl = C.c_int64(), C.c_int64()
        if groups is None:
            ng = self.stats["n_groups"]
            fn = lambda *a: lib().octgrav_lists_ex(self._h, float(theta), fl, *a)
        else:
            sel = np.ascontiguousarray(groups, np.int32)
            ng = sel.size
            fn = lambda *a: lib().octgrav_lists_select(self._h, float(theta), fl, _ptr(sel),
                                                       sel.size, *a)
        _check(fn(None, None, None, None, C.byref(nc), C.byref(nl)))
        c_off = np.zeros(ng + 1, np.int64)
        l_off = np.zeros(ng + 1, np.int64)
        c_ids = np.zeros(max(1, nc.value), np.int32)
        l_ids = np.zeros(max(1, nl.value), np.int32)
        _check(fn(_ptr(c_off), _ptr(c_ids), _ptr(l_off), _ptr(l_ids), C.byref(nc), C.byref(nl)))
        return c_off, c_ids[:nc.value], l_off, l_ids[:nl.value]

    def direct(self, eps, targets=None):
        """FP32 compensated GPU direct sum: (acc [nt,3], pot [nt]) torch tensors
        for the caller indices `targets` (a sequence or tensor; None = all)."""
        import torch
        self._bind_stream()
        tg = None
        if targets is not None:
            tg = torch.as_tensor(targets, dtype=torch.int32, device="cuda").contiguous()
        nt = self.n if tg is None else tg.numel()
        acc = torch.empty((nt, 3), dtype=torch.float32, device="cuda")
        pot = torch.empty(nt, dtype=torch.float32, device="cuda")
        if nt == 0:  # an empty tensor has no address; NULL targets would mean "all"
            return acc, pot
        _check(lib().octgrav_direct(self._h, float(eps),
                                    None if tg is None else C.c_void_p(tg.data_ptr()), nt,
                                    C.c_void_p(acc.data_ptr()), C.c_void_p(pot.data_ptr())))
        return acc, pot

    def mac_collect(self, eps, acc_direct, theta_lo=0.3, theta_hi=1.0, stride=1, cap=1 << 22):
        """Band pairs' features [k,12], labels [k], group ids, cell ids (torch)."""
        import torch
        self._bind_stream()
        feat = torch.empty((cap, 12), dtype=torch.float32, device="cuda")
        lab = torch.empty(cap, dtype=torch.float32, device="cuda")
        gid = torch.empty(cap, dtype=torch.int32, device="cuda")
        cid = torch.empty(cap, dtype=torch.int32, device="cuda")
        n = C.c_int64()
        acc_direct = acc_direct.contiguous()
        _check(lib().octgrav_mac_collect(self._h, float(theta_lo), float(theta_hi), float(eps),
                                         C.c_void_p(acc_direct.data_ptr()), int(stride),
                                         C.c_void_p(feat.data_ptr()), C.c_void_p(lab.data_ptr()),
                                         C.c_void_p(gid.data_ptr()), C.c_void_p(cid.data_ptr()),
                                         cap, C.byref(n)))
        k = n.value
        return feat[:k], lab[:k], gid[:k], cid[:k]

    def set_mac(self, mlp=None, theta_lo=0.3, theta_hi=1.0, tau_pair=1e-3, budget=float("inf")):
        """Learned acceptance criterion with network `mlp` (an Mlp), or the
        opening angle alone (mlp=None)."""
        _check(lib().octgrav_set_mac(self._h, None if mlp is None else mlp._h, float(theta_lo),
                                     float(theta_hi), float(tau_pair), float(budget)))

    def mac_stats(self):
        out = np.zeros(2, np.int64)
        _check(lib().octgrav_mac_stats(self._h, _ptr(out)))
        return dict(band=int(out[0]), fell_back=int(out[1]))

    def mac_trace(self, theta, groups=None):
        """(off [ng+1], cells, scores, fell_back [ng]) of the learned walks;
        with `groups` (group indices), only those groups', in that order."""
        self._bind_stream()
        if groups is None:
            ng = self.stats["n_groups"]
            fn = lambda *a: lib().octgrav_mac_trace(self._h, float(theta), *a)
        else:
            sel = np.ascontiguousarray(groups, np.int32)
            ng = sel.size
            fn = lambda *a: lib().octgrav_mac_trace_select(self._h, float(theta), _ptr(sel),
                                                           sel.size, *a)
        off = np.zeros(ng + 1, np.int64)
        fb = np.zeros(ng, np.int32)
        n = C.c_int64()
        _check(fn(_ptr(off), None, None, 0, C.byref(n), _ptr(fb)))
        cells = np.zeros(max(1, n.value), np.int32)
        scores = np.zeros(max(1, n.value), np.float32)
        _check(fn(_ptr(off), _ptr(cells), _ptr(scores), cells.size, C.byref(n), _ptr(fb)))
        return off, cells[:n.value], scores[:n.value], fb

    def export(self):
        s = self.stats
        n, nc, ng = s["n"], s["n_cells"], s["n_groups"]
        out = dict(perm=np.zeros(n, np.int32), topo=np.zeros((nc, 4), np.int32),
                   geo=np.zeros((nc, 4), np.float32), mp=np.zeros((nc, 12), np.float32),
                   mp64=np.zeros((nc, 10)), box=np.zeros((nc, 6)), depth=np.zeros(nc, np.int32),
                   groups=np.zeros(ng, np.int32), cube=np.zeros(4))
        v = TreeView(*(_ptr(out[k]) for k, _ in TreeView._fields_))
        _check(lib().octgrav_export_tree(self._h, C.byref(v)))
        return out

    def diagnostics(self):
        """(momentum sum m a [3], W = 1/2 sum m phi) in FP64 from the last forces call."""
        mom = np.zeros(3)
        w = np.zeros(1)
        _check(lib().octgrav_diagnostics(self._h, _ptr(mom), _ptr(w)))
        return mom, float(w[0])

    def last_counts(self):
        out = np.zeros(4, np.int64)
        _check(lib().octgrav_last_counts(self._h, _ptr(out)))
        return dict(n_c=int(out[0]), n_l=int(out[1]), n_pc=int(out[2]), n_pp=int(out[3]))

    def group_counts(self):
        """Per-group (|C_g|, |L_g|, n_src(L_g), flags) of the last forces/lists
        call, int32 [n_groups, 4] in the handle's group order."""
        out = np.zeros((self.stats["n_groups"], 4), np.int32)
        _check(lib().octgrav_group_counts(self._h, _ptr(out)))
        return out

    def last_timings(self):
        out = np.zeros(6)
        _check(lib().octgrav_last_timings(self._h, _ptr(out)))
        return dict(zip(("walk_count", "offsets", "walk_write", "eval", "diag", "total"),
                        out.tolist()))


class Mlp:
    """The learned criterion's network on the device (FP32 master parameters,
    Adam moments, BF16 inference image)."""

    def __init__(self, params=None):
        p = None
        if params is not None:
            p = np.ascontiguousarray(params, dtype=np.float32)
            if p.size != N_PARAMS:
                raise ValueError(f"need {N_PARAMS} parameters")
        h = lib().octgrav_mlp_create(_ptr(p))
        if not h:
            raise OctgravError(ENOMEM, last_error())
        self._h = C.c_void_p(h)

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.octgrav_mlp_free(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def _bind_stream(self):
        import torch
        _check(lib().octgrav_mlp_set_stream(self._h,
                                            C.c_void_p(torch.cuda.current_stream().cuda_stream)))

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != N_PARAMS:
            raise ValueError(f"need {N_PARAMS} parameters")
        self._bind_stream()
        _check(lib().octgrav_mlp_set_params(self._h, _ptr(p)))

    def params(self):
        p = np.zeros(N_PARAMS, np.float32)
        self._bind_stream()
        _check(lib().octgrav_mlp_get_params(self._h, _ptr(p)))
        return p

    def moments(self):
        """Adam's (first, second) moments, [5057] FP32 each."""
        m1 = np.zeros(N_PARAMS, np.float32)
        m2 = np.zeros(N_PARAMS, np.float32)
        self._bind_stream()
        _check(lib().octgrav_mlp_get_moments(self._h, _ptr(m1), _ptr(m2)))
        return m1, m2

    def set_state(self, params, mom1, mom2):
        """Restores parameters and Adam moments (a training checkpoint)."""
        a = [np.ascontiguousarray(v, dtype=np.float32) for v in (params, mom1, mom2)]
        if any(v.size != N_PARAMS for v in a):
            raise ValueError(f"need {N_PARAMS} values each")
        self._bind_stream()
        _check(lib().octgrav_mlp_set_state(self._h, *(_ptr(v) for v in a)))

    def forward(self, x):
        """x: float32 CUDA tensor [b, 12] -> y [b]."""
        import torch
        x = x.to(dtype=torch.float32).contiguous()
        y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        if x.shape[0] == 0:
            return y
        self._bind_stream()
        _check(lib().octgrav_mlp_forward(self._h, C.c_void_p(x.data_ptr()), x.shape[0],
                                         C.c_void_p(y.data_ptr())))
        return y

    def loss_grad(self, x, target, tau=0.9, want_grad=True):
        """(mean pinball loss, gradient [5057] numpy or None)."""
        import torch
        x = x.to(dtype=torch.float32).contiguous()
        target = target.to(dtype=torch.float32).contiguous()
        loss = np.zeros(1)
        g = np.zeros(N_PARAMS, np.float32) if want_grad else None
        self._bind_stream()
        _check(lib().octgrav_mlp_loss_grad(self._h, C.c_void_p(x.data_ptr()),
                                           C.c_void_p(target.data_ptr()), x.shape[0], float(tau),
                                           _ptr(loss), _ptr(g)))
        return float(loss[0]), g

    def adam(self, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self._bind_stream()
        _check(lib().octgrav_mlp_adam(self._h, float(lr), float(beta1), float(beta2), float(eps),
                                      int(step)))


class Sim:
    """A particle system on the device advanced with kick-drift-kick leapfrog,
    the tree rebuilt on the GPU every step."""

    def __init__(self, pos, vel, mass, n_leaf=16, n_group=64):
        pos = np.ascontiguousarray(pos, dtype=np.float32).reshape(-1, 3)
        vel = np.ascontiguousarray(vel, dtype=np.float32).reshape(-1, 3)
        mass = np.ascontiguousarray(mass, dtype=np.float32).reshape(-1)
        self.n = pos.shape[0]
        if vel.shape[0] != self.n or mass.shape[0] != self.n:
            raise ValueError("pos, vel and mass disagree on n")
        h = lib().octgrav_sim_create(_ptr(pos), _ptr(vel), _ptr(mass), self.n, int(n_leaf),
                                     int(n_group))
        if not h:
            raise OctgravError(EINVAL, last_error())
        self._h = C.c_void_p(h)

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.octgrav_sim_free(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def _bind_stream(self):
        import torch
        _check(lib().octgrav_sim_set_stream(self._h,
                                            C.c_void_p(torch.cuda.current_stream().cuda_stream)))

    def run(self, theta, eps, dt, steps):
        self._bind_stream()
        _check(lib().octgrav_sim_run(self._h, float(theta), float(eps), float(dt), int(steps)))

    def energy(self):
        """dict(K, W, E, P=[px, py, pz]) in FP64."""
        out = np.zeros(6)
        self._bind_stream()
        _check(lib().octgrav_sim_energy(self._h, _ptr(out)))
        return dict(K=out[0], W=out[1], E=out[2], P=out[3:6].copy())

    def state(self):
        pos = np.zeros((self.n, 3), np.float32)
        vel = np.zeros((self.n, 3), np.float32)
        acc = np.zeros((self.n, 3), np.float32)
        _check(lib().octgrav_sim_state(self._h, _ptr(pos), _ptr(vel), _ptr(acc)))
        return pos, vel, acc

    def timings(self):
        out = np.zeros(3)
        _check(lib().octgrav_sim_timings(self._h, _ptr(out)))
        return dict(step_ms=out[0], build_ms=out[1], forces_ms=out[2])
