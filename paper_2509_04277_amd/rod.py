"""Thin ctypes binding of libcorde_rod.so (C ABI in include/rod.h): argument marshalling only.

Every step of the rod method runs in the library's HIP kernels; this module converts Python
descriptions (``workloads.RodSpec``) to ``rod_params``, passes host numpy arrays or device
torch tensors by pointer, and raises ``RodError`` on a non-OK status.  There is no CPU
fallback: importing works anywhere, creating a handle needs the built library and a HIP device.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcorde_rod.so")

ROD_OK = 0
STATUS = {0: "ROD_OK", -1: "ROD_E_INVALID", -2: "ROD_E_NOMEM", -3: "ROD_E_DEVICE",
          -4: "ROD_E_UNSTABLE", -5: "ROD_E_ORDER", -6: "ROD_E_UNSUPPORTED", -7: "ROD_E_TIMEOUT"}


class RodError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


_DP = C.POINTER(C.c_double)
_FP = C.c_void_p


class rod_params(C.Structure):
    _fields_ = [
        ("n_elements", C.c_int32), ("inextensible", C.c_int32),
        ("n_constraint_iters", C.c_int32), ("clamp_end0", C.c_int32),
        ("dt", C.c_double), ("gravity", C.c_double * 3),
        ("damping_lin", C.c_double), ("damping_ang", C.c_double),
        ("poisson", C.c_double), ("density", C.c_double),
        ("kp_scale", C.c_double), ("bend_scale", C.c_double), ("twist_scale", C.c_double),
        ("seg_len", _DP), ("radius", _DP), ("young", _DP), ("u_hat", _DP),
        ("f_ext", _DP), ("tau_ext", _DP),
        ("clamp_x0", C.c_double * 3), ("clamp_q0", C.c_double * 4),
        ("clamp_amp", C.c_double * 3), ("clamp_twist_amp", C.c_double),
        ("clamp_twist_axis", C.c_double * 3), ("clamp_freq", C.c_double),
        ("clamp_phase_x", C.c_double), ("clamp_phase_twist", C.c_double),
        ("damping_int", C.c_double),
    ]


class rod_tuning(C.Structure):
    _fields_ = [("waves", C.c_int32), ("elems_per_lane", C.c_int32),
                ("steps_per_launch", C.c_int32), ("us_per_step", C.c_float)]


class rod_haptic_force(C.Structure):
    _fields_ = [("f", C.c_double * 3), ("step", C.c_uint32), ("pose", C.c_uint32),
                ("n_steps", C.c_uint32)]


# Exported entry points and their argument types (same names as include/rod.h).
_SIGS = {
    "rod_create": (C.c_int, [C.POINTER(rod_params), C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]),
    "rod_destroy": (C.c_int, [C.c_void_p]),
    "rod_set_state": (C.c_int, [C.c_void_p, _FP, _FP, _FP, _FP, C.c_int32, C.c_double]),
    "rod_get_state": (C.c_int, [C.c_void_p, _FP, _FP, _FP, _FP, C.c_int32]),
    "rod_step": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "rod_set_clamp": (C.c_int, [C.c_void_p, C.c_int32, _DP, _DP]),
    "rod_sync": (C.c_int, [C.c_void_p]),
    "rod_get_time": (C.c_int, [C.c_void_p, _DP, C.POINTER(C.c_int64)]),
    "rod_set_tuning": (C.c_int, [C.c_void_p, C.POINTER(rod_tuning)]),
    "rod_get_tuning": (C.c_int, [C.c_void_p, C.POINTER(rod_tuning)]),
    "rod_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(rod_tuning)]),
    "rod_bucket_info": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(rod_tuning), C.POINTER(C.c_int32)]),
    "rod_set_chunking": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "rod_set_bindings": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.c_int32]),
    "rod_set_contact": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.c_double]),
    "rod_haptic_attach": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "rod_haptic_detach": (C.c_int, [C.c_void_p, C.c_int32]),
    "rod_haptic_set_pose": (C.c_int, [C.c_void_p, C.c_int32, _DP, _DP]),
    "rod_haptic_get_force": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(rod_haptic_force)]),
    "rod_set_environment": (C.c_int, [C.c_void_p, C.c_int32, _DP, C.c_double]),
    "rod_environment_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "rod_stable_dt": (C.c_int, [C.POINTER(rod_params), _DP]),
    "rod_last_step_time": (C.c_int, [C.c_void_p, C.POINTER(C.c_float), C.POINTER(C.c_int32)]),
    "rod_set_stiffness_mult": (C.c_int, [C.c_void_p, C.POINTER(C.c_float), C.POINTER(C.c_float)]),
    "rod_step_state_noalloc": (C.c_int, [C.c_void_p, _FP, _FP, _FP, _FP, C.c_int64, C.c_int32,
                                        C.c_int32]),
    "rod_adjoint_forward": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, _FP, C.c_int32,
                                     C.POINTER(C.c_int64)]),
    "rod_adjoint_backward": (C.c_int, [C.c_void_p, C.c_int64, _FP, _FP, _FP, _FP, _FP, _FP, _FP,
                                       C.c_int32]),
    "rod_status_str": (C.c_char_p, [C.c_int]),
    "rod_last_error": (C.c_char_p, [C.c_void_p]),
}

_lib = None


def lib():
    """Load the built library (raises if it has not been built: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libcorde_rod.so is not built; run paper_2509_04277_amd/build.py")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc, handle=None):
    if rc != ROD_OK:
        msg = lib().rod_last_error(handle)
        raise RodError(rc, msg.decode() if msg else "")


def _f64(a, n=None):
    if a is None:
        return None
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64)).ravel()
    if n is not None and a.size != n:
        raise ValueError("array of %d values expected, got %d" % (n, a.size))
    return a


def make_params(spec):
    """rod_params for a ``RodSpec``; returns (params, arrays kept alive)."""
    n = int(spec.n)
    keep = [_f64(spec.seg_len, n), _f64(spec.radius, n), _f64(spec.young, n),
            _f64(spec.u_hat, 3 * (n - 1)) if spec.u_hat is not None else None,
            _f64(spec.f_ext, 3 * (n + 1)) if spec.f_ext is not None else None,
            _f64(spec.tau_ext, 3 * n) if spec.tau_ext is not None else None]
    p = rod_params()
    p.n_elements = n
    p.inextensible = int(bool(spec.inextensible))
    p.n_constraint_iters = int(spec.n_iter)
    p.clamp_end0 = int(bool(spec.clamp))
    p.dt = float(spec.dt)
    p.gravity[:] = [float(g) for g in spec.gravity]
    p.damping_lin, p.damping_ang = float(spec.damp_lin), float(spec.damp_ang)
    p.poisson, p.density = float(spec.poisson), float(spec.density)
    p.kp_scale, p.bend_scale = float(spec.kp_scale), float(spec.bend_scale)
    p.twist_scale = float(spec.twist_scale)
    for name, a in zip(("seg_len", "radius", "young", "u_hat", "f_ext", "tau_ext"), keep):
        setattr(p, name, a.ctypes.data_as(_DP) if a is not None else None)
    p.clamp_x0[:] = [float(c) for c in spec.clamp_x0]
    p.clamp_q0[:] = [float(c) for c in spec.clamp_q0]
    p.clamp_amp[:] = [float(c) for c in spec.clamp_amp]
    p.clamp_twist_amp = float(spec.clamp_twist_amp)
    p.clamp_twist_axis[:] = [float(c) for c in spec.clamp_twist_axis]
    p.clamp_freq = float(spec.clamp_freq)
    p.clamp_phase_x = float(spec.clamp_phase_x)
    p.clamp_phase_twist = float(spec.clamp_phase_twist)
    p.damping_int = float(spec.damp_int)
    return p, keep


def stable_dt(spec) -> float:
    """rod_stable_dt: the library's stability rule for one rod (host-only call)."""
    p, keep = make_params(spec.replace(dt=1.0) if not spec.dt > 0 else spec)
    out = C.c_double()
    _check(lib().rod_stable_dt(C.byref(p), C.byref(out)))
    return out.value


def _ptr(a):
    """(pointer, on_device) for a numpy array or a torch tensor."""
    if isinstance(a, np.ndarray):
        if a.dtype != np.float32 or not a.flags["C_CONTIGUOUS"]:
            raise ValueError("float32 C-contiguous array required")
        return a.ctypes.data, 0
    import torch
    if not isinstance(a, torch.Tensor) or a.dtype != torch.float32 or not a.is_contiguous():
        raise ValueError("float32 contiguous numpy array or torch tensor required")
    return a.data_ptr(), int(a.is_cuda)


class RodBatch:
    """A library handle holding one or more rods (rod_create ... rod_destroy)."""

    def __init__(self, specs: Sequence, stream=None):
        specs = list(specs)
        self.specs = specs
        self.n = [int(s.n) for s in specs]
        self.n_points = sum(n + 1 for n in self.n)
        self.n_frames = sum(self.n)
        arr = (rod_params * len(specs))()
        self._keep = []
        for i, s in enumerate(specs):
            p, keep = make_params(s)
            arr[i] = p
            self._keep.append(keep)
        if stream is None:
            try:
                import torch
                stream = torch.cuda.current_stream().cuda_stream if torch.cuda.is_available() else 0
            except Exception:
                stream = 0
        h = C.c_void_p()
        _check(lib().rod_create(arr, len(specs), C.c_void_p(stream), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().rod_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- state ------------------------------------------------------------------
    def set_state(self, x, v, q, w, t0: float = 0.0):
        ptrs = [_ptr(a) for a in (x, v, q, w)]
        dev = {d for _, d in ptrs}
        if len(dev) != 1:
            raise ValueError("all state arrays must be on the same side")
        sizes = (3 * self.n_points, 3 * self.n_points, 4 * self.n_frames, 3 * self.n_frames)
        for a, s in zip((x, v, q, w), sizes):
            if (a.size if isinstance(a, np.ndarray) else a.numel()) != s:
                raise ValueError("state array of %d values expected" % s)
        _check(lib().rod_set_state(self.h, *[C.c_void_p(p) for p, _ in ptrs], dev.pop(),
                                   float(t0)), self.h)

    def set_state_rods(self, states, t0: float = 0.0):
        """Set from a list of ``RodState`` (any float dtype), concatenated in rod order."""
        cat = lambda k: np.ascontiguousarray(
            np.concatenate([np.asarray(getattr(s, k), dtype=np.float64).reshape(-1) for s in states]),
            dtype=np.float32)
        self.set_state(cat("x"), cat("v"), cat("q"), cat("w"), t0)

    def get_state(self, out=None):
        """Host copy (x, v, q, w) as float32 arrays, or into device tensors ``out``."""
        if out is None:
            out = (np.empty(3 * self.n_points, np.float32), np.empty(3 * self.n_points, np.float32),
                   np.empty(4 * self.n_frames, np.float32), np.empty(3 * self.n_frames, np.float32))
        ptrs = [_ptr(a) for a in out]
        _check(lib().rod_get_state(self.h, *[C.c_void_p(p) for p, _ in ptrs], ptrs[0][1]), self.h)
        return out

    def get_positions(self, out):
        """Copy only the point positions (x) into ``out`` (host array or device tensor)."""
        p, dev = _ptr(out)
        _check(lib().rod_get_state(self.h, C.c_void_p(p), None, None, None, dev), self.h)
        return out

    def get_state_rods(self):
        """Per-rod (x, v, q, w) float32 arrays of shape (N+1,3), (N+1,3), (N,4), (N,3)."""
        x, v, q, w = self.get_state()
        res, po, fo = [], 0, 0
        for n in self.n:
            res.append((x[3 * po:3 * (po + n + 1)].reshape(n + 1, 3),
                        v[3 * po:3 * (po + n + 1)].reshape(n + 1, 3),
                        q[4 * fo:4 * (fo + n)].reshape(n, 4), w[3 * fo:3 * (fo + n)].reshape(n, 3)))
            po += n + 1
            fo += n
        return res

    # ---- stepping -----------------------------------------------------------------
    def step(self, n_steps: int, steps_per_launch: int = 0):
        _check(lib().rod_step(self.h, int(n_steps), int(steps_per_launch)), self.h)

    def sync(self):
        _check(lib().rod_sync(self.h), self.h)

    def last_step_time(self):
        ms, nl = C.c_float(), C.c_int32()
        _check(lib().rod_last_step_time(self.h, C.byref(ms), C.byref(nl)), self.h)
        return ms.value, nl.value

    def time(self):
        t, s = C.c_double(), C.c_int64()
        _check(lib().rod_get_time(self.h, C.byref(t), C.byref(s)), self.h)
        return t.value, s.value

    def set_clamp(self, rod: int, x0, q0):
        a, b = _f64(x0, 3), _f64(q0, 4)
        _check(lib().rod_set_clamp(self.h, int(rod), a.ctypes.data_as(_DP), b.ctypes.data_as(_DP)),
               self.h)

    def step_state_noalloc(self, x, v, q, w, first_step: int, n_steps: int,
                           steps_per_launch: int = 0):
        """rod_step_state_noalloc: steps caller-owned device state (float32 tensors in the
        handle's layout) in place, allocating nothing."""
        ptrs = [_ptr(a) for a in (x, v, q, w)]
        if any(not d for _, d in ptrs):
            raise ValueError("device arrays expected")
        _check(lib().rod_step_state_noalloc(self.h, *[C.c_void_p(p) for p, _ in ptrs],
                                            int(first_step), int(n_steps), int(steps_per_launch)),
               self.h)

    # ---- adjoint --------------------------------------------------------------------
    def set_stiffness_mult(self, bend, twist):
        b = np.ascontiguousarray(np.asarray(bend, dtype=np.float32).ravel())
        t = np.ascontiguousarray(np.asarray(twist, dtype=np.float32).ravel())
        if b.size != len(self.n) or t.size != len(self.n):
            raise ValueError("one multiplier per rod expected")
        _check(lib().rod_set_stiffness_mult(self.h, b.ctypes.data_as(C.POINTER(C.c_float)),
                                            t.ctypes.data_as(C.POINTER(C.c_float))), self.h)

    def adjoint_forward(self, n_steps: int, ckpt_every: int = 20, tips=None):
        """Rollout with checkpoints; returns the tip trajectory (rods, n_steps, 3).  The
        rollout's number is kept in ``self.rollout``."""
        if tips is None:
            tips = np.empty((len(self.n), int(n_steps), 3), np.float32)
        p, dev = _ptr(tips)
        rid = C.c_int64(0)
        _check(lib().rod_adjoint_forward(self.h, int(n_steps), int(ckpt_every), C.c_void_p(p),
                                         dev, C.byref(rid)), self.h)
        self.rollout = int(rid.value)
        return tips

    def adjoint_backward(self, dl_dtips, out=None, rollout: int = 0):
        """Gradients for dL/dtip: dict bend, twist (per rod) and x, v, q, w (state layout).
        rollout: the number of the rollout to reverse (0: the one the handle holds)."""
        if out is None:
            out = dict(bend=np.empty(len(self.n), np.float32), twist=np.empty(len(self.n), np.float32),
                       x=np.empty(3 * self.n_points, np.float32), v=np.empty(3 * self.n_points, np.float32),
                       q=np.empty(4 * self.n_frames, np.float32), w=np.empty(3 * self.n_frames, np.float32))
        pd, dev = _ptr(dl_dtips)
        ptrs = [_ptr(out[k]) for k in ("bend", "twist", "x", "v", "q", "w")]
        if any(d != dev for _, d in ptrs):
            raise ValueError("dL/dtip and the outputs must be on the same side")
        _check(lib().rod_adjoint_backward(self.h, int(rollout), C.c_void_p(pd),
                                          *[C.c_void_p(p) for p, _ in ptrs], dev), self.h)
        return out

    # ---- kernel shape ---------------------------------------------------------------
    @property
    def tuning(self):
        t = rod_tuning()
        _check(lib().rod_get_tuning(self.h, C.byref(t)), self.h)
        return dict(waves=t.waves, elems_per_lane=t.elems_per_lane,
                    steps_per_launch=t.steps_per_launch, us_per_step=t.us_per_step)

    def set_tuning(self, waves: int, elems_per_lane: int, steps_per_launch: int = 10):
        t = rod_tuning(int(waves), int(elems_per_lane), int(steps_per_launch), 0.0)
        _check(lib().rod_set_tuning(self.h, C.byref(t)), self.h)

    def buckets(self):
        """[(waves, elems_per_lane, n_rods, us_per_step)] of the handle's kernel-shape buckets."""
        out, b = [], 0
        while True:
            t, n = rod_tuning(), C.c_int32()
            if lib().rod_bucket_info(self.h, b, C.byref(t), C.byref(n)) != ROD_OK:
                return out
            out.append((t.waves, t.elems_per_lane, n.value, t.us_per_step))
            b += 1

    def set_bindings(self, pairs, one_way: bool):
        """Bind point pairs (k, 4) = (rod_a, point_a, rod_b, point_b) with zero-length distance
        constraints; one_way: rod_b is the master.  An empty list removes the bindings."""
        arr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 4))
        _check(lib().rod_set_bindings(self.h, int(arr.shape[0]),
                                      arr.ctypes.data_as(C.POINTER(C.c_int32)),
                                      1 if one_way else 2), self.h)

    def set_contact(self, sets, mu: float):
        """Contact sets (k, 2) = (rod_a, rod_b or -1) with friction coefficient mu; an empty list
        removes them."""
        arr = np.ascontiguousarray(np.asarray(sets, dtype=np.int32).reshape(-1, 2))
        _check(lib().rod_set_contact(self.h, int(arr.shape[0]),
                                     arr.ctypes.data_as(C.POINTER(C.c_int32)), float(mu)), self.h)

    def set_environment(self, tris, mu: float):
        """Static triangle mesh (k, 3, 3) the rods collide with; an empty list removes it."""
        t = np.ascontiguousarray(np.asarray(tris, dtype=np.float64).reshape(-1, 9))
        _check(lib().rod_set_environment(self.h, len(t), t.ctypes.data_as(_DP) if len(t) else None,
                                         float(mu)), self.h)

    def environment_info(self):
        """(tree nodes, triangles) of the environment."""
        a, b = C.c_int32(), C.c_int32()
        _check(lib().rod_environment_info(self.h, C.byref(a), C.byref(b)), self.h)
        return int(a.value), int(b.value)

    def haptic_attach(self, rod: int, steps_per_record: int = 1):
        _check(lib().rod_haptic_attach(self.h, rod, steps_per_record), self.h)

    def haptic_detach(self, rod: int):
        _check(lib().rod_haptic_detach(self.h, rod), self.h)

    def haptic_set_pose(self, rod: int, x0, q0):
        """Thread-safe against the stepping thread (no GPU call); errors name no handle."""
        x = (C.c_double * 3)(*[float(v) for v in x0])
        q = (C.c_double * 4)(*[float(v) for v in q0])
        _check(lib().rod_haptic_set_pose(self.h, rod, x, q))

    def haptic_get_force(self, rod: int, window: bool = False):
        """(mean force (3,) [N] on the clamped base over the newest record's window, steps taken
        at its end, pose number in use[, steps in the window if window])."""
        r = rod_haptic_force()
        _check(lib().rod_haptic_get_force(self.h, rod, C.byref(r)))
        out = (np.array(r.f[:]), int(r.step), int(r.pose))
        return out + (int(r.n_steps),) if window else out

    def set_chunking(self, min_elements: int, chunk_elements: int = 0):
        """Step rods longer than min_elements with the chunked multi-workgroup kernel, about
        chunk_elements owned elements per workgroup (0: the largest chunk)."""
        _check(lib().rod_set_chunking(self.h, int(min_elements), int(chunk_elements)), self.h)

    def autotune(self, probe_steps: int = 200, steps_per_launch: int = 10):
        """rod_autotune: time each admissible kernel shape per bucket and keep the fastest;
        steps_per_launch = 0 also picks the steps per launch (the smallest count whose time per
        step is within 5 % of the best).  State and step counter are left as they were."""
        t = rod_tuning()
        _check(lib().rod_autotune(self.h, int(probe_steps), int(steps_per_launch), C.byref(t)),
               self.h)
        return dict(waves=t.waves, elems_per_lane=t.elems_per_lane,
                    steps_per_launch=t.steps_per_launch, us_per_step=t.us_per_step)


def header_functions(path: Optional[str] = None):
    """Names of the functions declared in include/rod.h."""
    import re
    path = path or os.path.join(os.path.dirname(HERE), "include", "rod.h")
    src = open(path).read()
    return sorted(set(re.findall(r"^\s*(?:rod_status|const char\*)\s+(rod_\w+)\s*\(", src, re.M)))


def rollout_function():
    """torch.autograd.Function over the library's adjoint: tips = RodRollout.apply(batch,
    bend_mult, twist_mult, x0, v0, q0, w0, n_steps, ckpt_every).

    Inputs are device float32 tensors: bend_mult, twist_mult (n_rods,), initial state in the
    handle's layout.  Output: tip trajectory (n_rods, n_steps, 3).  backward() runs
    rod_adjoint_backward and returns gradients for the multipliers and the initial state."""
    import torch

    class RodRollout(torch.autograd.Function):
        @staticmethod
        def forward(ctx, batch, bend, twist, x0, v0, q0, w0, n_steps, ckpt_every):
            batch.set_stiffness_mult(bend.detach().cpu().numpy(), twist.detach().cpu().numpy())
            batch.set_state(x0.detach().contiguous(), v0.detach().contiguous(),
                            q0.detach().contiguous(), w0.detach().contiguous())
            tips = torch.empty((len(batch.n), int(n_steps), 3), dtype=torch.float32, device=x0.device)
            batch.adjoint_forward(int(n_steps), int(ckpt_every), tips)
            torch.cuda.synchronize(x0.device)
            ctx.batch = batch
            ctx.rollout = batch.rollout   # a later forward on the handle makes backward refuse
            return tips

        @staticmethod
        def backward(ctx, grad_tips):
            b = ctx.batch
            dev = grad_tips.device
            out = dict(bend=torch.empty(len(b.n), device=dev), twist=torch.empty(len(b.n), device=dev),
                       x=torch.empty(3 * b.n_points, device=dev), v=torch.empty(3 * b.n_points, device=dev),
                       q=torch.empty(4 * b.n_frames, device=dev), w=torch.empty(3 * b.n_frames, device=dev))
            b.adjoint_backward(grad_tips.contiguous().float(), out, rollout=ctx.rollout)
            torch.cuda.synchronize(dev)
            return (None, out["bend"], out["twist"], out["x"], out["v"], out["q"], out["w"], None, None)

    return RodRollout
