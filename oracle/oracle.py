"""ctypes binding of the FP64 CPU oracle (corde_oracle.c).

TEST INFRASTRUCTURE ONLY: the test-suite, the package smoke check and the CPU-baseline leg of
the benchmark use this module; the product library never imports it.  It shares no code with
the GPU path.  A rod is described by a ``RodSpec`` and a ``RodState`` from
``paper_2509_04277_amd.workloads`` (plain data, no method arithmetic).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "corde_oracle.c")
GRAD_SRC = os.path.join(HERE, "corde_oracle_grad.cpp")
HDR = os.path.join(HERE, "corde_oracle.h")
# CORDE_ORACLE_LIB names a library built elsewhere by build(src=..., lib=...): the mutation test
# loads copies of the oracle with planted mistakes this way, one process each.
PREBUILT = os.environ.get("CORDE_ORACLE_LIB")
LIB = PREBUILT or os.path.join(HERE, "libcorde_oracle.so")


def build(force: bool = False, src: str = SRC, lib: str = None, grad_src: str = GRAD_SRC) -> str:
    """Compile corde_oracle.c (or the copy ``src``) with gcc and corde_oracle_grad.cpp (or the
    copy ``grad_src``) with g++ into one library (FP64, -O2, no fast-math, no contraction)."""
    if lib is None:
        if PREBUILT:
            return PREBUILT
        lib = LIB
    deps = [src, grad_src, HDR]
    if force or not os.path.exists(lib) or any(os.path.getmtime(lib) < os.path.getmtime(d)
                                               for d in deps):
        tmp = lib + ".tmp%d" % os.getpid()
        obj_c, obj_cc = tmp + ".c.o", tmp + ".cc.o"
        common = ["-O2", "-fPIC", "-fno-fast-math", "-ffp-contract=off", "-Wall", "-I", HERE]
        try:
            subprocess.check_call(["gcc", "-std=c11"] + common + ["-c", "-o", obj_c, src])
            subprocess.check_call(["g++", "-std=c++17"] + common + ["-c", "-o", obj_cc, grad_src])
            subprocess.check_call(["g++", "-shared", "-pthread", "-o", tmp, obj_c, obj_cc, "-lm"])
        finally:
            for o in (obj_c, obj_cc):
                if os.path.exists(o):
                    os.remove(o)
        os.replace(tmp, lib)
    return lib


class _Rod(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("inextensible", C.c_int32), ("n_iter", C.c_int32),
        ("clamp", C.c_int32), ("dt", C.c_double), ("gravity", C.c_double * 3),
        ("damp_lin", C.c_double), ("damp_ang", C.c_double), ("poisson", C.c_double),
        ("density", C.c_double), ("kp_scale", C.c_double), ("bend_scale", C.c_double),
        ("twist_scale", C.c_double),
        ("seg_len", C.POINTER(C.c_double)), ("radius", C.POINTER(C.c_double)),
        ("young", C.POINTER(C.c_double)), ("u_hat", C.POINTER(C.c_double)),
        ("f_ext", C.POINTER(C.c_double)), ("tau_ext", C.POINTER(C.c_double)),
        ("clamp_x0", C.c_double * 3), ("clamp_q0", C.c_double * 4),
        ("clamp_amp", C.c_double * 3), ("clamp_twist_amp", C.c_double),
        ("clamp_twist_axis", C.c_double * 3), ("clamp_freq", C.c_double),
        ("clamp_phase_x", C.c_double), ("clamp_phase_twist", C.c_double),
        ("damp_int", C.c_double),
    ]


_lib = None
_DP = C.POINTER(C.c_double)


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        L.oracle_check.restype = C.c_int32
        L.oracle_check.argtypes = [C.POINTER(_Rod)]
        L.oracle_energy.restype = C.c_double
        L.oracle_energy.argtypes = [C.POINTER(_Rod), _DP, _DP]
        L.oracle_kinetic.restype = C.c_double
        L.oracle_kinetic.argtypes = [C.POINTER(_Rod), _DP, _DP]
        L.oracle_forces.restype = None
        L.oracle_forces.argtypes = [C.POINTER(_Rod), _DP, _DP, _DP, _DP]
        L.oracle_darboux.restype = None
        L.oracle_darboux.argtypes = [C.POINTER(_Rod), _DP, C.c_int32, _DP]
        L.oracle_clamp_pose.restype = None
        L.oracle_clamp_pose.argtypes = [C.POINTER(_Rod), C.c_double, _DP, _DP, _DP]
        L.oracle_step.restype = None
        L.oracle_step.argtypes = [C.POINTER(_Rod), C.c_double, _DP, _DP, _DP, _DP]
        L.oracle_rollout.restype = None
        L.oracle_rollout.argtypes = [C.POINTER(_Rod), C.c_double, C.c_int32,
                                     _DP, _DP, _DP, _DP, _DP]
        L.oracle_rollout_rounded.restype = None
        L.oracle_rollout_rounded.argtypes = [C.POINTER(_Rod), C.c_double, C.c_int32,
                                             _DP, _DP, _DP, _DP, C.c_int32]
        L.oracle_stable.restype = C.c_int32
        L.oracle_stable.argtypes = [C.POINTER(_Rod), C.c_double, C.c_int32,
                                    _DP, _DP, _DP, _DP, C.c_double]
        L.oracle_rotmat.restype = None
        L.oracle_rotmat.argtypes = [_DP, _DP]
        L.oracle_dt_rule.restype = C.c_double
        L.oracle_dt_rule.argtypes = [C.POINTER(_Rod)]
        L.oracle_max_strain.restype = C.c_double
        L.oracle_max_strain.argtypes = [C.POINTER(_Rod), _DP]
        L.oracle_bmat.restype = None
        L.oracle_bmat.argtypes = [C.c_int32, _DP]
        L.oracle_qmul.restype = None
        L.oracle_qmul.argtypes = [_DP, _DP, _DP]
        L.oracle_bind_impulse.restype = None
        L.oracle_bind_impulse.argtypes = [_DP, _DP, C.c_double, _DP, _DP, C.c_double, C.c_double,
                                          C.c_int32]
        L.oracle_rollout_fb.restype = None
        L.oracle_rollout_fb.argtypes = [C.POINTER(_Rod), C.c_double, C.c_int32, _DP, _DP, _DP, _DP,
                                        _DP]
        L.oracle_rollout_group.restype = None
        L.oracle_rollout_group.argtypes = [C.POINTER(C.POINTER(_Rod)), C.c_int32,
                                           C.POINTER(_Binding), C.POINTER(_Contact), C.c_double,
                                           C.c_int32] + [C.POINTER(_DP)] * 4 + [C.POINTER(C.c_int32)]
        L.oracle_rollout_group_rounded.restype = None
        L.oracle_rollout_group_rounded.argtypes = [
            C.POINTER(C.POINTER(_Rod)), C.c_int32, C.POINTER(_Binding), C.POINTER(_Contact),
            C.c_double, C.c_int32] + [C.POINTER(_DP)] * 4 + [C.c_int32, C.POINTER(C.c_int32)]
        L.oracle_self_skip.restype = C.c_int32
        L.oracle_self_skip.argtypes = [C.POINTER(_Rod)]
        L.oracle_rollout_pair.restype = None
        L.oracle_rollout_pair.argtypes = [C.POINTER(_Rod), C.POINTER(_Rod), C.POINTER(_Binding),
                                          C.c_double, C.c_int32] + [_DP] * 8
        L.oracle_dissipation.restype = C.c_double
        L.oracle_dissipation.argtypes = [C.POINTER(_Rod), _DP, _DP, _DP, _DP]
        L.oracle_damping_forces.restype = None
        L.oracle_damping_forces.argtypes = [C.POINTER(_Rod), _DP, _DP, _DP, _DP, _DP, _DP]
        L.oracle_closest_point_triangle.restype = None
        L.oracle_closest_point_triangle.argtypes = [_DP, _DP, _DP]
        L.oracle_env_response.restype = None
        L.oracle_env_response.argtypes = [C.POINTER(_Env), _DP, C.c_double, _DP, _DP,
                                          C.POINTER(C.c_int32)]
        L.oracle_env_impulse.restype = None
        L.oracle_env_impulse.argtypes = [_DP, C.c_double, C.c_double, C.c_double, C.c_double, _DP]
        L.oracle_rollout_env.restype = None
        L.oracle_rollout_env.argtypes = [C.POINTER(_Rod), C.POINTER(_Env), C.c_double, C.c_int32,
                                         _DP, _DP, _DP, _DP, C.POINTER(C.c_int32)]
        L.oracle_grad_rollout.restype = C.c_int32
        L.oracle_grad_rollout.argtypes = [C.POINTER(_Rod), C.c_double, C.c_int32] + [_DP] * 5
        L.oracle_jvp.restype = C.c_int32
        L.oracle_jvp.argtypes = ([C.POINTER(_Rod), C.c_double, C.c_int32] + [_DP] * 8 +
                                 [C.c_double, C.c_double, _DP, _DP])
        L.oracle_vjp.restype = C.c_int32
        L.oracle_vjp.argtypes = ([C.POINTER(_Rod), C.c_double, C.c_int32] + [_DP] * 5 +
                                 [C.c_int32] + [_DP] * 7)
        _PP = C.POINTER(_DP)
        L.oracle_vjp_many.restype = C.c_int32
        L.oracle_vjp_many.argtypes = ([C.c_int32, C.POINTER(_Rod), C.c_double, C.c_int32] +
                                      [_PP] * 5 + [C.c_int32] + [_PP] * 4 + [_DP, _DP, _PP, C.c_int32])
        L.oracle_rollout_many.restype = C.c_int32
        L.oracle_rollout_many.argtypes = ([C.c_int32, C.POINTER(_Rod), C.c_double, C.c_int32] +
                                          [_PP] * 4 + [C.c_int32])
        _lib = L
    return _lib


class _Binding(C.Structure):
    _fields_ = [("n_pairs", C.c_int32), ("point_a", C.POINTER(C.c_int32)),
                ("point_b", C.POINTER(C.c_int32)), ("one_way", C.c_int32)]


class _Contact(C.Structure):
    _fields_ = [("mu", C.c_double)]


class _Env(C.Structure):
    _fields_ = [("n_tris", C.c_int32), ("tris", _DP), ("mu", C.c_double)]


class Env:
    """A static triangle mesh (tris: (k, 3, 3) vertices, face normal (b - a) x (c - a) towards
    the rods) with friction coefficient mu, for the oracle's environment collision."""

    def __init__(self, tris, mu=0.0):
        self.tris = np.ascontiguousarray(np.asarray(tris, dtype=np.float64).reshape(-1, 9))
        self.c = _Env(len(self.tris), self.tris.ctypes.data_as(_DP), float(mu))

    def response(self, c, r):
        """(n (3,), depth, colliding triangles) of a sphere of centre c and radius r."""
        c = _f64(c, (3,))
        n, d, k = np.zeros(3), C.c_double(0.0), C.c_int32(0)
        lib().oracle_env_response(C.byref(self.c), _p(c), float(r), _p(n), C.byref(d), C.byref(k))
        return n, float(d.value), int(k.value)


def closest_point_triangle(p, tri):
    p, t, out = _f64(p, (3,)), _f64(tri, (9,)), np.zeros(3)
    lib().oracle_closest_point_triangle(_p(p), _p(t), _p(out))
    return out


def env_impulse(n, depth, winv, dt, mu, v):
    n, out = _f64(n, (3,)), _f64(v, (3,)).copy()
    lib().oracle_env_impulse(_p(n), float(depth), float(winv), float(dt), float(mu), _p(out))
    return out


def rollout_env(spec, state, n_steps, env, t0=0.0):
    """One rod against the mesh of ``env``; returns (new state, most colliding points)."""
    r = Rod(spec)
    o = state.copy()
    o.x, o.v = _f64(state.x, (r.n + 1, 3)).copy(), _f64(state.v, (r.n + 1, 3)).copy()
    o.q, o.w = _f64(state.q, (r.n, 4)).copy(), _f64(state.w, (r.n, 3)).copy()
    most = C.c_int32(0)
    lib().oracle_rollout_env(C.byref(r.c), C.byref(env.c), float(t0), int(n_steps), _p(o.x),
                             _p(o.v), _p(o.q), _p(o.w), C.byref(most))
    return o, int(most.value)


def _p(a):
    return None if a is None else a.ctypes.data_as(_DP)


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


class Rod:
    """An oracle rod: holds the C description and keeps its arrays alive."""

    def __init__(self, spec):
        n = int(spec.n)
        self.spec = spec
        self.n = n
        self._keep = dict(
            seg_len=_f64(spec.seg_len, (n,)), radius=_f64(spec.radius, (n,)),
            young=_f64(spec.young, (n,)),
            u_hat=_f64(spec.u_hat, (max(n - 1, 0), 3)) if spec.u_hat is not None else None,
            f_ext=_f64(spec.f_ext, (n + 1, 3)) if spec.f_ext is not None else None,
            tau_ext=_f64(spec.tau_ext, (n, 3)) if spec.tau_ext is not None else None)
        r = _Rod()
        r.n = n
        r.inextensible = int(bool(spec.inextensible))
        r.n_iter = int(spec.n_iter)
        r.clamp = int(bool(spec.clamp))
        r.dt = float(spec.dt)
        r.gravity[:] = [float(g) for g in spec.gravity]
        r.damp_lin = float(spec.damp_lin)
        r.damp_ang = float(spec.damp_ang)
        r.poisson = float(spec.poisson)
        r.density = float(spec.density)
        r.kp_scale = float(spec.kp_scale)
        r.bend_scale = float(spec.bend_scale)
        r.twist_scale = float(spec.twist_scale)
        for k in ("seg_len", "radius", "young", "u_hat", "f_ext", "tau_ext"):
            setattr(r, k, _p(self._keep[k]))
        r.clamp_x0[:] = [float(c) for c in spec.clamp_x0]
        r.clamp_q0[:] = [float(c) for c in spec.clamp_q0]
        r.clamp_amp[:] = [float(c) for c in spec.clamp_amp]
        r.clamp_twist_amp = float(spec.clamp_twist_amp)
        r.clamp_twist_axis[:] = [float(c) for c in spec.clamp_twist_axis]
        r.clamp_freq = float(spec.clamp_freq)
        r.clamp_phase_x = float(spec.clamp_phase_x)
        r.clamp_phase_twist = float(spec.clamp_phase_twist)
        r.damp_int = float(spec.damp_int)
        self.c = r
        rc = lib().oracle_check(C.byref(r))
        if rc != 0:
            raise ValueError("oracle rejected rod description (code %d)" % rc)

    def with_dt(self, dt):
        import dataclasses
        return Rod(dataclasses.replace(self.spec, dt=float(dt)))

    # --- queries -------------------------------------------------------------------
    def energy(self, x, q):
        x, q = _f64(x, (self.n + 1, 3)), _f64(q, (self.n, 4))
        return lib().oracle_energy(C.byref(self.c), _p(x), _p(q))

    def kinetic(self, v, w):
        v, w = _f64(v, (self.n + 1, 3)), _f64(w, (self.n, 3))
        return lib().oracle_kinetic(C.byref(self.c), _p(v), _p(w))

    def forces(self, x, q):
        x, q = _f64(x, (self.n + 1, 3)), _f64(q, (self.n, 4))
        F = np.zeros((self.n + 1, 3))
        tau = np.zeros((self.n, 3))
        lib().oracle_forces(C.byref(self.c), _p(x), _p(q), _p(F), _p(tau))
        return F, tau

    def dissipation(self, x, q, v, w):
        x, q = _f64(x, (self.n + 1, 3)), _f64(q, (self.n, 4))
        v, w = _f64(v, (self.n + 1, 3)), _f64(w, (self.n, 3))
        return lib().oracle_dissipation(C.byref(self.c), _p(x), _p(q), _p(v), _p(w))

    def damping_forces(self, x, q, v, w):
        x, q = _f64(x, (self.n + 1, 3)), _f64(q, (self.n, 4))
        v, w = _f64(v, (self.n + 1, 3)), _f64(w, (self.n, 3))
        F = np.zeros((self.n + 1, 3))
        tau = np.zeros((self.n, 3))
        lib().oracle_damping_forces(C.byref(self.c), _p(x), _p(q), _p(v), _p(w), _p(F), _p(tau))
        return F, tau

    def darboux(self, q, j):
        q = _f64(q, (self.n, 4))
        u = np.zeros(3)
        lib().oracle_darboux(C.byref(self.c), _p(q), int(j), _p(u))
        return u

    def clamp_pose(self, t):
        xc, qc, wc = np.zeros(3), np.zeros(4), np.zeros(3)
        lib().oracle_clamp_pose(C.byref(self.c), float(t), _p(xc), _p(qc), _p(wc))
        return xc, qc, wc

    def max_strain(self, x):
        x = _f64(x, (self.n + 1, 3))
        return lib().oracle_max_strain(C.byref(self.c), _p(x))

    def dt_rule(self):
        return lib().oracle_dt_rule(C.byref(self.c))

    # --- time stepping ---------------------------------------------------------------
    def rollout(self, state, n_steps, t0=0.0, tip=False):
        """Returns (new_state, tip trajectory or None); ``state`` is not modified."""
        st = state.copy()
        x, v = _f64(st.x, (self.n + 1, 3)).copy(), _f64(st.v, (self.n + 1, 3)).copy()
        q, w = _f64(st.q, (self.n, 4)).copy(), _f64(st.w, (self.n, 3)).copy()
        tr = np.zeros((int(n_steps), 3)) if tip else None
        lib().oracle_rollout(C.byref(self.c), float(t0), int(n_steps), _p(x), _p(v), _p(q),
                             _p(w), _p(tr))
        st.x, st.v, st.q, st.w = x, v, q, w
        return st, tr

    def rollout_rounded(self, state, n_steps, mask, t0=0.0):
        """rollout with the fields of mask (1 x, 2 v, 4 q, 8 w) rounded to FP32 after every
        step; returns the new state."""
        st = state.copy()
        x, v = _f64(st.x, (self.n + 1, 3)).copy(), _f64(st.v, (self.n + 1, 3)).copy()
        q, w = _f64(st.q, (self.n, 4)).copy(), _f64(st.w, (self.n, 3)).copy()
        lib().oracle_rollout_rounded(C.byref(self.c), float(t0), int(n_steps), _p(x), _p(v),
                                     _p(q), _p(w), int(mask))
        st.x, st.v, st.q, st.w = x, v, q, w
        return st

    def rollout_fb(self, state, n_steps, t0=0.0):
        """Returns (new_state, force on the base point for every step (n_steps, 3))."""
        st = state.copy()
        x, v = _f64(st.x, (self.n + 1, 3)).copy(), _f64(st.v, (self.n + 1, 3)).copy()
        q, w = _f64(st.q, (self.n, 4)).copy(), _f64(st.w, (self.n, 3)).copy()
        fb = np.zeros((int(n_steps), 3))
        lib().oracle_rollout_fb(C.byref(self.c), float(t0), int(n_steps), _p(x), _p(v), _p(q),
                                _p(w), _p(fb))
        st.x, st.v, st.q, st.w = x, v, q, w
        return st, fb

    # --- reference derivatives (corde_oracle_grad.cpp) -----------------------------
    def _state64(self, state):
        return (_f64(state.x, (self.n + 1, 3)).copy(), _f64(state.v, (self.n + 1, 3)).copy(),
                _f64(state.q, (self.n, 4)).copy(), _f64(state.w, (self.n, 3)).copy())

    def grad_rollout(self, state, n_steps, t0=0.0):
        """The rollout through the templated step of the gradient code, in doubles:
        (new state, tip trajectory); equals ``rollout`` bitwise."""
        x, v, q, w = self._state64(state)
        tr = np.zeros((int(n_steps), 3))
        rc = lib().oracle_grad_rollout(C.byref(self.c), float(t0), int(n_steps), _p(x), _p(v),
                                       _p(q), _p(w), _p(tr))
        if rc != 0:
            raise ValueError("oracle_grad_rollout refused the rod (code %d)" % rc)
        st = state.copy()
        st.x, st.v, st.q, st.w = x, v, q, w
        return st, tr

    def jvp(self, state, n_steps, dstate=None, dmb=0.0, dmt=0.0, t0=0.0):
        """Forward mode: (tip trajectory, its derivative along dstate (a RodState of
        directions, or None) and the multiplier directions dmb, dmt)."""
        x, v, q, w = self._state64(state)
        if dstate is not None:
            dx, dv, dq, dw = self._state64(dstate)
        else:
            dx = dv = dq = dw = None
        tip = np.zeros((int(n_steps), 3))
        dtip = np.zeros((int(n_steps), 3))
        rc = lib().oracle_jvp(C.byref(self.c), float(t0), int(n_steps), _p(x), _p(v), _p(q),
                              _p(w), _p(dx), _p(dv), _p(dq), _p(dw), float(dmb), float(dmt),
                              _p(tip), _p(dtip))
        if rc != 0:
            raise ValueError("oracle_jvp refused the rod (code %d)" % rc)
        return tip, dtip

    def vjp(self, state, n_steps, ct, round_fp32=False, t0=0.0):
        """Reverse mode: gradient of sum_s ct[s] . tip(s) as a dict with x, v, q, w (state
        shapes), bend, twist (multiplier gradients) and tip (the forward trajectory)."""
        x, v, q, w = self._state64(state)
        ct = _f64(ct, (int(n_steps), 3))
        g = {k: np.zeros_like(a) for k, a in (("x", x), ("v", v), ("q", q), ("w", w))}
        gb, gt = C.c_double(0.0), C.c_double(0.0)
        tip = np.zeros((int(n_steps), 3))
        rc = lib().oracle_vjp(C.byref(self.c), float(t0), int(n_steps), _p(x), _p(v), _p(q),
                              _p(w), _p(ct), int(round_fp32), _p(g["x"]), _p(g["v"]),
                              _p(g["q"]), _p(g["w"]), C.byref(gb), C.byref(gt), _p(tip))
        if rc != 0:
            raise ValueError("oracle_vjp refused the rod (code %d)" % rc)
        g["bend"], g["twist"], g["tip"] = float(gb.value), float(gt.value), tip
        return g

    def stable(self, state, n_steps, t0=0.0, energy_factor=1.01):
        x, v = _f64(state.x, (self.n + 1, 3)), _f64(state.v, (self.n + 1, 3))
        q, w = _f64(state.q, (self.n, 4)), _f64(state.w, (self.n, 3))
        return bool(lib().oracle_stable(C.byref(self.c), float(t0), int(n_steps), _p(x),
                                        _p(v), _p(q), _p(w), float(energy_factor)))


def bmat(k):
    out = np.zeros(16)
    lib().oracle_bmat(int(k), _p(out))
    return out.reshape(4, 4)


def rotmat(q):
    q = _f64(q, (4,))
    out = np.zeros(9)
    lib().oracle_rotmat(_p(q), _p(out))
    return out.reshape(3, 3)


def qmul(a, b):
    a, b = _f64(a, (4,)), _f64(b, (4,))
    r = np.zeros(4)
    lib().oracle_qmul(_p(a), _p(b), _p(r))
    return r


def bind_impulse(xa, va, wa, xb, vb, wb, dt, one_way):
    """One binding impulse (zero-length distance constraint); returns the new (va, vb)."""
    xa, xb = _f64(xa, (3,)), _f64(xb, (3,))
    va, vb = _f64(va, (3,)).copy(), _f64(vb, (3,)).copy()
    lib().oracle_bind_impulse(_p(xa), _p(va), float(wa), _p(xb), _p(vb), float(wb), float(dt),
                              int(bool(one_way)))
    return va, vb


def rollout_pair(spec_a, spec_b, state_a, state_b, point_a, point_b, one_way, n_steps, t0=0.0):
    """Two rods bound point_a[k] <-> point_b[k] (rod b the master if one_way), n_steps steps;
    returns the new (state_a, state_b); the inputs are not modified."""
    ra, rb = Rod(spec_a), Rod(spec_b)
    ia = np.ascontiguousarray(np.asarray(point_a, dtype=np.int32))
    ib = np.ascontiguousarray(np.asarray(point_b, dtype=np.int32))
    if ia.shape != ib.shape:
        raise ValueError("point_a and point_b differ in length")
    bd = _Binding(len(ia), ia.ctypes.data_as(C.POINTER(C.c_int32)),
                  ib.ctypes.data_as(C.POINTER(C.c_int32)), int(bool(one_way)))
    out = []
    arrs = []
    for r, st in ((ra, state_a), (rb, state_b)):
        o = st.copy()
        o.x, o.v = _f64(st.x, (r.n + 1, 3)).copy(), _f64(st.v, (r.n + 1, 3)).copy()
        o.q, o.w = _f64(st.q, (r.n, 4)).copy(), _f64(st.w, (r.n, 3)).copy()
        out.append(o)
        arrs += [o.x, o.v, o.q, o.w]
    lib().oracle_rollout_pair(C.byref(ra.c), C.byref(rb.c), C.byref(bd), float(t0), int(n_steps),
                              *[_p(a) for a in arrs])
    return out[0], out[1]


def self_skip(spec):
    return int(lib().oracle_self_skip(C.byref(Rod(spec).c)))


def rollout_group(specs, states, n_steps, mu=None, pairs=None, one_way=False, t0=0.0,
                  round_mask=0):
    """One or two rods stepped together: optional bindings (pairs: (k, 2) point indices of
    rod 0 and rod 1, rod 1 the master if one_way) and optional contact with friction
    coefficient mu.  round_mask (1 x, 2 v, 4 q, 8 w): those fields rounded to FP32 after every
    step.  Returns (new states, largest number of contacts of one point)."""
    rods = [Rod(s) for s in specs]
    outs, keep = [], []
    for r, st in zip(rods, states):
        o = st.copy()
        o.x, o.v = _f64(st.x, (r.n + 1, 3)).copy(), _f64(st.v, (r.n + 1, 3)).copy()
        o.q, o.w = _f64(st.q, (r.n, 4)).copy(), _f64(st.w, (r.n, 3)).copy()
        outs.append(o)
    rp = (C.POINTER(_Rod) * len(rods))(*[C.pointer(r.c) for r in rods])
    arr = lambda k: (_DP * len(outs))(*[_p(getattr(o, k)) for o in outs])
    bd = None
    if pairs is not None:
        pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
        ia, ib = np.ascontiguousarray(pr[:, 0]), np.ascontiguousarray(pr[:, 1])
        keep += [ia, ib]
        bd = _Binding(len(pr), ia.ctypes.data_as(C.POINTER(C.c_int32)),
                      ib.ctypes.data_as(C.POINTER(C.c_int32)), int(bool(one_way)))
    ct = _Contact(float(mu)) if mu is not None else None
    most = C.c_int32(0)
    bp = C.byref(bd) if bd is not None else None
    cp = C.byref(ct) if ct is not None else None
    if round_mask:
        lib().oracle_rollout_group_rounded(rp, len(rods), bp, cp, float(t0), int(n_steps),
                                           arr("x"), arr("v"), arr("q"), arr("w"),
                                           int(round_mask), C.byref(most))
    else:
        lib().oracle_rollout_group(rp, len(rods), bp, cp, float(t0), int(n_steps), arr("x"),
                                   arr("v"), arr("q"), arr("w"), C.byref(most))
    return outs, int(most.value)


def rollout_many(specs_states, n_steps, t0=0.0, tip=False):
    """Roll out several independent rods (one oracle call each)."""
    return [Rod(s).rollout(st, n_steps, t0, tip) for s, st in specs_states]


def bisect_dt_max(spec, state, n_steps, lo=1e-9, hi=1e-1, rel=1e-3, t0=0.0):
    """Largest stable dt by bisection in log space (stability as in ``Rod.stable``).

    ``lo`` must be stable and ``hi`` unstable; the interval is halved in log(dt) until
    hi / lo <= 1 + rel.  Returns the stable end ``lo``.
    """
    import dataclasses
    import math
    mk = lambda dt: Rod(dataclasses.replace(spec, dt=float(dt)))
    if not mk(lo).stable(state, n_steps, t0):
        raise ValueError("lower bracket is not stable")
    if mk(hi).stable(state, n_steps, t0):
        return hi
    while hi / lo > 1.0 + rel:
        mid = math.exp(0.5 * (math.log(lo) + math.log(hi)))
        if mk(mid).stable(state, n_steps, t0):
            lo = mid
        else:
            hi = mid
    return lo


def _ptrs(arrs):
    return (_DP * len(arrs))(*[_p(a) for a in arrs])


def vjp_many(specs_states, n_steps, cts, round_fp32=False, n_threads=0, t0=0.0):
    """``Rod.vjp`` for many independent rods, spread over n_threads threads in the oracle's
    own thread pool (0 = all hardware threads).  Returns a list of gradient dicts."""
    rods = [Rod(s) for s, _ in specs_states]
    arr = (_Rod * len(rods))(*[r.c for r in rods])
    ins = [r._state64(st) for r, (_, st) in zip(rods, specs_states)]
    cts = [_f64(c, (int(n_steps), 3)) for c in cts]
    outs = [{k: np.zeros_like(a) for k, a in zip(("x", "v", "q", "w"), s4)} for s4 in ins]
    tips = [np.zeros((int(n_steps), 3)) for _ in rods]
    gb = np.zeros(len(rods))
    gt = np.zeros(len(rods))
    rc = lib().oracle_vjp_many(len(rods), arr, float(t0), int(n_steps),
                               *[_ptrs([s4[k] for s4 in ins]) for k in range(4)], _ptrs(cts),
                               int(round_fp32),
                               *[_ptrs([o[k] for o in outs]) for k in ("x", "v", "q", "w")],
                               _p(gb), _p(gt), _ptrs(tips), int(n_threads))
    if rc != 0:
        raise ValueError("oracle_vjp_many refused a rod (code %d)" % rc)
    for o, b, t, tp in zip(outs, gb, gt, tips):
        o["bend"], o["twist"], o["tip"] = float(b), float(t), tp
    return outs


def rollout_many_threads(specs_states, n_steps, n_threads=0, t0=0.0):
    """oracle rollouts of many independent rods on n_threads threads of the oracle's own pool
    (0 = all hardware threads); returns the new states."""
    rods = [Rod(s) for s, _ in specs_states]
    arr = (_Rod * len(rods))(*[r.c for r in rods])
    ins = [r._state64(st) for r, (_, st) in zip(rods, specs_states)]
    rc = lib().oracle_rollout_many(len(rods), arr, float(t0), int(n_steps),
                                   *[_ptrs([s4[k] for s4 in ins]) for k in range(4)],
                                   int(n_threads))
    if rc != 0:
        raise ValueError("oracle_rollout_many refused a rod")
    out = []
    for (_, st), (x, v, q, w) in zip(specs_states, ins):
        o = st.copy()
        o.x, o.v, o.q, o.w = x, v, q, w
        out.append(o)
    return out
