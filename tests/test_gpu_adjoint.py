"""GPU adjoint: gradients of a tip-trajectory loss computed by the hand-written reverse kernel
(through the C ABI) against FP64 central finite differences of the oracle rollout on the same
inputs and targets.  Loss: L = mean over (rods, steps, xyz) of (tip - target)^2, targets from
the oracle with perturbed stiffness and initial velocity."""

import numpy as np
import pytest

from paper_2509_04277_amd import rod as R
from paper_2509_04277_amd import workloads as W
import parity_metrics as PM

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[gpu-test] " + msg, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    yield


def _mixed_rods(oracle):
    rng = np.random.default_rng(60)
    rods = []
    # c4-like clamped inextensible rod
    for spec, st in W.config4(n_rods=1, n=96).rods:
        rods.append((spec, st))
    # extensible rod with a driven clamp
    x, q = W.curved_rod(64, 1.0 / 64, rng, sigma=0.05, twist_sigma=0.05)
    spec = W.RodSpec(n=64, inextensible=False, n_iter=0, clamp=True, dt=0.0,
                     gravity=(0.0, 0.0, -9.81), damp_lin=0.1, damp_ang=0.1, poisson=0.5,
                     density=1000.0, seg_len=np.full(64, 1.0 / 64), radius=np.full(64, 0.01),
                     young=np.full(64, 1e6), clamp_x0=tuple(x[0]), clamp_q0=tuple(q[0]),
                     clamp_amp=(0.0, 2e-3, 1e-3), clamp_twist_amp=0.1,
                     clamp_twist_axis=(1.0, 0.0, 0.0), clamp_freq=3.0, clamp_phase_x=0.2,
                     clamp_phase_twist=0.9)
    st = W.RodState(x, np.zeros((65, 3)), q, np.zeros((64, 3)))
    xc, qc, _ = oracle.Rod(spec.replace(dt=1.0)).clamp_pose(0.0)
    st.x = st.x - st.x[0] + xc
    st.q[0] = qc
    rods.append((spec, st))
    # free inextensible rod with intrinsic curvature and non-uniform material
    x, q = W.curved_rod(40, 0.02, rng, sigma=0.1, twist_sigma=0.1)
    spec = W.RodSpec(n=40, inextensible=True, n_iter=6, clamp=False, dt=0.0,
                     gravity=(0.0, 0.0, -9.81), damp_lin=0.2, damp_ang=0.3, poisson=0.4,
                     density=1000.0, seg_len=np.full(40, 0.02), radius=rng.uniform(4e-3, 6e-3, 40),
                     young=rng.uniform(5e5, 2e6, 40), u_hat=rng.normal(0, 1.0, (39, 3)))
    st = W.RodState(x, rng.normal(0, 1e-2, (41, 3)), q, rng.normal(0, 0.1, (40, 3)))
    rods.append((spec, st))
    out = []
    for spec, st in rods:
        dt = oracle.Rod(spec.replace(dt=1.0)).dt_rule()
        spec = spec.replace(dt=dt)
        if spec.clamp_freq:
            spec = spec.replace(clamp_freq=1.0 / (60 * dt))
        out.append((spec, st))
    return PM.fp32_rods(out)   # the oracle starts from exactly the GPU's input


def _targets(oracle, rods, n_steps, rng):
    tg = []
    for spec, st in rods:
        sp = spec.replace(bend_scale=spec.bend_scale * (1 + rng.uniform(-0.3, 0.3)),
                          twist_scale=spec.twist_scale * (1 + rng.uniform(-0.3, 0.3)))
        s2 = st.copy()
        s2.v = s2.v + rng.normal(0, 1e-2, s2.v.shape)
        tg.append(oracle.Rod(sp).rollout(s2, n_steps, tip=True)[1])
    return np.stack(tg)


def _oracle_functional(oracle, rods, weights, n_steps, mult=None, states=None):
    """sum_r sum_s weights[r, s] . tip_r(s) with the FP64 oracle (a fixed cotangent)."""
    tot = 0.0
    for r, (spec, st) in enumerate(rods):
        if mult is not None:
            spec = spec.replace(bend_scale=spec.bend_scale * mult[r][0],
                                twist_scale=spec.twist_scale * mult[r][1])
        s = states[r] if states is not None else st
        tip = oracle.Rod(spec).rollout(s, n_steps, tip=True)[1]
        tot += float(np.sum(weights[r] * tip))
    return tot


def _oracle_loss(oracle, rods, targets, n_steps, mult=None, states=None):
    L = 0.0
    for r, (spec, st) in enumerate(rods):
        if mult is not None:
            spec = spec.replace(bend_scale=spec.bend_scale * mult[r][0],
                                twist_scale=spec.twist_scale * mult[r][1])
        s = states[r] if states is not None else st
        tip = oracle.Rod(spec).rollout(s, n_steps, tip=True)[1]
        L += np.sum((tip - targets[r]) ** 2)
    return L / (len(rods) * n_steps * 3)


def _gpu_vjp(rods, weights, n_steps, ckpt):
    b = R.RodBatch([s for s, _ in rods])
    b.set_state_rods([st for _, st in rods])
    tips = b.adjoint_forward(n_steps, ckpt)
    g = b.adjoint_backward(np.ascontiguousarray(weights, dtype=np.float32))
    b.close()
    return tips, g


def _gpu_grads(rods, targets, n_steps, ckpt):
    b = R.RodBatch([s for s, _ in rods])
    b.set_state_rods([st for _, st in rods])
    tips = b.adjoint_forward(n_steps, ckpt)
    M = len(rods) * n_steps * 3
    dtips = np.ascontiguousarray((2.0 / M) * (tips.astype(np.float64) - targets), dtype=np.float32)
    g = b.adjoint_backward(dtips)
    loss = float(np.sum((tips.astype(np.float64) - targets) ** 2) / M)
    b.close()
    return loss, g


def _split(rods, flat, k):
    out, o = [], 0
    for spec, _ in rods:
        m = (spec.n + 1) if k in ("x", "v") else spec.n
        c = 4 if k == "q" else 3
        out.append(flat[o:o + m * c].reshape(m, c))
        o += m * c
    return out


def _random_state_dirs(rods, rng):
    scale = {"x": 1e-3, "v": 1e-2, "q": 1e-3, "w": 1e-1}
    dirs = {k: [scale[k] * rng.normal(size=getattr(st, k).shape) for _, st in rods]
            for k in ("x", "v", "q", "w")}
    for r, (spec, _) in enumerate(rods):
        if spec.clamp:   # the base point and frame 0 follow the clamp: leave them fixed
            dirs["x"][r][0] = 0.0
            dirs["q"][r][0] = 0.0
    return dirs


def _shift(rods, dirs, eps):
    return [W.RodState(*(getattr(st, k) + eps * dirs[k][r] for k in ("x", "v", "q", "w")))
            for r, (_, st) in enumerate(rods)]


def _dot_state(rods, g, dirs):
    tot = 0.0
    for k in ("x", "v", "q", "w"):
        for gr, d in zip(_split(rods, g[k], k), dirs[k]):
            tot += float(np.sum(gr.astype(np.float64) * d))
    return tot


# Relative error in norm allowed per gradient block (bend and twist multipliers, x0, v0, q0,
# w0) against the FP64 oracle's reverse-mode gradient, and against central differences of the
# FP64 oracle rollout.
VJP_RTOL = 1e-4
BLOCKS = ("bend", "twist", "x", "v", "q", "w")


def _oracle_vjp(oracle, rods, weights, n_steps):
    """The FP64 oracle's reverse-mode gradient of sum_s weights[r, s] . tip_r(s), per rod."""
    return oracle.vjp_many(rods, n_steps, [weights[r] for r in range(len(rods))])


def _block_errors(rods, g, ref, idx=None):
    """Relative error in norm of each gradient block of the GPU result g (library layout)
    against the per-rod oracle gradients ref, over the rods idx (all by default)."""
    idx = range(len(rods)) if idx is None else idx
    out = {}
    for k in ("bend", "twist"):
        a = np.array([float(g[k][r]) for r in idx])
        b = np.array([ref[r][k] for r in idx])
        out[k] = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    for k in ("x", "v", "q", "w"):
        parts = _split(rods, g[k], k)
        a = np.concatenate([parts[r].astype(np.float64).ravel() for r in idx])
        b = np.concatenate([ref[r][k].ravel() for r in idx])
        out[k] = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    return out


def test_vjp_matches_oracle_gradient(oracle):
    """Vector-Jacobian product for a fixed random cotangent w on the tip trajectory: every
    block of the GPU adjoint against the FP64 oracle's reverse-mode gradient (three mixed rods:
    clamped inextensible, driven extensible, free inextensible with intrinsic curvature)."""
    rods = _mixed_rods(oracle)
    n_steps = 60
    rng = np.random.default_rng(64)
    weights = rng.normal(0, 1.0, (len(rods), n_steps, 3))
    _say("VJP vs oracle gradient: 3 mixed rods, %d steps, checkpoints every 16" % n_steps)
    tips, g = _gpu_vjp(rods, weights, n_steps, 16)
    ref = _oracle_vjp(oracle, rods, weights, n_steps)
    errs = _block_errors(rods, g, ref)
    _say("VJP relative error in norm per block: " +
         " ".join("%s %.2e" % (k, errs[k]) for k in BLOCKS))
    for k in BLOCKS:
        assert errs[k] <= VJP_RTOL, (k, errs[k])


def test_vjp_matches_finite_differences(oracle):
    """The same VJP against central differences of the FP64 oracle rollout: per-rod stiffness
    multipliers, and each initial-state block along a random direction."""
    rods = _mixed_rods(oracle)
    n_steps = 60
    rng = np.random.default_rng(64)
    weights = rng.normal(0, 1.0, (len(rods), n_steps, 3))
    tips, g = _gpu_vjp(rods, weights, n_steps, 16)
    h = 1e-4
    errs = {}
    for k, name in ((0, "bend"), (1, "twist")):
        fds, gots = [], []
        for r in range(len(rods)):
            mp = [[1.0, 1.0] for _ in rods]
            mm = [[1.0, 1.0] for _ in rods]
            mp[r][k] += h
            mm[r][k] -= h
            fds.append((_oracle_functional(oracle, rods, weights, n_steps, mp) -
                        _oracle_functional(oracle, rods, weights, n_steps, mm)) / (2 * h))
            gots.append(float(g[name][r]))
            _say("rod %d d<w,tip>/dm_%s: gpu %.8e fd %.8e" % (r, name, gots[-1], fds[-1]))
        errs[name] = np.linalg.norm(np.array(gots) - fds) / np.linalg.norm(fds)
    # initial state, one block at a time: a random direction d in the block, the error of
    # <g, d> against central differences relative to |g_block| |d| (a bound that follows from
    # the per-block relative error in norm, and does not blow up when <g, d> is near zero)
    worst_state = 0.0
    for blk in ("x", "v", "q", "w"):
        dirs = _random_state_dirs(rods, rng)
        for k in dirs:
            if k != blk:
                dirs[k] = [0.0 * d for d in dirs[k]]
        eps = 1e-4
        fd = (_oracle_functional(oracle, rods, weights, n_steps, states=_shift(rods, dirs, eps)) -
              _oracle_functional(oracle, rods, weights, n_steps, states=_shift(rods, dirs, -eps))) / (2 * eps)
        got = _dot_state(rods, g, dirs)
        gn = np.linalg.norm(g[blk].astype(np.float64))
        dn = np.sqrt(sum(float(np.sum(d * d)) for d in dirs[blk]))
        rel = abs(got - fd) / (gn * dn)
        worst_state = max(worst_state, rel)
        _say("state block %s: gpu %.8e fd %.8e, |err| / (|g| |d|) %.2e" % (blk, got, fd, rel))
    _say("VJP vs FD relative error: bend %.2e twist %.2e, initial state (worst block) %.2e"
         % (errs["bend"], errs["twist"], worst_state))
    assert errs["bend"] <= VJP_RTOL and errs["twist"] <= VJP_RTOL and worst_state <= VJP_RTOL


def test_loss_gradient_matches_finite_differences(oracle):
    """End-to-end gradient of the MSE tip loss (targets from perturbed stiffness and initial
    velocity): the GPU's residuals come from its own FP32 trajectory, so this also carries the
    forward's FP32 error in (tip - target)."""
    rods = _mixed_rods(oracle)
    n_steps = 60
    rng = np.random.default_rng(61)
    targets = _targets(oracle, rods, n_steps, rng)
    _say("loss gradient: 3 mixed rods, %d steps, checkpoints every 16" % n_steps)
    loss, g = _gpu_grads(rods, targets, n_steps, 16)
    loss_o = _oracle_loss(oracle, rods, targets, n_steps)
    _say("loss gpu %.8e oracle %.8e" % (loss, loss_o))
    assert abs(loss / loss_o - 1) < 1e-4
    h = 1e-4
    for k, name in ((0, "bend"), (1, "twist")):
        fds, gots = [], []
        for r in range(len(rods)):
            mp = [[1.0, 1.0] for _ in rods]
            mm = [[1.0, 1.0] for _ in rods]
            mp[r][k] += h
            mm[r][k] -= h
            fds.append((_oracle_loss(oracle, rods, targets, n_steps, mp) -
                        _oracle_loss(oracle, rods, targets, n_steps, mm)) / (2 * h))
            gots.append(float(g[name][r]))
            _say("rod %d dL/dm_%s: gpu %.8e fd %.8e" % (r, name, gots[-1], fds[-1]))
        rel = np.linalg.norm(np.array(gots) - fds) / np.linalg.norm(fds)
        _say("dL/dm_%s block: relative error in norm %.2e" % (name, rel))
        assert rel <= VJP_RTOL


def test_checkpointing_is_bitwise():
    rods = [(s.replace(dt=R.stable_dt(s)), st) for s, st in W.config4(n_rods=3, n=64).rods]
    n_steps = 45
    rng = np.random.default_rng(62)
    targets = np.stack([st.x[-1] + rng.normal(0, 1e-3, (n_steps, 3)) for _, st in rods])
    _say("adjoint checkpoints every 1 / 7 / 45 steps, 3 rods x 64")
    res = [_gpu_grads(rods, targets, n_steps, ck)[1] for ck in (1, 7, 45)]
    for k in ("bend", "twist", "x", "v", "q", "w"):
        assert np.array_equal(res[0][k], res[1][k]) and np.array_equal(res[0][k], res[2][k]), k


def test_adjoint_full_size(oracle):
    """256 rods x 256 elements, 400 steps, checkpoints every 20 (the adjoint workload): every
    gradient block of all 256 rods against the FP64 oracle's reverse-mode gradient, and the
    multiplier gradients of two sampled rods against oracle central differences."""
    wl = W.config4()
    rods = PM.fp32_rods([(s.replace(dt=R.stable_dt(s)), st) for s, st in wl.rods])
    n_steps = wl.n_steps
    rng = np.random.default_rng(63)
    weights = rng.normal(0, 1.0, (len(rods), n_steps, 3))
    _say("adjoint full size: 256 x 256, 400 steps, ckpt 20")
    tips, g = _gpu_vjp(rods, weights, n_steps, 20)
    ref = _oracle_vjp(oracle, rods, weights, n_steps)
    errs = _block_errors(rods, g, ref)
    per_rod = {k: max(_block_errors(rods, g, ref, [r])[k] for r in range(0, len(rods), 15))
               for k in ("bend", "twist")}
    _say("full size, all rods, relative error in norm per block: " +
         " ".join("%s %.2e" % (k, errs[k]) for k in BLOCKS) +
         "; worst single rod (every 15th): bend %.2e twist %.2e" % (per_rod["bend"], per_rod["twist"]))
    h = 1e-4
    for k, name in ((0, "bend"), (1, "twist")):
        for i in (5, 200):
            vals = []
            for sgn in (1, -1):
                spec, st = rods[i]
                m = [1.0, 1.0]
                m[k] += sgn * h
                sp = spec.replace(bend_scale=spec.bend_scale * m[0], twist_scale=spec.twist_scale * m[1])
                tip = oracle.Rod(sp).rollout(st, n_steps, tip=True)[1]
                vals.append(float(np.sum(weights[i] * tip)))
            fd = (vals[0] - vals[1]) / (2 * h)
            got = float(g[name][i])
            _say("rod %d d<w,tip>/dm_%s: gpu %.8e oracle %.8e fd %.8e rel(fd) %.2e" % (
                i, name, got, ref[i][name], fd, abs(got - fd) / abs(fd)))
            assert abs(got - fd) <= VJP_RTOL * abs(fd), (i, name)
    for k in BLOCKS:
        assert errs[k] <= VJP_RTOL, (k, errs[k])


def test_torch_autograd_function(oracle):
    """RodRollout (torch.autograd.Function): autograd through the library adjoint agrees with
    the direct C-ABI calls, and the gradient of a tip loss drives a decrease of the loss."""
    import torch
    rods = [(s.replace(dt=R.stable_dt(s)), st) for s, st in W.config4(n_rods=4, n=64).rods]
    n_steps = 50
    b = R.RodBatch([s for s, _ in rods])
    cat = lambda k: torch.tensor(np.concatenate([getattr(st, k).reshape(-1) for _, st in rods]),
                                 dtype=torch.float32, device="cuda")
    x0, v0, q0, w0 = (cat(k) for k in ("x", "v", "q", "w"))
    rng = np.random.default_rng(65)
    target = torch.tensor(np.stack([st.x[-1] + rng.normal(0, 2e-3, 3) for _, st in rods]),
                          dtype=torch.float32, device="cuda")
    bend = torch.ones(4, device="cuda", requires_grad=True)
    twist = torch.ones(4, device="cuda", requires_grad=True)
    v0 = v0.clone().requires_grad_(True)
    Fn = R.rollout_function()
    _say("torch autograd through the adjoint: 4 rods x 64, %d steps" % n_steps)
    tips = Fn.apply(b, bend, twist, x0, v0, q0, w0, n_steps, 10)
    loss = ((tips - target[:, None, :]) ** 2).mean()
    loss.backward()
    # same gradients through the raw calls
    b2 = R.RodBatch([s for s, _ in rods])
    b2.set_state(x0, v0.detach(), q0, w0)
    t2 = b2.adjoint_forward(n_steps, 10)
    d = (2.0 / t2.size) * (t2.astype(np.float64) - target.cpu().numpy()[:, None, :])
    g2 = b2.adjoint_backward(np.ascontiguousarray(d, dtype=np.float32))
    b2.close()
    # torch forms dL/dtip in FP32, the direct path in FP64: agreement to FP32 rounding
    gb, gv2 = bend.grad.cpu().numpy(), v0.grad.cpu().numpy()
    assert np.abs(gb - g2["bend"]).max() <= 1e-3 * np.abs(g2["bend"]).max()
    assert np.abs(gv2 - g2["v"]).max() <= 1e-3 * np.abs(g2["v"]).max()
    # one gradient step on the initial velocities lowers the loss
    with torch.no_grad():
        gv = v0.grad
        step = 0.1 * float(loss) / float((gv * gv).sum())
        v1 = (v0 - step * gv).detach()
    tips1 = Fn.apply(b, bend.detach(), twist.detach(), x0, v1, q0, w0, n_steps, 10)
    loss1 = ((tips1 - target[:, None, :]) ** 2).mean()
    _say("loss %.6e -> %.6e after one gradient step on v0" % (float(loss), float(loss1)))
    assert float(loss1) < float(loss)
    b.close()


def test_stale_rollout_is_refused():
    """Two RodRollout applications on one handle before backward: the second replaces the
    rollout the handle holds, so the first graph's backward is refused (ROD_E_ORDER) instead
    of returning the second rollout's gradients; the second graph's backward still works."""
    import torch
    rods = [(s.replace(dt=R.stable_dt(s)), st) for s, st in W.config4(n_rods=2, n=64).rods]
    b = R.RodBatch([s for s, _ in rods])
    cat = lambda k: torch.tensor(np.concatenate([getattr(st, k).reshape(-1) for _, st in rods]),
                                 dtype=torch.float32, device="cuda")
    x0, v0, q0, w0 = (cat(k) for k in ("x", "v", "q", "w"))
    Fn = R.rollout_function()
    bend1 = torch.ones(2, device="cuda", requires_grad=True)
    bend2 = torch.ones(2, device="cuda", requires_grad=True)
    twist = torch.ones(2, device="cuda")
    _say("two rollouts on one handle, backward of the first")
    t1 = Fn.apply(b, bend1, twist, x0, v0, q0, w0, 20, 5)
    t2 = Fn.apply(b, bend2, twist, x0, v0, q0, w0, 20, 5)
    with pytest.raises(R.RodError, match="ORDER"):
        t1.sum().backward()
    t2.sum().backward()
    assert bend2.grad is not None and torch.isfinite(bend2.grad).all()
    b.close()


def test_adjoint_in_two_exchange_forms():
    """Rods of 300 elements: the adjoint in four wavefronts of two elements per lane (whose
    exchanges merge the mailbox word into the lane move) and in eight wavefronts of one (plain
    exchanges) sees the same forward tips, bitwise, and returns the same gradients up to the
    rounding of the reverse pass's shape (two elements per lane share one impulse adjoint per
    in-lane segment): measured at most 2e-5 of the largest entry of a block (the same before
    the exchange had two forms), asserted at the adjoint's 1e-4 target; a lost base-point value
    or neighbour word moves a block by far more."""
    rods = [(s.replace(dt=R.stable_dt(s)), st) for s, st in W.config4(n_rods=2, n=300).rods]
    n_steps = 40
    rng = np.random.default_rng(71)
    targets = np.stack([st.x[-1] + rng.normal(0, 1e-3, (n_steps, 3)) for _, st in rods])
    res = []
    for shape in ((4, 2), (8, 1)):
        b = R.RodBatch([s for s, _ in rods])
        b.set_tuning(shape[0], shape[1], 10)
        b.set_state_rods([st for _, st in rods])
        tips = b.adjoint_forward(n_steps, 20)
        M = len(rods) * n_steps * 3
        dtips = np.ascontiguousarray((2.0 / M) * (tips.astype(np.float64) - targets), dtype=np.float32)
        g = b.adjoint_backward(dtips)
        b.close()
        res.append((tips, g))
    assert np.array_equal(res[0][0], res[1][0])
    for k in ("x", "v", "q", "w", "bend", "twist"):
        a, c = (np.asarray(r[1][k], dtype=np.float64) for r in res)
        rel = float(np.abs(a - c).max() / max(np.abs(a).max(), 1e-30))
        _say("(4, 2) against (8, 1), %s: largest difference %.2e of the largest entry" % (k, rel))
        assert rel <= 1e-4, k
