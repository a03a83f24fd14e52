"""Benchmark of the CoRdE rod stepper on one MI355X.

Workload: two inextensible 512-element rods (catheter / guidewire-like: rod A r = 0.5 mm,
E = 2 GPa; rod B r = 0.2 mm, E = 50 GPa with a 5 GPa tip), driven clamps, 10 constraint
iterations, 10 time steps per kernel launch.  A benchmark "step" is one time step of both
rods (forces, force integration, constraint impulses, velocity integration).

Prints one JSON line: element-steps/s over the timed steps (device state resident in HBM),
microseconds per step, the roofline of the step kernel (HBM, 104 algorithmic bytes per
element-step: the 52-byte FP32 state read and written) with the kernel duration measured by
HIP events on the library's stream, and the FP64 CPU oracle timed on the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

REPO = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, REPO)

BYTES_PER_ELEMENT_STEP = 104          # 13 FP32 state values read + written per element
HBM_PEAK_GBS = 8000.0                 # MI355X HBM3E

# Floating-point operations of the method per element (one segment, point, frame and joint)
# and step, by part of the step (add, subtract, multiply: 1; a multiply-add: 2; division,
# square root, reciprocal square root: 1), with shared subexpressions evaluated once and
# per-element material coefficients computed once per rod (Sec. 2.1):
#   segment   segment vector, tangent, directors d1..d3 of the frame, penalty force and torque
#             (eqs. (7)-(8)); stretch: the extensible variant's stretch force (eq. (2));
#   joint     relative rotation of neighbouring frames, moment K (u - u_hat) (eqs. (3), (5),
#             (6)) and the torques on both frames;
#   accumulate  the net force on a point and torque on a frame from their neighbours;
#   point, frame  force and torque integration with damping and the gyroscopic term;
#   impulse   one distance-constraint impulse per segment and constraint iteration;
#   advance   the velocity integration of the point and of the frame's quaternion, renormalised.
# The per-rod clamp pose is not counted.
FLOPS_PER_ROW = {"segment": 70, "stretch": 9, "joint": 52, "accumulate": 8, "point": 18,
                 "frame": 21, "advance": 46, "impulse": 32}
# MI355X FP32 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 (multiply-add) x 2.4 GHz = 78.6
# TFLOP/s, twice that with packed FP32 instructions (the published 157.3; the kernels here are
# built without packed FP32).
FP32_VECTOR_PEAK_TFLOPS = 157.3
FP32_UNPACKED_PEAK_TFLOPS = 78.6


def flops_per_element_step(inextensible, n_iter):
    r = FLOPS_PER_ROW
    base = r["segment"] + r["joint"] + r["accumulate"] + r["point"] + r["frame"] + r["advance"]
    return base + (r["impulse"] * n_iter if inextensible else r["stretch"])


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("paper_2509_04277_amd/csrc/rod_kernels.hpp", "paper_2509_04277_amd/csrc/rod_lib.hip",
              "paper_2509_04277_amd/build.py"):
        h.update(open(os.path.join(REPO, f), "rb").read())
    return h.hexdigest()[:16]


def _counters(kernel_name, elements, spl):
    """Figures of committed rocprofv3 counter runs of this kernel on this workload, if they
    were taken on the current kernel sources (else None)."""
    path = os.path.join(REPO, "profiles", "counters.json")
    if not os.path.exists(path):
        return None
    e = json.load(open(path)).get(kernel_name)
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    if e.get("elements") != elements or e.get("steps_per_launch") != spl:
        return None
    return e


def measured_batch_issue(wl, ms, buckets):
    """VALU issue of the batched rollout: the wave-level VALU instructions that the committed
    counter run of this workload counted (same kernel sources and buckets), each 4 cycles of a
    16-lane SIMD, over the chip's 1024 SIMDs at 2.4 GHz, as a fraction of the rollout time;
    with the executed FP32 operations (a multiply-add counted twice).  None without counters."""
    path = os.path.join(REPO, "profiles", "counters.json")
    if not os.path.exists(path):
        return None
    e = json.load(open(path)).get("c3_batch")
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    if e.get("elements") != wl.n_elements or e.get("steps") != wl.n_steps:
        return None
    if [list(b) for b in e["buckets"]] != [[w, k, n] for w, k, n, _ in buckets]:
        return None
    issue_s = e["valu_insts_per_rollout"] * 4 / (256 * 4) / 2.4e9
    return {"valu_issue_frac": issue_s / (ms / 1e3),
            "valu_insts_per_rollout": e["valu_insts_per_rollout"],
            "executed_fp32_tflops": e["fp32_flops_per_rollout"] / (ms / 1e3) / 1e12}


def measured_traffic(kernel_name, elements, spl):
    """HBM bytes per launch (copy-calibrated FETCH_SIZE + WRITE_SIZE), or None."""
    e = _counters(kernel_name, elements, spl)
    return None if e is None else e["fetch_bytes_per_launch"] + e["write_bytes_per_launch"]


def measured_wave_shares(kernel_name, elements, spl):
    """Shares of wavefront time from SQ counters: VALU issue (SQ_ACTIVE_INST_VALU /
    SQ_WAVE_CYCLES) and waiting (SQ_WAIT_ANY / SQ_WAVE_CYCLES: barriers, and the few memory
    waits of a register-resident kernel), or None."""
    e = _counters(kernel_name, elements, spl)
    if e is None or "valu_active_share" not in e:
        return None
    return {"valu_issue_frac": e["valu_active_share"], "barrier_share": e["wait_any_share"],
            "valu_insts_per_wave_step": e.get("valu_insts_per_wave_step"),
            "fp32_flops_per_element_step": e.get("fp32_flops_per_element_step")}


def host_cpu():
    """Model name and logical CPU counts of the machine running the oracle."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def oracle_threads():
    """Worker threads for the oracle's own pool: the CPUs this process may use, at most 16
    (the host share of one GPU)."""
    return max(1, min(16, host_cpu()["usable_cpus"] or 1))


COPY_FLOATS = 64 << 20                # 256 MiB FP32 copy: 512 MiB of HBM traffic per dispatch


def copy_bandwidth(torch, reps=20):
    """STREAM-style copy (one elementwise copy kernel of 256 MiB read + 256 MiB written): the
    measured HBM rate, and the dispatch whose FETCH_SIZE / WRITE_SIZE calibrate the counters."""
    src = torch.ones(COPY_FLOATS, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = 2 * 4 * COPY_FLOATS
    del src, dst
    return {"bytes_per_dispatch": nbytes, "ms": ms, "GB/s": nbytes / (ms / 1e3) / 1e9}


def cpu_baseline(wl, n_steps):
    from oracle import oracle as O
    t = time.perf_counter()
    for spec, st in wl.rods:
        O.Rod(spec).rollout(st, n_steps)
    dt = time.perf_counter() - t
    return {"value": wl.n_elements * n_steps / dt, "unit": "element-steps/s", "cores": 1,
            "kind": "oracle", "host": host_cpu(),
            "sample": "FP64 C oracle, both 512-element rods of the same workload, %d steps "
                      "(%.1f s), one thread (each rod's steps are a sequential chain)" % (n_steps, dt)}


def cpu_oracle_many(W, R):
    """The FP64 oracle on the batched (4096 rods) and adjoint (256 x 256) workloads, rods spread
    over the host's cores by the oracle's thread pool: a bounded sample of each."""
    from oracle import oracle as O
    nt = oracle_threads()
    out = {"threads": nt, "host": host_cpu()}
    wl = W.config3()
    rods = [(s.replace(dt=R.stable_dt(s)), st) for s, st in wl.rods]
    steps = 20
    t = time.perf_counter()
    O.rollout_many_threads(rods, steps, n_threads=nt)
    dt = time.perf_counter() - t
    out["batch"] = {"element_steps_per_s": wl.n_elements * steps / dt, "seconds": dt,
                    "sample": "all 4096 rods, %d of the %d steps" % (steps, wl.n_steps)}
    wl = W.config4()
    rods = [(s.replace(dt=R.stable_dt(s)), st) for s, st in wl.rods][:64]
    t = time.perf_counter()
    O.rollout_many_threads(rods, wl.n_steps, n_threads=nt)
    f_s = time.perf_counter() - t
    import numpy as np
    ct = [np.ones((wl.n_steps, 3)) for _ in rods]
    t = time.perf_counter()
    O.vjp_many(rods, wl.n_steps, ct, n_threads=nt)
    g_s = time.perf_counter() - t
    out["adjoint"] = {"forward_s": f_s, "vjp_s": g_s, "vjp_over_forward": g_s / f_s,
                      "sample": "64 of the 256 rods, all %d steps (forward rollout; reverse-mode "
                                "gradient with its own forward pass)" % wl.n_steps}
    return out


def batch_extras(R, W):
    """c3: 4096 uneven rods, per-rod dt, 1000 steps in one launch per kernel-shape bucket,
    against one launch per rod (same kernel) on every 32nd rod, extrapolated by rod count.
    The 1000-step rollout runs three times from the same initial state; the median counts."""
    import numpy as np
    wl = W.config3()
    rods = [(s.replace(dt=R.stable_dt(s)), st) for s, st in wl.rods]
    b = R.RodBatch([s for s, _ in rods])
    b.set_state_rods([st for _, st in rods])
    tune = b.autotune(probe_steps=50, steps_per_launch=1000)
    runs_ms = []
    for _ in range(3):
        b.set_state_rods([st for _, st in rods])
        b.step(wl.n_steps, wl.n_steps)
        b.sync()
        ms, launches = b.last_step_time()
        runs_ms.append(ms)
    ms = float(np.median(runs_ms))
    buckets = b.buckets()
    b.close()
    elements = wl.n_elements
    value = elements * wl.n_steps / (ms / 1e3)
    sample = rods[::32]
    per_rod_ms = []
    for spec, st in sample:
        h = R.RodBatch([spec])
        h.set_state_rods([st])
        h.step(wl.n_steps, wl.n_steps)
        h.sync()
        per_rod_ms.append(h.last_step_time()[0])
        h.close()
    single_ms = float(np.mean(per_rod_ms)) * len(rods)
    # the same launches spread over 8 streams (default priority), all in flight together
    import torch
    streams = [torch.cuda.Stream() for _ in range(8)]
    handles = []
    for i, (spec, st) in enumerate(sample):
        h = R.RodBatch([spec], stream=streams[i % 8].cuda_stream)
        h.set_state_rods([st])
        handles.append(h)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for h in handles:
        h.step(wl.n_steps, wl.n_steps)
    torch.cuda.synchronize()
    streams8_ms = 1e3 * (time.perf_counter() - t) * len(rods) / len(sample)
    for h in handles:
        h.close()
    achieved = BYTES_PER_ELEMENT_STEP * elements * wl.n_steps / (ms / 1e3) / 1e9
    tflops = (sum(s.n * flops_per_element_step(s.inextensible, s.n_iter) for s, _ in rods)
              * wl.n_steps / (ms / 1e3) / 1e12)
    issue = measured_batch_issue(wl, ms, buckets)
    return {
        "workload": "4096 rods, N log-uniform [32, 2048] (sum %d), half inextensible, per-rod dt, "
                    "%d steps" % (elements, wl.n_steps),
        "element_steps_per_s": value, "ms": ms, "runs_ms": runs_ms, "launches": launches,
        "buckets": [{"waves": w, "elems_per_lane": e, "rods": n} for w, e, n, _ in buckets],
        "hbm_roofline_frac": achieved / HBM_PEAK_GBS,
        # many rods per compute unit: the launches are bound by VALU issue, so the method's
        # floating-point rate against the FP32 vector peak (packed, and without packed FP32)
        "alu_roofline": {"bound": "alu", "achieved": tflops, "unit": "TFLOP/s",
                         "peak": FP32_VECTOR_PEAK_TFLOPS, "frac": tflops / FP32_VECTOR_PEAK_TFLOPS,
                         "peak_unpacked": FP32_UNPACKED_PEAK_TFLOPS,
                         "frac_unpacked": tflops / FP32_UNPACKED_PEAK_TFLOPS,
                         "valu_issue_frac": issue and issue["valu_issue_frac"],
                         "executed_fp32_tflops": issue and issue["executed_fp32_tflops"]},
        "one_rod_per_launch": {"element_steps_per_s": elements * wl.n_steps / (single_ms / 1e3),
                               "ms_extrapolated": single_ms, "sampled_rods": len(sample),
                               "hbm_roofline_frac": BYTES_PER_ELEMENT_STEP * elements * wl.n_steps
                               / (single_ms / 1e3) / 1e9 / HBM_PEAK_GBS},
        "one_rod_per_launch_8_streams": {
            "element_steps_per_s": elements * wl.n_steps / (streams8_ms / 1e3),
            "ms_extrapolated": streams8_ms, "sampled_rods": len(sample)},
        "speedup_vs_one_rod_per_launch": single_ms / ms,
        "speedup_vs_one_rod_per_launch_8_streams": streams8_ms / ms,
    }


def adjoint_extras(R, W):
    """c4: 256 rods x 256 elements, 400 steps: plain forward vs checkpointed adjoint."""
    import numpy as np
    import torch
    wl = W.config4()
    rods = [(s.replace(dt=R.stable_dt(s)), st) for s, st in wl.rods]
    n_steps, ckpt = wl.n_steps, 20
    b = R.RodBatch([s for s, _ in rods])

    def timed(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, 1e3 * (time.perf_counter() - t)

    # device-resident tips, loss gradient and outputs (no PCIe in the timed region); one
    # untimed round first (it also allocates the checkpoint buffers), then the median of 3
    dev = torch.device("cuda")
    tips = torch.empty((len(rods), n_steps, 3), dtype=torch.float32, device=dev)
    gen = torch.Generator(device="cpu").manual_seed(4)
    dtips = torch.randn((len(rods), n_steps, 3), generator=gen, dtype=torch.float32).to(dev)
    out = {k: torch.empty(n, dtype=torch.float32, device=dev) for k, n in (
        ("bend", len(rods)), ("twist", len(rods)), ("x", 3 * b.n_points), ("v", 3 * b.n_points),
        ("q", 4 * b.n_frames), ("w", 3 * b.n_frames))}
    fwd, afwd, bwd = [], [], []
    for rep in range(4):
        b.set_state_rods([st for _, st in rods])
        _, t_f = timed(lambda: (b.step(n_steps, ckpt), b.sync()))
        b.set_state_rods([st for _, st in rods])
        _, t_af = timed(lambda: (b.adjoint_forward(n_steps, ckpt, tips=tips), b.sync()))
        _, t_b = timed(lambda: b.adjoint_backward(dtips, out=out))
        if rep:
            fwd.append(t_f)
            afwd.append(t_af)
            bwd.append(t_b)
    # the plain forward at the autotuned kernel shape and steps per launch
    b.set_state_rods([st for _, st in rods])
    tuned = b.autotune(probe_steps=n_steps, steps_per_launch=0)
    tfwd = []
    for rep in range(4):
        b.set_state_rods([st for _, st in rods])
        _, t_f = timed(lambda: (b.step(n_steps), b.sync()))
        if rep:
            tfwd.append(t_f)
    b.close()
    fwd_ms, afwd_ms, bwd_ms, tfwd_ms = (float(np.median(v)) for v in (fwd, afwd, bwd, tfwd))
    return {"workload": "256 rods x 256 elements, inextensible, %d steps, checkpoints every %d"
                        % (n_steps, ckpt),
            "forward_ms": fwd_ms, "adjoint_forward_ms": afwd_ms, "adjoint_backward_ms": bwd_ms,
            "adjoint_over_forward": (afwd_ms + bwd_ms) / fwd_ms,
            "tuned_forward": {"ms": tfwd_ms, "tuning": tuned},
            "adjoint_over_tuned_forward": (afwd_ms + bwd_ms) / tfwd_ms}


def binding_extras(R, W):
    """Catheter / guidewire pair (2 x 512, 384 bound points): us/step unbound (variant 0),
    one-way (1) and two-way (2) bindings, 10 steps per launch."""
    out = {}
    for name, one_way in (("v0", None), ("v1", True), ("v2", False)):
        wl, pairs = W.config5(bool(one_way))
        b = R.RodBatch([s for s, _ in wl.rods])
        if one_way is not None:
            b.set_bindings(pairs, one_way)
        b.set_state_rods([st for _, st in wl.rods])
        b.step(500, 10)
        b.step(5000, 10)
        b.sync()
        ms, launches = b.last_step_time()
        b.close()
        out[name] = {"us_per_step": 1e3 * ms / 5000,
                     "kernel": ("rod_resident_kernel<4,2>, one workgroup per rod" if one_way is None
                                else "rod_group_kernel<4,2>, both rods in one workgroup")}
    for v in ("v1", "v2"):
        out[v]["overhead_vs_v0"] = out[v]["us_per_step"] / out["v0"]["us_per_step"] - 1.0
    out["workload"] = ("catheter/guidewire 2x512 inextensible, guidewire coaxial and bound at 384 "
                       "points, 5000 steps at 10 per launch")
    return out


def contact_extras(R, W):
    """Crossing rods (2 x 128, falling onto each other): us/step without and with sphere
    contact (friction 0.3), 10 steps per launch."""
    wl = W.config6()
    dt = min(R.stable_dt(s) for s, _ in wl.rods)
    rods = [(s.replace(dt=dt), st) for s, st in wl.rods]
    out = {}
    for name, sets in (("no_contact", None), ("contact", [[0, 1]])):
        b = R.RodBatch([s for s, _ in rods])
        if sets is not None:
            b.set_contact(sets, 0.3)
        b.set_state_rods([st for _, st in rods])
        b.step(200, 10)
        b.step(2000, 10)
        b.sync()
        ms, _ = b.last_step_time()
        b.close()
        out[name] = {"us_per_step": 1e3 * ms / 2000}
    out["overhead"] = out["contact"]["us_per_step"] / out["no_contact"]["us_per_step"] - 1.0
    out["workload"] = ("2 x 128-element inextensible rods crossing, one falling onto the other; "
                       "contact: both rods in one workgroup, candidate lists rebuilt when a point "
                       "has moved past their margin")
    return out


def haptic_extras(R, W):
    """Haptic mailbox on the two-instrument workload with static clamps (2 x 512): us/step
    without and with both rods' mailboxes attached (a record every step, or every 20 steps; 10
    steps per launch), and, with a record every step, during one long
    launch, the latency from a pose written by a 1 kHz haptic thread to the first force record
    that names it, plus how often a new force record appears."""
    import threading
    import numpy as np
    wl = W.config1(static_clamp=True)
    specs = [s for s, _ in wl.rods]
    out = {}
    for name, every in (("no_mailbox", 0), ("mailbox", 1), ("mailbox_window_20", 20)):
        b = R.RodBatch(specs)
        if every:
            b.haptic_attach(0, every)
            b.haptic_attach(1, every)
        b.set_state_rods([st for _, st in wl.rods])
        b.step(500, 10)
        b.step(5000, 10)
        b.sync()
        ms, _ = b.last_step_time()
        b.close()
        out[name] = {"us_per_step": 1e3 * ms / 5000}
    for name in ("mailbox", "mailbox_window_20"):
        out[name]["overhead"] = out[name]["us_per_step"] / out["no_mailbox"]["us_per_step"] - 1.0
    b = R.RodBatch(specs)
    b.haptic_attach(0)
    b.haptic_attach(1)
    b.set_state_rods([st for _, st in wl.rods])
    b.step(10, 10)
    b.sync()
    n_long = int(0.5e6 / max(out["mailbox"]["us_per_step"], 1e-3))   # about half a second
    lat, gaps = [], []
    stop = threading.Event()
    base = np.asarray(specs[0].clamp_x0)

    def haptic():
        k = 0
        last_step, last_t = None, None
        while not stop.is_set():
            k += 1
            t0 = time.perf_counter()
            b.haptic_set_pose(0, base + np.array([0.0, 1e-7 * k, 0.0]), specs[0].clamp_q0)
            seen = False
            while time.perf_counter() - t0 < 1e-3:
                _, s, p = b.haptic_get_force(0)
                now = time.perf_counter()
                if last_step is not None and s != last_step:
                    gaps.append((now - last_t) / max(s - last_step, 1))
                if s != last_step:
                    last_step, last_t = s, now
                if not seen and p >= k:
                    lat.append(now - t0)
                    seen = True
            if stop.is_set():
                break

    th = threading.Thread(target=haptic)
    th.start()
    b.step(n_long, n_long)
    b.sync()
    stop.set()
    th.join()
    b.close()
    lat_us = 1e6 * np.asarray(lat[1:-1]) if len(lat) > 2 else np.zeros(1)
    out["pose_to_force_latency_us"] = {"median": float(np.median(lat_us)),
                                       "p99": float(np.percentile(lat_us, 99)),
                                       "poses": int(len(lat_us))}
    out["host_seen_us_per_step"] = float(1e6 * np.median(gaps)) if gaps else None
    out["workload"] = ("two-instrument 2 x 512 inextensible rods, static clamps, mailboxes on both; "
                       "latency: one launch of %d steps, pose of rod 0 written at 1 kHz from a "
                       "host thread, polled until a force record names it" % n_long)
    return out


def environment_extras(R, W):
    """Environment collision on the bent-tube workload with 512 elements (a guidewire in a
    vessel): us/step without the mesh, with the mesh (3072 triangles) and with a mesh four times
    finer around; collision detection runs for every point every step, 10 steps per launch."""
    out = {}
    for name, n_around in (("plain", 0), ("tube_3072", 12), ("tube_12288", 48)):
        wl, tris = W.config7(n=512, n_around=max(n_around, 12))
        spec, st = wl.rods[0]
        spec = spec.replace(dt=R.stable_dt(spec))
        b = R.RodBatch([spec])
        if n_around:
            b.set_environment(tris, 0.3)
        b.set_state_rods([st])
        b.step(500, 10)
        b.step(5000, 10)
        b.sync()
        ms, _ = b.last_step_time()
        nodes, nt = b.environment_info()
        b.close()
        out[name] = {"us_per_step": 1e3 * ms / 5000, "triangles": nt, "tree_nodes": nodes}
    for name in ("tube_3072", "tube_12288"):
        out[name]["overhead"] = out[name]["us_per_step"] / out["plain"]["us_per_step"] - 1.0
    out["workload"] = ("512-element inextensible rod (1 m, r = 2 mm) laid along a bent tube of radius "
                       "1 cm, clamped at its entrance, 5000 steps after 500 of settling")
    return out


def long_rod_extras(R, W, sizes=(1024, 2048, 4096, 16384, 65536), variants=(False, True),
                    ks=(1, 10, 100)):
    """c2: us/step vs rod length and steps per launch over the workload's 5000 steps.  Rods up
    to 2048 elements run in one workgroup ("single") and, for comparison, split over several
    ("chunked"); longer rods are always chunked (one workgroup per ~500 elements, halo exchange
    through global memory every few steps)."""
    out = []
    for n in sizes:
        for inext in variants:
            wl = W.config2(n, inext)
            spec, st = wl.rods[0]
            for mode in (("single", "chunked") if n <= 2048 else ("chunked",)):
                for spl in ks:
                    b = R.RodBatch([spec])
                    if mode == "chunked" and n <= 2048:
                        b.set_chunking(n - 1)
                    b.set_state_rods([st])
                    b.step(200, spl)
                    b.set_state_rods([st])
                    b.step(wl.n_steps, spl)
                    b.sync()
                    ms, launches = b.last_step_time()
                    b.close()
                    us = 1e3 * ms / wl.n_steps
                    out.append({"n": n, "inextensible": inext, "mode": mode,
                                "steps_per_launch": spl, "steps": wl.n_steps, "us_per_step": us,
                                "element_steps_per_s": n / (us / 1e6)})
                    print("[bench] long rod n=%d %s %s k=%d: %.2f us/step" % (
                        n, "inext" if inext else "ext", mode, spl, us), file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--steps-per-launch", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=60000)
    ap.add_argument("--shape", default="", help="W,E kernel shape (default: autotune)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched (4096 rods), long-rod and adjoint measurements")
    ap.add_argument("--extras", default="batch,long_rod,adjoint,binding,contact,haptic,environment",
                    help="comma-separated subset of batch,long_rod,adjoint,binding,contact,"
                         "haptic,environment")
    ap.add_argument("--long-sizes", default="1024,2048,4096,16384,65536",
                    help="rod lengths of the long-rod sweep")
    ap.add_argument("--long-variants", default="ext,inext", help="ext, inext or both")
    ap.add_argument("--long-k", default="1,10,100", help="steps per launch of the long-rod sweep")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the rods of this workload are independent and a "
              "multi-GPU run would only shard rods across devices; run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2509_04277_amd import rod as R
    from paper_2509_04277_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    copy = copy_bandwidth(torch)
    print("copy: %.0f GB/s" % copy["GB/s"], file=sys.stderr, flush=True)
    spl = args.steps_per_launch
    wl = W.config1()
    specs = [s for s, _ in wl.rods]
    b = R.RodBatch(specs)
    b.set_state_rods([st for _, st in wl.rods])
    if args.shape:
        w, e = (int(v) for v in args.shape.split(","))
        b.set_tuning(w, e, spl)
        tune = b.tuning
    else:
        tune = b.autotune(probe_steps=1000, steps_per_launch=spl)
    print("kernel shape: %s" % tune, file=sys.stderr, flush=True)
    b.set_state_rods([st for _, st in wl.rods])
    if args.warmup:
        b.step(args.warmup, spl)
    b.sync()
    torch.cuda.synchronize()
    t = time.perf_counter()
    b.step(args.steps, spl)
    b.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    ms_dev, launches = b.last_step_time()
    elements = wl.n_elements
    value = elements * args.steps / wall
    # host-visible latency of one 10-step update including the position read-back (Sec. 3.1)
    pos = torch.empty(3 * b.n_points, dtype=torch.float32).pin_memory()
    lat = []
    for _ in range(200):
        t1 = time.perf_counter()
        b.step(spl, spl)
        b.get_positions(pos.numpy())
        lat.append(time.perf_counter() - t1)
    b.sync()
    b.close()
    kernel = "rod_resident_kernel<%d,%d>" % (tune["waves"], tune["elems_per_lane"])
    launch_s = ms_dev / 1e3 / launches
    bytes_per_launch = BYTES_PER_ELEMENT_STEP * elements * spl
    achieved = bytes_per_launch / launch_s / 1e9
    traffic = measured_traffic(kernel, elements, spl)
    shares = measured_wave_shares(kernel, elements, spl)
    flops = sum(s.n * flops_per_element_step(s.inextensible, s.n_iter) for s, _ in wl.rods)
    tflops = flops * spl / launch_s / 1e12
    out = {
        "metric": "element-steps/s",
        "value": value,
        "unit": "element-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "2x512-element inextensible rods (catheter/guidewire pair, "
                               "no contact), driven clamps, 10 constraint iterations, "
                               "%d steps per launch" % spl,
                   "rods": 2, "elements": elements, "steps_per_launch": spl,
                   "kernel": kernel},
        "us_per_step": 1e6 * wall / args.steps,
        "us_per_step_device": 1e3 * ms_dev / args.steps,
        "host_visible_ms_per_update": {"steps": spl, "median": 1e3 * float(np.median(lat)),
                                       "p99": 1e3 * float(np.percentile(lat, 99))},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "measured_copy_GBs": copy["GB/s"],
                     "frac_of_measured_copy": achieved / copy["GB/s"],
                     # what binds this small workload (two rods, one workgroup each): VALU issue
                     # and waiting (mostly the cross-wavefront exchanges' barriers), as shares
                     # of wavefront time from SQ counters of the same kernel and workload
                     "valu_issue_frac": shares and shares["valu_issue_frac"],
                     "barrier_share": shares and shares["barrier_share"],
                     "valu_insts_per_wave_step": shares and shares["valu_insts_per_wave_step"],
                     # the method's floating-point operations per element-step and the rate
                     # of the same launches against the chip's FP32 vector peak
                     "flops_per_element_step": flops / elements,
                     "executed_fp32_flops_per_element_step":
                         shares and shares["fp32_flops_per_element_step"],
                     "alu": {"achieved": tflops, "peak": FP32_VECTOR_PEAK_TFLOPS,
                             "unit": "TFLOP/s", "frac": tflops / FP32_VECTOR_PEAK_TFLOPS}},
    }
    if not args.no_extras:
        sizes = tuple(int(v) for v in args.long_sizes.split(",") if v)
        variants = tuple(v == "inext" for v in args.long_variants.split(",") if v)
        ks = tuple(int(v) for v in args.long_k.split(",") if v)
        fns = {"batch": batch_extras,
               "long_rod": lambda R_, W_: long_rod_extras(R_, W_, sizes, variants, ks),
               "adjoint": adjoint_extras,
               "binding": binding_extras, "contact": contact_extras, "haptic": haptic_extras,
               "environment": environment_extras}
        out["extras"] = {k: fns[k](R, W) for k in args.extras.split(",") if k}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_steps)
        if not args.no_extras:
            out["cpu_oracle_all_cores"] = cpu_oracle_many(W, R)
    torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
