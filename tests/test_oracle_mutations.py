"""The oracle's pins catch plausible mistakes: each case below plants one mistake in a scratch
copy of oracle/corde_oracle.c or of its derivative code oracle/corde_oracle_grad.cpp (a flipped
sign, a wrong index, a dropped term, a wrong material constant, a wrong differentiation rule),
builds it as its own library and runs the CPU pin tests against it in a fresh process.  Every
mutant must fail at least one pin; the unchanged copy, built the same way, must pass them all.
Each planted text must occur exactly once in its file, so the cases follow the source as it
changes."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(HERE)
SRC = os.path.join(REPO, "oracle", "corde_oracle.c")
GRAD_SRC = os.path.join(REPO, "oracle", "corde_oracle_grad.cpp")

PINS = ["test_oracle_algebra.py", "test_oracle_mechanics.py", "test_oracle_binding.py",
        "test_oracle_contact.py", "test_oracle_env.py", "test_oracle_damping.py",
        "test_oracle_feedback.py", "test_oracle_grad.py"]

# (name, text in the oracle, planted replacement); GRAD_MUTANTS: the same in the derivative code
MUTANTS = [
    ("gyroscopic sign (Euler's equations)",
     "tq[a] = tau[3 * j + a] - gyro[a];", "tq[a] = tau[3 * j + a] + gyro[a];"),
    ("penalty stiffness from E instead of G (eq. 8)",
     "e->Kp = rod->kp_scale * e->G * e->A;", "e->Kp = rod->kp_scale * e->E * e->A;"),
    ("axial moment of inertia doubled",
     "e->I3 = e->m * e->r * e->r / 2.0;", "e->I3 = e->m * e->r * e->r;"),
    ("penalty force without the projection (I - t t^T)",
     "g[c] += e.Kp * e.l * (r[c] - tr * t[c]) / len;", "g[c] += e.Kp * e.l * r[c] / len;"),
    ("distance impulse weighted by the wrong end",
     "v[3 * (j + 1) + c] -= winv[j + 1] * lambda * nc;",
     "v[3 * (j + 1) + c] -= winv[j] * lambda * nc;"),
    ("intrinsic curvature sign in the bend/twist moment",
     "double mk = jt.K[k] * (u[k] - jt.uhat[k]);", "double mk = jt.K[k] * (u[k] + jt.uhat[k]);"),
    ("twist stiffness taken from the bending stiffness",
     "jt->K[2] = 0.5 * (a.K3 + b.K3);", "jt->K[2] = 0.5 * (a.K1 + b.K1);"),
    ("linear velocity damping dropped",
     "double a = F[3 * i + c] / M - rod->damp_lin * v[3 * i + c];",
     "double a = F[3 * i + c] / M;"),
    ("quaternion rate doubled (eq. of q-dot)",
     "qj[a] += 0.5 * dt * dq[a];", "qj[a] += dt * dq[a];"),
    ("B_1 with its lower block transposed (eq. 6)",
     "{{0, -1, 0, 0}, {1, 0, 0, 0}, {0, 0, 0, 1}, {0, 0, -1, 0}}",
     "{{0, -1, 0, 0}, {1, 0, 0, 0}, {0, 0, 0, -1}, {0, 0, 1, 0}}"),
    ("Darboux vector without the 2 / rest length factor (eq. 5)",
     "u[k] = (2.0 / jt.lbar) * dot4(Bq, q + 4 * (j + 1));",
     "u[k] = (1.0 / jt.lbar) * dot4(Bq, q + 4 * (j + 1));"),
    ("one-way binding moves the master too",
     "const double wsum = one_way ? wa : wa + wb;", "const double wsum = wa + wb;"),
    ("rod-rod friction not bounded by the Coulomb cone",
     "if (lt > contact->mu * lam) lt = contact->mu * lam;", "if (0) lt = contact->mu * lam;"),
    ("environment penetration depth with the wrong sign",
     "const double sep = dt * dot3(v, n) - depth;", "const double sep = dt * dot3(v, n) + depth;"),
    ("internal friction force on one end with the wrong sign",
     "F[3 * (j + 1) + c] -= td * e.Ks * sd * t[c];", "F[3 * (j + 1) + c] += td * e.Ks * sd * t[c];"),
]

GRAD_MUTANTS = [
    ("forward mode: product rule without the second term",
     "return Dual(a.v * b.v, a.d * b.v + a.v * b.d);", "return Dual(a.v * b.v, a.d * b.v);"),
    ("forward mode: derivative of the square root without its 1/2",
     "return Dual(s, a.d / (2.0 * s));", "return Dual(s, a.d / s);"),
    ("reverse mode: quotient rule with the wrong sign on the divisor",
     "return make(r, a.i, 1.0 / b.v, b.i, -r / b.v);", "return make(r, a.i, 1.0 / b.v, b.i, r / b.v);"),
    ("reverse mode: square-root partial doubled",
     "return make(s, a.i, 0.5 / s, -1, 0.0);", "return make(s, a.i, 1.0 / s, -1, 0.0);"),
    ("templated step: gyroscopic sign flipped",
     "tq[a] = tau[3 * j + a] - gyro[a];", "tq[a] = tau[3 * j + a] + gyro[a];"),
]


def _run_pins(lib, log):
    env = dict(os.environ, CORDE_ORACLE_LIB=lib)
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
           "--timeout", "120"] + [os.path.join(HERE, f) for f in PINS]
    r = subprocess.run(cmd, cwd=REPO, env=env, capture_output=True, text=True, timeout=900)
    with open(log, "w") as f:
        f.write(r.stdout + r.stderr)
    return r.returncode, r.stdout


@pytest.mark.slow
def test_every_planted_mistake_fails_a_pin(tmp_path):
    from oracle import oracle as O
    src = {SRC: open(SRC).read(), GRAD_SRC: open(GRAD_SRC).read()}
    jobs = ([("unchanged", SRC, None, None)] + [(n, SRC, o, w) for n, o, w in MUTANTS] +
            [(n, GRAD_SRC, o, w) for n, o, w in GRAD_MUTANTS])
    libs = []
    for k, (name, target, old, new) in enumerate(jobs):
        paths = {}
        for f, text in src.items():
            if f == target and old is not None:
                assert text.count(old) == 1, "planted text for %r not found once" % name
                text = text.replace(old, new)
            paths[f] = tmp_path / ("m%02d_%s" % (k, os.path.basename(f)))
            paths[f].write_text(text)
        libs.append(O.build(force=True, src=str(paths[SRC]), grad_src=str(paths[GRAD_SRC]),
                            lib=str(tmp_path / ("m%02d.so" % k))))
    with ThreadPoolExecutor(max_workers=max(1, min(8, os.cpu_count() or 1))) as ex:
        results = list(ex.map(lambda a: _run_pins(*a),
                              [(lib, str(tmp_path / ("m%02d.log" % k))) for k, lib in enumerate(libs)]))
    rc0, out0 = results[0]
    assert rc0 == 0, "the unchanged oracle fails its pins:\n" + out0[-2000:]
    survivors = [jobs[k][0] for k, (rc, _) in enumerate(results) if k and rc != 1]
    assert not survivors, "mistakes no pin catches (or pytest errors): %s" % survivors
