"""Host-only checks of the C ABI (include/rod.h): the library loads, exports every declared
entry point, validates arguments before touching a device, and its stability rule agrees with
the oracle's.  No kernel is launched here."""
import ctypes as C

import numpy as np
import pytest

from paper_2509_04277_amd import rod as R
from paper_2509_04277_amd import workloads as W


@pytest.fixture(scope="module")
def L():
    import os
    from paper_2509_04277_amd import build
    if not os.path.exists(R.LIB_PATH):
        build.build()
    return R.lib()


def test_exports_every_declared_function(L):
    names = R.header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(R._SIGS), "binding and header disagree"


def test_status_strings(L):
    for s in R.STATUS:
        assert L.rod_status_str(s).decode().startswith(R.STATUS[s])
    assert L.rod_status_str(123) is not None
    assert L.rod_last_error(None) is not None


def _create_status(L, specs):
    arr = (R.rod_params * max(1, len(specs)))()
    keep = []
    for i, s in enumerate(specs):
        p, k = R.make_params(s)
        arr[i] = p
        keep.append(k)
    h = C.c_void_p()
    rc = L.rod_create(arr, len(specs), None, C.byref(h))
    return rc, h


@pytest.mark.parametrize("mut", [
    dict(n=0), dict(dt=0.0), dict(dt=float("nan")), dict(density=-1.0), dict(poisson=0.7),
    dict(damp_lin=-0.1), dict(kp_scale=-1.0), dict(gravity=(0.0, float("inf"), 0.0)),
    dict(clamp_q0=(1.0, 1.0, 0.0, 0.0)),
])
def test_create_rejects_invalid_params(L, mut):
    spec, _ = W.straight_rod(8)
    if "n" in mut:
        spec = spec.replace(n=0, seg_len=np.zeros(0), radius=np.zeros(0), young=np.zeros(0))
    else:
        spec = spec.replace(**mut)
    rc, h = _create_status(L, [spec])
    assert rc == -1 and not h.value
    assert len(L.rod_last_error(None)) > 0


def test_create_rejects_bad_arrays_and_counts(L):
    spec, _ = W.straight_rod(8)
    bad = spec.replace(young=np.array([1e6] * 7 + [-1.0]))
    assert _create_status(L, [bad])[0] == -1
    assert _create_status(L, [])[0] == -1          # n_rods = 0
    h = C.c_void_p()
    assert L.rod_create(None, 1, None, C.byref(h)) == -1
    p, keep = R.make_params(spec)
    assert L.rod_create(C.byref(p), 1, None, None) == -1


def test_rod_too_long_is_unsupported(L):
    for n in (1 << 20, (1 << 17) + 1):   # the longest accepted rod has 2^17 elements
        spec, _ = W.straight_rod(n)
        assert _create_status(L, [spec])[0] == -6


def test_null_handle_calls(L):
    assert L.rod_step(None, 1, 1) == -1
    assert L.rod_sync(None) == -1
    assert L.rod_destroy(None) == -1
    assert L.rod_get_state(None, None, None, None, None, 0) == -1


def test_stable_dt_matches_oracle(L, oracle):
    specs = [W.config0(dt=1e-6).rods[0][0]] + [s for s, _ in W.config1(dt=1e-7).rods]
    specs += [s for s, _ in W.config3(n_rods=40, n_min=8, n_max=64).rods[:40]]
    # with internal friction: weak (elastic limits bind) and strong (dashpot limits bind)
    specs += [s.replace(damp_int=td) for s in specs[:6] for td in (1e-9, 1e-3)]
    for s in specs:
        s = s.replace(dt=1.0)
        a = R.stable_dt(s)
        b = oracle.Rod(s).dt_rule()
        assert abs(a / b - 1) < 1e-12
