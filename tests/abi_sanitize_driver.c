/* Walks the host-side argument checks and refusal paths of the C ABI so that a build of the
 * library with host address and undefined-behaviour sanitizers can check them (built and run
 * by tests/test_abi_sanitizers.py; no GPU needed: every call here is refused before any device
 * work, or, for the one valid rod_create, fails on a machine without a GPU or succeeds and is
 * destroyed).  Exits 0 and prints "ok" when every refusal carries the documented status. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "rod.h"

static int bad = 0;

static void expect(const char* what, int got, int want) {
    if (got != want) {
        printf("%s: status %d, expected %d\n", what, got, want);
        bad = 1;
    }
}

#define N 8

int main(void) {
    double lens[N], rad[N], young[N];
    for (int j = 0; j < N; ++j) {
        lens[j] = 0.125;
        rad[j] = 0.01;
        young[j] = 1e6;
    }
    rod_params p;
    memset(&p, 0, sizeof(p));
    p.n_elements = N;
    p.inextensible = 1;
    p.n_constraint_iters = 10;
    p.clamp_end0 = 1;
    p.dt = 1e-5;
    p.gravity[2] = -9.81;
    p.poisson = 0.5;
    p.density = 1000.0;
    p.kp_scale = 1.0;
    p.bend_scale = 1.0;
    p.twist_scale = 1.0;
    p.seg_len = lens;
    p.radius = rad;
    p.young = young;
    p.clamp_q0[0] = 1.0;

    /* status strings and the handle-less error text */
    for (int s = 0; s >= -8; --s)
        if (!rod_status_str((rod_status)s)) bad = 1;
    if (!rod_last_error(NULL)) bad = 1;

    /* stable dt: host-only arithmetic */
    double dt = 0.0;
    expect("stable_dt", rod_stable_dt(&p, &dt), ROD_OK);
    if (!(dt > 0.0 && isfinite(dt))) bad = 1;
    expect("stable_dt null", rod_stable_dt(NULL, &dt), ROD_E_INVALID);

    /* rod_create refusals */
    rod_ctx* h = NULL;
    expect("create null params", rod_create(NULL, 1, NULL, &h), ROD_E_INVALID);
    expect("create no rods", rod_create(&p, 0, NULL, &h), ROD_E_INVALID);
    expect("create null out", rod_create(&p, 1, NULL, NULL), ROD_E_INVALID);
    rod_params q = p;
    q.n_elements = 0;
    expect("create n = 0", rod_create(&q, 1, NULL, &h), ROD_E_INVALID);
    q = p;
    q.dt = -1.0;
    expect("create dt < 0", rod_create(&q, 1, NULL, &h), ROD_E_INVALID);
    q = p;
    q.seg_len = NULL;
    expect("create no lengths", rod_create(&q, 1, NULL, &h), ROD_E_INVALID);
    double young_bad[N];
    memcpy(young_bad, young, sizeof(young));
    young_bad[N - 1] = -1.0;
    q = p;
    q.young = young_bad;
    expect("create E < 0", rod_create(&q, 1, NULL, &h), ROD_E_INVALID);
    double rad_nan[N];
    memcpy(rad_nan, rad, sizeof(rad));
    rad_nan[2] = NAN;
    q = p;
    q.radius = rad_nan;
    expect("create r = NaN", rod_create(&q, 1, NULL, &h), ROD_E_INVALID);
    q = p;
    q.damping_int = -1.0;
    expect("create tau_d < 0", rod_create(&q, 1, NULL, &h), ROD_E_INVALID);
    if (h) bad = 1;   /* no handle on any refusal */

    /* every entry point refuses a null handle */
    float f[4] = {0};
    double d4[4] = {1, 0, 0, 0};
    int32_t i2[4] = {0, 1, 0, 1};
    int64_t steps = 0;
    int32_t k = 0;
    rod_tuning t;
    rod_haptic_force hf;
    expect("destroy", rod_destroy(NULL), ROD_E_INVALID);
    expect("set_state", rod_set_state(NULL, f, f, f, f, 0, 0.0), ROD_E_INVALID);
    expect("get_state", rod_get_state(NULL, f, f, f, f, 0), ROD_E_INVALID);
    expect("step", rod_step(NULL, 1, 1), ROD_E_INVALID);
    expect("set_clamp", rod_set_clamp(NULL, 0, d4, d4), ROD_E_INVALID);
    expect("sync", rod_sync(NULL), ROD_E_INVALID);
    expect("get_time", rod_get_time(NULL, d4, &steps), ROD_E_INVALID);
    expect("set_tuning", rod_set_tuning(NULL, &t), ROD_E_INVALID);
    expect("get_tuning", rod_get_tuning(NULL, &t), ROD_E_INVALID);
    expect("bucket_info", rod_bucket_info(NULL, 0, &t, &k), ROD_E_INVALID);
    expect("set_chunking", rod_set_chunking(NULL, 100, 0), ROD_E_INVALID);
    expect("set_bindings", rod_set_bindings(NULL, 1, i2, 1), ROD_E_INVALID);
    expect("set_contact", rod_set_contact(NULL, 1, i2, 0.1), ROD_E_INVALID);
    expect("set_environment", rod_set_environment(NULL, 0, d4, 0.1), ROD_E_INVALID);
    expect("environment_info", rod_environment_info(NULL, &k, &k), ROD_E_INVALID);
    expect("haptic_attach", rod_haptic_attach(NULL, 0, 1), ROD_E_INVALID);
    expect("haptic_detach", rod_haptic_detach(NULL, 0), ROD_E_INVALID);
    expect("haptic_set_pose", rod_haptic_set_pose(NULL, 0, d4, d4), ROD_E_INVALID);
    expect("haptic_get_force", rod_haptic_get_force(NULL, 0, &hf), ROD_E_INVALID);
    expect("autotune", rod_autotune(NULL, 10, 10, &t), ROD_E_INVALID);
    expect("last_step_time", rod_last_step_time(NULL, f, &k), ROD_E_INVALID);
    expect("stiffness_mult", rod_set_stiffness_mult(NULL, f, f), ROD_E_INVALID);
    expect("adjoint_forward", rod_adjoint_forward(NULL, 10, 5, f, 0, NULL), ROD_E_INVALID);
    expect("adjoint_backward", rod_adjoint_backward(NULL, 0, f, f, f, f, f, f, f, 0), ROD_E_INVALID);

    /* one valid handle: without a GPU rod_create fails cleanly (and frees what it made) */
    int rc = rod_create(&p, 1, NULL, &h);
    if (rc == ROD_OK) {
        expect("step before state", rod_step(h, 1, 1), ROD_E_ORDER);
        expect("destroy", rod_destroy(h), ROD_OK);
    } else if (h) {
        bad = 1;
    }

    if (bad) return 1;
    printf("ok\n");
    return 0;
}
