/* Drives every entry point of the FP64 oracle on small rods so that a build with address and
 * undefined-behaviour sanitizers can check the oracle's own memory accesses and arithmetic
 * (built and run by tests/test_oracle_sanitizers.py, on the host only).  Prints "ok" and exits
 * 0 when every result is finite; a sanitizer finding aborts the program. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/corde_oracle.h"

#define N 16
#define M (N + 1)

static int bad = 0;

static void check_finite(const char* what, const double* a, int n) {
    for (int i = 0; i < n; ++i)
        if (!isfinite(a[i])) {
            printf("non-finite %s[%d]\n", what, i);
            bad = 1;
            return;
        }
}

/* a straight rod of N elements along +x from base, frames aligned (third axis along +x) */
static void straight(oracle_rod* r, double* lens, double* rad, double* young, const double* base,
                     double* x, double* v, double* q, double* w, int inext) {
    memset(r, 0, sizeof(*r));
    const double l = 1.0 / N;
    for (int j = 0; j < N; ++j) {
        lens[j] = l;
        rad[j] = 0.01;
        young[j] = 1e6;
    }
    r->n = N;
    r->inextensible = inext;
    r->n_iter = inext ? 10 : 0;
    r->clamp = 1;
    r->gravity[2] = -9.81;
    r->damp_lin = 0.5;
    r->damp_ang = 0.5;
    r->poisson = 0.5;
    r->density = 1000.0;
    r->kp_scale = 1.0;
    r->bend_scale = 1.0;
    r->twist_scale = 1.0;
    r->seg_len = lens;
    r->radius = rad;
    r->young = young;
    const double qa[4] = {cos(M_PI / 4), 0.0, sin(M_PI / 4), 0.0};   /* e3 -> +x */
    for (int i = 0; i < M; ++i) {
        x[3 * i] = base[0] + i * l;
        x[3 * i + 1] = base[1];
        x[3 * i + 2] = base[2];
        v[3 * i] = v[3 * i + 1] = v[3 * i + 2] = 0.0;
    }
    for (int j = 0; j < N; ++j) {
        memcpy(q + 4 * j, qa, sizeof(qa));
        w[3 * j] = w[3 * j + 1] = w[3 * j + 2] = 0.0;
    }
    memcpy(r->clamp_x0, base, 3 * sizeof(double));
    memcpy(r->clamp_q0, qa, sizeof(qa));
    r->dt = 0.5 * oracle_dt_rule(r);
}

int main(void) {
    double lens[N], rad[N], young[N], x[3 * M], v[3 * M], q[4 * N], w[3 * N];
    double F[3 * M], tau[3 * N], u[3], xc[3], qc[4], wc[3], tip[3 * 40], fb[3 * 40];
    const double origin[3] = {0.0, 0.0, 0.0};
    oracle_rod rod;

    /* single rods: both variants, a driven clamp, internal friction, energies and forces */
    for (int inext = 0; inext < 2; ++inext) {
        straight(&rod, lens, rad, young, origin, x, v, q, w, inext);
        rod.clamp_amp[1] = 0.01;
        rod.clamp_freq = 2.0;
        rod.clamp_twist_amp = 0.1;
        rod.clamp_twist_axis[0] = 1.0;
        rod.damp_int = 2.0 * rod.dt;
        if (oracle_check(&rod) != 0) {
            printf("oracle_check refused the rod\n");
            return 1;
        }
        rod.dt = 0.5 * oracle_dt_rule(&rod);
        oracle_rollout(&rod, 0.0, 40, x, v, q, w, tip);
        check_finite("x", x, 3 * M);
        check_finite("tip", tip, 3 * 40);
        double e = oracle_energy(&rod, x, q) + oracle_kinetic(&rod, v, w) +
                   oracle_dissipation(&rod, x, q, v, w) + oracle_max_strain(&rod, x);
        check_finite("energy", &e, 1);
        oracle_forces(&rod, x, q, F, tau);
        oracle_damping_forces(&rod, x, q, v, w, F, tau);
        check_finite("F", F, 3 * M);
        check_finite("tau", tau, 3 * N);
        for (int j = 0; j + 1 < N; ++j) oracle_darboux(&rod, q, j, u);
        check_finite("u", u, 3);
        oracle_clamp_pose(&rod, 0.37, xc, qc, wc);
        check_finite("qc", qc, 4);
        oracle_rollout_fb(&rod, 40 * rod.dt, 40, x, v, q, w, fb);
        check_finite("fb", fb, 3 * 40);
        (void)oracle_stable(&rod, 0.0, 20, x, v, q, w, 1.5);   /* (the driven clamp adds energy) */
    }
    double B[16], R[9], r4[4];
    for (int k = 0; k < 3; ++k) oracle_bmat(k, B);
    oracle_rotmat(q, R);
    oracle_qmul(q, q + 4, r4);
    check_finite("R", R, 9);

    /* two rods: a one-way and a two-way binding, then contact between and within them */
    double lens2[N], rad2[N], young2[N], x2[3 * M], v2[3 * M], q2[4 * N], w2[3 * N];
    const double off[3] = {0.0, 0.015, 0.0};
    oracle_rod a, b;
    straight(&a, lens, rad, young, origin, x, v, q, w, 1);
    straight(&b, lens2, rad2, young2, off, x2, v2, q2, w2, 1);
    b.dt = a.dt;
    int32_t pa[8], pb[8];
    for (int k = 0; k < 8; ++k) {
        pa[k] = 8 + k;
        pb[k] = 8 + k;
    }
    for (int one_way = 0; one_way < 2; ++one_way) {
        oracle_binding bind = {8, pa, pb, one_way};
        oracle_rollout_pair(&a, &b, &bind, 0.0, 20, x, v, q, w, x2, v2, q2, w2);
    }
    check_finite("xa", x, 3 * M);
    check_finite("xb", x2, 3 * M);
    const oracle_rod* rods[2] = {&a, &b};
    double* xs[2] = {x, x2};
    double* vs[2] = {v, v2};
    double* qs[2] = {q, q2};
    double* ws[2] = {w, w2};
    oracle_contact ct = {0.3};
    int32_t most = 0;
    oracle_rollout_group(rods, 2, NULL, &ct, 0.0, 20, xs, vs, qs, ws, &most);
    oracle_rollout_group(rods, 1, NULL, &ct, 0.0, 20, xs, vs, qs, ws, &most);
    (void)oracle_self_skip(&a);
    check_finite("xa", x, 3 * M);
    check_finite("xb", x2, 3 * M);

    /* one rod against a floor of two triangles just below it */
    const double tris[18] = {-2, -2, -0.005, 2, -2, -0.005, 2, 2, -0.005,
                             -2, -2, -0.005, 2, 2, -0.005, -2, 2, -0.005};
    oracle_env env = {2, tris, 0.4};
    straight(&a, lens, rad, young, origin, x, v, q, w, 1);
    double n[3], depth, cp[3];
    int32_t hits;
    oracle_closest_point_triangle(x + 3, tris, cp);
    oracle_env_response(&env, x + 3, 0.01, n, &depth, &hits);
    oracle_env_impulse(n, depth, 1.0, a.dt, 0.4, v + 3);
    oracle_rollout_env(&a, &env, 0.0, 30, x, v, q, w, &most);
    check_finite("x env", x, 3 * M);

    if (bad) return 1;
    printf("ok\n");
    return 0;
}
