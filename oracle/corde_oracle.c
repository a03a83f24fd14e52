/*
 * corde_oracle.c -- FP64 CPU oracle of the discrete CoRdE Cosserat rod stepper.
 *
 * TEST INFRASTRUCTURE ONLY (see corde_oracle.h).  Written for clarity, not speed: every
 * quantity is recomputed from the material description where it is used, every gradient
 * is the chain rule of the energy written out, and torques come from quaternion gradients
 * through the B_k matrices exactly as eq. (6) defines the strain.
 *
 * Readings taken where the paper is silent or garbled (each is also listed in the design
 * notes of the repository):
 *   - bending/twist stiffness use the second moment of area: K_1 = K_2 = E pi r^4 / 4,
 *     K_3 = G pi r^4 / 2 (eq. (3) prints r^2, which has the wrong dimension);
 *   - K_p = G pi r^2 (eq. (8) only says it depends on the material);
 *   - G = E / (2 (1 + nu)); point masses lump half of each adjacent element;
 *   - frames are integrated as rigid cylinders, I = diag(m(3r^2+l^2)/12 twice, m r^2/2),
 *     gyroscopic term included;
 *   - joint j couples frames j and j+1 over lbar_j = (l_j + l_{j+1}) / 2 with the mean of
 *     the two elements' stiffnesses;
 *   - B_k are derived from (0, u) = 2 conj(q) (x) q' for scalar-first Hamilton quaternions
 *     (the paper defers them to the appendix of its reference [17]);
 *   - distance constraints: red-black Gauss-Seidel over segments (even, then odd), each
 *     impulse linearised at the predicted positions p = x + dt v;
 *   - semi-implicit Euler: v (and omega) first, then x (and q) with the new velocities,
 *     followed by quaternion renormalisation;
 *   - damping is plain velocity damping (a -= gamma v, alpha -= gamma omega), plus, when a rod
 *     sets a retardation time, Kelvin-Voigt internal friction on the stretch and bend/twist
 *     strain rates (the paper names the dissipation terms but gives no formula).
 */
#include "corde_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ---------------------------------------------------------------- quaternion algebra -- */

/* B_k, eq. (6): B_k q = q (x) (0, e_k); skew-symmetric. */
static const double BMAT[3][4][4] = {
    {{0, -1, 0, 0}, {1, 0, 0, 0}, {0, 0, 0, 1}, {0, 0, -1, 0}},
    {{0, 0, -1, 0}, {0, 0, 0, -1}, {1, 0, 0, 0}, {0, 1, 0, 0}},
    {{0, 0, 0, -1}, {0, 0, 1, 0}, {0, -1, 0, 0}, {1, 0, 0, 0}},
};

void oracle_bmat(int32_t k, double* out16) {
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) out16[4 * r + c] = BMAT[k][r][c];
}

static void bmul(int k, const double* q, double* out) {
    for (int r = 0; r < 4; ++r) {
        out[r] = 0.0;
        for (int c = 0; c < 4; ++c) out[r] += BMAT[k][r][c] * q[c];
    }
}

static double dot4(const double* a, const double* b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3];
}

static double dot3(const double* a, const double* b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static double norm3(const double* a) { return sqrt(dot3(a, a)); }

static void cross3(const double* a, const double* b, double* r) {
    double t0 = a[1] * b[2] - a[2] * b[1];
    double t1 = a[2] * b[0] - a[0] * b[2];
    double t2 = a[0] * b[1] - a[1] * b[0];
    r[0] = t0;
    r[1] = t1;
    r[2] = t2;
}

void oracle_qmul(const double* a, const double* b, double* r) {
    double w = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    double x = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    double y = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    double z = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
    r[0] = w;
    r[1] = x;
    r[2] = y;
    r[3] = z;
}

/* Rotation matrix R(q) (body -> world), written for unit q; column k is director d_{k+1}. */
static void rotmat(const double* q, double R[3][3]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0][0] = w * w + x * x - y * y - z * z;
    R[0][1] = 2 * (x * y - w * z);
    R[0][2] = 2 * (x * z + w * y);
    R[1][0] = 2 * (x * y + w * z);
    R[1][1] = w * w - x * x + y * y - z * z;
    R[1][2] = 2 * (y * z - w * x);
    R[2][0] = 2 * (x * z - w * y);
    R[2][1] = 2 * (y * z + w * x);
    R[2][2] = w * w - x * x - y * y + z * z;
}

void oracle_rotmat(const double* q, double* out9) {
    double R[3][3];
    rotmat(q, R);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) out9[3 * r + c] = R[r][c];
}

/* Third director d_3(q) and its Jacobian with respect to (w, x, y, z). */
static void director3(const double* q, double* d3, double J[3][4]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    d3[0] = 2 * (x * z + w * y);
    d3[1] = 2 * (y * z - w * x);
    d3[2] = w * w - x * x - y * y + z * z;
    if (J) {
        J[0][0] = 2 * y;  J[0][1] = 2 * z;  J[0][2] = 2 * w;  J[0][3] = 2 * x;
        J[1][0] = -2 * x; J[1][1] = -2 * w; J[1][2] = 2 * z;  J[1][3] = 2 * y;
        J[2][0] = 2 * w;  J[2][1] = -2 * x; J[2][2] = -2 * y; J[2][3] = 2 * z;
    }
}

/* ------------------------------------------------------------------ material model -- */

typedef struct {
    double l, r, E, G, A, m, Ks, Kp, K1, K3, I1, I3;
} elem_t;

static void element(const oracle_rod* rod, int j, elem_t* e) {
    e->l = rod->seg_len[j];
    e->r = rod->radius[j];
    e->E = rod->young[j];
    e->G = e->E / (2.0 * (1.0 + rod->poisson));
    e->A = M_PI * e->r * e->r;
    e->m = rod->density * e->A * e->l;
    e->Ks = e->E * e->A;                                      /* eq. (2) */
    e->Kp = rod->kp_scale * e->G * e->A;                      /* eq. (8) */
    double r4 = e->r * e->r * e->r * e->r;
    e->K1 = rod->bend_scale * e->E * M_PI * r4 / 4.0;          /* eq. (3), second moment */
    e->K3 = rod->twist_scale * e->G * M_PI * r4 / 2.0;
    e->I1 = e->m * (3.0 * e->r * e->r + e->l * e->l) / 12.0;  /* rigid cylinder */
    e->I3 = e->m * e->r * e->r / 2.0;
}

static double point_mass(const oracle_rod* rod, int i) {
    double M = 0.0;
    elem_t e;
    if (i > 0) {
        element(rod, i - 1, &e);
        M += 0.5 * e.m;
    }
    if (i < rod->n) {
        element(rod, i, &e);
        M += 0.5 * e.m;
    }
    return M;
}

typedef struct {
    double lbar, K[3];
    double uhat[3];
} joint_t;

static void joint(const oracle_rod* rod, int j, joint_t* jt) {
    elem_t a, b;
    element(rod, j, &a);
    element(rod, j + 1, &b);
    jt->lbar = 0.5 * (a.l + b.l);
    jt->K[0] = 0.5 * (a.K1 + b.K1);
    jt->K[1] = jt->K[0];
    jt->K[2] = 0.5 * (a.K3 + b.K3);
    for (int k = 0; k < 3; ++k) jt->uhat[k] = rod->u_hat ? rod->u_hat[3 * j + k] : 0.0;
}

int32_t oracle_check(const oracle_rod* rod) {
    if (!rod || rod->n < 1) return -1;
    if (!rod->seg_len || !rod->radius || !rod->young) return -2;
    if (!(rod->dt > 0.0)) return -3;
    if (rod->inextensible && rod->n_iter < 0) return -4;
    for (int j = 0; j < rod->n; ++j)
        if (!(rod->seg_len[j] > 0 && rod->radius[j] > 0 && rod->young[j] > 0)) return -5;
    if (!(rod->density > 0)) return -6;
    return 0;
}

/* ----------------------------------------------------------------- energy and forces -- */

void oracle_darboux(const oracle_rod* rod, const double* q, int32_t j, double* u) {
    joint_t jt;
    joint(rod, j, &jt);
    double Bq[4];
    for (int k = 0; k < 3; ++k) {
        bmul(k, q + 4 * j, Bq);
        u[k] = (2.0 / jt.lbar) * dot4(Bq, q + 4 * (j + 1));  /* eq. (6) with eq. (5) */
    }
}

double oracle_energy(const oracle_rod* rod, const double* x, const double* q) {
    const int n = rod->n;
    double V = 0.0;
    for (int j = 0; j < n; ++j) {
        elem_t e;
        element(rod, j, &e);
        double d[3], t[3], d3[3];
        for (int c = 0; c < 3; ++c) d[c] = x[3 * (j + 1) + c] - x[3 * j + c];
        double len = norm3(d);
        for (int c = 0; c < 3; ++c) t[c] = d[c] / len;
        if (!rod->inextensible) {
            double s = len / e.l - 1.0;                        /* v_3 - 1, eq. (2) */
            V += 0.5 * e.Ks * s * s * e.l;
        }
        director3(q + 4 * j, d3, NULL);
        double diff[3] = {t[0] - d3[0], t[1] - d3[1], t[2] - d3[2]};
        V += 0.5 * e.Kp * dot3(diff, diff) * e.l;              /* eq. (8) */
    }
    for (int j = 0; j + 1 < n; ++j) {
        joint_t jt;
        joint(rod, j, &jt);
        double u[3];
        oracle_darboux(rod, q, j, u);
        for (int k = 0; k < 3; ++k) {
            double du = u[k] - jt.uhat[k];
            V += 0.5 * jt.K[k] * du * du * jt.lbar;            /* eq. (3) */
        }
    }
    for (int i = 0; i <= n; ++i) {
        double M = point_mass(rod, i);
        V -= M * dot3(rod->gravity, x + 3 * i);
        if (rod->f_ext) V -= dot3(rod->f_ext + 3 * i, x + 3 * i);
    }
    return V;
}

double oracle_kinetic(const oracle_rod* rod, const double* v, const double* w) {
    double T = 0.0;
    for (int i = 0; i <= rod->n; ++i) T += 0.5 * point_mass(rod, i) * dot3(v + 3 * i, v + 3 * i);
    for (int j = 0; j < rod->n; ++j) {
        elem_t e;
        element(rod, j, &e);
        const double* wj = w + 3 * j;
        T += 0.5 * (e.I1 * wj[0] * wj[0] + e.I1 * wj[1] * wj[1] + e.I3 * wj[2] * wj[2]);
    }
    return T;
}

void oracle_forces(const oracle_rod* rod, const double* x, const double* q, double* F,
                   double* tau) {
    const int n = rod->n;
    double* gq = (double*)calloc((size_t)4 * n, sizeof(double)); /* dV/dq */
    memset(F, 0, sizeof(double) * 3 * (n + 1));

    for (int j = 0; j < n; ++j) {
        elem_t e;
        element(rod, j, &e);
        double d[3], t[3], d3[3], J[3][4];
        for (int c = 0; c < 3; ++c) d[c] = x[3 * (j + 1) + c] - x[3 * j + c];
        double len = norm3(d);
        for (int c = 0; c < 3; ++c) t[c] = d[c] / len;
        /* dV/dd for this segment */
        double g[3] = {0, 0, 0};
        if (!rod->inextensible) {
            double s = len / e.l - 1.0;
            for (int c = 0; c < 3; ++c) g[c] += e.Ks * s * t[c];  /* d/dd of 1/2 Ks l s^2 */
        }
        director3(q + 4 * j, d3, J);
        double r[3] = {t[0] - d3[0], t[1] - d3[1], t[2] - d3[2]};
        /* d/dd of 1/2 Kp l |t - d3|^2 = Kp l (I - t t^T) r / |d| */
        double tr = dot3(t, r);
        for (int c = 0; c < 3; ++c) g[c] += e.Kp * e.l * (r[c] - tr * t[c]) / len;
        for (int c = 0; c < 3; ++c) {
            F[3 * (j + 1) + c] -= g[c];
            F[3 * j + c] += g[c];
        }
        /* d/dq of 1/2 Kp l |t - d3(q)|^2 = -Kp l J^T r */
        for (int a = 0; a < 4; ++a) {
            double s = 0.0;
            for (int c = 0; c < 3; ++c) s += J[c][a] * r[c];
            gq[4 * j + a] -= e.Kp * e.l * s;
        }
    }
    for (int j = 0; j + 1 < n; ++j) {
        joint_t jt;
        joint(rod, j, &jt);
        double u[3];
        oracle_darboux(rod, q, j, u);
        for (int k = 0; k < 3; ++k) {
            /* V_k = 1/2 K lbar (u_k - uhat)^2 with u_k = (2/lbar) q_j^T B_k^T q_{j+1} */
            double mk = jt.K[k] * (u[k] - jt.uhat[k]);
            double Bqj[4], Bqn[4];
            bmul(k, q + 4 * j, Bqj);
            bmul(k, q + 4 * (j + 1), Bqn);
            for (int a = 0; a < 4; ++a) {
                gq[4 * (j + 1) + a] += 2.0 * mk * Bqj[a];   /* B_k q_j */
                gq[4 * j + a] -= 2.0 * mk * Bqn[a];         /* B_k^T q_{j+1} = -B_k q_{j+1} */
            }
        }
    }
    for (int i = 0; i <= n; ++i) {
        double M = point_mass(rod, i);
        for (int c = 0; c < 3; ++c) {
            F[3 * i + c] += M * rod->gravity[c];
            if (rod->f_ext) F[3 * i + c] += rod->f_ext[3 * i + c];
        }
    }
    /* body torque about body axis a: virtual rotation q -> q (x) (1, eps e_a / 2) moves q by
     * eps/2 B_a q, so tau_a = -1/2 (dV/dq) . (B_a q) */
    for (int j = 0; j < n; ++j) {
        for (int a = 0; a < 3; ++a) {
            double Bq[4];
            bmul(a, q + 4 * j, Bq);
            tau[3 * j + a] = -0.5 * dot4(gq + 4 * j, Bq);
        }
    }
    free(gq);
}

/* ---------------------------------------------------------------- internal friction -- */

/* time derivative of the stretch s_j = |x_{j+1} - x_j| / l_j - 1 of element j */
static double stretch_rate(const oracle_rod* rod, int j, const double* x, const double* v,
                           double* t) {
    double d[3], dv[3];
    for (int c = 0; c < 3; ++c) {
        d[c] = x[3 * (j + 1) + c] - x[3 * j + c];
        dv[c] = v[3 * (j + 1) + c] - v[3 * j + c];
    }
    const double len = norm3(d);
    for (int c = 0; c < 3; ++c) t[c] = d[c] / len;
    return dot3(t, dv) / rod->seg_len[j];
}

/* d/dt of the Darboux vector of joint j, eq. (6): u_k = (2/lbar) (B_k q_j) . q_{j+1} with
 * dq/dt = 1/2 q (x) (0, omega); also its coefficients a[k][b] = d udot_k / d omega_j,b and
 * bb[k][b] = d udot_k / d omega_{j+1},b */
static void darboux_rate(const oracle_rod* rod, const double* q, const double* w, int j,
                         double* ud, double a[3][3], double bb[3][3]) {
    joint_t jt;
    joint(rod, j, &jt);
    const double* qj = q + 4 * j;
    const double* qn = q + 4 * (j + 1);
    for (int k = 0; k < 3; ++k) {
        double Bqj[4];
        bmul(k, qj, Bqj);
        ud[k] = 0.0;
        for (int b = 0; b < 3; ++b) {
            const double eb[4] = {0.0, b == 0, b == 1, b == 2};
            double qe[4], Bqe[4], ne[4];
            oracle_qmul(qj, eb, qe);          /* q_j (x) e_b */
            bmul(k, qe, Bqe);
            oracle_qmul(qn, eb, ne);          /* q_{j+1} (x) e_b */
            a[k][b] = dot4(Bqe, qn) / jt.lbar;   /* (2/lbar) (B_k (1/2 q_j (x) e_b)) . q_{j+1} */
            bb[k][b] = dot4(Bqj, ne) / jt.lbar;  /* (2/lbar) (B_k q_j) . (1/2 q_{j+1} (x) e_b) */
            ud[k] += a[k][b] * w[3 * j + b] + bb[k][b] * w[3 * (j + 1) + b];
        }
    }
}

double oracle_dissipation(const oracle_rod* rod, const double* x, const double* q,
                          const double* v, const double* w) {
    const double td = rod->damp_int;
    double D = 0.0;
    for (int j = 0; j < rod->n; ++j) {
        if (rod->inextensible) break;
        elem_t e;
        element(rod, j, &e);
        double t[3];
        const double sd = stretch_rate(rod, j, x, v, t);
        D += 0.5 * td * e.Ks * e.l * sd * sd;                 /* eq. (2) at the strain rate */
    }
    for (int j = 0; j + 1 < rod->n; ++j) {
        joint_t jt;
        joint(rod, j, &jt);
        double ud[3], a[3][3], bb[3][3];
        darboux_rate(rod, q, w, j, ud, a, bb);
        for (int k = 0; k < 3; ++k) D += 0.5 * td * jt.K[k] * ud[k] * ud[k] * jt.lbar;   /* eq. (3) */
    }
    return D;
}

void oracle_damping_forces(const oracle_rod* rod, const double* x, const double* q,
                           const double* v, const double* w, double* F, double* tau) {
    const double td = rod->damp_int;
    if (!(td > 0.0)) return;
    for (int j = 0; j < rod->n && !rod->inextensible; ++j) {
        elem_t e;
        element(rod, j, &e);
        double t[3];
        const double sd = stretch_rate(rod, j, x, v, t);
        /* -dD/dv: D_j = 1/2 td Ks l sd^2, d sd / d v_{j+1} = t / l */
        for (int c = 0; c < 3; ++c) {
            F[3 * (j + 1) + c] -= td * e.Ks * sd * t[c];
            F[3 * j + c] += td * e.Ks * sd * t[c];
        }
    }
    for (int j = 0; j + 1 < rod->n; ++j) {
        joint_t jt;
        joint(rod, j, &jt);
        double ud[3], a[3][3], bb[3][3];
        darboux_rate(rod, q, w, j, ud, a, bb);
        for (int b = 0; b < 3; ++b)
            for (int k = 0; k < 3; ++k) {
                const double g = td * jt.K[k] * ud[k] * jt.lbar;   /* dD / d udot_k */
                tau[3 * j + b] -= g * a[k][b];
                tau[3 * (j + 1) + b] -= g * bb[k][b];
            }
    }
}

/* -------------------------------------------------------------------------- clamp -- */

void oracle_clamp_pose(const oracle_rod* rod, double t, double* xc, double* qc, double* wc) {
    const double two_pi_f = 2.0 * M_PI * rod->clamp_freq;
    double sx = sin(two_pi_f * t + rod->clamp_phase_x);
    for (int c = 0; c < 3; ++c) xc[c] = rod->clamp_x0[c] + rod->clamp_amp[c] * sx;
    double psi = rod->clamp_twist_amp * sin(two_pi_f * t + rod->clamp_phase_twist);
    double psidot = rod->clamp_twist_amp * two_pi_f * cos(two_pi_f * t + rod->clamp_phase_twist);
    const double* ax = rod->clamp_twist_axis;
    double an = norm3(ax);
    double axis[3] = {0, 0, 0};
    if (an > 0) for (int c = 0; c < 3; ++c) axis[c] = ax[c] / an;
    double rq[4] = {cos(0.5 * psi), sin(0.5 * psi) * axis[0], sin(0.5 * psi) * axis[1],
                    sin(0.5 * psi) * axis[2]};
    oracle_qmul(rq, rod->clamp_q0, qc);
    /* world rate psidot * axis, expressed in the body axes of q_c: R(q_c)^T (psidot axis) */
    double R[3][3];
    rotmat(qc, R);
    for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (int c = 0; c < 3; ++c) s += R[c][a] * psidot * axis[c];
        wc[a] = s;
    }
}

/* --------------------------------------------------------------------------- step -- */

static void project_segment(const oracle_rod* rod, int j, const double* x, double* v,
                            const double* winv, double* imp0) {
    const double dt = rod->dt;
    double p0[3], p1[3], d[3];
    for (int c = 0; c < 3; ++c) {
        p0[c] = x[3 * j + c] + dt * v[3 * j + c];
        p1[c] = x[3 * (j + 1) + c] + dt * v[3 * (j + 1) + c];
        d[c] = p1[c] - p0[c];
    }
    double len = norm3(d);
    double wsum = winv[j] + winv[j + 1];
    if (!(wsum > 0.0) || !(len > 0.0)) return;
    double C = len - rod->seg_len[j];                  /* C_d: length error */
    double lambda = C / (dt * wsum);                   /* J M^-1 J^T = w_j + w_{j+1} */
    for (int c = 0; c < 3; ++c) {
        double nc = d[c] / len;
        v[3 * j + c] += winv[j] * lambda * nc;
        v[3 * (j + 1) + c] -= winv[j + 1] * lambda * nc;
        if (j == 0 && imp0) imp0[c] += lambda * nc;   /* impulse of segment 0 on point 0 */
    }
}

/* The phases of one step (Sec. 2.1; Fig. 5 without collisions): forces and their integration
 * with the clamp velocities (first), the distance constraints of one iteration (middle), and the
 * velocity integration with the clamp pose (last). */
typedef struct {
    double* winv;
    double xc[3], qc[4], wc[3];
    double fb[3];   /* force on the base point: internal force, then + impulses / dt */
} step_scratch;

static void step_first(const oracle_rod* rod, double t, const double* x, double* v, const double* q,
                       double* w, step_scratch* sc) {
    const int n = rod->n;
    const double dt = rod->dt;
    double* F = (double*)malloc(sizeof(double) * 3 * (n + 1));
    double* tau = (double*)malloc(sizeof(double) * 3 * n);
    sc->winv = (double*)malloc(sizeof(double) * (n + 1));
    double* winv = sc->winv;

    /* forces and torques from the start-of-step configuration, internal friction from the
     * start-of-step velocities */
    oracle_forces(rod, x, q, F, tau);
    oracle_damping_forces(rod, x, q, v, w, F, tau);
    {   /* internal force on point 0: without its weight and external load */
        const double M0 = point_mass(rod, 0);
        for (int c = 0; c < 3; ++c)
            sc->fb[c] = F[c] - M0 * rod->gravity[c] - (rod->f_ext ? rod->f_ext[c] : 0.0);
    }

    /* integrate forces: points as particles */
    for (int i = 0; i <= n; ++i) {
        double M = point_mass(rod, i);
        winv[i] = (rod->clamp && i == 0) ? 0.0 : 1.0 / M;
        if (rod->clamp && i == 0) continue;
        for (int c = 0; c < 3; ++c) {
            double a = F[3 * i + c] / M - rod->damp_lin * v[3 * i + c];
            v[3 * i + c] += dt * a;
        }
    }
    /* integrate torques: frames as rigid bodies, Euler's equations in body axes */
    for (int j = 0; j < n; ++j) {
        if (rod->clamp && j == 0) continue;
        elem_t e;
        element(rod, j, &e);
        double I[3] = {e.I1, e.I1, e.I3};
        double* wj = w + 3 * j;
        double Iw[3] = {I[0] * wj[0], I[1] * wj[1], I[2] * wj[2]};
        double gyro[3];
        cross3(wj, Iw, gyro);
        double tq[3];
        for (int a = 0; a < 3; ++a) {
            tq[a] = tau[3 * j + a] - gyro[a];
            if (rod->tau_ext) tq[a] += rod->tau_ext[3 * j + a];
        }
        for (int a = 0; a < 3; ++a) wj[a] += dt * (tq[a] / I[a] - rod->damp_ang * wj[a]);
    }
    if (rod->clamp) {
        oracle_clamp_pose(rod, t + dt, sc->xc, sc->qc, sc->wc);
        for (int c = 0; c < 3; ++c) {
            v[c] = (sc->xc[c] - x[c]) / dt;
            w[c] = sc->wc[c];
        }
    }
    free(F);
    free(tau);
}

/* one constraint iteration of the inextensible variant: red-black Gauss-Seidel sweeps */
static void step_sweeps(const oracle_rod* rod, const double* x, double* v, step_scratch* sc) {
    double imp0[3] = {0.0, 0.0, 0.0};
    for (int parity = 0; parity < 2; ++parity)
        for (int j = parity; j < rod->n; j += 2) project_segment(rod, j, x, v, sc->winv, imp0);
    for (int c = 0; c < 3; ++c) sc->fb[c] += imp0[c] / rod->dt;
}

static void step_last(const oracle_rod* rod, double* x, const double* v, double* q, const double* w,
                      step_scratch* sc) {
    const int n = rod->n;
    const double dt = rod->dt;
    /* integrate velocities */
    for (int i = 0; i <= n; ++i)
        for (int c = 0; c < 3; ++c) x[3 * i + c] += dt * v[3 * i + c];
    for (int j = 0; j < n; ++j) {
        double* qj = q + 4 * j;
        double om[4] = {0.0, w[3 * j], w[3 * j + 1], w[3 * j + 2]};
        double dq[4];
        oracle_qmul(qj, om, dq);                       /* dq/dt = 1/2 q (x) (0, omega) */
        double nq = 0.0;
        for (int a = 0; a < 4; ++a) {
            qj[a] += 0.5 * dt * dq[a];
            nq += qj[a] * qj[a];
        }
        nq = sqrt(nq);
        for (int a = 0; a < 4; ++a) qj[a] /= nq;
    }
    if (rod->clamp) {
        for (int c = 0; c < 3; ++c) x[c] = sc->xc[c];
        for (int a = 0; a < 4; ++a) q[a] = sc->qc[a];
    }
    free(sc->winv);
    sc->winv = NULL;
}

void oracle_step(const oracle_rod* rod, double t, double* x, double* v, double* q, double* w) {
    oracle_step_fb(rod, t, x, v, q, w, NULL);
}

void oracle_step_fb(const oracle_rod* rod, double t, double* x, double* v, double* q, double* w,
                    double* fbase) {
    step_scratch sc;
    step_first(rod, t, x, v, q, w, &sc);
    if (rod->inextensible)
        for (int it = 0; it < rod->n_iter; ++it) step_sweeps(rod, x, v, &sc);
    if (fbase)
        for (int c = 0; c < 3; ++c) fbase[c] = sc.fb[c];
    step_last(rod, x, v, q, w, &sc);
}

void oracle_rollout_fb(const oracle_rod* rod, double t0, int32_t n_steps, double* x, double* v,
                       double* q, double* w, double* fbase) {
    for (int s = 0; s < n_steps; ++s)
        oracle_step_fb(rod, t0 + s * rod->dt, x, v, q, w, fbase ? fbase + 3 * s : NULL);
}

/* ------------------------------------------------------------------------ binding -- */

/* One binding constraint (Sec. 2.1 "Constraints": a distance constraint whose rest length is
 * zero, solved as a velocity impulse like the distance constraints) between point a (position
 * xa, velocity va, inverse mass wa) and point b.  two-way: both points respond by their inverse
 * masses; one-way: point b belongs to the master instrument and does not move. */
void oracle_bind_impulse(const double* xa, double* va, double wa, const double* xb, double* vb,
                         double wb, double dt, int32_t one_way) {
    double d[3];
    for (int c = 0; c < 3; ++c) d[c] = (xa[c] + dt * va[c]) - (xb[c] + dt * vb[c]);
    const double len = norm3(d);
    const double wsum = one_way ? wa : wa + wb;
    if (!(wsum > 0.0) || !(len > 0.0)) return;
    const double lambda = (len - 0.0) / (dt * wsum);   /* C = |d| - 0 */
    for (int c = 0; c < 3; ++c) {
        const double nc = d[c] / len;
        va[c] -= wa * lambda * nc;
        if (!one_way) vb[c] += wb * lambda * nc;
    }
}

void oracle_step_pair(const oracle_rod* a, const oracle_rod* b, const oracle_binding* bind,
                      double t, double* xa, double* va, double* qa, double* wa, double* xb,
                      double* vb, double* qb, double* wb) {
    step_scratch sa, sb;
    step_first(a, t, xa, va, qa, wa, &sa);
    step_first(b, t, xb, vb, qb, wb, &sb);
    /* per iteration: distance constraints of both rods, then the binding impulses (Fig. 5) */
    for (int it = 0; it < a->n_iter; ++it) {
        if (a->inextensible) step_sweeps(a, xa, va, &sa);
        if (b->inextensible) step_sweeps(b, xb, vb, &sb);
        for (int k = 0; k < bind->n_pairs; ++k) {
            const int i = bind->point_a[k], j = bind->point_b[k];
            oracle_bind_impulse(xa + 3 * i, va + 3 * i, sa.winv[i], xb + 3 * j, vb + 3 * j,
                                sb.winv[j], a->dt, bind->one_way);
        }
    }
    step_last(a, xa, va, qa, wa, &sa);
    step_last(b, xb, vb, qb, wb, &sb);
}

/* ------------------------------------------------------------------------ contact -- */

/* Sphere radius of point i: the radius of its element, the mean of both at interior points. */
static double point_radius(const oracle_rod* rod, int i) {
    if (i == 0) return rod->radius[0];
    if (i == rod->n) return rod->radius[rod->n - 1];
    return 0.5 * (rod->radius[i - 1] + rod->radius[i]);
}

int32_t oracle_self_skip(const oracle_rod* rod) {
    double rmax = 0.0, lmin = INFINITY;
    for (int j = 0; j < rod->n; ++j) {
        if (rod->radius[j] > rmax) rmax = rod->radius[j];
        if (rod->seg_len[j] < lmin) lmin = rod->seg_len[j];
    }
    int32_t s = (int32_t)ceil(2.0 * rmax / lmin);
    return s < 1 ? 1 : s;
}

/* contacts of point i of rod ra: (rod, point) pairs with overlapping spheres at positions x */
typedef struct {
    int rod, pt;
    double n[3], D;
} contact_t;

static int find_contacts(const oracle_rod* const* rods, int n_rods, double* const* x, int ra,
                         int i, contact_t* out, int cap) {
    int k = 0;
    const double ri = point_radius(rods[ra], i);
    for (int rb = 0; rb < n_rods; ++rb) {
        const int skip = oracle_self_skip(rods[rb]);
        for (int j = 1; j <= rods[rb]->n; ++j) {
            if (rb == ra && abs(j - i) <= skip) continue;
            double d[3];
            for (int c = 0; c < 3; ++c) d[c] = x[ra][3 * i + c] - x[rb][3 * j + c];
            const double len = norm3(d);
            const double D = ri + point_radius(rods[rb], j);
            if (!(len < D) || !(len > 0.0)) continue;
            if (k < cap) {
                out[k].rod = rb;
                out[k].pt = j;
                for (int c = 0; c < 3; ++c) out[k].n[c] = d[c] / len;
                out[k].D = D;
            }
            ++k;
        }
    }
    return k;
}

void oracle_step_group(const oracle_rod* const* rods, int32_t n_rods, const oracle_binding* bind,
                       const oracle_contact* contact, double t, double* const* x, double* const* v,
                       double* const* q, double* const* w, int32_t* max_contacts) {
    step_scratch sc[2];
    const oracle_rod* a = rods[0];
    const double dt = a->dt;
    for (int r = 0; r < n_rods; ++r) step_first(rods[r], t, x[r], v[r], q[r], w[r], &sc[r]);
    /* contacts from the start-of-step positions (Fig. 5: detection first), points 1..n */
    contact_t* cl[2] = {NULL, NULL};
    int* cn[2] = {NULL, NULL};
    int cap = 0, most = 0;
    if (contact) {
        for (int r = 0; r < n_rods; ++r) cap += rods[r]->n;
        for (int r = 0; r < n_rods; ++r) {
            cl[r] = (contact_t*)malloc(sizeof(contact_t) * (size_t)(rods[r]->n + 1) * cap);
            cn[r] = (int*)calloc((size_t)rods[r]->n + 1, sizeof(int));
            for (int i = 1; i <= rods[r]->n; ++i) {
                cn[r][i] = find_contacts(rods, n_rods, x, r, i, cl[r] + (size_t)i * cap, cap);
                if (cn[r][i] > most) most = cn[r][i];
            }
        }
    }
    if (max_contacts) *max_contacts = most;
    double* dv[2] = {NULL, NULL};
    if (contact)
        for (int r = 0; r < n_rods; ++r) dv[r] = (double*)malloc(sizeof(double) * 3 * (rods[r]->n + 1));
    /* per iteration: distance constraints, bindings, then the contact impulses (Fig. 5) */
    for (int it = 0; it < a->n_iter; ++it) {
        for (int r = 0; r < n_rods; ++r)
            if (rods[r]->inextensible) step_sweeps(rods[r], x[r], v[r], &sc[r]);
        if (bind && n_rods == 2)
            for (int k = 0; k < bind->n_pairs; ++k) {
                const int i = bind->point_a[k], j = bind->point_b[k];
                oracle_bind_impulse(x[0] + 3 * i, v[0] + 3 * i, sc[0].winv[i], x[1] + 3 * j,
                                    v[1] + 3 * j, sc[1].winv[j], dt, bind->one_way);
            }
        if (!contact) continue;
        /* Jacobi: every point's contacts from the same velocities; a point applies the mean of
         * its active contacts' impulses */
        for (int r = 0; r < n_rods; ++r)
            for (int i = 0; i <= rods[r]->n; ++i) {
                double acc[3] = {0.0, 0.0, 0.0};
                int active = 0;
                for (int k = 0; i > 0 && k < cn[r][i]; ++k) {
                    const contact_t* ct = cl[r] + (size_t)i * cap + k;
                    const double* xi = x[r] + 3 * i;
                    const double* vi = v[r] + 3 * i;
                    const double* xj = x[ct->rod] + 3 * ct->pt;
                    const double* vj = v[ct->rod] + 3 * ct->pt;
                    const double wi = sc[r].winv[i], wj = sc[ct->rod].winv[ct->pt];
                    if (!(wi + wj > 0.0)) continue;
                    double sep = -ct->D;   /* predicted separation along the contact normal */
                    for (int c = 0; c < 3; ++c) sep += ((xi[c] + dt * vi[c]) - (xj[c] + dt * vj[c])) * ct->n[c];
                    if (!(sep < 0.0)) continue;
                    const double lam = -sep / (dt * (wi + wj));       /* normal impulse */
                    double vr[3], vrn = 0.0;
                    for (int c = 0; c < 3; ++c) {
                        vr[c] = vi[c] - vj[c];
                        vrn += vr[c] * ct->n[c];
                    }
                    double vt[3];
                    for (int c = 0; c < 3; ++c) vt[c] = vr[c] - vrn * ct->n[c];
                    const double vtl = norm3(vt);
                    double lt = 0.0;                                   /* Coulomb friction */
                    if (vtl > 0.0) {
                        lt = vtl / (wi + wj);
                        if (lt > contact->mu * lam) lt = contact->mu * lam;
                    }
                    for (int c = 0; c < 3; ++c)
                        acc[c] += wi * lam * ct->n[c] - (vtl > 0.0 ? wi * lt * vt[c] / vtl : 0.0);
                    ++active;
                }
                for (int c = 0; c < 3; ++c) dv[r][3 * i + c] = active ? acc[c] / active : 0.0;
            }
        for (int r = 0; r < n_rods; ++r)
            for (int i = 0; i <= rods[r]->n; ++i)
                for (int c = 0; c < 3; ++c) v[r][3 * i + c] += dv[r][3 * i + c];
    }
    for (int r = 0; r < n_rods; ++r) {
        step_last(rods[r], x[r], v[r], q[r], w[r], &sc[r]);
        free(cl[r]);
        free(cn[r]);
        free(dv[r]);
    }
}

/* Rounds n values to the nearest FP32 number (kept as doubles). */
static void round_fp32(double* a, int n) {
    for (int i = 0; i < n; ++i) a[i] = (double)(float)a[i];
}

/* The fields of one rod's state named by the bits of mask (1 x, 2 v, 4 q, 8 w), rounded. */
static void round_state(int n, double* x, double* v, double* q, double* w, int32_t mask) {
    if (mask & 1) round_fp32(x, 3 * (n + 1));
    if (mask & 2) round_fp32(v, 3 * (n + 1));
    if (mask & 4) round_fp32(q, 4 * n);
    if (mask & 8) round_fp32(w, 3 * n);
}

void oracle_rollout_group_rounded(const oracle_rod* const* rods, int32_t n_rods,
                                  const oracle_binding* bind, const oracle_contact* contact,
                                  double t0, int32_t n_steps, double* const* x,
                                  double* const* v, double* const* q, double* const* w,
                                  int32_t mask, int32_t* max_contacts) {
    int32_t most = 0;
    for (int s = 0; s < n_steps; ++s) {
        int32_t m = 0;
        oracle_step_group(rods, n_rods, bind, contact, t0 + s * rods[0]->dt, x, v, q, w, &m);
        if (m > most) most = m;
        for (int r = 0; r < n_rods; ++r) round_state(rods[r]->n, x[r], v[r], q[r], w[r], mask);
    }
    if (max_contacts) *max_contacts = most;
}

void oracle_rollout_group(const oracle_rod* const* rods, int32_t n_rods,
                          const oracle_binding* bind, const oracle_contact* contact, double t0,
                          int32_t n_steps, double* const* x, double* const* v, double* const* q,
                          double* const* w, int32_t* max_contacts) {
    int32_t most = 0;
    for (int s = 0; s < n_steps; ++s) {
        int32_t m = 0;
        oracle_step_group(rods, n_rods, bind, contact, t0 + s * rods[0]->dt, x, v, q, w, &m);
        if (m > most) most = m;
    }
    if (max_contacts) *max_contacts = most;
}

/* -------------------------------------------------------------- environment -- */

static void segment_closest(const double* p, const double* a, const double* b, double* out) {
    double ab[3], ap[3];
    for (int c = 0; c < 3; ++c) {
        ab[c] = b[c] - a[c];
        ap[c] = p[c] - a[c];
    }
    const double L2 = dot3(ab, ab);
    double t = L2 > 0.0 ? dot3(ap, ab) / L2 : 0.0;
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    for (int c = 0; c < 3; ++c) out[c] = a[c] + t * ab[c];
}

void oracle_closest_point_triangle(const double* p, const double* tri, double* out) {
    const double* A = tri;
    const double* B = tri + 3;
    const double* Cv = tri + 6;
    double ab[3], ac[3], N[3];
    for (int c = 0; c < 3; ++c) {
        ab[c] = B[c] - A[c];
        ac[c] = Cv[c] - A[c];
    }
    cross3(ab, ac, N);
    const double nn = dot3(N, N);
    if (nn > 0.0) {
        /* projection onto the plane; inside if it lies on the inner side of all three edges */
        double ap[3];
        for (int c = 0; c < 3; ++c) ap[c] = p[c] - A[c];
        const double h = dot3(ap, N) / nn;
        double pp[3];
        for (int c = 0; c < 3; ++c) pp[c] = p[c] - h * N[c];
        const double* V[3] = {A, B, Cv};
        int inside = 1;
        for (int k = 0; k < 3; ++k) {
            const double* P0 = V[k];
            const double* P1 = V[(k + 1) % 3];
            double e[3], d[3], cr[3];
            for (int c = 0; c < 3; ++c) {
                e[c] = P1[c] - P0[c];
                d[c] = pp[c] - P0[c];
            }
            cross3(e, d, cr);
            if (dot3(cr, N) < 0.0) inside = 0;
        }
        if (inside) {
            for (int c = 0; c < 3; ++c) out[c] = pp[c];
            return;
        }
    }
    /* otherwise the nearest point of the three edges */
    double best = INFINITY;
    const double* E[3][2] = {{A, B}, {B, Cv}, {Cv, A}};
    for (int k = 0; k < 3; ++k) {
        double q[3], d[3];
        segment_closest(p, E[k][0], E[k][1], q);
        for (int c = 0; c < 3; ++c) d[c] = p[c] - q[c];
        const double dd = dot3(d, d);
        if (dd < best) {
            best = dd;
            for (int c = 0; c < 3; ++c) out[c] = q[c];
        }
    }
}

void oracle_env_response(const oracle_env* env, const double* c, double r, double* n,
                         double* depth, int32_t* hits) {
    double acc[3] = {0.0, 0.0, 0.0};
    double dmax = 0.0;
    int k = 0;
    for (int t = 0; t < env->n_tris; ++t) {
        const double* tri = env->tris + 9 * t;
        double q[3], d[3], ab[3], ac[3], N[3];
        oracle_closest_point_triangle(c, tri, q);
        for (int a = 0; a < 3; ++a) {
            d[a] = c[a] - q[a];
            ab[a] = tri[3 + a] - tri[a];
            ac[a] = tri[6 + a] - tri[a];
        }
        const double dist = norm3(d);
        if (!(dist < r)) continue;
        cross3(ab, ac, N);
        const double nl = norm3(N);
        if (!(nl > 0.0)) continue;
        for (int a = 0; a < 3; ++a) N[a] /= nl;
        double cp[3];
        for (int a = 0; a < 3; ++a) cp[a] = c[a] - tri[a];
        /* penetration depth: the sphere reaches r - dist past the face, or, with its centre
         * behind the face, r + dist */
        const double dep = dot3(cp, N) >= 0.0 ? r - dist : r + dist;
        for (int a = 0; a < 3; ++a) acc[a] += dep * N[a];
        if (dep > dmax) dmax = dep;
        ++k;
    }
    const double al = norm3(acc);
    if (k > 0 && al > 0.0) {
        for (int a = 0; a < 3; ++a) n[a] = acc[a] / al;
        *depth = dmax;
    } else {
        for (int a = 0; a < 3; ++a) n[a] = 0.0;
        *depth = 0.0;
    }
    if (hits) *hits = k;
}

void oracle_env_impulse(const double* n, double depth, double winv, double dt, double mu,
                        double* v) {
    if (!(depth > 0.0) || !(winv > 0.0)) return;
    const double sep = dt * dot3(v, n) - depth;   /* predicted motion along n minus the depth */
    if (!(sep < 0.0)) return;
    const double lam = -sep / (dt * winv);       /* normal impulse (the wall does not move) */
    const double vn = dot3(v, n);
    double vt[3];
    for (int c = 0; c < 3; ++c) vt[c] = v[c] - vn * n[c];
    const double vtl = norm3(vt);
    double lt = 0.0;                              /* Coulomb friction */
    if (vtl > 0.0) {
        lt = vtl / winv;
        if (lt > mu * lam) lt = mu * lam;
    }
    for (int c = 0; c < 3; ++c)
        v[c] += winv * lam * n[c] - (vtl > 0.0 ? winv * lt * vt[c] / vtl : 0.0);
}

void oracle_step_env(const oracle_rod* rod, const oracle_env* env, double t, double* x, double* v,
                     double* q, double* w, int32_t* colliding) {
    step_scratch sc;
    step_first(rod, t, x, v, q, w, &sc);
    /* detection from the start-of-step positions (Fig. 5: detection first), points 1..n */
    const int n = rod->n;
    double* nrm = (double*)calloc((size_t)3 * (n + 1), sizeof(double));
    double* dep = (double*)calloc((size_t)n + 1, sizeof(double));
    int count = 0;
    for (int i = 1; i <= n; ++i) {
        oracle_env_response(env, x + 3 * i, point_radius(rod, i), nrm + 3 * i, dep + i, NULL);
        if (dep[i] > 0.0) ++count;
    }
    if (colliding) *colliding = count;
    /* per iteration: distance constraints, then the collision response (Fig. 5); a rod
     * without constraint iterations takes the response once */
    const int iters = (rod->inextensible && rod->n_iter > 0) ? rod->n_iter : 1;
    for (int it = 0; it < iters; ++it) {
        if (rod->inextensible && it < rod->n_iter) step_sweeps(rod, x, v, &sc);
        for (int i = 1; i <= n; ++i)
            oracle_env_impulse(nrm + 3 * i, dep[i], sc.winv[i], rod->dt, env->mu, v + 3 * i);
    }
    free(nrm);
    free(dep);
    step_last(rod, x, v, q, w, &sc);
}

void oracle_rollout_env(const oracle_rod* rod, const oracle_env* env, double t0, int32_t n_steps,
                        double* x, double* v, double* q, double* w, int32_t* most) {
    int32_t m = 0;
    for (int s = 0; s < n_steps; ++s) {
        int32_t c = 0;
        oracle_step_env(rod, env, t0 + s * rod->dt, x, v, q, w, &c);
        if (c > m) m = c;
    }
    if (most) *most = m;
}

void oracle_rollout_pair(const oracle_rod* a, const oracle_rod* b, const oracle_binding* bind,
                         double t0, int32_t n_steps, double* xa, double* va, double* qa, double* wa,
                         double* xb, double* vb, double* qb, double* wb) {
    for (int s = 0; s < n_steps; ++s)
        oracle_step_pair(a, b, bind, t0 + s * a->dt, xa, va, qa, wa, xb, vb, qb, wb);
}

void oracle_rollout(const oracle_rod* rod, double t0, int32_t n_steps, double* x, double* v,
                    double* q, double* w, double* tip) {
    for (int s = 0; s < n_steps; ++s) {
        oracle_step(rod, t0 + s * rod->dt, x, v, q, w);
        if (tip)
            for (int c = 0; c < 3; ++c) tip[3 * s + c] = x[3 * rod->n + c];
    }
}


void oracle_rollout_rounded(const oracle_rod* rod, double t0, int32_t n_steps, double* x,
                            double* v, double* q, double* w, int32_t mask) {
    for (int s = 0; s < n_steps; ++s) {
        oracle_step(rod, t0 + s * rod->dt, x, v, q, w);
        round_state(rod->n, x, v, q, w, mask);
    }
}

double oracle_max_strain(const oracle_rod* rod, const double* x) {
    double m = 0.0;
    for (int j = 0; j < rod->n; ++j) {
        double d[3];
        for (int c = 0; c < 3; ++c) d[c] = x[3 * (j + 1) + c] - x[3 * j + c];
        double s = fabs(norm3(d) / rod->seg_len[j] - 1.0);
        if (!(s == s)) return INFINITY;
        if (s > m) m = s;
    }
    return m;
}

int32_t oracle_stable(const oracle_rod* rod, double t0, int32_t n_steps, const double* x0,
                      const double* v0, const double* q0, const double* w0,
                      double energy_factor) {
    const int n = rod->n;
    double* x = (double*)malloc(sizeof(double) * 3 * (n + 1));
    double* v = (double*)malloc(sizeof(double) * 3 * (n + 1));
    double* q = (double*)malloc(sizeof(double) * 4 * n);
    double* w = (double*)malloc(sizeof(double) * 3 * n);
    memcpy(x, x0, sizeof(double) * 3 * (n + 1));
    memcpy(v, v0, sizeof(double) * 3 * (n + 1));
    memcpy(q, q0, sizeof(double) * 4 * n);
    memcpy(w, w0, sizeof(double) * 3 * n);
    double E0 = oracle_kinetic(rod, v, w) + oracle_energy(rod, x, q);
    int ok = 1;
    for (int s = 0; s < n_steps && ok; ++s) {
        oracle_step(rod, t0 + s * rod->dt, x, v, q, w);
        double E = oracle_kinetic(rod, v, w) + oracle_energy(rod, x, q);
        if (!(E == E) || !isfinite(E)) ok = 0;
        else if (E > E0 + (energy_factor - 1.0) * fabs(E0) + 1e-9) ok = 0;
        else if (!(oracle_max_strain(rod, x) < 0.5)) ok = 0;
    }
    free(x);
    free(v);
    free(q);
    free(w);
    return ok;
}

double oracle_dt_rule(const oracle_rod* rod) {
    double best = INFINITY;
    for (int j = 0; j < rod->n; ++j) {
        elem_t e;
        element(rod, j, &e);
        double om[5];
        int nm = 0;
        /* one-element mode frequencies of a uniform chain: 2 sqrt(k / m) for the
         * alternating translational modes, sqrt(k_rot / I) for the rotational ones */
        int damped[5];
        if (!rod->inextensible) {
            damped[nm] = 1;
            om[nm++] = 2.0 * sqrt(e.Ks / e.l / e.m);
        }
        damped[nm] = 0;
        om[nm++] = 2.0 * sqrt(e.Kp / e.l / e.m);
        damped[nm] = 0;
        om[nm++] = sqrt(e.l * e.Kp / e.I1);
        damped[nm] = 1;
        om[nm++] = sqrt(4.0 * e.K1 / (e.l * e.I1));
        damped[nm] = 1;
        om[nm++] = sqrt(4.0 * e.K3 / (e.l * e.I3));
        for (int k = 0; k < nm; ++k) {
            double dt = 2.0 / om[k];
            /* a Kelvin-Voigt damper on the mode decays at tau_d om^2: explicit in dt too */
            if (damped[k] && rod->damp_int > 0.0) {
                const double dd = 2.0 / (rod->damp_int * om[k] * om[k]);
                if (dd < dt) dt = dd;
            }
            if (dt < best) best = dt;
        }
    }
    return 0.5 * best;
}
