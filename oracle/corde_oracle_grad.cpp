/*
 * corde_oracle_grad.cpp -- FP64 reference derivatives of the oracle's rod rollout.
 *
 * TEST INFRASTRUCTURE ONLY (see corde_oracle.h): the test-suite and the CPU-baseline leg of the
 * benchmark use it; the product library never does.  It shares no code with the GPU path.
 *
 * What is differentiated: the tip trajectory tip(s) = x_N after step s of a rollout of the
 * plain step (Sec. 2.1; Fig. 5 without collision, self-collision and binding lines), with
 * respect to the initial state (x, v, q, w -- q by its four stored components, not projected
 * on the unit sphere) and two per-rod multipliers: m_b of the bending stiffness K_1 = K_2 and
 * m_t of the twisting stiffness K_3 of eq. (3) (the oracle's bend_scale and twist_scale are
 * multiplied by them).  Material, dt and the clamp motion are constants.
 *
 * How: the oracle step of corde_oracle.c is written out once more below as a template over the
 * scalar type, in the oracle's own order of operations (the quaternion matrices B_k and the
 * clamp pose are taken from the oracle itself), and instantiated three times:
 *   double -- must reproduce oracle_step bitwise, which ties this copy to the pinned oracle;
 *   Dual   -- forward mode: each number carries one directional derivative (JVP);
 *   Var    -- reverse mode: every operation is recorded on a tape with its local partial
 *             derivatives, and the tape is swept backward (VJP).  The rollout is replayed one
 *             step at a time from stored step-start states, newest first, so a tape holds one
 *             step.
 * Only elementary rules are involved: d(a+b), d(a-b), d(ab) = b da + a db,
 * d(a/b) = (da - (a/b) db)/b, d sqrt(a) = da / (2 sqrt(a)).
 * Internal friction (damp_int > 0) is not covered and is refused.
 */
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

#include "corde_oracle.h"

namespace {

// ------------------------------------------------------------------ forward mode --

struct Dual {
    double v, d;
    Dual(double a = 0.0, double b = 0.0) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
    const double r = a.v / b.v;
    return Dual(r, (a.d - r * b.d) / b.v);
}
inline Dual sqrt(Dual a) {
    const double s = std::sqrt(a.v);
    return Dual(s, a.d / (2.0 * s));
}
inline double value(Dual a) { return a.v; }

// ------------------------------------------------------------------ reverse mode --

// One recorded operation: result = f(parent a, parent b) with partials pa, pb (-1: no parent).
struct Tape {
    std::vector<int32_t> a, b;
    std::vector<double> pa, pb;
    int32_t push(int32_t i, double p, int32_t j, double q) {
        a.push_back(i);
        pa.push_back(p);
        b.push_back(j);
        pb.push_back(q);
        return (int32_t)a.size() - 1;
    }
    void clear() {
        a.clear();
        b.clear();
        pa.clear();
        pb.clear();
    }
    // adj[k] holds the seeds on entry and d(seeded output)/d(node k) on return
    void sweep(std::vector<double>& adj) const {
        for (int32_t k = (int32_t)a.size() - 1; k >= 0; --k) {
            const double g = adj[k];
            if (g == 0.0) continue;
            if (a[k] >= 0) adj[a[k]] += pa[k] * g;
            if (b[k] >= 0) adj[b[k]] += pb[k] * g;
        }
    }
};

thread_local Tape* g_tape = nullptr;

struct Var {
    double v;
    int32_t i;   // tape index; -1 for a constant
    Var(double x = 0.0) : v(x), i(-1) {}
};
inline Var make(double v, int32_t i, double pi, int32_t j, double pj) {
    Var r(v);
    if (i >= 0 || j >= 0) r.i = g_tape->push(i, pi, j, pj);
    return r;
}
inline Var operator+(Var a, Var b) { return make(a.v + b.v, a.i, 1.0, b.i, 1.0); }
inline Var operator-(Var a, Var b) { return make(a.v - b.v, a.i, 1.0, b.i, -1.0); }
inline Var operator-(Var a) { return make(-a.v, a.i, -1.0, -1, 0.0); }
inline Var operator*(Var a, Var b) { return make(a.v * b.v, a.i, b.v, b.i, a.v); }
inline Var operator/(Var a, Var b) {
    const double r = a.v / b.v;
    return make(r, a.i, 1.0 / b.v, b.i, -r / b.v);
}
inline Var sqrt(Var a) {
    const double s = std::sqrt(a.v);
    return make(s, a.i, 0.5 / s, -1, 0.0);
}
inline double value(Var a) { return a.v; }
// a tape leaf (an independent variable)
inline Var leaf(double v) {
    Var r(v);
    r.i = g_tape->push(-1, 0.0, -1, 0.0);
    return r;
}

inline double value(double a) { return a; }
inline double sqrt(double a) { return std::sqrt(a); }

template <class S> inline S& operator+=(S& a, const S& b) { return a = a + b; }
template <class S> inline S& operator-=(S& a, const S& b) { return a = a - b; }
template <class S> inline S& operator/=(S& a, const S& b) { return a = a / b; }
inline Dual& operator+=(Dual& a, double b) { return a = a + Dual(b); }
inline Var& operator+=(Var& a, double b) { return a = a + Var(b); }

// ------------------------------------------------------- the step, over a scalar S --

// B_k q for the oracle's matrices (entries 0 and +-1, so the product is a signed permutation,
// which is exactly what the oracle's 4x4 product evaluates to in floating point).
struct BTable {
    double m[3][16];
    BTable() {
        for (int k = 0; k < 3; ++k) oracle_bmat(k, m[k]);
    }
};
const BTable& btable() {
    static const BTable t;
    return t;
}

template <class S>
inline void bmul(int k, const S* q, S* out) {
    const double* B = btable().m[k];
    for (int r = 0; r < 4; ++r) {
        S acc = S(0.0);
        for (int c = 0; c < 4; ++c) {
            const double e = B[4 * r + c];
            if (e == 1.0) acc = acc + q[c];
            else if (e == -1.0) acc = acc - q[c];
        }
        out[r] = acc;
    }
}

template <class S> inline S dot3(const S* a, const S* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
template <class S> inline S dot4(const S* a, const S* b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3];
}
template <class S> inline S norm3(const S* a) { return sqrt(dot3(a, a)); }
template <class S> inline void cross3(const S* a, const S* b, S* r) {
    S t0 = a[1] * b[2] - a[2] * b[1];
    S t1 = a[2] * b[0] - a[0] * b[2];
    S t2 = a[0] * b[1] - a[1] * b[0];
    r[0] = t0;
    r[1] = t1;
    r[2] = t2;
}
template <class S> inline void qmul(const S* a, const S* b, S* r) {
    S w = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    S x = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    S y = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    S z = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
    r[0] = w;
    r[1] = x;
    r[2] = y;
    r[3] = z;
}
// third director d_3(q) and its Jacobian d d_3 / d(w, x, y, z)
template <class S> inline void director3(const S* q, S* d3, S J[3][4]) {
    S w = q[0], x = q[1], y = q[2], z = q[3];
    d3[0] = S(2.0) * (x * z + w * y);
    d3[1] = S(2.0) * (y * z - w * x);
    d3[2] = w * w - x * x - y * y + z * z;
    J[0][0] = S(2.0) * y;  J[0][1] = S(2.0) * z;  J[0][2] = S(2.0) * w;  J[0][3] = S(2.0) * x;
    J[1][0] = -2.0 * x;    J[1][1] = -2.0 * w;    J[1][2] = S(2.0) * z;  J[1][3] = S(2.0) * y;
    J[2][0] = S(2.0) * w;  J[2][1] = -2.0 * x;    J[2][2] = -2.0 * y;    J[2][3] = S(2.0) * z;
}

// Element constants; K1 (= K2) and K3 carry the multipliers and are of type S.
template <class S> struct Elem {
    double l, r, E, G, A, m, Ks, Kp, I1, I3;
    S K1, K3;
};
template <class S>
inline void element(const oracle_rod* rod, int j, const S& mb, const S& mt, Elem<S>* e) {
    e->l = rod->seg_len[j];
    e->r = rod->radius[j];
    e->E = rod->young[j];
    e->G = e->E / (2.0 * (1.0 + rod->poisson));
    e->A = M_PI * e->r * e->r;
    e->m = rod->density * e->A * e->l;
    e->Ks = e->E * e->A;                                   /* eq. (2) */
    e->Kp = rod->kp_scale * e->G * e->A;                   /* eq. (8) */
    const double r4 = e->r * e->r * e->r * e->r;
    e->K1 = S(rod->bend_scale) * mb * S(e->E) * S(M_PI) * S(r4) / S(4.0);    /* eq. (3) */
    e->K3 = S(rod->twist_scale) * mt * S(e->G) * S(M_PI) * S(r4) / S(2.0);
    e->I1 = e->m * (3.0 * e->r * e->r + e->l * e->l) / 12.0;
    e->I3 = e->m * e->r * e->r / 2.0;
}

template <class S> inline double point_mass(const oracle_rod* rod, int i) {
    double M = 0.0;
    Elem<S> e;
    const S one(1.0);
    if (i > 0) {
        element(rod, i - 1, one, one, &e);
        M += 0.5 * e.m;
    }
    if (i < rod->n) {
        element(rod, i, one, one, &e);
        M += 0.5 * e.m;
    }
    return M;
}

template <class S>
void forces(const oracle_rod* rod, const S& mb, const S& mt, const S* x, const S* q, S* F, S* tau) {
    const int n = rod->n;
    std::vector<S> gq((size_t)4 * n, S(0.0));   // dV/dq
    for (int i = 0; i < 3 * (n + 1); ++i) F[i] = S(0.0);
    for (int j = 0; j < n; ++j) {
        Elem<S> e;
        element(rod, j, mb, mt, &e);
        S d[3], t[3], d3[3], J[3][4];
        for (int c = 0; c < 3; ++c) d[c] = x[3 * (j + 1) + c] - x[3 * j + c];
        S len = norm3(d);
        for (int c = 0; c < 3; ++c) t[c] = d[c] / len;
        S g[3] = {S(0.0), S(0.0), S(0.0)};
        if (!rod->inextensible) {
            S s = len / S(e.l) - S(1.0);                         /* eq. (2) */
            for (int c = 0; c < 3; ++c) g[c] += S(e.Ks) * s * t[c];
        }
        director3(q + 4 * j, d3, J);
        S r[3] = {t[0] - d3[0], t[1] - d3[1], t[2] - d3[2]};
        S tr = dot3(t, r);
        for (int c = 0; c < 3; ++c) g[c] += S(e.Kp * e.l) * (r[c] - tr * t[c]) / len;   /* eq. (8) */
        for (int c = 0; c < 3; ++c) {
            F[3 * (j + 1) + c] -= g[c];
            F[3 * j + c] += g[c];
        }
        for (int a = 0; a < 4; ++a) {
            S s = S(0.0);
            for (int c = 0; c < 3; ++c) s += J[c][a] * r[c];
            gq[4 * j + a] -= S(e.Kp * e.l) * s;
        }
    }
    for (int j = 0; j + 1 < n; ++j) {
        Elem<S> a, b;
        element(rod, j, mb, mt, &a);
        element(rod, j + 1, mb, mt, &b);
        const double lbar = 0.5 * (a.l + b.l);
        S K[3];
        K[0] = S(0.5) * (a.K1 + b.K1);
        K[1] = K[0];
        K[2] = S(0.5) * (a.K3 + b.K3);
        for (int k = 0; k < 3; ++k) {
            const double uhat = rod->u_hat ? rod->u_hat[3 * j + k] : 0.0;
            S Bqj[4], Bqn[4];
            bmul(k, q + 4 * j, Bqj);
            S u = S(2.0 / lbar) * dot4(Bqj, q + 4 * (j + 1));  /* eqs. (5), (6) */
            S mk = K[k] * (u - S(uhat));                       /* eq. (3) */
            bmul(k, q + 4 * (j + 1), Bqn);
            for (int c = 0; c < 4; ++c) {
                gq[4 * (j + 1) + c] += S(2.0) * mk * Bqj[c];
                gq[4 * j + c] -= S(2.0) * mk * Bqn[c];
            }
        }
    }
    for (int i = 0; i <= n; ++i) {
        const double M = point_mass<S>(rod, i);
        for (int c = 0; c < 3; ++c) {
            F[3 * i + c] += S(M * rod->gravity[c]);
            if (rod->f_ext) F[3 * i + c] += S(rod->f_ext[3 * i + c]);
        }
    }
    for (int j = 0; j < n; ++j)
        for (int a = 0; a < 3; ++a) {
            S Bq[4];
            bmul(a, q + 4 * j, Bq);
            tau[3 * j + a] = S(-0.5) * dot4(&gq[4 * j], Bq);
        }
}

template <class S>
void project_segment(const oracle_rod* rod, int j, const S* x, S* v, const double* winv) {
    const double dt = rod->dt;
    S p0[3], p1[3], d[3];
    for (int c = 0; c < 3; ++c) {
        p0[c] = x[3 * j + c] + S(dt) * v[3 * j + c];
        p1[c] = x[3 * (j + 1) + c] + S(dt) * v[3 * (j + 1) + c];
        d[c] = p1[c] - p0[c];
    }
    S len = norm3(d);
    const double wsum = winv[j] + winv[j + 1];
    if (!(wsum > 0.0) || !(value(len) > 0.0)) return;
    S C = len - S(rod->seg_len[j]);
    S lambda = C / S(dt * wsum);
    for (int c = 0; c < 3; ++c) {
        S nc = d[c] / len;
        v[3 * j + c] += S(winv[j]) * lambda * nc;
        v[3 * (j + 1) + c] -= S(winv[j + 1]) * lambda * nc;
    }
}

// One step from time t, in place (the oracle's step_first, sweeps and step_last).
template <class S>
void step(const oracle_rod* rod, double t, const S& mb, const S& mt, S* x, S* v, S* q, S* w) {
    const int n = rod->n;
    const double dt = rod->dt;
    std::vector<S> F((size_t)3 * (n + 1)), tau((size_t)3 * n);
    std::vector<double> winv((size_t)n + 1);
    forces(rod, mb, mt, x, q, F.data(), tau.data());
    for (int i = 0; i <= n; ++i) {
        const double M = point_mass<S>(rod, i);
        winv[i] = (rod->clamp && i == 0) ? 0.0 : 1.0 / M;
        if (rod->clamp && i == 0) continue;
        for (int c = 0; c < 3; ++c) {
            S a = F[3 * i + c] / S(M) - S(rod->damp_lin) * v[3 * i + c];
            v[3 * i + c] += S(dt) * a;
        }
    }
    const S one(1.0);
    for (int j = 0; j < n; ++j) {
        if (rod->clamp && j == 0) continue;
        Elem<S> e;
        element(rod, j, one, one, &e);
        const double I[3] = {e.I1, e.I1, e.I3};
        S* wj = w + 3 * j;
        S Iw[3] = {S(I[0]) * wj[0], S(I[1]) * wj[1], S(I[2]) * wj[2]};
        S gyro[3];
        cross3(wj, Iw, gyro);
        S tq[3];
        for (int a = 0; a < 3; ++a) {
            tq[a] = tau[3 * j + a] - gyro[a];
            if (rod->tau_ext) tq[a] += S(rod->tau_ext[3 * j + a]);
        }
        for (int a = 0; a < 3; ++a) wj[a] += S(dt) * (tq[a] / S(I[a]) - S(rod->damp_ang) * wj[a]);
    }
    double xc[3], qc[4], wc[3];
    if (rod->clamp) {
        oracle_clamp_pose(rod, t + dt, xc, qc, wc);
        for (int c = 0; c < 3; ++c) {
            v[c] = (S(xc[c]) - x[c]) / S(dt);
            w[c] = S(wc[c]);
        }
    }
    if (rod->inextensible)
        for (int it = 0; it < rod->n_iter; ++it)
            for (int parity = 0; parity < 2; ++parity)
                for (int j = parity; j < n; j += 2) project_segment(rod, j, x, v, winv.data());
    for (int i = 0; i <= n; ++i)
        for (int c = 0; c < 3; ++c) x[3 * i + c] += S(dt) * v[3 * i + c];
    for (int j = 0; j < n; ++j) {
        S* qj = q + 4 * j;
        S om[4] = {S(0.0), w[3 * j], w[3 * j + 1], w[3 * j + 2]};
        S dq[4];
        qmul(qj, om, dq);                                      /* dq/dt = 1/2 q (x) (0, omega) */
        S nq = S(0.0);
        for (int a = 0; a < 4; ++a) {
            qj[a] += S(0.5 * dt) * dq[a];
            nq += qj[a] * qj[a];
        }
        nq = sqrt(nq);
        for (int a = 0; a < 4; ++a) qj[a] /= nq;
    }
    if (rod->clamp) {
        for (int c = 0; c < 3; ++c) x[c] = S(xc[c]);
        for (int a = 0; a < 4; ++a) q[a] = S(qc[a]);
    }
}

inline size_t state_size(int n) { return (size_t)3 * (n + 1) * 2 + (size_t)4 * n + (size_t)3 * n; }

int32_t check(const oracle_rod* rod) {
    const int32_t rc = oracle_check(rod);
    if (rc != 0) return rc;
    if (rod->damp_int > 0.0) return -20;   // internal friction is not differentiated here
    return 0;
}

float to_f32(double a) { return (float)a; }

}  // namespace

extern "C" {

int32_t oracle_grad_rollout(const oracle_rod* rod, double t0, int32_t n_steps, double* x, double* v,
                            double* q, double* w, double* tip) {
    const int32_t rc = check(rod);
    if (rc != 0) return rc;
    const double one = 1.0;
    for (int s = 0; s < n_steps; ++s) {
        step<double>(rod, t0 + s * rod->dt, one, one, x, v, q, w);
        if (tip)
            for (int c = 0; c < 3; ++c) tip[3 * s + c] = x[3 * rod->n + c];
    }
    return 0;
}

int32_t oracle_jvp(const oracle_rod* rod, double t0, int32_t n_steps, const double* x,
                   const double* v, const double* q, const double* w, const double* dx,
                   const double* dv, const double* dq, const double* dw, double dmb, double dmt,
                   double* tip, double* dtip) {
    const int32_t rc = check(rod);
    if (rc != 0) return rc;
    const int n = rod->n;
    std::vector<Dual> X((size_t)3 * (n + 1)), Vv((size_t)3 * (n + 1)), Q((size_t)4 * n),
        Wv((size_t)3 * n);
    for (int i = 0; i < 3 * (n + 1); ++i) {
        X[i] = Dual(x[i], dx ? dx[i] : 0.0);
        Vv[i] = Dual(v[i], dv ? dv[i] : 0.0);
    }
    for (int i = 0; i < 4 * n; ++i) Q[i] = Dual(q[i], dq ? dq[i] : 0.0);
    for (int i = 0; i < 3 * n; ++i) Wv[i] = Dual(w[i], dw ? dw[i] : 0.0);
    const Dual mb(1.0, dmb), mt(1.0, dmt);
    for (int s = 0; s < n_steps; ++s) {
        step<Dual>(rod, t0 + s * rod->dt, mb, mt, X.data(), Vv.data(), Q.data(), Wv.data());
        for (int c = 0; c < 3; ++c) {
            if (tip) tip[3 * s + c] = X[3 * n + c].v;
            dtip[3 * s + c] = X[3 * n + c].d;
        }
    }
    return 0;
}

int32_t oracle_vjp(const oracle_rod* rod, double t0, int32_t n_steps, const double* x,
                   const double* v, const double* q, const double* w, const double* ct,
                   int32_t round_fp32, double* gx, double* gv, double* gq, double* gw,
                   double* gmb, double* gmt, double* tip) {
    const int32_t rc = check(rod);
    if (rc != 0) return rc;
    const int n = rod->n;
    const size_t nx = (size_t)3 * (n + 1), nqs = (size_t)4 * n, nw = (size_t)3 * n;
    const size_t ns = state_size(n);
    // forward: every step's start state, packed x | v | q | w
    std::vector<double> traj((size_t)(n_steps + 1) * ns);
    double* s0 = traj.data();
    std::memcpy(s0, x, nx * sizeof(double));
    std::memcpy(s0 + nx, v, nx * sizeof(double));
    std::memcpy(s0 + 2 * nx, q, nqs * sizeof(double));
    std::memcpy(s0 + 2 * nx + nqs, w, nw * sizeof(double));
    const double one = 1.0;
    for (int s = 0; s < n_steps; ++s) {
        double* a = traj.data() + (size_t)s * ns;
        double* b = a + ns;
        std::memcpy(b, a, ns * sizeof(double));
        step<double>(rod, t0 + s * rod->dt, one, one, b, b + nx, b + 2 * nx, b + 2 * nx + nqs);
        // the rounded replay: the fields of the state named by the bits of round_fp32 (1 x,
        // 2 v, 4 q, 8 w) are rounded to FP32 after every step (the rounding's derivative taken
        // as 1)
        if (round_fp32) {
            const size_t lo[4] = {0, nx, 2 * nx, 2 * nx + nqs};
            const size_t hi[4] = {nx, 2 * nx, 2 * nx + nqs, ns};
            for (int f = 0; f < 4; ++f)
                if (round_fp32 & (1 << f))
                    for (size_t k = lo[f]; k < hi[f]; ++k) b[k] = (double)to_f32(b[k]);
        }
        if (tip)
            for (int c = 0; c < 3; ++c) tip[3 * s + c] = b[3 * n + c];
    }
    // reverse, newest step first: lambda = dL/d(state at the end of the step)
    std::vector<double> lam(ns, 0.0);
    double amb = 0.0, amt = 0.0;
    Tape tape;
    g_tape = &tape;
    std::vector<Var> S(ns);
    std::vector<double> adj;
    for (int s = n_steps - 1; s >= 0; --s) {
        for (int c = 0; c < 3; ++c) lam[3 * n + c] += ct[3 * s + c];   // tip(s) = x_N after step s
        tape.clear();
        const double* a = traj.data() + (size_t)s * ns;
        for (size_t k = 0; k < ns; ++k) S[k] = leaf(a[k]);
        const Var mb = leaf(1.0), mt = leaf(1.0);
        std::vector<int32_t> in_idx(ns);
        for (size_t k = 0; k < ns; ++k) in_idx[k] = S[k].i;
        step<Var>(rod, t0 + s * rod->dt, mb, mt, S.data(), S.data() + nx, S.data() + 2 * nx,
                  S.data() + 2 * nx + nqs);
        adj.assign(tape.a.size(), 0.0);
        for (size_t k = 0; k < ns; ++k)
            if (S[k].i >= 0) adj[S[k].i] += lam[k];
        tape.sweep(adj);
        for (size_t k = 0; k < ns; ++k) lam[k] = adj[in_idx[k]];
        amb += adj[mb.i];
        amt += adj[mt.i];
    }
    g_tape = nullptr;
    std::memcpy(gx, lam.data(), nx * sizeof(double));
    std::memcpy(gv, lam.data() + nx, nx * sizeof(double));
    std::memcpy(gq, lam.data() + 2 * nx, nqs * sizeof(double));
    std::memcpy(gw, lam.data() + 2 * nx + nqs, nw * sizeof(double));
    *gmb = amb;
    *gmt = amt;
    return 0;
}

/* Many independent rods, spread over n_threads threads (0 = all hardware threads).  Arrays of
 * per-rod pointers; a NULL tip array skips the tips. */
int32_t oracle_vjp_many(int32_t n_rods, const oracle_rod* rods, double t0, int32_t n_steps,
                        const double* const* x, const double* const* v, const double* const* q,
                        const double* const* w, const double* const* ct, int32_t round_fp32,
                        double* const* gx, double* const* gv, double* const* gq,
                        double* const* gw, double* gmb, double* gmt, double* const* tip,
                        int32_t n_threads) {
    if (n_threads <= 0) n_threads = (int32_t)std::thread::hardware_concurrency();
    if (n_threads <= 0) n_threads = 1;
    std::vector<int32_t> rcs((size_t)n_rods, 0);
    std::vector<std::thread> pool;
    for (int32_t t = 0; t < n_threads; ++t)
        pool.emplace_back([&, t]() {
            for (int32_t r = t; r < n_rods; r += n_threads)
                rcs[r] = oracle_vjp(&rods[r], t0, n_steps, x[r], v[r], q[r], w[r], ct[r], round_fp32,
                                    gx[r], gv[r], gq[r], gw[r], &gmb[r], &gmt[r], tip ? tip[r] : nullptr);
        });
    for (auto& th : pool) th.join();
    for (int32_t r = 0; r < n_rods; ++r)
        if (rcs[r] != 0) return rcs[r];
    return 0;
}

/* Plain rollouts of many independent rods with the oracle's own oracle_rollout, spread over
 * n_threads threads (0 = all hardware threads). */
int32_t oracle_rollout_many(int32_t n_rods, const oracle_rod* rods, double t0, int32_t n_steps,
                            double* const* x, double* const* v, double* const* q, double* const* w,
                            int32_t n_threads) {
    if (n_threads <= 0) n_threads = (int32_t)std::thread::hardware_concurrency();
    if (n_threads <= 0) n_threads = 1;
    for (int32_t r = 0; r < n_rods; ++r)
        if (oracle_check(&rods[r]) != 0) return -1;
    std::vector<std::thread> pool;
    for (int32_t t = 0; t < n_threads; ++t)
        pool.emplace_back([&, t]() {
            for (int32_t r = t; r < n_rods; r += n_threads)
                oracle_rollout(&rods[r], t0, n_steps, x[r], v[r], q[r], w[r], nullptr);
        });
    for (auto& th : pool) th.join();
    return 0;
}

}  // extern "C"
