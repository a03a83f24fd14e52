/*
 * corde_oracle.h -- FP64 CPU oracle of the discrete CoRdE Cosserat rod stepper.
 *
 * TEST INFRASTRUCTURE ONLY.  This header and corde_oracle.c are the slow, plainly written
 * reference that the GPU library is checked against.  Only the test-suite, the package smoke
 * check and the CPU-baseline leg of the benchmark may build, load or call it.  It shares no
 * code, header, table or constant with the product library under paper_2509_04277_amd/.
 *
 * Model (Korzeniowski, Hald, Bello: "Massively-Parallel Implementation of Inextensible
 * Elastic Rods Using Inter-block GPU Synchronization", Sec. 2.1):
 *   - N elements (segments), N+1 mass points x_0..x_N, N material frames q_0..q_{N-1}
 *     stored as unit quaternions (w, x, y, z), Hamilton product, body -> world.
 *   - stretch energy, eq. (2), extensible variant only;
 *   - bend/twist energy, eq. (3), with the discrete Darboux vector of eqs. (5)-(6);
 *   - parallel-constraint penalty energy, eqs. (7)-(8);
 *   - inextensible variant: eq. (2) dropped, segment lengths enforced by iterative local
 *     velocity impulses (the J M^-1 J^T projection of Sec. 2.1, "Constraints");
 *   - time integration: forces -> velocities -> impulses -> positions, semi-implicit Euler
 *     (Sec. 2.1 last paragraph and the step loop of Fig. 5, without collision, self-collision
 *     and binding lines).
 *
 * Array layouts (all row-major, contiguous):
 *   x, v          : (N+1) x 3   world positions [m] and velocities [m/s]
 *   q             : N x 4       (w, x, y, z) unit quaternions, body -> world
 *   w (omega)     : N x 3       angular velocities in each frame's body axes [rad/s]
 *   seg_len, radius, young : N  per element rest length [m], radius [m], Young modulus [Pa]
 *   u_hat         : (N-1) x 3   intrinsic Darboux vector per joint [1/m] (NULL = zero)
 *   f_ext         : (N+1) x 3   constant external world force per point [N] (NULL = none)
 *   tau_ext       : N x 3       constant external body-frame torque per frame [N m] (NULL)
 */
#ifndef CORDE_ORACLE_H
#define CORDE_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct oracle_rod {
    int32_t n;             /* number of elements N >= 1 */
    int32_t inextensible;  /* 0: stretch energy eq. (2); 1: distance constraints */
    int32_t n_iter;        /* constraint iterations per step (inextensible only) */
    int32_t clamp;         /* 1: point 0 and frame 0 follow the prescribed clamp motion */
    double dt;             /* time step [s] */
    double gravity[3];     /* [m/s^2] */
    double damp_lin;       /* linear velocity damping gamma [1/s]: a -= gamma v */
    double damp_ang;       /* angular velocity damping [1/s]: alpha -= gamma omega */
    double poisson;        /* G = E / (2 (1 + nu)) */
    double density;        /* [kg/m^3] */
    double kp_scale;       /* K_p = kp_scale * G * pi r^2 */
    double bend_scale;     /* multiplies K_1 = K_2 (1 = E pi r^4 / 4) */
    double twist_scale;    /* multiplies K_3 (1 = G pi r^4 / 2) */
    const double* seg_len;
    const double* radius;
    const double* young;
    const double* u_hat;
    const double* f_ext;
    const double* tau_ext;
    /* clamp trajectory: x_c(t) = clamp_x0 + clamp_amp * sin(2 pi f t + phase_x);
     * q_c(t) = (cos(psi/2), sin(psi/2) axis) (x) clamp_q0, psi = twist_amp sin(2 pi f t + phase_tw) */
    double clamp_x0[3];
    double clamp_q0[4];
    double clamp_amp[3];
    double clamp_twist_amp;
    double clamp_twist_axis[3];
    double clamp_freq;
    double clamp_phase_x;
    double clamp_phase_twist;
    /* internal friction (Kelvin-Voigt): retardation time tau_d [s], 0 = none; the dissipation
     * function is the elastic energy's quadratic form at the strain rates (see
     * oracle_dissipation) */
    double damp_int;
} oracle_rod;

/* 0 if the description is usable, else a negative code. */
int32_t oracle_check(const oracle_rod* rod);

/* Total potential energy V(x, q): stretch (extensible only) + penalty + bend/twist
 * - sum_i M_i g . x_i - sum_i f_ext_i . x_i.  [J] */
double oracle_energy(const oracle_rod* rod, const double* x, const double* q);

/* Kinetic energy 1/2 sum M v^2 + 1/2 sum w^T I w over all points and frames. [J] */
double oracle_kinetic(const oracle_rod* rod, const double* v, const double* w);

/* Conservative forces F = -dV/dx on every point (includes gravity and f_ext), and body
 * torques tau_a = -1/2 (dV/dq) . (B_a q) on every frame (without tau_ext). */
void oracle_forces(const oracle_rod* rod, const double* x, const double* q,
                   double* F, double* tau);

/* Internal friction (the CoRdE dissipation terms, translational and angular), read as
 * Kelvin-Voigt: the Rayleigh dissipation function is the elastic energy's quadratic form at the
 * strain rates, D = sum_j 1/2 tau_d K_s l_j sdot_j^2 (extensible variant; s_j = |e_j|/l_j - 1)
 * + sum_joints 1/2 tau_d lbar sum_k K_k udot_k^2, udot the time derivative of eq. (6) under
 * dq/dt = 1/2 q (x) (0, omega).  oracle_damping_forces adds F = -dD/dv and body torques
 * tau = -dD/domega to F and tau (nothing if damp_int = 0). */
double oracle_dissipation(const oracle_rod* rod, const double* x, const double* q,
                          const double* v, const double* w);
void oracle_damping_forces(const oracle_rod* rod, const double* x, const double* q,
                           const double* v, const double* w, double* F, double* tau);

/* Discrete Darboux vector of joint j, eq. (6): u_k = (2 / lbar_j) (B_k q_j) . q_{j+1}. */
void oracle_darboux(const oracle_rod* rod, const double* q, int32_t j, double* u);

/* Prescribed clamp pose and body-frame angular rate at time t. */
void oracle_clamp_pose(const oracle_rod* rod, double t, double* xc, double* qc, double* wc);

/* One step from time t to t + dt, in place. */
void oracle_step(const oracle_rod* rod, double t, double* x, double* v, double* q, double* w);

/* One step like oracle_step that also returns the force the rod exerts on its base point 0
 * during the step (the force feedback of a haptic clamp, Sec. 2.2): the internal elastic
 * force on point 0 (element 0's stretch and penalty forces, eqs. (2), (8)) plus the impulses
 * of segment 0's distance constraints on point 0 summed over the iterations, divided by dt.
 * Gravity and the external load on point 0 itself are not part of it. */
void oracle_step_fb(const oracle_rod* rod, double t, double* x, double* v, double* q, double* w,
                    double* fbase);

/* n_steps of oracle_step_fb; fbase (n_steps x 3, nullable) receives every step's force. */
void oracle_rollout_fb(const oracle_rod* rod, double t0, int32_t n_steps, double* x, double* v,
                       double* q, double* w, double* fbase);

/* n_steps steps starting at time t0, in place.  If tip != NULL it receives x_N after every
 * step (n_steps x 3). */
void oracle_rollout(const oracle_rod* rod, double t0, int32_t n_steps,
                    double* x, double* v, double* q, double* w, double* tip);

/* oracle_rollout (no tips) with the state fields named by the bits of mask (1 x, 2 v, 4 q,
 * 8 w) rounded to FP32 after every step, FP64 arithmetic otherwise: the effect of storing
 * those fields in FP32 between steps (the floor against which FP32 results are judged). */
void oracle_rollout_rounded(const oracle_rod* rod, double t0, int32_t n_steps, double* x,
                            double* v, double* q, double* w, int32_t mask);

/* Same as oracle_rollout, on a private copy of the state, and returns 1 if every step is
 * stable: all values finite, max_j | |e_j| / l_j - 1 | < 0.5, and total energy
 * (kinetic + V) <= E_0 + (energy_factor - 1) |E_0| + 1e-9 J at every step (for E_0 > 0 this
 * is E <= energy_factor E_0 + 1e-9; the |E_0| form stays meaningful when the gravity
 * potential makes E_0 negative); 0 otherwise. */
int32_t oracle_stable(const oracle_rod* rod, double t0, int32_t n_steps,
                      const double* x, const double* v, const double* q, const double* w,
                      double energy_factor);

/* Time-step stability rule: 0.5 * min over elements and modes of 2 / omega_mode, with
 * omega from the axial (extensible only), penalty-shear, penalty-rotation, bending and
 * twisting one-element modes. */
double oracle_dt_rule(const oracle_rod* rod);

/* Largest relative segment-length error max_j | |x_{j+1} - x_j| / l_j - 1 |. */
double oracle_max_strain(const oracle_rod* rod, const double* x);

/* The constant skew-symmetric matrix B_k (k = 0, 1, 2), row-major 4x4, of eq. (6). */
void oracle_bmat(int32_t k, double* out16);

/* Rotation matrix R(q), row-major 3x3, body -> world: column k is director d_{k+1}. */
void oracle_rotmat(const double* q, double* out9);

/* Hamilton product r = a (x) b of (w, x, y, z) quaternions. */
void oracle_qmul(const double* a, const double* b, double* r);

/* ---- Binding constraints between two rods (Sec. 2.1 "Constraints"; Sec. 3.4 variants) ----
 * Distance constraints of rest length zero between point point_a[k] of rod a and point
 * point_b[k] of rod b, solved as velocity impulses after the distance constraints in every
 * constraint iteration (Fig. 5).  one_way = 1: rod b is the master instrument and is not moved
 * by the bindings (variant 1); 0: both rods respond by their inverse masses (variant 2). */
typedef struct {
    int32_t n_pairs;
    const int32_t* point_a;   /* point indices 0..n of rod a */
    const int32_t* point_b;   /* point indices 0..n of rod b */
    int32_t one_way;
} oracle_binding;

/* One binding impulse between point a (position xa, velocity va, inverse mass wa) and point b:
 * d = (xa + dt va) - (xb + dt vb), lambda = |d| / (dt (wa + wb)) (wa alone if one_way), and
 * va -= wa lambda d/|d|, vb += wb lambda d/|d| (vb unchanged if one_way). */
void oracle_bind_impulse(const double* xa, double* va, double wa, const double* xb, double* vb,
                         double wb, double dt, int32_t one_way);

/* One step of two bound rods from time t, in place.  Both rods step with a's dt and a's number
 * of constraint iterations (the caller gives them equal dt and n_iter). */
void oracle_step_pair(const oracle_rod* a, const oracle_rod* b, const oracle_binding* bind,
                      double t, double* xa, double* va, double* qa, double* wa, double* xb,
                      double* vb, double* qb, double* wb);

/* ---- Contact (Sec. 2.2 "Collisions and self-collisions"; Sec. 2.1 "Constraints") -------
 * Every point 1..n carries a sphere of its element's radius (the mean of its two elements'
 * at interior points).  Two points are in contact when their spheres overlap at the start of
 * the step (points of one rod only if they are more than oracle_self_skip() apart along it,
 * so resting neighbours never count); the contact keeps that normal n (from the other point
 * towards this one) and target distance D = sum of the radii for the step.  In every
 * constraint iteration, after the distance constraints and bindings, every point computes the
 * impulse of each of its contacts from the same velocities: a normal impulse removing the
 * predicted penetration, lambda = -s / (dt (w_i + w_j)) with s = (p_i - p_j) . n - D < 0,
 * p = x + dt v, and a Coulomb friction impulse opposing the relative tangential velocity,
 * at most mu lambda; the point applies the mean of its active contacts' impulses. */
typedef struct {
    double mu;   /* friction coefficient */
} oracle_contact;

/* Index distance along one rod within which points never collide: ceil(2 r_max / l_min), at
 * least 1. */
int32_t oracle_self_skip(const oracle_rod* rod);

/* One step of a group of 1 or 2 rods (bindings need 2; either may be NULL), from time t, in
 * place; x[r], v[r], q[r], w[r] are rod r's arrays.  All rods step with rods[0]'s dt and
 * number of constraint iterations.  max_contacts (nullable) receives the largest number of
 * contacts of one point. */
void oracle_step_group(const oracle_rod* const* rods, int32_t n_rods, const oracle_binding* bind,
                       const oracle_contact* contact, double t, double* const* x, double* const* v,
                       double* const* q, double* const* w, int32_t* max_contacts);

/* oracle_rollout_group with every rod's state fields named by mask (as for
 * oracle_rollout_rounded) rounded to FP32 after every step. */
void oracle_rollout_group_rounded(const oracle_rod* const* rods, int32_t n_rods,
                                  const oracle_binding* bind, const oracle_contact* contact,
                                  double t0, int32_t n_steps, double* const* x,
                                  double* const* v, double* const* q, double* const* w,
                                  int32_t mask, int32_t* max_contacts);

/* n_steps of oracle_step_group from time t0; max_contacts over all steps. */
void oracle_rollout_group(const oracle_rod* const* rods, int32_t n_rods,
                          const oracle_binding* bind, const oracle_contact* contact, double t0,
                          int32_t n_steps, double* const* x, double* const* v, double* const* q,
                          double* const* w, int32_t* max_contacts);

/* ---- Environment collision (Sec. 2.2 "Collisions") ------------------------------------
 * A static triangle mesh; each triangle's face normal (b - a) x (c - a), normalised, points to
 * the side the rods are on.  At the start of a step every point 1..n (sphere of its element's
 * radius r, as for contact) collides with every triangle whose nearest point lies closer than
 * r; per colliding triangle the penetration depth is r - dist (centre in front of the face) or
 * r + dist (centre behind it).  The point's response is n = normalise(sum_k depth_k N_k), the
 * depth-weighted mean of the colliding triangles' normals, with depth = max_k depth_k.  In
 * every constraint iteration, after the distance constraints, a colliding point whose
 * predicted motion along n falls short of the depth, s = dt v . n - depth < 0, takes the
 * impulse lambda = -s / (dt w) along n (the mesh does not move) and a Coulomb friction impulse
 * against its tangential velocity, at most mu lambda.  A rod without constraint iterations
 * (the extensible variant) takes the response once per step. */
typedef struct {
    int32_t n_tris;
    const double* tris;   /* n_tris x 9: vertices a, b, c */
    double mu;            /* friction coefficient */
} oracle_env;

/* Nearest point of triangle tri (9 values: a, b, c) to p. */
void oracle_closest_point_triangle(const double* p, const double* tri, double* out);

/* Response of a sphere (centre c, radius r) against the mesh: unit n, depth (0 with n = 0 if
 * it touches nothing or the normals cancel), hits = colliding triangles (nullable). */
void oracle_env_response(const oracle_env* env, const double* c, double r, double* n,
                         double* depth, int32_t* hits);

/* The collision impulse of one point (inverse mass winv) on its velocity v, in place. */
void oracle_env_impulse(const double* n, double depth, double winv, double dt, double mu,
                        double* v);

/* One step of one rod against the mesh, from time t, in place; colliding (nullable) receives
 * the number of colliding points. */
void oracle_step_env(const oracle_rod* rod, const oracle_env* env, double t, double* x, double* v,
                     double* q, double* w, int32_t* colliding);

/* n_steps of oracle_step_env from time t0; most = the largest number of colliding points. */
void oracle_rollout_env(const oracle_rod* rod, const oracle_env* env, double t0, int32_t n_steps,
                        double* x, double* v, double* q, double* w, int32_t* most);

/* n_steps of oracle_step_pair starting at time t0, in place. */
void oracle_rollout_pair(const oracle_rod* a, const oracle_rod* b, const oracle_binding* bind,
                         double t0, int32_t n_steps, double* xa, double* va, double* qa, double* wa,
                         double* xb, double* vb, double* qb, double* wb);


/* ---- Reference derivatives (corde_oracle_grad.cpp, C++) --------------------------------
 * Derivatives of the tip trajectory tip(s) = x_N after step s (s = 0 .. n_steps-1) of a
 * rollout of the plain step from time t0, with respect to the initial state (x, v, q, w; q by
 * its four stored components) and the multipliers m_b of K_1 = K_2 and m_t of K_3 (eq. (3)),
 * taken at m_b = m_t = 1.  Rods with internal friction are refused (nonzero return); 0 = done. */

/* The rollout through the templated restatement of the step in corde_oracle_grad.cpp,
 * evaluated in plain doubles; it must equal oracle_rollout bitwise.  tip nullable. */
int32_t oracle_grad_rollout(const oracle_rod* rod, double t0, int32_t n_steps, double* x,
                            double* v, double* q, double* w, double* tip);

/* Forward mode: tip (nullable, n_steps x 3) and its directional derivative dtip (n_steps x 3)
 * along the initial-state direction (dx, dv, dq, dw; each nullable = 0) and multiplier
 * direction (dmb, dmt). */
int32_t oracle_jvp(const oracle_rod* rod, double t0, int32_t n_steps, const double* x,
                   const double* v, const double* q, const double* w, const double* dx,
                   const double* dv, const double* dq, const double* dw, double dmb, double dmt,
                   double* tip, double* dtip);

/* Reverse mode: for the cotangent ct (n_steps x 3) the gradient of L = sum_s ct[s] . tip(s):
 * gx, gv ((N+1) x 3), gq (N x 4), gw (N x 3), gmb, gmt.  round_fp32 = 1 rounds the stored state
 * to FP32 after every step of the forward pass (the rounding's derivative taken as 1): the
 * gradient of an FP32-storage trajectory.  tip (nullable) receives the forward trajectory. */
int32_t oracle_vjp(const oracle_rod* rod, double t0, int32_t n_steps, const double* x,
                   const double* v, const double* q, const double* w, const double* ct,
                   int32_t round_fp32, double* gx, double* gv, double* gq, double* gw,
                   double* gmb, double* gmt, double* tip);

/* oracle_vjp for n_rods independent rods on n_threads threads (0 = all hardware threads);
 * per-rod pointer arrays; tip nullable. */
int32_t oracle_vjp_many(int32_t n_rods, const oracle_rod* rods, double t0, int32_t n_steps,
                        const double* const* x, const double* const* v, const double* const* q,
                        const double* const* w, const double* const* ct, int32_t round_fp32,
                        double* const* gx, double* const* gv, double* const* gq,
                        double* const* gw, double* gmb, double* gmt, double* const* tip,
                        int32_t n_threads);

/* oracle_rollout of n_rods independent rods (in place, no tips) on n_threads threads
 * (0 = all hardware threads). */
int32_t oracle_rollout_many(int32_t n_rods, const oracle_rod* rods, double t0, int32_t n_steps,
                            double* const* x, double* const* v, double* const* q,
                            double* const* w, int32_t n_threads);

#ifdef __cplusplus
}
#endif

#endif
