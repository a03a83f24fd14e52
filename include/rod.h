/*
 * rod.h -- C ABI of the MI355X (gfx950) CoRdE Cosserat-rod stepper, libcorde_rod.so.
 *
 * Method: Korzeniowski, Hald, Bello, "Massively-Parallel Implementation of Inextensible
 * Elastic Rods Using Inter-block GPU Synchronization".
 *   - Model: discrete Cosserat rod of Sec. 2.1 -- N elements, N+1 mass points, N material
 *     frames as unit quaternions; stretch energy eq. (2) (extensible variant), bend/twist
 *     energy eq. (3) with the discrete Darboux vector of eqs. (5)-(6), parallel-constraint
 *     penalty eqs. (7)-(8); the inextensible variant drops eq. (2) and enforces segment
 *     lengths with iterative local velocity impulses (J M^-1 J^T projection, Sec. 2.1
 *     "Constraints").
 *   - Step (Sec. 2.1 last paragraph, Fig. 5 without collision/self-collision/binding):
 *     external + elastic forces and torques -> integrate forces -> n_iter constraint
 *     iterations -> integrate velocities (semi-implicit Euler), quaternion renormalisation.
 *   - The paper's kernel takes the number of time-steps, the number of constraint
 *     iterations, material properties and the user input (Sec. 2.2): rod_step() takes the
 *     step count, the handle carries the rest; rod_set_clamp() is the user (haptic) input.
 *
 * Conventions
 *   - Every call returns a rod_status; ROD_OK == 0, errors are negative.  No C++ exception
 *     crosses the ABI.  On error, output buffers are left untouched and rod_last_error()
 *     describes the failure.
 *   - A handle (rod_ctx) holds R >= 1 independent rods ("batch"); all its device memory is
 *     owned by the library and freed by rod_destroy().  Caller buffers are never retained.
 *   - State layout, concatenated over the rods of a handle in rod order (FP32, row-major):
 *       x, v : sum_r (N_r + 1) x 3     point positions [m] / velocities [m/s], world axes
 *       q    : sum_r N_r x 4           frame quaternions (w, x, y, z), body -> world
 *       w    : sum_r N_r x 3           frame angular velocities in body axes [rad/s]
 *   - on_device = 1: pointers are device pointers on the handle's device (e.g. a torch
 *     tensor's data_ptr()); the copy is enqueued on the handle's stream and the call returns
 *     without waiting.  on_device = 0: host pointers; the call synchronises the stream.
 *   - All work is enqueued on the HIP stream given at creation (NULL = default stream) and is
 *     stream-ordered.  Calls on one handle must not be made concurrently from two threads.
 *   - A handle lives on the device that is current at rod_create (its stream must belong to
 *     it); later calls must be made with that device current (rod_step: ROD_E_DEVICE if not).
 *   - Non-finite state seen by a kernel is latched on the device; the next call that
 *     synchronises (rod_sync, host rod_get_state) returns ROD_E_UNSTABLE.
 */
#ifndef CORDE_ROD_H
#define CORDE_ROD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rod_status {
    ROD_OK = 0,
    ROD_E_INVALID = -1,     /* bad argument (null pointer, size, value out of range) */
    ROD_E_NOMEM = -2,       /* device or host allocation failed */
    ROD_E_DEVICE = -3,      /* a HIP call failed */
    ROD_E_UNSTABLE = -4,    /* a kernel saw a non-finite state value */
    ROD_E_ORDER = -5,       /* call made in the wrong order */
    ROD_E_UNSUPPORTED = -6, /* valid request this build cannot run */
    ROD_E_TIMEOUT = -7      /* a long-rod workgroup waited too long for a neighbour */
} rod_status;

/* Description of one rod, SI units.  Arrays are read during rod_create() only. */
typedef struct rod_params {
    int32_t n_elements;          /* N >= 1: N+1 points, N frames */
    int32_t inextensible;        /* 0: stretch energy eq. (2); 1: distance impulses */
    int32_t n_constraint_iters;  /* iterations per step (inextensible only, paper: 10) */
    int32_t clamp_end0;          /* 1: point 0 and frame 0 follow the clamp trajectory */
    double dt;                   /* time step [s] > 0 */
    double gravity[3];           /* [m/s^2] */
    double damping_lin;          /* gamma [1/s]: acceleration -= gamma * v */
    double damping_ang;          /* [1/s]: angular acceleration -= gamma * omega */
    double poisson;              /* nu, G = E / (2 (1 + nu)) */
    double density;              /* rho [kg/m^3] */
    double kp_scale;             /* penalty eq. (8): K_p = kp_scale * G * pi r^2 */
    double bend_scale;           /* K_1 = K_2 = bend_scale * E * pi r^4 / 4, eq. (3) */
    double twist_scale;          /* K_3 = twist_scale * G * pi r^4 / 2, eq. (3) */
    const double* seg_len;       /* [N] rest length of each element [m] (required) */
    const double* radius;        /* [N] cross-section radius [m] (required) */
    const double* young;         /* [N] Young modulus [Pa] (required) */
    const double* u_hat;         /* [(N-1) x 3] intrinsic Darboux vector per joint, or NULL */
    const double* f_ext;         /* [(N+1) x 3] constant world force per point [N], or NULL */
    const double* tau_ext;       /* [N x 3] constant body torque per frame [N m], or NULL */
    /* clamp trajectory (used when clamp_end0 = 1):
     *   x_c(t) = clamp_x0 + clamp_amp * sin(2 pi f t + phase_x)
     *   q_c(t) = (cos(psi/2), sin(psi/2) axis) (x) clamp_q0,  psi = twist_amp sin(2 pi f t + phase_tw) */
    double clamp_x0[3];
    double clamp_q0[4];
    double clamp_amp[3];
    double clamp_twist_amp;
    double clamp_twist_axis[3];
    double clamp_freq;
    double clamp_phase_x;
    double clamp_phase_twist;
    /* Internal friction (Sec. 2.1: the CoRdE dissipation terms damping relative motion,
     * translational and angular), Kelvin-Voigt: retardation time tau_d [s] >= 0.  Element j's
     * stretch force uses (len - l) + tau_d d(len)/dt (extensible variant), joint k's bend/twist
     * moment K (u - u_hat + tau_d du/dt); du/dt follows from the frames' angular velocities.
     * 0 = none.  rod_stable_dt also keeps tau_d omega^2 dt <= 2 on the damped modes.  Rods
     * with internal friction step in a variant of the one-rod-per-workgroup kernel only:
     * rod_create refuses them above the chunking threshold, rod_set_bindings and
     * rod_set_contact refuse to group them, rod_set_environment refuses handles holding them,
     * and the adjoint refuses them (ROD_E_UNSUPPORTED). */
    double damping_int;
} rod_params;

typedef struct rod_ctx rod_ctx;

/* Kernel shape used for a handle: waves per workgroup and elements per lane. */
typedef struct rod_tuning {
    int32_t waves;            /* wavefronts (64 lanes) per rod */
    int32_t elems_per_lane;   /* consecutive elements held in each lane's registers */
    int32_t steps_per_launch; /* time steps run inside one kernel launch */
    float us_per_step;        /* measured device time per step (autotune), else 0 */
} rod_tuning;

/* Create a handle for n_rods rods described by params[0..n_rods-1] on the current HIP device,
 * enqueuing work on hip_stream (a hipStream_t, NULL = default).  Derives all per-element
 * coefficients (masses, inertias, stiffnesses of eqs. (2), (3), (8)) in FP64 on the host.
 * Rods of up to 2048 elements are stepped by one workgroup each; longer rods are split into
 * chunks of up to about 500 elements, one workgroup per chunk, that exchange halos once every
 * few steps (see rod_set_chunking)
 * (all chunks of a handle must be resident on the device at once: ROD_E_UNSUPPORTED if not,
 * and for any rod longer than 131072 elements).
 * The state is zero until rod_set_state().  Errors: INVALID (bad sizes/values), NOMEM,
 * DEVICE, UNSUPPORTED. */
rod_status rod_create(const rod_params* params, int32_t n_rods, void* hip_stream, rod_ctx** out);

/* Free all device and host memory of the handle (after finishing its stream's work). */
rod_status rod_destroy(rod_ctx* ctx);

/* Copy a full state in (layouts above): the arrays the paper uploads once at initialisation
 * (Sec. 2.2).  Resets the simulation time to t0 [s].  Inside the handle, positions and
 * quaternions are kept as pairs of floats (value + a low part below half its ulp) so that
 * the small per-step increments are not rounded away; this call sets the low parts to 0. */
rod_status rod_set_state(rod_ctx* ctx, const float* x, const float* v, const float* q,
                         const float* w, int32_t on_device, double t0);

/* Copy the full state out into caller-owned buffers (any pointer may be NULL to skip): the
 * positions the paper reads back for rendering every launch (Sec. 2.2, Sec. 3.1).  x and q
 * are the FP32 values nearest to the handle's pairs; a get / set round trip therefore rounds
 * them once (a resumed run differs from a straight one by that rounding). */
rod_status rod_get_state(rod_ctx* ctx, float* x, float* v, float* q, float* w, int32_t on_device);

/* Advance every rod by n_steps time steps (Sec. 2.1 last paragraph; Fig. 5 without its
 * collision lines unless a mesh, contact or bindings are set), steps_per_launch steps per
 * kernel launch (0 = the handle's tuned value; the paper runs several time steps per kernel
 * launch, Sec. 2.2).  Each launch loads the state once, keeps it in registers across its
 * steps and stores it once. */
rod_status rod_step(rod_ctx* ctx, int32_t n_steps, int32_t steps_per_launch);

/* Override the static clamp pose of rod `rod` (haptic input, Sec. 2.2); takes effect at the
 * next step.  x0[3], q0[4] as in rod_params; the sinusoidal amplitudes are kept. */
rod_status rod_set_clamp(rod_ctx* ctx, int32_t rod, const double* x0, const double* q0);

/* Wait for the handle's stream (the calls above are stream-ordered and return before the
 * device finishes; their device-side conditions surface here): ROD_E_UNSTABLE if a non-finite
 * state was seen, ROD_E_TIMEOUT if chunked long-rod workgroups lost step synchronisation,
 * ROD_E_UNSUPPORTED if a point had more contacts than the kernel holds (the conditions stay
 * latched until the next rod_set_state). */
rod_status rod_sync(rod_ctx* ctx);

/* Simulation time [s] and number of steps taken since rod_set_state(). */
rod_status rod_get_time(const rod_ctx* ctx, double* t, int64_t* steps);

/* Rods of a handle are grouped into buckets that share one kernel shape (by default the
 * smallest shape that holds each rod); rod_step() launches every bucket per chunk of steps.
 * Rods longer than 2048 elements form one last bucket stepped by the chunked kernel (shape
 * 4 waves x 2 elements per lane per chunk), which tuning does not change.
 * rod_set_tuning() puts all other rods into one bucket of the given shape (waves in
 * {1,2,4,8,16}, elems_per_lane in {1,2,4,8} as built; ROD_E_UNSUPPORTED if not built or too
 * small for the longest of them).  rod_get_tuning() reports the first bucket's shape and the
 * summed per-step time of the buckets measured by rod_autotune(). */
rod_status rod_set_tuning(rod_ctx* ctx, const rod_tuning* t);
rod_status rod_get_tuning(const rod_ctx* ctx, rod_tuning* t);

/* Shape, measured time (0 if not measured) and rod count of bucket `bucket` (0-based; the
 * bound-pair buckets follow the single-rod ones, and the long-rod bucket, if any, is last;
 * a pair bucket's shape is per rod); ROD_E_INVALID past the end. */
rod_status rod_bucket_info(const rod_ctx* ctx, int32_t bucket, rod_tuning* t, int32_t* n_rods);

/* Step every rod longer than min_elements (1..2048; default 2048) with the chunked long-rod
 * kernel: one workgroup per chunk, neighbouring chunks trading H = T (2 n_constraint_iters + 2)
 * + 2 (rounded up to even) halo elements per side once every T steps, so a rod of up to 2048
 * elements can also be spread over several compute units.  T (1..16) is the largest for which
 * each halo takes at most a quarter of a 512-element window, 2 H + 2 <= chunk_elements (if
 * set) and the rod needs at most one chunk per compute unit.  chunk_elements sets the owned
 * elements per chunk (0 = the most a 512-element window holds, 512 - 2 H; otherwise clamped to
 * [2 H + 2, 512 - 2 H]; chunk sizes are even and about equal).  The other rods return to their
 * default shapes (as after rod_create).  A held adjoint rollout is dropped if any rod ends up
 * chunked.  All chunks of a handle must be resident on the device together: the handle's
 * chunked steps run after those of any other handle of the process on the same device (stream
 * order through one event per device), and a chunk whose neighbour does not arrive gives up
 * after a bounded wait (rod_sync then reports ROD_E_TIMEOUT), for instance when another
 * process holds the compute units.  Errors: INVALID, UNSUPPORTED (too many constraint
 * iterations to split a rod, or more chunks than the device holds at once; the default split
 * is then restored), DEVICE. */
rod_status rod_set_chunking(rod_ctx* ctx, int32_t min_elements, int32_t chunk_elements);

/* ---- Binding constraints (Sec. 2.1 "Constraints"; Sec. 3.4 variants 1 and 2) ----------
 * Bind point pairs of two rods with distance constraints of rest length zero, solved as
 * velocity impulses after the distance constraints of every constraint iteration (Fig. 5).
 * pairs: n_pairs x 4 int32 (rod_a, point_a, rod_b, point_b), points 1..n (the base point 0 is
 * not bindable); every point at most once; a rod may be bound to one other rod only.
 * mode 1 = one-way (rod_b is the master and is not moved; all pairs of two rods must name the
 * same master), 2 = two-way (both rods respond by their inverse masses).  n_pairs = 0 removes
 * all bindings.  Bound rods must be inextensible with equal n_constraint_iters and dt and at
 * most 1024 elements; each bound pair is stepped by one workgroup (the two rods exchange
 * their points through LDS).  Replaces earlier bindings; takes effect at the next rod_step.
 * The adjoint refuses handles with bound rods.  Errors: INVALID, UNSUPPORTED, NOMEM, DEVICE. */
rod_status rod_set_bindings(rod_ctx* ctx, int32_t n_pairs, const int32_t* pairs, int32_t mode);

/* ---- Contact (Sec. 2.2 "Collisions and self-collisions"; Sec. 2.1 contact constraints) ---
 * sets: n_sets x 2 int32 (rod_a, rod_b), rod_b = -1 for a rod alone: the points of the set's
 * rods touch each other and themselves.  Every point 1..n carries a sphere of its element's
 * radius (the mean of its two elements' radii inside the rod); at the start of each step,
 * points whose spheres overlap are in contact (points of one rod only if more than
 * ceil(2 r_max / l_min) apart along it) with the step-start normal and the sum of the radii as
 * target distance; every constraint iteration, after the distance constraints and bindings,
 * each point applies the mean of its active contacts' impulses: one removing the predicted
 * penetration and a Coulomb friction impulse (coefficient mu) opposing the relative tangential
 * velocity.  A set's rods share one workgroup (with a bound pair: the same two rods); they
 * must be inextensible with equal dt and n_constraint_iters, at most 512 elements each, and
 * a point may have at most 8 contacts (more: rod_sync reports ROD_E_UNSUPPORTED).  The first
 * call with contact allocates 48 bytes per element of the handle for per-point candidate lists
 * (pairs within contact distance + half the largest radius of the set), which the kernel keeps
 * between launches and rebuilds only when a point has moved far enough to need it; the
 * contacts found are those of a check of all point pairs.  n_sets = 0 removes all contact
 * sets.  Errors: INVALID, UNSUPPORTED, NOMEM, DEVICE. */
rod_status rod_set_contact(rod_ctx* ctx, int32_t n_sets, const int32_t* sets, double mu);

/* ---- Environment collision (Sec. 2.2 "Collisions"; Sec. 2.1 contact constraints) --------
 * A static triangle mesh that every rod of the handle collides with.  tris: n_tris x 9
 * doubles, the vertices a, b, c of each triangle; the face normal (b - a) x (c - a) points to
 * the side the rods are on (into the lumen of a vessel).  Degenerate triangles are dropped.
 * The library builds an AABB tree over them by volume partitioning (leaves of at most 2
 * triangles) and copies it to the device.  At the start of every step each point 1..n (a
 * sphere of its element's radius, as for contact) finds the triangles whose nearest point is
 * closer than its radius; each has a depth, radius - distance (centre in front of the face) or
 * radius + distance (behind it); the point's response is the depth-weighted mean of their face
 * normals, normalised, with the largest depth.  In every constraint iteration, after the
 * distance constraints, a colliding point whose predicted motion along that normal falls
 * short of the depth is pushed out by a velocity impulse, with Coulomb friction (coefficient
 * mu) against its tangential velocity; rods without constraint iterations take the response
 * once per step.  n_tris = 0 removes the mesh.  Rods collide in kernel variants of their own
 * (default shapes only, as for the haptic mailbox).  Grouped (bound, contact) and chunked rods
 * do not collide: with any, this returns ROD_E_UNSUPPORTED, and so do rod_set_bindings,
 * rod_set_contact, rod_set_chunking and the adjoint while a mesh is set.
 * Errors: INVALID, UNSUPPORTED, NOMEM, DEVICE. */
rod_status rod_set_environment(rod_ctx* ctx, int32_t n_tris, const double* tris, double mu);

/* Size of the environment's tree: nodes and (non-degenerate) triangles, 0 without a mesh. */
rod_status rod_environment_info(const rod_ctx* ctx, int32_t* n_nodes, int32_t* n_tris);

/* ---- Haptic mailbox (Sec. 2.2: the haptic thread hands a new device position to the
 * running simulation and reads its force-feedback vector at any time, at 0.5-1 kHz) ---------
 * rod_haptic_attach() gives rod `rod` a mailbox in pinned host memory that its kernel reads
 * and writes while it runs, so the pose and force calls below never wait for a launch and make
 * no GPU call.  The kernel works in windows of steps_per_record (>= 1) steps, counted from the
 * first step of each launch (a launch's last window may be shorter): at the clamp of a window's
 * first step it takes the newest whole pose; after its last step it writes one force record,
 * the mean over the window.  The rod must be clamped with a static clamp (clamp_amp and
 * clamp_twist_amp 0 or clamp_freq 0) and stepped by the one-rod-per-workgroup kernel: not
 * bound, in a contact set or chunked (those calls then return ROD_E_UNSUPPORTED, and so does
 * the adjoint).  Rods with a mailbox step in buckets of their own, with a kernel variant that
 * holds the mailbox code (shapes (1,1), (1,2), (2,2), (4,2), (4,4), (4,8), (8,4); a tuned shape
 * without it falls back to the default shape).  Attaching again only changes steps_per_record.
 * Errors: INVALID (rod index, unclamped rod, steps_per_record), UNSUPPORTED, NOMEM, DEVICE.
 * rod_haptic_detach() waits for the handle's kernels and frees the mailbox (no-op without). */
rod_status rod_haptic_attach(rod_ctx* ctx, int32_t rod, int32_t steps_per_record);
rod_status rod_haptic_detach(rod_ctx* ctx, int32_t rod);

/* New clamp pose of rod `rod`: x0[3] [m], q0[4] (w, x, y, z; must have unit norm within 1e-6,
 * normalised here).  Taken at the start of the next window (of a running launch, or of the
 * next launch); a read that overlaps this write keeps the previous pose for one more window.
 * Every launch re-applies the newest pose at its first step.  Once a pose is set, it replaces
 * the pose of rod_set_clamp().  Poses are numbered 1, 2, ... per rod.  rod_step() returns
 * before its launches end: a pose set afterwards may be taken by them.  May be called from
 * another thread while the handle's owner steps it; one caller per rod.
 * Errors: INVALID, ORDER (no mailbox). */
rod_status rod_haptic_set_pose(rod_ctx* ctx, int32_t rod, const double* x0, const double* q0);

typedef struct {
  double f[3];        /* [N] mean force of the rod on its clamped base point over the window */
  uint32_t step;      /* steps taken when the window ended (low 32 bits of the step count;
                         0 with f = 0 before the first window after attaching) */
  uint32_t pose;      /* number of the pose in use in the window (0: the rod_set_clamp pose) */
  uint32_t n_steps;   /* steps in the window */
} rod_haptic_force;

/* Newest force record of rod `rod`.  The force on the base over one step is the internal
 * (stretch and penalty) force of element 0 on point 0 plus the impulses of the distance
 * constraint of element 0 on point 0, summed over the constraint iterations, divided by dt;
 * gravity and the external load of point 0 are not included.  The record holds its mean over
 * the window (the momentum passed to the base divided by the window's duration).  Thread rules
 * as for rod_haptic_set_pose().  Errors: INVALID, ORDER (no mailbox), TIMEOUT (no whole record
 * read in 2^20 attempts). */
rod_status rod_haptic_get_force(rod_ctx* ctx, int32_t rod, rod_haptic_force* out);

/* The autotuner of the batched form (kernel shape per bucket and steps per launch picked by
 * measuring; the paper fixes them by hand, Sec. 3.1).
 * Per bucket, time every built shape that holds its longest rod on probe_steps steps (the
 * state is saved and restored, the step counter unchanged) and keep the fastest, or a shape
 * that another bucket keeps if it is within 2 % of the fastest (the buckets then share one
 * launch); sets the handle's steps_per_launch.  steps_per_launch = 0: first, while the long-rod split is the
 * default one, the whole handle is timed with its rods of more than 512 elements in one
 * workgroup each and chunked as by rod_set_chunking(ctx, 512, 0), and the faster split is kept
 * (a chunked rod is not differentiated by the adjoint); then the shapes are timed at 10 steps
 * per launch, then the whole handle at 1, 2, 5, 10, 20, 50, ..., 1000 steps per launch (up to
 * probe_steps), and the smallest that comes within 5 % of the best time per step is kept.  Rods with a haptic
 * mailbox read its pose and write force records during the probes.  out (nullable) receives
 * rod_get_tuning(). */
rod_status rod_autotune(rod_ctx* ctx, int32_t probe_steps, int32_t steps_per_launch,
                        rod_tuning* out);

/* Stability rule for one rod: 0.5 * min over elements and one-element modes (axial for the
 * extensible variant, penalty shear, penalty rotation, bending, twisting) of 2 / omega. */
rod_status rod_stable_dt(const rod_params* p, double* dt_out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): rod_step on caller-owned state instead of the
 * handle's.  x, v, q, w are device arrays on the handle's device in the handle's layout (as for
 * rod_set_state with on_device = 1), read and written in place; the handle's own state, step
 * counter and tuning are left as they are.  Steps are numbered from first_step (a driven
 * clamp is evaluated at t0 + (first_step + s + 1) dt, t0 from the last rod_set_state, else 0).
 * Positions and quaternions are compensated within the call only (their low parts start at 0
 * and are dropped at its end), so a run split over several calls rounds them to FP32 at each
 * call's end; one call gives bitwise the state of rod_set_state + rod_step from the same state
 * and time.  steps_per_launch = 0 uses the handle's.  The call allocates nothing and creates no
 * stream: its one scratch buffer (those low parts, 3 floats per point and 4 per frame) is a
 * fixed array in device memory that each GPU holds from the first rod_create on it until the
 * process ends (56 MiB); every bucket steps on the handle's stream.  Calls on one GPU share that array, so
 * calls that overlap on one GPU (other streams, other threads) race: order them.  Stream-
 * ordered like rod_step; a non-finite state is reported by rod_sync.  Errors: INVALID (null
 * pointer, negative count, more than 2^21 points), UNSUPPORTED (handles with chunked rods,
 * bindings, contact, a haptic mailbox or an environment), DEVICE. */
rod_status rod_step_state_noalloc(rod_ctx* ctx, float* x, float* v, float* q, float* w,
                                  int64_t first_step, int32_t n_steps, int32_t steps_per_launch);

/* Device time of the last rod_step() call measured with HIP events on the handle's stream
 * [ms], and the number of kernel launches it made. */
rod_status rod_last_step_time(rod_ctx* ctx, float* ms, int32_t* launches);

/* ---- Adjoint (reverse-mode gradients of a rollout) ------------------------------------
 * Differentiates the rollout of rod_step() with respect to the per-rod multipliers of the
 * bend stiffness (K_1 = K_2 of eq. (3)) and twist stiffness (K_3), and the initial state.
 * The loss is any function of the tip trajectory tip(s) = x_N after step s; the caller passes
 * dL/dtip.  Supported: at most 10 constraint iterations, rods of at most 512 elements. */

/* Set the stiffness multipliers m_b[r], m_t[r] >= 0 (host arrays of n_rods; default 1).
 * Invalidates a recorded adjoint rollout. */
rod_status rod_set_stiffness_mult(rod_ctx* ctx, const float* bend, const float* twist);

/* Advance every rod by n_steps steps from the current state (like rod_step), recording a
 * checkpoint of the whole state every ckpt_every steps (ckpt_every = 1 stores every step and
 * needs no recomputation), and write the tip trajectory to tips (n_rods x n_steps x 3, rod
 * major; nullable).  The handle holds one rollout at a time: this one replaces the previous.
 * rollout (nullable) receives its number (1, 2, ... per handle), which rod_adjoint_backward
 * checks.  Device memory: ceil(n_steps / ckpt_every) + ckpt_every states. */
rod_status rod_adjoint_forward(rod_ctx* ctx, int32_t n_steps, int32_t ckpt_every, float* tips,
                               int32_t on_device, int64_t* rollout);

/* Reverse pass of the last rod_adjoint_forward() (ROD_E_ORDER without one, or if rollout is
 * not 0 and not the number of the held rollout, i.e. a later forward replaced it).  dl_dtips:
 * n_rods x n_steps x 3.  Outputs (any may be NULL): dL/dm_b, dL/dm_t (n_rods each), and
 * dL/d(initial state) in the state layout; dl_dq is the gradient with respect to the four
 * quaternion components as stored (not projected on the unit sphere).  Each checkpoint
 * segment is recomputed forward, then reversed by one kernel launch per bucket.  Synchronises
 * the stream; ROD_E_UNSTABLE if a non-finite adjoint appears. */
rod_status rod_adjoint_backward(rod_ctx* ctx, int64_t rollout, const float* dl_dtips,
                                float* dl_dbend, float* dl_dtwist, float* dl_dx, float* dl_dv,
                                float* dl_dq, float* dl_dw, int32_t on_device);

const char* rod_status_str(rod_status s);
/* Detail of the last error on this handle (never NULL; "" if none; NULL ctx = global). */
const char* rod_last_error(const rod_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif
