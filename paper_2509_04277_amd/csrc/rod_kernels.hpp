// rod_kernels.hpp -- gfx950 kernels of the CoRdE Cosserat-rod stepper.
//
// One workgroup of W wavefronts steps one rod for k time steps per launch with the whole rod
// state held in registers.  Lane g (0 <= g < 64 W) owns E consecutive "slots"; slot j holds
// material frame j (q_j, omega_j) and mass point j+1 (x_{j+1}, v_{j+1}), i.e. segment j's
// right end.  Point 0 (the clamped base) is held separately by lane 0.  With this split a rod
// of N elements needs exactly N slots.
//
// Neighbour data moves between lanes of a wavefront with DPP whole-wave shifts (wave_shr:1,
// wave_shl:1), and between wavefronts through a double-buffered LDS mailbox with one
// s_barrier per exchange.  One time step needs, in order (Sec. 2.1, Fig. 5 of the paper):
//   A  exchange x of the left point and q of the right frame,
//   F  segment forces (stretch eq. (2), penalty eq. (8)), joint torques (bend/twist eq. (3)
//      with the Darboux vector of eqs. (5)-(6)),
//   B  exchange each segment's force on its left point and each joint's torque on its right
//      frame (and, inextensible, the right neighbour's segment vector),
//   V  integrate forces: points as particles, frames as rigid bodies (Euler's equations),
//   C  inextensible: n_iter x {even segments, odd segments} velocity impulses; with an even
//      number of slots per lane only the even half-sweep crosses lanes,
//   X  integrate velocities (semi-implicit Euler) and renormalise the quaternions.
// No barrier is needed inside a wavefront; a workgroup of W > 1 waves pays one barrier per
// exchange (A, B and one per constraint iteration).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace corde {

// Per-slot coefficient rows (FP32, derived in FP64 on the host), stored row-major:
// prm[row * stride + slot].
enum PrmRow : int {
  P_WINV = 0,    // inverse mass of point j+1
  P_WINV_PREV,   // inverse mass of point j (0 for a clamped base)
  P_CI,          // segment j: 1 / (dt (w_j + w_{j+1}))   (J M^-1 J^T of the distance constraint)
  P_CIL,         // segment j: l_j / (dt (w_j + w_{j+1}))
  P_CI_NEXT,     // the same for segment j+1 (0 if j = N-1: no segment)
  P_CIL_NEXT,
  P_LEN,         // rest length l_j
  P_KS_L,        // K_s / l_j, stretch, eq. (2) (0 for the inextensible variant)
  P_LKP,         // l_j K_p, penalty, eq. (8)
  P_IINV1,       // 1 / I_1 of frame j
  P_IINV3,       // 1 / I_3
  P_GYRO,        // (I_3 - I_1) / I_1
  P_C1,          // joint j: 2 K_1 / lbar_j (0 if j = N-1: no joint)
  P_C3,          // joint j: 2 K_3 / lbar_j
  P_D0,          // joint j: K_k uhat_k
  P_D1,
  P_D2,
  P_NROWS
};

// Clamp poses are evaluated for up to kClampChunk steps at a time, one step per lane, into LDS.
constexpr int kClampChunk = 64;

// Haptic mailbox of one clamped rod, in pinned host memory mapped for the device (Sec. 2.2:
// the haptic thread writes the device position and reads the force feedback at any time,
// while the kernel runs).  Every word is a 64-bit value (tag << 32 | bits of a float), read
// and written whole; a record is taken only when all its words carry the same tag, so a read
// that overlaps a write is never taken and no ordering between words is needed.
//   pose: x, y, z, qw, qx, qy, qz               tag = the host's pose number (1, 2, ...)
//   fb:   fx, fy, fz, pose number, window steps  tag = steps completed (low 32 bits)
struct HapticBox {
  uint64_t pose[8];
  uint64_t fb[8];
};

// Mailbox words are accessed through global-address-space pointers: a flat access would also
// count against the LDS wait counter, so every LDS exchange would wait for the PCIe round trip.
using GlobalWord = __attribute__((address_space(1))) uint64_t;
__device__ __forceinline__ uint64_t mailbox_load(const uint64_t* p) {
  return __hip_atomic_load((GlobalWord*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void mailbox_store(uint64_t* p, uint64_t v) {
  __hip_atomic_store((GlobalWord*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Static triangle mesh of the environment (Sec. 2.2 "Collisions"): an AABB tree by volume
// partitioning, its nodes in depth-first order so that a query walks it without a stack: at a
// node whose box the sphere reaches, go to the next node (its first child), or test a leaf's
// triangles and go to `skip`; elsewhere jump to `skip`, the node after its subtree.
struct alignas(16) EnvNode {
  float lo[3];
  int32_t skip;   // index of the first node after this subtree
  float hi[3];
  int32_t leaf;   // -1: interior node; else (first triangle << 3) | triangle count
};
struct alignas(16) EnvTri {
  float a[3], e1[3], e2[3], n[3];   // vertex a, b - a, c - a, unit face normal
};

struct RodDev {
  int32_t n;          // elements
  int32_t slot_off;   // first slot in the coefficient rows
  int32_t pt_off;     // first point in x, v
  int32_t fr_off;     // first frame in q, w
  int32_t n_iter;     // constraint iterations (0: extensible)
  int32_t clamp;      // 1: base point and frame 0 kinematic
  int32_t self_skip;  // points of this rod closer than this along it never touch
  int32_t driven;     // 1: clamp trajectory has non-zero amplitudes
  int32_t has_ext;    // 1: read f_ext / tau_ext
  float dt, damp_lin, damp_ang, winv0;
  float g[3];
  float ctw;          // twist amplitude
  float cx0[3], camp[3], caxis[3];
  float cq0[4];
  float mult_bend;    // learnable multipliers of the bend (K_1 = K_2) and twist (K_3) stiffness
  float mult_twist;
  double dt_d, t0, omega, ph_x, ph_t;
  HapticBox* hbox;    // haptic mailbox (device address of pinned host memory), or null
  int32_t hstride;    // steps per force record (>= 1 with a mailbox)
  int32_t env_n_nodes;   // environment tree (0: none)
  const EnvNode* env_nodes;
  const EnvTri* env_tris;
  float4* env_cache;  // per slot: where its candidate list was built, list length (int bits)
  int2* env_cand;     // per slot: kEnvCand candidates (triangle, bits of its build distance)
  const float* rho;   // per slot: sphere radius of point slot + 1
  float env_mu;       // friction coefficient against the environment
  float damp_int;     // internal friction: Kelvin-Voigt retardation time tau_d [s] (0: none)
};

// Kernel feature bits of rod_resident_kernel's variants.
constexpr int kFeatHaptic = 1;
constexpr int kFeatEnv = 2;
constexpr int kFeatDamp = 4;   // internal friction

struct V3 {
  float x, y, z;
};
struct Q4 {
  float w, x, y, z;
};

__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 operator*(float s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
// s a + b and b - s a with one rounding per component (explicit, so that the fused forms do
// not depend on what the compiler sees around an inlined call)
__device__ __forceinline__ V3 fma3(float s, V3 a, V3 b) {
  return {__builtin_fmaf(s, a.x, b.x), __builtin_fmaf(s, a.y, b.y), __builtin_fmaf(s, a.z, b.z)};
}
__device__ __forceinline__ V3 fnma3(float s, V3 a, V3 b) {
  return {__builtin_fmaf(-s, a.x, b.x), __builtin_fmaf(-s, a.y, b.y), __builtin_fmaf(-s, a.z, b.z)};
}
__device__ __forceinline__ float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ V3 sel(bool c, V3 a, V3 b) {
  return {c ? a.x : b.x, c ? a.y : b.y, c ? a.z : b.z};
}
__device__ __forceinline__ Q4 sel4(bool c, Q4 a, Q4 b) {
  return {c ? a.w : b.w, c ? a.x : b.x, c ? a.y : b.y, c ? a.z : b.z};
}

// DPP whole-wavefront shifts.  from_lower_lane / from_upper_lane: the lane without a source
// (lane 0 / lane 63) receives 0 (bound_ctrl).  The `_or` forms leave that lane's destination
// unwritten, so it keeps `edge`: one instruction moves the neighbour's value and merges what the
// wavefront's edge lane takes from elsewhere.
__device__ __forceinline__ float from_lower_lane(float v) {  // lane i <- lane i-1
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_upper_lane(float v) {  // lane i <- lane i+1
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_lower_lane_or(float edge, float v) {  // lane i <- lane i-1
  return __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float from_upper_lane_or(float edge, float v) {  // lane i <- lane i+1
  return __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), 0x130, 0xf, 0xf, false));
}

// Neighbour exchange across the rod's lanes.  `lo` receives the KL values `mine_hi` of the
// lane below (its last slot), `hi` receives the KH values `mine_lo` of the lane above (its
// first slot).  The rod's last lane receives 0.  Its first lane (g = 0) receives `base` (B:
// values that stand for what lies below the rod, such as its base point) in the merged form;
// otherwise 0, and the caller substitutes (the substitution inside the plain form kept a lane
// mask live across the step loop, which spilled scalar registers).  E (the elements per lane)
// only sets how much register room the reads may use.
constexpr int kMailboxWords = 11;  // the widest exchange: quaternion (two parts), angular velocity
// buf: what each wavefront's edge lanes publish ([0]: lane 0's, [1]: lane 63's), per parity.
// edge (merged form, M): [1] is what lane 0 of wavefront 0 reads from below (written by that
// lane at every exchange: the base values, or zeros), [0] what the last wavefront's lane 63
// reads from above (zero, set once by mailbox_init and never written).
template <int W, bool M = false>
struct Mailbox {
  float buf[2][W][2][kMailboxWords];
  float edge[2][2][kMailboxWords];
};

// Two forms of the exchange move the same values (the states are bitwise the same).  The
// merged form (M) reads the mailbox words into the DPP moves' kept operand (one instruction per
// word, the base values travelling through the mailbox); the plain form moves before the
// barrier and selects the mailbox words into the edge lanes afterwards.  Measured (device time
// per step, 2 rods and 2048 rods per launch, every shape): the merged form is faster for four
// wavefronts of 2 or 4 elements per lane, one per SIMD, and slower for every other shape, for
// two rods of four wavefronts in one workgroup (two wavefronts per SIMD), and in the chunked
// long-rod kernel's extensible steps (two exchanges per step); those use the plain form.
template <int W, int E>
constexpr bool kMergedExchange = (W == 4) && (E == 2 || E == 4);

// Zeroes the words above the last wavefront (merged form only); must run before the kernel's
// first exchange (whose barrier orders it before the reads).  It touches no word that an
// exchange writes.
template <int W, bool M>
__device__ __forceinline__ void mailbox_init(Mailbox<W, M>& mb) {
  if constexpr (M) {
    if (threadIdx.x < kMailboxWords) {
      mb.edge[0][0][threadIdx.x] = 0.f;
      mb.edge[1][0][threadIdx.x] = 0.f;
    }
  }
}

template <int W, int E, int KL, int KH, bool B, bool M>
__device__ __forceinline__ void exchange(const float (&mine_hi)[KL], float (&lo)[KL],
                                         const float (&mine_lo)[KH], float (&hi)[KH],
                                         const float (&base)[KL], Mailbox<W, M>& mb, int& parity) {
  static_assert(KL <= kMailboxWords && KH <= kMailboxWords, "exchange wider than the mailbox");
  const int lane = threadIdx.x & 63;
  if constexpr (W == 1) {
#pragma unroll
    for (int k = 0; k < KL; ++k) lo[k] = from_lower_lane(mine_hi[k]);
#pragma unroll
    for (int k = 0; k < KH; ++k) hi[k] = from_upper_lane(mine_lo[k]);
  } else if constexpr (M) {
    const int wave = (threadIdx.x >> 6) & (W - 1);   // wavefront within the rod's W
    if (lane == 63) {
#pragma unroll
      for (int k = 0; k < KL; ++k) mb.buf[parity][wave][1][k] = mine_hi[k];
    }
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < KH; ++k) mb.buf[parity][wave][0][k] = mine_lo[k];
      if (wave == 0) {   // (zeros without B: faster on c1 than reading the zero words)
#pragma unroll
        for (int k = 0; k < KL; ++k) mb.edge[parity][1][k] = B ? base[k] : 0.f;
      }
    }
    __syncthreads();
    // every lane reads the same (broadcast) words; the DPP move keeps them only in the
    // wavefront's edge lane, which has no source inside the wavefront
    const float* from_lo = wave > 0 ? mb.buf[parity][wave - 1][1] : mb.edge[parity][1];
    const float* from_hi = wave < W - 1 ? mb.buf[parity][wave + 1][0] : mb.edge[parity][0];
#pragma unroll
    for (int k = 0; k < KL; ++k) lo[k] = from_lower_lane_or(from_lo[k], mine_hi[k]);
#pragma unroll
    for (int k = 0; k < KH; ++k) hi[k] = from_upper_lane_or(from_hi[k], mine_lo[k]);
    parity ^= 1;
  } else {
    static_assert((W & (W - 1)) == 0, "W must be a power of two");
#pragma unroll
    for (int k = 0; k < KL; ++k) lo[k] = from_lower_lane(mine_hi[k]);
#pragma unroll
    for (int k = 0; k < KH; ++k) hi[k] = from_upper_lane(mine_lo[k]);
    const int wave = (threadIdx.x >> 6) & (W - 1);   // wavefront within the rod's W
    if (lane == 63) {
#pragma unroll
      for (int k = 0; k < KL; ++k) mb.buf[parity][wave][1][k] = mine_hi[k];
    }
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < KH; ++k) mb.buf[parity][wave][0][k] = mine_lo[k];
    }
    __syncthreads();
    // every lane reads the same (broadcast) words and only the wave's edge lanes keep them.
    // Where registers allow, an empty asm consumes the loaded values so the loads stay
    // unconditional (a load moved under the lane test becomes an exec-mask branch per word);
    // 8 waves x 4 elements (256 registers) and 16 waves (128) would spill with all words live.
    constexpr bool kPinLoads = (W <= 4) || (W <= 8 && E <= 2);
    const int wl = wave > 0 ? wave - 1 : 0;
    const int wh = wave < W - 1 ? wave + 1 : W - 1;
    const bool take_lo = (lane == 0) && (wave > 0);
    const bool take_hi = (lane == 63) && (wave < W - 1);
    if constexpr (kPinLoads) {
      float tl[KL], th[KH];
#pragma unroll
      for (int k = 0; k < KL; ++k) tl[k] = mb.buf[parity][wl][1][k];
#pragma unroll
      for (int k = 0; k < KH; ++k) th[k] = mb.buf[parity][wh][0][k];
#pragma unroll
      for (int k = 0; k < KL; ++k) {
        asm volatile("" : "+v"(tl[k]));
        lo[k] = take_lo ? tl[k] : lo[k];
      }
#pragma unroll
      for (int k = 0; k < KH; ++k) {
        asm volatile("" : "+v"(th[k]));
        hi[k] = take_hi ? th[k] : hi[k];
      }
    } else {
#pragma unroll
      for (int k = 0; k < KL; ++k) {
        const float t = mb.buf[parity][wl][1][k];
        lo[k] = take_lo ? t : lo[k];
      }
#pragma unroll
      for (int k = 0; k < KH; ++k) {
        const float t = mb.buf[parity][wh][0][k];
        hi[k] = take_hi ? t : hi[k];
      }
    }
    parity ^= 1;
  }
}

// Velocity impulse of one distance constraint (Sec. 2.1, "Constraints"), linearised at the
// predicted positions p = x + dt v, returned as lambda n:
//   d = p_hi - p_lo = e + dt (v_hi - v_lo),  C = |d| - l,  lambda = C / (dt (w_lo + w_hi)),
//   lambda n = ci (1 - l / |d|) d   with ci = 1 / (dt (w_lo + w_hi)), cil = ci l.
// Both owners of a segment compute it from identical operands, so both apply the same impulse.
// A missing segment has ci = cil = 0 and yields 0 (the max keeps the reciprocal finite).
__device__ __forceinline__ V3 impulse_d(V3 d, float ci, float cil) {
  const float il = rsqrtf(fmaxf(dot(d, d), 1e-30f));
  const float s = ci - cil * il;
  return s * d;
}

// x <- x + dt v on a position held as the pair (hi, lo): y = lo + dt v (one rounding), then
// the Fast2Sum of hi and y, whose rounding error becomes the new low part.
__device__ __forceinline__ void add_compensated(float& hi, float& lo, float v, float dt) {
  const float y = __builtin_fmaf(dt, v, lo);
  const float s = hi + y;
  lo = y - (s - hi);
  hi = s;
}
__device__ __forceinline__ void advance_position(V3& hi, V3& lo, V3 v, float dt) {
  add_compensated(hi.x, lo.x, v.x, dt);
  add_compensated(hi.y, lo.y, v.y, dt);
  add_compensated(hi.z, lo.z, v.z, dt);
}

// hi + lo <- hi + lo + d with the Fast2Sum of hi and lo + d.
__device__ __forceinline__ void add_pair(float& hi, float& lo, float d) {
  const float y = lo + d;
  const float s = hi + y;
  lo = y - (s - hi);
  hi = s;
}

// q <- normalize(q + dt/2 q (x) (0, omega)) on a quaternion held as the pair (h, l) (the
// rotation increment per step is far below the ulp of a unit quaternion's components).  The
// increment d, from the high part, is orthogonal to it (a rotation), so |h + d|^2 = |h|^2 +
// |d|^2 and the normalised result is (h + d)(1 + eps) with eps = 1/|h + d| - 1: the increment
// and the normalisation enter as one correction d + eps (h + d), added to the pair with
// Fast2Sum per component.  The FP32 rounding of eps only changes the norm, not the rotation.
__device__ __forceinline__ void advance_quat(Q4& h, Q4& l, V3 o, float dt) {
  const float hdt = 0.5f * dt;
  const Q4 d = {hdt * (-h.x * o.x - h.y * o.y - h.z * o.z), hdt * (h.w * o.x + h.y * o.z - h.z * o.y),
                hdt * (h.w * o.y - h.x * o.z + h.z * o.x), hdt * (h.w * o.z + h.x * o.y - h.y * o.x)};
  const float n2 = (h.w * h.w + h.x * h.x + h.y * h.y + h.z * h.z) +
                   (d.w * d.w + d.x * d.x + d.y * d.y + d.z * d.z);
  const float eps = rsqrtf(n2) - 1.f;
  add_pair(h.w, l.w, __builtin_fmaf(eps, h.w, __builtin_fmaf(eps, d.w, d.w)));
  add_pair(h.x, l.x, __builtin_fmaf(eps, h.x, __builtin_fmaf(eps, d.x, d.x)));
  add_pair(h.y, l.y, __builtin_fmaf(eps, h.y, __builtin_fmaf(eps, d.y, d.y)));
  add_pair(h.z, l.z, __builtin_fmaf(eps, h.z, __builtin_fmaf(eps, d.z, d.z)));
}

__device__ __forceinline__ Q4 qmul(Q4 a, Q4 b) {
  return {a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z,
          a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y,
          a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x,
          a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w};
}

// Prescribed clamp pose at time t: position, orientation, body angular rate.
__device__ __forceinline__ void clamp_pose(const RodDev& rd, double t, V3& xc, Q4& qc, V3& wc) {
  const double two_pi = 6.283185307179586;
  double px = rd.omega * t + rd.ph_x;
  double pt = rd.omega * t + rd.ph_t;
  px -= two_pi * rint(px * (1.0 / two_pi));
  pt -= two_pi * rint(pt * (1.0 / two_pi));
  float sx = sinf((float)px);
  float st, ct;
  sincosf((float)pt, &st, &ct);
  xc = {rd.cx0[0] + rd.camp[0] * sx, rd.cx0[1] + rd.camp[1] * sx, rd.cx0[2] + rd.camp[2] * sx};
  float psi = rd.ctw * st;
  float psidot = rd.ctw * (float)rd.omega * ct;
  float sh, ch;
  sincosf(0.5f * psi, &sh, &ch);
  Q4 r = {ch, sh * rd.caxis[0], sh * rd.caxis[1], sh * rd.caxis[2]};
  Q4 q0 = {rd.cq0[0], rd.cq0[1], rd.cq0[2], rd.cq0[3]};
  qc = qmul(r, q0);
  // body rate = R(qc)^T (psidot axis): rotate by the conjugate
  V3 a = {psidot * rd.caxis[0], psidot * rd.caxis[1], psidot * rd.caxis[2]};
  V3 u = {-qc.x, -qc.y, -qc.z};
  V3 tt = 2.0f * cross(u, a);
  wc = a + qc.w * tt + cross(u, tt);
}


// Nearest point of triangle t to the point a + ap (a its first vertex), as its offset from
// a, by the Voronoi region of the point (vertex, edge or face) found from the signs of dot
// products with the edges (Ericson, Real-Time Collision Detection, 5.1.5).  Working from a
// keeps every quantity at the scale of the triangle and the sphere, not of the coordinates.
// face: set when the nearest point lies inside the face (the point projects onto it).
__device__ __forceinline__ V3 tri_closest(const EnvTri& t, V3 ap, bool& face) {
  face = false;
  const V3 ab = {t.e1[0], t.e1[1], t.e1[2]};
  const V3 ac = {t.e2[0], t.e2[1], t.e2[2]};
  const float d1 = dot(ab, ap), d2 = dot(ac, ap);
  if (d1 <= 0.f && d2 <= 0.f) return {0.f, 0.f, 0.f};
  const V3 bp = ap - ab;
  const float d3 = dot(ab, bp), d4 = dot(ac, bp);
  if (d3 >= 0.f && d4 <= d3) return ab;
  const float vc = d1 * d4 - d3 * d2;
  if (vc <= 0.f && d1 >= 0.f && d3 <= 0.f) return (d1 / (d1 - d3)) * ab;
  const V3 cp = ap - ac;
  const float d5 = dot(ab, cp), d6 = dot(ac, cp);
  if (d6 >= 0.f && d5 <= d6) return ac;
  const float vb = d5 * d2 - d1 * d6;
  if (vb <= 0.f && d2 >= 0.f && d6 <= 0.f) return (d2 / (d2 - d6)) * ac;
  const float va = d3 * d6 - d5 * d4;
  if (va <= 0.f && d4 - d3 >= 0.f && d5 - d6 >= 0.f) {
    const float u = (d4 - d3) / ((d4 - d3) + (d5 - d6));
    return fma3(u, ac - ab, ab);
  }
  face = true;
  const float den = 1.0f / (va + vb + vc);
  return fma3(vc * den, ac, (vb * den) * ab);
}

// Walks the environment's tree for a sphere of centre c and radius reach, calling leaf(k) for
// every triangle k of every leaf whose box the sphere reaches, in tree order.
template <class Leaf>
__device__ __forceinline__ void env_walk(const RodDev& rd, V3 c, float reach, Leaf&& leaf) {
  const float r2 = reach * reach;
  int i = 0;
  while (i < rd.env_n_nodes) {
    const EnvNode nd = rd.env_nodes[i];
    const float bx = fmaxf(fmaxf(nd.lo[0] - c.x, c.x - nd.hi[0]), 0.f);
    const float by = fmaxf(fmaxf(nd.lo[1] - c.y, c.y - nd.hi[1]), 0.f);
    const float bz = fmaxf(fmaxf(nd.lo[2] - c.z, c.z - nd.hi[2]), 0.f);
    const bool in = bx * bx + by * by + bz * bz < r2;
    if (in && nd.leaf >= 0) {
      const int first = nd.leaf >> 3, cnt = nd.leaf & 7;
      for (int k = 0; k < cnt; ++k) leaf(first + k);
    }
    i = (in && nd.leaf < 0) ? i + 1 : nd.skip;
  }
}

// Narrow phase of one triangle against a sphere (centre c + cl, a compensated position;
// radius r): a triangle collides when its nearest point is closer than r; its depth is r - dist
// with the centre in front of the face, r + dist behind it; acc gathers depth x face normal,
// dmax the largest depth.  Returns the distance.  The centre is taken relative to the
// triangle's first vertex in FP64 (exact for these float operands); where the nearest point
// is inside the face the signed distance is the height over the face's plane, dot(c + cl - a,
// n) in FP64, and the depth is r minus that height on either side: resting contact keeps the
// height within a step's sinking of r, far below the ulp of the coordinates.
__device__ __forceinline__ float env_hit(const EnvTri& t, V3 c, V3 cl, float r, V3& acc,
                                         float& dmax) {
  const double hx = ((double)c.x - (double)t.a[0]) + (double)cl.x;
  const double hy = ((double)c.y - (double)t.a[1]) + (double)cl.y;
  const double hz = ((double)c.z - (double)t.a[2]) + (double)cl.z;
  const V3 ca = {(float)hx, (float)hy, (float)hz};
  const V3 nf = {t.n[0], t.n[1], t.n[2]};
  bool face;
  const V3 d = ca - tri_closest(t, ca, face);
  float dist, dep;
  if (face) {
    const double H = __builtin_fma(hx, (double)nf.x, __builtin_fma(hy, (double)nf.y, hz * (double)nf.z));
    dep = (float)((double)r - H);
    dist = fabsf((float)H);
  } else {
    dist = sqrtf(dot(d, d));
    dep = dot(ca, nf) >= 0.f ? r - dist : r + dist;
  }
  if (dist < r) {
    acc = fma3(dep, nf, acc);
    dmax = fmaxf(dmax, dep);
  }
  return dist;
}

// Collision response from the gathered hits: the depth-weighted mean normal, the largest depth.
__device__ __forceinline__ void env_finish(V3 acc, float dmax, V3& n, float& depth) {
  const float al2 = dot(acc, acc);
  if (dmax > 0.f && al2 > 0.f) {
    n = rsqrtf(al2) * acc;
    depth = dmax;
  } else {
    n = {0.f, 0.f, 0.f};
    depth = 0.f;
  }
}

// Candidate triangles cached per point: every triangle within (1 + m) r of the point where the
// list was built, m = kEnvMargin, with its distance from there.  While the point stays within
// m r of that place, the triangles within r of it are all on the list, so the narrow phase runs
// over the list alone (in tree order, as a walk would visit them), and skips, without loading
// it, every triangle whose build distance minus the point's movement is still at least r (its
// distance now is no smaller).  A point that moved farther rebuilds its list with a walk.  A
// list that overflows makes the point walk the tree every step until its next rebuild.
constexpr int kEnvCand = 32;
constexpr float kEnvMargin = 1.0f;

// Whole-handle state arrays in device memory: x, v (3 floats per point), q (4 per frame, w x y
// z), w (3 per frame), and the low parts of x and q (layouts of x and q; null: read as 0 and
// not written).
struct StateArrays {
  float *x, *v, *q, *w, *xl, *ql;
};
// One whole-handle state stored contiguously (trajectories, checkpoints):
//   [x (3 n_pts) | v (3 n_pts) | q (4 n_frames) | w (3 n_frames) | xl (3 n_pts) | ql (4 n_frames)]
__host__ __device__ __forceinline__ StateArrays state_at(float* base, long long n_pts,
                                                         long long n_frames) {
  return {base, base + 3 * n_pts, base + 6 * n_pts, base + 6 * n_pts + 4 * n_frames,
          base + 6 * n_pts + 7 * n_frames, base + 9 * n_pts + 7 * n_frames};
}
__host__ __device__ __forceinline__ long long state_floats(long long n_pts, long long n_frames) {
  return 9 * n_pts + 11 * n_frames;
}

// Registers of one lane of a rod's workgroup: E slots (frame j, point j+1) plus, in lane 0,
// the base point.  The member functions are the phases of one time step; the forward kernel
// and the adjoint kernel call the same functions, so a recomputed step is bit-identical.
//
// Positions and quaternions are held as unevaluated sums of two floats (X + XL, Qf + QL; the
// low part below half an ulp of the high one): the per-step increments dt v and
// dt/2 q (x) (0, omega) are far below the ulp of a coordinate of a metres-long rod or of a unit
// quaternion's component, and rounding the sums to one float every step perturbs the
// trajectory, and the gradients of a rollout, far more than the FP32 rounding of v and omega
// does.  Increments are added with compensated (Fast2Sum) updates; segment vectors and the
// quaternion differences of the Darboux vectors take the two parts' differences separately;
// the low parts travel through HBM between launches.
template <int W, int E>
struct RodLane {
  V3 X[E], XL[E], Vv[E], Om[E];
  Q4 Qf[E], QL[E];
  float P[P_NROWS][E];
  bool ok[E];
  V3 bx, bxl, bv;
  int g, j0, n;
  int off, nloc;   // window of the rod held by this workgroup: slots [off, off + nloc)
  bool ghost;      // off > 0: lane 0's "base point" is point `off`, held fixed (a halo edge)
  V3 imp0;         // lane 0: momentum passed to point 0 (forces x dt + impulses)
  V3 en[E];        // environment collision of each slot's point this step: normal, depth
  float ed[E];
  bool env_any;    // some point of this wavefront collides this step (uniform over the wave)
  float dt;

  // Loads the coefficients of slots [off, off + nloc) (the whole rod by default).  A window
  // that does not reach the rod's end drops its last slot's outward segment and joint; one
  // that does not start at the rod's base sees point `off` as a fixed (infinite-mass) point.
  // Both only perturb slots within one step's dependency radius of the window edges.
  __device__ __forceinline__ void load_params(const RodDev& rd, const float* __restrict__ prm,
                                              int prm_stride, int win_off = 0, int win_n = -1) {
    g = threadIdx.x & (64 * W - 1);   // lane within the rod's 64 W (a workgroup may hold two)
    n = rd.n;
    off = win_off;
    nloc = win_n < 0 ? rd.n : win_n;
    ghost = off > 0;
    j0 = g * E;
    dt = rd.dt;
    const bool cut_right = off + nloc < n;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int jl = j0 + e;
      ok[e] = jl < nloc;
#pragma unroll
      for (int r = 0; r < P_NROWS; ++r)
        P[r][e] = ok[e] ? prm[r * prm_stride + rd.slot_off + off + jl] : 0.f;
      // learnable stiffness multipliers scale the joint coefficients
      P[P_C1][e] *= rd.mult_bend;
      P[P_D0][e] *= rd.mult_bend;
      P[P_D1][e] *= rd.mult_bend;
      P[P_C3][e] *= rd.mult_twist;
      P[P_D2][e] *= rd.mult_twist;
      if (ghost && jl == 0) P[P_WINV_PREV][e] = 0.f;
      if (cut_right && jl == nloc - 1) {
        P[P_CI_NEXT][e] = 0.f;
        P[P_CIL_NEXT][e] = 0.f;
        P[P_C1][e] = P[P_C3][e] = P[P_D0][e] = P[P_D1][e] = P[P_D2][e] = 0.f;
      }
    }
  }

  __device__ __forceinline__ void load_state(const RodDev& rd, const StateArrays& sa) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int j = off + j0 + e;
      X[e] = XL[e] = Vv[e] = Om[e] = {0.f, 0.f, 0.f};
      Qf[e] = {1.f, 0.f, 0.f, 0.f};
      QL[e] = {0.f, 0.f, 0.f, 0.f};
      if (ok[e]) {
        const float* px = sa.x + 3 * (rd.pt_off + j + 1);
        const float* pv = sa.v + 3 * (rd.pt_off + j + 1);
        const float* pq = sa.q + 4 * (rd.fr_off + j);
        const float* pw = sa.w + 3 * (rd.fr_off + j);
        X[e] = {px[0], px[1], px[2]};
        Vv[e] = {pv[0], pv[1], pv[2]};
        Qf[e] = {pq[0], pq[1], pq[2], pq[3]};
        Om[e] = {pw[0], pw[1], pw[2]};
        if (sa.xl) {
          const float* pl = sa.xl + 3 * (rd.pt_off + j + 1);
          XL[e] = {pl[0], pl[1], pl[2]};
        }
        if (sa.ql) {
          const float* pl = sa.ql + 4 * (rd.fr_off + j);
          QL[e] = {pl[0], pl[1], pl[2], pl[3]};
        }
      }
    }
    bx = bxl = bv = {0.f, 0.f, 0.f};
    if (g == 0) {
      const float* px = sa.x + 3 * (rd.pt_off + off);
      const float* pv = sa.v + 3 * (rd.pt_off + off);
      bx = {px[0], px[1], px[2]};
      bv = {pv[0], pv[1], pv[2]};
      if (sa.xl) {
        const float* pl = sa.xl + 3 * (rd.pt_off + off);
        bxl = {pl[0], pl[1], pl[2]};
      }
    }
  }

  // Writes the slots [own_lo, own_hi) of the window (all by default) and, for a window at the
  // rod's base, the base point; returns a sum of the written values (non-finite if any is).
  __device__ __forceinline__ float store_state(const RodDev& rd, const StateArrays& sa,
                                               int own_lo = 0, int own_hi = 1 << 30) const {
    float chk = 0.f;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int jl = j0 + e;
      const int j = off + jl;
      if (ok[e] && jl >= own_lo && jl < own_hi) {
        float* px = sa.x + 3 * (rd.pt_off + j + 1);
        float* pv = sa.v + 3 * (rd.pt_off + j + 1);
        float* pq = sa.q + 4 * (rd.fr_off + j);
        float* pw = sa.w + 3 * (rd.fr_off + j);
        px[0] = X[e].x; px[1] = X[e].y; px[2] = X[e].z;
        pv[0] = Vv[e].x; pv[1] = Vv[e].y; pv[2] = Vv[e].z;
        pq[0] = Qf[e].w; pq[1] = Qf[e].x; pq[2] = Qf[e].y; pq[3] = Qf[e].z;
        pw[0] = Om[e].x; pw[1] = Om[e].y; pw[2] = Om[e].z;
        if (sa.xl) {
          float* pl = sa.xl + 3 * (rd.pt_off + j + 1);
          pl[0] = XL[e].x; pl[1] = XL[e].y; pl[2] = XL[e].z;
        }
        if (sa.ql) {
          float* pl = sa.ql + 4 * (rd.fr_off + j);
          pl[0] = QL[e].w; pl[1] = QL[e].x; pl[2] = QL[e].y; pl[3] = QL[e].z;
        }
        chk += X[e].x + X[e].y + X[e].z + Vv[e].x + Vv[e].y + Vv[e].z + Qf[e].w + Om[e].x +
               Om[e].y + Om[e].z;
      }
    }
    if (g == 0 && off == 0) {
      float* px = sa.x + 3 * rd.pt_off;
      float* pv = sa.v + 3 * rd.pt_off;
      px[0] = bx.x; px[1] = bx.y; px[2] = bx.z;
      pv[0] = bv.x; pv[1] = bv.y; pv[2] = bv.z;
      if (sa.xl) {
        float* pl = sa.xl + 3 * rd.pt_off;
        pl[0] = bxl.x; pl[1] = bxl.y; pl[2] = bxl.z;
      }
      chk += bx.x + bx.y + bx.z + bv.x + bv.y + bv.z;
    }
    return chk;
  }

  // Exchange A: the left neighbour point's position (both parts: xl, xll; the base point for
  // lane 0) and the next frame's quaternion (both parts: qn, qnl; from the lane above); with
  // internal friction (D) also that point's velocity vl and that frame's angular velocity wn.
  template <bool D, bool M>
  __device__ __forceinline__ void exchange_a(Mailbox<W, M>& mb, int& par, V3& xl, V3& xll, Q4& qn,
                                             Q4& qnl, V3& vl, V3& wn) const {
    const V3 a = X[E - 1], al = XL[E - 1];
    const Q4 b = Qf[0], bl = QL[0];
    if constexpr (D) {
      const V3 c = Vv[E - 1], o = Om[0];
      float mh[9] = {a.x, a.y, a.z, al.x, al.y, al.z, c.x, c.y, c.z};
      float ml[11] = {b.w, b.x, b.y, b.z, bl.w, bl.x, bl.y, bl.z, o.x, o.y, o.z};
      const float base[9] = {bx.x, bx.y, bx.z, bxl.x, bxl.y, bxl.z, bv.x, bv.y, bv.z};
      float lo[9], hi[11];
      exchange<W, E, 9, 11, true, M>(mh, lo, ml, hi, base, mb, par);
      xl = {lo[0], lo[1], lo[2]};
      xll = {lo[3], lo[4], lo[5]};
      vl = {lo[6], lo[7], lo[8]};
      if (!M && g == 0) {
        xl = bx;
        xll = bxl;
        vl = bv;
      }
      qn = {hi[0], hi[1], hi[2], hi[3]};
      qnl = {hi[4], hi[5], hi[6], hi[7]};
      wn = {hi[8], hi[9], hi[10]};
    } else {
      float mh[6] = {a.x, a.y, a.z, al.x, al.y, al.z};
      float ml[8] = {b.w, b.x, b.y, b.z, bl.w, bl.x, bl.y, bl.z};
      const float base[6] = {bx.x, bx.y, bx.z, bxl.x, bxl.y, bxl.z};
      float lo[6], hi[8];
      exchange<W, E, 6, 8, true, M>(mh, lo, ml, hi, base, mb, par);
      xl = {lo[0], lo[1], lo[2]};
      xll = {lo[3], lo[4], lo[5]};
      if (!M && g == 0) {
        xl = bx;
        xll = bxl;
      }
      qn = {hi[0], hi[1], hi[2], hi[3]};
      qnl = {hi[4], hi[5], hi[6], hi[7]};
      vl = {0.f, 0.f, 0.f};
      wn = {0.f, 0.f, 0.f};
    }
  }
  template <bool M>
  __device__ __forceinline__ void exchange_a(Mailbox<W, M>& mb, int& par, V3& xl, V3& xll, Q4& qn,
                                             Q4& qnl) const {
    V3 vl, wn;
    exchange_a<false>(mb, par, xl, xll, qn, qnl, vl, wn);
  }

  // F: segment forces (stretch eq. (2), penalty eq. (8)) and joint torques (eq. (3) with the
  // discrete Darboux vector of eqs. (5)-(6)), accumulated per slot; then exchange B.
  // F[e]: force on point j+1; T[e]: body torque on frame j; Ev[e]: segment vector e_j;
  // fs0: force of the lane's first segment on its left point (negated); enext: e_{j+1} of the
  // last slot.  With internal friction (D, Kelvin-Voigt, retardation time td), a segment's stretch uses
  // (len - l) + td d(len)/dt and a joint's moment K (u - uhat + td du/dt), where
  // du/dt = (rw (w_{j+1} - w_j) + rv x (w_{j+1} + w_j)) / lbar for the relative rotation
  // r = conj(q_j) q_{j+1}; vl and wn are the exchanged neighbour velocities.
  template <bool D = false, bool M = false>
  __device__ __forceinline__ void forces(Mailbox<W, M>& mb, int& par, V3 xl, V3 xll, Q4 qn, Q4 qnl,
                                         V3 (&F)[E],
                                         V3 (&T)[E], V3 (&Ev)[E], V3& fs0, V3& enext,
                                         float td = 0.f, V3 vl = {0.f, 0.f, 0.f},
                                         V3 wn = {0.f, 0.f, 0.f}) const {
    V3 tn_prev = {0.f, 0.f, 0.f};
    fs0 = {0.f, 0.f, 0.f};
#pragma unroll
    for (int e = 0; e < E; ++e) {
      // segment vector from both parts: the high parts of neighbouring points differ by little
      // (their difference is exact or nearly so), then the low parts are added
      const V3 xa = (e == 0) ? xl : X[e - 1];
      const V3 xal = (e == 0) ? xll : XL[e - 1];
      const V3 d = (X[e] - xa) + (XL[e] - xal);
      Ev[e] = d;
      const float len2 = dot(d, d);
      const float il = rsqrtf(len2);
      const V3 t = il * d;
      const Q4 q = Qf[e];
      const float ww = q.w * q.w, xx = q.x * q.x, yy = q.y * q.y, zz = q.z * q.z;
      const float xy = q.x * q.y, xz = q.x * q.z, yz = q.y * q.z;
      const float wx = q.w * q.x, wy = q.w * q.y, wz = q.w * q.z;
      const V3 d1 = {ww + xx - yy - zz, 2.f * (xy + wz), 2.f * (xz - wy)};
      const V3 d2 = {2.f * (xy - wz), ww - xx + yy - zz, 2.f * (yz + wx)};
      const V3 d3 = {2.f * (xz + wy), 2.f * (yz - wx), ww - xx - yy + zz};
      const float lkp = P[P_LKP][e];
      const float td3 = dot(t, d3);
      V3 f = (lkp * il) * fnma3(td3, t, d3);                     // penalty, eq. (8)
      const float len = len2 * il;
      float sd = len - P[P_LEN][e];
      if constexpr (D) sd = fmaf(td, dot(t, Vv[e] - ((e == 0) ? vl : Vv[e - 1])), sd);
      f = fnma3(P[P_KS_L][e] * sd, t, f);                         // stretch, eq. (2)
      f = sel(ok[e], f, V3{0.f, 0.f, 0.f});                      // force on point j+1
      const V3 tpen = {-lkp * dot(d2, t), lkp * dot(d1, t), 0.f};  // l K_p e_3 x R^T t
      const Q4 qb = (e == E - 1) ? qn : Qf[e + 1];
      const Q4 qbl = (e == E - 1) ? qnl : QL[e + 1];
      const Q4 ql = QL[e];
      // q_{j+1} - q_j from both parts (neighbouring frames differ by little)
      const Q4 dq = {(qb.w - q.w) + (qbl.w - ql.w), (qb.x - q.x) + (qbl.x - ql.x),
                     (qb.y - q.y) + (qbl.y - ql.y), (qb.z - q.z) + (qbl.z - ql.z)};
      const float rw = q.w * qb.w + q.x * qb.x + q.y * qb.y + q.z * qb.z;
      const V3 va = {q.x, q.y, q.z}, dv = {dq.x, dq.y, dq.z};
      const V3 rv = {q.w * dv.x - dq.w * va.x - (va.y * dv.z - va.z * dv.y),
                     q.w * dv.y - dq.w * va.y - (va.z * dv.x - va.x * dv.z),
                     q.w * dv.z - dq.w * va.z - (va.x * dv.y - va.y * dv.x)};  // vec(conj(q_j) (x) q_{j+1})
      V3 m = {P[P_C1][e] * rv.x - P[P_D0][e], P[P_C1][e] * rv.y - P[P_D1][e],
              P[P_C3][e] * rv.z - P[P_D2][e]};                   // K (u - uhat)
      if constexpr (D) {   // + td K du/dt (P_C = 2 K / lbar)
        const V3 wj = Om[e];
        const V3 wb = (e == E - 1) ? wn : Om[e + 1];
        const V3 gs = fma3(rw, wb - wj, cross(rv, wb + wj));   // lbar du/dt
        const float h = 0.5f * td;
        m = {fmaf(h * P[P_C1][e], gs.x, m.x), fmaf(h * P[P_C1][e], gs.y, m.y),
             fmaf(h * P[P_C3][e], gs.z, m.z)};
      }
      const V3 rxm = cross(rv, m);
      const V3 tj = sel(ok[e], fma3(rw, m, rxm), V3{0.f, 0.f, 0.f});   // on frame j
      const V3 tn = sel(ok[e], fnma3(rw, m, rxm), V3{0.f, 0.f, 0.f});  // on frame j+1
      F[e] = f;
      if (e == 0) fs0 = f;
      else F[e - 1] = F[e - 1] - f;                              // reaction on point j
      T[e] = (tpen + tj) + tn_prev;
      tn_prev = tn;
    }
    float mh[3] = {tn_prev.x, tn_prev.y, tn_prev.z};
    float ml[6] = {fs0.x, fs0.y, fs0.z, Ev[0].x, Ev[0].y, Ev[0].z};
    const float base[3] = {0.f, 0.f, 0.f};   // no joint below frame 0
    float lo[3], hi[6];
    exchange<W, E, 3, 6, false, M>(mh, lo, ml, hi, base, mb, par);
    T[0] = T[0] + V3{lo[0], lo[1], lo[2]};
    F[E - 1] = F[E - 1] - V3{hi[0], hi[1], hi[2]};
    enext = {hi[3], hi[4], hi[5]};
  }

  // V: integrate forces (points as particles) and torques (frames as rigid bodies).
  __device__ __forceinline__ void integrate_forces(const RodDev& rd, const V3 (&F)[E],
                                                   const V3 (&T)[E], V3 fs0, V3 xc, V3 wc,
                                                   const float* __restrict__ fext,
                                                   const float* __restrict__ text) {
    const V3 grav = {rd.g[0], rd.g[1], rd.g[2]};
#pragma unroll
    for (int e = 0; e < E; ++e) {
      V3 Fe = F[e];
      V3 tau = T[e];
      if (rd.has_ext && ok[e]) {
        const float* pf = fext + 3 * (rd.pt_off + off + j0 + e + 1);
        const float* pt = text + 3 * (rd.fr_off + off + j0 + e);
        Fe = Fe + V3{pf[0], pf[1], pf[2]};
        tau = tau + V3{pt[0], pt[1], pt[2]};
      }
      const V3 a = fma3(P[P_WINV][e], Fe, fnma3(rd.damp_lin, Vv[e], grav));
      Vv[e] = fma3(dt, a, Vv[e]);
      const V3 o = Om[e];
      const float i1 = P[P_IINV1][e], i3 = P[P_IINV3][e], kg = P[P_GYRO][e];
      const V3 al = {i1 * tau.x - kg * o.y * o.z - rd.damp_ang * o.x,
                     i1 * tau.y + kg * o.x * o.z - rd.damp_ang * o.y,
                     i3 * tau.z - rd.damp_ang * o.z};
      Om[e] = fma3(dt, al, o);
    }
    if (g == 0) {
      if (ghost) {
        bv = {0.f, 0.f, 0.f};                                  // fixed halo-edge point
      } else if (rd.clamp) {
        bv = (1.0f / dt) * ((xc - bx) - bxl);
        Om[0] = wc;
      } else {
        V3 Fb = V3{0.f, 0.f, 0.f} - fs0;
        if (rd.has_ext) {
          const float* pf = fext + 3 * rd.pt_off;
          Fb = Fb + V3{pf[0], pf[1], pf[2]};
        }
        bv = fma3(dt, fma3(rd.winv0, Fb, fnma3(rd.damp_lin, bv, grav)), bv);
      }
    }
  }

  // One red-black half-sweep h of the distance impulses.  If dsnap is given, the segment
  // vector d of the slot's segment in this half-sweep is saved (for the adjoint).
  template <bool M>
  __device__ __forceinline__ void half_sweep(const RodDev& rd, Mailbox<W, M>& mb, int& par, int h,
                                             const V3 (&Ev)[E], V3 enext, V3* dsnap) {
    const bool cross_lanes = (E % 2 == 1) || (h == 0);
    V3 vlo = {0.f, 0.f, 0.f}, vhi = {0.f, 0.f, 0.f};
    if (cross_lanes) {
      float mh[3] = {Vv[E - 1].x, Vv[E - 1].y, Vv[E - 1].z};
      float ml[3] = {Vv[0].x, Vv[0].y, Vv[0].z};
      const float base[3] = {bv.x, bv.y, bv.z};
      float lo[3], hi[3];
      exchange<W, E, 3, 3, true, M>(mh, lo, ml, hi, base, mb, par);
      vlo = {lo[0], lo[1], lo[2]};
      vhi = {hi[0], hi[1], hi[2]};
      if (!M && g == 0) vlo = bv;
    }
    V3 dvb = {0.f, 0.f, 0.f};
    V3 nv[E];
    if constexpr (E % 2 == 0) {
      // Even E: slot e has the parity of e (lane and window starts are even).  Half-sweep 1
      // pairs slots (0, 1), (2, 3), ..., half-sweep 0 pairs (1, 2), (3, 4), ...: the two slots
      // of a pair are the ends of one segment, whose impulse is computed once from the
      // operands both ends would use (slot a's next-segment coefficients are slot a + 1's own),
      // so the result is the same as computing it at each end.  In half-sweep 0 slots 0 and
      // E - 1 act on the segments that cross to the lanes below and above.
      auto pair = [&](int a) {   // the segment between slots a and a + 1 (slot a + 1's)
        const V3 d = fma3(dt, Vv[a + 1] - Vv[a], Ev[a + 1]);
        const V3 im = impulse_d(d, P[P_CI][a + 1], P[P_CIL][a + 1]);
        nv[a] = fma3(P[P_WINV][a], im, Vv[a]);
        nv[a + 1] = fnma3(P[P_WINV][a + 1], im, Vv[a + 1]);
        if (dsnap) {
          dsnap[a] = d;
          dsnap[a + 1] = d;
        }
      };
      if (h == 0) {
        const V3 d0 = fma3(dt, Vv[0] - vlo, Ev[0]);
        const V3 im0 = impulse_d(d0, P[P_CI][0], P[P_CIL][0]);
        nv[0] = fnma3(P[P_WINV][0], im0, Vv[0]);
        if (dsnap) dsnap[0] = d0;
        dvb = P[P_WINV_PREV][0] * im0;   // base point: left end of segment 0
        imp0 = imp0 + im0;
#pragma unroll
        for (int a = 1; a + 1 < E; a += 2) pair(a);
        const V3 dl = fma3(dt, vhi - Vv[E - 1], enext);
        const V3 iml = impulse_d(dl, P[P_CI_NEXT][E - 1], P[P_CIL_NEXT][E - 1]);
        nv[E - 1] = fma3(P[P_WINV][E - 1], iml, Vv[E - 1]);
        if (dsnap) dsnap[E - 1] = dl;
      } else {
#pragma unroll
        for (int a = 0; a < E; a += 2) pair(a);
      }
#pragma unroll
      for (int e = 0; e < E; ++e) Vv[e] = nv[e];
      if (g == 0 && h == 0 && !rd.clamp && !ghost) bv = bv + dvb;
      return;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int j = j0 + e;
      const bool is_hi = ((j & 1) == h);   // slot is the right end of segment j
      const float w_me = P[P_WINV][e];
      // as right end of segment j (partner: point j) or left end of segment j+1
      // (partner: point j+2); only one of the two is live for even E
      const V3 v_lo = (e == 0) ? vlo : Vv[e - 1];
      const V3 v_hi = (e == E - 1) ? vhi : Vv[e + 1];
      const V3 e_next = (e == E - 1) ? enext : Ev[e + 1];
      const V3 d_hi = fma3(dt, Vv[e] - v_lo, Ev[e]);
      const V3 d_lo = fma3(dt, v_hi - Vv[e], e_next);
      const V3 im_hi = impulse_d(d_hi, P[P_CI][e], P[P_CIL][e]);
      const V3 im_lo = impulse_d(d_lo, P[P_CI_NEXT][e], P[P_CIL_NEXT][e]);
      nv[e] = sel(is_hi, fnma3(w_me, im_hi, Vv[e]), fma3(w_me, im_lo, Vv[e]));
      if (dsnap) dsnap[e] = sel(is_hi, d_hi, d_lo);
      if (e == 0) dvb = P[P_WINV_PREV][e] * im_hi;   // base point: left end of segment 0
      if (e == 0 && h == 0) imp0 = imp0 + im_hi;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) Vv[e] = nv[e];
    if (g == 0 && h == 0 && !rd.clamp && !ghost) bv = bv + dvb;
  }

  // Candidate lists of the slots (see kEnvCand): where each was built and its length, in HBM
  // between launches and in LDS (lc, one float4 per slot) during one; lr: the slots' sphere
  // radii, in LDS for the launch.
  __device__ __forceinline__ void env_load(const RodDev& rd, float4* lc, float* lr) const {
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (ok[e]) {
        lc[j0 + e] = rd.env_cache[rd.slot_off + off + j0 + e];
        lr[j0 + e] = rd.rho[rd.slot_off + off + j0 + e];
      }
  }
  __device__ __forceinline__ void env_store(const RodDev& rd, const float4* lc) const {
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (ok[e]) rd.env_cache[rd.slot_off + off + j0 + e] = lc[j0 + e];
  }

  // Environment collision detection from the step-start positions (points 1..n).  Each thread
  // reads and writes only its own slots' entries of lc and lr.
  __device__ __forceinline__ void env_detect(const RodDev& rd, float4* lc, const float* lr) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      en[e] = {0.f, 0.f, 0.f};
      ed[e] = 0.f;
      if (!ok[e]) continue;
      const int slot = rd.slot_off + off + j0 + e;
      const float r = lr[j0 + e];
      const V3 c = X[e], cl = XL[e];
      int2* list = rd.env_cand + (size_t)slot * kEnvCand;
      V3 acc = {0.f, 0.f, 0.f};
      float dmax = 0.f;
      const float4 cp = lc[j0 + e];
      const int have = __float_as_int(cp.w);
      const V3 mv = c - V3{cp.x, cp.y, cp.z};
      const float moved2 = dot(mv, mv);
      if (moved2 > (kEnvMargin * r) * (kEnvMargin * r)) {   // rebuild the list here
        const float reach = (1.f + kEnvMargin) * r;
        int cnt = 0;
        env_walk(rd, c, reach, [&](int k) {
          const float dist = env_hit(rd.env_tris[k], c, cl, r, acc, dmax);
          if (dist < reach) {
            if (cnt < kEnvCand) list[cnt] = make_int2(k, __float_as_int(dist));
            ++cnt;
          }
        });
        lc[j0 + e] = make_float4(c.x, c.y, c.z, __int_as_float(cnt));
      } else if (have <= kEnvCand) {
        // a candidate can touch the sphere only if its build distance, less the movement since
        // (and a rounding margin), is below r; four entries at a time: one load of the entries,
        // then the triangles that can touch together
        const float moved = sqrtf(moved2);
        for (int k0 = 0; k0 < have; k0 += 4) {
          const int4 e01 = *reinterpret_cast<const int4*>(list + k0);
          const int4 e23 = *reinterpret_cast<const int4*>(list + k0 + 2);
          const int id[4] = {e01.x, e01.z, e23.x, e23.z};
          const float db[4] = {__int_as_float(e01.y), __int_as_float(e01.w), __int_as_float(e23.y),
                               __int_as_float(e23.w)};
          bool near[4];
          EnvTri t[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            near[u] = k0 + u < have && db[u] - moved < r * (1.f + 1e-5f) + 1e-5f * db[u];
            if (near[u]) t[u] = rd.env_tris[id[u]];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (near[u]) env_hit(t[u], c, cl, r, acc, dmax);
        }
      } else {
        env_walk(rd, c, r, [&](int k) { env_hit(rd.env_tris[k], c, cl, r, acc, dmax); });
      }
      env_finish(acc, dmax, en[e], ed[e]);
    }
    bool mine = false;
#pragma unroll
    for (int e = 0; e < E; ++e) mine = mine || ed[e] > 0.f;
    env_any = __ballot(mine) != 0ull;
  }

  // Collision response impulses (after a constraint iteration's distance sweeps): a point whose
  // predicted motion along n falls short of its depth is pushed out, with Coulomb friction
  // against its tangential velocity, at most mu times the normal impulse.
  __device__ __forceinline__ void env_impulses(const RodDev& rd) {
    if (!env_any) return;   // nothing of this wavefront touches the mesh (a uniform branch)
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const V3 n = en[e];
      const V3 v = Vv[e];
      const float vn = dot(v, n);
      const float sep = fmaf(dt, vn, -ed[e]);
      const float w = P[P_WINV][e];
      if (ed[e] > 0.f && sep < 0.f && w > 0.f) {
        const float dvn = -sep / dt;                   // w lambda: the normal velocity change
        const V3 vt = fnma3(vn, n, v);
        const float vtl2 = dot(vt, vt);
        V3 nv = fma3(dvn, n, v);
        if (vtl2 > 0.f) {
          const float il = rsqrtf(vtl2);
          const float dvt = fminf(vtl2 * il, rd.env_mu * dvn);   // w times the friction impulse
          nv = fnma3(dvt * il, vt, nv);
        }
        Vv[e] = nv;
      }
    }
  }

  // X: integrate velocities (semi-implicit Euler), renormalise, impose the clamp pose.
  __device__ __forceinline__ void integrate_velocities(const RodDev& rd, V3 xc, Q4 qc) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      advance_position(X[e], XL[e], Vv[e], dt);
      advance_quat(Qf[e], QL[e], Om[e], dt);
    }
    if (g == 0 && !ghost) {
      if (rd.clamp) {
        bx = xc;
        bxl = {0.f, 0.f, 0.f};
        Qf[0] = qc;
        QL[0] = {0.f, 0.f, 0.f, 0.f};
      } else {
        advance_position(bx, bxl, bv, dt);
      }
    }
  }
};

// Prescribed clamp pose of step s (global step index steps_done + s), evaluated kClampChunk
// steps at a time, one step per lane (g: the lane within the rod), into LDS.  Must be reached
// by every thread; any_driven (uniform over the workgroup) says whether any rod in the
// workgroup has a driven clamp, i.e. whether the chunk barriers are taken.
template <int W>
__device__ __forceinline__ void clamp_for_step(const RodDev& rd, float (*cbuf)[10], int s,
                                               int n_steps, long long steps_done, V3& xc, Q4& qc,
                                               V3& wc, bool any_driven, int g) {
  if (!any_driven) return;
  const bool mine = rd.driven && rd.clamp;
  const int cs = s % kClampChunk;
  if (cs == 0) {
    __syncthreads();
    if (mine && g < kClampChunk && s + g < n_steps) {
      V3 pxc, pwc;
      Q4 pqc;
      clamp_pose(rd, rd.t0 + (double)(steps_done + s + g + 1) * rd.dt_d, pxc, pqc, pwc);
      float* c = cbuf[g];
      c[0] = pxc.x; c[1] = pxc.y; c[2] = pxc.z;
      c[3] = pqc.w; c[4] = pqc.x; c[5] = pqc.y; c[6] = pqc.z;
      c[7] = pwc.x; c[8] = pwc.y; c[9] = pwc.z;
    }
    __syncthreads();
  }
  if (!mine) return;
  const float* c = cbuf[cs];
  xc = {c[0], c[1], c[2]};
  qc = {c[3], c[4], c[5], c[6]};
  wc = {c[7], c[8], c[9]};
}

// Forward kernel: steps one rod per workgroup n_steps times with the state in registers.
// traj (nullable): the whole-handle state at the start of step s < traj_steps is written to
// traj + s * traj_stride in the contiguous layout of state_at (traj_steps = 1 writes a
// checkpoint of the launch's initial state).
// tips (nullable): x_N after step s goes to tips[(rod * tip_steps + steps_done - tip_base + s) * 3].
// store_final = 0 leaves gx..gw untouched (a recomputation that only needs traj).
template <int W, int E, int F = 0>
__global__ __launch_bounds__(64 * W) void rod_resident_kernel(
    const RodDev* __restrict__ rods, const int* __restrict__ rod_ids, const float* __restrict__ prm,
    int prm_stride, StateArrays st, const float* __restrict__ fext,
    const float* __restrict__ text, int n_steps, long long steps_done, int* __restrict__ status,
    float* __restrict__ traj,
    long long traj_stride, int n_pts, int n_frames, float* __restrict__ tips, int tip_steps,
    long long tip_base, int traj_steps, int store_final) {
  __shared__ Mailbox<W, kMergedExchange<W, E>> mb;
  mailbox_init(mb);
  __shared__ float cbuf[kClampChunk][10];
  const int rod = rod_ids[blockIdx.x];
  const RodDev rd = rods[rod];
  RodLane<W, E> L;
  L.load_params(rd, prm, prm_stride);
  L.load_state(rd, st);
  __shared__ float4 lcand[(F & kFeatEnv) ? 64 * W * E : 1];
  __shared__ float lrad[(F & kFeatEnv) ? 64 * W * E : 1];
  if (F & kFeatEnv) L.env_load(rd, lcand, lrad);
  int par = 0;
  V3 xc = {rd.cx0[0], rd.cx0[1], rd.cx0[2]}, wc = {0.f, 0.f, 0.f};
  Q4 qc = {rd.cq0[0], rd.cq0[1], rd.cq0[2], rd.cq0[3]};
  const int tip_lane = (rd.n - 1) / E, tip_e = (rd.n - 1) % E;
  // haptic mailbox: records cover windows of hstride steps (the last one of a launch may be
  // shorter); the pose is taken at the clamp of each window's first step.  Lanes 0..6 of wave 0
  // hold one pose word each, loaded a whole window before it is needed.
  HapticBox* const hb = (F & kFeatHaptic) ? rd.hbox : nullptr;   // the mailbox variant only
  const int hk = rd.hstride;
  uint32_t htag = 0;   // pose number in use (0: the rod's own clamp pose)
  int hn = 0;          // steps in the current window
  uint64_t pw = 0;
  if (hb && L.g < 7)
    pw = mailbox_load(&hb->pose[L.g]);

  for (int s = 0; s < n_steps; ++s) {
    if (traj && s < traj_steps) {
      L.store_state(rd, state_at(traj + (long long)s * traj_stride, n_pts, n_frames));
    }
    if (F & kFeatEnv) L.env_detect(rd, lcand, lrad);   // environment collisions (Fig. 5: detection first)
    V3 xl, xll, vl, wn;
    Q4 qn, qnl;
    L.template exchange_a<(F & kFeatDamp) != 0>(mb, par, xl, xll, qn, qnl, vl, wn);
    V3 Fo[E], T[E], Ev[E], fs0, enext;
    L.template forces<(F & kFeatDamp) != 0>(mb, par, xl, xll, qn, qnl, Fo, T, Ev, fs0, enext,
                                            rd.damp_int, vl, wn);
    clamp_for_step<W>(rd, cbuf, s, n_steps, steps_done, xc, qc, wc, rd.driven && rd.clamp, L.g);
    const bool hfirst = hb && hn == 0;
    if (hfirst && L.g < 64) {   // wave 0, all lanes: take the pose if whole and new
      const uint32_t tag = (uint32_t)(pw >> 32);
      const int word = (int)(uint32_t)pw;
      const uint32_t tag0 = __builtin_amdgcn_readfirstlane(tag);
      const bool whole = (__ballot(L.g < 7 && tag == tag0) & 0x7full) == 0x7full;
      if (whole && tag0 != htag) {
        htag = tag0;
        auto lane = [&](int k) { return __int_as_float(__builtin_amdgcn_readlane(word, k)); };
        xc = {lane(0), lane(1), lane(2)};
        qc = {lane(3), lane(4), lane(5), lane(6)};
      }
      if (L.g < 7 && s + hk < n_steps)   // the next window's pose
        pw = mailbox_load(&hb->pose[L.g]);
    }
    L.integrate_forces(rd, Fo, T, fs0, xc, wc, fext, text);
    // momentum the base point receives over the window: internal force x dt, plus segment 0's
    // constraint impulses (accumulated by the sweeps)
    L.imp0 = fnma3(rd.dt, fs0, hn == 0 ? V3{0.f, 0.f, 0.f} : L.imp0);
    for (int it = 0; it < rd.n_iter; ++it) {
      L.half_sweep(rd, mb, par, 0, Ev, enext, nullptr);
      L.half_sweep(rd, mb, par, 1, Ev, enext, nullptr);
      if (F & kFeatEnv) L.env_impulses(rd);   // then the collision response (Fig. 5)
    }
    if ((F & kFeatEnv) && rd.n_iter == 0) L.env_impulses(rd);   // without iterations: once
    L.integrate_velocities(rd, xc, qc);
    if (hb) {
      ++hn;
      if (hn == hk || s + 1 == n_steps) {   // window done: mean force of the rod on its base
        if (L.g == 0) {
          const V3 f = (1.0f / ((float)hn * rd.dt)) * L.imp0;
          const uint64_t tag = (uint64_t)(uint32_t)(steps_done + s + 1) << 32;
          const uint32_t rec[5] = {__float_as_uint(f.x), __float_as_uint(f.y), __float_as_uint(f.z),
                                   htag, (uint32_t)hn};
#pragma unroll
          for (int k = 0; k < 5; ++k)
            mailbox_store(&hb->fb[k], tag | rec[k]);
        }
        hn = 0;
      }
    }
    if (tips && (int)threadIdx.x == tip_lane) {
#pragma unroll
      for (int e = 0; e < E; ++e)
        if (e == tip_e) {
          float* pt = tips + ((long long)rod * tip_steps + steps_done - tip_base + s) * 3;
          pt[0] = L.X[e].x; pt[1] = L.X[e].y; pt[2] = L.X[e].z;
        }
    }
  }
  if (F & kFeatEnv) L.env_store(rd, lcand);
  if (store_final) {
    const float chk = L.store_state(rd, st);
    if (!__builtin_isfinite(chk)) atomicOr(status, 1);
  }
}

// ---------------------------------------------------------------------------------------
// Groups of one or two rods per workgroup, for the constraints that couple points across rods
// or far apart along one rod: bindings (Sec. 2.1 "Constraints": distance constraints of rest
// length zero between points of two rods; Sec. 3.4 variants 1 and 2) and sphere contact with
// Coulomb friction (Sec. 2.2 "Collisions and self-collisions").  Threads [0, 64 W) step the
// group's first rod and [64 W, 128 W) the second, each exactly as rod_resident_kernel steps
// one rod; a single rod leaves the second half idle (a rod of no elements taking the same
// barriers).  Both rods have the same number of constraint iterations.
//   Step start: every point writes its position (both floats of the pair) and sphere radius
//   to LDS; separations between points of the group are taken as (x_i - x_j) + (l_i - l_j),
//   and the contact test and separation from them by sphere_gap, so that the compensated
//   positions decide contacts, alike on both sides of a pair.  With contact
//   (compiled in when CT), every point then lists (in (rod, point) order, at most
//   kMaxContacts) the points whose spheres overlap its own, leaving out points of its own rod
//   within self_skip of it.  It takes them from a candidate list (at most kContactCand
//   points, same order) of the points that were within contact distance + margin of it when
//   the list was built; the lists are rebuilt, for the whole group, only when some point has
//   moved more than 0.45 x margin since, so every contact is among the candidates and the
//   contacts found are exactly those of a scan of all points.  A build groups 8 consecutive
//   points into a bounding sphere (one thread each), marks the pairs of spheres that come
//   within the margin of each other, and scans the points of those spheres; a point with too
//   many candidates falls back to its exact contacts and forces a new build next step.  The
//   build positions and lists are kept in device memory between launches.
//   Every constraint iteration, after the distance sweeps: points publish velocity and inverse
//   mass; bound points apply the zero-length distance impulse (two-way, or one-way with the
//   second rod the master); then, with contact, points publish again and every point applies
//   the mean of its active contacts' impulses, computed from the published values: a normal
//   impulse removing the predicted penetration along the step-start normal and a friction
//   impulse opposing the relative tangential velocity, at most mu times the normal one.
constexpr int kMaxContacts = 8;    // contacts per point (more sets status bit 8)
constexpr int kContactCand = 16;   // candidate partners per point kept between list builds
constexpr int kSphereSize = 8;     // points per bounding sphere
// slack [m] of the fallback's FP32 candidate test over the exact contact test (sphere_gap)
constexpr float kExactSlack = 1e-6f;

struct GroupDev {
  int32_t rod[2];      // rod[1] = -1: a single rod
  int32_t bind_mode;   // 0 none, 1 one-way (rod[1] is the master), 2 two-way
  int32_t contact;     // 1: sphere contact between and within the group's rods
  float mu;            // friction coefficient
  float margin;        // contact candidates: pairs within contact distance + margin [m]
};

// 16-bit entry k (0..3) of a quad of list entries
__device__ __forceinline__ int quad_get(uint2 q, int k) {
  const uint32_t w = k < 2 ? q.x : q.y;
  return (int)((k & 1) ? w >> 16 : w & 0xffffu);
}
__device__ __forceinline__ void quad_put(uint2& q, int k, uint32_t v) {
  uint32_t& w = k < 2 ? q.x : q.y;
  w = (k & 1) ? ((w & 0xffffu) | (v << 16)) : ((w & 0xffff0000u) | v);
}

// Gap |d| - D between two spheres whose radii sum to D (ri + rj) and whose centres are the
// compensated positions xi + li and xj + lj; d returns the centre difference (rounded, for
// the normal).  Resting contact keeps |d| within a step's sinking (g dt^2, often below
// 1e-8 m) of D, where the difference of two FP32 lengths would carry an error of ulp(D):
// instead the centre difference is formed in FP64 (exact for these float operands), |d|^2 -
// D^2 in FP64, and the gap is that over |d| + D, to FP32 precision of the gap itself.  (FP64
// fused multiply-adds issue at the rate of the unpacked FP32 ones this library uses.)
__device__ __forceinline__ float sphere_gap(V3 xi, V3 li, V3 xj, V3 lj, float ri, float rj,
                                            V3& d) {
  const double dx = ((double)xi.x - (double)xj.x) + ((double)li.x - (double)lj.x);
  const double dy = ((double)xi.y - (double)xj.y) + ((double)li.y - (double)lj.y);
  const double dz = ((double)xi.z - (double)xj.z) + ((double)li.z - (double)lj.z);
  d = {(float)dx, (float)dy, (float)dz};
  const double S = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
  const double D = (double)ri + (double)rj;
  return (float)__builtin_fma(-D, D, S) / (sqrtf((float)S) + (float)D);
}

template <int W, int E, bool CT>
__global__ __launch_bounds__(128 * W) void rod_group_kernel(
    const RodDev* __restrict__ rods, const GroupDev* __restrict__ groups,
    const int* __restrict__ partner, const float* __restrict__ rho_slot,
    float4* __restrict__ cbuild, uint16_t* __restrict__ ccand,
    const float* __restrict__ prm, int prm_stride, StateArrays st,
    const float* __restrict__ fext, const float* __restrict__ text, int n_steps,
    long long steps_done, int* __restrict__ status) {
  constexpr int CAP = 64 * W * E;                                   // slots per rod
  constexpr int CC = CT ? CAP : 1;                                  // contact-list slots
  constexpr int SMAX = CT ? 2 * ((CAP + kSphereSize - 1) / kSphereSize) : 1;  // spheres
  constexpr int SW = (SMAX + 31) / 32;
  __shared__ Mailbox<W, false> mb[2];   // two rods per workgroup: the plain exchange
  __shared__ float cbuf[2][kClampChunk][10];
  // step-start position and sphere radius, and the low parts of the position (the positions
  // are pairs of floats; separations between points take both); rewritten at every step start
  // after a barrier, so that no wavefront still reads the previous step's
  __shared__ float4 xs[2][CAP];
  __shared__ float4 xsl[2][CAP];
  // velocity and inverse mass, double-buffered by publication parity: the reads after one
  // publication and the writes two publications later are separated by a barrier
  __shared__ float4 vw[2][2][CAP];
  __shared__ float4 sph[SMAX];                            // bounding spheres: centre, radius
  __shared__ uint32_t sov[SMAX][SW];                      // sphere pairs within the margin
  // candidates (sub * CAP + slot) and this step's contacts, four 16-bit entries per quad,
  // quad-major so that a wavefront reads consecutive quads
  __shared__ uint2 cand[2][kContactCand / 4][CC];
  __shared__ uint2 lst[2][kMaxContacts / 4][CC];
  // the gap |d| - D of each listed contact, stored once per step where LDS has room (a group
  // of one or two wavefronts per rod); the larger shape recomputes it in every iteration
  constexpr bool GC = CT && W <= 2;
  __shared__ float gapc[2][GC ? kMaxContacts : 1][GC ? CC : 1];
  __shared__ float4 xbl[2][CC];      // each point's position when its candidates were listed
  __shared__ int moved[2][2 * W];                         // per wavefront and step parity
  __shared__ int touching[2][2 * W];                      // ditto: some point has a contact
  const GroupDev gp = groups[blockIdx.x];
  const int sub = threadIdx.x >= 64 * W ? 1 : 0;
  const bool active = gp.rod[sub] >= 0;
  RodDev rd = rods[active ? gp.rod[sub] : gp.rod[0]];
  if (!active) rd.n = 0;   // idle half: no slots, same barriers
  const RodDev& r0 = rods[gp.rod[0]];
  bool any_driven = r0.driven && r0.clamp;
  int nrod[2] = {r0.n, 0};
  if (gp.rod[1] >= 0) {
    const RodDev& r1 = rods[gp.rod[1]];
    any_driven = any_driven || (r1.driven && r1.clamp);
    nrod[1] = r1.n;
  }
  const bool moved_rod = !(gp.bind_mode == 1 && sub == 1);
  const bool contact = CT && gp.contact != 0;
  RodLane<W, E> L;
  L.load_params(rd, prm, prm_stride);
  L.load_state(rd, st);
  int part[E], cnt[E], ncand[E];
  float rho[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    part[e] = (L.ok[e] && gp.bind_mode) ? partner[rd.slot_off + L.j0 + e] : -1;
    rho[e] = L.ok[e] ? rho_slot[rd.slot_off + L.j0 + e] : 0.f;
    cnt[e] = 0;
    ncand[e] = 0;
  }
  if (contact) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (!L.ok[e]) continue;
      const int i = L.j0 + e, gs = rd.slot_off + i;
      const float4 b = cbuild[gs];   // NaN position: no valid list
      xbl[sub][i] = b;
      ncand[e] = min(max(__float_as_int(b.w), 0), kContactCand);
      for (int c = 0; c < ncand[e]; ++c)
        quad_put(cand[sub][c >> 2][i], c & 3, ccand[(size_t)gs * kContactCand + c]);
    }
  }
  const int skip = rd.self_skip;
  const float reb2 = (0.45f * gp.margin) * (0.45f * gp.margin);
  const int s0 = (nrod[0] + kSphereSize - 1) / kSphereSize;
  const int ns = s0 + (nrod[1] + kSphereSize - 1) / kSphereSize;
  int par = 0;
  V3 xc = {rd.cx0[0], rd.cx0[1], rd.cx0[2]}, wc = {0.f, 0.f, 0.f};
  Q4 qc = {rd.cq0[0], rd.cq0[1], rd.cq0[2], rd.cq0[3]};
  const float dt = rd.dt;
  int bpar = 0;
  bool overflow = false;
  bool touch = false;   // some point of the group has a contact this step
  auto publish = [&]() {
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (L.ok[e]) vw[bpar][sub][L.j0 + e] = make_float4(L.Vv[e].x, L.Vv[e].y, L.Vv[e].z, L.P[P_WINV][e]);
    __syncthreads();
  };
  // candidates of slot e's point: points of overlapping spheres (sov) within contact distance
  // + mm, in (rod, point) order; returns how many there are (only the first kContactCand kept)
  auto scan = [&](int e, float mm) {
    const int i = L.j0 + e;
    const int own = sub * s0 + i / kSphereSize;
    const V3 xi = L.X[e], li = L.XL[e];
    int n = 0;
    for (int wd = 0; wd < SW; ++wd) {
      uint32_t bits = wd * 32 < ns ? sov[own][wd] : 0u;
      while (bits) {
        const int k = wd * 32 + __builtin_ctz(bits);
        bits &= bits - 1;
        const int r = k < s0 ? 0 : 1, kk = k < s0 ? k : k - s0;
        const int a = kk * kSphereSize, b = min(a + kSphereSize, nrod[r]);
        for (int j = a; j < b; ++j) {
          if (r == sub && abs(j - i) <= skip) continue;
          const float4 p = xs[r][j], pl = xsl[r][j];
          const V3 lj = {pl.x, pl.y, pl.z};
          const float dx = (xi.x - p.x) + (li.x - lj.x), dy = (xi.y - p.y) + (li.y - lj.y);
          const float dz = (xi.z - p.z) + (li.z - lj.z), D = rho[e] + p.w + mm;
          const float d2 = dx * dx + dy * dy + dz * dz;   // (the listing takes the exact test)
          if (!(d2 < D * D) || !(d2 > 0.f)) continue;
          if (n < kContactCand) quad_put(cand[sub][n >> 2][i], n & 3, (uint32_t)(r * CAP + j));
          ++n;
        }
      }
    }
    return n;
  };

  for (int s = 0; s < n_steps; ++s) {
    // ---- step start: positions and radii; contact lists
    __syncthreads();   // every wavefront is done with the previous step's xs and xsl
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (!L.ok[e]) continue;
      xs[sub][L.j0 + e] = make_float4(L.X[e].x, L.X[e].y, L.X[e].z, rho[e]);
      xsl[sub][L.j0 + e] = make_float4(L.XL[e].x, L.XL[e].y, L.XL[e].z, 0.f);
    }
    if (contact) {
      bool mv = false;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if (!L.ok[e]) continue;
        const float4 b = xbl[sub][L.j0 + e];
        const V3 d = L.X[e] - V3{b.x, b.y, b.z};
        mv = mv || !(dot(d, d) <= reb2);
      }
      const bool wmv = __ballot(mv) != 0ull;
      if ((threadIdx.x & 63) == 0) moved[s & 1][threadIdx.x >> 6] = wmv ? 1 : 0;
    }
    __syncthreads();
    if (contact) {
      bool rebuild = false;
#pragma unroll
      for (int k = 0; k < 2 * W; ++k) rebuild = rebuild || moved[s & 1][k] != 0;
      if (rebuild) {   // uniform over the workgroup
        const int t = threadIdx.x;
        if (t < ns) {
          const int r = t < s0 ? 0 : 1, k = t < s0 ? t : t - s0;
          const int a = k * kSphereSize, b = min(a + kSphereSize, nrod[r]);
          float cx = 0.f, cy = 0.f, cz = 0.f, rm = 0.f;
          for (int j = a; j < b; ++j) {
            const float4 p = xs[r][j];
            cx += p.x; cy += p.y; cz += p.z;
            rm = fmaxf(rm, p.w);
          }
          const float inv = 1.0f / (float)(b - a);
          cx *= inv; cy *= inv; cz *= inv;
          float d2 = 0.f;
          for (int j = a; j < b; ++j) {
            const float4 p = xs[r][j];
            d2 = fmaxf(d2, (p.x - cx) * (p.x - cx) + (p.y - cy) * (p.y - cy) + (p.z - cz) * (p.z - cz));
          }
          sph[t] = make_float4(cx, cy, cz, sqrtf(d2) + rm);
        }
        __syncthreads();
        // one 32-sphere word of one sphere's row per thread; neighbouring threads take
        // neighbouring rows of the same word (same sphere read by all of them)
        for (int task = t; task < ns * SW; task += 128 * W) {
          const int row = task % ns, wd = task / ns;
          const float4 me = sph[row];
          uint32_t bits = 0;
          for (int bb = 0; bb < 32; ++bb) {
            const int k = wd * 32 + bb;
            if (k < ns) {
              const float4 o = sph[k];
              const float dx = me.x - o.x, dy = me.y - o.y, dz = me.z - o.z;
              const float rr = me.w + o.w + gp.margin;
              if (dx * dx + dy * dy + dz * dz < rr * rr) bits |= 1u << bb;
            }
          }
          sov[row][wd] = bits;
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) {
          if (!L.ok[e]) continue;
          int n = scan(e, gp.margin);
          float4 b = make_float4(L.X[e].x, L.X[e].y, L.X[e].z, 0.f);
          if (n > kContactCand) {   // too many candidates: this step's exact contacts only
            n = min(scan(e, kExactSlack), kContactCand);
            b.x = __int_as_float(0x7fc00000);   // build again next step
          }
          ncand[e] = n;
          b.w = __int_as_float(n);
          xbl[sub][L.j0 + e] = b;
        }
      }
#pragma unroll
      for (int e = 0; e < E; ++e) {
        cnt[e] = 0;
        if (!L.ok[e]) continue;
        const int i = L.j0 + e;
        const V3 xi = L.X[e], li = L.XL[e];
        const float4* xsp = &xs[0][0];   // indexed by sub * CAP + slot
        const float4* xlp = &xsl[0][0];
        // four candidates at a time: one quad read, then their four position reads together
#pragma unroll
        for (int q = 0; q < kContactCand; q += 4) {
          if (q >= ncand[e]) break;
          const uint2 w = cand[sub][q >> 2][i];
          int g[4];
          float4 p[4];
          float4 pl[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) g[k] = q + k < ncand[e] ? quad_get(w, k) : quad_get(w, 0);
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            p[k] = xsp[g[k]];
            pl[k] = xlp[g[k]];
          }
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            if (q + k >= ncand[e]) break;
            const V3 lj = {pl[k].x, pl[k].y, pl[k].z};
            V3 d;
            const float gap = sphere_gap(xi, li, V3{p[k].x, p[k].y, p[k].z}, lj, rho[e], p[k].w, d);
            if (!(gap < 0.f) || !(dot(d, d) > 0.f)) continue;
            if (cnt[e] < kMaxContacts) {
              quad_put(lst[sub][cnt[e] >> 2][i], cnt[e] & 3, (uint32_t)g[k]);
              if constexpr (GC) gapc[sub][cnt[e]][i] = gap;
              ++cnt[e];
            } else {
              overflow = true;
            }
          }
        }
      }
      // the iterations' contact rounds (a publication and its barrier each) are skipped in
      // steps where no point of the group touches anything
      bool mine = false;
#pragma unroll
      for (int e = 0; e < E; ++e) mine = mine || cnt[e] > 0;
      const bool wt = __ballot(mine) != 0ull;
      if ((threadIdx.x & 63) == 0) touching[s & 1][threadIdx.x >> 6] = wt ? 1 : 0;
      __syncthreads();
      touch = false;
#pragma unroll
      for (int k = 0; k < 2 * W; ++k) touch = touch || touching[s & 1][k] != 0;
    }

    // ---- the step
    V3 xl, xll;
    Q4 qn, qnl;
    L.exchange_a(mb[sub], par, xl, xll, qn, qnl);
    V3 F[E], T[E], Ev[E], fs0, enext;
    L.forces(mb[sub], par, xl, xll, qn, qnl, F, T, Ev, fs0, enext);
    clamp_for_step<W>(rd, cbuf[sub], s, n_steps, steps_done, xc, qc, wc, any_driven, L.g);
    L.integrate_forces(rd, F, T, fs0, xc, wc, fext, text);
    for (int it = 0; it < rd.n_iter; ++it) {
      L.half_sweep(rd, mb[sub], par, 0, Ev, enext, nullptr);
      L.half_sweep(rd, mb[sub], par, 1, Ev, enext, nullptr);
      if (gp.bind_mode) {
        publish();
#pragma unroll
        for (int e = 0; e < E; ++e) {
          if (part[e] >= 0 && moved_rod) {
            const float4 ox = xs[1 - sub][part[e]];
            const float4 ov = vw[bpar][1 - sub][part[e]];
            const float4 ol = xsl[1 - sub][part[e]];
            const V3 lo = {ol.x, ol.y, ol.z};
            // predicted separation: (x - xo) + (l - lo) + dt (v - vo)
            const V3 d0 = (L.X[e] - V3{ox.x, ox.y, ox.z}) + (L.XL[e] - lo);
            const V3 d = fma3(dt, L.Vv[e] - V3{ov.x, ov.y, ov.z}, d0);
            const float wm = L.P[P_WINV][e];
            const float ws = gp.bind_mode == 2 ? wm + ov.w : wm;
            if (ws > 0.f) L.Vv[e] = fnma3(wm / (dt * ws), d, L.Vv[e]);
          }
        }
        bpar ^= 1;
      }
      if (contact && touch) {   // (uniform over the workgroup)
        publish();
#pragma unroll
        for (int e = 0; e < E; ++e) {
          if (!cnt[e]) continue;
          const int i = L.j0 + e;
          const V3 xi = L.X[e], vi = L.Vv[e], li = L.XL[e];
          const float wi = L.P[P_WINV][e];
          const float4* xsp = &xs[0][0];     // indexed by sub * CAP + slot
          const float4* xlp = &xsl[0][0];
          const float4* vwp = &vw[bpar][0][0];
          // the impulse on this point from partner (ox + its low parts oxl, ov); false if that
          // contact is inactive
          auto impulse = [&](float4 ox, float4 oxl, float4 ov, int c, V3& imp) {
            const V3 xj = {ox.x, ox.y, ox.z}, vj = {ov.x, ov.y, ov.z};
            const float wsum = wi + ov.w;
            if (!(wsum > 0.f)) return false;
            const V3 lj = {oxl.x, oxl.y, oxl.z};
            // the listing's gap (stored, or formed again alike); the normal from the centre
            // difference in FP32, the same in every shape and exactly opposite for the partner
            float gap;
            if constexpr (GC) {
              gap = gapc[sub][c][i];
            } else {
              V3 dd;
              gap = sphere_gap(xi, li, xj, lj, rho[e], ox.w, dd);
            }
            const V3 d0 = (xi - xj) + (li - lj);
            const V3 nrm = rsqrtf(dot(d0, d0)) * d0;        // step-start normal, towards i
            const V3 vr = vi - vj;
            // predicted separation along the normal: |d0| - D + dt (vi - vj).n
            const float sep = __builtin_fmaf(dt, dot(vr, nrm), gap);
            if (!(sep < 0.f)) return false;
            const float lam = -sep / (dt * wsum);
            const V3 vt = fnma3(dot(vr, nrm), nrm, vr);
            const float vtl = sqrtf(dot(vt, vt));
            imp = (wi * lam) * nrm;
            if (vtl > 0.f) imp = fnma3(wi * fminf(vtl / wsum, gp.mu * lam) / vtl, vt, imp);
            return true;
          };
          V3 acc = {0.f, 0.f, 0.f};
          int act = 0;
          // two contacts at a time (their four reads together), summed in list order
#pragma unroll
          for (int c = 0; c < kMaxContacts; c += 2) {
            if (c >= cnt[e]) break;
            const uint2 w = lst[sub][c >> 2][i];
            const int ga = quad_get(w, c & 3);
            const int gb = c + 1 < cnt[e] ? quad_get(w, (c & 3) + 1) : ga;
            const float4 oxa = xsp[ga], ova = vwp[ga], oxb = xsp[gb], ovb = vwp[gb];
            const float4 la = xlp[ga], lb = xlp[gb];
            V3 imp;
            if (impulse(oxa, la, ova, c, imp)) {
              acc = acc + imp;
              ++act;
            }
            if (c + 1 < cnt[e] && impulse(oxb, lb, ovb, c + 1, imp)) {
              acc = acc + imp;
              ++act;
            }
          }
          if (act) L.Vv[e] = fma3(1.0f / (float)act, acc, L.Vv[e]);
        }
        bpar ^= 1;
      }
    }
    L.integrate_velocities(rd, xc, qc);
  }
  if (active) {
    const float chk = L.store_state(rd, st);
    if (!__builtin_isfinite(chk)) atomicOr(status, 1);
  }
  if (contact) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (!L.ok[e]) continue;
      const int i = L.j0 + e, gs = rd.slot_off + i;
      cbuild[gs] = xbl[sub][i];
      for (int c = 0; c < ncand[e]; ++c)
        ccand[(size_t)gs * kContactCand + c] = (uint16_t)quad_get(cand[sub][c >> 2][i], c & 3);
    }
  }
  if (overflow) atomicOr(status, 8);
}

// ---------------------------------------------------------------------------------------
// Long rods: several workgroups per rod.  Chunk k owns slots [s0, s0 + c) and holds the window
// [win0, win0 + nwin) = owned slots plus a halo of H slots on each side (fewer at the rod
// ends).  Every step is computed on the whole window; the window edges perturb the slots within
// one step's dependency radius (2 n_iter + 2) of them, and that front moves inwards by the
// radius every step, so with H >= T radius the owned slots stay exact for T steps.  Every T
// steps (except after the launch's last, whose owned slots are stored and whose halos the
// next launch loads from the neighbours' stored slots) the chunk publishes its first H owned
// slots (for the left neighbour's right halo) and its last H + 1 owned slots (for the right
// neighbour's left halo and halo-edge point) to a double-buffered mailbox in global memory,
// raises its flag to the step count, waits for both neighbours' flags and refills its halos:
// one exchange per T steps instead of one per phase.
struct GridChunk {
  int32_t rod;             // rod index
  int32_t s0, c;           // owned slots
  int32_t win0, nwin;      // window slots
  int32_t left, right;     // neighbour chunk indices (-1 at the rod's ends)
  int32_t halo;            // H
  int32_t every;           // T: steps between halo exchanges (H >= T (2 n_iter + 2))
};

// Mailbox part: the 20 words (x, v of point j+1; q, w of frame j; the low parts of x and q) of
// up to pub_slots slots, word-major (word k of slot i at k pub_slots + i), so that a
// wavefront's store or load of one word covers consecutive addresses.
constexpr int kPubSlotFloats = 20;

// Mailbox words are read and written as device-scope relaxed atomics (coherent across the
// XCDs' L2 caches without writing back or invalidating them); the step flags order them.
__device__ __forceinline__ void put_coherent(float* p, float v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float get_coherent(const float* p) {
  return __hip_atomic_load(const_cast<float*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int W, int E>
__global__ __launch_bounds__(64 * W) void rod_grid_kernel(
    const RodDev* __restrict__ rods, const GridChunk* __restrict__ chunks,
    const int* __restrict__ block_chunk, const float* __restrict__ prm, int prm_stride,
    StateArrays st, const float* __restrict__ fext, const float* __restrict__ text, int n_steps,
    long long steps_done, int* __restrict__ status, float* pub, int pub_slots, int n_chunks,
    int* flags, int spin_limit) {
  __shared__ Mailbox<W, false> mb;   // the plain exchange (see kMergedExchange)
  __shared__ float cbuf[kClampChunk][10];
  __shared__ int abort_flag;
  const int ci = block_chunk[blockIdx.x];
  const GridChunk ck = chunks[ci];
  const RodDev rd = rods[ck.rod];
  RodLane<W, E> L;
  L.load_params(rd, prm, prm_stride, ck.win0, ck.nwin);
  L.load_state(rd, st);
  int par = 0;
  V3 xc = {rd.cx0[0], rd.cx0[1], rd.cx0[2]}, wc = {0.f, 0.f, 0.f};
  Q4 qc = {rd.cq0[0], rd.cq0[1], rd.cq0[2], rd.cq0[3]};
  const int own_lo = ck.s0 - ck.win0, own_hi = own_lo + ck.c;
  const int H = ck.halo;
  int xk = 0;   // halo exchanges so far in this launch
  if (threadIdx.x == 0) abort_flag = 0;
  __syncthreads();

  for (int s = 0; s < n_steps; ++s) {
    const long long gs = steps_done + s;
    V3 xl, xll;
    Q4 qn, qnl;
    L.exchange_a(mb, par, xl, xll, qn, qnl);
    V3 F[E], T[E], Ev[E], fs0, enext;
    L.forces(mb, par, xl, xll, qn, qnl, F, T, Ev, fs0, enext);
    if (ck.win0 == 0)
      clamp_for_step<W>(rd, cbuf, s, n_steps, steps_done, xc, qc, wc, rd.driven && rd.clamp, L.g);
    L.integrate_forces(rd, F, T, fs0, xc, wc, fext, text);
    for (int it = 0; it < rd.n_iter; ++it) {
      L.half_sweep(rd, mb, par, 0, Ev, enext, nullptr);
      L.half_sweep(rd, mb, par, 1, Ev, enext, nullptr);
    }
    L.integrate_velocities(rd, xc, qc);

    if ((s + 1) % ck.every != 0 || s + 1 == n_steps) continue;   // (uniform over the chunk)
    // ---- publish boundary slots: part 0 = owned [0, H), part 1 = owned [c - H - 1, c), into
    // the mailbox buffer of this launch's exchange count parity
    const int pp = xk & 1;
    ++xk;
    float* mine = pub + ((long long)(pp * n_chunks + ci) * 2) * pub_slots * kPubSlotFloats;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int o = L.j0 + e - own_lo;   // owned index
      // (with several chunks c >= 2 H + 2, so no slot is in both parts)
      const bool p0 = L.ok[e] && o >= 0 && o < H && ck.left >= 0;
      const bool p1 = L.ok[e] && o >= ck.c - H - 1 && o < ck.c && ck.right >= 0;
      if (p0 || p1) {
        float* d = p0 ? mine + o : mine + pub_slots * kPubSlotFloats + (o - (ck.c - H - 1));
        const float v[kPubSlotFloats] = {L.X[e].x,  L.X[e].y,  L.X[e].z,  L.Vv[e].x,
                                         L.Vv[e].y, L.Vv[e].z, L.Qf[e].w, L.Qf[e].x,
                                         L.Qf[e].y, L.Qf[e].z, L.Om[e].x, L.Om[e].y,
                                         L.Om[e].z, L.XL[e].x, L.XL[e].y, L.XL[e].z,
                                         L.QL[e].w, L.QL[e].x, L.QL[e].y, L.QL[e].z};
#pragma unroll
        for (int k = 0; k < kPubSlotFloats; ++k) put_coherent(d + k * pub_slots, v[k]);
      }
    }
    // this thread's mailbox stores are complete (device-visible) before the barrier, and the
    // flag is raised after it
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) {
      __hip_atomic_store(&flags[ci], (int)(gs + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      // wait for both neighbours to have published this step (bounded spin)
      int spins = 0;
      for (int side = 0; side < 2; ++side) {
        const int nb = side == 0 ? ck.left : ck.right;
        if (nb < 0) continue;
        while (__hip_atomic_load(&flags[nb], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (int)(gs + 1)) {
          __builtin_amdgcn_s_sleep(1);
          if (++spins > spin_limit) {
            abort_flag = 1;
            break;
          }
        }
      }
    }
    __syncthreads();   // the neighbours' words are read (device-coherent) only after this
    if (abort_flag) {
      if (threadIdx.x == 0) atomicOr(status, 4);
      break;
    }
    // ---- refill the halos from the neighbours' parts
    const float* lp = ck.left >= 0
        ? pub + ((long long)(pp * n_chunks + ck.left) * 2 + 1) * pub_slots * kPubSlotFloats
        : nullptr;
    const float* rp = ck.right >= 0
        ? pub + ((long long)(pp * n_chunks + ck.right) * 2) * pub_slots * kPubSlotFloats
        : nullptr;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int o = L.j0 + e - own_lo;
      const float* src = nullptr;
      if (L.ok[e] && o < 0 && lp) src = lp + (o + H + 1);   // slot s0 + o
      if (L.ok[e] && o >= ck.c && rp) src = rp + (o - ck.c);
      if (src) {
        float v[kPubSlotFloats];
#pragma unroll
        for (int k = 0; k < kPubSlotFloats; ++k) v[k] = get_coherent(src + k * pub_slots);
        L.X[e] = {v[0], v[1], v[2]};
        L.Vv[e] = {v[3], v[4], v[5]};
        L.Qf[e] = {v[6], v[7], v[8], v[9]};
        L.Om[e] = {v[10], v[11], v[12]};
        L.XL[e] = {v[13], v[14], v[15]};
        L.QL[e] = {v[16], v[17], v[18], v[19]};
      }
    }
    if (L.g == 0 && L.ghost && lp) {   // halo-edge point: point win0 = point of slot win0 - 1
      const int ps = pub_slots;
      L.bx = {get_coherent(lp), get_coherent(lp + ps), get_coherent(lp + 2 * ps)};
      L.bxl = {get_coherent(lp + 13 * ps), get_coherent(lp + 14 * ps), get_coherent(lp + 15 * ps)};
      L.bv = {get_coherent(lp + 3 * ps), get_coherent(lp + 4 * ps), get_coherent(lp + 5 * ps)};
    }
  }
  const float chk = L.store_state(rd, st, own_lo, own_hi);
  if (!__builtin_isfinite(chk)) atomicOr(status, 1);
}

}  // namespace corde
