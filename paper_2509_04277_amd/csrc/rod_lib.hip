// rod_lib.hip -- host side of libcorde_rod.so: the C ABI declared in include/rod.h.
//
// rod_create() derives every per-element coefficient of the discrete Cosserat rod (Sec. 2.1
// of the paper) in FP64 on the host and stores it as FP32 rows on the device; rod_step()
// launches the register-resident kernel of rod_kernels.hpp, one workgroup per rod, running
// steps_per_launch time steps per launch.  Everything is enqueued on the handle's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/rod.h"
#include "rod_adjoint.hpp"

using corde::RodDev;

namespace {

constexpr double kPi = 3.14159265358979323846;

using corde::StateArrays;
using KernelFn = void (*)(const RodDev*, const int*, const float*, int, StateArrays, const float*,
                          const float*, int, long long, int*, float*, long long, int, int, float*,
                          int, long long, int, int);
using GridFn = void (*)(const RodDev*, const corde::GridChunk*, const int*, const float*, int,
                        StateArrays, const float*, const float*, int, long long, int*, float*, int,
                        int, int*, int);
// Long-rod kernel shape: 4 wavefronts (one per SIMD) x 2 elements per lane = 512-slot windows.
constexpr int kGridWaves = 4, kGridElems = 2;
constexpr int kResidentMax = 2048;   // longest rod stepped by a single workgroup
constexpr int kChunkTry = 512;       // rods longer than this may be chunked by rod_autotune
constexpr int kMaxDevices = 64;       // devices of one process the library keeps state for
constexpr int kLongMax = 1 << 17;
constexpr int kMaxExchangeEvery = 16;  // most steps between two halo exchanges of a chunked rod    // longest rod accepted (its chunks must be co-resident)

using AdjointFn = void (*)(const RodDev*, const int*, const float*, int, const float*, long long,
                           int, int, int, long long, int, const float*, int, float*, float*,
                           float*, float*, double*, const float*, const float*, int*);

struct AdjointEntry {
  int waves, elems;
  AdjointFn fn;
};

// Adjoint kernel shapes (one or two elements per lane: the reverse keeps 60 snapshot values
// per element in registers).
const AdjointEntry kAdjoints[] = {
    {1, 1, corde::rod_adjoint_kernel<1, 1>}, {1, 2, corde::rod_adjoint_kernel<1, 2>},
    {2, 1, corde::rod_adjoint_kernel<2, 1>}, {2, 2, corde::rod_adjoint_kernel<2, 2>},
    {4, 1, corde::rod_adjoint_kernel<4, 1>}, {4, 2, corde::rod_adjoint_kernel<4, 2>},
    {8, 1, corde::rod_adjoint_kernel<8, 1>},
};

struct KernelEntry {
  int waves, elems;
  KernelFn fn[8];   // by feature bits (kFeatHaptic, kFeatEnv, kFeatDamp); the variants exist
                    // for the default shapes only, without environment + internal friction
};

// Built kernel shapes: (waves per rod, elements per lane).  Capacity = 64 * waves * elems.
#define ROD_SHAPE(w, e) {w, e, {corde::rod_resident_kernel<w, e, 0>}}
#define ROD_SHAPE_F(w, e)                                                                   \
  {w, e, {corde::rod_resident_kernel<w, e, 0>, corde::rod_resident_kernel<w, e, 1>,       \
          corde::rod_resident_kernel<w, e, 2>, corde::rod_resident_kernel<w, e, 3>,       \
          corde::rod_resident_kernel<w, e, 4>, corde::rod_resident_kernel<w, e, 5>}}
const KernelEntry kKernels[] = {
    ROD_SHAPE_F(1, 1), ROD_SHAPE_F(1, 2), ROD_SHAPE(1, 4),    ROD_SHAPE(1, 8),
    ROD_SHAPE(2, 1),   ROD_SHAPE_F(2, 2), ROD_SHAPE(2, 4),    ROD_SHAPE(4, 1),
    ROD_SHAPE_F(4, 2), ROD_SHAPE_F(4, 4), ROD_SHAPE_F(4, 8),  ROD_SHAPE(8, 1),
    ROD_SHAPE(8, 2),   ROD_SHAPE_F(8, 4), ROD_SHAPE(16, 1),
};
#undef ROD_SHAPE
#undef ROD_SHAPE_F

const KernelEntry* find_kernel(int w, int e) {
  for (const auto& k : kKernels)
    if (k.waves == w && k.elems == e) return &k;
  return nullptr;
}

GridFn grid_kernel() { return corde::rod_grid_kernel<kGridWaves, kGridElems>; }

using GroupFn = void (*)(const RodDev*, const corde::GroupDev*, const int*, const float*,
                         float4*, uint16_t*,
                         const float*, int, StateArrays, const float*, const float*, int,
                         long long, int*);
struct GroupEntry {
  int waves, elems;
  bool contact;   // contact compiled in (binding-only kernels leave its LDS out)
  GroupFn fn;
};
// Shapes of the rod-group kernel (bindings, contact), per rod; a workgroup holds 2 x 64 waves
// threads (at most 8 wavefronts: with 16 the register budget halves and the kernel spills).
const GroupEntry kGroups[] = {
    {1, 2, false, corde::rod_group_kernel<1, 2, false>},
    {2, 2, false, corde::rod_group_kernel<2, 2, false>},
    {4, 2, false, corde::rod_group_kernel<4, 2, false>},
    {2, 4, false, corde::rod_group_kernel<2, 4, false>},
    {2, 8, false, corde::rod_group_kernel<2, 8, false>},
    {1, 2, true, corde::rod_group_kernel<1, 2, true>},
    {2, 2, true, corde::rod_group_kernel<2, 2, true>},
    {4, 2, true, corde::rod_group_kernel<4, 2, true>},
};
// contact candidate lists: pairs within contact distance + this fraction of the largest
// sphere radius of the group's rods
constexpr float kContactMarginRel = 0.5f;
constexpr int kGroupMax = 1024;     // longest rod a group may hold
constexpr int kContactMax = 512;    // longest rod of a group with contact

thread_local std::string g_last_error;

}  // namespace

struct rod_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int n_rods = 0;
  int max_n = 0;
  int total_pts = 0, total_frames = 0;
  std::vector<int> n;
  std::vector<RodDev> rods;
  RodDev* d_rods = nullptr;
  float* d_prm = nullptr;
  int prm_stride = 0;
  float *d_x = nullptr, *d_v = nullptr, *d_q = nullptr, *d_w = nullptr;
  // low parts of the positions and quaternions (x = d_x + d_xl, q = d_q + d_ql), zeroed by
  // rod_set_state
  float *d_xl = nullptr, *d_ql = nullptr;
  float *d_fext = nullptr, *d_text = nullptr;
  int* d_status = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool have_state = false;
  long long steps_done = 0;
  double t0 = 0.0;
  // rods grouped by kernel shape; rod_ids lists the rods bucket by bucket (longest first)
  struct Bucket {
    int waves, elems, first, count, max_n;
    float us_per_step;
    int feat = 0;   // kernel feature bits of its rods (mailbox, environment)
  };
  // long rods (more than chunk_above elements): chunked, one workgroup per chunk
  int chunk_above = kResidentMax;
  int chunk_target = 0;   // owned elements per chunk (0: as many as a window holds)
  std::vector<int> long_rods;
  int n_chunks = 0, pub_slots = 0;
  corde::GridChunk* d_chunks = nullptr;
  int* d_block_chunk = nullptr;
  float* d_pub = nullptr;
  int* d_flags = nullptr;
  std::vector<Bucket> buckets;
  // rod groups (bindings, contact): one or two rods per workgroup, grouped by kernel shape
  std::vector<std::array<int, 2>> bind_pairs;   // as set: bound rod pairs (second = master)
  int bind_mode = 0;
  std::vector<int> partner;                     // per slot: slot of the bound point, or -1
  std::vector<std::array<int, 2>> contact_sets; // as set: rods in contact (second -1: alone)
  float contact_mu = 0.f;
  std::vector<char> bound;                      // per rod: stepped by the group kernel
  std::vector<corde::GroupDev> groups;          // bucket by bucket
  std::vector<Bucket> pair_buckets;             // shapes of the group buckets
  corde::GroupDev* d_groups = nullptr;
  int* d_partner = nullptr;
  float* d_rho = nullptr;                       // per slot: sphere radius of point slot + 1
  std::vector<float> rmax;                      // per rod: largest sphere radius
  // contact candidate lists per slot: build position + count, kContactCand partner indices
  float4* d_cbuild = nullptr;
  uint16_t* d_ccand = nullptr;
  std::vector<int> rod_ids;
  int* d_rod_ids = nullptr;
  int steps_per_launch = 10;
  // haptic mailboxes (pinned host memory mapped for the device), per rod; seq: last pose number
  struct Haptic {
    corde::HapticBox* host = nullptr;
    corde::HapticBox* dev = nullptr;
    uint32_t seq = 0;
  };
  std::vector<Haptic> haptic;
  int n_haptic = 0;
  // environment mesh (rod_set_environment): AABB tree and triangles on the device
  corde::EnvNode* d_env_nodes = nullptr;
  corde::EnvTri* d_env_tris = nullptr;
  float4* d_env_cache = nullptr;   // per slot: candidate-list position and length
  int2* d_env_cand = nullptr;      // per slot: candidate triangles and build distances
  int env_nodes = 0, env_tris = 0;
  // adjoint rollout (rod_adjoint_forward / rod_adjoint_backward)
  bool adj_ready = false;
  long long adj_serial = 0;   // number of the held rollout (rollouts are numbered 1, 2, ...)
  long long adj_count = 0;    // rollouts recorded so far
  int adj_steps = 0, adj_ckpt = 0, adj_nckpt = 0;
  long long adj_step0 = 0;
  float* d_ckpt = nullptr;   // adj_nckpt whole-handle states (checkpoints)
  float* d_traj = nullptr;   // states at the start of each step of a segment (or of all steps)
  size_t cap_ckpt = 0, cap_traj = 0, cap_tips = 0, cap_dtips = 0, cap_state = 0;
  float* d_tips = nullptr;   // n_rods x adj_steps x 3
  float* d_dtips = nullptr;
  float* d_adj = nullptr;    // adjoint state, whole-handle state layout
  double* d_gacc = nullptr;  // n_rods x 512 lanes x 2: FP64 multiplier-gradient accumulators
  // the backward pass recomputes segment k-1 on a second stream while segment k is reversed
  hipStream_t aux = nullptr;
  hipEvent_t ev_start = nullptr, ev_rec[2] = {nullptr, nullptr}, ev_rev[2] = {nullptr, nullptr};
  // one stream per bucket (and one for the chunked long rods): buckets step concurrently
  std::vector<hipStream_t> bstreams;
  std::vector<hipEvent_t> bevents;
  hipEvent_t ev_fork = nullptr;
  float last_ms = 0.f;
  int last_launches = 0;
  bool timed = false;
  std::string err;
};

namespace {

rod_status fail(rod_ctx* c, rod_status s, const std::string& msg) {
  if (c) c->err = msg;
  g_last_error = msg;
  return s;
}

rod_status hip_fail(rod_ctx* c, hipError_t e, const char* what) {
  return fail(c, ROD_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(ctx, call)                                   \
  do {                                                       \
    hipError_t _e = (call);                                  \
    if (_e != hipSuccess) return hip_fail((ctx), _e, #call); \
  } while (0)

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Kernel feature bits rod r needs (a mailbox, the environment).
int rod_features(const rod_ctx* c, int r) {
  return (c->haptic[r].host ? corde::kFeatHaptic : 0) | (c->env_nodes ? corde::kFeatEnv : 0) |
         (c->rods[r].damp_int > 0.f ? corde::kFeatDamp : 0);
}

// Validates one rod description; returns "" or a message.
std::string check_params(const rod_params& p, int idx) {
  char buf[256];
  auto bad = [&](const char* what) {
    std::snprintf(buf, sizeof buf, "rod %d: %s", idx, what);
    return std::string(buf);
  };
  if (p.n_elements < 1) return bad("n_elements must be >= 1");
  if (p.inextensible != 0 && p.inextensible != 1) return bad("inextensible must be 0 or 1");
  if (p.inextensible && (p.n_constraint_iters < 0 || p.n_constraint_iters > 100000))
    return bad("n_constraint_iters out of range");
  if (!finite_pos(p.dt)) return bad("dt must be finite and > 0");
  if (!finite_pos(p.density)) return bad("density must be > 0");
  if (!(std::isfinite(p.poisson) && p.poisson > -1.0 && p.poisson < 0.5 + 1e-12))
    return bad("poisson must be in (-1, 0.5]");
  if (!(std::isfinite(p.kp_scale) && p.kp_scale >= 0) || !(std::isfinite(p.bend_scale) && p.bend_scale >= 0) ||
      !(std::isfinite(p.twist_scale) && p.twist_scale >= 0))
    return bad("stiffness scales must be finite and >= 0");
  if (!(std::isfinite(p.damping_lin) && p.damping_lin >= 0 && std::isfinite(p.damping_ang) &&
        p.damping_ang >= 0 && std::isfinite(p.damping_int) && p.damping_int >= 0))
    return bad("damping must be finite and >= 0");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(p.gravity[k])) return bad("gravity must be finite");
  if (!p.seg_len || !p.radius || !p.young) return bad("seg_len, radius and young are required");
  for (int j = 0; j < p.n_elements; ++j)
    if (!finite_pos(p.seg_len[j]) || !finite_pos(p.radius[j]) || !finite_pos(p.young[j]))
      return bad("seg_len, radius and young must be finite and > 0");
  if (p.clamp_end0 != 0 && p.clamp_end0 != 1) return bad("clamp_end0 must be 0 or 1");
  if (p.clamp_end0) {
    double qn = 0;
    for (int k = 0; k < 4; ++k) qn += p.clamp_q0[k] * p.clamp_q0[k];
    if (!(std::fabs(qn - 1.0) < 1e-6)) return bad("clamp_q0 must be a unit quaternion");
    double an = 0;
    for (int k = 0; k < 3; ++k) an += p.clamp_twist_axis[k] * p.clamp_twist_axis[k];
    if (p.clamp_twist_amp != 0.0 && !(an > 0)) return bad("clamp_twist_axis must be non-zero");
    if (!std::isfinite(p.clamp_freq)) return bad("clamp_freq must be finite");
  }
  return "";
}

// Material coefficients of element j (FP64): Sec. 2.1, with the second moment of area in
// eq. (3), K_p = kp_scale G pi r^2 in eq. (8), rigid-cylinder frame inertia.
struct Elem {
  double l, m, Ks, Kp, K1, K3, I1, I3;
};

Elem element(const rod_params& p, int j) {
  Elem e;
  const double r = p.radius[j], E = p.young[j];
  const double G = E / (2.0 * (1.0 + p.poisson));
  const double A = kPi * r * r;
  e.l = p.seg_len[j];
  e.m = p.density * A * e.l;
  e.Ks = E * A;
  e.Kp = p.kp_scale * G * A;
  e.K1 = p.bend_scale * E * kPi * r * r * r * r / 4.0;
  e.K3 = p.twist_scale * G * kPi * r * r * r * r / 2.0;
  e.I1 = e.m * (3.0 * r * r + e.l * e.l) / 12.0;
  e.I3 = e.m * r * r / 2.0;
  return e;
}

// Per-slot coefficient rows of one rod into rows[r * stride + off + j].
void fill_rows(const rod_params& p, std::vector<float>& rows, int stride, int off, double* winv0) {
  const int n = p.n_elements;
  std::vector<Elem> el(n);
  for (int j = 0; j < n; ++j) el[j] = element(p, j);
  std::vector<double> winv(n + 1);
  for (int i = 0; i <= n; ++i) {
    double M = 0.0;
    if (i > 0) M += 0.5 * el[i - 1].m;
    if (i < n) M += 0.5 * el[i].m;
    winv[i] = 1.0 / M;
  }
  if (p.clamp_end0) winv[0] = 0.0;
  *winv0 = winv[0];
  auto put = [&](int row, int j, double v) { rows[(size_t)row * stride + off + j] = (float)v; };
  // distance-constraint coefficients of segment k: 1 / (dt (w_k + w_{k+1})) and l_k times it
  auto ci = [&](int k) { return 1.0 / (p.dt * (winv[k] + winv[k + 1])); };
  for (int j = 0; j < n; ++j) {
    const Elem& e = el[j];
    put(corde::P_WINV, j, winv[j + 1]);
    put(corde::P_WINV_PREV, j, winv[j]);
    put(corde::P_WINV_NEXT, j, j + 2 <= n ? winv[j + 2] : 0.0);
    put(corde::P_CI, j, p.inextensible ? ci(j) : 0.0);
    put(corde::P_CIL, j, p.inextensible ? ci(j) * e.l : 0.0);
    put(corde::P_CI_NEXT, j, p.inextensible && j + 1 < n ? ci(j + 1) : 0.0);
    put(corde::P_CIL_NEXT, j, p.inextensible && j + 1 < n ? ci(j + 1) * el[j + 1].l : 0.0);
    put(corde::P_LEN, j, e.l);
    put(corde::P_KS_L, j, p.inextensible ? 0.0 : e.Ks / e.l);
    put(corde::P_LKP, j, e.l * e.Kp);
    put(corde::P_IINV1, j, 1.0 / e.I1);
    put(corde::P_IINV3, j, 1.0 / e.I3);
    put(corde::P_GYRO, j, (e.I3 - e.I1) / e.I1);
    if (j + 1 < n) {
      const Elem& f = el[j + 1];
      const double lbar = 0.5 * (e.l + f.l);
      const double K1 = 0.5 * (e.K1 + f.K1), K3 = 0.5 * (e.K3 + f.K3);
      put(corde::P_C1, j, 2.0 * K1 / lbar);
      put(corde::P_C3, j, 2.0 * K3 / lbar);
      const double* uh = p.u_hat ? p.u_hat + 3 * j : nullptr;
      put(corde::P_D0, j, uh ? K1 * uh[0] : 0.0);
      put(corde::P_D1, j, uh ? K1 * uh[1] : 0.0);
      put(corde::P_D2, j, uh ? K3 * uh[2] : 0.0);
    } else {
      put(corde::P_C1, j, 0.0);
      put(corde::P_C3, j, 0.0);
      put(corde::P_D0, j, 0.0);
      put(corde::P_D1, j, 0.0);
      put(corde::P_D2, j, 0.0);
    }
  }
}

RodDev make_dev(const rod_params& p, int slot_off, int pt_off, int fr_off, double winv0) {
  RodDev d{};
  d.n = p.n_elements;
  d.slot_off = slot_off;
  d.pt_off = pt_off;
  d.fr_off = fr_off;
  d.n_iter = p.inextensible ? p.n_constraint_iters : 0;
  d.clamp = p.clamp_end0;
  d.damp_int = (float)p.damping_int;
  {  // contact: points closer than 2 r_max along the rod (in elements of l_min) never touch
    double rmax = 0.0, lmin = INFINITY;
    for (int j = 0; j < p.n_elements; ++j) {
      rmax = std::max(rmax, p.radius[j]);
      lmin = std::min(lmin, p.seg_len[j]);
    }
    d.self_skip = std::max(1, (int)std::ceil(2.0 * rmax / lmin));
  }
  d.has_ext = (p.f_ext || p.tau_ext) ? 1 : 0;
  d.dt = (float)p.dt;
  d.dt_d = p.dt;
  d.damp_lin = (float)p.damping_lin;
  d.damp_ang = (float)p.damping_ang;
  d.winv0 = (float)winv0;
  for (int k = 0; k < 3; ++k) d.g[k] = (float)p.gravity[k];
  double an = 0;
  for (int k = 0; k < 3; ++k) an += p.clamp_twist_axis[k] * p.clamp_twist_axis[k];
  an = an > 0 ? std::sqrt(an) : 1.0;
  bool moving = p.clamp_twist_amp != 0.0;
  for (int k = 0; k < 3; ++k) {
    d.cx0[k] = (float)p.clamp_x0[k];
    d.camp[k] = (float)p.clamp_amp[k];
    d.caxis[k] = (float)(p.clamp_twist_axis[k] / an);
    moving = moving || p.clamp_amp[k] != 0.0;
  }
  for (int k = 0; k < 4; ++k) d.cq0[k] = (float)p.clamp_q0[k];
  d.ctw = (float)p.clamp_twist_amp;
  d.driven = (p.clamp_end0 && moving) ? 1 : 0;
  d.omega = 2.0 * kPi * p.clamp_freq;
  d.ph_x = p.clamp_phase_x;
  d.ph_t = p.clamp_phase_twist;
  d.t0 = 0.0;
  d.mult_bend = 1.f;
  d.mult_twist = 1.f;
  return d;
}

// Default kernel shape for a rod of n elements: one wavefront while it fits, then up to four
// (one per SIMD), then more elements per lane.
void default_shape(int n, int* w, int* e) {
  static const int order[][2] = {{1, 1}, {1, 2}, {2, 2}, {4, 2}, {4, 4}, {8, 4}, {4, 8}};
  for (const auto& o : order) {
    if (64 * o[0] * o[1] >= n) {
      *w = o[0];
      *e = o[1];
      return;
    }
  }
  *w = 4;
  *e = 8;
}

// Groups the rods into buckets of equal kernel shape (shape(r) gives it), longest rod first
// within a bucket, and uploads the resulting rod order.
template <class ShapeFn>
rod_status make_buckets(rod_ctx* c, ShapeFn shape) {
  std::vector<std::pair<long long, int>> key;
  std::vector<int> wr(c->n_rods), er(c->n_rods);
  std::vector<int> hr(c->n_rods);
  for (int r = 0; r < c->n_rods; ++r) {
    if (c->n[r] > c->chunk_above) continue;   // long rods run chunked
    if (!c->bound.empty() && c->bound[r]) continue;   // bound pairs have their own kernel
    int w, e;
    shape(r, &w, &e);
    const int h = rod_features(c, r);
    if (h) {   // a shape built with the feature code
      const KernelEntry* k = find_kernel(w, e);
      if (!k || !k->fn[h]) default_shape(c->n[r], &w, &e);
    }
    wr[r] = w, er[r] = e, hr[r] = h;
    // within a bucket, most work first (a constraint iteration costs about a quarter of the
    // rest of a step), so the last workgroups dispatched are the cheap ones
    const long long cost = (long long)c->n[r] * (4 + c->rods[r].n_iter);
    key.push_back({((long long)((w * 16 + e) * 8 + h) << 32) | (0x7fffffffLL - cost), r});
  }
  std::sort(key.begin(), key.end());
  c->buckets.clear();
  c->rod_ids.assign(std::max(c->n_rods, 1), 0);
  for (int i = 0; i < (int)key.size(); ++i) {
    const int r = key[i].second;
    const int w = wr[r], e = er[r];
    const int h = hr[r];
    c->rod_ids[i] = r;
    if (c->buckets.empty() || c->buckets.back().waves != w || c->buckets.back().elems != e ||
        c->buckets.back().feat != h)
      c->buckets.push_back({w, e, i, 0, 0, 0.f, h});
    c->buckets.back().count++;
    c->buckets.back().max_n = std::max(c->buckets.back().max_n, c->n[r]);
  }
  HIP_TRY(c, hipMemcpyAsync(c->d_rod_ids, c->rod_ids.data(), sizeof(int) * c->n_rods,
                            hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return ROD_OK;
}

// AABB tree of a triangle mesh by volume partitioning: the triangles of a node are split at
// the median of their centroids along the longest axis of the centroids' bounds, down to leaves
// of at most kLeafTris triangles; nodes are emitted depth-first (see corde::EnvNode), leaf
// triangles in leaf order.  Boxes are padded by pad so that the FP32 box test never rejects a
// triangle the FP32 narrow phase would accept.
constexpr int kLeafTris = 2;
struct BuildTri {
  double v[3][3];
  double cen[3];
};

void build_env_node(std::vector<BuildTri>& t, int b, int e, float pad,
                    std::vector<corde::EnvNode>& nodes, std::vector<corde::EnvTri>& out) {
  const int me = (int)nodes.size();
  nodes.push_back({});
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int i = b; i < e; ++i)
    for (int a = 0; a < 3; ++a) {
      for (int k = 0; k < 3; ++k) {
        lo[a] = std::min(lo[a], (float)t[i].v[k][a]);
        hi[a] = std::max(hi[a], (float)t[i].v[k][a]);
      }
      clo[a] = std::min(clo[a], t[i].cen[a]);
      chi[a] = std::max(chi[a], t[i].cen[a]);
    }
  corde::EnvNode nd;
  for (int a = 0; a < 3; ++a) {
    nd.lo[a] = lo[a] - pad;
    nd.hi[a] = hi[a] + pad;
  }
  if (e - b <= kLeafTris) {
    nd.leaf = ((int)out.size() << 3) | (e - b);
    for (int i = b; i < e; ++i) {
      corde::EnvTri tr;
      double e1[3], e2[3], n[3];
      for (int a = 0; a < 3; ++a) {
        e1[a] = t[i].v[1][a] - t[i].v[0][a];
        e2[a] = t[i].v[2][a] - t[i].v[0][a];
      }
      n[0] = e1[1] * e2[2] - e1[2] * e2[1];
      n[1] = e1[2] * e2[0] - e1[0] * e2[2];
      n[2] = e1[0] * e2[1] - e1[1] * e2[0];
      const double nl = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
      for (int a = 0; a < 3; ++a) {
        tr.a[a] = (float)t[i].v[0][a];
        tr.e1[a] = (float)e1[a];
        tr.e2[a] = (float)e2[a];
        tr.n[a] = (float)(n[a] / nl);
      }
      out.push_back(tr);
    }
    nd.skip = me + 1;
    nodes[me] = nd;
    return;
  }
  int axis = 0;
  for (int a = 1; a < 3; ++a)
    if (chi[a] - clo[a] > chi[axis] - clo[axis]) axis = a;
  const int mid = (b + e) / 2;
  std::nth_element(t.begin() + b, t.begin() + mid, t.begin() + e,
                   [axis](const BuildTri& x, const BuildTri& y) { return x.cen[axis] < y.cen[axis]; });
  build_env_node(t, b, mid, pad, nodes, out);
  build_env_node(t, mid, e, pad, nodes, out);
  nd.leaf = -1;
  nd.skip = (int)nodes.size();
  nodes[me] = nd;
}

// Rebuilds the buckets with every rod keeping its current shape (after a mailbox change).
rod_status rebucket(rod_ctx* c) {
  std::vector<int> shape_of(c->n_rods, 0);
  for (const auto& b : c->buckets)
    for (int i = 0; i < b.count; ++i) shape_of[c->rod_ids[b.first + i]] = b.waves * 16 + b.elems;
  return make_buckets(c, [&](int r, int* w, int* e) {
    if (shape_of[r]) {
      *w = shape_of[r] / 16;
      *e = shape_of[r] % 16;
    } else {
      default_shape(c->n[r], w, e);
    }
  });
}

// Splits every rod longer than chunk_above into chunks owning c slots (even, at least 2 H + 2
// when there are several, about chunk_target if set) with windows of at most
// 64 kGridWaves kGridElems slots and H = T (2 n_iter + 2) + 2 (rounded up to even) halo slots
// per side, enough for T steps between halo exchanges; T (at most kMaxExchangeEvery) is the
// largest whose halos take at most a quarter of a window each, fit chunk_target if set, and
// keep the rod within one chunk per compute unit (or 1).  Maps chunks to blocks so that
// neighbours share an XCD.
rod_status setup_long_rods(rod_ctx* c) {
  std::vector<corde::GridChunk> ch;
  int hmax = 0;
  const int K = 64 * kGridWaves * kGridElems;
  int cus = 0;
  HIP_TRY(c, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device));
  for (int r = 0; r < c->n_rods; ++r) {
    const int n = c->n[r];
    if (n <= c->chunk_above) continue;
    if (c->rods[r].damp_int > 0.f)
      return fail(c, ROD_E_UNSUPPORTED, "rods with internal friction cannot be chunked");
    c->long_rods.push_back(r);
    const int rad = 2 * c->rods[r].n_iter + 2;   // one step's dependency radius in slots
    auto halo_of = [&](int t) { const int h = t * rad + 2; return h + (h & 1); };
    auto chunks_of = [&](int h) {
      int cm = (K - 2 * h) & ~1;
      if (c->chunk_target > 0) cm = std::min(cm, std::max(c->chunk_target, 2 * h + 2) & ~1);
      int g = (n + cm - 1) / cm;
      while (g > 1 && ((n / g) & ~1) < 2 * h + 2) --g;
      return g;
    };
    int T = 1;
    for (int t = 2; t <= kMaxExchangeEvery; ++t) {
      const int h = halo_of(t);
      if (4 * h > K || (c->chunk_target > 0 && 2 * h + 2 > c->chunk_target) || chunks_of(h) > cus)
        break;
      T = t;
    }
    const int H = halo_of(T);
    hmax = std::max(hmax, H);
    const int G = chunks_of(H);
    int base = (n / G) & ~1;
    int rem = n - base * G;   // distributed two slots at a time
    int s0 = 0;
    const int first = (int)ch.size();
    for (int k = 0; k < G; ++k) {
      int cc = base;
      if (rem >= 2) { cc += 2; rem -= 2; }
      if (k == G - 1) cc = n - s0;
      corde::GridChunk g{};
      g.rod = r;
      g.s0 = s0;
      g.c = cc;
      g.win0 = std::max(0, s0 - H);
      g.nwin = std::min(n, s0 + cc + H) - g.win0;
      g.left = k > 0 ? first + k - 1 : -1;
      g.right = k < G - 1 ? first + k + 1 : -1;
      g.halo = H;
      g.every = T;
      if (g.nwin > K || (G > 1 && cc < 2 * H + 2))
        return fail(c, ROD_E_UNSUPPORTED, "rod " + std::to_string(r) +
                    ": too many constraint iterations to split it into chunks");
      ch.push_back(g);
      s0 += cc;
    }
  }
  c->n_chunks = (int)ch.size();
  if (!c->n_chunks) return ROD_OK;
  c->pub_slots = hmax + 1;
  // blocks are dealt to the 8 XCDs round-robin: give XCD x the chunks [x G / 8, (x+1) G / 8)
  const int G = c->n_chunks;
  std::vector<int> block_chunk(G);
  {
    std::vector<int> per_xcd(8, 0), start(9, 0);
    for (int x = 0; x < 8; ++x) start[x + 1] = (int)((long long)G * (x + 1) / 8);
    std::vector<int> next(start.begin(), start.end() - 1);
    for (int b = 0; b < G; ++b) {
      int x = b % 8;
      // fall back to any XCD with chunks left if this one is exhausted
      for (int t = 0; t < 8 && next[x] >= start[x + 1]; ++t) x = (x + 1) % 8;
      block_chunk[b] = next[x]++;
    }
  }
  auto dm = [&](void** p, size_t n) { return hipMalloc(p, std::max<size_t>(n, 4)) == hipSuccess; };
  if (!dm((void**)&c->d_chunks, sizeof(corde::GridChunk) * G) ||
      !dm((void**)&c->d_block_chunk, sizeof(int) * G) ||
      !dm((void**)&c->d_pub, sizeof(float) * 2 * (size_t)G * 2 * c->pub_slots * corde::kPubSlotFloats) ||
      !dm((void**)&c->d_flags, sizeof(int) * G))
    return fail(c, ROD_E_NOMEM, "long-rod buffers");
  HIP_TRY(c, hipMemcpy(c->d_chunks, ch.data(), sizeof(corde::GridChunk) * G, hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(c->d_block_chunk, block_chunk.data(), sizeof(int) * G, hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemset(c->d_flags, 0, sizeof(int) * G));
  // every chunk must be resident at once (the chunks wait on each other)
  int per_cu = 0;
  HIP_TRY(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, grid_kernel(), 64 * kGridWaves, 0));
  if ((long long)per_cu * cus < G)
    return fail(c, ROD_E_UNSUPPORTED, "long rods need " + std::to_string(G) +
                " resident workgroups, the device holds " + std::to_string(per_cu * cus));
  return ROD_OK;
}

// Chunked long rods: one ordinary launch of ks steps.  The chunks wait on their neighbours, so
// all workgroups of the grid must be resident together: the grid fits the device (checked when
// the chunks are set up), and every chunked run of the process is ordered after the previous
// one on the same device (LongGate), so two such grids never hold the compute units against
// each other.  A workgroup whose neighbour still does not arrive gives up after a bounded wait
// (status 4) instead of hanging.
rod_status launch_long(rod_ctx* c, StateArrays sa, int ks, long long done, hipStream_t stream) {
  if (!c->n_chunks) return ROD_OK;
  int spin = 1 << 22;
  const RodDev* rods = c->d_rods;
  const corde::GridChunk* chunks = c->d_chunks;
  const int* bc = c->d_block_chunk;
  const float* prm = c->d_prm;
  int stride = c->prm_stride;
  const float* fe = c->d_fext;
  const float* te = c->d_text;
  int* st = c->d_status;
  float* pub = c->d_pub;
  int ps = c->pub_slots, nc = c->n_chunks;
  int* fl = c->d_flags;
  void* args[] = {&rods, &chunks, &bc, &prm, &stride, &sa, &fe, &te, &ks, &done,
                  &st, &pub, &ps, &nc, &fl, &spin};
  HIP_TRY(c, hipLaunchKernel((const void*)grid_kernel(), dim3(c->n_chunks), dim3(64 * kGridWaves),
                             args, 0, stream));
  return ROD_OK;
}

// Orders the chunked runs of all handles of the process, per device: a run waits for the
// event recorded after the previous one (if another stream recorded it) and records it anew.
// The events live until the process ends.
struct LongGate {
  std::mutex m;
  hipEvent_t ev[kMaxDevices] = {};
  hipStream_t last[kMaxDevices] = {};   // stream of the last record (valid where rec)
  bool rec[kMaxDevices] = {};
};
LongGate& long_gate() {
  static LongGate* g = new LongGate;   // never destroyed: handles may outlive static teardown
  return *g;
}

// Zeroes the long-rod step flags (whenever the step counter restarts).
rod_status reset_flags(rod_ctx* c) {
  if (c->d_flags) HIP_TRY(c, hipMemsetAsync(c->d_flags, 0, sizeof(int) * c->n_chunks, c->stream));
  return ROD_OK;
}

// ---- scratch of rod_step_state_noalloc -----------------------------------------------------
// The low parts of the positions and quaternions of one call (3 floats per point, 4 per frame;
// a handle has fewer frames than points).  Every GPU the library runs
// on holds its own copy of this array until the process ends.  In host code its name is not a
// device address: the address of each GPU's copy is looked up once per device, with that
// device current (scratch_address), and only that address is passed to kernels.
constexpr long long kNoAllocMaxPoints = 1LL << 21;   // 56 MiB
static __device__ __align__(256) float scratch[7 * kNoAllocMaxPoints];

struct ScratchTable {
  std::mutex m;
  float* ptr[kMaxDevices] = {};
};
ScratchTable& scratch_table() {
  static ScratchTable* t = new ScratchTable;   // never destroyed, like the device copies
  return *t;
}

// Device address of device dev's copy of the scratch array (dev must be current).
rod_status scratch_address(rod_ctx* c, int dev, float** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(c, ROD_E_DEVICE, "device index out of range");
  ScratchTable& t = scratch_table();
  std::lock_guard<std::mutex> lock(t.m);
  if (!t.ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(c, ROD_E_DEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") +
                                       hipGetErrorString(e));
    t.ptr[dev] = static_cast<float*>(p);
  }
  *out = t.ptr[dev];
  return ROD_OK;
}

// Clears n floats with a kernel (a fill that also works where a caller captures the stream).
__global__ void zero_floats(float* __restrict__ p, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = 0.f;
}

// State arrays of a launch: the handle's own, or (rod_step_state_noalloc) the caller's with
// the low parts in the device's scratch array.
StateArrays handle_state(rod_ctx* c) { return {c->d_x, c->d_v, c->d_q, c->d_w, c->d_xl, c->d_ql}; }

rod_status launch_bucket(rod_ctx* c, const rod_ctx::Bucket& b, int ks, long long done,
                         hipStream_t stream, const StateArrays& sp) {
  const KernelEntry* k = find_kernel(b.waves, b.elems);
  const KernelFn fn = k ? k->fn[b.feat] : nullptr;
  if (!fn) return fail(c, ROD_E_UNSUPPORTED, "kernel shape not built");
  hipLaunchKernelGGL(fn, dim3(b.count), dim3(64 * k->waves), 0, stream, c->d_rods,
                     c->d_rod_ids + b.first, c->d_prm, c->prm_stride, sp, c->d_fext,
                     c->d_text, ks, done, c->d_status, nullptr, 0LL,
                     c->total_pts, c->total_frames, nullptr, 0, 0LL, 0, 1);
  HIP_TRY(c, hipGetLastError());
  return ROD_OK;
}

rod_status launch_pair_bucket(rod_ctx* c, const rod_ctx::Bucket& b, int ks, long long done,
                              hipStream_t stream) {
  const GroupEntry* k = nullptr;
  for (const auto& e : kGroups)
    if (e.waves == b.waves && e.elems == b.elems && (int)e.contact == b.feat) k = &e;
  if (!k) return fail(c, ROD_E_UNSUPPORTED, "group kernel shape not built");
  hipLaunchKernelGGL(k->fn, dim3(b.count), dim3(128 * k->waves), 0, stream, c->d_rods,
                     c->d_groups + b.first, c->d_partner, c->d_rho, c->d_cbuild, c->d_ccand,
                     c->d_prm, c->prm_stride,
                     handle_state(c), c->d_fext, c->d_text, ks, done, c->d_status);
  HIP_TRY(c, hipGetLastError());
  return ROD_OK;
}

// Merges the bindings and contact sets into workgroup groups (a rod in one group at most),
// checks them, and rebuilds the group and single-rod buckets.
rod_status rebuild_groups(rod_ctx* c) {
  std::vector<corde::GroupDev> gs;
  std::vector<int> group_of(c->n_rods, -1);
  for (const auto& p : c->bind_pairs) {
    group_of[p[0]] = group_of[p[1]] = (int)gs.size();
    gs.push_back({{p[0], p[1]}, c->bind_mode, 0, 0.f, 0.f});
  }
  for (const auto& cs : c->contact_sets) {
    const int a = cs[0], b = cs[1];
    int g = group_of[a];
    if (g >= 0) {
      if (b >= 0 && !(gs[g].rod[0] == b || gs[g].rod[1] == b))
        return fail(c, ROD_E_INVALID, "contact set of rods in different groups");
    } else if (b >= 0 && group_of[b] >= 0) {
      return fail(c, ROD_E_INVALID, "contact set of rods in different groups");
    } else {
      g = (int)gs.size();
      gs.push_back({{a, b}, 0, 0, 0.f, 0.f});
      group_of[a] = g;
      if (b >= 0) group_of[b] = g;
    }
    gs[g].contact = 1;
    gs[g].mu = c->contact_mu;
    gs[g].margin = kContactMarginRel * std::max(c->rmax[gs[g].rod[0]],
                                                gs[g].rod[1] >= 0 ? c->rmax[gs[g].rod[1]] : 0.f);
  }
  if (!gs.empty() && c->env_nodes)
    return fail(c, ROD_E_UNSUPPORTED, "rods in groups do not collide with the environment");
  for (const auto& g : gs)
    if (c->rods[g.rod[0]].damp_int > 0.f || (g.rod[1] >= 0 && c->rods[g.rod[1]].damp_int > 0.f))
      return fail(c, ROD_E_UNSUPPORTED, "rods with internal friction cannot be grouped");
  for (const auto& g : gs) {
    if (c->haptic[g.rod[0]].host || (g.rod[1] >= 0 && c->haptic[g.rod[1]].host))
      return fail(c, ROD_E_UNSUPPORTED, "a rod with a haptic mailbox cannot be grouped");
    const RodDev& a = c->rods[g.rod[0]];
    const int n = std::max(a.n, g.rod[1] >= 0 ? c->rods[g.rod[1]].n : 0);
    if (a.n_iter < 1) return fail(c, ROD_E_UNSUPPORTED, "grouped rods must be inextensible");
    if (g.rod[1] >= 0) {
      const RodDev& b = c->rods[g.rod[1]];
      if (b.n_iter != a.n_iter) return fail(c, ROD_E_UNSUPPORTED, "grouped rods need equal constraint iterations");
      if (b.dt_d != a.dt_d) return fail(c, ROD_E_UNSUPPORTED, "grouped rods need equal dt");
    }
    if (n > std::min(g.contact ? kContactMax : kGroupMax, c->chunk_above))
      return fail(c, ROD_E_UNSUPPORTED, "grouped rods are limited to 1024 elements (512 with contact) "
                                        "and must not be chunked");
  }
  auto shape_of = [&](int n, int* w, int* e) {
    *w = n <= 128 ? 1 : n <= 256 ? 2 : n <= 512 ? 4 : 2;
    *e = n <= 512 ? 2 : 8;
  };
  auto nmax = [&](const corde::GroupDev& g) {
    return std::max(c->n[g.rod[0]], g.rod[1] >= 0 ? c->n[g.rod[1]] : 0);
  };
  std::vector<std::pair<long long, int>> key;
  for (int g = 0; g < (int)gs.size(); ++g) {
    int w, e;
    shape_of(nmax(gs[g]), &w, &e);
    const long long cost = (long long)(c->n[gs[g].rod[0]] + (gs[g].rod[1] >= 0 ? c->n[gs[g].rod[1]] : 0)) *
                           (4 + c->rods[gs[g].rod[0]].n_iter);
    key.push_back({((long long)((w * 16 + e) * 2 + gs[g].contact) << 32) | (0x7fffffffLL - cost), g});
  }
  std::sort(key.begin(), key.end());
  HIP_TRY(c, hipStreamSynchronize(c->stream));   // no launch may still read the old tables
  for (hipStream_t st : c->bstreams) HIP_TRY(c, hipStreamSynchronize(st));
  c->groups.clear();
  c->pair_buckets.clear();
  c->bound.assign(c->n_rods, 0);
  for (int i = 0; i < (int)key.size(); ++i) {
    const auto& g = gs[key[i].second];
    int w, e;
    shape_of(nmax(g), &w, &e);
    c->groups.push_back(g);
    c->bound[g.rod[0]] = 1;
    if (g.rod[1] >= 0) c->bound[g.rod[1]] = 1;
    if (c->pair_buckets.empty() || c->pair_buckets.back().waves != w ||
        c->pair_buckets.back().elems != e || c->pair_buckets.back().feat != g.contact)
      c->pair_buckets.push_back({w, e, i, 0, 0, 0.f, g.contact});
    c->pair_buckets.back().count++;
    c->pair_buckets.back().max_n = std::max(c->pair_buckets.back().max_n, nmax(g));
  }
  if (c->d_groups) (void)hipFree(c->d_groups);
  c->d_groups = nullptr;
  if (!c->groups.empty()) {
    if (hipMalloc((void**)&c->d_groups, sizeof(corde::GroupDev) * c->groups.size()) != hipSuccess)
      return fail(c, ROD_E_NOMEM, "group tables");
    HIP_TRY(c, hipMemcpy(c->d_groups, c->groups.data(), sizeof(corde::GroupDev) * c->groups.size(),
                         hipMemcpyHostToDevice));
    if (!c->d_partner && hipMalloc((void**)&c->d_partner, sizeof(int) * c->partner.size()) != hipSuccess)
      return fail(c, ROD_E_NOMEM, "group tables");
    HIP_TRY(c, hipMemcpy(c->d_partner, c->partner.data(), sizeof(int) * c->partner.size(),
                         hipMemcpyHostToDevice));
    c->adj_ready = false;   // the adjoint does not step grouped rods
    bool any_contact = false;
    for (const auto& g : c->groups) any_contact = any_contact || g.contact;
    if (any_contact) {
      const size_t slots = (size_t)c->total_frames;
      if (!c->d_cbuild && (hipMalloc((void**)&c->d_cbuild, sizeof(float4) * slots) != hipSuccess ||
                           hipMalloc((void**)&c->d_ccand, sizeof(uint16_t) * corde::kContactCand * slots) !=
                               hipSuccess))
        return fail(c, ROD_E_NOMEM, "contact lists");
      // all bytes 0xff: NaN build positions, so every group builds its lists at its first step
      HIP_TRY(c, hipMemsetAsync(c->d_cbuild, 0xff, sizeof(float4) * slots, c->stream));
    }
  }
  return make_buckets(c, [&](int r, int* w, int* e) { default_shape(c->n[r], w, e); });
}

// n_steps steps of every rod, spl steps per launch; bucket < 0: all buckets, else that one.
rod_status launch_steps(rod_ctx* c, int n_steps, int spl, bool time_it, int bucket = -1) {
  // the buckets (and the bound-pair buckets) are independent: with several, each steps on its
  // own stream (forked from and joined back to the handle's stream)
  const int nb = bucket >= 0 ? 1 : (int)c->buckets.size();
  const int np = bucket >= 0 ? 0 : (int)c->pair_buckets.size();
  const int ng = nb + np;
  const bool fork = ng > 1;
  if (fork) {   // streams and events made on first use, before the timed interval opens
    while ((int)c->bstreams.size() < ng) {
      hipStream_t st = nullptr;
      hipEvent_t ev = nullptr;
      HIP_TRY(c, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      c->bstreams.push_back(st);
      HIP_TRY(c, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      c->bevents.push_back(ev);
    }
    if (!c->ev_fork) HIP_TRY(c, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
  }
  if (time_it) HIP_TRY(c, hipEventRecord(c->ev0, c->stream));
  int launches = 0;
  if (fork) HIP_TRY(c, hipEventRecord(c->ev_fork, c->stream));
  for (int gi = 0; gi < ng; ++gi) {
    hipStream_t st = c->stream;
    if (fork) {
      st = c->bstreams[gi];
      HIP_TRY(c, hipStreamWaitEvent(st, c->ev_fork, 0));
    }
    for (int done = 0; done < n_steps; done += spl) {
      const int ks = std::min(spl, n_steps - done);
      rod_status rs =
          gi < nb ? launch_bucket(c, c->buckets[bucket >= 0 ? bucket : gi], ks, c->steps_done + done, st,
                                  handle_state(c))
                  : launch_pair_bucket(c, c->pair_buckets[gi - nb], ks, c->steps_done + done, st);
      if (rs != ROD_OK) return rs;
      ++launches;
    }
    if (fork) {
      HIP_TRY(c, hipEventRecord(c->bevents[gi], st));
      HIP_TRY(c, hipStreamWaitEvent(c->stream, c->bevents[gi], 0));
    }
  }
  // chunked long rods on the handle's stream, after the buckets (all of a chunked grid's
  // workgroups must be resident together), and after any other handle's chunked run
  if (bucket < 0 && c->n_chunks) {
    const int dev = c->device;
    if (dev < 0 || dev >= kMaxDevices) return fail(c, ROD_E_DEVICE, "device index out of range");
    LongGate& g = long_gate();
    std::lock_guard<std::mutex> lock(g.m);
    if (!g.ev[dev]) HIP_TRY(c, hipEventCreateWithFlags(&g.ev[dev], hipEventDisableTiming));
    if (g.rec[dev] && g.last[dev] != c->stream) HIP_TRY(c, hipStreamWaitEvent(c->stream, g.ev[dev], 0));
    for (int done = 0; done < n_steps; done += spl) {
      const int ks = std::min(spl, n_steps - done);
      rod_status rs = launch_long(c, handle_state(c), ks, c->steps_done + done,
                                  c->stream);
      if (rs != ROD_OK) return rs;
      ++launches;
    }
    HIP_TRY(c, hipEventRecord(g.ev[dev], c->stream));
    g.last[dev] = c->stream;
    g.rec[dev] = true;
  }
  if (time_it) HIP_TRY(c, hipEventRecord(c->ev1, c->stream));
  c->timed = time_it;
  c->last_launches = launches;
  c->steps_done += n_steps;
  return ROD_OK;
}

// Adjoint shape for a bucket: the bucket's forward shape when it is built (an even number of
// elements per lane halves the constraint work), else the smallest one that holds the rods.
const AdjointEntry* adjoint_shape(int max_n, int waves = 0, int elems = 0) {
  for (const auto& a : kAdjoints)
    if (a.waves == waves && a.elems == elems && 64 * a.waves * a.elems >= max_n) return &a;
  for (const auto& a : kAdjoints)
    if (64 * a.waves * a.elems >= max_n) return &a;
  return nullptr;
}

// floats of one whole-handle state in the contiguous layout of corde::state_at
size_t state_floats(const rod_ctx* c) {
  return (size_t)corde::state_floats(c->total_pts, c->total_frames);
}

void free_adjoint(rod_ctx* c) {
  for (float** p : {&c->d_ckpt, &c->d_traj, &c->d_tips, &c->d_dtips, &c->d_adj}) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
  }
  if (c->d_gacc) (void)hipFree(c->d_gacc);
  c->d_gacc = nullptr;
  c->cap_ckpt = c->cap_traj = c->cap_tips = c->cap_dtips = c->cap_state = 0;
  c->adj_ready = false;
}

// Grows the adjoint buffers to hold a rollout of n_steps with checkpoints every ck steps
// (allocations are kept between rollouts; a larger rollout reallocates).
bool ensure_adjoint(rod_ctx* c, int n_steps, int ck) {
  const size_t S = state_floats(c);
  const int nck = (n_steps + ck - 1) / ck;
  const size_t need_ckpt = ck == 1 ? 1 : (size_t)nck * S;
  const size_t need_traj = (ck == 1 ? (size_t)n_steps : 2 * (size_t)ck) * S;   // 2: ping-pong
  const size_t need_tips = (size_t)3 * c->n_rods * n_steps;
  auto grow = [&](float** p, size_t* cap, size_t n) {
    if (*p && *cap >= n) return true;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    if (hipMalloc((void**)p, sizeof(float) * std::max<size_t>(n, 1)) != hipSuccess) {
      *p = nullptr;
      return false;
    }
    *cap = n;
    return true;
  };
  if (!c->aux) {
    if (hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) != hipSuccess) {
      c->aux = nullptr;
      return false;
    }
    for (hipEvent_t* e : {&c->ev_start, &c->ev_rec[0], &c->ev_rec[1], &c->ev_rev[0], &c->ev_rev[1]})
      if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) return false;
  }
  return grow(&c->d_ckpt, &c->cap_ckpt, need_ckpt) && grow(&c->d_traj, &c->cap_traj, need_traj) &&
         grow(&c->d_tips, &c->cap_tips, need_tips) && grow(&c->d_dtips, &c->cap_dtips, need_tips) &&
         grow(&c->d_adj, &c->cap_state, S) &&
         (c->d_gacc || hipMalloc((void**)&c->d_gacc, sizeof(double) * 2 * corde::kAdjointMaxLanes *
                                                         (size_t)c->n_rods) == hipSuccess);
}

// Launches the forward kernel of every bucket on the given state arrays.
rod_status launch_forward_on(rod_ctx* c, StateArrays sa, int ks,
                             long long step, float* traj, float* tips, long long tip_base,
                             int traj_steps, int store_final, hipStream_t stream = nullptr) {
  if (!stream) stream = c->stream;
  const long long S = (long long)state_floats(c);
  for (const auto& b : c->buckets) {
    const KernelEntry* k = find_kernel(b.waves, b.elems);
    if (!k) return fail(c, ROD_E_UNSUPPORTED, "kernel shape not built");
    if (b.feat) return fail(c, ROD_E_UNSUPPORTED, "the adjoint steps plain rods only");
    hipLaunchKernelGGL(k->fn[0], dim3(b.count), dim3(64 * k->waves), 0, stream, c->d_rods,
                       c->d_rod_ids + b.first, c->d_prm, c->prm_stride, sa, c->d_fext,
                       c->d_text, ks, step, c->d_status, traj, S, c->total_pts, c->total_frames,
                       tips, c->adj_steps, tip_base, traj_steps, store_final);
    HIP_TRY(c, hipGetLastError());
  }
  return ROD_OK;
}

}  // namespace

extern "C" {

const char* rod_status_str(rod_status s) {
  switch (s) {
    case ROD_OK: return "ROD_OK";
    case ROD_E_INVALID: return "ROD_E_INVALID: invalid argument";
    case ROD_E_NOMEM: return "ROD_E_NOMEM: out of memory";
    case ROD_E_DEVICE: return "ROD_E_DEVICE: HIP runtime error";
    case ROD_E_UNSTABLE: return "ROD_E_UNSTABLE: non-finite state";
    case ROD_E_ORDER: return "ROD_E_ORDER: call out of order";
    case ROD_E_UNSUPPORTED: return "ROD_E_UNSUPPORTED: not supported by this build";
    case ROD_E_TIMEOUT: return "ROD_E_TIMEOUT: long-rod workgroups lost step synchronisation";
  }
  return "unknown rod_status";
}

const char* rod_last_error(const rod_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_last_error.c_str();
}

rod_status rod_stable_dt(const rod_params* p, double* dt_out) {
  if (!p || !dt_out) return fail(nullptr, ROD_E_INVALID, "null argument");
  rod_params q = *p;
  q.dt = 1.0;  // dt itself is not needed for the rule
  std::string msg = check_params(q, 0);
  if (!msg.empty()) return fail(nullptr, ROD_E_INVALID, msg);
  double best = INFINITY;
  for (int j = 0; j < p->n_elements; ++j) {
    const Elem e = element(*p, j);
    // one-element modes: alternating translation 2 sqrt(k/m) with k = K/l, rotation
    // sqrt(k_rot / I) with k_rot = l K_p (penalty), 4 K_1 / l (bend), 4 K_3 / l (twist)
    // (the stretch, bend and twist modes carry the internal-friction dashpot: its decay rate
    // tau_d w^2 must stay below 2 / dt as well)
    double w[5];
    bool dashpot[5];
    int nw = 0;
    if (!p->inextensible) {
      dashpot[nw] = true;
      w[nw++] = 2.0 * std::sqrt(e.Ks / (e.l * e.m));
    }
    dashpot[nw] = false;
    w[nw++] = 2.0 * std::sqrt(e.Kp / (e.l * e.m));
    dashpot[nw] = false;
    w[nw++] = std::sqrt(e.l * e.Kp / e.I1);
    dashpot[nw] = true;
    w[nw++] = std::sqrt(4.0 * e.K1 / (e.l * e.I1));
    dashpot[nw] = true;
    w[nw++] = std::sqrt(4.0 * e.K3 / (e.l * e.I3));
    for (int k = 0; k < nw; ++k) {
      if (!(w[k] > 0)) continue;
      best = std::min(best, 2.0 / w[k]);
      if (dashpot[k] && p->damping_int > 0) best = std::min(best, 2.0 / (p->damping_int * w[k] * w[k]));
    }
  }
  if (!std::isfinite(best)) return fail(nullptr, ROD_E_INVALID, "rod has no elastic mode");
  *dt_out = 0.5 * best;
  return ROD_OK;
}

rod_status rod_create(const rod_params* params, int32_t n_rods, void* hip_stream, rod_ctx** out) {
  if (!params || !out) return fail(nullptr, ROD_E_INVALID, "null argument");
  if (n_rods < 1 || n_rods > (1 << 24)) return fail(nullptr, ROD_E_INVALID, "n_rods out of range");
  long long pts = 0, frames = 0;
  int max_n = 0;
  for (int r = 0; r < n_rods; ++r) {
    std::string msg = check_params(params[r], r);
    if (!msg.empty()) return fail(nullptr, ROD_E_INVALID, msg);
    pts += params[r].n_elements + 1;
    frames += params[r].n_elements;
    max_n = std::max(max_n, params[r].n_elements);
  }
  if (max_n > kLongMax)
    return fail(nullptr, ROD_E_UNSUPPORTED, "rod of " + std::to_string(max_n) +
                " elements exceeds the longest supported (" + std::to_string(kLongMax) + ")");
  if (frames > (1LL << 30)) return fail(nullptr, ROD_E_INVALID, "too many elements");
  rod_ctx* c = new (std::nothrow) rod_ctx();
  if (!c) return fail(nullptr, ROD_E_NOMEM, "host allocation failed");
  auto cleanup = [&](rod_status s) {
    rod_destroy(c);
    return s;
  };
  hipError_t e = hipGetDevice(&c->device);
  if (e != hipSuccess) return cleanup(hip_fail(nullptr, e, "hipGetDevice"));
  c->stream = (hipStream_t)hip_stream;
  c->n_rods = n_rods;
  c->max_n = max_n;
  c->total_pts = (int)pts;
  c->total_frames = (int)frames;
  c->prm_stride = (int)frames;
  std::vector<float> rows((size_t)(corde::P_NROWS + 1) * c->prm_stride, 0.f);
  std::vector<float> fext, text;
  std::vector<float> rho((size_t)std::max<long long>(frames, 1), 0.f);   // sphere radius per slot
  bool any_ext = false;
  for (int r = 0; r < n_rods; ++r) any_ext = any_ext || params[r].f_ext || params[r].tau_ext;
  if (any_ext) {
    fext.assign((size_t)3 * pts, 0.f);
    text.assign((size_t)3 * frames, 0.f);
  }
  int slot = 0, pt = 0, fr = 0;
  for (int r = 0; r < n_rods; ++r) {
    const rod_params& p = params[r];
    double winv0 = 0;
    fill_rows(p, rows, c->prm_stride, slot, &winv0);
    for (int j = 0; j < p.n_elements; ++j)   // point j + 1: its element's radius, the mean inside
      rho[(size_t)slot + j] = (float)(j + 1 == p.n_elements ? p.radius[j]
                                                             : 0.5 * (p.radius[j] + p.radius[j + 1]));
    c->rods.push_back(make_dev(p, slot, pt, fr, winv0));
    c->haptic.push_back({});
    c->n.push_back(p.n_elements);
    {
      double rm = 0.0;
      for (int j = 0; j < p.n_elements; ++j) rm = std::max(rm, p.radius[j]);
      c->rmax.push_back((float)rm);
    }
    if (p.f_ext)
      for (int i = 0; i < 3 * (p.n_elements + 1); ++i) fext[(size_t)3 * pt + i] = (float)p.f_ext[i];
    if (p.tau_ext)
      for (int i = 0; i < 3 * p.n_elements; ++i) text[(size_t)3 * fr + i] = (float)p.tau_ext[i];
    slot += p.n_elements;
    pt += p.n_elements + 1;
    fr += p.n_elements;
  }
  auto dmalloc = [&](void** ptr, size_t bytes) -> bool {
    return hipMalloc(ptr, std::max<size_t>(bytes, 4)) == hipSuccess;
  };
  if (!dmalloc((void**)&c->d_rods, sizeof(RodDev) * n_rods) ||
      !dmalloc((void**)&c->d_prm, sizeof(float) * rows.size()) ||
      !dmalloc((void**)&c->d_x, sizeof(float) * 3 * pts) ||
      !dmalloc((void**)&c->d_xl, sizeof(float) * 3 * pts) ||
      !dmalloc((void**)&c->d_v, sizeof(float) * 3 * pts) ||
      !dmalloc((void**)&c->d_q, sizeof(float) * 4 * frames) ||
      !dmalloc((void**)&c->d_ql, sizeof(float) * 4 * frames) ||
      !dmalloc((void**)&c->d_w, sizeof(float) * 3 * frames) ||
      !dmalloc((void**)&c->d_status, sizeof(int)) ||
      !dmalloc((void**)&c->d_rod_ids, sizeof(int) * n_rods) ||
      !dmalloc((void**)&c->d_rho, sizeof(float) * rho.size()))
    return cleanup(fail(nullptr, ROD_E_NOMEM, "device allocation failed"));
  if (any_ext && (!dmalloc((void**)&c->d_fext, sizeof(float) * fext.size()) ||
                  !dmalloc((void**)&c->d_text, sizeof(float) * text.size())))
    return cleanup(fail(nullptr, ROD_E_NOMEM, "device allocation failed"));
  for (auto& d : c->rods) d.rho = c->d_rho;
  e = hipMemcpy(c->d_rods, c->rods.data(), sizeof(RodDev) * n_rods, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->d_prm, rows.data(), sizeof(float) * rows.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->d_rho, rho.data(), sizeof(float) * rho.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && any_ext) {
    e = hipMemcpy(c->d_fext, fext.data(), sizeof(float) * fext.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->d_text, text.data(), sizeof(float) * text.size(), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipMemset(c->d_x, 0, sizeof(float) * 3 * pts);
  if (e == hipSuccess) e = hipMemset(c->d_xl, 0, sizeof(float) * 3 * pts);
  if (e == hipSuccess) e = hipMemset(c->d_v, 0, sizeof(float) * 3 * pts);
  if (e == hipSuccess) e = hipMemset(c->d_q, 0, sizeof(float) * 4 * frames);
  if (e == hipSuccess) e = hipMemset(c->d_ql, 0, sizeof(float) * 4 * frames);
  if (e == hipSuccess) e = hipMemset(c->d_w, 0, sizeof(float) * 3 * frames);
  if (e == hipSuccess) e = hipMemset(c->d_status, 0, sizeof(int));
  if (e == hipSuccess) e = hipEventCreate(&c->ev0);
  if (e == hipSuccess) e = hipEventCreate(&c->ev1);
  if (e != hipSuccess) return cleanup(hip_fail(nullptr, e, "rod_create device setup"));
  {
    rod_status st = setup_long_rods(c);
    if (st != ROD_OK) return cleanup(st);
    st = make_buckets(c, [&](int r, int* w, int* e) { default_shape(c->n[r], w, e); });
    if (st != ROD_OK) return cleanup(st);
  }
  {
    // set-up of rod_step_state_noalloc on this device (a failure is reported by that call)
    float* sp = nullptr;
    if (scratch_address(c, c->device, &sp) != ROD_OK) c->err.clear();
  }
  *out = c;
  return ROD_OK;
}

rod_status rod_destroy(rod_ctx* c) {
  if (!c) return fail(nullptr, ROD_E_INVALID, "null handle");
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  for (void* p : {(void*)c->d_rods, (void*)c->d_prm, (void*)c->d_x, (void*)c->d_xl,
                  (void*)c->d_ql, (void*)c->d_v,
                  (void*)c->d_q, (void*)c->d_w, (void*)c->d_fext, (void*)c->d_text,
                  (void*)c->d_status, (void*)c->d_rod_ids, (void*)c->d_ckpt, (void*)c->d_traj,
                  (void*)c->d_tips, (void*)c->d_dtips, (void*)c->d_adj,
                  (void*)c->d_gacc, (void*)c->d_groups, (void*)c->d_partner, (void*)c->d_rho,
                  (void*)c->d_chunks, (void*)c->d_block_chunk, (void*)c->d_pub,
                  (void*)c->d_flags, (void*)c->d_env_nodes, (void*)c->d_env_tris,
                  (void*)c->d_env_cache, (void*)c->d_env_cand, (void*)c->d_cbuild,
                  (void*)c->d_ccand})
    if (p) (void)hipFree(p);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  if (c->aux) {
    (void)hipStreamSynchronize(c->aux);
    (void)hipStreamDestroy(c->aux);
  }
  for (hipStream_t st : c->bstreams) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  for (hipEvent_t e : c->bevents) (void)hipEventDestroy(e);
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  for (hipEvent_t e : {c->ev_start, c->ev_rec[0], c->ev_rec[1], c->ev_rev[0], c->ev_rev[1]})
    if (e) (void)hipEventDestroy(e);
  for (auto& h : c->haptic)
    if (h.host) (void)hipHostFree(h.host);
  delete c;
  return ROD_OK;
}

rod_status rod_set_state(rod_ctx* c, const float* x, const float* v, const float* q,
                         const float* w, int32_t on_device, double t0) {
  if (!c) return fail(nullptr, ROD_E_INVALID, "null handle");
  if (!x || !v || !q || !w) return fail(c, ROD_E_INVALID, "null state pointer");
  if (!std::isfinite(t0)) return fail(c, ROD_E_INVALID, "t0 must be finite");
  const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  HIP_TRY(c, hipMemcpyAsync(c->d_x, x, sizeof(float) * 3 * c->total_pts, k, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->d_xl, 0, sizeof(float) * 3 * c->total_pts, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->d_v, v, sizeof(float) * 3 * c->total_pts, k, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->d_q, q, sizeof(float) * 4 * c->total_frames, k, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->d_ql, 0, sizeof(float) * 4 * c->total_frames, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->d_w, w, sizeof(float) * 3 * c->total_frames, k, c->stream));
  if (!on_device) HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->t0 = t0;
  c->steps_done = 0;
  {
    rod_status st = reset_flags(c);
    if (st != ROD_OK) return st;
  }
  for (auto& r : c->rods) r.t0 = t0;
  HIP_TRY(c, hipMemcpyAsync(c->d_rods, c->rods.data(), sizeof(RodDev) * c->n_rods,
                            hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));  // c->rods is host memory read by the copy
  c->have_state = true;
  return ROD_OK;
}

rod_status rod_get_state(rod_ctx* c, float* x, float* v, float* q, float* w, int32_t on_device) {
  if (!c) return fail(nullptr, ROD_E_INVALID, "null handle");
  if (!c->have_state) return fail(c, ROD_E_ORDER, "rod_get_state before rod_set_state");
  const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (x) HIP_TRY(c, hipMemcpyAsync(x, c->d_x, sizeof(float) * 3 * c->total_pts, k, c->stream));
  if (v) HIP_TRY(c, hipMemcpyAsync(v, c->d_v, sizeof(float) * 3 * c->total_pts, k, c->stream));
  if (q) HIP_TRY(c, hipMemcpyAsync(q, c->d_q, sizeof(float) * 4 * c->total_frames, k, c->stream));
  if (w) HIP_TRY(c, hipMemcpyAsync(w, c->d_w, sizeof(float) * 3 * c->total_frames, k, c->stream));
  if (!on_device) return rod_sync(c);
  return ROD_OK;
}

rod_status rod_step(rod_ctx* c, int32_t n_steps, int32_t steps_per_launch) {
  if (!c) return fail(nullptr, ROD_E_INVALID, "null handle");
  if (!c->have_state) return fail(c, ROD_E_ORDER, "rod_step before rod_set_state");
  if (n_steps < 0) return fail(c, ROD_E_INVALID, "n_steps must be >= 0");
  if (steps_per_launch < 0) return fail(c, ROD_E_INVALID, "steps_per_launch must be >= 0");
  if (n_steps == 0) return ROD_OK;
  int dev = -1;
  HIP_TRY(c, hipGetDevice(&dev));
  if (dev != c->device)
    return fail(c, ROD_E_DEVICE, "the handle's device (" + std::to_string(c->device) +
                ") is not the current device (" + std::to_string(dev) + ")");
  const int spl = steps_per_launch > 0 ? steps_per_launch : std::max(1, c->steps_per_launch);
  return launch_steps(c, n_steps, spl, true);
}

rod_status rod_set_clamp(rod_ctx* c, int32_t rod, const double* x0, const double* q0) {
  if (!c) return fail(nullptr, ROD_E_INVALID, "null handle");
  if (rod < 0 || rod >= c->n_rods) return fail(c, ROD_E_INVALID, "rod index out of range");
  if (!x0 || !q0) return fail(c, ROD_E_INVALID, "null clamp pose");
  double qn = 0;
  for (int k = 0; k < 4; ++k) qn += q0[k] * q0[k];
  if (!(std::fabs(qn - 1.0) < 1e-6)) return fail(c, ROD_E_INVALID, "q0 must be a unit quaternion");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(x0[k])) return fail(c, ROD_E_INVALID, "x0 must be finite");
  RodDev& d = c->rods[rod];
  for (int k = 0; k < 3; ++k) d.cx0[k] = (float)x0[k];
  for (int k = 0; k < 4; ++k) d.cq0[k] = (float)q0[k];
  HIP_TRY(c, hipMemcpyAsync(c->d_rods + rod, &d, sizeof(RodDev), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return ROD_OK;
}

rod_status rod_step_state_noalloc(rod_ctx* c, float* x, float* v, float* q, float* w,
                                  int64_t first_step, int32_t n_steps, int32_t steps_per_launch) {
  if (!c) return fail(nullptr, ROD_E_INVALID, "null handle");
  if (!x || !v || !q || !w) return fail(c, ROD_E_INVALID, "null state pointer");
  if (n_steps < 0 || steps_per_launch < 0 || first_step < 0)
    return fail(c, ROD_E_INVALID, "n_steps, steps_per_launch and first_step must be >= 0");
  if (c->n_chunks || !c->pair_buckets.empty() || c->n_haptic || c->env_nodes)
    return fail(c, ROD_E_UNSUPPORTED, "rod_step_state_noalloc steps handles without chunked rods, "
                                      "bindings, contact, haptic mailboxes or an environment");
  if ((long long)c->total_pts > kNoAllocMaxPoints)
    return fail(c, ROD_E_INVALID, "rod_step_state_noalloc holds at most " +
                                      std::to_string(kNoAllocMaxPoints) + " points; the handle has " +
                                      std::to_string(c->total_pts));
  int dev = -1;
  HIP_TRY(c, hipGetDevice(&dev));
  if (dev != c->device)
    return fail(c, ROD_E_DEVICE, "the handle's device (" + std::to_string(c->device) +
                ") is not the current device (" + std::to_string(dev) + ")");
  if (n_steps == 0) return ROD_OK;
  float* lo = nullptr;
  {
    rod_status st = scratch_address(c, dev, &lo);
    if (st != ROD_OK) return st;
  }
  const long long nl = 3LL * c->total_pts + 4LL * c->total_frames;
  hipLaunchKernelGGL(zero_floats, dim3((unsigned)std::min<long long>((nl + 255) / 256, 1024)),
                     dim3(256), 0, c->stream, lo, nl);
  HIP_TRY(c, hipGetLastError());
  const int spl = steps_per_launch > 0 ? steps_per_launch : c->steps_per_launch;
  const StateArrays sp = {x, v, q, w, lo, lo + 3LL * c->total_pts};
  for (const auto& b : c->buckets)   // all on the handle's stream: no stream is created
    for (int done = 0; done < n_steps; done += spl) {
      const int ks = std::min(spl, n_steps - done);
      rod_status rs = launch_bucket(c, b, ks, (long long)first_step + done, c->stream, sp);
      if (rs != ROD_OK) return rs;
    }
  return ROD_OK;
}

rod_status rod_sync(rod_ctx* c) {
  if (!c) return fail(nullptr, ROD_E_INVALID, "null handle");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  int st = 0;
  HIP_TRY(c, hipMemcpy(&st, c->d_status, sizeof(int), hipMemcpyDeviceToHost));
  if (st & 4) return fail(c, ROD_E_TIMEOUT, "a long-rod chunk waited too long for a neighbour");
  if (st & 8) return fail(c, ROD_E_UNSUPPORTED, "a point had more than 8 contacts in one step");
  if (st) return fail(c, ROD_E_UNSTABLE, "non-finite state detected by the step kernel");
  return ROD_OK;
}

rod_status rod_get_time(const rod_ctx* c, double* t, int64_t* steps) {
  if (!c || !t || !steps) return fail(nullptr, ROD_E_INVALID, "null argument");
  *steps = c->steps_done;
  *t = c->t0 + (double)c->steps_done * c->rods[0].dt_d;
  return ROD_OK;
}

rod_status rod_set_tuning(rod_ctx* c, const rod_tuning* t) {
  if (!c || !t) return fail(nullptr, ROD_E_INVALID, "null argument");
  if (t->steps_per_launch < 1) return fail(c, ROD_E_INVALID, "steps_per_launch must be >= 1");
  const KernelEntry* k = find_kernel(t->waves, t->elems_per_lane);
  if (!k) return fail(c, ROD_E_UNSUPPORTED, "kernel shape not built");
  int max_res = 0;
  for (int r = 0; r < c->n_rods; ++r)
    if (c->n[r] <= c->chunk_above) max_res = std::max(max_res, c->n[r]);
  if (64 * k->waves * k->elems < max_res) return fail(c, ROD_E_UNSUPPORTED, "shape cannot hold the longest rod");
  rod_status st = make_buckets(c, [&](int, int* w, int* e) { *w = t->waves; *e = t->elems_per_lane; });
  if (st != ROD_OK) return st;
  c->steps_per_launch = t->steps_per_launch;
  return ROD_OK;
}

rod_status rod_get_tuning(const rod_ctx* c, rod_tuning* t) {
  if (!c || !t) return fail(nullptr, ROD_E_INVALID, "null argument");
  t->waves = c->buckets.empty() ? kGridWaves : c->buckets.front().waves;
  t->elems_per_lane = c->buckets.empty() ? kGridElems : c->buckets.front().elems;
  t->steps_per_launch = c->steps_per_launch;
  float us = 0.f;
  for (const auto& bb : c->buckets) us += bb.us_per_step;
  t->us_per_step = us;
  return ROD_OK;
}

rod_status rod_bucket_info(const rod_ctx* c, int32_t bucket, rod_tuning* t, int32_t* n_rods) {
  if (!c || !t || !n_rods) return fail(nullptr, ROD_E_INVALID, "null argument");
  const int nb0 = (int)c->buckets.size();
  if (bucket >= nb0 && bucket < nb0 + (int)c->pair_buckets.size()) {
    const auto& b = c->pair_buckets[bucket - nb0];
    t->waves = b.waves;
    t->elems_per_lane = b.elems;
    t->steps_per_launch = c->steps_per_launch;
    t->us_per_step = 0.f;
    int nr = 0;
    for (int i = 0; i < b.count; ++i) nr += c->groups[b.first + i].rod[1] >= 0 ? 2 : 1;
    *n_rods = nr;
    return ROD_OK;
  }
  const int nb = nb0 + (int)c->pair_buckets.size();
  if (bucket == nb && c->n_chunks) {
    t->waves = kGridWaves;
    t->elems_per_lane = kGridElems;
    t->steps_per_launch = c->steps_per_launch;
    t->us_per_step = 0.f;
    *n_rods = (int)c->long_rods.size();
    return ROD_OK;
  }
  if (bucket < 0 || bucket >= nb0)
    return fail(const_cast<rod_ctx*>(c), ROD_E_INVALID, "bucket index out of range");
  const auto& b = c->buckets[bucket];
  t->waves = b.waves;
  t->elems_per_lane = b.elems;
  t->steps_per_launch = c->steps_per_launch;
  t->us_per_step = b.us_per_step;
  *n_rods = b.count;
  return ROD_OK;
}

rod_status rod_set_chunking(rod_ctx* c, int32_t min_elements, int32_t chunk_elements) {
  if (!c) return fail(nullptr, ROD_E_INVALID, "null handle");
  if (min_elements < 1 || min_elements > kResidentMax)
    return fail(c, ROD_E_INVALID, "min_elements must be in [1, 2048]");
  if (chunk_elements < 0) return fail(c, ROD_E_INVALID, "chunk_elements must be >= 0");
  for (int r = 0; r < c->n_rods; ++r) {
    if (!c->bound.empty() && c->bound[r] && c->n[r] > min_elements)
      return fail(c, ROD_E_UNSUPPORTED, "a bound rod cannot be chunked");
    if (c->haptic[r].host && c->n[r] > min_elements)
      return fail(c, ROD_E_UNSUPPORTED, "a rod with a haptic mailbox cannot be chunked");
    if (c->env_nodes && c->n[r] > min_elements)
      return fail(c, ROD_E_UNSUPPORTED, "chunked rods do not collide with the environment");
    if (c->rods[r].damp_int > 0.f && c->n[r] > min_elements)
      return fail(c, ROD_E_UNSUPPORTED, "rods with internal friction cannot be chunked");
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (void** p : {(void**)&c->d_chunks, (void**)&c->d_block_chunk, (void**)&c->d_pub,
                   (void**)&c->d_flags}) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
  }
  c->long_rods.clear();
  c->n_chunks = 0;
  c->pub_slots = 0;
  c->chunk_above = min_elements;
  c->chunk_target = chunk_elements;
  rod_status st = setup_long_rods(c);
  if (st == ROD_OK) st = make_buckets(c, [&](int r, int* w, int* e) { default_shape(c->n[r], w, e); });
  if (st != ROD_OK) {   // back to the default split, which rod_create accepted
    for (void** p : {(void**)&c->d_chunks, (void**)&c->d_block_chunk, (void**)&c->d_pub,
                     (void**)&c->d_flags}) {
      if (*p) (void)hipFree(*p);
      *p = nullptr;
    }
    c->long_rods.clear();
    c->n_chunks = 0;
    c->chunk_above = kResidentMax;
    c->chunk_target = 0;
    const std::string err = c->err;
    if (setup_long_rods(c) == ROD_OK)
      (void)make_buckets(c, [&](int r, int* w, int* e) { default_shape(c->n[r], w, e); });
    return fail(c, st, err);
  }
  if (c->n_chunks) c->adj_ready = false;   // the adjoint does not step chunked rods
  return ROD_OK;
}

rod_status rod_set_bindings(rod_ctx* c, int32_t n_pairs, const int32_t* pairs, int32_t mode) {
  if (!c) return fail(nullptr, ROD_E_INVALID, "null handle");
  if (n_pairs < 0 || (n_pairs > 0 && !pairs)) return fail(c, ROD_E_INVALID, "bad pair list");
  if (n_pairs > 0 && mode != 1 && mode != 2)
    return fail(c, ROD_E_INVALID, "mode must be 1 (one-way) or 2 (two-way)");
  std::vector<int> partner((size_t)std::max(c->total_frames, 1), -1);
  std::vector<int> group_of(c->n_rods, -1);
  std::vector<std::array<int, 2>> groups;   // (first, second); second = master if one-way
  for (int k = 0; k < n_pairs; ++k) {
    const int ra = pairs[4 * k], pa = pairs[4 * k + 1], rb = pairs[4 * k + 2], pb = pairs[4 * k + 3];
    if (ra < 0 || ra >= c->n_rods || rb < 0 || rb >= c->n_rods || ra == rb)
      return fail(c, ROD_E_INVALID, "pair " + std::to_string(k) + ": bad rod index");
    if (pa < 1 || pa > c->n[ra] || pb < 1 || pb > c->n[rb])
      return fail(c, ROD_E_INVALID, "pair " + std::to_string(k) + ": point index outside 1..n");
    int g = group_of[ra];
    if (g < 0 && group_of[rb] < 0) {
      g = (int)groups.size();
      groups.push_back({ra, rb});
      group_of[ra] = group_of[rb] = g;
    } else if (g < 0 || group_of[rb] != g) {
      return fail(c, ROD_E_INVALID, "pair " + std::to_string(k) + ": a rod is bound to two others");
    } else if (mode == 1 && groups[g][1] != rb) {
      return fail(c, ROD_E_INVALID, "pair " + std::to_string(k) + ": one-way pairs must name the same master");
    }
    const int sa = c->rods[ra].slot_off + pa - 1, sb = c->rods[rb].slot_off + pb - 1;
    if (partner[sa] >= 0 || partner[sb] >= 0)
      return fail(c, ROD_E_INVALID, "pair " + std::to_string(k) + ": a point is bound twice");
    partner[sa] = pb - 1;
    partner[sb] = pa - 1;
  }
  const auto old_pairs = c->bind_pairs;
  const auto old_partner = c->partner;
  const int old_mode = c->bind_mode;
  c->bind_pairs = groups;
  c->partner = partner;
  c->bind_mode = groups.empty() ? 0 : mode;
  rod_status st = rebuild_groups(c);
  if (st != ROD_OK) {   // keep the previous configuration
    const std::string err = c->err;
    c->bind_pairs = old_pairs;
    c->partner = old_partner;
    c->bind_mode = old_mode;
    (void)rebuild_groups(c);
    return fail(c, st, err);
  }
  return ROD_OK;
}

rod_status rod_set_contact(rod_ctx* c, int32_t n_sets, const int32_t* sets, double mu) {
  if (!c) return fail(nullptr, ROD_E_INVALID, "null handle");
  if (n_sets < 0 || (n_sets > 0 && !sets)) return fail(c, ROD_E_INVALID, "bad contact list");
  if (!(std::isfinite(mu) && mu >= 0.0)) return fail(c, ROD_E_INVALID, "mu must be finite and >= 0");
  std::vector<std::array<int, 2>> cs;
  std::vector<char> seen(c->n_rods, 0);
  for (int k = 0; k < n_sets; ++k) {
    const int a = sets[2 * k], b = sets[2 * k + 1];
    if (a < 0 || a >= c->n_rods || b < -1 || b >= c->n_rods || a == b)
      return fail(c, ROD_E_INVALID, "contact set " + std::to_string(k) + ": bad rod index");
    if (seen[a] || (b >= 0 && seen[b]))
      return fail(c, ROD_E_INVALID, "contact set " + std::to_string(k) + ": a rod is in two sets");
    seen[a] = 1;
    if (b >= 0) seen[b] = 1;
    cs.push_back({a, b});
  }
  const auto old = c->contact_sets;
  const float old_mu = c->contact_mu;
  c->contact_sets = cs;
  c->contact_mu = (float)mu;
  if (c->partner.empty()) c->partner.assign((size_t)std::max(c->total_frames, 1), -1);
  rod_status st = rebuild_groups(c);
  if (st != ROD_OK) {
    const std::string err = c->err;
    c->contact_sets = old;
    c->contact_mu = old_mu;
    (void)rebuild_groups(c);
    return fail(c, st, err);
  }
  return ROD_OK;
}

rod_status rod_last_step_time(rod_ctx* c, float* ms, int32_t* launches) {
  if (!c || !ms || !launches) return fail(nullptr, ROD_E_INVALID, "null argument");
  if (!c->timed) return fail(c, ROD_E_ORDER, "no timed rod_step yet");
  HIP_TRY(c, hipEventSynchronize(c->ev1));
  HIP_TRY(c, hipEventElapsedTime(&c->last_ms, c->ev0, c->ev1));
  *ms = c->last_ms;
  *launches = c->last_launches;
  return ROD_OK;
}

rod_status rod_haptic_attach(rod_ctx* c, int32_t rod, int32_t steps_per_record) {
  if (!c) return fail(nullptr, ROD_E_INVALID, "null handle");
  if (rod < 0 || rod >= c->n_rods) return fail(c, ROD_E_INVALID, "rod index out of range");
  if (steps_per_record < 1) return fail(c, ROD_E_INVALID, "steps_per_record must be >= 1");
  RodDev& d = c->rods[rod];
  if (!d.clamp) return fail(c, ROD_E_INVALID, "a haptic mailbox drives a clamped base");
  if (d.driven) return fail(c, ROD_E_UNSUPPORTED, "the rod's clamp is driven by its sinusoid");
  if (!c->bound.empty() && c->bound[rod])
    return fail(c, ROD_E_UNSUPPORTED, "a rod with a haptic mailbox cannot be grouped");
  if (c->n[rod] > c->chunk_above)
    return fail(c, ROD_E_UNSUPPORTED, "a rod with a haptic mailbox cannot be chunked");
  auto& hh = c->haptic[rod];
  const bool fresh = hh.host == nullptr;
  corde::HapticBox* h = hh.host;
  corde::HapticBox* hd = hh.dev;
  if (fresh) {
    if (hipHostMalloc((void**)&h, sizeof(corde::HapticBox), hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess || !h)
      return fail(c, ROD_E_NOMEM, "haptic mailbox");
    std::memset((void*)h, 0, sizeof(corde::HapticBox));
    hipError_t e = hipHostGetDevicePointer((void**)&hd, h, 0);
    if (e != hipSuccess) {
      (void)hipHostFree(h);
      return hip_fail(c, e, "hipHostGetDevicePointer");
    }
  }
  const RodDev before = d;
  d.hbox = hd;
  d.hstride = steps_per_record;
  hipError_t e = hipMemcpyAsync(c->d_rods + rod, &d, sizeof(RodDev), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    d = before;
    if (fresh) (void)hipHostFree(h);
    return hip_fail(c, e, "rod_haptic_attach");
  }
  if (!fresh) return ROD_OK;
  hh = {h, hd, 0};
  c->n_haptic++;
  c->adj_ready = false;
  return rebucket(c);   // the rod moves to a bucket of the kernel variant with the mailbox code
}

rod_status rod_haptic_detach(rod_ctx* c, int32_t rod) {
  if (!c) return fail(nullptr, ROD_E_INVALID, "null handle");
  if (rod < 0 || rod >= c->n_rods) return fail(c, ROD_E_INVALID, "rod index out of range");
  auto& h = c->haptic[rod];
  if (!h.host) return ROD_OK;
  RodDev& d = c->rods[rod];
  d.hbox = nullptr;
  d.hstride = 0;
  HIP_TRY(c, hipMemcpyAsync(c->d_rods + rod, &d, sizeof(RodDev), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));   // no kernel still uses the mailbox
  for (hipStream_t st : c->bstreams) HIP_TRY(c, hipStreamSynchronize(st));
  (void)hipHostFree(h.host);
  h = {};
  c->n_haptic--;
  return rebucket(c);
}

rod_status rod_haptic_set_pose(rod_ctx* c, int32_t rod, const double* x0, const double* q0) {
  // called from the haptic thread: no GPU call, no write to the handle other than the mailbox
  if (!c || rod < 0 || rod >= c->n_rods || !x0 || !q0)
    return fail(nullptr, ROD_E_INVALID, "bad handle, rod index or pose");
  auto& h = c->haptic[rod];
  if (!h.host) return fail(nullptr, ROD_E_ORDER, "rod has no haptic mailbox");
  double qn = 0;
  for (int k = 0; k < 4; ++k) qn += q0[k] * q0[k];
  if (!(std::fabs(qn - 1.0) < 1e-6)) return fail(nullptr, ROD_E_INVALID, "q0 must be a unit quaternion");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(x0[k])) return fail(nullptr, ROD_E_INVALID, "x0 must be finite");
  if (++h.seq == 0) h.seq = 1;   // pose number 0 means "no pose"
  const uint64_t tag = (uint64_t)h.seq << 32;
  const double inv = 1.0 / std::sqrt(qn);
  const float w[7] = {(float)x0[0], (float)x0[1], (float)x0[2], (float)(q0[0] * inv),
                      (float)(q0[1] * inv), (float)(q0[2] * inv), (float)(q0[3] * inv)};
  for (int k = 0; k < 7; ++k) {
    uint32_t bits;
    std::memcpy(&bits, &w[k], 4);
    __atomic_store_n(&h.host->pose[k], tag | bits, __ATOMIC_RELAXED);
  }
  return ROD_OK;
}

rod_status rod_haptic_get_force(rod_ctx* c, int32_t rod, rod_haptic_force* out) {
  // called from the haptic thread: no GPU call, no write to the handle
  if (!c || rod < 0 || rod >= c->n_rods || !out)
    return fail(nullptr, ROD_E_INVALID, "bad handle, rod index or output");
  const auto& h = c->haptic[rod];
  if (!h.host) return fail(nullptr, ROD_E_ORDER, "rod has no haptic mailbox");
  for (int attempt = 0; attempt < (1 << 20); ++attempt) {
    uint64_t w[5];
    for (int k = 0; k < 5; ++k) w[k] = __atomic_load_n(&h.host->fb[k], __ATOMIC_RELAXED);
    const uint32_t tag = (uint32_t)(w[0] >> 32);
    bool whole = true;
    for (int k = 1; k < 5; ++k) whole = whole && (uint32_t)(w[k] >> 32) == tag;
    if (!whole) continue;   // a record being written: read again
    for (int k = 0; k < 3; ++k) {
      const uint32_t bits = (uint32_t)w[k];
      float v;
      std::memcpy(&v, &bits, 4);
      out->f[k] = v;
    }
    out->step = tag;
    out->pose = (uint32_t)w[3];
    out->n_steps = (uint32_t)w[4];
    return ROD_OK;
  }
  return fail(nullptr, ROD_E_TIMEOUT, "no whole force record could be read");
}

rod_status rod_set_environment(rod_ctx* c, int32_t n_tris, const double* tris, double mu) {
  if (!c) return fail(nullptr, ROD_E_INVALID, "null handle");
  if (n_tris < 0 || n_tris > (1 << 26) || (n_tris > 0 && !tris))
    return fail(c, ROD_E_INVALID, "bad triangle list");
  if (!(std::isfinite(mu) && mu >= 0.0)) return fail(c, ROD_E_INVALID, "mu must be finite and >= 0");
  std::vector<BuildTri> bt;
  double cmax = 0.0;
  for (int i = 0; i < n_tris; ++i) {
    BuildTri t;
    bool fin = true;
    for (int k = 0; k < 3; ++k)
      for (int a = 0; a < 3; ++a) {
        t.v[k][a] = tris[9 * i + 3 * k + a];
        fin = fin && std::isfinite(t.v[k][a]);
        cmax = std::max(cmax, std::fabs(t.v[k][a]));
      }
    if (!fin) return fail(c, ROD_E_INVALID, "triangle coordinates must be finite");
    double e1[3], e2[3];
    for (int a = 0; a < 3; ++a) {
      e1[a] = t.v[1][a] - t.v[0][a];
      e2[a] = t.v[2][a] - t.v[0][a];
      t.cen[a] = (t.v[0][a] + t.v[1][a] + t.v[2][a]) / 3.0;
    }
    const double nx = e1[1] * e2[2] - e1[2] * e2[1], ny = e1[2] * e2[0] - e1[0] * e2[2],
                 nz = e1[0] * e2[1] - e1[1] * e2[0];
    if (nx * nx + ny * ny + nz * nz > 0.0) bt.push_back(t);   // degenerate triangles have no face
  }
  if (!bt.empty()) {
    if (!c->groups.empty())
      return fail(c, ROD_E_UNSUPPORTED, "rods in groups do not collide with the environment");
    for (const auto& d : c->rods)
      if (d.damp_int > 0.f)
        return fail(c, ROD_E_UNSUPPORTED, "rods with internal friction do not collide with the environment");
    if (c->n_chunks) return fail(c, ROD_E_UNSUPPORTED, "chunked rods do not collide with the environment");
  }
  std::vector<corde::EnvNode> nodes;
  std::vector<corde::EnvTri> out;
  if (!bt.empty()) build_env_node(bt, 0, (int)bt.size(), (float)(1e-6 * (1.0 + cmax)), nodes, out);
  HIP_TRY(c, hipStreamSynchronize(c->stream));   // no launch still reads the old mesh
  for (hipStream_t st : c->bstreams) HIP_TRY(c, hipStreamSynchronize(st));
  // first back to no mesh: plain kernels, no pointers to the old tables, which are freed
  auto set_rods = [&](int n_nodes, float mu) -> hipError_t {
    for (auto& d : c->rods) {
      d.env_n_nodes = n_nodes;
      d.env_nodes = n_nodes ? c->d_env_nodes : nullptr;
      d.env_tris = n_nodes ? c->d_env_tris : nullptr;
      d.env_cache = n_nodes ? c->d_env_cache : nullptr;
      d.env_cand = n_nodes ? c->d_env_cand : nullptr;
      d.env_mu = mu;
    }
    return hipMemcpy(c->d_rods, c->rods.data(), sizeof(RodDev) * c->n_rods, hipMemcpyHostToDevice);
  };
  auto free_env = [&]() {
    for (void** p : {(void**)&c->d_env_nodes, (void**)&c->d_env_tris, (void**)&c->d_env_cache,
                     (void**)&c->d_env_cand}) {
      if (*p) (void)hipFree(*p);
      *p = nullptr;
    }
  };
  c->env_nodes = c->env_tris = 0;
  HIP_TRY(c, set_rods(0, 0.f));
  free_env();
  rod_status st = rebucket(c);
  if (st != ROD_OK || nodes.empty()) return st;
  size_t slots = 0;
  for (int r = 0; r < c->n_rods; ++r) slots += (size_t)c->n[r];
  if (hipMalloc((void**)&c->d_env_nodes, sizeof(corde::EnvNode) * nodes.size()) != hipSuccess ||
      hipMalloc((void**)&c->d_env_tris, sizeof(corde::EnvTri) * out.size()) != hipSuccess ||
      hipMalloc((void**)&c->d_env_cache, sizeof(float4) * slots) != hipSuccess ||
      hipMalloc((void**)&c->d_env_cand, sizeof(int2) * slots * corde::kEnvCand) != hipSuccess) {
    free_env();
    return fail(c, ROD_E_NOMEM, "environment tables");
  }
  // no candidate list yet: every point builds one at its first step
  const std::vector<float4> far(slots, make_float4(1e30f, 1e30f, 1e30f, 0.f));
  hipError_t e = hipMemcpy(c->d_env_nodes, nodes.data(), sizeof(corde::EnvNode) * nodes.size(),
                           hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(c->d_env_tris, out.data(), sizeof(corde::EnvTri) * out.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->d_env_cache, far.data(), sizeof(float4) * slots, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = set_rods((int)nodes.size(), (float)mu);
  if (e != hipSuccess) {
    (void)set_rods(0, 0.f);
    free_env();
    return hip_fail(c, e, "rod_set_environment");
  }
  c->env_nodes = (int)nodes.size();
  c->env_tris = (int)out.size();
  c->adj_ready = false;
  return rebucket(c);   // the rods move to the kernel variant with the collision code
}

rod_status rod_environment_info(const rod_ctx* c, int32_t* n_nodes, int32_t* n_tris) {
  if (!c || !n_nodes || !n_tris) return fail(nullptr, ROD_E_INVALID, "null argument");
  *n_nodes = c->env_nodes;
  *n_tris = c->env_tris;
  return ROD_OK;
}

rod_status rod_autotune(rod_ctx* c, int32_t probe_steps, int32_t steps_per_launch, rod_tuning* out) {
  if (!c) return fail(nullptr, ROD_E_INVALID, "null handle");
  if (!c->have_state) return fail(c, ROD_E_ORDER, "rod_autotune before rod_set_state");
  if (probe_steps < 1 || steps_per_launch < 0) return fail(c, ROD_E_INVALID, "bad probe sizes");
  const bool pick_k = steps_per_launch == 0;   // also choose the steps per launch
  if (pick_k) steps_per_launch = std::min(10, probe_steps);
  // save the state, probe the candidate shapes of every bucket, restore
  const size_t bx = sizeof(float) * 3 * c->total_pts, bq = sizeof(float) * 4 * c->total_frames,
               bw = sizeof(float) * 3 * c->total_frames;
  float *sx = nullptr, *sxl = nullptr, *sv = nullptr, *sq = nullptr, *sql = nullptr, *sw = nullptr;
  if (hipMalloc(&sx, bx) != hipSuccess || hipMalloc(&sxl, bx) != hipSuccess ||
      hipMalloc(&sv, bx) != hipSuccess || hipMalloc(&sq, bq) != hipSuccess ||
      hipMalloc(&sql, bq) != hipSuccess || hipMalloc(&sw, bw) != hipSuccess) {
    for (float* p : {sx, sxl, sv, sq, sql, sw}) if (p) (void)hipFree(p);
    return fail(c, ROD_E_NOMEM, "autotune scratch allocation failed");
  }
  auto free_all = [&]() { for (float* p : {sx, sxl, sv, sq, sql, sw}) (void)hipFree(p); };
  auto copy = [&](float* d, const float* s, size_t b) {
    return hipMemcpyAsync(d, s, b, hipMemcpyDeviceToDevice, c->stream);
  };
  if (copy(sx, c->d_x, bx) || copy(sxl, c->d_xl, bx) || copy(sv, c->d_v, bx) ||
      copy(sq, c->d_q, bq) || copy(sql, c->d_ql, bq) || copy(sw, c->d_w, bw)) {
    free_all();
    return fail(c, ROD_E_DEVICE, "autotune state save failed");
  }
  const long long saved_steps = c->steps_done;
  rod_status st = ROD_OK;
  // whole-handle time per step at steps_per_launch (best of two probes)
  auto whole = [&](float* us) -> rod_status {
    float ms_best = INFINITY;
    for (int rep = 0; rep < 2; ++rep) {
      rod_status s2 = launch_steps(c, probe_steps, steps_per_launch, true);
      float ms = 0;
      int nl = 0;
      if (s2 == ROD_OK) s2 = rod_last_step_time(c, &ms, &nl);
      if (s2 != ROD_OK) return s2;
      ms_best = std::min(ms_best, ms);
    }
    *us = 1000.f * ms_best / probe_steps;
    return ROD_OK;
  };
  // steps_per_launch = 0 also decides whether the rods of more than kChunkTry elements step
  // chunked over several compute units or in one workgroup each (while the split is the
  // default one): the faster of the two is kept
  if (pick_k && c->chunk_above == kResidentMax && c->chunk_target == 0) {
    bool any = false;
    for (int r = 0; r < c->n_rods; ++r) any = any || (c->n[r] > kChunkTry && c->n[r] <= kResidentMax);
    float us_one = 0.f, us_chunked = 0.f;
    if (any) st = whole(&us_one);
    const std::string err0 = c->err;   // a refused split (e.g. a rod with a mailbox) is no error
    if (any && st == ROD_OK && rod_set_chunking(c, kChunkTry, 0) == ROD_OK) {
      st = whole(&us_chunked);
      if (st == ROD_OK && !(us_chunked < us_one)) st = rod_set_chunking(c, kResidentMax, 0);
    } else if (st == ROD_OK) {
      c->err = err0;
    }
  }
  // per bucket: time every built shape that holds its longest rod without idling most lanes
  std::vector<rod_ctx::Bucket> chosen = c->buckets;
  std::vector<std::vector<std::pair<int, float>>> tried(chosen.size());   // (shape, us) per bucket
  for (size_t bi = 0; bi < chosen.size() && st == ROD_OK; ++bi) {
    rod_ctx::Bucket& best = chosen[bi];
    best.us_per_step = INFINITY;
    for (const auto& k : kKernels) {
      const int cap = 64 * k.waves * k.elems;
      if (cap < best.max_n || cap >= 4 * std::max(best.max_n, 64)) continue;
      if (!k.fn[best.feat]) continue;
      c->buckets[bi].waves = k.waves;
      c->buckets[bi].elems = k.elems;
      float ms_best = INFINITY;
      for (int rep = 0; rep < 2 && st == ROD_OK; ++rep) {
        st = launch_steps(c, probe_steps, steps_per_launch, true, (int)bi);
        float ms = 0;
        int nl = 0;
        if (st == ROD_OK) st = rod_last_step_time(c, &ms, &nl);
        ms_best = std::min(ms_best, ms);
      }
      if (st != ROD_OK) break;
      const float us = 1000.f * ms_best / probe_steps;
      tried[bi].push_back({k.waves * 16 + k.elems, us});
      if (us < best.us_per_step) {
        best.us_per_step = us;
        best.waves = k.waves;
        best.elems = k.elems;
      }
    }
  }
  if (st == ROD_OK) {
    // Near ties go to a shape that another bucket (same kernel features) already uses: the
    // buckets step side by side, one launch each, and the shared shape saves a launch.  (The
    // shortest rods' bucket timed 1 x 1 and 1 x 2 within noise; split, the 4096-rod batch took
    // 38.6 ms against 37.4 merged.)
    auto key_of = [](const rod_ctx::Bucket& b) { return b.waves * 16 + b.elems; };
    auto used_elsewhere = [&](size_t bi, int key) {
      for (size_t o = 0; o < chosen.size(); ++o)
        if (o != bi && chosen[o].feat == chosen[bi].feat && key_of(chosen[o]) == key) return true;
      return false;
    };
    for (size_t bi = 0; bi < chosen.size(); ++bi) {
      rod_ctx::Bucket& b = chosen[bi];
      if (used_elsewhere(bi, key_of(b))) continue;
      for (const auto& t : tried[bi]) {
        if (t.first == key_of(b) || !(t.second <= 1.02f * b.us_per_step)) continue;
        if (used_elsewhere(bi, t.first)) {
          b.waves = t.first / 16;
          b.elems = t.first % 16;
          b.us_per_step = t.second;
          break;
        }
      }
    }
    // re-bucket: rods keep their bucket's chosen shape (equal shapes merge)
    std::vector<int> shape_of(c->n_rods);
    for (size_t bi = 0; bi < chosen.size(); ++bi)
      for (int i = 0; i < chosen[bi].count; ++i)
        shape_of[c->rod_ids[chosen[bi].first + i]] = chosen[bi].waves * 16 + chosen[bi].elems;
    std::vector<std::pair<int, float>> us_of;
    for (const auto& b : chosen)
      us_of.push_back({(b.waves * 16 + b.elems) * 8 + b.feat, b.us_per_step});
    st = make_buckets(c, [&](int r, int* w, int* e) { *w = shape_of[r] / 16; *e = shape_of[r] % 16; });
    for (auto& b : c->buckets) {
      b.us_per_step = 0.f;
      for (const auto& u : us_of)
        if (u.first == (b.waves * 16 + b.elems) * 8 + b.feat) b.us_per_step += u.second;
    }
  }
  if (st == ROD_OK && pick_k) {
    // steps per launch: time the whole handle at each k (probe steps rounded up to whole
    // launches) and keep the smallest k within 5 % of the best time per step (a larger k
    // only delays the host's view of the state)
    static const int ks[] = {1, 2, 5, 10, 20, 50, 100, 200, 500, 1000};
    float us_k[10];
    float best = INFINITY;
    int nk = 0;
    for (int k : ks) {
      if (k > probe_steps && nk > 0) break;
      const int steps = ((probe_steps + k - 1) / k) * k;
      float ms_best = INFINITY;
      for (int rep = 0; rep < 2 && st == ROD_OK; ++rep) {
        st = launch_steps(c, steps, k, true);
        float ms = 0;
        int nl = 0;
        if (st == ROD_OK) st = rod_last_step_time(c, &ms, &nl);
        ms_best = std::min(ms_best, ms);
      }
      if (st != ROD_OK) break;
      us_k[nk++] = 1000.f * ms_best / steps;
      best = std::min(best, us_k[nk - 1]);
    }
    if (st == ROD_OK)
      for (int i = 0; i < nk; ++i)
        if (us_k[i] <= 1.05f * best) {
          steps_per_launch = ks[i];
          break;
        }
  }
  c->steps_per_launch = steps_per_launch;
  c->steps_done = saved_steps;
  (void)reset_flags(c);
  if (copy(c->d_x, sx, bx) || copy(c->d_xl, sxl, bx) || copy(c->d_v, sv, bx) ||
      copy(c->d_q, sq, bq) || copy(c->d_ql, sql, bq) || copy(c->d_w, sw, bw)) {
    free_all();
    return fail(c, ROD_E_DEVICE, "autotune state restore failed");
  }
  (void)hipStreamSynchronize(c->stream);
  free_all();
  if (st != ROD_OK) return st;
  if (out) rod_get_tuning(c, out);
  return ROD_OK;
}

rod_status rod_set_stiffness_mult(rod_ctx* c, const float* bend, const float* twist) {
  if (!c || !bend || !twist) return fail(c, ROD_E_INVALID, "null argument");
  for (int r = 0; r < c->n_rods; ++r)
    if (!(std::isfinite(bend[r]) && bend[r] >= 0.f && std::isfinite(twist[r]) && twist[r] >= 0.f))
      return fail(c, ROD_E_INVALID, "multipliers must be finite and >= 0");
  for (int r = 0; r < c->n_rods; ++r) {
    c->rods[r].mult_bend = bend[r];
    c->rods[r].mult_twist = twist[r];
  }
  HIP_TRY(c, hipMemcpyAsync(c->d_rods, c->rods.data(), sizeof(RodDev) * c->n_rods,
                            hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->adj_ready = false;
  return ROD_OK;
}

rod_status rod_adjoint_forward(rod_ctx* c, int32_t n_steps, int32_t ckpt_every, float* tips,
                               int32_t on_device, int64_t* rollout) {
  if (!c) return fail(nullptr, ROD_E_INVALID, "null handle");
  if (!c->have_state) return fail(c, ROD_E_ORDER, "rod_adjoint_forward before rod_set_state");
  if (n_steps < 1 || ckpt_every < 1) return fail(c, ROD_E_INVALID, "n_steps and ckpt_every must be >= 1");
  for (const auto& r : c->rods)
    if (r.n_iter > corde::kAdjointMaxIter)
      return fail(c, ROD_E_UNSUPPORTED, "adjoint supports at most 10 constraint iterations");
  for (const auto& b : c->buckets)
    if (!adjoint_shape(b.max_n)) return fail(c, ROD_E_UNSUPPORTED, "rod too long for the adjoint kernel");
  if (c->n_chunks)
    return fail(c, ROD_E_UNSUPPORTED,
                "chunked rods are not differentiated (rod_set_chunking(ctx, 2048, 0) restores the default split)");
  if (!c->groups.empty()) return fail(c, ROD_E_UNSUPPORTED, "the adjoint does not step grouped rods");
  if (c->n_haptic) return fail(c, ROD_E_UNSUPPORTED, "the adjoint does not step rods with a haptic mailbox");
  if (c->env_nodes) return fail(c, ROD_E_UNSUPPORTED, "the adjoint does not step rods against an environment");
  for (const auto& r : c->rods)
    if (r.damp_int > 0.f) return fail(c, ROD_E_UNSUPPORTED, "the adjoint does not differentiate internal friction");
  c->adj_ready = false;
  const size_t S = state_floats(c);
  const int ck = std::min(ckpt_every, n_steps);
  const int nck = (n_steps + ck - 1) / ck;
  if (!ensure_adjoint(c, n_steps, ck)) {
    free_adjoint(c);
    return fail(c, ROD_E_NOMEM, "adjoint buffers do not fit");
  }
  c->adj_steps = n_steps;
  c->adj_ckpt = ck;
  c->adj_nckpt = nck;
  c->adj_step0 = c->steps_done;
  for (int seg = 0; seg < nck; ++seg) {
    const int len = std::min(ck, n_steps - seg * ck);
    // the launch writes its initial state: the checkpoint (or, with ck = 1, the stored step)
    float* traj = (ck == 1 ? c->d_traj : c->d_ckpt) + (size_t)seg * S;
    rod_status st = launch_forward_on(c, handle_state(c), len, c->steps_done, traj, c->d_tips,
                                      c->adj_step0, 1, 1);
    if (st != ROD_OK) return st;
    c->steps_done += len;
  }
  if (tips) {
    const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    HIP_TRY(c, hipMemcpyAsync(tips, c->d_tips, sizeof(float) * 3 * c->n_rods * n_steps, k, c->stream));
    if (!on_device) HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  c->adj_ready = true;
  c->adj_serial = ++c->adj_count;
  if (rollout) *rollout = c->adj_serial;
  return ROD_OK;
}

rod_status rod_adjoint_backward(rod_ctx* c, int64_t rollout, const float* dl_dtips,
                                float* dl_dbend, float* dl_dtwist, float* dl_dx, float* dl_dv,
                                float* dl_dq, float* dl_dw, int32_t on_device) {
  if (!c) return fail(nullptr, ROD_E_INVALID, "null handle");
  if (!c->adj_ready) return fail(c, ROD_E_ORDER, "rod_adjoint_backward without rod_adjoint_forward");
  if (rollout != 0 && rollout != c->adj_serial)
    return fail(c, ROD_E_ORDER, "rollout " + std::to_string(rollout) +
                " is no longer held (the handle holds rollout " + std::to_string(c->adj_serial) + ")");
  if (c->n_chunks)
    return fail(c, ROD_E_UNSUPPORTED,
                "chunked rods are not differentiated (rod_set_chunking(ctx, 2048, 0) restores the default split)");
  if (!dl_dtips) return fail(c, ROD_E_INVALID, "null dL/dtip");
  const size_t S = state_floats(c);
  const size_t P3 = (size_t)3 * c->total_pts, F4 = (size_t)4 * c->total_frames;
  const hipMemcpyKind kin = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  HIP_TRY(c, hipMemcpyAsync(c->d_dtips, dl_dtips, sizeof(float) * 3 * c->n_rods * c->adj_steps, kin, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->d_adj, 0, sizeof(float) * S, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->d_gacc, 0, sizeof(double) * 2 * corde::kAdjointMaxLanes * c->n_rods,
                            c->stream));
  const long long Sl = (long long)S;
  const int nck = c->adj_nckpt, ck = c->adj_ckpt;
  auto reverse = [&](int seg, const float* traj) -> rod_status {
    const int len = std::min(ck, c->adj_steps - seg * ck);
    const long long tstep0 = c->adj_step0 + (long long)seg * ck;
    for (const auto& b : c->buckets) {
      const AdjointEntry* a = adjoint_shape(b.max_n, b.waves, b.elems);
      if (!a || 64 * a->waves > corde::kAdjointMaxLanes)
        return fail(c, ROD_E_UNSUPPORTED, "no adjoint kernel for this bucket");
      hipLaunchKernelGGL(a->fn, dim3(b.count), dim3(64 * a->waves), 0, c->stream, c->d_rods,
                         c->d_rod_ids + b.first, c->d_prm, c->prm_stride, traj, Sl, c->total_pts,
                         c->total_frames, len, tstep0, seg * ck, c->d_dtips, c->adj_steps,
                         c->d_adj, c->d_adj + P3, c->d_adj + 2 * P3, c->d_adj + 2 * P3 + F4,
                         c->d_gacc, c->d_fext, c->d_text, c->d_status);
      HIP_TRY(c, hipGetLastError());
    }
    return ROD_OK;
  };
  if (ck == 1) {
    for (int seg = nck - 1; seg >= 0; --seg) {
      rod_status st = reverse(seg, c->d_traj + (size_t)seg * S);
      if (st != ROD_OK) return st;
    }
  } else {
    // segment k - 1 is recomputed from its checkpoint (every step start stored in one of two
    // buffers) on the second stream while segment k is reversed on the handle's stream
    float* tb[2] = {c->d_traj, c->d_traj + (size_t)ck * S};
    auto recompute = [&](int seg) -> rod_status {
      const int len = std::min(ck, c->adj_steps - seg * ck);
      const long long tstep0 = c->adj_step0 + (long long)seg * ck;
      float* cp = c->d_ckpt + (size_t)seg * S;
      rod_status st = launch_forward_on(c, corde::state_at(cp, c->total_pts, c->total_frames), len,
                                        tstep0, tb[seg & 1], nullptr, 0, len, 0, c->aux);
      if (st != ROD_OK) return st;
      HIP_TRY(c, hipEventRecord(c->ev_rec[seg & 1], c->aux));
      return ROD_OK;
    };
    HIP_TRY(c, hipEventRecord(c->ev_start, c->stream));
    HIP_TRY(c, hipStreamWaitEvent(c->aux, c->ev_start, 0));
    rod_status st = recompute(nck - 1);
    if (st != ROD_OK) return st;
    for (int seg = nck - 1; seg >= 0; --seg) {
      HIP_TRY(c, hipStreamWaitEvent(c->stream, c->ev_rec[seg & 1], 0));
      st = reverse(seg, tb[seg & 1]);
      if (st != ROD_OK) return st;
      HIP_TRY(c, hipEventRecord(c->ev_rev[seg & 1], c->stream));
      if (seg > 0) {
        // buffer (seg - 1) & 1 was last read by the reverse pass of segment seg + 1
        if (seg + 1 < nck) HIP_TRY(c, hipStreamWaitEvent(c->aux, c->ev_rev[(seg + 1) & 1], 0));
        st = recompute(seg - 1);
        if (st != ROD_OK) return st;
      }
    }
  }
  const hipMemcpyKind kout = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (dl_dx) HIP_TRY(c, hipMemcpyAsync(dl_dx, c->d_adj, sizeof(float) * P3, kout, c->stream));
  if (dl_dv) HIP_TRY(c, hipMemcpyAsync(dl_dv, c->d_adj + P3, sizeof(float) * P3, kout, c->stream));
  if (dl_dq) HIP_TRY(c, hipMemcpyAsync(dl_dq, c->d_adj + 2 * P3, sizeof(float) * F4, kout, c->stream));
  if (dl_dw) HIP_TRY(c, hipMemcpyAsync(dl_dw, c->d_adj + 2 * P3 + F4, sizeof(float) * 3 * c->total_frames, kout, c->stream));
  if (dl_dbend || dl_dtwist) {
    // fixed-order FP64 sums over the steps, into the first 2 n_rods floats of d_dtips (the
    // loss gradient is no longer needed) and from there to the caller
    float* gb = c->d_dtips;
    float* gt = c->d_dtips + c->n_rods;
    hipLaunchKernelGGL(corde::sum_multiplier_grads, dim3((c->n_rods + 63) / 64), dim3(64), 0,
                       c->stream, c->d_gacc, c->n_rods, gb, gt);
    HIP_TRY(c, hipGetLastError());
    if (dl_dbend) HIP_TRY(c, hipMemcpyAsync(dl_dbend, gb, sizeof(float) * c->n_rods, kout, c->stream));
    if (dl_dtwist) HIP_TRY(c, hipMemcpyAsync(dl_dtwist, gt, sizeof(float) * c->n_rods, kout, c->stream));
  }
  int stt = 0;
  HIP_TRY(c, hipMemcpyAsync(&stt, c->d_status, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (stt) return fail(c, ROD_E_UNSTABLE, "non-finite value in the adjoint");
  return ROD_OK;
}

}  // extern "C"
