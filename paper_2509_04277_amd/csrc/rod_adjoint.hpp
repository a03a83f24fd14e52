// rod_adjoint.hpp -- reverse-mode (adjoint) kernel of the CoRdE rod stepper for gfx950.
//
// The forward step S_{n+1} = Phi(S_n; m_b, m_t) is the semi-implicit Euler step of the paper's
// Sec. 2.1 (rod_kernels.hpp); m_b, m_t are per-rod multipliers of the bend and twist
// stiffness (eq. (3)).  Given lambda_{n+1} = dL/dS_{n+1}, this kernel computes
//   lambda_n = (dPhi/dS_n)^T lambda_{n+1} + dL/dS_n,   dL/dm += (dPhi/dm)^T lambda_{n+1}
// for the steps of one checkpoint segment, newest first, with lambda held in registers.  For
// each step it reloads S_n, recomputes the step's internals with the forward code (saving the
// predicted segment vector of every constraint half-sweep), then applies the transposed
// Jacobians in reverse order:
//   X  positions / quaternions:  q' = p / |p|, p = q + dt/2 q (x) (0, omega')
//   C  the red-black distance impulses, last half-sweep first
//   V  force integration (particles; rigid bodies with the gyroscopic term)
//   F  segment forces (eqs. (2), (4), (7), (8)) and joint torques (eqs. (3), (5), (6))
// The loss enters through dL/d tip(s): tip(s) = x_N after step s.
#pragma once

#include "rod_kernels.hpp"

namespace corde {

constexpr int kAdjointMaxIter = 10;   // constraint iterations the adjoint kernel holds
constexpr int kAdjointMaxLanes = 512;  // lanes per rod of the widest adjoint kernel (8 waves)
constexpr int P_WINV_NEXT = P_NROWS;  // extra coefficient row: inverse mass of point j+2

__device__ __forceinline__ Q4 q_add(Q4 a, Q4 b) { return {a.w + b.w, a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ Q4 q_scale(float s, Q4 a) { return {s * a.w, s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ float q_dot(Q4 a, Q4 b) { return a.w * b.w + a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ Q4 qfma(float s, Q4 a, Q4 b) {   // s a + b, fused per component
  return {__builtin_fmaf(s, a.w, b.w), __builtin_fmaf(s, a.x, b.x), __builtin_fmaf(s, a.y, b.y),
          __builtin_fmaf(s, a.z, b.z)};
}

// Adjoint of one distance impulse.  Inputs: predicted segment vector d (before the impulse),
// coefficients ci, cil, inverse masses, and the adjoints gl, gh of the two end velocities after
// the impulse.  Returns dbar = dL/dd; the end-velocity adjoints before the impulse are
// gh + dt dbar (right end) and gl - dt dbar (left end).
__device__ __forceinline__ V3 impulse_adjoint(V3 d, float ci, float cil, float wl, float wh, V3 gl,
                                              V3 gh) {
  const float il = rsqrtf(fmaxf(dot(d, d), 1e-30f));
  const float s = ci - cil * il;
  const V3 Db = fnma3(wh, gh, wl * gl);     // Delta = s d; v_hi -= w_hi Delta; v_lo += w_lo Delta
  const float sb = dot(Db, d);
  return fma3(sb * cil * il * il * il, d, s * Db);
}

template <int W, int E>
__global__ __launch_bounds__(64 * W) void rod_adjoint_kernel(
    const RodDev* __restrict__ rods, const int* __restrict__ rod_ids, const float* __restrict__ prm,
    int prm_stride, const float* __restrict__ traj, long long traj_stride, int n_pts, int n_frames,
    int n_seg, long long tstep0, int tip0, const float* __restrict__ dtips, int tip_steps,
    float* __restrict__ ax, float* __restrict__ av, float* __restrict__ aq, float* __restrict__ aw,
    double* __restrict__ gacc, const float* __restrict__ fext, const float* __restrict__ text,
    int* __restrict__ status) {
  __shared__ Mailbox<W, kMergedExchange<W, E>> mb;
  mailbox_init(mb);
  const int rod = rod_ids[blockIdx.x];
  const RodDev rd = rods[rod];
  RodLane<W, E> L;
  L.load_params(rd, prm, prm_stride);
  const int g = L.g, j0 = L.j0;
  const float dt = L.dt;
  int par = 0;

  // coefficients without the stiffness multipliers, and the right-neighbour inverse mass
  float C1b[E], C3b[E], D0b[E], D1b[E], D2b[E], WN[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int o = rd.slot_off + j0 + e;
    const bool ok = L.ok[e];
    C1b[e] = ok ? prm[P_C1 * prm_stride + o] : 0.f;
    C3b[e] = ok ? prm[P_C3 * prm_stride + o] : 0.f;
    D0b[e] = ok ? prm[P_D0 * prm_stride + o] : 0.f;
    D1b[e] = ok ? prm[P_D1 * prm_stride + o] : 0.f;
    D2b[e] = ok ? prm[P_D2 * prm_stride + o] : 0.f;
    WN[e] = ok ? prm[P_WINV_NEXT * prm_stride + o] : 0.f;
  }

  // adjoint state lambda (same slot layout as the state)
  V3 AX[E], AV[E], AW[E];
  Q4 AQ[E];
  V3 abx = {0.f, 0.f, 0.f}, abv = {0.f, 0.f, 0.f};
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int j = j0 + e;
    if (L.ok[e]) {
      const float* p = ax + 3 * (rd.pt_off + j + 1);
      AX[e] = {p[0], p[1], p[2]};
      p = av + 3 * (rd.pt_off + j + 1);
      AV[e] = {p[0], p[1], p[2]};
      p = aq + 4 * (rd.fr_off + j);
      AQ[e] = {p[0], p[1], p[2], p[3]};
      p = aw + 3 * (rd.fr_off + j);
      AW[e] = {p[0], p[1], p[2]};
    } else {
      AX[e] = AV[e] = AW[e] = {0.f, 0.f, 0.f};
      AQ[e] = {0.f, 0.f, 0.f, 0.f};
    }
  }
  if (g == 0) {
    const float* p = ax + 3 * rd.pt_off;
    abx = {p[0], p[1], p[2]};
    p = av + 3 * rd.pt_off;
    abv = {p[0], p[1], p[2]};
  }
  const int tip_lane = (rd.n - 1) / E, tip_e = (rd.n - 1) % E;
  const bool clamp0 = rd.clamp && g == 0;   // this lane holds the kinematic frame 0 / point 0
  // this lane's multiplier gradients, accumulated in FP64 over all steps newest first (the
  // same sequence of additions for every checkpoint interval) and kept between launches
  double* acc = gacc + ((long long)rod * kAdjointMaxLanes + threadIdx.x) * 2;
  double gb_acc = acc[0], gt_acc = acc[1];

  // S_n and dL/dtip(n) of the next step to reverse are loaded one step ahead
  RodLane<W, E> S;
  S.off = 0;
#pragma unroll
  for (int e = 0; e < E; ++e) S.ok[e] = L.ok[e];
  S.g = g;
  S.j0 = j0;
  auto fetch = [&](int i, V3& dtip) {
    const float* base = traj + (long long)i * traj_stride;
    S.load_state(rd, state_at(const_cast<float*>(base), n_pts, n_frames));
    dtip = {0.f, 0.f, 0.f};
    if (dtips && g == tip_lane) {
      const float* pt = dtips + ((long long)rod * tip_steps + tip0 + i) * 3;
      dtip = {pt[0], pt[1], pt[2]};
    }
  };
  V3 dtip_next;
  fetch(n_seg - 1, dtip_next);

  for (int i = n_seg - 1; i >= 0; --i) {
    float gb = 0.f, gt = 0.f;
    // ---- S_n, loss gradient of the tip after this step, clamp pose
#pragma unroll
    for (int e = 0; e < E; ++e) {
      L.X[e] = S.X[e];
      L.XL[e] = S.XL[e];
      L.Vv[e] = S.Vv[e];
      L.Qf[e] = S.Qf[e];
      L.QL[e] = S.QL[e];
      L.Om[e] = S.Om[e];
    }
    L.bx = S.bx;
    L.bxl = S.bxl;
    L.bv = S.bv;
    const V3 dtip = dtip_next;
    if (i > 0) fetch(i - 1, dtip_next);
    if (dtips && g == tip_lane) {
#pragma unroll
      for (int e = 0; e < E; ++e)
        if (e == tip_e) AX[e] = AX[e] + dtip;
    }
    V3 xc = {rd.cx0[0], rd.cx0[1], rd.cx0[2]}, wc = {0.f, 0.f, 0.f};
    Q4 qc = {rd.cq0[0], rd.cq0[1], rd.cq0[2], rd.cq0[3]};
    if (rd.driven && rd.clamp) clamp_pose(rd, rd.t0 + (double)(tstep0 + i + 1) * rd.dt_d, xc, qc, wc);

    // ---- recompute the forward step, keeping what the reverse needs
    V3 xl, xll;
    Q4 qn, qnl;
    L.exchange_a(mb, par, xl, xll, qn, qnl);
    V3 Om0[E];
    Q4 Q0[E], Q0L[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      Om0[e] = L.Om[e];
      Q0[e] = L.Qf[e];
      Q0L[e] = L.QL[e];
    }
    {
      V3 F[E], T[E], Ev[E], fs0, enext;
      L.forces(mb, par, xl, xll, qn, qnl, F, T, Ev, fs0, enext);
      L.integrate_forces(rd, F, T, fs0, xc, wc, fext, text);
      V3 ds[kAdjointMaxIter][2][E];
#pragma unroll
      for (int it = 0; it < kAdjointMaxIter; ++it) {
        if (it < rd.n_iter) {
          L.half_sweep(rd, mb, par, 0, Ev, enext, ds[it][0]);
          L.half_sweep(rd, mb, par, 1, Ev, enext, ds[it][1]);
        }
      }
      // L.Om = omega' (after force integration), L.Vv = v'' (after the impulses)

      // ---- reverse X: x' = x + dt v'', q' = normalize(q + dt/2 q (x) (0, omega'))
      V3 AVc[E], AWp[E];
      Q4 AQn[E];
      V3 AXn[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        AXn[e] = AX[e];
        AVc[e] = fma3(dt, AX[e], AV[e]);
        const Q4 q = Q0[e];
        const V3 o = L.Om[e];
        const float hdt = 0.5f * dt;
        const Q4 p = {q.w + hdt * (-q.x * o.x - q.y * o.y - q.z * o.z),
                      q.x + hdt * (q.w * o.x + q.y * o.z - q.z * o.y),
                      q.y + hdt * (q.w * o.y - q.x * o.z + q.z * o.x),
                      q.z + hdt * (q.w * o.z + q.x * o.y - q.y * o.x)};
        const float ip = rsqrtf(q_dot(p, p));
        const Q4 qo = q_scale(ip, p);
        Q4 pb = q_scale(ip, qfma(-q_dot(qo, AQ[e]), qo, AQ[e]));
        if (clamp0 && e == 0) pb = {0.f, 0.f, 0.f, 0.f};   // q'_0 = q_c
        // dq: p_bar - dt/2 p_bar (x) (0, omega');  domega': dt/2 vec(conj(q) (x) p_bar)
        const Q4 po = qmul(pb, Q4{0.f, o.x, o.y, o.z});
        AQn[e] = {pb.w - hdt * po.w, pb.x - hdt * po.x, pb.y - hdt * po.y, pb.z - hdt * po.z};
        const Q4 cq = qmul(Q4{q.w, -q.x, -q.y, -q.z}, pb);
        AWp[e] = fma3(hdt, V3{cq.x, cq.y, cq.z}, AW[e]);
        if (clamp0 && e == 0) AWp[e] = {0.f, 0.f, 0.f};      // omega'_0 = omega_c
      }
      V3 abxn, abvc;
      if (rd.clamp) {
        abxn = {0.f, 0.f, 0.f};                               // x'_0 = x_c
        abvc = abv;
      } else {
        abxn = abx;
        abvc = fma3(dt, abx, abv);
      }

      // ---- reverse C: half-sweeps in reverse order
      V3 EB[E];
#pragma unroll
      for (int e = 0; e < E; ++e) EB[e] = {0.f, 0.f, 0.f};
#pragma unroll
      for (int it = kAdjointMaxIter - 1; it >= 0; --it) {
        if (it < rd.n_iter) {
#pragma unroll
          for (int h = 1; h >= 0; --h) {
            const bool cross_lanes = (E % 2 == 1) || (h == 0);
            V3 glo = {0.f, 0.f, 0.f}, ghi = {0.f, 0.f, 0.f};
            if (cross_lanes) {
              float mh[3] = {AVc[E - 1].x, AVc[E - 1].y, AVc[E - 1].z};
              float ml[3] = {AVc[0].x, AVc[0].y, AVc[0].z};
              const float base[3] = {abvc.x, abvc.y, abvc.z};
              float lo[3], hi[3];
              exchange<W, E, 3, 3, true, kMergedExchange<W, E>>(mh, lo, ml, hi, base, mb, par);
              glo = {lo[0], lo[1], lo[2]};
              ghi = {hi[0], hi[1], hi[2]};
              if (!kMergedExchange<W, E> && g == 0) glo = abvc;
            }
            V3 nv[E];
            V3 dbase = {0.f, 0.f, 0.f};
            if constexpr (E % 2 == 0) {
              // even E: the slots pair up as the two ends of one segment as in the forward
              // half-sweep (both ends saw the same segment vector and their coefficients agree:
              // a slot's next-segment ones are the next slot's own, its inverse mass is the next
              // slot's previous one), so one adjoint serves both ends
              auto pair = [&](int a) {
                const V3 db = impulse_adjoint(ds[it][h][a + 1], L.P[P_CI][a + 1], L.P[P_CIL][a + 1],
                                              L.P[P_WINV_PREV][a + 1], L.P[P_WINV][a + 1], AVc[a],
                                              AVc[a + 1]);
                nv[a] = fnma3(dt, db, AVc[a]);           // left end
                nv[a + 1] = fma3(dt, db, AVc[a + 1]);    // right end
                EB[a + 1] = EB[a + 1] + db;
              };
              if (h == 0) {
                const V3 db0 = impulse_adjoint(ds[it][0][0], L.P[P_CI][0], L.P[P_CIL][0],
                                               L.P[P_WINV_PREV][0], L.P[P_WINV][0], glo, AVc[0]);
                nv[0] = fma3(dt, db0, AVc[0]);
                EB[0] = EB[0] + db0;
                dbase = db0;
#pragma unroll
                for (int a = 1; a + 1 < E; a += 2) pair(a);
                const V3 dbl = impulse_adjoint(ds[it][0][E - 1], L.P[P_CI_NEXT][E - 1],
                                               L.P[P_CIL_NEXT][E - 1], L.P[P_WINV][E - 1], WN[E - 1],
                                               AVc[E - 1], ghi);
                nv[E - 1] = fnma3(dt, dbl, AVc[E - 1]);
              } else {
#pragma unroll
                for (int a = 0; a < E; a += 2) pair(a);
              }
            } else {
#pragma unroll
            for (int e = 0; e < E; ++e) {
              const int j = j0 + e;
              const bool is_hi = ((j & 1) == h);
              const float w_me = L.P[P_WINV][e];
              const V3 g_lo = (e == 0) ? glo : AVc[e - 1];
              const V3 g_hi = (e == E - 1) ? ghi : AVc[e + 1];
              const V3 d = ds[it][h][e];
              // as right end of segment j
              const V3 db_h = impulse_adjoint(d, L.P[P_CI][e], L.P[P_CIL][e], L.P[P_WINV_PREV][e],
                                              w_me, g_lo, AVc[e]);
              // as left end of segment j+1
              const V3 db_l = impulse_adjoint(d, L.P[P_CI_NEXT][e], L.P[P_CIL_NEXT][e], w_me,
                                              WN[e], AVc[e], g_hi);
              nv[e] = sel(is_hi, fma3(dt, db_h, AVc[e]), fnma3(dt, db_l, AVc[e]));
              EB[e] = sel(is_hi, EB[e] + db_h, EB[e]);
              if (e == 0) dbase = db_h;
            }
            }
#pragma unroll
            for (int e = 0; e < E; ++e) AVc[e] = nv[e];
            if (g == 0 && h == 0) abvc = fnma3(dt, dbase, abvc);  // base point: left end of segment 0
          }
        }
      }

      // ---- reverse V: v' = v + dt (w F + g - gamma v); omega' = omega + dt alpha(tau, omega)
      V3 FB[E], TB[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        FB[e] = (dt * L.P[P_WINV][e]) * AVc[e];
        AV[e] = (1.f - dt * rd.damp_lin) * AVc[e];
        const V3 a = dt * AWp[e];
        const float i1 = L.P[P_IINV1][e], i3 = L.P[P_IINV3][e], kg = L.P[P_GYRO][e];
        TB[e] = {i1 * a.x, i1 * a.y, i3 * a.z};
        const V3 o = Om0[e];
        const float ga = rd.damp_ang;
        AW[e] = {AWp[e].x - ga * a.x + kg * o.z * a.y, AWp[e].y - kg * o.z * a.x - ga * a.y,
                 AWp[e].z - kg * o.y * a.x + kg * o.x * a.y - ga * a.z};
        if (clamp0 && e == 0) {
          TB[e] = {0.f, 0.f, 0.f};
          AW[e] = {0.f, 0.f, 0.f};
        }
      }
      V3 fb0 = {0.f, 0.f, 0.f};   // adjoint of the base point's force (free base only)
      if (rd.clamp) {
        abxn = fnma3(1.0f / dt, abvc, abxn);                  // v'_0 = (x_c - x_0) / dt
        abv = {0.f, 0.f, 0.f};
      } else {
        fb0 = (dt * rd.winv0) * abvc;
        abv = (1.f - dt * rd.damp_lin) * abvc;
      }

      // ---- reverse F: segment and joint adjoints
      V3 fb_lo, tb_hi;
      {
        float mh[3] = {FB[E - 1].x, FB[E - 1].y, FB[E - 1].z};
        float ml[3] = {TB[0].x, TB[0].y, TB[0].z};
        const float base[3] = {fb0.x, fb0.y, fb0.z};
        float lo[3], hi[3];
        exchange<W, E, 3, 3, true, kMergedExchange<W, E>>(mh, lo, ml, hi, base, mb, par);
        fb_lo = {lo[0], lo[1], lo[2]};
        tb_hi = {hi[0], hi[1], hi[2]};
        if (!kMergedExchange<W, E> && g == 0) fb_lo = fb0;
      }
      V3 dneg_first = {0.f, 0.f, 0.f};
      Q4 qb_last = {0.f, 0.f, 0.f, 0.f};
      Q4 qb_prev = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const V3 d = Ev[e];                                   // the forward's segment vector
        const float len2 = dot(d, d);
        const float il = rsqrtf(len2);
        const V3 t = il * d;
        const float len = len2 * il;
        const Q4 q = Q0[e];
        const float ww = q.w * q.w, xx = q.x * q.x, yy = q.y * q.y, zz = q.z * q.z;
        const float xy = q.x * q.y, xz = q.x * q.z, yz = q.y * q.z;
        const float wx = q.w * q.x, wy = q.w * q.y, wz = q.w * q.z;
        const V3 d1 = {ww + xx - yy - zz, 2.f * (xy + wz), 2.f * (xz - wy)};
        const V3 d2 = {2.f * (xy - wz), ww - xx + yy - zz, 2.f * (yz + wx)};
        const V3 d3 = {2.f * (xz + wy), 2.f * (yz - wx), ww - xx - yy + zz};
        const float lkp = L.P[P_LKP][e], ksl = L.P[P_KS_L][e];
        const float td3 = dot(t, d3);
        // segment j: f (on point j+1, minus on point j) and the penalty torque on frame j
        const V3 fbar = sel(L.ok[e], FB[e] - ((e == 0) ? fb_lo : FB[e - 1]), V3{0.f, 0.f, 0.f});
        const V3 tpb = sel(L.ok[e], TB[e], V3{0.f, 0.f, 0.f});
        const float tf = dot(t, fbar);
        const V3 d3b = (lkp * il) * fnma3(tf, t, fbar);
        V3 tb = fnma3(ksl * (len - L.P[P_LEN][e]), fbar, (-lkp * il) * fma3(td3, fbar, tf * d3));
        tb = fma3(lkp, fnma3(tpb.x, d2, tpb.y * d1), tb);
        const V3 d2b = (-lkp * tpb.x) * t;
        const V3 d1b = (lkp * tpb.y) * t;
        const float ilb = lkp * (dot(d3, fbar) - td3 * tf);
        const float lenb = -ksl * tf;
        V3 db = fma3(lenb - ilb * il * il, t, il * fnma3(dot(t, tb), t, tb));
        db = sel(L.ok[e], db + EB[e], V3{0.f, 0.f, 0.f});     // + constraint use of e_j
        AXn[e] = AXn[e] + db;                                 // d = x_{j+1} - x_j
        if (e == 0) dneg_first = db;
        else AXn[e - 1] = AXn[e - 1] - db;
        // director Jacobians: q_bar += J1^T d1b + J2^T d2b + J3^T d3b
        const V3 a = d1b, b = d2b, c = d3b;
        Q4 qs = {2.f * (q.w * a.x + q.z * a.y - q.y * a.z) + 2.f * (-q.z * b.x + q.w * b.y + q.x * b.z) +
                     2.f * (q.y * c.x - q.x * c.y + q.w * c.z),
                 2.f * (q.x * a.x + q.y * a.y + q.z * a.z) + 2.f * (q.y * b.x - q.x * b.y + q.w * b.z) +
                     2.f * (q.z * c.x - q.w * c.y - q.x * c.z),
                 2.f * (-q.y * a.x + q.x * a.y - q.w * a.z) + 2.f * (q.x * b.x + q.y * b.y + q.z * b.z) +
                     2.f * (q.w * c.x + q.z * c.y - q.y * c.z),
                 2.f * (-q.z * a.x + q.w * a.y + q.x * a.z) + 2.f * (-q.w * b.x - q.z * b.y + q.y * b.z) +
                     2.f * (q.x * c.x + q.y * c.y + q.z * c.z)};
        // joint j between frames j (qa = q) and j+1 (qb)
        const Q4 qb = (e == E - 1) ? qn : Q0[e + 1];
        const Q4 qbl = (e == E - 1) ? qnl : Q0L[e + 1];
        const Q4 ql = Q0L[e];
        const Q4 dq = {(qb.w - q.w) + (qbl.w - ql.w), (qb.x - q.x) + (qbl.x - ql.x),
                       (qb.y - q.y) + (qbl.y - ql.y), (qb.z - q.z) + (qbl.z - ql.z)};
        const float rw = q.w * qb.w + q.x * qb.x + q.y * qb.y + q.z * qb.z;
        const V3 va = {q.x, q.y, q.z}, vb = {qb.x, qb.y, qb.z}, dv = {dq.x, dq.y, dq.z};
        const V3 rv = {q.w * dv.x - dq.w * va.x - (va.y * dv.z - va.z * dv.y),
                       q.w * dv.y - dq.w * va.y - (va.z * dv.x - va.x * dv.z),
                       q.w * dv.z - dq.w * va.z - (va.x * dv.y - va.y * dv.x)};
        const float C1 = L.P[P_C1][e], C3 = L.P[P_C3][e];
        const V3 m = {C1 * rv.x - L.P[P_D0][e], C1 * rv.y - L.P[P_D1][e], C3 * rv.z - L.P[P_D2][e]};
        const V3 tjb = tpb;                                   // tj goes to frame j
        const V3 tnb = sel(L.ok[e], (e == E - 1) ? tb_hi : TB[e + 1], V3{0.f, 0.f, 0.f});
        const float rwb = dot(m, tjb - tnb);
        const V3 cb = tjb + tnb;
        const V3 mb_ = fma3(rw, tjb - tnb, cross(cb, rv));
        const V3 rvb = {m.y * cb.z - m.z * cb.y + C1 * mb_.x, m.z * cb.x - m.x * cb.z + C1 * mb_.y,
                        m.x * cb.y - m.y * cb.x + C3 * mb_.z};
        gb += mb_.x * (C1b[e] * rv.x - D0b[e]) + mb_.y * (C1b[e] * rv.y - D1b[e]);
        gt += mb_.z * (C3b[e] * rv.z - D2b[e]);
        // rw = qa . qb ; rv = qa_w qb_v - qb_w qa_v - qa_v x qb_v
        const V3 qav = fnma3(qb.w, rvb, cross(rvb, vb));
        const V3 qbv = fma3(q.w, rvb, cross(va, rvb));
        const Q4 qa_b = {rwb * qb.w + dot(rvb, vb), rwb * qb.x + qav.x, rwb * qb.y + qav.y,
                         rwb * qb.z + qav.z};
        const Q4 qb_b = {rwb * q.w - dot(rvb, va), rwb * q.x + qbv.x, rwb * q.y + qbv.y,
                         rwb * q.z + qbv.z};
        qs = q_add(qs, qa_b);
        if (e > 0) qs = q_add(qs, qb_prev);
        AQn[e] = sel4(L.ok[e], q_add(AQn[e], qs), AQn[e]);
        qb_prev = qb_b;
        if (e == E - 1) qb_last = qb_b;
      }
      {
        float mh[4] = {qb_last.w, qb_last.x, qb_last.y, qb_last.z};
        float ml[3] = {dneg_first.x, dneg_first.y, dneg_first.z};
        const float base[4] = {0.f, 0.f, 0.f, 0.f};   // frame 0 has no joint below
        float lo[4], hi[3];
        exchange<W, E, 4, 3, false, kMergedExchange<W, E>>(mh, lo, ml, hi, base, mb, par);
        // joint j-1's adjoint for frame j (from below); segment j+1's -d for point j+1 (above)
        const Q4 qfrom = {lo[0], lo[1], lo[2], lo[3]};
        const V3 dfrom = {hi[0], hi[1], hi[2]};
        if (g != 0) AQn[0] = sel4(L.ok[0], q_add(AQn[0], qfrom), AQn[0]);
        AXn[E - 1] = sel(L.ok[E - 1], AXn[E - 1] - dfrom, AXn[E - 1]);
      }
      if (g == 0) abxn = abxn - dneg_first;                  // point 0 is segment 0's left end
#pragma unroll
      for (int e = 0; e < E; ++e) {
        AX[e] = AXn[e];
        AQ[e] = AQn[e];
      }
      abx = abxn;
    }
    gb_acc += (double)gb;
    gt_acc += (double)gt;
  }

  // ---- write lambda and this lane's multiplier-gradient accumulators
  acc[0] = gb_acc;
  acc[1] = gt_acc;
  if (!__builtin_isfinite(gb_acc + gt_acc)) atomicOr(status, 2);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int j = j0 + e;
    if (L.ok[e]) {
      float* p = ax + 3 * (rd.pt_off + j + 1);
      p[0] = AX[e].x; p[1] = AX[e].y; p[2] = AX[e].z;
      p = av + 3 * (rd.pt_off + j + 1);
      p[0] = AV[e].x; p[1] = AV[e].y; p[2] = AV[e].z;
      p = aq + 4 * (rd.fr_off + j);
      p[0] = AQ[e].w; p[1] = AQ[e].x; p[2] = AQ[e].y; p[3] = AQ[e].z;
      p = aw + 3 * (rd.fr_off + j);
      p[0] = AW[e].x; p[1] = AW[e].y; p[2] = AW[e].z;
    }
  }
  if (g == 0) {
    float* p = ax + 3 * rd.pt_off;
    p[0] = abx.x; p[1] = abx.y; p[2] = abx.z;
    p = av + 3 * rd.pt_off;
    p[0] = abv.x; p[1] = abv.y; p[2] = abv.z;
  }
  if (g == 0 && !__builtin_isfinite(abx.x + abx.y + abx.z + abv.x + abv.y + abv.z)) atomicOr(status, 2);
}

// Per-rod stiffness-multiplier gradients: the lanes' FP64 accumulators summed in lane order
// (one thread per rod; unused lanes hold 0).
__global__ void sum_multiplier_grads(const double* __restrict__ gacc, int n_rods,
                                     float* __restrict__ dbend, float* __restrict__ dtwist) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_rods) return;
  double sb = 0.0, st = 0.0;
  const double* g = gacc + (long long)r * kAdjointMaxLanes * 2;
  for (int l = 0; l < kAdjointMaxLanes; ++l) {
    sb += g[2 * l];
    st += g[2 * l + 1];
  }
  dbend[r] = (float)sb;
  dtwist[r] = (float)st;
}

}  // namespace corde
