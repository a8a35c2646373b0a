// Per-sample arithmetic of one rollout step shared by the rollout kernels:
// the Euler step and its Jacobian, the covariance propagation, the
// chance-constraint geometry and the stage cost (Eqs. 1, 10-16), and the
// per-step trace rows.
#pragma once
#include "device_common.hpp"
#include "kernels.hpp"

namespace gpmppi {

// Tightened distance to one obstacle (Eqs. 14, 16): the centre distance rho
// less the radius, less z_p times the position deviation along the centre
// direction n = (dx, dy) / rho, n^T Sigma n = (sa dx^2 + 2 sb dx dy + sc dy^2) / rho^2;
// at rho = 0 the direction is undefined and the largest eigenvalue stands in.
// One reciprocal square root gives both rho and 1 / rho^2.
__device__ __forceinline__ float obstacle_margin(float dx, float dy, float radius, float sa, float sb, float sc,
                                                 float lmax, float z_p) {
    const float rho2 = dx * dx + dy * dy;
    const bool pos = rho2 > 0.0f;
    const float rs = __builtin_amdgcn_rsqf(rho2);
    const float rho = pos ? rho2 * rs : 0.0f;
    const float quad = sa * dx * dx + 2.0f * sb * dx * dy + sc * dy * dy;
    const float vn = pos ? quad * (rs * rs) : lmax;
    return (rho - radius) - z_p * __builtin_amdgcn_sqrtf(fmaxf(vn, 0.0f));
}

// The 15 entries of a sample's symmetric 5x5 state covariance (Eq. 10).
struct Cov {
    float p00, p01, p02, p03, p04, p11, p12, p13, p14, p22, p23, p24, p33, p34, p44;
};

// Jacobian of the Euler step: identity plus a02, a03 (row x), a12, a13 (row y),
// a24 (row theta), diagonal a33, a44 for the velocities.
struct StepJac {
    float a02, a03, a12, a13, a24, a33, a44;
};

__device__ __forceinline__ StepJac step_jacobian(const Dyn &dy, float v, float sth, float cth) {
    const float dt = dy.dt;
    return StepJac{-dt * v * sth, dt * cth, dt * v * cth, dt * sth, dt, dy.a33, dy.a44};
}

// Sigma <- A Sigma A^T (Eq. 10, without the GP variance, which the caller adds):
// B = A Sigma by rows, then Sigma+_ij = sum_n B_in A_jn for i <= j.  Every
// product-sum is an explicit fused multiply-add, so the rounding does not depend
// on how the compiler contracts the surrounding code (the split rollout computes
// the position block apart from the rest and must reproduce it exactly).
__device__ __forceinline__ void propagate_cov(Cov &c, const StepJac &j) {
    const float a02 = j.a02, a03 = j.a03, a12 = j.a12, a13 = j.a13, a24 = j.a24, a33 = j.a33, a44 = j.a44;
    const float b00 = fmaf(a03, c.p03, fmaf(a02, c.p02, c.p00)), b01 = fmaf(a03, c.p13, fmaf(a02, c.p12, c.p01)),
                b02 = fmaf(a03, c.p23, fmaf(a02, c.p22, c.p02)), b03 = fmaf(a03, c.p33, fmaf(a02, c.p23, c.p03)),
                b04 = fmaf(a03, c.p34, fmaf(a02, c.p24, c.p04));
    const float b11 = fmaf(a13, c.p13, fmaf(a12, c.p12, c.p11)), b12 = fmaf(a13, c.p23, fmaf(a12, c.p22, c.p12)),
                b13 = fmaf(a13, c.p33, fmaf(a12, c.p23, c.p13)), b14 = fmaf(a13, c.p34, fmaf(a12, c.p24, c.p14));
    const float b22 = fmaf(a24, c.p24, c.p22), b23 = fmaf(a24, c.p34, c.p23), b24 = fmaf(a24, c.p44, c.p24);
    const float b33 = a33 * c.p33, b34 = a33 * c.p34;
    const float b44 = a44 * c.p44;
    c.p00 = fmaf(a03, b03, fmaf(a02, b02, b00));
    c.p01 = fmaf(a13, b03, fmaf(a12, b02, b01));
    c.p02 = fmaf(a24, b04, b02);
    c.p03 = a33 * b03;
    c.p04 = a44 * b04;
    c.p11 = fmaf(a13, b13, fmaf(a12, b12, b11));
    c.p12 = fmaf(a24, b14, b12);
    c.p13 = a33 * b13;
    c.p14 = a44 * b14;
    c.p22 = fmaf(a24, b24, b22);
    c.p23 = a33 * b23;
    c.p24 = a44 * b24;
    c.p33 = a33 * b33;
    c.p34 = a44 * b34;
    c.p44 = a44 * b44;
}

// The position block (Sigma_xx, Sigma_xy, Sigma_yy) of A Sigma A^T alone, by the
// same operations as propagate_cov; it does not involve the velocity variances'
// own entries p04, p14, p24, p34, p44.
__device__ __forceinline__ void propagate_pos_block(const Cov &c, const StepJac &j, float &sa, float &sb,
                                                    float &sc) {
    const float a02 = j.a02, a03 = j.a03, a12 = j.a12, a13 = j.a13;
    const float b00 = fmaf(a03, c.p03, fmaf(a02, c.p02, c.p00)), b01 = fmaf(a03, c.p13, fmaf(a02, c.p12, c.p01)),
                b02 = fmaf(a03, c.p23, fmaf(a02, c.p22, c.p02)), b03 = fmaf(a03, c.p33, fmaf(a02, c.p23, c.p03));
    const float b11 = fmaf(a13, c.p13, fmaf(a12, c.p12, c.p11)), b12 = fmaf(a13, c.p23, fmaf(a12, c.p22, c.p12)),
                b13 = fmaf(a13, c.p33, fmaf(a12, c.p23, c.p13));
    sa = fmaf(a03, b03, fmaf(a02, b02, b00));
    sb = fmaf(a13, b03, fmaf(a12, b02, b01));
    sc = fmaf(a13, b13, fmaf(a12, b12, b11));
}

// The GP variance s2 of a step into a velocity variance (Eq. 10): p += dt^2 s2.
__device__ __forceinline__ void add_gp_variance(float &p, float dt, float s2) { p = fmaf(dt * dt, s2, p); }

// Position and heading after one explicit Euler step (Eqs. 1, 10), as explicit
// fused multiply-adds (both roles of the split rollout integrate them and must
// agree bit for bit).
__device__ __forceinline__ void advance_pose(const Dyn &dy, float v, float w, float sth, float cth, float &X, float &Y,
                                             float &th) {
    const float dv = dy.dt * v;
    X = fmaf(dv, cth, X);
    Y = fmaf(dv, sth, Y);
    th = fmaf(dy.dt, w, th);
}

// Velocities after one explicit Euler step of the dynamic unicycle plus the GP
// residual means m0, m1 (Eqs. 1, 2, 10).
__device__ __forceinline__ void advance_velocities(const Dyn &dy, float2 u, float m0, float m1, float &v, float &w) {
    const float v_old = v, w_old = w;
    v = v_old + (dy.dt_tau_v * (u.x - v_old) + dy.dt * m0);
    w = w_old + (dy.dt_tau_w * (u.y - w_old) + dy.dt * m1);
}

// One wave's share of the polyline (oo = 0) or obstacle (oo = 1) loop at the
// position (Xs, Ys) and position covariance (sa, sb, sc), for waves wv < LW:
// the squared distance to segments wv, wv + LW, ... goes to ored[wv][sl], the
// least tightened obstacle distance over obstacles wv, wv + LW, ... to
// ored[LW + wv][sl].  Segments and obstacles are wave-uniform (scalar cache).
template <int LW, int B>
__device__ __forceinline__ void world_loop(const Geometry &geo, int oo, int wv, int sl, float Xs, float Ys, float sa,
                                           float sb, float sc, float lmax, float *ored) {
    if (wv >= LW) return;
    if (oo == 0) {
        if (geo.path_kind == 0) return;
        float best = INFINITY;
        const const_v4p segs = (const_v4p)geo.seg;
        const const_fp sinv = (const_fp)geo.seg_inv;
#pragma unroll 4
        for (int i = wv; i < geo.P; i += LW) {
            const v4f sgm = segs[i];
            const float rx = Xs - sgm.x, ry = Ys - sgm.y;
            float t = (rx * sgm.z + ry * sgm.w) * sinv[i];
            t = fminf(fmaxf(t, 0.0f), 1.0f);
            const float ex = rx - t * sgm.z, ey = ry - t * sgm.w;
            best = fminf(best, ex * ex + ey * ey);
        }
        ored[wv * B + sl] = best;
    } else {
        float om = INFINITY;
        const const_v4p obs = (const_v4p)geo.obs;
#pragma unroll 2
        for (int j = wv; j < geo.n_obs; j += LW) {
            const v4f ob = obs[j];
            om = fminf(om, obstacle_margin(Xs - ob.x, Ys - ob.y, ob.z, sa, sb, sc, lmax, geo.z_p));
        }
        ored[(LW + wv) * B + sl] = om;
    }
}

// What a step's cost needs besides the GP variances: the lane deviation dl and
// tightened half-width rbar (Eqs. 13, 15), the least tightened obstacle
// distance om (Eqs. 14, 16), the speed error dv and the goal distance dg.
struct StageIn {
    float dl, rbar, om, dv, dg;
};

// Reduces the loop results of ored (written before the contraction's last
// barrier) and forms the step's StageIn at the position (X, Y) and speed v.
// POLY = false: the polyline part is left to the caller (dl = 0 on a polyline).
template <int LW, int B, bool POLY = true>
__device__ __forceinline__ StageIn stage_inputs(const Geometry &geo, const CostWeights &cw, const float *ored, int sl,
                                                float X, float Y, float v, float lmax, float &dgoal_min) {
    float best_all = INFINITY, om = INFINITY;
#pragma unroll
    for (int p = 0; p < LW; ++p) {
        if (POLY && geo.path_kind != 0) best_all = fminf(best_all, ored[p * B + sl]);
        om = fminf(om, ored[(LW + p) * B + sl]);
    }
    StageIn t;
    if (geo.path_kind == 0) {
        const float dx = X - geo.cx, dyy = Y - geo.cy;
        t.dl = fabsf(sqrtf(dx * dx + dyy * dyy) - geo.R);
    } else {
        t.dl = POLY ? sqrtf(best_all) : 0.0f;
    }
    t.rbar = geo.half_width - geo.c_p * sqrtf(fmaxf(lmax, 0.0f));
    t.om = om;
    t.dv = cw.v_des - v;
    t.dg = 0.0f;
    if (cw.w_goal != 0.0f || cw.w_term != 0.0f) {   // goal terms (Eq. 12)
        const float gx = X - cw.goal_x, gy = Y - cw.goal_y;
        t.dg = sqrtf(gx * gx + gy * gy);
        dgoal_min = fminf(dgoal_min, t.dg);
    }
    return t;
}

// Stage cost (Eqs. 11-12 terms) added to the Kahan-compensated sum (S, Sc) of
// Eq. (5); the lane term is discounted by disc, which then advances.
__device__ __forceinline__ void add_stage_cost(const CostWeights &cw, const Geometry &geo, const StageIn &t, float s2a,
                                               float s2b, float &disc, float &S, float &Sc) {
    float c = cw.w_var * (s2a + s2b) + cw.w_dev * (t.dl * geo.inv_half_width) + cw.w_speed * (t.dv * t.dv);
    if (t.dl > t.rbar) c += cw.w_lane * disc;
    if (t.om <= 0.0f) c += cw.w_obs;
    if (cw.w_goal != 0.0f || cw.w_term != 0.0f) c += cw.w_goal * t.dg;
    const float yk = c - Sc;
    const float tk = S + yk;
    Sc = (tk - S) - yk;
    S = tk;
    disc *= cw.discount;
}

// Per-step trace rows of sample sg (K samples) at step k; var1 = false skips
// the second output's variance and lane = false the lane rows, which the split
// rollout writes one step later (write_deferred_trace).
__device__ __forceinline__ void write_trace(const gpmppi_trace &tr, int K, int sg, int k, float X, float Y, float th,
                                            float v, float w, const Cov &P, float m0, float m1, float s20, float s21,
                                            const StageIn &t, float2 u, bool var1, bool lane = true) {
    const size_t kk = (size_t)k;
    if (tr.x_d) {
        float *xd = tr.x_d + (kk + 1) * 5 * K;
        xd[0 * K + sg] = X;
        xd[1 * K + sg] = Y;
        xd[2 * K + sg] = th;
        xd[3 * K + sg] = v;
        xd[4 * K + sg] = w;
    }
    if (tr.sxy_d) {
        float *sd = tr.sxy_d + (kk + 1) * 3 * K;
        sd[0 * K + sg] = P.p00;
        sd[1 * K + sg] = P.p01;
        sd[2 * K + sg] = P.p11;
    }
    if (tr.gp_mean_d) {
        tr.gp_mean_d[(kk * 2 + 0) * K + sg] = m0;
        tr.gp_mean_d[(kk * 2 + 1) * K + sg] = m1;
    }
    if (tr.gp_var_d) {
        tr.gp_var_d[(kk * 2 + 0) * K + sg] = s20;
        if (var1) tr.gp_var_d[(kk * 2 + 1) * K + sg] = s21;
    }
    if (lane && tr.d_lane_d) tr.d_lane_d[kk * K + sg] = t.dl;
    if (lane && tr.lane_margin_d) tr.lane_margin_d[kk * K + sg] = t.rbar - t.dl;
    if (tr.obs_margin_d) tr.obs_margin_d[kk * K + sg] = t.om;
    if (tr.u_d) {
        tr.u_d[(kk * 2 + 0) * K + sg] = u.x;
        tr.u_d[(kk * 2 + 1) * K + sg] = u.y;
    }
}

// The rows write_trace(..., false, false) left out: the second variance and the lane rows.
__device__ __forceinline__ void write_deferred_trace(const gpmppi_trace &tr, int K, int sg, int k, float s21,
                                                     const StageIn &t) {
    const size_t kk = (size_t)k;
    if (tr.gp_var_d) tr.gp_var_d[(kk * 2 + 1) * K + sg] = s21;
    if (tr.d_lane_d) tr.d_lane_d[kk * K + sg] = t.dl;
    if (tr.lane_margin_d) tr.lane_margin_d[kk * K + sg] = t.rbar - t.dl;
}

}  // namespace gpmppi
