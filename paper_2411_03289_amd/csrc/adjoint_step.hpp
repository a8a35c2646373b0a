// Per-sample algebra of the adjoint rollout (host and device): the
// covariance update Sigma+ = A Sigma A^T + dt^2 diag(0, 0, 0, s2_v, s2_w)
// (Eq. 10) on the 15 stored entries and its reverse, and one reversed step of
// everything but the GP: the smoothed stage cost (Eqs. 11-16 with sigmoid
// indicators), the covariance update, the Euler step (Eqs. 1, 2) and the
// Jacobian A(theta, v).
#pragma once
#include <math.h>

#include "kernels.hpp"

namespace gpmppi {

// p index: 00 01 02 03 04 11 12 13 14 22 23 24 33 34 44
struct Jac {
    float a02, a03, a12, a13;
};

__host__ __device__ inline void cov_forward(const float p[15], const Jac &J, float a24, float a33, float a44,
                                            float e3, float e4, float P[15]) {
    const float p00 = p[0], p01 = p[1], p02 = p[2], p03 = p[3], p04 = p[4], p11 = p[5], p12 = p[6], p13 = p[7],
                p14 = p[8], p22 = p[9], p23 = p[10], p24 = p[11], p33 = p[12], p34 = p[13], p44 = p[14];
    const float b00 = p00 + J.a02 * p02 + J.a03 * p03, b01 = p01 + J.a02 * p12 + J.a03 * p13,
                b02 = p02 + J.a02 * p22 + J.a03 * p23, b03 = p03 + J.a02 * p23 + J.a03 * p33,
                b04 = p04 + J.a02 * p24 + J.a03 * p34;
    const float b11 = p11 + J.a12 * p12 + J.a13 * p13, b12 = p12 + J.a12 * p22 + J.a13 * p23,
                b13 = p13 + J.a12 * p23 + J.a13 * p33, b14 = p14 + J.a12 * p24 + J.a13 * p34;
    const float b22 = p22 + a24 * p24, b23 = p23 + a24 * p34, b24 = p24 + a24 * p44;
    const float b33 = a33 * p33, b34 = a33 * p34, b44 = a44 * p44;
    P[0] = b00 + J.a02 * b02 + J.a03 * b03;
    P[1] = b01 + J.a12 * b02 + J.a13 * b03;
    P[2] = b02 + a24 * b04;
    P[3] = a33 * b03;
    P[4] = a44 * b04;
    P[5] = b11 + J.a12 * b12 + J.a13 * b13;
    P[6] = b12 + a24 * b14;
    P[7] = a33 * b13;
    P[8] = a44 * b14;
    P[9] = b22 + a24 * b24;
    P[10] = a33 * b23;
    P[11] = a44 * b24;
    P[12] = a33 * b33 + e3;
    P[13] = a44 * b34;
    P[14] = a44 * b44 + e4;
}

// Reverse of cov_forward: Pb (adjoint of P) -> pb (adjoint of p, overwritten),
// adjoints of a02 a03 a12 a13 added to Jb, of e3 and e4 returned.
__host__ __device__ inline void cov_backward(const float p[15], const Jac &J, float a24, float a33, float a44,
                                             const float Pb[15], float pb[15], Jac &Jb, float &e3b, float &e4b) {
    const float p02 = p[2], p03 = p[3], p12 = p[6], p13 = p[7], p22 = p[9], p23 = p[10], p24 = p[11], p33 = p[12],
                p34 = p[13];
    // forward intermediates needed by the reverse
    const float b02 = p02 + J.a02 * p22 + J.a03 * p23, b03 = p03 + J.a02 * p23 + J.a03 * p33;
    const float b12 = p12 + J.a12 * p22 + J.a13 * p23, b13 = p13 + J.a12 * p23 + J.a13 * p33;
    float bb00 = 0, bb01 = 0, bb02 = 0, bb03 = 0, bb04 = 0, bb11 = 0, bb12 = 0, bb13 = 0, bb14 = 0, bb22 = 0,
          bb23 = 0, bb24 = 0, bb33 = 0, bb34 = 0, bb44 = 0;
    // P00 = b00 + a02 b02 + a03 b03
    bb00 += Pb[0]; bb02 += J.a02 * Pb[0]; bb03 += J.a03 * Pb[0];
    Jb.a02 += b02 * Pb[0]; Jb.a03 += b03 * Pb[0];
    // P01 = b01 + a12 b02 + a13 b03
    bb01 += Pb[1]; bb02 += J.a12 * Pb[1]; bb03 += J.a13 * Pb[1];
    Jb.a12 += b02 * Pb[1]; Jb.a13 += b03 * Pb[1];
    // P02 = b02 + a24 b04; P03 = a33 b03; P04 = a44 b04
    bb02 += Pb[2]; bb04 += a24 * Pb[2];
    bb03 += a33 * Pb[3];
    bb04 += a44 * Pb[4];
    // P11 = b11 + a12 b12 + a13 b13
    bb11 += Pb[5]; bb12 += J.a12 * Pb[5]; bb13 += J.a13 * Pb[5];
    Jb.a12 += b12 * Pb[5]; Jb.a13 += b13 * Pb[5];
    // P12 = b12 + a24 b14; P13 = a33 b13; P14 = a44 b14
    bb12 += Pb[6]; bb14 += a24 * Pb[6];
    bb13 += a33 * Pb[7];
    bb14 += a44 * Pb[8];
    // P22 = b22 + a24 b24; P23 = a33 b23; P24 = a44 b24
    bb22 += Pb[9]; bb24 += a24 * Pb[9];
    bb23 += a33 * Pb[10];
    bb24 += a44 * Pb[11];
    // P33 = a33 b33 + e3; P34 = a44 b34; P44 = a44 b44 + e4
    bb33 += a33 * Pb[12]; e3b = Pb[12];
    bb34 += a44 * Pb[13];
    bb44 += a44 * Pb[14]; e4b = Pb[14];
    // b rows -> p
    float q[15] = {};
    // b00 = p00 + a02 p02 + a03 p03
    q[0] += bb00; q[2] += J.a02 * bb00; q[3] += J.a03 * bb00; Jb.a02 += p02 * bb00; Jb.a03 += p03 * bb00;
    // b01 = p01 + a02 p12 + a03 p13
    q[1] += bb01; q[6] += J.a02 * bb01; q[7] += J.a03 * bb01; Jb.a02 += p12 * bb01; Jb.a03 += p13 * bb01;
    // b02 = p02 + a02 p22 + a03 p23
    q[2] += bb02; q[9] += J.a02 * bb02; q[10] += J.a03 * bb02; Jb.a02 += p22 * bb02; Jb.a03 += p23 * bb02;
    // b03 = p03 + a02 p23 + a03 p33
    q[3] += bb03; q[10] += J.a02 * bb03; q[12] += J.a03 * bb03; Jb.a02 += p23 * bb03; Jb.a03 += p33 * bb03;
    // b04 = p04 + a02 p24 + a03 p34
    q[4] += bb04; q[11] += J.a02 * bb04; q[13] += J.a03 * bb04; Jb.a02 += p24 * bb04; Jb.a03 += p34 * bb04;
    // b11 = p11 + a12 p12 + a13 p13
    q[5] += bb11; q[6] += J.a12 * bb11; q[7] += J.a13 * bb11; Jb.a12 += p12 * bb11; Jb.a13 += p13 * bb11;
    // b12 = p12 + a12 p22 + a13 p23
    q[6] += bb12; q[9] += J.a12 * bb12; q[10] += J.a13 * bb12; Jb.a12 += p22 * bb12; Jb.a13 += p23 * bb12;
    // b13 = p13 + a12 p23 + a13 p33
    q[7] += bb13; q[10] += J.a12 * bb13; q[12] += J.a13 * bb13; Jb.a12 += p23 * bb13; Jb.a13 += p33 * bb13;
    // b14 = p14 + a12 p24 + a13 p34
    q[8] += bb14; q[11] += J.a12 * bb14; q[13] += J.a13 * bb14; Jb.a12 += p24 * bb14; Jb.a13 += p34 * bb14;
    // b22 = p22 + a24 p24; b23 = p23 + a24 p34; b24 = p24 + a24 p44
    q[9] += bb22; q[11] += a24 * bb22;
    q[10] += bb23; q[13] += a24 * bb23;
    q[11] += bb24; q[14] += a24 * bb24;
    // b33 = a33 p33; b34 = a33 p34; b44 = a44 p44
    q[12] += a33 * bb33;
    q[13] += a33 * bb34;
    q[14] += a44 * bb44;
#pragma unroll
    for (int i = 0; i < 15; ++i) pb[i] = q[i];
}

__host__ __device__ inline float sigm(float x) { return 1.0f / (1.0f + expf(-x)); }

// Largest eigenvalue of [[a, b], [b, c]] and its partial derivatives (the
// root's derivative taken as 0 where the root is 0).
__host__ __device__ inline float lmax_grad(float a, float b, float c, float &da, float &db, float &dc) {
    const float h = 0.5f * (a - c);
    const float s = sqrtf(h * h + b * b);
    if (s > 0.0f) {
        da = 0.5f + 0.5f * h / s;
        dc = 0.5f - 0.5f * h / s;
        db = b / s;
    } else {
        da = 0.5f;
        dc = 0.5f;
        db = 0.0f;
    }
    return 0.5f * (a + c) + s;
}


// Lane distance at (X, Y) (circle, or polyline segment iseg) and its gradient.
__host__ __device__ inline float lane_dist_grad(const Geometry &geo, float X, float Y, int iseg, float &gx,
                                                float &gy) {
    gx = 0.0f;
    gy = 0.0f;
    if (geo.path_kind == 0) {
        const float dx = X - geo.cx, dyy = Y - geo.cy;
        const float rho = sqrtf(dx * dx + dyy * dyy);
        const float d = rho - geo.R;
        if (rho > 0.0f && d != 0.0f) {
            const float sg = d > 0.0f ? 1.0f : -1.0f;
            gx = sg * dx / rho;
            gy = sg * dyy / rho;
        }
        return fabsf(d);
    }
    if (iseg < 0) return INFINITY;
    const float4 sgm = geo.seg[iseg];
    const float rx = X - sgm.x, ry = Y - sgm.y;
    float t = (rx * sgm.z + ry * sgm.w) * geo.seg_inv[iseg];
    t = fminf(fmaxf(t, 0.0f), 1.0f);
    const float ex = rx - t * sgm.z, ey = ry - t * sgm.w;
    const float dl = sqrtf(ex * ex + ey * ey);
    if (dl > 0.0f) {
        gx = ex / dl;
        gy = ey / dl;
    }
    return dl;
}

// Smoothed stage cost of Eqs. (11)-(16) at (x_{k+1}, Sigma_{k+1}, s2_k), given
// the argmin polyline segment iseg and obstacle iobs (-1 where there is none).
__host__ __device__ inline float smoothed_stage(const Geometry &geo, const CostWeights &cw, float inv_tau, float disc_k,
                                                const float x1[5], const float p1[15], const float s2[2], int iseg,
                                                int iobs) {
    const float sa = p1[0], sb = p1[1], sc = p1[5];
    float da, db, dc;
    const float lmax = lmax_grad(sa, sb, sc, da, db, dc);
    float gx, gy;
    const float dl = lane_dist_grad(geo, x1[0], x1[1], iseg, gx, gy);
    const float rbar = geo.half_width - geo.c_p * sqrtf(fmaxf(lmax, 0.0f));
    const float dv = cw.v_des - x1[3];
    float c = cw.w_var * (s2[0] + s2[1]) + cw.w_dev * (dl * geo.inv_half_width) + cw.w_speed * (dv * dv);
    c += cw.w_lane * disc_k * sigm((dl - rbar) * inv_tau);
    if (iobs >= 0) {
        const float4 ob = geo.obs[iobs];
        const float dx = x1[0] - ob.x, dyy = x1[1] - ob.y;
        const float rho2 = dx * dx + dyy * dyy;
        const float rho = sqrtf(rho2);
        const float var = rho > 0.0f ? (sa * dx * dx + 2.0f * sb * dx * dyy + sc * dyy * dyy) / rho2 : lmax;
        const float om = (rho - ob.z) - geo.z_p * sqrtf(fmaxf(var, 0.0f));
        c += cw.w_obs * sigm(-om * inv_tau);
    }
    return c;
}

// Adjoints produced by one reversed step besides the state's.
struct StepAdj {
    float s2b[2];   // of the GP variances s2_k
    float mb[2];    // of the GP means m_k
    float ub[2];    // of the sampled, clipped controls u_k (their GP-input share excluded)
};

// One reversed step of one sample, GP excluded.  On entry xb, pb hold the
// adjoint of (x_{k+1}, Sigma_{k+1}) carried from the later steps; the stage
// cost's adjoint at (x_{k+1}, Sigma_{k+1}, s2_k) (weight cbar, discount disc_k,
// argmin segment iseg and obstacle iobs) is added, then the covariance
// update, the Euler step and the Jacobian are reversed: on return xb, pb hold
// the adjoint of (x_k, Sigma_k) without the GP inputs' share.
__host__ __device__ inline void step_adjoint(const Geometry &geo, const CostWeights &cw, const Dyn &dy, float inv_tau,
                                             float cbar, float disc_k, const float xk[5], const float pk[15],
                                             const float x1[5], const float p1[15], int iseg, int iobs, float xb[5],
                                             float pb[15], StepAdj &out) {
    const float dt = dy.dt;
    const float X1 = x1[0], Y1 = x1[1], v1 = x1[3];
    const float sa = p1[0], sb = p1[1], sc = p1[5];
    float da, db, dc;
    const float lmax = lmax_grad(sa, sb, sc, da, db, dc);
    float gx, gy;
    const float dl = lane_dist_grad(geo, X1, Y1, iseg, gx, gy);
    const float sq = sqrtf(fmaxf(lmax, 0.0f));
    const float rbar = geo.half_width - geo.c_p * sq;
    out.s2b[0] = cbar * cw.w_var;
    out.s2b[1] = cbar * cw.w_var;
    float lamb = 0.0f;   // adjoint of lambda_max(Sigma_XY)
    float dlb = cbar * cw.w_dev * geo.inv_half_width;
    {
        const float sL = sigm((dl - rbar) * inv_tau);
        const float gL = cbar * cw.w_lane * disc_k * sL * (1.0f - sL) * inv_tau;
        dlb += gL;
        if (sq > 0.0f) lamb += gL * geo.c_p * 0.5f / sq;   // r_bar = r - c_p sqrt(lambda)
    }
    float Xb1 = gx * dlb, Yb1 = gy * dlb;
    float Sab = 0.0f, Sbb = 0.0f, Scb = 0.0f;
    if (iobs >= 0) {
        const float4 ob = geo.obs[iobs];
        const float dx = X1 - ob.x, dyy = Y1 - ob.y;
        const float rho2 = dx * dx + dyy * dyy;
        const float rho = sqrtf(rho2);
        const float var = rho > 0.0f ? (sa * dx * dx + 2.0f * sb * dx * dyy + sc * dyy * dyy) / rho2 : lmax;
        const float sv = sqrtf(fmaxf(var, 0.0f));
        const float om = (rho - ob.z) - geo.z_p * sv;
        const float sO = sigm(-om * inv_tau);
        const float omb = -cbar * cw.w_obs * sO * (1.0f - sO) * inv_tau;
        const float varb = sv > 0.0f ? omb * (-geo.z_p) * 0.5f / sv : 0.0f;
        if (rho > 0.0f) {
            Xb1 += omb * dx / rho + varb * 2.0f * (sa * dx + sb * dyy - var * dx) / rho2;
            Yb1 += omb * dyy / rho + varb * 2.0f * (sb * dx + sc * dyy - var * dyy) / rho2;
            Sab += varb * dx * dx / rho2;
            Sbb += varb * 2.0f * dx * dyy / rho2;
            Scb += varb * dyy * dyy / rho2;
        } else {
            lamb += varb;
        }
    }
    Sab += lamb * da;
    Sbb += lamb * db;
    Scb += lamb * dc;
    const float Xn_b = xb[0] + Xb1, Yn_b = xb[1] + Yb1, thn_b = xb[2];
    const float vn_b = xb[3] + cbar * cw.w_speed * (-2.0f) * (cw.v_des - v1), wn_b = xb[4];
    pb[0] += Sab;
    pb[1] += Sbb;
    pb[5] += Scb;

    // covariance update at x_k
    const float vk = xk[3];
    float sth, cth;
    sincosf(xk[2], &sth, &cth);
    const Jac Jk{-dt * vk * sth, dt * cth, dt * vk * cth, dt * sth};
    Jac Jb{0.0f, 0.0f, 0.0f, 0.0f};
    float e3b, e4b, pbk[15];
    cov_backward(pk, Jk, dt, dy.a33, dy.a44, pb, pbk, Jb, e3b, e4b);
    out.s2b[0] += dt * dt * e3b;
    out.s2b[1] += dt * dt * e4b;

    // Euler step, and the Jacobian's dependence on (theta, v)
    xb[0] = Xn_b;
    xb[1] = Yn_b;
    xb[2] = -Xn_b * dt * vk * sth + Yn_b * dt * vk * cth + thn_b + Jb.a02 * (-dt * vk * cth) + Jb.a03 * (-dt * sth) +
            Jb.a12 * (-dt * vk * sth) + Jb.a13 * (dt * cth);
    xb[3] = Xn_b * dt * cth + Yn_b * dt * sth + vn_b * (1.0f - dy.dt_tau_v) + Jb.a02 * (-dt * sth) +
            Jb.a12 * (dt * cth);
    xb[4] = thn_b * dt + wn_b * (1.0f - dy.dt_tau_w);
    out.ub[0] = vn_b * dy.dt_tau_v;
    out.ub[1] = wn_b * dy.dt_tau_w;
    out.mb[0] = vn_b * dt;
    out.mb[1] = wn_b * dt;
    for (int i = 0; i < 15; ++i) pb[i] = pbk[i];
}

}  // namespace gpmppi
