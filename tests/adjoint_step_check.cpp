// Host build of the adjoint rollout's per-sample algebra (the library's
// adjoint_step.hpp) with a C interface, for the CPU tests that compare it with
// reverse-mode autodiff of one float64 step.
#include "adjoint_step.hpp"

using namespace gpmppi;

namespace {
Geometry make_geo(int path_kind, const float *circle, int P, const float *seg, const float *seg_inv, int n_obs,
                  const float *obs, float half_width, float z_p, float c_p) {
    Geometry g{};
    g.path_kind = path_kind;
    g.cx = circle[0];
    g.cy = circle[1];
    g.R = circle[2];
    g.P = P;
    g.seg = reinterpret_cast<const float4 *>(seg);
    g.seg_inv = seg_inv;
    g.half_width = half_width;
    g.inv_half_width = 1.0f / half_width;
    g.n_obs = n_obs;
    g.obs = reinterpret_cast<const float4 *>(obs);
    g.z_p = z_p;
    g.c_p = c_p;
    return g;
}
CostWeights make_cw(const float *c) {
    CostWeights w{};
    w.w_var = c[0];
    w.w_dev = c[1];
    w.w_lane = c[2];
    w.w_speed = c[3];
    w.w_obs = c[4];
    w.v_des = c[5];
    w.discount = c[6];
    return w;
}
Dyn make_dyn(const float *d) { return Dyn{d[0], d[1], d[2], d[3], d[4]}; }
}  // namespace

extern "C" {

void adj_cov_forward(const float *p, const float *jac, float a24, float a33, float a44, float e3, float e4, float *P) {
    cov_forward(p, Jac{jac[0], jac[1], jac[2], jac[3]}, a24, a33, a44, e3, e4, P);
}

float adj_stage(int path_kind, const float *circle, int P, const float *seg, const float *seg_inv, int n_obs,
                const float *obs, float half_width, float z_p, float c_p, const float *cw, float inv_tau, float disc_k,
                const float *x1, const float *p1, const float *s2, int iseg, int iobs) {
    const Geometry g = make_geo(path_kind, circle, P, seg, seg_inv, n_obs, obs, half_width, z_p, c_p);
    return smoothed_stage(g, make_cw(cw), inv_tau, disc_k, x1, p1, s2, iseg, iobs);
}

void adj_step(int path_kind, const float *circle, int P, const float *seg, const float *seg_inv, int n_obs,
              const float *obs, float half_width, float z_p, float c_p, const float *cw, const float *dyn,
              float inv_tau, float cbar, float disc_k, const float *xk, const float *pk, const float *x1,
              const float *p1, int iseg, int iobs, float *xb, float *pb, float *out6) {
    const Geometry g = make_geo(path_kind, circle, P, seg, seg_inv, n_obs, obs, half_width, z_p, c_p);
    StepAdj o;
    step_adjoint(g, make_cw(cw), make_dyn(dyn), inv_tau, cbar, disc_k, xk, pk, x1, p1, iseg, iobs, xb, pb, o);
    out6[0] = o.s2b[0];
    out6[1] = o.s2b[1];
    out6[2] = o.mb[0];
    out6[3] = o.mb[1];
    out6[4] = o.ub[0];
    out6[5] = o.ub[1];
}

}  // extern "C"
