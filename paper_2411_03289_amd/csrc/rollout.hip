// K-sample x T-step rollout of the GP-augmented chance-constrained MPPI
// controller on gfx950 (Alg. 1 Step 1 with Eqs. 1-3, 10, 11-16).
//
// Work decomposition: one workgroup of NW wave64s (NW = 4 or 8) owns
// B = 32 G samples (G = 1 or 2 column groups of the 32x32 matrix-core tiles).
// Every wave keeps the state x (5) and covariance Sigma (15 symmetric entries)
// of all B samples in registers for the whole horizon, lane l holding sample
// l % B; the waves split the training points and the blocks of W between them.
//
// Per step:
//  0. noise and sampled control; position, heading and A Sigma A^T, none of
//     which needs the GP at this step (the GP variance reaches the position
//     block of Sigma one step later).
//  Per GP output o (gp_tiles.hpp):
//  1. kernel vector k_oj = sf^2 exp(-|q - z_j|^2_ell / 2) for every sample and
//     training point; k goes to LDS in the matrix-core operand layout and the
//     GP mean k^T alpha is summed in FP32.
//  2. variance: v = W k with W = L^-1 lower triangular, on the matrix cores:
//     each wave walks its share of the 32x32 blocks of W, streamed from L2
//     through a register ring; each W block serves G sample groups.
//     s2 = sn^2 + max(0, sf^2 - |v|^2).  Odd steps take the outputs and the
//     blocks in reverse order, so the blocks walked last stay in L2 for the
//     next step.  While the later waves finish their blocks, the first waves
//     run the polyline (first output) and obstacle (second output) loops at
//     x_{k+1}, Sigma_{k+1}.
//  3. velocities with the GP mean, the GP variance into Sigma, lane/obstacle
//     tightening and the stage cost.
#include "gp_tiles.hpp"

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

// The rollout of sample block blk (samples blk * B .. blk * B + B - 1) of one
// problem; called by all threads of a workgroup.
template <int PREC, int G, int NW = kWaves, int WALK = kWalkAny>
__device__ __forceinline__ void rollout_block(const RolloutArgs &a, int blk, unsigned char *lds, float *pred,
                                              float *ored, float *vred) {
    using S = Shapes<PREC, G, NW>;
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int sl = lane % S::B;                     // sample within the block
    const int part = (G == 2) ? w : 2 * w + (lane >> 5);
    const int sg = blk * S::B + sl;
    const bool valid = sg < a.K;
    const bool writer = valid && w == 0 && lane < S::B;
    const int K = a.K;
    const int Mpad = a.gp.Mpad;
    const size_t zs_off = G * kgroup_bytes<PREC>(Mpad);

    NoiseParams np = a.noise;
    {
        uint64_t seed = a.seed;
        if (a.step_counter) seed += (uint64_t)(*a.step_counter);
        np.key0 = (uint32_t)seed;
        np.key1 = (uint32_t)(seed >> 32);
    }
    const Dyn dy = a.dyn;
    const CostWeights cw = a.cw;
    const Geometry &geo = a.geo;

    float X = a.x0[0], Y = a.x0[1], th = a.x0[2], v = a.x0[3], w_ = a.x0[4];
    float p00 = 0, p01 = 0, p02 = 0, p03 = 0, p04 = 0, p11 = 0, p12 = 0, p13 = 0, p14 = 0, p22 = 0,
          p23 = 0, p24 = 0, p33 = 0, p34 = 0, p44 = 0;
    float S_ = 0.0f, Sc = 0.0f, disc = 1.0f;
    float dgoal_min = INFINITY;

    if (writer && a.trace.x_d) {
        a.trace.x_d[0 * K + sg] = X;
        a.trace.x_d[1 * K + sg] = Y;
        a.trace.x_d[2 * K + sg] = th;
        a.trace.x_d[3 * K + sg] = v;
        a.trace.x_d[4 * K + sg] = w_;
    }
    if (writer && a.trace.sxy_d) {
        a.trace.sxy_d[0 * K + sg] = 0.0f;
        a.trace.sxy_d[1 * K + sg] = 0.0f;
        a.trace.sxy_d[2 * K + sg] = 0.0f;
    }

    if constexpr (mfma_gen<PREC>()) {   // alpha of both outputs, for the whole horizon
        stage_alpha<NW>(a.gp, lds, zs_off);
    } else if constexpr (!scalar_inputs<G>()) {   // inputs of output 0 (the first output of step 0)
        StagedInputs st;
        stage_load<PREC, NW>(st, a.gp, 0);
        stage_store<PREC, NW>(st, a.gp, lds, zs_off);
    }
    for (int k = 0; k < a.T; ++k) {
        // even steps: outputs 0 then 1; odd steps: 1 then 0 (and blocks reversed)
        const bool rev = (k & 1) != 0;
        const float2 u = sampled_control(np, k, sg, a.U[2 * k], a.U[2 * k + 1]);
        const float q[4] = {v, w_, u.x, u.y};

        // ---- the parts of the step that do not need the GP at step k: position and heading
        // (Eqs. 1, 10) and the covariance propagation A Sigma A^T (Eq. 10); the GP variance
        // enters Sigma_vv and Sigma_ww below, and reaches the position block one step later
        float sth, cth;
        sincosf(th, &sth, &cth);
        const float dt = dy.dt;
        const float a02 = -dt * v * sth, a03 = dt * cth, a12 = dt * v * cth, a13 = dt * sth, a24 = dt;
        const float a33 = dy.a33, a44 = dy.a44;
        const float v_old = v, w_old = w_;
        X = X + dt * v * cth;
        Y = Y + dt * v * sth;
        th = th + dt * w_;
        {   // B = A Sigma (rows), then Sigma+_ij = sum_n B_in A_jn for i <= j
            const float b00 = p00 + a02 * p02 + a03 * p03, b01 = p01 + a02 * p12 + a03 * p13,
                        b02 = p02 + a02 * p22 + a03 * p23, b03 = p03 + a02 * p23 + a03 * p33,
                        b04 = p04 + a02 * p24 + a03 * p34;
            const float b11 = p11 + a12 * p12 + a13 * p13, b12 = p12 + a12 * p22 + a13 * p23,
                        b13 = p13 + a12 * p23 + a13 * p33, b14 = p14 + a12 * p24 + a13 * p34;
            const float b22 = p22 + a24 * p24, b23 = p23 + a24 * p34, b24 = p24 + a24 * p44;
            const float b33 = a33 * p33, b34 = a33 * p34;
            const float b44 = a44 * p44;
            p00 = b00 + a02 * b02 + a03 * b03;
            p01 = b01 + a12 * b02 + a13 * b03;
            p02 = b02 + a24 * b04;
            p03 = a33 * b03;
            p04 = a44 * b04;
            p11 = b11 + a12 * b12 + a13 * b13;
            p12 = b12 + a24 * b14;
            p13 = a33 * b13;
            p14 = a44 * b14;
            p22 = b22 + a24 * b24;
            p23 = a33 * b23;
            p24 = a44 * b24;
            p33 = a33 * b33;
            p34 = a44 * b34;
            p44 = a44 * b44;
        }

        // ---- chance-constraint geometry at (x_{k+1}, Sigma_{k+1}) (Eqs. 13-16); with Step 2
        // tightening the covariance is the nominal sequence's, shared by all samples
        float sa = p00, sb = p01, sc = p11;
        if (a.tight_sxy) {
            sa = a.tight_sxy[3 * (k + 1)];
            sb = a.tight_sxy[3 * (k + 1) + 1];
            sc = a.tight_sxy[3 * (k + 1) + 2];
        }
        const float hh = 0.5f * (sa - sc);
        const float lmax = 0.5f * (sa + sc) + sqrtf(hh * hh + sb * sb);
        // Loops over polyline segments (during the first output's contraction) and obstacles
        // (during the second's), run by the first S::lwaves waves, which finish their share of
        // W first: wave w's squared distance to segments w, w + lwaves, ... and least tightened
        // distance to obstacles w, w + lwaves, ..., to ored[w] and ored[lwaves + w] (with one
        // sample group both half-waves hold the same samples and write the same values).
        const float Xs = X, Ys = Y;
        auto loops = [&](int oo, int wv) {
            if (wv >= S::lwaves) return;   // wave-uniform: segments and obstacles through the scalar cache
            if (oo == 0) {
                if (geo.path_kind == 0) return;
                float best = INFINITY;
                const const_v4p segs = (const_v4p)geo.seg;
                const const_fp sinv = (const_fp)geo.seg_inv;
#pragma unroll 4
                for (int i = wv; i < geo.P; i += S::lwaves) {
                    const v4f sgm = segs[i];
                    const float rx = Xs - sgm.x, ry = Ys - sgm.y;
                    float t = (rx * sgm.z + ry * sgm.w) * sinv[i];
                    t = fminf(fmaxf(t, 0.0f), 1.0f);
                    const float ex = rx - t * sgm.z, ey = ry - t * sgm.w;
                    best = fminf(best, ex * ex + ey * ey);
                }
                ored[wv * S::B + sl] = best;
            } else {
                float om = INFINITY;
                const const_v4p obs = (const_v4p)geo.obs;
#pragma unroll 2
                for (int j = wv; j < geo.n_obs; j += S::lwaves) {
                    const v4f ob = obs[j];
                    om = fminf(om, obstacle_margin(Xs - ob.x, Ys - ob.y, ob.z, sa, sb, sc, lmax, geo.z_p));
                }
                ored[(S::lwaves + wv) * S::B + sl] = om;
            }
        };

        float m[2], s2[2];
#pragma unroll
        for (int oo = 0; oo < 2; ++oo) {
            const int o = rev ? 1 - oo : oo;
            __syncthreads();   // staged inputs visible; previous k-operand readers are done
            const float qs[4] = {q[0] * a.gp.scale[o][0], q[1] * a.gp.scale[o][1], q[2] * a.gp.scale[o][2],
                                 q[3] * a.gp.scale[o][3]};
            m[o] = gp_gen<PREC, G, NW>(a.gp, o, qs, part, sl, lds, pred);
            s2[o] = gp_walk<PREC, G, NW, WALK>(a.gp, o, oo == 0 ? 1 - o : -1, rev, a.rotate, blk, lds, vred, sl,
                                               [&](int wv) { loops(oo, wv); });
        }

        // ---- velocities: explicit Euler of the dynamic unicycle plus the GP residual (Eqs. 1, 2,
        // 10)
        v = v_old + (dy.dt_tau_v * (u.x - v_old) + dt * m[0]);
        w_ = w_old + (dy.dt_tau_w * (u.y - w_old) + dt * m[1]);

        // ---- the GP variance into the covariance (Eq. 10)
        p33 += dt * dt * s2[0];
        p44 += dt * dt * s2[1];

        // the loop parts' partial results were written before the contraction's last barrier
        float best_all = INFINITY, om = INFINITY;
#pragma unroll
        for (int p = 0; p < S::lwaves; ++p) {
            if (geo.path_kind != 0) best_all = fminf(best_all, ored[p * S::B + sl]);
            om = fminf(om, ored[(S::lwaves + p) * S::B + sl]);
        }
        float dl;
        if (geo.path_kind == 0) {
            const float dx = X - geo.cx, dyy = Y - geo.cy;
            dl = fabsf(sqrtf(dx * dx + dyy * dyy) - geo.R);
        } else {
            dl = sqrtf(best_all);
        }
        const float rbar = geo.half_width - geo.c_p * sqrtf(fmaxf(lmax, 0.0f));

        // ---- stage cost (Eqs. 11-12 terms), Kahan-compensated sum (Eq. 5)
        const float dv = cw.v_des - v;
        float c = cw.w_var * (s2[0] + s2[1]) + cw.w_dev * (dl * geo.inv_half_width) + cw.w_speed * (dv * dv);
        if (dl > rbar) c += cw.w_lane * disc;
        if (om <= 0.0f) c += cw.w_obs;
        if (cw.w_goal != 0.0f || cw.w_term != 0.0f) {   // goal terms (Eq. 12)
            const float gx = X - cw.goal_x, gy = Y - cw.goal_y;
            const float dg = sqrtf(gx * gx + gy * gy);
            dgoal_min = fminf(dgoal_min, dg);
            c += cw.w_goal * dg;
        }
        {
            const float yk = c - Sc;
            const float tk = S_ + yk;
            Sc = (tk - S_) - yk;
            S_ = tk;
        }
        disc *= cw.discount;

        if (writer) {
            const gpmppi_trace &tr = a.trace;
            const size_t kk = (size_t)k;
            if (tr.x_d) {
                float *xd = tr.x_d + (kk + 1) * 5 * K;
                xd[0 * K + sg] = X;
                xd[1 * K + sg] = Y;
                xd[2 * K + sg] = th;
                xd[3 * K + sg] = v;
                xd[4 * K + sg] = w_;
            }
            if (tr.sxy_d) {
                float *sd = tr.sxy_d + (kk + 1) * 3 * K;
                sd[0 * K + sg] = p00;
                sd[1 * K + sg] = p01;
                sd[2 * K + sg] = p11;
            }
            if (tr.gp_mean_d) {
                tr.gp_mean_d[(kk * 2 + 0) * K + sg] = m[0];
                tr.gp_mean_d[(kk * 2 + 1) * K + sg] = m[1];
            }
            if (tr.gp_var_d) {
                tr.gp_var_d[(kk * 2 + 0) * K + sg] = s2[0];
                tr.gp_var_d[(kk * 2 + 1) * K + sg] = s2[1];
            }
            if (tr.d_lane_d) tr.d_lane_d[kk * K + sg] = dl;
            if (tr.lane_margin_d) tr.lane_margin_d[kk * K + sg] = rbar - dl;
            if (tr.obs_margin_d) tr.obs_margin_d[kk * K + sg] = om;
            if (tr.u_d) {
                tr.u_d[(kk * 2 + 0) * K + sg] = u.x;
                tr.u_d[(kk * 2 + 1) * K + sg] = u.y;
            }
        }
    }
    if (cw.w_term != 0.0f && !(dgoal_min <= cw.goal_tol)) {
        const float yk = cw.w_term - Sc;
        S_ = S_ + yk;
    }
    if (writer) a.costs[sg] = S_;
}

template <int PREC, int G, int NW, int WALK>
__global__ __launch_bounds__(64 * NW) void rollout_kernel(RolloutArgs a) {
    using S = Shapes<PREC, G, NW>;
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ float pred[S::rparts * S::B];
    __shared__ float ored[2 * S::lwaves * S::B];
    __shared__ float vred[NW * S::B];
    rollout_block<PREC, G, NW, WALK>(a, blockIdx.x, lds, pred, ored, vred);
}

// Persistent rollout of many independent problems: every workgroup takes
// (problem, sample block) items from a shared counter until the list (sorted
// longest first) is exhausted.  Results do not depend on which workgroup
// runs an item.  *counter must be 0 at launch.
template <int PREC, int G, int NW>
__global__ __launch_bounds__(64 * NW) void rollout_batch_kernel(const RolloutArgs *probs, const int2 *items,
                                                                 int n_items, uint32_t *counter) {
    using S = Shapes<PREC, G, NW>;
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ float pred[S::rparts * S::B];
    __shared__ float ored[2 * S::lwaves * S::B];
    __shared__ float vred[NW * S::B];
    __shared__ int next_item;
    for (;;) {
        __syncthreads();   // every thread has read the previous item
        if (threadIdx.x == 0) next_item = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(next_item);
        if (it >= n_items) break;
        const int2 pb = items[it];
        const int p = __builtin_amdgcn_readfirstlane(pb.x);
        const int b = __builtin_amdgcn_readfirstlane(pb.y);
        rollout_block<PREC, G, NW>(probs[p], b, lds, pred, ored, vred);
    }
}

template <int PREC, int G>
__global__ __launch_bounds__(kThreads) void gp_predict_kernel(GpDev g, const float *q, int n, float *mean,
                                                              float *var) {
    using S = Shapes<PREC, G>;
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ float pred[S::rparts * S::B];
    __shared__ float vred[kWaves * S::B];
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int sl = lane % S::B;
    const int part = (G == 2) ? w : 2 * w + (lane >> 5);
    const int sg = blockIdx.x * S::B + sl;
    const int sc = sg < n ? sg : n - 1;
    const float4 qq = reinterpret_cast<const float4 *>(q)[sc];
    const float qv[4] = {qq.x, qq.y, qq.z, qq.w};
    const size_t zs_off = G * kgroup_bytes<PREC>(g.Mpad);
    if constexpr (mfma_gen<PREC>()) {
        stage_alpha<kWaves>(g, lds, zs_off);
    } else if constexpr (!scalar_inputs<G>()) {
        StagedInputs st;
        stage_load<PREC>(st, g, 0);
        stage_store<PREC>(st, g, lds, zs_off);
    }
#pragma unroll
    for (int o = 0; o < 2; ++o) {
        __syncthreads();
        const float qs[4] = {qv[0] * g.scale[o][0], qv[1] * g.scale[o][1], qv[2] * g.scale[o][2],
                             qv[3] * g.scale[o][3]};
        float m, s2;
        gp_output<PREC, G>(g, o, o == 0 ? 1 : -1, qs, part, sl, false, 0, blockIdx.x, lds, pred, vred, m, s2);
        if (sg < n && w == 0 && lane < S::B) {
            mean[(size_t)o * n + sg] = m;
            var[(size_t)o * n + sg] = s2;
        }
    }
}

// Sample groups per block: two when both groups' k operand and the staged
// inputs fit the 160 KB LDS of a CDNA4 compute unit, else one.
static int groups_for(int precision, int Mpad) {
    const size_t budget = 160 * 1024 - 8 * 1024;
    size_t need2 = 0;
    switch (precision) {
        case GPMPPI_FP32: need2 = dyn_lds_bytes<GPMPPI_FP32, 2>(Mpad); break;
        case GPMPPI_BF16: need2 = dyn_lds_bytes<GPMPPI_BF16, 2>(Mpad); break;
        default: need2 = dyn_lds_bytes<GPMPPI_BF16X3, 2>(Mpad); break;
    }
    return need2 <= budget ? 2 : 1;
}

size_t rollout_lds_bytes(int precision, int G, int Mpad) {
    switch (precision) {
        case GPMPPI_FP32: return G == 2 ? dyn_lds_bytes<GPMPPI_FP32, 2>(Mpad) : dyn_lds_bytes<GPMPPI_FP32, 1>(Mpad);
        case GPMPPI_BF16: return G == 2 ? dyn_lds_bytes<GPMPPI_BF16, 2>(Mpad) : dyn_lds_bytes<GPMPPI_BF16, 1>(Mpad);
        default: return G == 2 ? dyn_lds_bytes<GPMPPI_BF16X3, 2>(Mpad) : dyn_lds_bytes<GPMPPI_BF16X3, 1>(Mpad);
    }
}

template <typename F>
static hipError_t set_lds(F *fn, size_t bytes) {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// One problem: the kernel carries only the walk over W that its size takes.
template <int PREC, int G, int NW, int WALK>
static hipError_t launch_rollout_w(const RolloutArgs &a, hipStream_t st) {
    const size_t lds = dyn_lds_bytes<PREC, G>(a.gp.Mpad);
    hipError_t e = set_lds(rollout_kernel<PREC, G, NW, WALK>, lds);
    if (e != hipSuccess) return e;
    const dim3 grid((a.K + 32 * G - 1) / (32 * G));
    hipLaunchKernelGGL((rollout_kernel<PREC, G, NW, WALK>), grid, dim3(64 * NW), lds, st, a);
    return hipGetLastError();
}

template <int PREC, int G, int NW>
static hipError_t launch_rollout_t(const RolloutArgs &a, hipStream_t st) {
    return walk_by_rows(a.gp.NT, NW) ? launch_rollout_w<PREC, G, NW, kWalkRows>(a, st)
                                     : launch_rollout_w<PREC, G, NW, kWalkPairs>(a, st);
}

template <int PREC>
static hipError_t launch_rollout_p(const RolloutArgs &a, int G, int NW, hipStream_t st) {
    if (NW == 8) return G == 2 ? launch_rollout_t<PREC, 2, 8>(a, st) : launch_rollout_t<PREC, 1, 8>(a, st);
    return G == 2 ? launch_rollout_t<PREC, 2, kWaves>(a, st) : launch_rollout_t<PREC, 1, kWaves>(a, st);
}

template <int PREC, int G, int NW>
static hipError_t launch_rollout_batch_t(const RolloutArgs *probs, const int2 *items, int n_items, uint32_t *counter,
                                         int Mpad_max, int grid, hipStream_t st) {
    const size_t lds = dyn_lds_bytes<PREC, G>(Mpad_max);
    hipError_t e = set_lds(rollout_batch_kernel<PREC, G, NW>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((rollout_batch_kernel<PREC, G, NW>), dim3(grid), dim3(64 * NW), lds, st, probs, items, n_items,
                       counter);
    return hipGetLastError();
}

template <int PREC>
static hipError_t launch_rollout_batch_p(const RolloutArgs *probs, const int2 *items, int n_items, uint32_t *counter,
                                         int G, int NW, int Mpad_max, int grid, hipStream_t st) {
    if (NW == 8)
        return G == 2 ? launch_rollout_batch_t<PREC, 2, 8>(probs, items, n_items, counter, Mpad_max, grid, st)
                      : launch_rollout_batch_t<PREC, 1, 8>(probs, items, n_items, counter, Mpad_max, grid, st);
    return G == 2 ? launch_rollout_batch_t<PREC, 2, kWaves>(probs, items, n_items, counter, Mpad_max, grid, st)
                  : launch_rollout_batch_t<PREC, 1, kWaves>(probs, items, n_items, counter, Mpad_max, grid, st);
}

int rollout_groups(int precision, int Mpad) { return groups_for(precision, Mpad); }

hipError_t launch_rollout_batch(const RolloutArgs *probs_d, const int2 *items_d, int n_items, uint32_t *counter,
                                int precision, int G, int NW, int Mpad_max, int grid, hipStream_t st) {
    if (G < 1 || G > groups_for(precision, Mpad_max) || grid < 1 || (NW != kWaves && NW != 8))
        return hipErrorInvalidValue;
    switch (precision) {
        case GPMPPI_FP32:
            return launch_rollout_batch_p<GPMPPI_FP32>(probs_d, items_d, n_items, counter, G, NW, Mpad_max, grid, st);
        case GPMPPI_BF16:
            return launch_rollout_batch_p<GPMPPI_BF16>(probs_d, items_d, n_items, counter, G, NW, Mpad_max, grid, st);
        default:
            return launch_rollout_batch_p<GPMPPI_BF16X3>(probs_d, items_d, n_items, counter, G, NW, Mpad_max, grid,
                                                         st);
    }
}

hipError_t launch_rollout(const RolloutArgs &a, int precision, int G, int NW, hipStream_t st) {
    if (G < 1 || G > groups_for(precision, a.gp.Mpad) || (NW != kWaves && NW != 8)) return hipErrorInvalidValue;
    switch (precision) {
        case GPMPPI_FP32: return launch_rollout_p<GPMPPI_FP32>(a, G, NW, st);
        case GPMPPI_BF16: return launch_rollout_p<GPMPPI_BF16>(a, G, NW, st);
        default: return launch_rollout_p<GPMPPI_BF16X3>(a, G, NW, st);
    }
}

template <int PREC, int G>
static hipError_t launch_predict_t(const GpDev &g, const float *q, int n, float *mean, float *var,
                                   hipStream_t st) {
    const size_t lds = dyn_lds_bytes<PREC, G>(g.Mpad);
    hipError_t e = set_lds(gp_predict_kernel<PREC, G>, lds);
    if (e != hipSuccess) return e;
    const dim3 grid((n + 32 * G - 1) / (32 * G));
    hipLaunchKernelGGL((gp_predict_kernel<PREC, G>), grid, dim3(kThreads), lds, st, g, q, n, mean, var);
    return hipGetLastError();
}

hipError_t launch_gp_predict(const GpDev &g, int precision, const float *q, int n, float *mean, float *var,
                             hipStream_t st) {
    const int G = groups_for(precision, g.Mpad);
    switch (precision) {
        case GPMPPI_FP32: return G == 2 ? launch_predict_t<GPMPPI_FP32, 2>(g, q, n, mean, var, st)
                                        : launch_predict_t<GPMPPI_FP32, 1>(g, q, n, mean, var, st);
        case GPMPPI_BF16: return G == 2 ? launch_predict_t<GPMPPI_BF16, 2>(g, q, n, mean, var, st)
                                        : launch_predict_t<GPMPPI_BF16, 1>(g, q, n, mean, var, st);
        default: return G == 2 ? launch_predict_t<GPMPPI_BF16X3, 2>(g, q, n, mean, var, st)
                               : launch_predict_t<GPMPPI_BF16X3, 1>(g, q, n, mean, var, st);
    }
}

}  // namespace gpmppi
