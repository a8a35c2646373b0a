// Adjoint rollout on gfx950: gradient of the smoothed expected cost
//   J(U, log ell, log sf) = (1/K) sum_s S~^s
// where S~ is the rollout cost of Alg. 1 Step 1 (Eqs. 1-3, 10-16, one
// combined stage cost) with the lane-exit and collision indicators replaced by
// sigmoid((d_lane - r_bar)/tau) and sigmoid(-min_j d_bar_j / tau).  The noise
// is fixed by the seed; u = clip(U + eps) has derivative 1 strictly inside the
// box.  The derivative in the GP hyperparameters is total (through k, alpha and
// A^-1, A = K(Z, Z) + sn^2 I).
//
// grad_kernel: one workgroup of 256 threads per 32 samples (one 32-column
// matrix-core group; 8 loop parts = 4 waves x 2 half-waves), or, split, two
// workgroups per 32 samples, workgroup 2 blk + r doing the GP work of output r
// (kernel vectors, variance walk, r = Q k and its sums) and both doing the
// per-sample algebra; they exchange, per forward step, their output's GP mean
// and variance and, per reversed step, their output's share of the GP inputs'
// adjoint.  The exchanged values enter the same arithmetic in the same order
// as in the unsplit kernel, so the results are the same bit for bit.  A
// workgroup whose bounded exchange wait gives up marks its block for the
// repair launch of the unsplit kernel that follows every split launch.
//   job 0   forward over all T steps: costs, the state (x, Sigma) every C
//           steps (checkpoints), and the last segment's per-step record;
//   job j   for segment n - j (last first): recompute the segment's C steps
//           from its checkpoint (not for j = 1, recorded by job 0), keeping
//           per-step state, controls, GP means and variances in a scratch
//           array, then step backwards through it.
// Both passes run the same forward code, so the recomputed trajectory is the
// first pass's bit for bit.  Per backward step, per sample, in registers: the
// adjoints of the stage cost, of Sigma+ = A Sigma A^T + dt^2 diag(s2) (the
// 15 stored entries as independent scalars), of the Euler step and of the
// Jacobian A(theta, v).  Per output o, for the whole block: the kernel vector
// k (VALU) and r = Q k with Q = A^-1 = W^T W (dense 32x32 FP32 tiles on the
// matrix cores); with beta_j = k_j (-mbar alpha_j + 2 s2bar r_j):
//   dq_d        = 2 ln2 s_d sum_j beta_j (qs_d - zs_jd)
//   d log ell_d = -2 ln2 sum_j beta_j (qs_d - zs_jd)^2       (through k)
// and the length-scales' dependence through A: sum_ij (P_ij - b_i alpha_j)
// dA_ij/dlog ell_d with b = sum mbar r and P = sum s2bar r r^T over all
// sample-steps.  b is summed in registers; P is formed by grad_syrk_kernel from
// the stored r (FP32 [T K][Mpad] per output) and contracted on the fly.
// The signal variance scales k and K(Z, Z) alike (dA/dlog sf = 2 (A - sn^2 I)),
// so with A r = k and A alpha = y its total derivative folds into per-sample
// terms in which the large parts through k and through A^-1 cancel exactly:
//   d log sf    = 2 s2bar (s2 - sn^2 - sn^2 |r|^2) + 2 sn^2 mbar r^T alpha
// (s2 - sn^2 = sf^2 - k^T r, the latent variance of the forward pass).
#include "adjoint_step.hpp"
#include "gp_tiles.hpp"

namespace gpmppi {

namespace {

constexpr int kB = 32;           // samples per workgroup
constexpr int kParts = 8;        // loop splitters
constexpr int kSegF = 28;        // per step: x 5, p 15, u 2, m 2, s2 2, latent-positive flags 2
constexpr int kCkF = 20;         // per checkpoint: x 5, p 15
constexpr float kLn2 = 0.69314718055994531f;

}  // namespace


namespace {

// Dynamic LDS: [k operand 32 x Mpad FP32][staged inputs][r: 32 x (Mpad + 1) FP32]
__host__ __device__ constexpr size_t grad_rbuf_off(int Mpad) {
    return kgroup_bytes<GPMPPI_FP32>(Mpad) + (size_t)staged_slots<GPMPPI_FP32>(Mpad) * 16;
}
__host__ __device__ constexpr size_t grad_lds_bytes(int Mpad) {
    return grad_rbuf_off(Mpad) + (size_t)kB * (Mpad + 1) * 4;
}

__device__ __forceinline__ void restage(const GpDev &g, int o, unsigned char *lds) {
    __syncthreads();
    StagedInputs st;
    stage_load<GPMPPI_FP32>(st, g, o);
    stage_store<GPMPPI_FP32>(st, g, lds, kgroup_bytes<GPMPPI_FP32>(g.Mpad));
    __syncthreads();
}

// FP32 kernel vector of output o for this thread's sample into the k operand.
__device__ __forceinline__ void gen_kvec(const GpDev &g, int o, const float qs[4], int part, int sl,
                                         unsigned char *lds) {
    const int Mpad = g.Mpad, nchunk = Mpad >> 3;
    const float4 *zs = reinterpret_cast<const float4 *>(lds + kgroup_bytes<GPMPPI_FP32>(Mpad));
    const float c2 = g.c2[o];
    for (int c = part; c < nchunk; c += kParts) {
        float kv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float4 z = zs[8 * c + e];
            const float d0 = qs[0] - z.x, d1 = qs[1] - z.y, d2 = qs[2] - z.z, d3 = qs[3] - z.w;
            float acc = c2;
            acc = fmaf(-d0, d0, acc);
            acc = fmaf(-d1, d1, acc);
            acc = fmaf(-d2, d2, acc);
            acc = fmaf(-d3, d3, acc);
            kv[e] = __builtin_amdgcn_exp2f(acc);
        }
        float4 *Kp = reinterpret_cast<float4 *>(lds) + (size_t)c * 64;
        Kp[sl] = make_float4(kv[0], kv[2], kv[4], kv[6]);
        Kp[32 + sl] = make_float4(kv[1], kv[3], kv[5], kv[7]);
    }
}

// r = Q k for the block's 32 samples: wave w computes row tiles t = w, w+4, ...
// over all column tiles, writing r[s][j] (row stride Mpad + 1) to LDS.  Q blocks
// rotate through four register slots with static indices: block it + 3 is loaded
// into the slot of block it - 1 before the products of block it (loads past the
// row's end repeat its last block), three blocks of products ahead of its use.
__device__ __forceinline__ void qk_walk(const GradArgs &a, int o, unsigned char *lds) {
    const int Mpad = a.gp.Mpad, NT = Mpad >> 5;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const float4 *Qo = a.q32 + (size_t)o * a.q_stride;
    float *rb = reinterpret_cast<float *>(lds + grad_rbuf_off(Mpad));
    for (int t = w; t < NT; t += kWaves) {
        const float4 *Qt = Qo + (size_t)(t * NT) * 256 + lane;
        v16f acc = v16f{};
        WBlock<GPMPPI_FP32> b[4];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const float4 *p = Qt + (size_t)(r < NT ? r : NT - 1) * 256;
            b[r].v[0] = p[0];
            b[r].v[1] = p[64];
            b[r].v[2] = p[128];
            b[r].v[3] = p[192];
        }
        for (int it0 = 0; it0 < NT; it0 += 4) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int it = it0 + r;
                if (it < NT) {
                    {   // block it + 3 into the slot freed by block it - 1
                        const int nx = it + 3 < NT ? it + 3 : NT - 1;
                        const float4 *p = Qt + (size_t)nx * 256;
                        WBlock<GPMPPI_FP32> &d = b[(r + 3) % 4];
                        d.v[0] = p[0];
                        d.v[1] = p[64];
                        d.v[2] = p[128];
                        d.v[3] = p[192];
                    }
                    KOp<GPMPPI_FP32> kop;
                    load_kop<GPMPPI_FP32>(kop, lds, it, lane, Mpad);
                    mma_block<GPMPPI_FP32>(acc, b[r], kop);
                }
            }
        }
        const int s = lane & 31;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int row = 32 * t + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
            rb[s * (Mpad + 1) + row] = acc[e];
        }
    }
}

// Argmin over this part's polyline segments and obstacles, reduced over the
// parts through LDS (smallest value, then smallest index).
__device__ __forceinline__ void constraint_scan(const Geometry &geo, float X, float Y, float sa, float sb, float sc,
                                                float lmax, int part, int sl, float *vb, int *ib, float *vo, int *io,
                                                float &best_all, int &iseg, float &om_all, int &iobs) {
    float best = INFINITY, om = INFINITY;
    int bi = -1, oi = -1;
    // wave-uniform indices (both half-waves take the same segments and obstacles and
    // store the same results): the geometry comes through the scalar cache
    const int wu = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (geo.path_kind != 0) {
        const const_v4p segs = (const_v4p)geo.seg;
        const const_fp sinv = (const_fp)geo.seg_inv;
#pragma unroll 4
        for (int i = wu; i < geo.P; i += kWaves) {
            const v4f sgm = segs[i];
            const float rx = X - sgm.x, ry = Y - sgm.y;
            float t = (rx * sgm.z + ry * sgm.w) * sinv[i];
            t = fminf(fmaxf(t, 0.0f), 1.0f);
            const float ex = rx - t * sgm.z, ey = ry - t * sgm.w;
            const float d2 = ex * ex + ey * ey;
            if (d2 < best) {
                best = d2;
                bi = i;
            }
        }
    }
    const const_v4p obs = (const_v4p)geo.obs;
#pragma unroll 2
    for (int j = wu; j < geo.n_obs; j += kWaves) {
        const v4f ob = obs[j];
        const float dx = X - ob.x, dyy = Y - ob.y;
        const float rho2 = dx * dx + dyy * dyy;
        const float rho = sqrtf(rho2);
        const float vn = rho > 0.0f ? (sa * dx * dx + 2.0f * sb * dx * dyy + sc * dyy * dyy) / rho2 : lmax;
        const float m = (rho - ob.z) - geo.z_p * sqrtf(fmaxf(vn, 0.0f));
        if (m < om) {
            om = m;
            oi = j;
        }
    }
    __syncthreads();
    vb[part * kB + sl] = best;
    ib[part * kB + sl] = bi;
    vo[part * kB + sl] = om;
    io[part * kB + sl] = oi;
    __syncthreads();
    best_all = INFINITY;
    om_all = INFINITY;
    iseg = -1;
    iobs = -1;
#pragma unroll
    for (int p = 0; p < kParts; ++p) {
        const float b = vb[p * kB + sl], m = vo[p * kB + sl];
        const int bx = ib[p * kB + sl], mx = io[p * kB + sl];
        if (b < best_all || (b == best_all && bx >= 0 && (iseg < 0 || bx < iseg))) {
            best_all = b;
            iseg = bx;
        }
        if (m < om_all || (m == om_all && mx >= 0 && (iobs < 0 || mx < iobs))) {
            om_all = m;
            iobs = mx;
        }
    }
}

__device__ __forceinline__ void seg_put(float *base, int f, float v) { base[f * kB] = v; }

// a + b, never fused with the product that formed b: the split kernel adds the
// partner's share after receiving it as a value, and the unsplit kernel must round alike.
__device__ __forceinline__ float add_rounded(float a, float b) {
#pragma clang fp contract(off)
    return a + b;
}

}  // namespace

// SPLIT: role = blockIdx.x & 1 of block blockIdx.x >> 1 (see above).  REPAIR
// (unsplit): the repair launch, only the blocks a split launch marked.
template <bool SPLIT, bool REPAIR = false>
__global__ __launch_bounds__(kThreads) void grad_kernel(GradArgs a) {
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ float pred[kParts * kB];
    __shared__ float vred[kWaves * kB];
    __shared__ float vb[kParts * kB], vo[kParts * kB];
    __shared__ int ib[kParts * kB], io[kParts * kB];
    __shared__ __align__(16) float gred[11 * kParts * kB];
    __shared__ float mb_s[2][kB], sb_s[2][kB], ub_s[2][kB];
    __shared__ float xv[5 * kB + 1];   // split: values received from the partner, and a give-up flag

    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int sl = lane & 31;
    const int part = 2 * w + (lane >> 5);
    const int blk = SPLIT ? (int)(blockIdx.x >> 1) : (int)blockIdx.x;
    const int role = SPLIT ? (int)(blockIdx.x & 1) : 0;   // split: the GP output this workgroup computes
    if (REPAIR && __hip_atomic_load(a.repair + blk, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) return;
    const int sg = blk * kB + sl;
    const bool valid = sg < a.K;
    const bool writer = w == 0 && lane < kB;   // one copy of each sample
    const int K = a.K, T = a.T, C = a.C;
    const int Mpad = a.gp.Mpad;
    const GpDev &g = a.gp;
    const Geometry &geo = a.geo;
    const CostWeights cw = a.cw;
    const Dyn dy = a.dyn;
    const float dt = dy.dt;
    const float cbar = valid ? a.inv_K : 0.0f;
    // per-(block, role) segment scratch [e][f][32] and per-role checkpoints
    float *segw = a.seg + ((size_t)blk * 2 + role) * (C + 1) * kSegF * kB + sl;
    float *ckpt = a.ckpt + (size_t)role * a.nck * kCkF * K;
    float *rb = reinterpret_cast<float *>(lds + grad_rbuf_off(Mpad));

    NoiseParams np = a.noise;

    // split exchange: event e (the same sequence in both roles) uses slot e % 4 of the
    // writer's records [block][writer role][slot][kind][32]; records are zeroed before
    // the launch, and the tag e + 1 names the event
    unsigned long long *xrec = SPLIT ? a.xrec + (size_t)blk * kGradXchPerBlock : nullptr;
    auto xslot = [&](int wr, uint32_t e, int kind) {
        return xrec + ((size_t)(wr * 4 + (int)(e & 3u)) * 4 + kind) * kB;
    };
    uint32_t ev = 0;
    bool broken = false, alone = false;

    // per-sample accumulators of the hyperparameter terms through k (o, theta)
    double hyp[2][5] = {};
    // this thread's share of b = sum mbar r (points j = tid + 256 i)
    double bacc[2][2] = {};

    const int nseg = (T + C - 1) / C;
    float X = 0, Y = 0, th = 0, v = 0, w_ = 0;
    float p[15];
    // adjoint of the state after the step being reversed, carried between segments
    float xb[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    float pb[15] = {};
    float S_ = 0.0f, Sc = 0.0f, disc = 1.0f;

    // the last segment's per-step record is written by the forward pass itself, so
    // its backward job (job 1) needs no recompute
    const int kl0 = (nseg - 1) * C;
    for (int job = 0; job <= nseg; ++job) {
        const bool first = job == 0;
        const int segi = first ? 0 : nseg - job;
        const int k0 = first ? 0 : segi * C;
        const int k1 = first ? T : min(T, k0 + C);
        const int kf = job == 1 ? k0 : k1;   // end of the forward (re)computation: job 1's is recorded
        if (first) {
            X = a.x0[0]; Y = a.x0[1]; th = a.x0[2]; v = a.x0[3]; w_ = a.x0[4];
#pragma unroll
            for (int i = 0; i < 15; ++i) p[i] = 0.0f;
        } else {
            const float *ck = ckpt + (size_t)segi * kCkF * K + (valid ? sg : 0);
            X = ck[0 * (size_t)K]; Y = ck[1 * (size_t)K]; th = ck[2 * (size_t)K]; v = ck[3 * (size_t)K];
            w_ = ck[4 * (size_t)K];
#pragma unroll
            for (int i = 0; i < 15; ++i) p[i] = ck[(5 + i) * (size_t)K];
        }
        restage(g, SPLIT ? role : ((k0 & 1) ? 1 : 0), lds);
        // ---------------------------------------------------------- forward
        for (int k = k0; k < kf; ++k) {
            if (writer) {
                if (first && k % C == 0 && valid) {
                    float *ck = ckpt + (size_t)(k / C) * kCkF * K + sg;
                    ck[0 * (size_t)K] = X; ck[1 * (size_t)K] = Y; ck[2 * (size_t)K] = th; ck[3 * (size_t)K] = v;
                    ck[4 * (size_t)K] = w_;
#pragma unroll
                    for (int i = 0; i < 15; ++i) ck[(5 + i) * (size_t)K] = p[i];
                }
                if (!first || k >= kl0) {
                    float *e = segw + (size_t)(k - (first ? kl0 : k0)) * kSegF * kB;
                    seg_put(e, 0, X); seg_put(e, 1, Y); seg_put(e, 2, th); seg_put(e, 3, v); seg_put(e, 4, w_);
#pragma unroll
                    for (int i = 0; i < 15; ++i) seg_put(e, 5 + i, p[i]);
                }
            }
            const bool rev = (k & 1) != 0;
            const float2 u = sampled_control(np, k, sg, a.U[2 * k], a.U[2 * k + 1]);
            const float q[4] = {v, w_, u.x, u.y};
            float m[2], s2[2];
            if constexpr (SPLIT) {   // this role's output, then the partner's mean and variance
                const int o = role;
                __syncthreads();
                const float qs[4] = {q[0] * g.scale[o][0], q[1] * g.scale[o][1], q[2] * g.scale[o][2],
                                     q[3] * g.scale[o][3]};
                gp_output<GPMPPI_FP32, 1>(g, o, -1, qs, part, sl, rev, 0, blk, lds, pred, vred, m[o], s2[o]);
                const uint32_t tag = ev + 1;
                if (w == 0) {
                    xch_put(xslot(role, ev, 0), lane, m[o], tag);
                    xch_put(xslot(role, ev, 1), lane, s2[o], tag);
                    const float mp = xch_get(xslot(1 - role, ev, 0), lane, tag, a.xspin, broken);
                    const float sp = xch_get(xslot(1 - role, ev, 1), lane, tag, a.xspin, broken);
                    if (lane < kB) {
                        xv[lane] = mp;
                        xv[kB + lane] = sp;
                    }
                    if (lane == 0) xv[5 * kB] = broken ? 1.0f : 0.0f;
                }
                ++ev;
                __syncthreads();
                if (xv[5 * kB] != 0.0f) {
                    alone = true;
                    break;
                }
                m[1 - o] = xv[sl];
                s2[1 - o] = xv[kB + sl];
            } else {
#pragma unroll
                for (int oo = 0; oo < 2; ++oo) {
                    const int o = rev ? 1 - oo : oo;
                    __syncthreads();
                    const float qs[4] = {q[0] * g.scale[o][0], q[1] * g.scale[o][1], q[2] * g.scale[o][2],
                                         q[3] * g.scale[o][3]};
                    gp_output<GPMPPI_FP32, 1>(g, o, oo == 0 ? 1 - o : -1, qs, part, sl, rev, 0, blk, lds, pred,
                                              vred, m[o], s2[o]);
                }
            }
            float sth, cth;
            sincosf(th, &sth, &cth);
            const Jac J{-dt * v * sth, dt * cth, dt * v * cth, dt * sth};
            const float Xn = X + dt * v * cth;
            const float Yn = Y + dt * v * sth;
            const float thn = th + dt * w_;
            const float vn = v + (dy.dt_tau_v * (u.x - v) + dt * m[0]);
            const float wn = w_ + (dy.dt_tau_w * (u.y - w_) + dt * m[1]);
            float P[15];
            cov_forward(p, J, dt, dy.a33, dy.a44, dt * dt * s2[0], dt * dt * s2[1], P);
#pragma unroll
            for (int i = 0; i < 15; ++i) p[i] = P[i];
            X = Xn; Y = Yn; th = thn; v = vn; w_ = wn;
            if ((!first || k >= kl0) && writer) {
                float *e = segw + (size_t)(k - (first ? kl0 : k0)) * kSegF * kB;
                seg_put(e, 20, u.x); seg_put(e, 21, u.y); seg_put(e, 22, m[0]); seg_put(e, 23, m[1]);
                seg_put(e, 24, s2[0]); seg_put(e, 25, s2[1]);
                seg_put(e, 26, s2[0] > g.sn2[0] ? 1.0f : 0.0f);
                seg_put(e, 27, s2[1] > g.sn2[1] ? 1.0f : 0.0f);
            }
            if (first) {
                // smoothed stage cost on (x_{k+1}, Sigma_{k+1})
                float da, db, dc;
                const float lmax = lmax_grad(p[0], p[1], p[5], da, db, dc);
                float best_all, om_all;
                int iseg, iobs;
                constraint_scan(geo, X, Y, p[0], p[1], p[5], lmax, part, sl, vb, ib, vo, io, best_all, iseg, om_all,
                                iobs);
                const float x1[5] = {X, Y, th, v, w_};
                const float c = smoothed_stage(geo, cw, a.inv_tau, disc, x1, p, s2, iseg, iobs);
                const float yk = c - Sc;
                const float tk = S_ + yk;
                Sc = (tk - S_) - yk;
                S_ = tk;
                disc *= cw.discount;
            }
        }
        if (alone) break;
        if (first) {
            if (writer && valid && role == 0) a.costs[sg] = S_;
            if (writer) {   // the last segment's final state
                float *e = segw + (size_t)(T - kl0) * kSegF * kB;
                seg_put(e, 0, X); seg_put(e, 1, Y); seg_put(e, 2, th); seg_put(e, 3, v); seg_put(e, 4, w_);
#pragma unroll
                for (int i = 0; i < 15; ++i) seg_put(e, 5 + i, p[i]);
            }
            continue;
        }
        if (job != 1 && writer) {   // the segment's final state
            float *e = segw + (size_t)(k1 - k0) * kSegF * kB;
            seg_put(e, 0, X); seg_put(e, 1, Y); seg_put(e, 2, th); seg_put(e, 3, v); seg_put(e, 4, w_);
#pragma unroll
            for (int i = 0; i < 15; ++i) seg_put(e, 5 + i, p[i]);
        }
        __syncthreads();   // segment scratch visible to every copy of each sample

        // ---------------------------------------------------------- backward
        for (int k = k1 - 1; k >= k0; --k) {
            const float *e1 = segw + (size_t)(k + 1 - k0) * kSegF * kB;   // x_{k+1}, p_{k+1}
            const float *e0 = segw + (size_t)(k - k0) * kSegF * kB;       // x_k, p_k, u, m, s2, flags
            const float vk = e0[3 * kB], wk = e0[4 * kB];
            float pk[15];
#pragma unroll
            for (int i = 0; i < 15; ++i) pk[i] = e0[(5 + i) * kB];
            const float ux = e0[20 * kB], uy = e0[21 * kB];
            const float flag[2] = {e0[26 * kB], e0[27 * kB]};
            const float s2k[2] = {e0[24 * kB], e0[25 * kB]};

            float x1[5], p1[15], xk[5];
#pragma unroll
            for (int i = 0; i < 5; ++i) {
                x1[i] = e1[i * kB];
                xk[i] = e0[i * kB];
            }
#pragma unroll
            for (int i = 0; i < 15; ++i) p1[i] = e1[(5 + i) * kB];
            float da, db, dc;
            const float lmax = lmax_grad(p1[0], p1[1], p1[5], da, db, dc);
            float best_all, om_all;
            int iseg, iobs;
            constraint_scan(geo, x1[0], x1[1], p1[0], p1[1], p1[5], lmax, part, sl, vb, ib, vo, io, best_all, iseg,
                            om_all, iobs);
            float discount_k = 1.0f;
            for (int i = 0; i < k; ++i) discount_k *= cw.discount;
            StepAdj sa_out;
            step_adjoint(geo, cw, dy, a.inv_tau, cbar, discount_k, xk, pk, x1, p1, iseg, iobs, xb, pb, sa_out);
            float vbk = xb[3], wbk = xb[4];
            float uxb = sa_out.ub[0], uyb = sa_out.ub[1];
            const float mb[2] = {sa_out.mb[0], sa_out.mb[1]};
            const float s2b[2] = {sa_out.s2b[0], sa_out.s2b[1]};

            // ---- GP adjoint, both outputs
            const float qk[4] = {vk, wk, ux, uy};
            float qb[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            float qown[4];   // split: this role's output's share of the GP inputs' adjoint
            for (int o = 0; o < 2; ++o) {
                if (SPLIT && o != role) continue;
                const float sbo = s2b[o] * flag[o];
                if (writer) {
                    mb_s[o][sl] = mb[o];
                    sb_s[o][sl] = sbo;
                }
                restage(g, o, lds);   // also publishes mb_s / sb_s
                const float qs[4] = {qk[0] * g.scale[o][0], qk[1] * g.scale[o][1], qk[2] * g.scale[o][2],
                                     qk[3] * g.scale[o][3]};
                gen_kvec(g, o, qs, part, sl, lds);
                __syncthreads();
                qk_walk(a, o, lds);
                __syncthreads();
                // per-sample sums over this part's points
                const float4 *zs = reinterpret_cast<const float4 *>(lds + kgroup_bytes<GPMPPI_FP32>(Mpad));
                const float *al = reinterpret_cast<const float *>(zs + Mpad);
                float Sd[4] = {0, 0, 0, 0}, Sdd[4] = {0, 0, 0, 0}, Srr = 0.0f, Sra = 0.0f;
                for (int c = part; c < (Mpad >> 3); c += kParts) {
                    const float4 *Kp = reinterpret_cast<const float4 *>(lds) + (size_t)c * 64;
                    const float4 lo = Kp[sl], hi = Kp[32 + sl];
                    const float kv[8] = {lo.x, hi.x, lo.y, hi.y, lo.z, hi.z, lo.w, hi.w};
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int j = 8 * c + e;
                        const float4 z = zs[j];
                        const float rj = rb[sl * (Mpad + 1) + j];
                        const float beta = kv[e] * (2.0f * sbo * rj - mb[o] * al[j]);
                        const float d0 = qs[0] - z.x, d1 = qs[1] - z.y, d2 = qs[2] - z.z, d3 = qs[3] - z.w;
                        Srr = fmaf(rj, rj, Srr);
                        Sra = fmaf(rj, al[j], Sra);
                        Sd[0] = fmaf(beta, d0, Sd[0]);
                        Sd[1] = fmaf(beta, d1, Sd[1]);
                        Sd[2] = fmaf(beta, d2, Sd[2]);
                        Sd[3] = fmaf(beta, d3, Sd[3]);
                        Sdd[0] = fmaf(beta * d0, d0, Sdd[0]);
                        Sdd[1] = fmaf(beta * d1, d1, Sdd[1]);
                        Sdd[2] = fmaf(beta * d2, d2, Sdd[2]);
                        Sdd[3] = fmaf(beta * d3, d3, Sdd[3]);
                    }
                }
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    gred[((1 + d) * kParts + part) * kB + sl] = Sd[d];
                    gred[((5 + d) * kParts + part) * kB + sl] = Sdd[d];
                }
                gred[(9 * kParts + part) * kB + sl] = Srr;
                gred[(10 * kParts + part) * kB + sl] = Sra;
                // b += sum_s mbar_s r_s over this thread's points; the r rows for P
                for (int jj = 0; jj < 2; ++jj) {
                    const int j = tid + kThreads * jj;
                    if (j < Mpad) {
                        double acc = bacc[o][jj];
                        float *Rrow = a.R + ((size_t)o * T * K + (size_t)k * K + (size_t)blk * kB) * Mpad + j;
                        for (int s = 0; s < kB; ++s) {
                            if (blk * kB + s < K) {
                                const float rv = rb[s * (Mpad + 1) + j];
                                acc += (double)(mb_s[o][s] * rv);
                                Rrow[(size_t)s * Mpad] = rv;
                            }
                        }
                        bacc[o][jj] = acc;
                    }
                }
                if (writer && valid) a.Gw[(size_t)o * T * K + (size_t)k * K + sg] = sbo;
                __syncthreads();
                float tot[11];
#pragma unroll
                for (int i = 1; i < 11; ++i) {
                    float sum = 0.0f;
#pragma unroll
                    for (int pp = 0; pp < kParts; ++pp) sum += gred[(i * kParts + pp) * kB + sl];
                    tot[i] = sum;
                }
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    const float qd = 2.0f * kLn2 * g.scale[o][d] * tot[1 + d];
                    if constexpr (SPLIT) qown[d] = qd;
                    else qb[d] = add_rounded(qb[d], qd);
                    hyp[o][d] += (double)(-2.0f * kLn2 * tot[5 + d]);
                }
                {   // log sf: the folded per-sample terms (k and A^-1 parts cancelled)
                    const double sn2 = (double)g.sn2[o];
                    hyp[o][4] += 2.0 * (double)sbo * (((double)s2k[o] - sn2) - sn2 * (double)tot[9]) +
                                 2.0 * sn2 * (double)mb[o] * (double)tot[10];
                }
            }
            if constexpr (SPLIT) {   // the partner's share, received in exchange for ours
                const uint32_t tag = ev + 1;
                if (w == 0) {
#pragma unroll
                    for (int d = 0; d < 4; ++d) xch_put(xslot(role, ev, d), lane, qown[d], tag);
#pragma unroll
                    for (int d = 0; d < 4; ++d) {
                        const float vq = xch_get(xslot(1 - role, ev, d), lane, tag, a.xspin, broken);
                        if (lane < kB) xv[d * kB + lane] = vq;
                    }
                    if (lane == 0) xv[5 * kB] = broken ? 1.0f : 0.0f;
                }
                ++ev;
                __syncthreads();
                if (xv[5 * kB] != 0.0f) {
                    alone = true;
                    break;
                }
                // in output order, as the unsplit kernel accumulates them
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    const float qp = xv[d * kB + sl];
                    qb[d] = add_rounded(qb[d], role == 0 ? qown[d] : qp);
                    qb[d] = add_rounded(qb[d], role == 0 ? qp : qown[d]);
                }
            }
            vbk += qb[0];
            wbk += qb[1];
            uxb += qb[2];
            uyb += qb[3];

            // ---- the nominal control's adjoint through the clip (1 strictly inside the box)
            {
                const float2 raw = sampled_raw(np, k, sg, a.U[2 * k], a.U[2 * k + 1]);
                const float m0 = (raw.x > np.umin0 && raw.x < np.umax0) ? 1.0f : 0.0f;
                const float m1 = (raw.y > np.umin1 && raw.y < np.umax1) ? 1.0f : 0.0f;
                if (writer) {
                    ub_s[0][sl] = valid ? uxb * m0 : 0.0f;
                    ub_s[1][sl] = valid ? uyb * m1 : 0.0f;
                }
                __syncthreads();
                if (tid < 2 && role == 0) {
                    float sum = 0.0f;
                    for (int i = 0; i < kB; ++i) sum += ub_s[tid][i];
                    a.upart[((size_t)blk * T + k) * 2 + tid] = sum;
                }
            }
            xb[3] = vbk;
            xb[4] = wbk;
        }
        if (alone) break;
    }
    (void)np;
    if (SPLIT && alone) {   // uniform: leave the block to the repair launch
        if (tid == 0) {
            __hip_atomic_store(a.repair + blk, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (a.flags)
                __hip_atomic_fetch_or(a.flags, GPMPPI_FLAG_EXCHANGE_TIMEOUT, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
        }
        return;
    }
    // ---- per-workgroup partial sums (split: this role's output only)
    __syncthreads();
    double *hred = reinterpret_cast<double *>(gred);   // 10 x 32 doubles
    if (writer) {
#pragma unroll
        for (int o = 0; o < 2; ++o)
#pragma unroll
            for (int i = 0; i < 5; ++i) hred[(o * 5 + i) * kB + sl] = valid ? hyp[o][i] : 0.0;
    }
    __syncthreads();
    if (tid < 10 && (!SPLIT || tid / 5 == role)) {
        double s = 0.0;
        for (int i = 0; i < kB; ++i) s += hred[tid * kB + i];
        a.hpart[(size_t)blk * 10 + tid] = s;
    }
    for (int o = 0; o < 2; ++o) {
        if (SPLIT && o != role) continue;
        for (int jj = 0; jj < 2; ++jj) {
            const int j = tid + kThreads * jj;
            if (j < Mpad) a.bpart[((size_t)blk * 2 + o) * Mpad + j] = bacc[o][jj];
        }
    }
    if (REPAIR && tid == 0)   // the block is done
        __hip_atomic_store(a.repair + blk, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Zeroes the split gradient's exchange records and repair marks before a launch.
__global__ __launch_bounds__(kThreads) void grad_clear_kernel(unsigned long long *rec, size_t n_rec, uint32_t *repair,
                                                              int n_blk) {
    const size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n_rec) rec[i] = 0ull;
    if (i < (size_t)n_blk) repair[i] = 0u;
}


// dA_ij / dlog ell_d contracted with a weight c_ij: K_ij = exp2(c2 - |zs_i - zs_j|^2),
// dA/dlog ell_d = K 2 ln2 (zs_id - zs_jd)^2 (the sn^2 I part does not depend on it).
__device__ __forceinline__ void dA_contract(float cval, const float4 &zi, const float4 &zj, float c2, double acc[4]) {
    const float d0 = zi.x - zj.x, d1 = zi.y - zj.y, d2 = zi.z - zj.z, d3 = zi.w - zj.w;
    const float e0 = d0 * d0, e1 = d1 * d1, e2 = d2 * d2, e3 = d3 * d3;
    const float Kij = __builtin_amdgcn_exp2f(c2 - (e0 + e1 + e2 + e3));
    const float ck = cval * Kij;
    const float c2l = 2.0f * kLn2 * ck;
    acc[0] += (double)(c2l * e0);
    acc[1] += (double)(c2l * e1);
    acc[2] += (double)(c2l * e2);
    acc[3] += (double)(c2l * e3);
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
    return x;
}

// P = sum_n g_n r_n r_n^T over rows n in [n0, n1) of one output, for one
// 128 x 128 block (bi <= bj) of the Mpad x Mpad result, contracted with dA/dlog ell:
// ppart[((o * npairs + pair) * nsplit + split) * 4 + d].  Wave w owns the
// 32 x 32 tiles (2 (w >> 1) + {0, 1}, 2 (w & 1) + {0, 1}) of the block.
__global__ __launch_bounds__(kThreads) void grad_syrk_kernel(const float *R, const float *Gw, long long TK, int Mpad,
                                                             const float *zs, float c20, float c21, int nsplit,
                                                             double *ppart) {
    __shared__ double red[kWaves][4];
    const int pair = blockIdx.x, split = blockIdx.y, o = blockIdx.z;
    const int npairs = gridDim.x;
    const int nb = (Mpad + 127) / 128;
    int bi = 0, rem = pair;
    while (rem >= nb - bi) {
        rem -= nb - bi;
        ++bi;
    }
    const int bj = bi + rem;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ti0 = 4 * bi + 2 * (w >> 1), tj0 = 4 * bj + 2 * (w & 1);
    const int NT = Mpad >> 5;
    const bool vi[2] = {ti0 < NT, ti0 + 1 < NT}, vj[2] = {tj0 < NT, tj0 + 1 < NT};
    const long long chunk = (TK + nsplit - 1) / nsplit;
    const long long n0 = (long long)split * chunk;
    const long long n1 = n0 + chunk < TK ? n0 + chunk : TK;
    const float *Ro = R + (size_t)o * TK * Mpad;
    const float *Go = Gw + (size_t)o * TK;
    v16f acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = v16f{};
    const int col = lane & 31, rsel = lane >> 5;
    // rows in chunks of kD row pairs: every load of a chunk is issued before its first
    // product, so the loads' latency is paid once per chunk
    constexpr int kD = 8;
    for (long long n = n0; n < n1; n += 2 * kD) {
        float gq[kD], ra[kD][2], rbq[kD][2];
        bool okq[kD];
#pragma unroll
        for (int q = 0; q < kD; ++q) {
            const long long row = n + 2 * q + rsel;
            okq[q] = row < n1;
            const float *rp = Ro + (size_t)(okq[q] ? row : n0) * Mpad;
            gq[q] = Go[okq[q] ? row : n0];
#pragma unroll
            for (int i = 0; i < 2; ++i) ra[q][i] = vi[i] ? rp[32 * (ti0 + i) + col] : 0.0f;
#pragma unroll
            for (int j = 0; j < 2; ++j) rbq[q][j] = vj[j] ? rp[32 * (tj0 + j) + col] : 0.0f;
        }
#pragma unroll
        for (int q = 0; q < kD; ++q) {
            const float gv = gq[q];
            float av[2], bv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) av[i] = okq[q] ? gv * ra[q][i] : 0.0f;
#pragma unroll
            for (int j = 0; j < 2; ++j) bv[j] = okq[q] ? rbq[q][j] : 0.0f;
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i], bv[j], acc[i][j], 0, 0, 0);
        }
    }
    // epilogue: sum_ij P_ij dA_ij/dtheta over the wave's tiles (both triangles of a
    // diagonal block; off-diagonal blocks stand for their mirror image too)
    const float c2 = o ? c21 : c20;
    const float4 *z = reinterpret_cast<const float4 *>(zs) + (size_t)o * Mpad;
    const float weight = bi == bj ? 1.0f : 2.0f;
    double cacc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            if (!vi[i] || !vj[j]) continue;
            const float4 zj = z[32 * (tj0 + j) + col];
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int row = 32 * (ti0 + i) + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
                dA_contract(weight * acc[i][j][e], z[row], zj, c2, cacc);
            }
        }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const double v = wave_sum(cacc[t]);
        if (lane == 0) red[w][t] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const double v = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
        ppart[((size_t)(o * npairs + pair) * nsplit + split) * 4 + threadIdx.x] = v;
    }
}

// b = sum over workgroups of the partial b, then sum_ij b_i alpha_j dA_ij/dlog ell_d:
// one thread per row i; bterm[(o * gridDim.x + block) * 4 + d].
__global__ __launch_bounds__(kThreads) void grad_bterm_kernel(const double *bpart, int nwg, int Mpad, const float *zs,
                                                              const float *alpha, float c20, float c21,
                                                              double *bterm) {
    __shared__ double red[kWaves][4];
    const int o = blockIdx.y;
    const int i = blockIdx.x * kThreads + threadIdx.x;
    const float c2 = o ? c21 : c20;
    const float4 *z = reinterpret_cast<const float4 *>(zs) + (size_t)o * Mpad;
    const float *al = alpha + (size_t)o * Mpad;
    double cacc[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < Mpad) {
        double b = 0.0;
        for (int wg = 0; wg < nwg; ++wg) b += bpart[((size_t)wg * 2 + o) * Mpad + i];
        const float4 zi = z[i];
        const float bf = (float)b;
        for (int j = 0; j < Mpad; ++j) dA_contract(bf * al[j], zi, z[j], c2, cacc);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const double v = wave_sum(cacc[t]);
        if (lane == 0) red[w][t] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const double v = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
        bterm[((size_t)o * gridDim.x + blockIdx.x) * 4 + threadIdx.x] = v;
    }
}

// Fixed-order final sums: J = mean smoothed cost, dU[k][c], and the
// hyperparameter gradient: log ell_d = direct (through k) + (P - b alpha^T) : dA/dlog ell_d;
// log sf = its folded per-sample terms.
__global__ __launch_bounds__(kThreads) void grad_final_kernel(const float *costs, int K, int T, int nwg,
                                                              const float *upart, const double *hpart,
                                                              const double *ppart, int nppart, const double *bterm,
                                                              int nbterm, float *J, float *dU, float *dlog_ell,
                                                              float *dlog_sf) {
    __shared__ float red[kThreads];
    const int tid = threadIdx.x;
    float s = 0.0f;
    for (int i = tid; i < K; i += kThreads) s += costs[i];
    red[tid] = s;
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
        if (tid < h) red[tid] += red[tid + h];
        __syncthreads();
    }
    if (tid == 0) J[0] = red[0] / (float)K;
    for (int kc = tid; kc < 2 * T; kc += kThreads) {
        double v = 0.0;
        for (int wg = 0; wg < nwg; ++wg) v += upart[(size_t)wg * 2 * T + kc];
        dU[kc] = (float)v;
    }
    if (tid < 10) {
        const int o = tid / 5, t = tid % 5;
        double direct = 0.0, mat = 0.0, bt = 0.0;
        for (int wg = 0; wg < nwg; ++wg) direct += hpart[(size_t)wg * 10 + tid];
        if (t < 4) {
            for (int i = 0; i < nppart; ++i) mat += ppart[((size_t)o * nppart + i) * 4 + t];
            for (int i = 0; i < nbterm; ++i) bt += bterm[((size_t)o * nbterm + i) * 4 + t];
        }
        const float g = (float)(direct + mat - bt);
        if (t < 4) dlog_ell[o * 4 + t] = g;
        else dlog_sf[o] = g;
    }
}

size_t grad_lds(int Mpad) { return grad_lds_bytes(Mpad); }

int grad_split_capacity(int Mpad) {
    const size_t lds = grad_lds_bytes(Mpad);
    int dev = 0, ncu = 0, per_cu = 0;
    if (hipFuncSetAttribute(reinterpret_cast<const void *>(grad_kernel<true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(grad_kernel<true>),
                                                     kThreads, lds) != hipSuccess)
        return 0;
    return per_cu * ncu;
}

hipError_t launch_grad(const GradArgs &args, const GradLaunch &l, hipStream_t st) {
    const size_t lds = grad_lds_bytes(args.gp.Mpad);
    GradArgs a = args;
    hipError_t e;
    if (a.split) {
        if (!a.xrec || !a.repair || 2 * l.nwg > grad_split_capacity(a.gp.Mpad)) return hipErrorInvalidValue;
        const size_t n_rec = (size_t)l.nwg * kGradXchPerBlock;
        const size_t n = n_rec > (size_t)l.nwg ? n_rec : (size_t)l.nwg;
        hipLaunchKernelGGL(grad_clear_kernel, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, st,
                           a.xrec, n_rec, a.repair, l.nwg);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = hipFuncSetAttribute(reinterpret_cast<const void *>(grad_kernel<true>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) != hipSuccess)
            return e;
        hipLaunchKernelGGL(grad_kernel<true>, dim3(2 * l.nwg), dim3(kThreads), lds, st, a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        // the repair launch: the unsplit kernel for the blocks whose exchange gave up
        if ((e = hipFuncSetAttribute(reinterpret_cast<const void *>(grad_kernel<false, true>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) != hipSuccess)
            return e;
        hipLaunchKernelGGL((grad_kernel<false, true>), dim3(l.nwg), dim3(kThreads), lds, st, a);
    } else {
        if ((e = hipFuncSetAttribute(reinterpret_cast<const void *>(grad_kernel<false>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) != hipSuccess)
            return e;
        hipLaunchKernelGGL(grad_kernel<false>, dim3(l.nwg), dim3(kThreads), lds, st, a);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const long long TK = (long long)a.T * a.K;
    hipLaunchKernelGGL(grad_syrk_kernel, dim3(l.npairs, l.nsplit, 2), dim3(kThreads), 0, st, a.R, a.Gw, TK, a.gp.Mpad,
                       a.gp.zs, a.gp.c2[0], a.gp.c2[1], l.nsplit, l.ppart);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(grad_bterm_kernel, dim3(l.nbterm, 2), dim3(kThreads), 0, st, a.bpart, l.nwg, a.gp.Mpad,
                       a.gp.zs, a.gp.alpha, a.gp.c2[0], a.gp.c2[1], l.bterm);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(grad_final_kernel, dim3(1), dim3(kThreads), 0, st, a.costs, a.K, a.T, l.nwg, a.upart, a.hpart,
                       l.ppart, l.npairs * l.nsplit, l.bterm, l.nbterm, l.J, l.dU, l.dlog_ell, l.dlog_sf);
    return hipGetLastError();
}

}  // namespace gpmppi
