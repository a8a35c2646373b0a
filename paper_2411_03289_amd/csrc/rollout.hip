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
#include "sample_step.hpp"

namespace gpmppi {

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
    Cov P{};
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
        const StepJac jac = step_jacobian(dy, v, sth, cth);
        advance_pose(dy, v, w_, sth, cth, X, Y, th);
        propagate_cov(P, jac);

        // ---- chance-constraint geometry at (x_{k+1}, Sigma_{k+1}) (Eqs. 13-16); with Step 2
        // tightening the covariance is the nominal sequence's, shared by all samples
        float sa = P.p00, sb = P.p01, sc = P.p11;
        if (a.tight_sxy) {
            sa = a.tight_sxy[3 * (k + 1)];
            sb = a.tight_sxy[3 * (k + 1) + 1];
            sc = a.tight_sxy[3 * (k + 1) + 2];
        }
        const float hh = 0.5f * (sa - sc);
        const float lmax = 0.5f * (sa + sc) + sqrtf(hh * hh + sb * sb);
        // The polyline loop runs during the first output's contraction and the obstacle loop
        // during the second's, on the first S::lwaves waves, which finish their share of W first
        // (with one sample group both half-waves hold the same samples and write the same values).
        const float Xs = X, Ys = Y;
        float m[2], s2[2];
#pragma unroll
        for (int oo = 0; oo < 2; ++oo) {
            const int o = rev ? 1 - oo : oo;
            __syncthreads();   // staged inputs visible; previous k-operand readers are done
            const float qs[4] = {q[0] * a.gp.scale[o][0], q[1] * a.gp.scale[o][1], q[2] * a.gp.scale[o][2],
                                 q[3] * a.gp.scale[o][3]};
            m[o] = gp_gen<PREC, G, NW>(a.gp, o, qs, part, sl, lds, pred);
            s2[o] = gp_walk<PREC, G, NW, WALK>(a.gp, o, oo == 0 ? 1 - o : -1, rev, a.rotate, blk, lds, vred, sl,
                                               [&](int wv) {
                                                   world_loop<S::lwaves, S::B>(geo, oo, wv, sl, Xs, Ys, sa, sb, sc,
                                                                               lmax, ored);
                                               });
        }

        advance_velocities(dy, u, m[0], m[1], v, w_);
        // ---- the GP variance into the covariance (Eq. 10)
        add_gp_variance(P.p33, dt, s2[0]);
        add_gp_variance(P.p44, dt, s2[1]);

        const StageIn t = stage_inputs<S::lwaves, S::B>(geo, cw, ored, sl, X, Y, v, lmax, dgoal_min);
        add_stage_cost(cw, geo, t, s2[0], s2[1], disc, S_, Sc);
        if (writer) write_trace(a.trace, K, sg, k, X, Y, th, v, w_, P, m[0], m[1], s2[0], s2[1], t, u, true);
    }
    if (cw.w_term != 0.0f && !(dgoal_min <= cw.goal_tol)) {
        const float yk = cw.w_term - Sc;
        S_ = S_ + yk;
    }
    if (writer) a.costs[sg] = S_;
}

// ---- output split
// The two GP outputs of one sample block can run on two workgroups of a doubled
// grid, workgroup 2 blk + r computing output r: where the sample count alone
// would leave compute units idle, this halves each workgroup's kernel-vector
// and variance work.  Role 0 carries the full sample state, the covariance, the
// obstacle loop and the cost; role 1 the pose and velocities that its queries
// and the polyline loop need.  Both loops are dealt over all of a role's waves.
// The roles exchange, per step, the two GP means, the second output's variance
// and the squared distance to the polyline as 64-bit records (value, tag)
// stored and loaded at agent scope, one
// record per sample: a record is valid once its tag names this launch's epoch
// and the step, so no flag and no store-completion wait is needed.  Slots cycle
// over four steps (a writer runs at most two steps ahead of a slot's reader).
// The values reach the same arithmetic as in rollout_block, so the results are
// bitwise those of the unsplit kernel.  The launcher admits the shape only
// where the whole doubled grid fits the device at once, but other work on the
// device can still keep one role waiting: every wait is bounded
// (RolloutArgs::xspin polls), and a workgroup whose wait gives up abandons the
// exchange, marks its block in RolloutArgs::repair and sets the exchange
// time-out bit of the context's status word (its partner, waiting in turn,
// does the same).  The launcher follows every split launch with a repair
// launch of the unsplit kernel that recomputes exactly the marked blocks (the
// same results bit for bit) and exits at once elsewhere.

constexpr int kXvFail = 3 * 32;   // xv slot of wave 0's "an exchange wait gave up" flag

__device__ __forceinline__ uint32_t xch_tag(uint32_t epoch, int k) {
    return ((epoch & 0x7FFFFu) << 13) | (uint32_t)(k + 1);   // k + 1 <= 4096 < 2^13
}

// Role `role` of sample block blk (one sample group, G = 1); see above.
template <int PREC, int NW, int WALK>
__device__ __forceinline__ void rollout_block_split(const RolloutArgs &a, int blk, int role, unsigned char *lds,
                                                    float *pred, float *ored, float *vred, float *xv) {
    constexpr int G = 1;
    using S = Shapes<PREC, G, NW>;
    static_assert(S::B == 32, "exchange records hold one 32-sample group");
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int sl = lane % S::B;
    const int part = 2 * w + (lane >> 5);
    const int sg = blk * S::B + sl;
    const int K = a.K;
    const bool writer = role == 0 && sg < K && w == 0 && lane < S::B;
    const size_t zs_off = kgroup_bytes<PREC>(a.gp.Mpad);

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
    const float dt = dy.dt;
    const uint32_t epoch =
        __builtin_amdgcn_readfirstlane(__hip_atomic_load(a.xep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    unsigned long long *rec = a.xrec + (size_t)blk * kXchRecPerBlock;
    // kind: m0, m1, s2 of output 1, squared polyline distance at x_{k+1}
    auto slot = [&](int k, int kind) { return rec + ((k & 3) * 4 + kind) * 32; };
    bool broken = false;
    bool alone = false;   // set (uniformly) when an exchange wait gave up: the block is left to the repair
    const int spin = a.xspin;

    float X = a.x0[0], Y = a.x0[1], th = a.x0[2], v = a.x0[3], w_ = a.x0[4];
    Cov P{};
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
    if constexpr (mfma_gen<PREC>()) {
        stage_alpha<NW>(a.gp, lds, zs_off);
    } else {   // the inputs of this role's output, for the whole horizon
        StagedInputs st;
        stage_load<PREC, NW>(st, a.gp, role);
        stage_store<PREC, NW>(st, a.gp, lds, zs_off);
    }

    StageIn prev{};        // role 0: the previous step's cost inputs, completed by that step's s2 of output 1
    float s20_prev = 0.0f;
    for (int k = 0; k < a.T; ++k) {
        const bool rev = (k & 1) != 0;
        const uint32_t tag = xch_tag(epoch, k);
        const float2 u = sampled_control(np, k, sg, a.U[2 * k], a.U[2 * k + 1]);
        const float qs[4] = {v * a.gp.scale[role][0], w_ * a.gp.scale[role][1], u.x * a.gp.scale[role][2],
                             u.y * a.gp.scale[role][3]};
        float sth, cth;
        sincosf(th, &sth, &cth);
        if (role == 1) {
            advance_pose(dy, v, w_, sth, cth, X, Y, th);
            const float Xs = X, Ys = Y;
            __syncthreads();   // the previous step's k-operand and loop-result readers are done
            const float m1 = gp_gen<PREC, G, NW>(a.gp, 1, qs, part, sl, lds, pred);
            if (w == 0) xch_put(slot(k, 1), lane, m1, tag);
            const float s21 = gp_walk<PREC, G, NW, WALK>(a.gp, 1, -1, rev, a.rotate, blk, lds, vred, sl, [&](int wv) {
                world_loop<NW, S::B>(geo, 0, wv, sl, Xs, Ys, 0.0f, 0.0f, 0.0f, 0.0f, ored);
                if (wv == 0) {
                    const float m0 = xch_get(slot(k, 0), lane, tag, spin, broken);
                    if (lane < 32) xv[lane] = m0;
                    if (lane == 0) xv[kXvFail] = broken ? 1.0f : 0.0f;
                }
            });
            if (xv[kXvFail] != 0.0f) {   // the partner did not answer: leave the block to the repair
                alone = true;
                break;
            }
            if (w == 0) {
                xch_put(slot(k, 2), lane, s21, tag);
                if (geo.path_kind != 0) {
                    float best = INFINITY;
#pragma unroll
                    for (int p = 0; p < NW; ++p) best = fminf(best, ored[p * S::B + sl]);
                    xch_put(slot(k, 3), lane, best, tag);
                }
            }
            advance_velocities(dy, u, xv[sl], m1, v, w_);
            continue;
        }

        // ---- role 0: position and heading (Eqs. 1, 10)
        const StepJac jac = step_jacobian(dy, v, sth, cth);
        advance_pose(dy, v, w_, sth, cth, X, Y, th);
        __syncthreads();
        const float m0 = gp_gen<PREC, G, NW>(a.gp, 0, qs, part, sl, lds, pred);
        if (w == 0) xch_put(slot(k, 0), lane, m0, tag);

        // ---- chance-constraint geometry at (x_{k+1}, Sigma_{k+1}) (Eqs. 13-16): the position
        // block of A Sigma A^T does not involve the second output's variance of step k - 1,
        // which arrives during this step's contraction
        float sa, sb, sc;
        propagate_pos_block(P, jac, sa, sb, sc);
        if (a.tight_sxy) {
            sa = a.tight_sxy[3 * (k + 1)];
            sb = a.tight_sxy[3 * (k + 1) + 1];
            sc = a.tight_sxy[3 * (k + 1) + 2];
        }
        const float hh = 0.5f * (sa - sc);
        const float lmax = 0.5f * (sa + sc) + sqrtf(hh * hh + sb * sb);
        const float Xs = X, Ys = Y;
        const float s20 = gp_walk<PREC, G, NW, WALK>(a.gp, 0, -1, rev, a.rotate, blk, lds, vred, sl, [&](int wv) {
            world_loop<NW, S::B>(geo, 1, wv, sl, Xs, Ys, sa, sb, sc, lmax, ored);
            if (wv == 0) {
                const float m1 = xch_get(slot(k, 1), lane, tag, spin, broken);
                const uint32_t tp = xch_tag(epoch, k - 1);
                const float s21p = k > 0 ? xch_get(slot(k - 1, 2), lane, tp, spin, broken) : 0.0f;
                const float bestp =
                    k > 0 && geo.path_kind != 0 ? xch_get(slot(k - 1, 3), lane, tp, spin, broken) : 0.0f;
                if (lane < 32) {
                    xv[lane] = m1;
                    xv[32 + lane] = s21p;
                    xv[64 + lane] = bestp;
                }
                if (lane == 0) xv[kXvFail] = broken ? 1.0f : 0.0f;
            }
        });
        if (xv[kXvFail] != 0.0f) {   // the partner did not answer: leave the block to the repair
            alone = true;
            break;
        }
        const float m1 = xv[sl];
        if (k > 0) {   // step k - 1 completed: its second variance into Sigma_ww, its lane distance, its cost
            const float s21p = xv[32 + sl];
            add_gp_variance(P.p44, dt, s21p);
            if (geo.path_kind != 0) prev.dl = sqrtf(xv[64 + sl]);
            add_stage_cost(cw, geo, prev, s20_prev, s21p, disc, S_, Sc);
            if (writer) write_deferred_trace(a.trace, K, sg, k - 1, s21p, prev);
        }
        propagate_cov(P, jac);
        advance_velocities(dy, u, m0, m1, v, w_);
        add_gp_variance(P.p33, dt, s20);
        prev = stage_inputs<NW, S::B, false>(geo, cw, ored, sl, X, Y, v, lmax, dgoal_min);
        s20_prev = s20;
        if (writer) write_trace(a.trace, K, sg, k, X, Y, th, v, w_, P, m0, m1, s20, 0.0f, prev, u, false, false);
    }
    if (role == 0 && !alone) {
        const uint32_t tl = xch_tag(epoch, a.T - 1);
        const float s21p = xch_get(slot(a.T - 1, 2), lane, tl, spin, broken);
        if (geo.path_kind != 0) prev.dl = sqrtf(xch_get(slot(a.T - 1, 3), lane, tl, spin, broken));
        alone = __syncthreads_or(broken) != 0;
        if (!alone) {
            add_stage_cost(cw, geo, prev, s20_prev, s21p, disc, S_, Sc);
            if (writer) write_deferred_trace(a.trace, K, sg, a.T - 1, s21p, prev);
            if (cw.w_term != 0.0f && !(dgoal_min <= cw.goal_tol)) {
                const float yk = cw.w_term - Sc;
                S_ = S_ + yk;
            }
            if (writer) a.costs[sg] = S_;
        }
    }
    if (alone && tid == 0) {   // hand the block to the repair launch that follows
        __hip_atomic_store(a.repair + blk, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (a.flags)
            __hip_atomic_fetch_or(a.flags, GPMPPI_FLAG_EXCHANGE_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // the last workgroup to finish advances the epoch for the next launch
    __syncthreads();
    if (tid == 0) {
        const uint32_t n = __hip_atomic_fetch_add(a.xep + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (n == gridDim.x - 1) {
            __hip_atomic_store(a.xep + 1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(a.xep, epoch + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <int PREC, int NW, int WALK>
__global__ __launch_bounds__(64 * NW) void rollout_split_kernel(RolloutArgs a) {
    using S = Shapes<PREC, 1, NW>;
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ float pred[S::rparts * S::B];
    __shared__ float ored[2 * NW * S::B];   // both loops on every wave (rollout_block_split)
    __shared__ float vred[NW * S::B];
    __shared__ float xv[kXvFail + 1];
    const int role = __builtin_amdgcn_readfirstlane((int)(blockIdx.x & 1));
    rollout_block_split<PREC, NW, WALK>(a, blockIdx.x >> 1, role, lds, pred, ored, vred, xv);
}

// a.repair == NULL: every block.  Otherwise the repair launch after an output
// split (G = 1): only the blocks the split launch marked, whose marks it clears.
template <int PREC, int G, int NW, int WALK>
__global__ __launch_bounds__(64 * NW) void rollout_kernel(RolloutArgs a) {
    using S = Shapes<PREC, G, NW>;
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ float pred[S::rparts * S::B];
    __shared__ float ored[2 * S::lwaves * S::B];
    __shared__ float vred[NW * S::B];
    if (a.repair && __hip_atomic_load(a.repair + blockIdx.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) return;
    rollout_block<PREC, G, NW, WALK>(a, blockIdx.x, lds, pred, ored, vred);
    if (a.repair && threadIdx.x == 0)
        __hip_atomic_store(a.repair + blockIdx.x, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The problems of a batch, read-only for the whole launch: through the constant
// address space their fields come in by scalar loads the compiler may repeat
// where they are used, as a kernel argument's do, instead of vector loads kept
// live in registers across the item (which spilled the eight-wave shapes).
typedef const RolloutArgs __attribute__((address_space(4))) ConstRolloutArgs;

// Persistent rollout of many independent problems: every workgroup takes
// (problem, sample block) items from a shared counter until the list (sorted
// longest first) is exhausted.  Results do not depend on which workgroup
// runs an item.  *counter must be 0 at launch.
template <int PREC, int G, int NW>
__global__ __launch_bounds__(64 * NW) void rollout_batch_kernel(ConstRolloutArgs *probs, const int2 *items,
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
        rollout_block<PREC, G, NW>(*(const RolloutArgs *)&probs[p], b, lds, pred, ored, vred);
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

// Workgroups of fn (64 NW threads, lds bytes of dynamic LDS) resident at once on the device.
template <typename F>
static hipError_t resident_blocks(F *fn, int NW, size_t lds, int &n) {
    int dev = 0, ncu = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(fn), 64 * NW, lds);
    n = e == hipSuccess ? per_cu * ncu : 0;
    return e;
}

template <int PREC, int NW, int WALK>
static hipError_t split_capacity_w(int Mpad, int &n) {
    const size_t lds = dyn_lds_bytes<PREC, 1>(Mpad);
    hipError_t e = set_lds(rollout_split_kernel<PREC, NW, WALK>, lds);
    if (e != hipSuccess) return e;
    return resident_blocks(rollout_split_kernel<PREC, NW, WALK>, NW, lds, n);
}

template <int PREC, int NW>
static int split_capacity_t(int Mpad) {
    int n = 0;
    const hipError_t e = walk_by_rows(Mpad / 32, NW) ? split_capacity_w<PREC, NW, kWalkRows>(Mpad, n)
                                                    : split_capacity_w<PREC, NW, kWalkPairs>(Mpad, n);
    return e == hipSuccess ? 32 * (n / 2) : 0;
}

template <int PREC, int NW, int WALK>
static hipError_t launch_rollout_split_w(const RolloutArgs &a, hipStream_t st) {
    if (!a.xrec || !a.xep || !a.repair) return hipErrorInvalidValue;
    const size_t lds = dyn_lds_bytes<PREC, 1>(a.gp.Mpad);
    int cap = 0;
    hipError_t e = split_capacity_w<PREC, NW, WALK>(a.gp.Mpad, cap);
    if (e != hipSuccess) return e;
    const int nblk = (a.K + 31) / 32;
    if (2 * nblk > cap) return hipErrorCooperativeLaunchTooLarge;   // both roles of every block resident together
    hipLaunchKernelGGL((rollout_split_kernel<PREC, NW, WALK>), dim3(2 * nblk), dim3(64 * NW), lds, st, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // the repair launch: the unsplit kernel recomputes the blocks whose exchange gave up
    return launch_rollout_w<PREC, 1, NW, WALK>(a, st);
}

template <int PREC, int NW>
static hipError_t launch_rollout_split_t(const RolloutArgs &a, hipStream_t st) {
    return walk_by_rows(a.gp.NT, NW) ? launch_rollout_split_w<PREC, NW, kWalkRows>(a, st)
                                     : launch_rollout_split_w<PREC, NW, kWalkPairs>(a, st);
}

template <int PREC>
static hipError_t launch_rollout_p(const RolloutArgs &a, int G, int NW, int split, hipStream_t st) {
    if (split) return NW == 8 ? launch_rollout_split_t<PREC, 8>(a, st) : launch_rollout_split_t<PREC, kWaves>(a, st);
    if (NW == 8) return G == 2 ? launch_rollout_t<PREC, 2, 8>(a, st) : launch_rollout_t<PREC, 1, 8>(a, st);
    return G == 2 ? launch_rollout_t<PREC, 2, kWaves>(a, st) : launch_rollout_t<PREC, 1, kWaves>(a, st);
}

template <int PREC, int G, int NW>
static hipError_t launch_rollout_batch_t(const RolloutArgs *probs, const int2 *items, int n_items, uint32_t *counter,
                                         int Mpad_max, int grid, hipStream_t st) {
    const size_t lds = dyn_lds_bytes<PREC, G>(Mpad_max);
    hipError_t e = set_lds(rollout_batch_kernel<PREC, G, NW>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((rollout_batch_kernel<PREC, G, NW>), dim3(grid), dim3(64 * NW), lds, st,
                       (ConstRolloutArgs *)probs, items, n_items, counter);
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

hipError_t launch_rollout(const RolloutArgs &args, int precision, int G, int NW, int split, hipStream_t st) {
    if (NW == kPipeWaves) {
        if (split) return hipErrorInvalidValue;
        RolloutArgs a = args;
        a.repair = nullptr;
        return launch_rollout_pipe(a, precision, G, st);
    }
    if (G < 1 || G > groups_for(precision, args.gp.Mpad) || (NW != kWaves && NW != 8) || (split != 0 && split != 1) ||
        (split && G != 1))
        return hipErrorInvalidValue;
    RolloutArgs a = args;
    if (!split) a.repair = nullptr;   // an unsplit launch computes every block
    switch (precision) {
        case GPMPPI_FP32: return launch_rollout_p<GPMPPI_FP32>(a, G, NW, split, st);
        case GPMPPI_BF16: return launch_rollout_p<GPMPPI_BF16>(a, G, NW, split, st);
        default: return launch_rollout_p<GPMPPI_BF16X3>(a, G, NW, split, st);
    }
}

int rollout_split_capacity(int precision, int Mpad, int NW) {
    if (NW != kWaves && NW != 8) return 0;
    switch (precision) {
        case GPMPPI_FP32: return NW == 8 ? split_capacity_t<GPMPPI_FP32, 8>(Mpad) : split_capacity_t<GPMPPI_FP32, kWaves>(Mpad);
        case GPMPPI_BF16: return NW == 8 ? split_capacity_t<GPMPPI_BF16, 8>(Mpad) : split_capacity_t<GPMPPI_BF16, kWaves>(Mpad);
        default: return NW == 8 ? split_capacity_t<GPMPPI_BF16X3, 8>(Mpad) : split_capacity_t<GPMPPI_BF16X3, kWaves>(Mpad);
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
