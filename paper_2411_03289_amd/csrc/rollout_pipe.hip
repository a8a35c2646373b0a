// Wave-specialised K-sample x T-step rollout for the BF16 forms at M_pad = 1024
// (Alg. 1 Step 1 with Eqs. 1-3, 10, 11-16): the arithmetic of rollout_kernel,
// laid out so that the kernel-vector generation and the per-sample step run
// beside the variance contraction instead of between its passes.
//
// A workgroup of twelve wave64s owns B = 32 G samples.
//  * Waves 0-7, the walkers, only contract v = W k on the matrix cores.
//    Walker w takes the row-tile pairs 15 - w and w of W (34 iterations of two
//    32x32 blocks, the same count for every walker), always columns descending,
//    for the output slots e = 2 k + o of all steps one after another; W streams
//    through a register ring three iterations deep that runs on from one slot
//    into the next.  The walkers issue at a raised wave priority, so that a
//    walker's next matrix-core product goes ahead of the state waves' vector
//    instructions on the same SIMD.
//  * Waves 8-11, the state waves, keep the sample state (every state wave all B
//    samples, as every wave of rollout_kernel does), draw the noise, generate
//    the kernel vectors (the other shapes' matrix-core generation, bit for bit
//    the same operand), the GP means, the chance-constraint geometry and the
//    costs.  State wave g writes the column tiles 31 - g, 27 - g, ..., 3 - g of
//    every slot's k operand.
//
// One k operand region in LDS (128 KB; alpha of both outputs beside it) serves all slots in turn, and
// per column tile c two LDS counters hand it back and forth:
//   ready[c] = e + 1 once a state wave has written tile c for slot e;
//   freed[c] counts the walkers' last reads of tile c over all slots: it may be
//            rewritten for slot e once the count reaches users(c) e.
// A walker's first pair reads tiles 31 - 2w .. 0 and its second 2w + 1 .. 0, so
// the high tiles are released early in a slot and refilled for the next slot
// while the walkers are still on the low tiles, and the next slot starts on the
// high tiles: the walkers do not wait for the generation.  The walkers leave
// each slot's partial |v|^2 per sample in one of four LDS rows and count their
// finished slots; the state waves read the variances of step k - 1 after
// generating the first output of step k (the covariance needs them only from
// the propagation of step k on) and meet once per step at an LDS counter to
// combine their partial means and constraint partials.
//
// Every hand-over is inside one workgroup, whose waves are resident together.
// Every wait polls a bounded number of times (RolloutArgs::xspin, the exchange
// spin of the context); one that gives up marks the workgroup, after which every
// wait returns at once, so the launch ends; the workgroup's costs are then NaN
// and GPMPPI_FLAG_PIPELINE_STALL is set.
#include "gp_tiles.hpp"
#include "sample_step.hpp"

namespace gpmppi {

namespace {

constexpr int kPipeWalkers = 8;
constexpr int kPipeStateWaves = 4;
constexpr int kPipeNT = 32;     // column tiles of W at M_pad = 1024
constexpr int kPipeVRows = 4;   // slots of walker partials held in LDS

struct PipeSync {
    uint32_t ready[kPipeNT];
    uint32_t freed[kPipeNT];
    uint32_t vdone[kPipeWalkers];   // slots finished by each walker
    uint32_t sbar;                  // state-wave meeting counter
    uint32_t stall;                 // a wait gave up
    int spin;                       // polls per wait before it gives up (RolloutArgs::xspin; < 0: none)
};

// The GP output of slot e: 0, 1, 1, 0, 0, 1, ... (step k takes output k % 2 first), so that
// consecutive slots walk the same W where the steps meet and its blocks are still in L2.
__device__ __forceinline__ int slot_output(int e) { return (e ^ (e >> 1)) & 1; }

// Walkers that read column tile c in a slot: walker w reads c <= 31 - 2w.
__device__ __forceinline__ uint32_t pipe_users(int c) { return c <= 17 ? 8u : (uint32_t)((31 - c) / 2 + 1); }

__device__ __forceinline__ uint32_t lds_get(const uint32_t *p) {
    return __builtin_amdgcn_readfirstlane(__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
}
__device__ __forceinline__ void lds_put(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_add(uint32_t *p, uint32_t v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// A hand-over orders LDS accesses: the hardware performs one wave's LDS
// instructions in issue order, and this keeps the compiler from moving data
// accesses across the counter access next to it.
__device__ __forceinline__ void lds_order() { __asm__ __volatile__("" ::: "memory"); }

// Waits until *p >= target (bounded; see above).
__device__ __forceinline__ void pipe_wait(const uint32_t *p, uint32_t target, PipeSync &sy) {
    if (__builtin_expect(lds_get(p) >= target, 1)) return;
    const int polls = sy.spin;
    for (int n = 0; n < polls; ++n) {
        __builtin_amdgcn_s_sleep(1);
        if (lds_get(p) >= target || lds_get(&sy.stall) != 0u) return;
    }
    lds_put(&sy.stall, 1u);
}

// ---------------------------------------------------------------- walkers
template <int PREC, int G>
__device__ __forceinline__ void pipe_walker(const RolloutArgs &a, int w, int lane, unsigned char *lds, PipeSync &sy,
                                            float *vred) {
    constexpr int B = 32 * G;
    const int Mpad = a.gp.Mpad;
    const int nslot = 2 * a.T;
    // row-tile pairs hi = 15 - w then lo = w (34 iterations per slot for every walker), the
    // list repeated (the cursor reads it modulo 8 pairs)
    const int hi = kPipeNT / 2 - 1 - w, lo = w;
    const uint64_t two = (uint64_t)hi | ((uint64_t)lo << 8);
    const uint64_t plist = two | (two << 16) | (two << 32) | (two << 48);
    const WRsrc<PREC> wr0 = w_rsrc<PREC>(a.gp, 0), wr1 = w_rsrc<PREC>(a.gp, 1);
    const int voff = 16 * lane;
    const unsigned char *kgrp[G];
#pragma unroll
    for (int gg = 0; gg < G; ++gg) kgrp[gg] = lds + gg * kgroup_bytes<PREC>(Mpad);

    WBlock<PREC> ring[3][2];   // W blocks of the next three iterations
    KOp<PREC> kb[G];           // k operand of the current iteration
    v16f acc[2][G];
    float sq[G];
#pragma unroll
    for (int gg = 0; gg < G; ++gg) {
        acc[0][gg] = v16f{};
        acc[1][gg] = v16f{};
        sq[gg] = 0.0f;
    }
    Cursor pc, mc;   // prefetch and compute cursors; a slot is two pairs
    cursor_start<true>(pc, plist);
    cursor_start<true>(mc, plist);
    int pe = 0, me = 0;   // their slots
    // W blocks of the prefetch cursor's iteration (the diagonal block twice in place of the
    // zero block above it, so every iteration issues the same loads)
    auto fetch = [&](int r) {
        WRsrc<PREC> wr;
        wr.h = slot_output(pe) ? wr1.h : wr0.h;
        wr.l = slot_output(pe) ? wr1.l : wr0.l;
        const int b0 = pair_block(pc);
        load_wblock_rs<PREC>(ring[r][0], wr, pair_zero(pc) ? b0 + 1 : b0, voff);
        load_wblock_rs<PREC>(ring[r][1], wr, b0 + 1, voff);
        if (cursor_next<true>(pc, plist) && (pc.n & 1) == 0) ++pe;
    };
    // Tiles known to be ready for slot kslot (bit c: tile c), refreshed from all 32 ready
    // counters at once only when a tile not yet known is needed: the state waves usually run
    // ahead, so most iterations need no LDS round trip before their operand reads.
    uint32_t known = 0u;
    int kslot = 0;
    auto need = [&](int c, int e) {
        if (e != kslot) {
            known = 0u;
            kslot = e;
        }
        if ((known >> c) & 1u) return;
        const uint32_t r = __hip_atomic_load(&sy.ready[lane & 31], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        known = (uint32_t)__builtin_amdgcn_ballot_w64(r >= (uint32_t)e + 1u);
        if ((known >> c) & 1u) return;
        pipe_wait(&sy.ready[c], (uint32_t)e + 1u, sy);
        known |= 1u << c;
    };
    fetch(0);
    fetch(1);
    fetch(2);
    if (nslot > 0) need(mc.it, 0);
    lds_order();
#pragma unroll
    for (int gg = 0; gg < G; ++gg) load_kop<PREC>(kb[gg], kgrp[gg], mc.it, lane, Mpad);

    // the ring slot of an iteration is its index mod 3; the fetches past the last iteration
    // read W blocks of the repeated pair list and are never used
    const int total = nslot * (2 * hi + 2 * lo + 4);
    for (int base = 0; base < total; base += 3) {
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            if (base + r >= total) break;
            if (!pair_zero(mc)) {
#pragma unroll
                for (int gg = 0; gg < G; ++gg) mma_block<PREC>(acc[0][gg], ring[r][0], kb[gg]);
            }
#pragma unroll
            for (int gg = 0; gg < G; ++gg) mma_block<PREC>(acc[1][gg], ring[r][1], kb[gg]);
            // the wave's last read of this tile in the slot: hand it back (its operand is in
            // registers: the products above waited for it)
            if ((mc.n & 1) != 0 || mc.it > 2 * lo + 1) {
                lds_order();
                if (lane == 0) lds_add(&sy.freed[mc.it], 1u);
            }
            fetch(r);
            const bool pair_end = cursor_next<true>(mc, plist);
            const bool slot_end = pair_end && (mc.n & 1) == 0;
            const int ne = me + (slot_end ? 1 : 0);
            if (ne < nslot) need(mc.it, ne);
            lds_order();
#pragma unroll
            for (int gg = 0; gg < G; ++gg) load_kop<PREC>(kb[gg], kgrp[gg], mc.it, lane, Mpad);
            if (__builtin_expect(pair_end, 0)) {
#pragma unroll
                for (int gg = 0; gg < G; ++gg) {
#pragma unroll
                    for (int e = 0; e < 16; ++e) {
                        sq[gg] = fmaf(acc[0][gg][e], acc[0][gg][e], sq[gg]);
                        sq[gg] = fmaf(acc[1][gg][e], acc[1][gg][e], sq[gg]);
                    }
                    acc[0][gg] = v16f{};
                    acc[1][gg] = v16f{};
                }
                if (slot_end) {
                    float *vr = vred + ((me % kPipeVRows) * kPipeWalkers + w) * B;
#pragma unroll
                    for (int gg = 0; gg < G; ++gg) {
                        const float t = sq[gg] + shfl_xor(sq[gg], 32);
                        if (lane < 32) vr[gg * 32 + lane] = t;
                        sq[gg] = 0.0f;
                    }
                    lds_order();
                    if (lane == 0) lds_put(&sy.vdone[w], (uint32_t)ne);
                    me = ne;
                }
            }
        }
    }
}

// ---------------------------------------------------------------- state waves
__device__ __forceinline__ int pipe_tile(int g, int n) { return kPipeNT - 1 - g - kPipeStateWaves * n; }

// Kernel vectors of output o for slot e into the state wave's column tiles
// jt = 31 - g - 4n of the k operand, each once the walkers have released it, by
// the matrix-core generation of the other shapes (gen_bop, then gen_tile's and
// gen_store's arithmetic and layout one sample group at a time: the same operand
// bits); the points' A operands stream from memory one tile ahead, alpha comes
// from LDS.  Returns the lane's sample's partial GP mean over
// the wave's tiles (lane l: sample l % B).
template <int PREC, int G>
__device__ __forceinline__ float pipe_gen(const GpDev &gp, int o, const float qs[4], int e, int g, int lane,
                                          unsigned char *lds, const float *alds, PipeSync &sy) {
    const int Mpad = gp.Mpad, hl = lane >> 5;
    // the A operands through a buffer resource: one lane offset, the tile in the scalar offset
    const __amdgpu_buffer_rsrc_t zr = uniform_rsrc(gp.zop + o * gp.zop_stride, (long long)gp.NT * 128 * 16);
    const float *al = alds + (size_t)o * Mpad;
    uint4 bop[G][2];
    gen_bop<G>(qs, hl, bop);
    float ms[G];
#pragma unroll
    for (int gg = 0; gg < G; ++gg) ms[gg] = 0.0f;
    auto fetch = [&](uint4 (&d)[2], int n) {
        const int jt = pipe_tile(g, n);
        d[0] = buf_load16(zr, 16 * lane, jt * 2048);
        d[1] = buf_load16(zr, 16 * lane, jt * 2048 + 1024);
    };
    auto tile = [&](const uint4 (&d)[2], int n) {
        const int jt = pipe_tile(g, n);
        if (e > 0) pipe_wait(&sy.freed[jt], pipe_users(jt) * (uint32_t)e, sy);
        lds_order();
        const v4f *ap = reinterpret_cast<const v4f *>(al + 32 * jt + 8 * hl);
        const v4f alv[4] = {ap[0], ap[1], ap[4], ap[5]};
        // one sample group at a time (gen_tile's arithmetic), its operand stored at once
#pragma unroll
        for (int gg = 0; gg < G; ++gg) {
            v16f ex = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf(d[0]), as_bf(bop[gg][0]), v16f{}, 0, 0, 0);
            ex = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf(d[1]), as_bf(bop[gg][1]), ex, 0, 0, 0);
            float kv[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) kv[r] = __builtin_amdgcn_exp2f(ex[r]);
#pragma unroll
            for (int r = 0; r < 16; ++r) ms[gg] = fmaf(kv[r], alv[r >> 2][r & 3], ms[gg]);
            uint32_t hv[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) hv[i] = pack_bf16x2(kv[2 * i], kv[2 * i + 1]);
            uint4 *K = reinterpret_cast<uint4 *>(lds + gg * kgroup_bytes<PREC>(Mpad)) + (size_t)jt * 128;
            K[lane] = make_uint4(hv[0], hv[1], hv[2], hv[3]);
            K[64 + lane] = make_uint4(hv[4], hv[5], hv[6], hv[7]);
            if constexpr (PREC == GPMPPI_BF16X3) {
                uint32_t lv[8];
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    lv[i] = pack_bf16x2(kv[2 * i] - bf16_to_f32((uint16_t)hv[i]),
                                        kv[2 * i + 1] - bf16_to_f32((uint16_t)(hv[i] >> 16)));
                uint4 *L = reinterpret_cast<uint4 *>(lds + gg * kgroup_bytes<PREC>(Mpad) + (size_t)Mpad * 64) +
                           (size_t)jt * 128;
                L[lane] = make_uint4(lv[0], lv[1], lv[2], lv[3]);
                L[64 + lane] = make_uint4(lv[4], lv[5], lv[6], lv[7]);
            }
            // the group's mean products here and now: deferred into the next tile (the compiler
            // would rotate them), its 16 kernel values would stay live across the waits
            __asm__ __volatile__("" : "+v"(ms[gg]));
        }
        lds_order();
        if (lane == 0) lds_put(&sy.ready[jt], (uint32_t)e + 1u);
    };
    // the A operands of the current and the next tile (the wave's tile count is even)
    uint4 za[2], zb[2];
    fetch(za, 0);
#pragma unroll 1
    for (int n = 0; n < kPipeNT / kPipeStateWaves; n += 2) {
        fetch(zb, n + 1);
        tile(za, n);
        if (n + 2 < kPipeNT / kPipeStateWaves) fetch(za, n + 2);
        tile(zb, n + 1);
    }
    // lane l holds sample 32 gg + l % 32's partial over the rows of half-wave l / 32
    const float t0 = ms[0] + shfl_xor(ms[0], 32);
    if constexpr (G == 2) {
        const float t1 = ms[1] + shfl_xor(ms[1], 32);
        return hl ? t1 : t0;
    }
    return t0;
}

// Trace rows through buffer resources built per row block from the array's
// wave-uniform base (scalar registers) and the sample's byte offset (one
// register): no per-lane 64-bit addresses stay live across the steps.  A NULL
// array gets an empty range, where stores are dropped.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t trace_rows(float *base, size_t first, int count) {
    return uniform_rsrc(base ? base + first : nullptr, base ? (long long)count * 4 : 0);
}
__device__ __forceinline__ void trace_put(__amdgpu_buffer_rsrc_t r, int row, int K, int soff, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, soff, row * K * 4, 0);
}

// write_trace's rows of step k but the GP variances (state after the step: row
// k + 1 of x and Sigma_XY, whose position block the variances of step k do not
// reach).
__device__ __forceinline__ void pipe_trace_step(const gpmppi_trace &tr, int K, int soff, int k, float X, float Y,
                                                float th, float v, float w, const Cov &P, float m0, float m1,
                                                const StageIn &t, float2 u) {
    const size_t kk = (size_t)k, KK = (size_t)K;
    const __amdgpu_buffer_rsrc_t rx = trace_rows(tr.x_d, (kk + 1) * 5 * KK, 5 * K);
    trace_put(rx, 0, K, soff, X);
    trace_put(rx, 1, K, soff, Y);
    trace_put(rx, 2, K, soff, th);
    trace_put(rx, 3, K, soff, v);
    trace_put(rx, 4, K, soff, w);
    const __amdgpu_buffer_rsrc_t rs = trace_rows(tr.sxy_d, (kk + 1) * 3 * KK, 3 * K);
    trace_put(rs, 0, K, soff, P.p00);
    trace_put(rs, 1, K, soff, P.p01);
    trace_put(rs, 2, K, soff, P.p11);
    const __amdgpu_buffer_rsrc_t rm = trace_rows(tr.gp_mean_d, kk * 2 * KK, 2 * K);
    trace_put(rm, 0, K, soff, m0);
    trace_put(rm, 1, K, soff, m1);
    trace_put(trace_rows(tr.d_lane_d, kk * KK, K), 0, K, soff, t.dl);
    trace_put(trace_rows(tr.lane_margin_d, kk * KK, K), 0, K, soff, t.rbar - t.dl);
    trace_put(trace_rows(tr.obs_margin_d, kk * KK, K), 0, K, soff, t.om);
    const __amdgpu_buffer_rsrc_t ru = trace_rows(tr.u_d, kk * 2 * KK, 2 * K);
    trace_put(ru, 0, K, soff, u.x);
    trace_put(ru, 1, K, soff, u.y);
}

__device__ __forceinline__ void pipe_trace_var(const gpmppi_trace &tr, int K, int soff, int k, float s20, float s21) {
    const __amdgpu_buffer_rsrc_t rv = trace_rows(tr.gp_var_d, (size_t)k * 2 * K, 2 * K);
    trace_put(rv, 0, K, soff, s20);
    trace_put(rv, 1, K, soff, s21);
}

// add_stage_cost in two parts: the terms without the GP variances, when the
// step's constraint inputs are known (disc then advances) ...
__device__ __forceinline__ float stage_cost_rest(const CostWeights &cw, const Geometry &geo, const StageIn &t,
                                                 float &disc) {
    float c = cw.w_dev * (t.dl * geo.inv_half_width) + cw.w_speed * (t.dv * t.dv);
    if (t.dl > t.rbar) c += cw.w_lane * disc;
    if (t.om <= 0.0f) c += cw.w_obs;
    if (cw.w_goal != 0.0f || cw.w_term != 0.0f) c += cw.w_goal * t.dg;
    disc *= cw.discount;
    return c;
}

// ... and, once the variances arrive, the whole stage cost into the
// Kahan-compensated sum (S, Sc) of Eq. (5).
__device__ __forceinline__ void add_stage_cost_var(const CostWeights &cw, float rest, float s2a, float s2b, float &S,
                                                   float &Sc) {
    const float c = cw.w_var * (s2a + s2b) + rest;
    const float yk = c - Sc;
    const float tk = S + yk;
    Sc = (tk - S) - yk;
    S = tk;
}

template <int PREC, int G>
__device__ __forceinline__ void pipe_state(const RolloutArgs &a, int blk, int g, int lane, unsigned char *lds,
                                           PipeSync &sy, const float *vred, float *pred, float *ored) {
    constexpr int B = 32 * G, LW = kPipeStateWaves;
    const int sl = lane % B;
    const int sg = blk * B + sl;
    const int K = a.K;
    const bool writer = g == 0 && lane < B && sg < K;

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
    const GpDev &gp = a.gp;
    const float *alds = reinterpret_cast<const float *>(lds + G * kgroup_bytes<PREC>(gp.Mpad));

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

    // the GP variances of step k from the walkers' partials
    auto variances = [&](int k, float &s20, float &s21) {
        for (int w = 0; w < kPipeWalkers; ++w) pipe_wait(&sy.vdone[w], (uint32_t)(2 * k + 2), sy);
        lds_order();
        // slot 2k holds output k % 2, slot 2k + 1 the other
        const int first = k & 1;
        const float *r0 = vred + ((2 * k + first) % kPipeVRows) * kPipeWalkers * B;
        const float *r1 = vred + ((2 * k + 1 - first) % kPipeVRows) * kPipeWalkers * B;
        float v0 = 0.0f, v1 = 0.0f;
#pragma unroll
        for (int w = 0; w < kPipeWalkers; ++w) {
            v0 += r0[w * B + sl];
            v1 += r1[w * B + sl];
        }
        s20 = gp.vscale[0] * (gp.sn2[0] + fmaxf(0.0f, gp.sf2[0] - v0));
        s21 = gp.vscale[1] * (gp.sn2[1] + fmaxf(0.0f, gp.sf2[1] - v1));
    };

    float rest = 0.0f;   // step k - 1's stage cost without its GP variances
    uint32_t met = 0;
    for (int k = 0; k < a.T; ++k) {
        const float2 u = sampled_control(np, k, sg, a.U[2 * k], a.U[2 * k + 1]);
        const float q[4] = {v, w_, u.x, u.y};
        float qs[4];
        const int oa = k & 1, ob = 1 - oa;   // the outputs of slots 2k and 2k + 1
#pragma unroll
        for (int d = 0; d < 4; ++d) qs[d] = q[d] * gp.scale[oa][d];
        const float msa = pipe_gen<PREC, G>(gp, oa, qs, 2 * k, g, lane, lds, alds, sy);

        if (k > 0) {   // step k - 1's variances: Sigma_k complete, its cost
            float s20, s21;
            variances(k - 1, s20, s21);
            add_gp_variance(P.p33, dy.dt, s20);
            add_gp_variance(P.p44, dy.dt, s21);
            add_stage_cost_var(cw, rest, s20, s21, S_, Sc);
            if (writer) pipe_trace_var(a.trace, K, 4 * sg, k - 1, s20, s21);
        }

        // position, heading and A Sigma A^T (Eqs. 1, 10)
        float sth, cth;
        sincosf(th, &sth, &cth);
        const StepJac jac = step_jacobian(dy, v, sth, cth);
        advance_pose(dy, v, w_, sth, cth, X, Y, th);
        propagate_cov(P, jac);

        // chance-constraint geometry at (x_{k+1}, Sigma_{k+1}) (Eqs. 13-16), this wave's share
        float sa = P.p00, sb = P.p01, sc = P.p11;
        if (a.tight_sxy) {
            sa = a.tight_sxy[3 * (k + 1)];
            sb = a.tight_sxy[3 * (k + 1) + 1];
            sc = a.tight_sxy[3 * (k + 1) + 2];
        }
        const float hh = 0.5f * (sa - sc);
        const float lmax = 0.5f * (sa + sc) + sqrtf(hh * hh + sb * sb);
        float *orow = ored + (k & 1) * 2 * LW * B;
        world_loop<LW, B>(geo, 0, g, sl, X, Y, sa, sb, sc, lmax, orow);
        world_loop<LW, B>(geo, 1, g, sl, X, Y, sa, sb, sc, lmax, orow);

#pragma unroll
        for (int d = 0; d < 4; ++d) qs[d] = q[d] * gp.scale[ob][d];
        const float msb = pipe_gen<PREC, G>(gp, ob, qs, 2 * k + 1, g, lane, lds, alds, sy);

        // the state waves meet: means (row o: output o) and constraint partials of all four
        float *prow = pred + (k & 1) * 2 * LW * B;
        if (lane < B) {
            prow[(oa * LW + g) * B + sl] = msa;
            prow[(ob * LW + g) * B + sl] = msb;
        }
        lds_order();
        met += LW;
        if (lane == 0) lds_add(&sy.sbar, 1u);
        pipe_wait(&sy.sbar, met, sy);
        lds_order();
        float m0 = 0.0f, m1 = 0.0f;
#pragma unroll
        for (int p = 0; p < LW; ++p) {
            m0 += prow[p * B + sl];
            m1 += prow[(LW + p) * B + sl];
        }
        advance_velocities(dy, u, m0, m1, v, w_);
        const StageIn t = stage_inputs<LW, B>(geo, cw, orow, sl, X, Y, v, lmax, dgoal_min);
        rest = stage_cost_rest(cw, geo, t, disc);
        if (writer) pipe_trace_step(a.trace, K, 4 * sg, k, X, Y, th, v, w_, P, m0, m1, t, u);
    }
    if (a.T > 0) {
        float s20, s21;
        variances(a.T - 1, s20, s21);
        add_stage_cost_var(cw, rest, s20, s21, S_, Sc);
        if (writer) pipe_trace_var(a.trace, K, 4 * sg, a.T - 1, s20, s21);
    }
    if (cw.w_term != 0.0f && !(dgoal_min <= cw.goal_tol)) {
        const float yk = cw.w_term - Sc;
        S_ = S_ + yk;
    }
    if (lds_get(&sy.stall) != 0u) {
        S_ = __builtin_nanf("");
        if (writer && lane == 0 && a.flags)
            __hip_atomic_fetch_or(a.flags, GPMPPI_FLAG_PIPELINE_STALL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (writer) a.costs[sg] = S_;
}

}  // namespace

template <int PREC, int G>
__global__ __launch_bounds__(64 * (kPipeWalkers + kPipeStateWaves)) void rollout_pipe_kernel(RolloutArgs a) {
    constexpr int B = 32 * G;
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ PipeSync sy;
    __shared__ float vred[kPipeVRows * kPipeWalkers * B];
    __shared__ float pred[2 * 2 * kPipeStateWaves * B];
    __shared__ float ored[2 * 2 * kPipeStateWaves * B];
    const int tid = threadIdx.x;
    if (tid < (int)(offsetof(PipeSync, spin) / 4)) reinterpret_cast<uint32_t *>(&sy)[tid] = 0u;
    if (tid == 0) sy.spin = a.xspin;
    stage_alpha<kPipeWalkers + kPipeStateWaves>(a.gp, lds, G * kgroup_bytes<PREC>(a.gp.Mpad));   // both outputs
    __syncthreads();
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    if (w < kPipeWalkers) {
        __builtin_amdgcn_s_setprio(1);
        pipe_walker<PREC, G>(a, w, lane, lds, sy, vred);
    } else
        pipe_state<PREC, G>(a, blockIdx.x, w - kPipeWalkers, lane, lds, sy, vred, pred, ored);
}

namespace {

template <int PREC, int G>
hipError_t launch_pipe_t(const RolloutArgs &a, hipStream_t st) {
    const size_t lds = (size_t)G * kgroup_bytes<PREC>(a.gp.Mpad) + (size_t)2 * a.gp.Mpad * sizeof(float);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(rollout_pipe_kernel<PREC, G>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const dim3 grid((a.K + 32 * G - 1) / (32 * G));
    hipLaunchKernelGGL((rollout_pipe_kernel<PREC, G>), grid, dim3(64 * (kPipeWalkers + kPipeStateWaves)), lds, st, a);
    return hipGetLastError();
}

}  // namespace

bool rollout_pipe_admissible(int precision, int G, int Mpad) {
    return (precision == GPMPPI_BF16 && G == 2 && Mpad == 32 * kPipeNT) ||
           (precision == GPMPPI_BF16X3 && G == 1 && Mpad == 32 * kPipeNT);
}

hipError_t launch_rollout_pipe(const RolloutArgs &a, int precision, int G, hipStream_t st) {
    if (!rollout_pipe_admissible(precision, G, a.gp.Mpad) || a.gp.NT != kPipeNT) return hipErrorInvalidValue;
    return precision == GPMPPI_BF16 ? launch_pipe_t<GPMPPI_BF16, 2>(a, st) : launch_pipe_t<GPMPPI_BF16X3, 1>(a, st);
}

}  // namespace gpmppi
