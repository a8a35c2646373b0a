// K-sample x T-step rollout of the GP-augmented chance-constrained MPPI
// controller on gfx950 (Alg. 1 Step 1 with Eqs. 1-3, 10, 11-16).
//
// Work decomposition: one workgroup of 256 threads (4 wave64s) owns 32
// samples.  Thread t serves sample s = t / 8 with sub-lane r = t % 8; the 8
// lanes of a sample hold identical copies of its state x (5) and covariance
// Sigma (15 symmetric entries) in registers for the whole horizon and split
// the sample's loops (kernel vector chunks, polyline segments, obstacles).
//
// Per step and per GP output o:
//  1. kernel vector: k_oj = exp2(c2_o - |q s_o - zs_oj|^2) for the 32 samples
//     of the block and every training point j (VALU exp), written to LDS in
//     the matrix-core operand layout; the GP mean k^T alpha is summed in FP32.
//  2. variance: v = W k with W = L^-1 lower triangular, on the matrix cores:
//     each wave walks its share of the 32x32 blocks (t, jt <= t) of W,
//     streaming W from L2 through a register ring and reading k from LDS,
//     and sums |v|^2 per sample; s2 = sn^2 + max(0, sf^2 - |v|^2).
//  3. per-sample Euler step, covariance A Sigma A^T + dt^2 diag(0,0,0,s2),
//     lane/obstacle tightening and the stage cost.
#include "device_common.hpp"
#include "kernels.hpp"

namespace gpmppi {

// ---------------------------------------------------------------- W blocks
// Packed block (t, jt) of W (rows 32t.., columns 32jt..), index
// b = t (t + 1) / 2 + jt, lane l of a wave:
//   FP32: float4 [b][q][l], component c: W[32t + l%32][32jt + 2(4q+c) + l/32]
//   BF16: uint4  [b][h][l], element e:   W[32t + l%32][32jt + 16h + 8(l/32) + e]
// The LDS operand holds k in the same lane order with the sample s = l % 32
// in place of the W row.
template <int PREC>
struct WBlock;
template <>
struct WBlock<GPMPPI_FP32> {
    float4 v[4];
};
template <>
struct WBlock<GPMPPI_BF16> {
    uint4 h[2];
};
template <>
struct WBlock<GPMPPI_BF16X3> {
    uint4 h[2];
    uint4 l[2];
};

template <int PREC>
__device__ __forceinline__ void load_wblock(WBlock<PREC> &b, const GpDev &g, int o, int blk, int lane) {
    if constexpr (PREC == GPMPPI_FP32) {
        const float4 *p = g.w32 + o * g.w32_stride + (size_t)blk * 256 + lane;
        b.v[0] = p[0];
        b.v[1] = p[64];
        b.v[2] = p[128];
        b.v[3] = p[192];
    } else {
        const uint4 *p = g.wbh + o * g.wb_stride + (size_t)blk * 128 + lane;
        b.h[0] = p[0];
        b.h[1] = p[64];
        if constexpr (PREC == GPMPPI_BF16X3) {
            const uint4 *q = g.wbl + o * g.wb_stride + (size_t)blk * 128 + lane;
            b.l[0] = q[0];
            b.l[1] = q[64];
        }
    }
}

__device__ __forceinline__ v8bf as_bf(uint4 u) {
    v8bf r;
    __builtin_memcpy(&r, &u, 16);
    return r;
}

template <int PREC>
__device__ __forceinline__ void mma_block(v16f &acc, const WBlock<PREC> &b, const unsigned char *lds,
                                          int jt, int lane, int Mpad) {
    if constexpr (PREC == GPMPPI_FP32) {
        const float4 *K = reinterpret_cast<const float4 *>(lds) + (size_t)jt * 256 + lane;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float4 kq = K[q * 64];
            const float4 wq = b.v[q];
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(wq.x, kq.x, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(wq.y, kq.y, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(wq.z, kq.z, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(wq.w, kq.w, acc, 0, 0, 0);
        }
    } else {
        const uint4 *Kh = reinterpret_cast<const uint4 *>(lds) + (size_t)jt * 128 + lane;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint4 kh = Kh[h * 64];
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf(b.h[h]), as_bf(kh), acc, 0, 0, 0);
            if constexpr (PREC == GPMPPI_BF16X3) {
                const uint4 *Kl = reinterpret_cast<const uint4 *>(lds + (size_t)Mpad * 64) +
                                  (size_t)jt * 128 + lane;
                const uint4 kl = Kl[h * 64];
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf(b.h[h]), as_bf(kl), acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf(b.l[h]), as_bf(kh), acc, 0, 0, 0);
            }
        }
    }
}

size_t rollout_lds_bytes(int precision, int Mpad) {
    const size_t per = (precision == GPMPPI_FP32) ? 4 : (precision == GPMPPI_BF16 ? 2 : 4);
    return (size_t)Mpad * kSamplesPerBlock * per;
}

// Tile list of a wave: round i holds tiles 4i .. 4i+3, assigned in snake
// order so that the sum of tile heights (t + 1) is balanced across waves.
__device__ __forceinline__ int wave_tile(int w, int i) { return (i & 1) ? 4 * i + 3 - w : 4 * i + w; }

constexpr int ring_depth(int prec) { return prec == GPMPPI_FP32 ? 4 : 8; }

// One GP output for the 32 samples of the block.  Must be called by all 256
// threads.  qs: this thread's sample query scaled by s_o.  Returns the GP
// mean and the predictive variance of that sample (identical on its 8 lanes).
template <int PREC>
__device__ __forceinline__ void gp_output(const GpDev &g, int o, const float qs[4], int s, int r,
                                          unsigned char *lds, float *red, float &mean_out,
                                          float &var_out) {
    const int Mpad = g.Mpad;
    const int nchunk = Mpad >> 3;
    const float4 *zs = reinterpret_cast<const float4 *>(g.zs) + (size_t)o * Mpad;
    const float *al = g.alpha + (size_t)o * Mpad;
    const float c2 = g.c2[o];
    float msum = 0.0f;
    for (int c = r; c < nchunk; c += kLanesPerSample) {
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
        const float4 a0 = *reinterpret_cast<const float4 *>(al + 8 * c);
        const float4 a1 = *reinterpret_cast<const float4 *>(al + 8 * c + 4);
        msum = fmaf(kv[0], a0.x, msum);
        msum = fmaf(kv[1], a0.y, msum);
        msum = fmaf(kv[2], a0.z, msum);
        msum = fmaf(kv[3], a0.w, msum);
        msum = fmaf(kv[4], a1.x, msum);
        msum = fmaf(kv[5], a1.y, msum);
        msum = fmaf(kv[6], a1.z, msum);
        msum = fmaf(kv[7], a1.w, msum);
        if constexpr (PREC == GPMPPI_FP32) {
            float4 *K = reinterpret_cast<float4 *>(lds) + (size_t)c * 64;
            K[s] = make_float4(kv[0], kv[2], kv[4], kv[6]);
            K[32 + s] = make_float4(kv[1], kv[3], kv[5], kv[7]);
        } else {
            uint16_t hb[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) hb[e] = bf16_rne(kv[e]);
            uint4 hv;
            hv.x = (uint32_t)hb[0] | ((uint32_t)hb[1] << 16);
            hv.y = (uint32_t)hb[2] | ((uint32_t)hb[3] << 16);
            hv.z = (uint32_t)hb[4] | ((uint32_t)hb[5] << 16);
            hv.w = (uint32_t)hb[6] | ((uint32_t)hb[7] << 16);
            const int idx = (c >> 1) * 64 + s + 32 * (c & 1);
            reinterpret_cast<uint4 *>(lds)[idx] = hv;
            if constexpr (PREC == GPMPPI_BF16X3) {
                uint16_t lb[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) lb[e] = bf16_rne(kv[e] - bf16_to_f32(hb[e]));
                uint4 lv;
                lv.x = (uint32_t)lb[0] | ((uint32_t)lb[1] << 16);
                lv.y = (uint32_t)lb[2] | ((uint32_t)lb[3] << 16);
                lv.z = (uint32_t)lb[4] | ((uint32_t)lb[5] << 16);
                lv.w = (uint32_t)lb[6] | ((uint32_t)lb[7] << 16);
                reinterpret_cast<uint4 *>(lds + (size_t)Mpad * 64)[idx] = lv;
            }
        }
    }
    msum += shfl_xor(msum, 1);
    msum += shfl_xor(msum, 2);
    msum += shfl_xor(msum, 4);
    __syncthreads();

    // ---- variance contraction on the matrix cores
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int NT = g.NT;
    const int rounds = (NT + 3) >> 2;
    int ntiles = rounds;
    if (wave_tile(w, rounds - 1) >= NT) ntiles = rounds - 1;
    int nsteps = 0;
    for (int i = 0; i < ntiles; ++i) nsteps += wave_tile(w, i) + 1;

    constexpr int D = ring_depth(PREC);
    WBlock<PREC> ring[D];
    int pi = 0, pjt = 0;   // prefetch position (tile list index, column block)
#pragma unroll
    for (int u = 0; u < D; ++u) {
        if (u < nsteps) {
            const int t = wave_tile(w, pi);
            load_wblock<PREC>(ring[u], g, o, t * (t + 1) / 2 + pjt, lane);
            if (++pjt > t) {
                ++pi;
                pjt = 0;
            }
        }
    }
    v16f acc = {};
    float sq = 0.0f;
    int ci = 0, cjt = 0;
    int ct = wave_tile(w, 0);
    for (int base = 0; base < nsteps; base += D) {
#pragma unroll
        for (int u = 0; u < D; ++u) {
            if (base + u < nsteps) {
                const WBlock<PREC> cur = ring[u];
                if (base + u + D < nsteps) {
                    const int t = wave_tile(w, pi);
                    load_wblock<PREC>(ring[u], g, o, t * (t + 1) / 2 + pjt, lane);
                    if (++pjt > t) {
                        ++pi;
                        pjt = 0;
                    }
                }
                mma_block<PREC>(acc, cur, lds, cjt, lane, Mpad);
                if (++cjt > ct) {
#pragma unroll
                    for (int e = 0; e < 16; ++e) sq = fmaf(acc[e], acc[e], sq);
                    acc = v16f{};
                    ++ci;
                    cjt = 0;
                    ct = wave_tile(w, ci);
                }
            }
        }
    }
    sq += shfl_xor(sq, 32);
    if (lane < 32) red[w * 32 + lane] = sq;
    __syncthreads();
    const float v2 = (red[s] + red[32 + s]) + (red[64 + s] + red[96 + s]);
    var_out = g.sn2[o] + fmaxf(0.0f, g.sf2[o] - v2);
    mean_out = msum;
}

__device__ __forceinline__ float min8(float v) {
    v = fminf(v, shfl_xor(v, 1));
    v = fminf(v, shfl_xor(v, 2));
    v = fminf(v, shfl_xor(v, 4));
    return v;
}

template <int PREC>
__global__ __launch_bounds__(kThreads) void rollout_kernel(RolloutArgs a) {
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ float red[kWaves * 32];
    const int tid = threadIdx.x;
    const int s = tid / kLanesPerSample, r = tid % kLanesPerSample;
    const int sg = blockIdx.x * kSamplesPerBlock + s;
    const bool valid = sg < a.K;
    const bool writer = valid && r == 0;
    const int K = a.K;

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

    float X = a.x0[0], Y = a.x0[1], th = a.x0[2], v = a.x0[3], w = a.x0[4];
    // Sigma (symmetric), Sigma(0) = 0
    float p00 = 0, p01 = 0, p02 = 0, p03 = 0, p04 = 0, p11 = 0, p12 = 0, p13 = 0, p14 = 0, p22 = 0,
          p23 = 0, p24 = 0, p33 = 0, p34 = 0, p44 = 0;
    float S = 0.0f, Sc = 0.0f, disc = 1.0f;

    if (writer && a.trace.x_d) {
        a.trace.x_d[0 * K + sg] = X;
        a.trace.x_d[1 * K + sg] = Y;
        a.trace.x_d[2 * K + sg] = th;
        a.trace.x_d[3 * K + sg] = v;
        a.trace.x_d[4 * K + sg] = w;
    }
    if (writer && a.trace.sxy_d) {
        a.trace.sxy_d[0 * K + sg] = 0.0f;
        a.trace.sxy_d[1 * K + sg] = 0.0f;
        a.trace.sxy_d[2 * K + sg] = 0.0f;
    }

    for (int k = 0; k < a.T; ++k) {
        const float2 u = sampled_control(np, k, sg, a.U[2 * k], a.U[2 * k + 1]);
        const float q[4] = {v, w, u.x, u.y};
        float m[2], s2[2];
#pragma unroll
        for (int o = 0; o < 2; ++o) {
            const float qs[4] = {q[0] * a.gp.scale[o][0], q[1] * a.gp.scale[o][1], q[2] * a.gp.scale[o][2],
                                 q[3] * a.gp.scale[o][3]};
            gp_output<PREC>(a.gp, o, qs, s, r, lds, red, m[o], s2[o]);
        }

        // ---- mean: explicit Euler of the dynamic unicycle plus the GP residual (Eqs. 1, 2, 10)
        float sth, cth;
        sincosf(th, &sth, &cth);
        const float dt = dy.dt;
        const float a02 = -dt * v * sth, a03 = dt * cth, a12 = dt * v * cth, a13 = dt * sth, a24 = dt;
        const float a33 = dy.a33, a44 = dy.a44;
        const float Xn = X + dt * v * cth;
        const float Yn = Y + dt * v * sth;
        const float thn = th + dt * w;
        const float vn = v + (dy.dt_tau_v * (u.x - v) + dt * m[0]);
        const float wn = w + (dy.dt_tau_w * (u.y - w) + dt * m[1]);

        // ---- covariance: Sigma+ = A Sigma A^T + dt^2 diag(0, 0, 0, s2_v, s2_w) (Eq. 10)
        // B = A Sigma (rows), then Sigma+_ij = sum_n B_in A_jn for i <= j.
        const float b00 = p00 + a02 * p02 + a03 * p03, b01 = p01 + a02 * p12 + a03 * p13,
                    b02 = p02 + a02 * p22 + a03 * p23, b03 = p03 + a02 * p23 + a03 * p33,
                    b04 = p04 + a02 * p24 + a03 * p34;
        const float b11 = p11 + a12 * p12 + a13 * p13, b12 = p12 + a12 * p22 + a13 * p23,
                    b13 = p13 + a12 * p23 + a13 * p33, b14 = p14 + a12 * p24 + a13 * p34;
        const float b10 = p01 + a12 * p02 + a13 * p03;
        const float b22 = p22 + a24 * p24, b23 = p23 + a24 * p34, b24 = p24 + a24 * p44;
        const float b20 = p02 + a24 * p04, b21 = p12 + a24 * p14;
        const float b33 = a33 * p33, b34 = a33 * p34;
        const float b44 = a44 * p44;
        (void)b20;
        (void)b21;
        (void)b10;
        const float n00 = b00 + a02 * b02 + a03 * b03;
        const float n01 = b01 + a12 * b02 + a13 * b03;
        const float n02 = b02 + a24 * b04;
        const float n03 = a33 * b03;
        const float n04 = a44 * b04;
        const float n11 = b11 + a12 * b12 + a13 * b13;
        const float n12 = b12 + a24 * b14;
        const float n13 = a33 * b13;
        const float n14 = a44 * b14;
        const float n22 = b22 + a24 * b24;
        const float n23 = a33 * b23;
        const float n24 = a44 * b24;
        const float n33 = a33 * b33 + dt * dt * s2[0];
        const float n34 = a44 * b34;
        const float n44 = a44 * b44 + dt * dt * s2[1];
        p00 = n00; p01 = n01; p02 = n02; p03 = n03; p04 = n04;
        p11 = n11; p12 = n12; p13 = n13; p14 = n14;
        p22 = n22; p23 = n23; p24 = n24;
        p33 = n33; p34 = n34; p44 = n44;
        X = Xn; Y = Yn; th = thn; v = vn; w = wn;

        // ---- chance constraints at (x_{k+1}, Sigma_{k+1}) (Eqs. 13-16)
        const float sa = p00, sb = p01, sc = p11;
        const float hh = 0.5f * (sa - sc);
        const float lmax = 0.5f * (sa + sc) + sqrtf(hh * hh + sb * sb);
        float dl;
        if (geo.path_kind == 0) {
            const float dx = X - geo.cx, dyy = Y - geo.cy;
            dl = fabsf(sqrtf(dx * dx + dyy * dyy) - geo.R);
        } else {
            float best = INFINITY;
            for (int i = r; i < geo.P; i += kLanesPerSample) {
                const float4 sgm = geo.seg[i];
                const float rx = X - sgm.x, ry = Y - sgm.y;
                float t = (rx * sgm.z + ry * sgm.w) * geo.seg_inv[i];
                t = fminf(fmaxf(t, 0.0f), 1.0f);
                const float ex = rx - t * sgm.z, ey = ry - t * sgm.w;
                best = fminf(best, ex * ex + ey * ey);
            }
            dl = sqrtf(min8(best));
        }
        const float rbar = geo.half_width - geo.c_p * sqrtf(fmaxf(lmax, 0.0f));
        float om = INFINITY;
        for (int j = r; j < geo.n_obs; j += kLanesPerSample) {
            const float4 ob = geo.obs[j];
            const float dx = X - ob.x, dyy = Y - ob.y;
            const float rho2 = dx * dx + dyy * dyy;
            const float rho = sqrtf(rho2);
            const float vn_dir = rho > 0.0f ? (sa * dx * dx + 2.0f * sb * dx * dyy + sc * dyy * dyy) / rho2 : lmax;
            om = fminf(om, (rho - ob.z) - geo.z_p * sqrtf(fmaxf(vn_dir, 0.0f)));
        }
        om = min8(om);

        // ---- stage cost (Eqs. 11-12 terms), Kahan-compensated sum (Eq. 5)
        const float dv = cw.v_des - v;
        float c = cw.w_var * (s2[0] + s2[1]) + cw.w_dev * (dl * geo.inv_half_width) + cw.w_speed * (dv * dv);
        if (dl > rbar) c += cw.w_lane * disc;
        if (om <= 0.0f) c += cw.w_obs;
        {
            const float yk = c - Sc;
            const float tk = S + yk;
            Sc = (tk - S) - yk;
            S = tk;
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
                xd[4 * K + sg] = w;
            }
            if (tr.sxy_d) {
                float *sd = tr.sxy_d + (kk + 1) * 3 * K;
                sd[0 * K + sg] = sa;
                sd[1 * K + sg] = sb;
                sd[2 * K + sg] = sc;
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
    if (writer) a.costs[sg] = S;
}

template <int PREC>
__global__ __launch_bounds__(kThreads) void gp_predict_kernel(GpDev g, const float *q, int n, float *mean,
                                                              float *var) {
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ float red[kWaves * 32];
    const int tid = threadIdx.x;
    const int s = tid / kLanesPerSample, r = tid % kLanesPerSample;
    const int sg = blockIdx.x * kSamplesPerBlock + s;
    const int sl = sg < n ? sg : n - 1;
    const float4 qq = reinterpret_cast<const float4 *>(q)[sl];
    const float qv[4] = {qq.x, qq.y, qq.z, qq.w};
#pragma unroll
    for (int o = 0; o < 2; ++o) {
        const float qs[4] = {qv[0] * g.scale[o][0], qv[1] * g.scale[o][1], qv[2] * g.scale[o][2],
                             qv[3] * g.scale[o][3]};
        float m, s2;
        gp_output<PREC>(g, o, qs, s, r, lds, red, m, s2);
        if (sg < n && r == 0) {
            mean[(size_t)o * n + sg] = m;
            var[(size_t)o * n + sg] = s2;
        }
    }
}

template <typename F>
static hipError_t set_lds(F *fn, size_t bytes) {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_rollout(const RolloutArgs &a, int precision, hipStream_t st) {
    const size_t lds = rollout_lds_bytes(precision, a.gp.Mpad);
    const dim3 grid((a.K + kSamplesPerBlock - 1) / kSamplesPerBlock);
    hipError_t e;
    switch (precision) {
        case GPMPPI_FP32:
            if ((e = set_lds(rollout_kernel<GPMPPI_FP32>, lds)) != hipSuccess) return e;
            hipLaunchKernelGGL(rollout_kernel<GPMPPI_FP32>, grid, dim3(kThreads), lds, st, a);
            break;
        case GPMPPI_BF16:
            if ((e = set_lds(rollout_kernel<GPMPPI_BF16>, lds)) != hipSuccess) return e;
            hipLaunchKernelGGL(rollout_kernel<GPMPPI_BF16>, grid, dim3(kThreads), lds, st, a);
            break;
        default:
            if ((e = set_lds(rollout_kernel<GPMPPI_BF16X3>, lds)) != hipSuccess) return e;
            hipLaunchKernelGGL(rollout_kernel<GPMPPI_BF16X3>, grid, dim3(kThreads), lds, st, a);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_gp_predict(const GpDev &g, int precision, const float *q, int n, float *mean, float *var,
                             hipStream_t st) {
    const size_t lds = rollout_lds_bytes(precision, g.Mpad);
    const dim3 grid((n + kSamplesPerBlock - 1) / kSamplesPerBlock);
    hipError_t e;
    switch (precision) {
        case GPMPPI_FP32:
            if ((e = set_lds(gp_predict_kernel<GPMPPI_FP32>, lds)) != hipSuccess) return e;
            hipLaunchKernelGGL(gp_predict_kernel<GPMPPI_FP32>, grid, dim3(kThreads), lds, st, g, q, n, mean, var);
            break;
        case GPMPPI_BF16:
            if ((e = set_lds(gp_predict_kernel<GPMPPI_BF16>, lds)) != hipSuccess) return e;
            hipLaunchKernelGGL(gp_predict_kernel<GPMPPI_BF16>, grid, dim3(kThreads), lds, st, g, q, n, mean, var);
            break;
        default:
            if ((e = set_lds(gp_predict_kernel<GPMPPI_BF16X3>, lds)) != hipSuccess) return e;
            hipLaunchKernelGGL(gp_predict_kernel<GPMPPI_BF16X3>, grid, dim3(kThreads), lds, st, g, q, n, mean, var);
            break;
    }
    return hipGetLastError();
}

}  // namespace gpmppi
