// Kernel argument blocks and host-side launchers of the GP-MPPI library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gpmppi.h"
#include "device_common.hpp"

namespace gpmppi {

// Device image of the two residual GPs, packed for the rollout.
//  zs     [2][Mpad][4]  inputs scaled by s_od = sqrt(log2(e)/2) / ell_od, so that
//                       k = exp2(c2_o - |q s_o - zs|^2) = sf_o^2 exp(-r^2/2)
//  alpha  [2][Mpad]     (K + sn^2 I)^-1 y, zero beyond M
//  w32    packed FP32 blocks of W = L^-1 (see pack layout in gp_build.hip)
//  wbh/wbl packed BF16 hi / lo splits of the same blocks
//  zop    BF16 A operands of the kernel-vector exponent products (BF16 forms)
struct GpDev {
    const float *zs;
    const float *alpha;
    const float4 *w32;
    const uint4 *wbh;
    const uint4 *wbl;
    const uint4 *zop;       // BF16 A operands of the exponent products [2][NT][2][64] (see pack_zop_kernel)
    long long w32_stride;   // float4 per output
    long long wb_stride;    // uint4 per output
    long long zop_stride;   // uint4 per output (NT * 128)
    float scale[2][4];
    float c2[2];
    float sf2[2];
    float sn2[2];
    float vscale[2];        // sum_i w_i^2 of a terrain ensemble (1 for a single terrain)
    int Mpad;
    int NT;                 // Mpad / 32
};

struct Geometry {
    int path_kind;          // 0 circle, 1 polyline
    float cx, cy, R;
    int P;
    const float4 *seg;      // [P] (ax, ay, ex, ey), e = b - a
    const float *seg_inv;   // [P] 1 / |e|^2
    float half_width, inv_half_width;
    int n_obs;
    const float4 *obs;      // [n_obs] (cx, cy, r, 0)
    float z_p, c_p;         // Phi^-1(p_x), sqrt(chi2_2(p_x))
};

struct CostWeights {
    float w_var, w_dev, w_lane, w_speed, w_obs, v_des, discount;
    float w_goal, w_term, goal_x, goal_y, goal_tol;
};

struct Dyn {
    float dt, dt_tau_v, dt_tau_w;   // dt, dt/tau_v, dt/tau_w
    float a33, a44;                 // 1 - dt/tau_v, 1 - dt/tau_w
};

struct RolloutArgs {
    GpDev gp;
    Geometry geo;
    CostWeights cw;
    Dyn dyn;
    NoiseParams noise;              // key words are the base seed's
    uint64_t seed;
    const uint32_t *step_counter;   // if non-NULL, seed + *step_counter keys the noise
    int K, T;
    int rotate;                     // start each block's walk over W at a block-dependent pair
    const float *x0;                // [5]
    const float *U;                 // [T][2]
    float *costs;                   // [K]
    const float *tight_sxy;         // [T+1][3] Sigma_XY along the nominal sequence, or NULL (per sample)
    gpmppi_trace trace;
    // output split (two workgroups per sample block): exchange records
    // [nblk][4 slots][4 kinds][32 samples] of (value, tag) and the launch epoch
    // and finished-workgroup count [2]; see rollout_block_split
    unsigned long long *xrec;
    uint32_t *xep;
    int xspin;                      // polls per exchange wait before it gives up; < 0: give up at once
    uint32_t *flags;                // context status word: GPMPPI_FLAG_EXCHANGE_TIMEOUT is set here
    uint32_t *repair;               // [nblk] split launches: blocks whose exchange gave up, recomputed and
                                    // cleared by the repair launch that follows (all 0 between launches)
};

struct UpdateArgs {
    NoiseParams noise;
    uint64_t seed;
    const uint32_t *step_counter;
    int K, T;
    float lambda;
    const float *costs;
    const float *U;
    float *U_out;
    float *weights;
    uint32_t *flags;
};

size_t rollout_lds_bytes(int precision, int G, int Mpad);
// largest sample-group count whose LDS plan fits a compute unit (1 or 2)
int rollout_groups(int precision, int Mpad);
// G sample groups of 32 per workgroup (<= rollout_groups), NW wave64s per workgroup (4 or 8; 12: the
// wave-specialised rollout, where rollout_pipe_admissible).
// split = 1: each sample block's two GP outputs on two workgroups (G = 1 only; a.xrec, a.xep, a.repair
// set), then a repair launch of the unsplit kernel for blocks whose exchange gave up;
// hipErrorCooperativeLaunchTooLarge if the doubled grid cannot be resident at once.
hipError_t launch_rollout(const RolloutArgs &a, int precision, int G, int NW, int split, hipStream_t st);
// Largest sample count whose split launch at this shape can be resident at once (0: not admissible).
int rollout_split_capacity(int precision, int Mpad, int NW);
// Wave-specialised rollout (twelve waves: eight walk W, four generate the kernel vectors and carry
// the sample state): the BF16 forms at Mpad = 1024 with the largest group count only.
constexpr int kPipeWaves = 12;
bool rollout_pipe_admissible(int precision, int G, int Mpad);
hipError_t launch_rollout_pipe(const RolloutArgs &a, int precision, int G, hipStream_t st);
constexpr int kXchRecPerBlock = 4 * 4 * 32;   // exchange records per sample block
constexpr int kXchSpin = 1 << 18;               // default polls of an exchange wait (~0.3 s)
hipError_t launch_rollout_batch(const RolloutArgs *probs_d, const int2 *items_d, int n_items, uint32_t *counter,
                                int precision, int G, int NW, int Mpad_max, int grid, hipStream_t st);
hipError_t launch_update_batch(const UpdateArgs *probs_d, const int2 *items_d, int n_items, hipStream_t st);
hipError_t launch_plant_shift_batch(float *x, float *U, const long long *U_off, const int *T, const Dyn *dyn,
                                    float amplitude, const uint32_t *step_counter, float *x_hist, int n,
                                    hipStream_t st);
hipError_t launch_counter_add(uint32_t *counter, uint32_t v, hipStream_t st);

// Pointers of one batched call, patched into the per-problem argument tables
// on the device (problem p: x0 + 5p, U + U_off[p], costs + K_off[p], ...).
struct BatchPtrs {
    const float *x0;
    const float *U;
    float *U_out;
    float *costs;
    float *weights;        // may be NULL
    uint64_t seed;
    const uint32_t *step_counter;   // may be NULL
    const long long *U_off;
    const long long *K_off;
};
hipError_t launch_batch_patch(RolloutArgs *ra, UpdateArgs *ua, int n, BatchPtrs ptrs, hipStream_t st);
hipError_t launch_gp_predict(const GpDev &g, int precision, const float *q, int n, float *mean,
                             float *var, hipStream_t st);
hipError_t launch_update(const UpdateArgs &a, hipStream_t st);
hipError_t launch_philox(uint64_t seed, const uint32_t *ctr, int n, uint32_t *out, hipStream_t st);
hipError_t launch_plant_shift(const float *x, float *x_out, float *U, int T, Dyn dyn, float amplitude,
                              uint32_t *step_counter, float *x_hist, float *U0_hist, hipStream_t st);
hipError_t launch_counter_reset(uint32_t *counter, hipStream_t st);

// FP64 GP build on the device (per output).
struct GpBuildBuffers {
    double *A;        // [Mpad][Mpad] K + sn^2 I, overwritten by L (lower)
    double *W;        // [Mpad][Mpad] L^-1
    double *Z;        // [M][4]
    double *y;        // [Mpad]
    double *u;        // [Mpad] scratch
    double *alpha;    // [Mpad]
    uint32_t *flag;   // non-PD flag
};
hipError_t build_gp_output(const GpBuildBuffers &b, int M, int Mpad, const double ell[4], double sf2,
                           double sn2, hipStream_t st);
struct TerrainWeights {
    double w[8];
};
// alpha_bar = sum_i w_i alpha_i (FP64 alpha_terr [n_terr][Mpad] of one output),
// written to out64 and, in FP32, to alpha32 [Mpad].
hipError_t combine_alpha(const double *alpha_terr, int n_terr, int Mpad, TerrainWeights w, double *out64,
                         float *alpha32, hipStream_t st);
hipError_t launch_terrain_means(const float *q, int n, const GpDev &g, const double *alpha_terr, int n_terr,
                                float *out, hipStream_t st);
// Differentiation form (the adjoint rollout and its reductions).
struct GradArgs {
    GpDev gp;
    Geometry geo;
    CostWeights cw;
    Dyn dyn;
    NoiseParams noise;
    int K, T, C, nck;
    float inv_tau, inv_K;
    const float4 *q32;       // dense packed Q per output
    long long q_stride;      // float4 per output
    const float *x0;         // [5]
    const float *U;          // [T][2]
    float *costs;            // [K] smoothed costs
    float *ckpt;             // [nck][20][K]
    float *seg;              // [nwg][C + 1][28][32] per-workgroup segment scratch
    float *R;                // [2][T K][Mpad]
    float *Gw;               // [2][T K]
    double *bpart;           // [nwg][2][Mpad]
    double *hpart;           // [nwg][10]
    float *upart;            // [nwg][T][2]
    // output split (two workgroups per 32 samples, one per GP output): ckpt holds [2 roles]
    // and seg [nwg][2 roles] copies; xrec [nwg][kGradXchPerBlock] exchange records, zeroed
    // with repair [nwg] before each split launch; repair marks blocks for the repair launch
    int split;
    unsigned long long *xrec;
    uint32_t *repair;
    int xspin;               // polls per exchange wait before it gives up; < 0: give up at once
    uint32_t *flags;         // context status word (GPMPPI_FLAG_EXCHANGE_TIMEOUT)
};

struct GradLaunch {
    int nwg;                 // grad_kernel workgroups = ceil(K / 32)
    int npairs, nsplit;      // grad_syrk_kernel grid: 128-blocks (bi <= bj) x row splits
    int nbterm;              // grad_bterm_kernel blocks per output
    double *ppart, *bterm;   // partial contractions
    float *J, *dU, *dlog_ell, *dlog_sf;   // outputs
};
// Dynamic LDS of grad_kernel at this Mpad (must be <= 160 KB minus its static LDS).
size_t grad_lds(int Mpad);
constexpr int kGradXchPerBlock = 2 * 4 * 4 * kSamplesPerBlock;   // split exchange records per block
// Workgroups of the split gradient kernel resident at once (a split launch needs 2 nwg).
int grad_split_capacity(int Mpad);
hipError_t launch_grad(const GradArgs &a, const GradLaunch &l, hipStream_t st);

// Q = A^-1 = W^T W packed dense (FP32 operand order); overwrites b.A.
hipError_t pack_q(const GpBuildBuffers &b, int M, int Mpad, float4 *q32, hipStream_t st);
hipError_t alpha_for_targets(const GpBuildBuffers &b, int Mpad, const double *y_d, double *alpha_d, hipStream_t st);
hipError_t pack_gp_output(const GpBuildBuffers &b, int M, int Mpad, const double scale[4], double c2, uint4 *zop, float *zs,
                          float *alpha, float *zs2, float *cz, float4 *w32, uint4 *wbh, uint4 *wbl,
                          hipStream_t st);

}  // namespace gpmppi
