// MPPI weights and control update (Alg. 1: trajectory weights and the
// weighted sum of the sampled controls), the closed-loop plant step with the
// warm-start shift, and a raw Philox probe.
#include "device_common.hpp"
#include "kernels.hpp"

namespace gpmppi {

constexpr int kUpdThreads = 256;

__device__ __forceinline__ float block_min(float v, float *sh) {
    for (int m = 32; m >= 1; m >>= 1) v = fminf(v, __shfl_xor(v, m, 64));
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    float r = sh[0];
    for (int i = 1; i < kUpdThreads / 64; ++i) r = fminf(r, sh[i]);
    return r;
}

// Fixed-order block sum of up to three values (identical in every block).
__device__ __forceinline__ void block_sum3(float &a, float &b, float &c, float *sh) {
    for (int m = 32; m >= 1; m >>= 1) {
        a += __shfl_xor(a, m, 64);
        b += __shfl_xor(b, m, 64);
        c += __shfl_xor(c, m, 64);
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) {
        sh[3 * w] = a;
        sh[3 * w + 1] = b;
        sh[3 * w + 2] = c;
    }
    __syncthreads();
    a = sh[0];
    b = sh[1];
    c = sh[2];
    for (int i = 1; i < kUpdThreads / 64; ++i) {
        a += sh[3 * i];
        b += sh[3 * i + 1];
        c += sh[3 * i + 2];
    }
}

// Block k computes U'_k = sum_s w^s u_k^s with w^s = exp(-(S^s - rho)/lambda) / Z,
// rho = min S.  Every block evaluates the same fixed-order min and sum, so the
// normaliser is identical everywhere; block 0 also writes the weights.
__device__ __forceinline__ void update_step(const UpdateArgs &a, int k, float *sh) {
    const int tid = threadIdx.x;
    NoiseParams np = a.noise;
    {
        uint64_t seed = a.seed;
        if (a.step_counter) seed += (uint64_t)(*a.step_counter);
        np.key0 = (uint32_t)seed;
        np.key1 = (uint32_t)(seed >> 32);
    }
    const float inv_lam = 1.0f / a.lambda;
    float mn = INFINITY;
    bool bad = false;
    for (int s = tid; s < a.K; s += kUpdThreads) {
        const float c = a.costs[s];
        bad |= !isfinite(c);
        mn = fminf(mn, c);
    }
    mn = block_min(mn, sh);
    const float U0 = a.U[2 * k], U1 = a.U[2 * k + 1];
    float z = 0.0f, n0 = 0.0f, n1 = 0.0f;
    for (int s = tid; s < a.K; s += kUpdThreads) {
        const float e = expf((mn - a.costs[s]) * inv_lam);
        const float2 u = sampled_control(np, k, s, U0, U1);
        z += e;
        n0 = fmaf(e, u.x, n0);
        n1 = fmaf(e, u.y, n1);
    }
    block_sum3(z, n0, n1, sh);
    const float iz = 1.0f / z;
    if (tid == 0) {
        a.U_out[2 * k] = n0 * iz;
        a.U_out[2 * k + 1] = n1 * iz;
    }
    if (k == 0) {
        if (a.weights)
            for (int s = tid; s < a.K; s += kUpdThreads) a.weights[s] = expf((mn - a.costs[s]) * inv_lam) * iz;
        if (bad && a.flags) atomicOr(a.flags, GPMPPI_FLAG_NONFINITE);
    }
}

__global__ __launch_bounds__(kUpdThreads) void update_kernel(UpdateArgs a) {
    __shared__ float sh[3 * kUpdThreads / 64];
    update_step(a, blockIdx.x, sh);
}

// One workgroup per (problem, horizon step) item of a batch.
__global__ __launch_bounds__(kUpdThreads) void update_batch_kernel(const UpdateArgs *probs, const int2 *items) {
    __shared__ float sh[3 * kUpdThreads / 64];
    const int2 pk = items[blockIdx.x];
    const int p = __builtin_amdgcn_readfirstlane(pk.x);
    const int k = __builtin_amdgcn_readfirstlane(pk.y);
    update_step(probs[p], k, sh);
}

hipError_t launch_update_batch(const UpdateArgs *probs_d, const int2 *items_d, int n_items, hipStream_t st) {
    hipLaunchKernelGGL(update_batch_kernel, dim3(n_items), dim3(kUpdThreads), 0, st, probs_d, items_d);
    return hipGetLastError();
}

hipError_t launch_update(const UpdateArgs &a, hipStream_t st) {
    hipLaunchKernelGGL(update_kernel, dim3(a.T), dim3(kUpdThreads), 0, st, a);
    return hipGetLastError();
}

__global__ void philox_kernel(uint32_t k0, uint32_t k1, const uint4 *ctr, int n, uint4 *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = philox4x32_10(ctr[i], k0, k1);
}

hipError_t launch_philox(uint64_t seed, const uint32_t *ctr, int n, uint32_t *out, hipStream_t st) {
    hipLaunchKernelGGL(philox_kernel, dim3((n + 255) / 256), dim3(256), 0, st, (uint32_t)seed,
                       (uint32_t)(seed >> 32), reinterpret_cast<const uint4 *>(ctr), n,
                       reinterpret_cast<uint4 *>(out));
    return hipGetLastError();
}

// Synthetic plant (nominal Euler step plus amplitude * sin(v w) on both
// velocity derivatives) driven by U_0, then the warm-start shift
// U <- [U_1 .. U_{T-1}, U_{T-1}].  One block; T <= 4096.
__device__ __forceinline__ void plant_shift_body(const float *x, float *x_out, float *U, int T, Dyn dy, float amp,
                                                 const uint32_t *step_counter, float *x_hist, float *U0_hist,
                                                 float *xs) {
    const int tid = threadIdx.x;
    const uint32_t t = step_counter ? *step_counter : 0u;
    if (tid == 0) {
        const float X = x[0], Y = x[1], th = x[2], v = x[3], w = x[4];
        const float u0 = U[0], u1 = U[1];
        const float dt = dy.dt;
        const float res = amp * sinf(v * w);
        xs[0] = X + dt * v * cosf(th);
        xs[1] = Y + dt * v * sinf(th);
        xs[2] = th + dt * w;
        xs[3] = v + (dy.dt_tau_v * (u0 - v) + dt * res);
        xs[4] = w + (dy.dt_tau_w * (u1 - w) + dt * res);
        if (U0_hist) {
            U0_hist[2 * t] = u0;
            U0_hist[2 * t + 1] = u1;
        }
    }
    // shift: every thread reads its elements before any thread writes
    float keep[2 * 16];
    int cnt = 0;
    for (int i = tid; i < 2 * T && cnt < 32; i += 256, ++cnt) {
        const int k = i >> 1, c = i & 1;
        const int src = k + 1 < T ? k + 1 : T - 1;
        keep[cnt] = U[2 * src + c];
    }
    __syncthreads();
    cnt = 0;
    for (int i = tid; i < 2 * T && cnt < 32; i += 256, ++cnt) U[i] = keep[cnt];
    if (tid < 5) {
        x_out[tid] = xs[tid];
        if (x_hist) x_hist[(size_t)(t + 1) * 5 + tid] = xs[tid];
    }
}

__global__ __launch_bounds__(256) void plant_shift_kernel(const float *x, float *x_out, float *U, int T, Dyn dy,
                                                          float amp, uint32_t *step_counter, float *x_hist,
                                                          float *U0_hist) {
    __shared__ float xs[5];
    plant_shift_body(x, x_out, U, T, dy, amp, step_counter, x_hist, U0_hist, xs);
    __syncthreads();
    if (threadIdx.x == 0 && step_counter) *step_counter = *step_counter + 1;
}

// Workgroup p: plant step and shift of problem p of a batch; x [n][5], U packed
// with offsets U_off (floats), x_hist [steps + 1][n][5].  The step counter
// is advanced by the separate counter kernel after all problems.
__global__ __launch_bounds__(256) void plant_shift_batch_kernel(float *x, float *U, const long long *U_off,
                                                                const int *T, const Dyn *dyn, float amp,
                                                                const uint32_t *step_counter, float *x_hist,
                                                                int n) {
    __shared__ float xs[5];
    const int p = blockIdx.x;
    const uint32_t t = *step_counter;
    plant_shift_body(x + 5 * p, x + 5 * p, U + U_off[p], T[p], dyn[p], amp, nullptr, nullptr, nullptr, xs);
    __syncthreads();
    if (x_hist && threadIdx.x < 5) x_hist[((size_t)(t + 1) * n + p) * 5 + threadIdx.x] = x[5 * p + threadIdx.x];
}

hipError_t launch_plant_shift_batch(float *x, float *U, const long long *U_off, const int *T, const Dyn *dyn,
                                    float amplitude, const uint32_t *step_counter, float *x_hist, int n,
                                    hipStream_t st) {
    hipLaunchKernelGGL(plant_shift_batch_kernel, dim3(n), dim3(256), 0, st, x, U, U_off, T, dyn, amplitude,
                       step_counter, x_hist, n);
    return hipGetLastError();
}

__global__ void batch_patch_kernel(RolloutArgs *ra, UpdateArgs *ua, int n, BatchPtrs q) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const long long uo = q.U_off[p], ko = q.K_off[p];
    ra[p].x0 = q.x0 + 5 * p;
    ra[p].U = q.U + uo;
    ra[p].costs = q.costs + ko;
    ra[p].seed = q.seed;
    ra[p].step_counter = q.step_counter;
    ua[p].U = q.U + uo;
    ua[p].U_out = q.U_out + uo;
    ua[p].costs = q.costs + ko;
    ua[p].weights = q.weights ? q.weights + ko : nullptr;
    ua[p].seed = q.seed;
    ua[p].step_counter = q.step_counter;
}

hipError_t launch_batch_patch(RolloutArgs *ra, UpdateArgs *ua, int n, BatchPtrs ptrs, hipStream_t st) {
    hipLaunchKernelGGL(batch_patch_kernel, dim3((n + 63) / 64), dim3(64), 0, st, ra, ua, n, ptrs);
    return hipGetLastError();
}

__global__ void counter_add_kernel(uint32_t *c, uint32_t v) {
    if (threadIdx.x == 0) c[0] += v;
}

hipError_t launch_counter_add(uint32_t *counter, uint32_t v, hipStream_t st) {
    hipLaunchKernelGGL(counter_add_kernel, dim3(1), dim3(64), 0, st, counter, v);
    return hipGetLastError();
}

hipError_t launch_plant_shift(const float *x, float *x_out, float *U, int T, Dyn dyn, float amplitude,
                              uint32_t *step_counter, float *x_hist, float *U0_hist, hipStream_t st) {
    hipLaunchKernelGGL(plant_shift_kernel, dim3(1), dim3(256), 0, st, x, x_out, U, T, dyn, amplitude,
                       step_counter, x_hist, U0_hist);
    return hipGetLastError();
}

__global__ void counter_reset_kernel(uint32_t *c) {
    if (threadIdx.x == 0) c[0] = 0u;
}

hipError_t launch_counter_reset(uint32_t *counter, hipStream_t st) {
    hipLaunchKernelGGL(counter_reset_kernel, dim3(1), dim3(64), 0, st, counter);
    return hipGetLastError();
}

}  // namespace gpmppi
