// Device helpers shared by the gfx950 kernels of the GP-MPPI library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gpmppi {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
// read-only kernel data at wave-uniform addresses: loads through the scalar cache
typedef const __attribute__((address_space(4))) v4f *const_v4p;
typedef const __attribute__((address_space(4))) float *const_fp;

constexpr int kSamplesPerBlock = 32;   // samples per workgroup (one MFMA column block)
constexpr int kThreads = 256;          // 4 wave64s
constexpr int kWaves = kThreads / 64;
constexpr int kLanesPerSample = kThreads / kSamplesPerBlock;   // 8
constexpr int kTile = 32;              // rows of W per MFMA tile
constexpr int kMaxM = 1024;

// Exchange records between the two workgroups of a split sample block: 64-bit
// (tag, value) words, one per sample, stored and loaded at agent scope
// (coherent across the XCDs' L2s).  A record is valid once its tag is the one
// the reader expects, so the writer needs no flag, fence or wait.
// Lanes 0..31 of the calling wave publish their sample's value.
__device__ __forceinline__ void xch_put(unsigned long long *rec, int lane, float val, uint32_t tag) {
    if (lane < 32) {
        const unsigned long long r = ((unsigned long long)tag << 32) | __float_as_uint(val);
        __hip_atomic_store(rec + lane, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Every lane of the calling wave waits, for at most spin polls, for the record
// of sample lane % 32 with this tag and returns its value (NaN once a wait of
// this wave has timed out, and broken is set; spin < 0 gives up at once).
__device__ __forceinline__ float xch_get(const unsigned long long *rec, int lane, uint32_t tag, int spin,
                                         bool &broken) {
    if (spin < 0) broken = true;
    if (broken) return __builtin_nanf("");
    unsigned long long r = 0;
    for (int n = 0;; ++n) {
        r = __hip_atomic_load(rec + (lane & 31), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (__all((uint32_t)(r >> 32) == tag)) break;
        if (n == spin) {
            broken = true;
            return __builtin_nanf("");
        }
        __builtin_amdgcn_s_sleep(2);
    }
    return __uint_as_float((uint32_t)r);
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32
// multiplies whose high halves are mixed with the other words and the key;
// the key advances by two Weyl constants between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
    const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t hi0 = __umulhi(m0, c.x), lo0 = m0 * c.x;
        const uint32_t hi1 = __umulhi(m1, c.z), lo1 = m1 * c.z;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    }
    return c;
}

// Open-interval uniform ((w >> 9) + 1/2) 2^-23: a multiple of 2^-24 below 1,
// hence exact in binary32.
__device__ __forceinline__ float uniform_open(uint32_t w) {
    return ((float)(w >> 9) + 0.5f) * 0x1p-23f;
}

// Clipped sampled control u = clip(U_k + eps) for step k of sample s
// (Alg. 1 Step 1 noise with Box-Muller normals; Eq. 8 box).
struct NoiseParams {
    uint32_t key0, key1;
    uint32_t pid;
    float sig_v, sig_w;
    float umin0, umin1, umax0, umax1;
};

// U_k + eps_k^s before the clip.
__device__ __forceinline__ float2 sampled_raw(const NoiseParams &np, int k, int s, float U0, float U1) {
    const uint4 w = philox4x32_10(make_uint4((uint32_t)k, (uint32_t)s, np.pid, 0u), np.key0, np.key1);
    const float u1 = uniform_open(w.x), u2 = uniform_open(w.y);
    const float r = sqrtf(-2.0f * logf(u1));
    float sn, cs;
    sincospif(2.0f * u2, &sn, &cs);
    return make_float2(U0 + np.sig_v * (r * cs), U1 + np.sig_w * (r * sn));
}

__device__ __forceinline__ float2 sampled_control(const NoiseParams &np, int k, int s, float U0,
                                                  float U1) {
    const float2 raw = sampled_raw(np, k, s, U0, U1);
    return make_float2(fminf(fmaxf(raw.x, np.umin0), np.umax0), fminf(fmaxf(raw.y, np.umin1), np.umax1));
}

// Round-to-nearest-even float -> bfloat16 bits (finite inputs).
__device__ __host__ __forceinline__ uint16_t bf16_rne(float x) {
    uint32_t b;
    __builtin_memcpy(&b, &x, 4);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

__device__ __host__ __forceinline__ float bf16_to_f32(uint16_t h) {
    const uint32_t b = (uint32_t)h << 16;
    float x;
    __builtin_memcpy(&x, &b, 4);
    return x;
}

// Wave-level helpers (wave64).
__device__ __forceinline__ float shfl_xor(float v, int m) { return __shfl_xor(v, m, 64); }

}  // namespace gpmppi
