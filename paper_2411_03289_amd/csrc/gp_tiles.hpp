// GP tile machinery shared by the rollout and its adjoint on gfx950:
// kernel-vector generation into LDS in the matrix-core operand layout,
// the pair-major walk over W = L^-1 on the matrix cores (FP32, BF16 and
// BF16x3 forms) and the staging of the per-point GP inputs.
#pragma once
#include "device_common.hpp"
#include "kernels.hpp"

namespace gpmppi {

// ---------------------------------------------------------------- W blocks
// W is walked in row-tile pairs (2u, 2u + 1), u < NP = NT / 2 (Mpad is a
// multiple of 64, so NT = Mpad / 32 is even): pair u
// takes 2u + 2 iterations it = 0 .. 2u + 1, each holding the two 32x32 blocks
// (2u, it) and (2u + 1, it) of W (rows 32t.., columns 32 it..).  Block (2u, 2u+1)
// lies above the diagonal and is stored as zeros, and so is every block of a
// row tile beyond the matrix, so all iterations are alike.  Packed block index
// b = 2 (u (u + 1) + it) + side, lane l of a wave:
//   FP32: float4 [b][q][l], component c: W[32t + l%32][32 it + 2(4q+c) + l/32]
//   BF16: uint4  [b][h][l], element e:   W[32t + l%32][32 it + 16h + 8(l/32) + e]
// The LDS operand of sample group g holds k in the same lane order with the
// sample 32g + l % 32 in place of the W row.
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

// k operand of one sample group for one block column.
template <int PREC>
struct KOp;
template <>
struct KOp<GPMPPI_FP32> {
    float4 v[4];
};
template <>
struct KOp<GPMPPI_BF16> {
    uint4 h[2];
};
template <>
struct KOp<GPMPPI_BF16X3> {
    uint4 h[2];
    uint4 l[2];
};

// Byte size of one sample group's k operand in LDS.
template <int PREC>
__host__ __device__ constexpr size_t kgroup_bytes(int Mpad) {
    return (size_t)Mpad * 32 * (PREC == GPMPPI_BF16 ? 2 : 4);
}

template <int PREC>
__device__ __forceinline__ void load_kop(KOp<PREC> &k, const unsigned char *kg, int jt, int lane, int Mpad) {
    if constexpr (PREC == GPMPPI_FP32) {
        const float4 *K = reinterpret_cast<const float4 *>(kg) + (size_t)jt * 256 + lane;
        k.v[0] = K[0];
        k.v[1] = K[64];
        k.v[2] = K[128];
        k.v[3] = K[192];
    } else {
        const uint4 *K = reinterpret_cast<const uint4 *>(kg) + (size_t)jt * 128 + lane;
        k.h[0] = K[0];
        k.h[1] = K[64];
        if constexpr (PREC == GPMPPI_BF16X3) {
            const uint4 *L = reinterpret_cast<const uint4 *>(kg + (size_t)Mpad * 64) + (size_t)jt * 128 + lane;
            k.l[0] = L[0];
            k.l[1] = L[64];
        }
    }
}

__device__ __forceinline__ v8bf as_bf(uint4 u) {
    v8bf r;
    __builtin_memcpy(&r, &u, 16);
    return r;
}

template <int PREC>
__device__ __forceinline__ void mma_block(v16f &acc, const WBlock<PREC> &b, const KOp<PREC> &k) {
    if constexpr (PREC == GPMPPI_FP32) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(b.v[q].x, k.v[q].x, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(b.v[q].y, k.v[q].y, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(b.v[q].z, k.v[q].z, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(b.v[q].w, k.v[q].w, acc, 0, 0, 0);
        }
    } else {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf(b.h[h]), as_bf(k.h[h]), acc, 0, 0, 0);
            if constexpr (PREC == GPMPPI_BF16X3) {
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf(b.h[h]), as_bf(k.l[h]), acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf(b.l[h]), as_bf(k.h[h]), acc, 0, 0, 0);
            }
        }
    }
}

// Pair list of wave w of NW: round i holds pairs NW i .. NW i + NW - 1,
// assigned in snake order so that the summed pair lengths (2u + 2) balance
// across waves.
template <int NW>
__device__ __forceinline__ int wave_pair(int w, int i) { return (i & 1) ? NW * i + NW - 1 - w : NW * i + w; }

// Row-tile list of wave w of NW for the single-row walk.  With eight waves,
// waves w and w + 4 share a SIMD and its matrix core, so the rows are dealt
// per SIMD: round i gives SIMD s = w % 4 the rows 8i + s (its first wave) and
// 8i + 7 - s (its second), which sum to the same block count on every SIMD.
// Walk over W: row-tile pairs (2u, 2u + 1) of 2u + 2 iterations, dealt to the
// waves in snake order, balance exactly when every wave takes an even number
// of them; otherwise the walk goes by single row tiles t (t + 1 blocks).
__host__ __device__ constexpr bool walk_by_rows(int NT, int NW) {
    return ((NT >> 1) % NW) != 0 || (((NT >> 1) / NW) & 1) != 0;
}
// Walk kinds a kernel is built for: either, decided per call, or one of them.
enum WalkKind { kWalkAny = 0, kWalkPairs = 1, kWalkRows = 2 };

template <int NW>
__device__ __forceinline__ int wave_row(int w, int i) {
    if constexpr (NW == 8) return (w < 4) ? 8 * i + w : 8 * i + 11 - w;
    else return wave_pair<NW>(w, i);
}

// Position in a wave's iteration sequence.  The wave's pairs, in visiting
// order, are packed 8 bits each into plist (at most 8 pairs: Mpad <= 1024);
// forward: pairs in order, it ascending; reverse: the exact reverse of that
// sequence.  Every pair has an even length.  The list is built once per output
// so that an iteration costs a few scalar additions and compares; past the
// end the cursor sits on pair 0 (a valid block).
struct Cursor {
    int n;      // pairs completed
    int it;     // current column tile
    int last;   // 2u + 1 for the current pair u
    int base;   // packed index of block (2u, 0): 2 u (u + 1)
};

template <bool REV>
__device__ __forceinline__ void cursor_pair(Cursor &c, uint64_t plist) {
    const int u = (int)((plist >> (8 * (c.n & 7))) & 0xFFu);
    c.last = 2 * u + 1;
    c.base = 2 * u * (u + 1);
    c.it = REV ? c.last : 0;
}

template <bool REV>
__device__ __forceinline__ void cursor_start(Cursor &c, uint64_t plist) {
    c.n = 0;
    cursor_pair<REV>(c, plist);
}

// Advances; returns true when the iteration just left closed its pair.
template <bool REV>
__device__ __forceinline__ bool cursor_next(Cursor &c, uint64_t plist) {
    if (!REV) {
        if (__builtin_expect(++c.it <= c.last, 1)) return false;
    } else {
        if (__builtin_expect(--c.it >= 0, 1)) return false;
    }
    ++c.n;
    cursor_pair<REV>(c, plist);
    return true;
}

__device__ __forceinline__ int pair_block(const Cursor &c) { return c.base + 2 * c.it; }
// The pair's last column tile: its block (2u, 2u + 1) lies above the diagonal.
__device__ __forceinline__ bool pair_zero(const Cursor &c) { return c.it == c.last; }

// Position in a wave's sequence of single row tiles t (blocks (t, 0) .. (t, t)),
// packed 8 bits each into rlist in visiting order (at most 8 rows); forward:
// columns ascending, reverse: the exact reverse sequence.  Past the end the
// cursor runs into the padded entries (row 0, a valid block).
struct RowCursor {
    int n;      // rows completed
    int c;      // current column tile
    int t;      // current row tile
    int base;   // packed index of block (t, 0): 2 u (u + 1) + t % 2 with u = t / 2
};

template <bool REV>
__device__ __forceinline__ void rcursor_row(RowCursor &c, uint64_t rlist) {
    const int t = (int)((rlist >> (8 * (c.n & 7))) & 0xFFu);
    const int u = t >> 1;
    c.t = t;
    c.base = 2 * u * (u + 1) + (t & 1);
    c.c = REV ? t : 0;
}

template <bool REV>
__device__ __forceinline__ void rcursor_start(RowCursor &c, uint64_t rlist) {
    c.n = 0;
    rcursor_row<REV>(c, rlist);
}

// Advances; returns true when the iteration just left closed its row.
template <bool REV>
__device__ __forceinline__ bool rcursor_next(RowCursor &c, uint64_t rlist) {
    if (!REV) {
        if (__builtin_expect(++c.c <= c.t, 1)) return false;
    } else {
        if (__builtin_expect(--c.c >= 0, 1)) return false;
    }
    ++c.n;
    rcursor_row<REV>(c, rlist);
    return true;
}

__device__ __forceinline__ int row_block(const RowCursor &c) { return c.base + 2 * c.c; }

// Buffer resources over one output's packed W: the block offset goes in the
// scalar offset, the lane offset stays in one VGPR, out-of-range reads return 0.
template <int PREC>
struct WRsrc {
    __amdgpu_buffer_rsrc_t h, l;
};

// Descriptor from wave-uniform base and size (the persistent batch kernel reads
// its GpDev from memory, where the compiler cannot prove uniformity and would
// otherwise wrap every load in a readfirstlane loop).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t uniform_rsrc(const void *base, long long bytes) {
    constexpr int kFlags = 0x00020000;   // raw (untyped) buffer, dword 3 of the descriptor
    const uint64_t a = (uint64_t)(uintptr_t)base;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    const int n = __builtin_amdgcn_readfirstlane((int)bytes);
    return __builtin_amdgcn_make_buffer_rsrc((void *)(uintptr_t)(((uint64_t)hi << 32) | lo), (short)0, n, kFlags);
}

template <int PREC>
__device__ __forceinline__ WRsrc<PREC> w_rsrc(const GpDev &g, int o) {
    WRsrc<PREC> r;
    if constexpr (PREC == GPMPPI_FP32) {
        r.h = uniform_rsrc(g.w32 + o * g.w32_stride, g.w32_stride * 16);
        r.l = r.h;
    } else {
        r.h = uniform_rsrc(g.wbh + o * g.wb_stride, g.wb_stride * 16);
        r.l = PREC == GPMPPI_BF16X3 ? uniform_rsrc(g.wbl + o * g.wb_stride, g.wb_stride * 16) : r.h;
    }
    return r;
}

__device__ __forceinline__ uint4 buf_load16(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    typedef unsigned int v4u __attribute__((ext_vector_type(4)));
    const v4u t = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
    uint4 u;
    __builtin_memcpy(&u, &t, 16);
    return u;
}

// W block blk of the packed layout for lane offset voff = 16 * lane.
template <int PREC>
__device__ __forceinline__ void load_wblock_rs(WBlock<PREC> &b, const WRsrc<PREC> &rs, int blk, int voff) {
    if constexpr (PREC == GPMPPI_FP32) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint4 t = buf_load16(rs.h, voff + 1024 * q, blk * 4096);
            __builtin_memcpy(&b.v[q], &t, 16);
        }
    } else {
        b.h[0] = buf_load16(rs.h, voff, blk * 2048);
        b.h[1] = buf_load16(rs.h, voff + 1024, blk * 2048);
        if constexpr (PREC == GPMPPI_BF16X3) {
            b.l[0] = buf_load16(rs.l, voff, blk * 2048);
            b.l[1] = buf_load16(rs.l, voff + 1024, blk * 2048);
        }
    }
}

template <int PREC>
__host__ __device__ constexpr int staged_slots(int Mpad);

template <int PREC, int G, int NW = kWaves>
struct Shapes {
    static constexpr int B = 32 * G;              // samples per block
    static constexpr int waves = NW;              // wave64s per workgroup
    static constexpr int threads = 64 * NW;
    static constexpr int parts = NW * (2 / G);    // loop splitters: waves (x half-waves for G = 1)
    static constexpr int rparts = 2 * NW;         // partial sums per sample in the reduction arrays
    // the waves that run the per-step geometry loops inside the variance contraction
    // (with two waves per SIMD, the first four, which get the matrix core first and finish
    // their share of W first)
    static constexpr int lwaves = NW == 8 ? 4 : NW;
    static constexpr int stage_iters = (1280 + threads - 1) / threads;   // staged-input slots per thread
};

// Per-point GP inputs: with two sample groups a wave's chunks of training
// points are wave-uniform, so the inputs are read through the scalar cache
// straight from global memory; with one group the two half-waves take
// different chunks and the inputs are staged in LDS.
template <int G>
__host__ __device__ constexpr bool scalar_inputs() { return G == 2; }

// The BF16 forms compute the kernel-vector exponents on the matrix cores from
// prepacked point operands (GpDev::zop) and need only alpha of both outputs in
// LDS, staged once per launch.
template <int PREC>
__host__ __device__ constexpr bool mfma_gen() { return PREC != GPMPPI_FP32; }

// Dynamic LDS layout: [G k-operand groups] then alpha [2][Mpad] (BF16 form),
// nothing (scalar-cache inputs) or the per-point inputs of one output.
template <int PREC, int G>
__host__ __device__ constexpr size_t dyn_lds_bytes(int Mpad) {
    return G * kgroup_bytes<PREC>(Mpad) +
           (mfma_gen<PREC>() ? (size_t)2 * Mpad * 4
                             : (scalar_inputs<G>() ? 0 : (size_t)staged_slots<PREC>(Mpad) * 16));
}

// Copies alpha of both outputs to LDS (all threads; the caller synchronises).
template <int NW>
__device__ __forceinline__ void stage_alpha(const GpDev &g, unsigned char *lds, size_t off) {
    const v4f *src = reinterpret_cast<const v4f *>(g.alpha);
    v4f *dst = reinterpret_cast<v4f *>(lds + off);
    for (int i = threadIdx.x; i < g.Mpad / 2; i += 64 * NW) dst[i] = src[i];
}

// Per-point inputs of output o staged in LDS for the FP32 form with one sample
// group (float4 slots): zs [Mpad] then alpha [Mpad / 4] (20 B per point), held in
// registers between their global load and their store to LDS; thread t of T
// owns slots t, t + T, ... (at most 1280 slots for Mpad <= 1024).
template <int PREC>
__host__ __device__ constexpr int staged_slots(int Mpad) {
    return PREC == GPMPPI_FP32 ? Mpad + (Mpad >> 2) : 0;
}

// Native vectors (not HIP's float4 struct, whose copies become memcpy of a
// private array that the compiler keeps in scratch memory).
struct StagedInputs {
    v4f v[6];
};

template <int PREC, int NW = kWaves>
__device__ __forceinline__ void stage_load(StagedInputs &st, const GpDev &g, int o) {
    static_assert(PREC == GPMPPI_FP32, "only the FP32 form stages its per-point inputs");
    const int Mpad = g.Mpad, nz = Mpad, ns = staged_slots<PREC>(Mpad);
    const v4f *zsrc = reinterpret_cast<const v4f *>(g.zs) + (size_t)o * Mpad;
    const v4f *asrc = reinterpret_cast<const v4f *>(g.alpha + (size_t)o * Mpad);
#pragma unroll
    for (int r = 0; r < Shapes<PREC, 1, NW>::stage_iters; ++r) {
        const int slot = threadIdx.x + r * (64 * NW);
        v4f val = {0.0f, 0.0f, 0.0f, 0.0f};
        if (slot < nz) val = zsrc[slot];
        else if (slot < ns) val = asrc[slot - nz];
        st.v[r] = val;
    }
}

template <int PREC, int NW = kWaves>
__device__ __forceinline__ void stage_store(const StagedInputs &st, const GpDev &g, unsigned char *lds,
                                            size_t zs_off) {
    const int ns = staged_slots<PREC>(g.Mpad);
    v4f *dst = reinterpret_cast<v4f *>(lds + zs_off);
#pragma unroll
    for (int r = 0; r < Shapes<PREC, 1, NW>::stage_iters; ++r) {
        const int slot = threadIdx.x + r * (64 * NW);
        if (slot < ns) dst[slot] = st.v[r];
    }
}

// BF16 bit patterns of three terms summing to the FP32 value x (round to
// nearest even at each stage; the remainders are exact in FP32).  Contraction
// is off: where x is a product, x - hi must not become a fused multiply-add of
// the unrounded product, or the split would depend on the code around it.
__device__ __forceinline__ void split3_bits(float x, uint32_t &h, uint32_t &m, uint32_t &l) {
#pragma clang fp contract(off)
    const __bf16 bh = (__bf16)x;
    const float r1 = x - (float)bh;
    const __bf16 bm = (__bf16)r1;
    const __bf16 bl = (__bf16)(r1 - (float)bm);
    uint16_t u;
    __builtin_memcpy(&u, &bh, 2);
    h = u;
    __builtin_memcpy(&u, &bm, 2);
    m = u;
    __builtin_memcpy(&u, &bl, 2);
    l = u;
}

__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
    typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
    typedef float v2f __attribute__((ext_vector_type(2)));
    const v2f x = {a, b};
    const v2bf h = __builtin_convertvector(x, v2bf);   // round to nearest even
    uint32_t r;
    __builtin_memcpy(&r, &h, 4);
    return r;
}

// The wave's share of |W k|^2 for the G sample groups: nit iterations over its
// pairs (plist, see Cursor) in direction REV.  W streams from L2 through a
// register ring two iterations deep, the k operand of the next iteration is
// read from LDS one iteration ahead.  Every iteration issues the same loads:
// past the end the cursors run into pair 0 of the padded list, and in place
// of the zero block above the diagonal the diagonal block is fetched twice, so
// the memory counters stay exact and each product waits for its own operands
// only.  Accumulators start from zero and are cleared after each pair.
template <int PREC, int G, bool REV>
__device__ __forceinline__ void walk_pairs(const WRsrc<PREC> &wrs, int voff, const unsigned char *lds, int lane,
                                           int Mpad, uint64_t plist, int nit, float sq[G]) {
    const unsigned char *kgrp[G];
#pragma unroll
    for (int gg = 0; gg < G; ++gg) kgrp[gg] = lds + gg * kgroup_bytes<PREC>(Mpad);
    WBlock<PREC> ring[2][2];
    KOp<PREC> kb[2][G];
    v16f acc[2][G];
#pragma unroll
    for (int gg = 0; gg < G; ++gg) {
        acc[0][gg] = v16f{};
        acc[1][gg] = v16f{};
        sq[gg] = 0.0f;
    }
    Cursor pc, mc;   // prefetch and compute cursors
    cursor_start<REV>(pc, plist);
    cursor_start<REV>(mc, plist);
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int b0 = pair_block(pc);
        load_wblock_rs<PREC>(ring[r][0], wrs, pair_zero(pc) ? b0 + 1 : b0, voff);
        load_wblock_rs<PREC>(ring[r][1], wrs, b0 + 1, voff);
        cursor_next<REV>(pc, plist);
    }
#pragma unroll
    for (int gg = 0; gg < G; ++gg) load_kop<PREC>(kb[0][gg], kgrp[gg], mc.it, lane, Mpad);
    for (int base = 0; base < nit; base += 2) {   // nit is even
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            if (!pair_zero(mc)) {
#pragma unroll
                for (int gg = 0; gg < G; ++gg) mma_block<PREC>(acc[0][gg], ring[r][0], kb[r][gg]);
            }
#pragma unroll
            for (int gg = 0; gg < G; ++gg) mma_block<PREC>(acc[1][gg], ring[r][1], kb[r][gg]);
            {   // refill this slot two iterations ahead
                const int b0 = pair_block(pc);
                load_wblock_rs<PREC>(ring[r][0], wrs, pair_zero(pc) ? b0 + 1 : b0, voff);
                load_wblock_rs<PREC>(ring[r][1], wrs, b0 + 1, voff);
                cursor_next<REV>(pc, plist);
            }
            const bool pair_end = cursor_next<REV>(mc, plist);
#pragma unroll
            for (int gg = 0; gg < G; ++gg) load_kop<PREC>(kb[1 - r][gg], kgrp[gg], mc.it, lane, Mpad);
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
            }
        }
    }
}

struct NoSideWork {
    __device__ void operator()(int) const {}
};

// The wave's share of |W k|^2 by single row tiles (rlist, see RowCursor), nb
// blocks in all: one block per iteration, W streamed through a register ring
// four blocks deep, the k operand of the next block read from LDS one block
// ahead.  Used where the row-tile pairs cannot be spread evenly over the
// waves; every block loads its own k operand, twice the LDS reads of the pair
// walk.  Iterations past nb (to a multiple of four) load but do not multiply.
template <int PREC, int G, bool REV>
__device__ __forceinline__ void walk_rows(const WRsrc<PREC> &wrs, int voff, const unsigned char *lds, int lane,
                                          int Mpad, uint64_t rlist, int nb, float sq[G]) {
    const unsigned char *kgrp[G];
#pragma unroll
    for (int gg = 0; gg < G; ++gg) kgrp[gg] = lds + gg * kgroup_bytes<PREC>(Mpad);
    WBlock<PREC> ring[4];
    KOp<PREC> kb[2][G];
    v16f acc[G];
#pragma unroll
    for (int gg = 0; gg < G; ++gg) {
        acc[gg] = v16f{};
        sq[gg] = 0.0f;
    }
    RowCursor pc, mc;   // prefetch and compute cursors
    rcursor_start<REV>(pc, rlist);
    rcursor_start<REV>(mc, rlist);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        load_wblock_rs<PREC>(ring[r], wrs, row_block(pc), voff);
        rcursor_next<REV>(pc, rlist);
    }
#pragma unroll
    for (int gg = 0; gg < G; ++gg) load_kop<PREC>(kb[0][gg], kgrp[gg], mc.c, lane, Mpad);
    for (int base = 0; base < nb; base += 4) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (base + r < nb) {
#pragma unroll
                for (int gg = 0; gg < G; ++gg) mma_block<PREC>(acc[gg], ring[r], kb[r & 1][gg]);
            }
            load_wblock_rs<PREC>(ring[r], wrs, row_block(pc), voff);   // four blocks ahead
            rcursor_next<REV>(pc, rlist);
            const bool row_end = rcursor_next<REV>(mc, rlist);
#pragma unroll
            for (int gg = 0; gg < G; ++gg) load_kop<PREC>(kb[(r + 1) & 1][gg], kgrp[gg], mc.c, lane, Mpad);
            if (__builtin_expect(row_end, 0)) {
#pragma unroll
                for (int gg = 0; gg < G; ++gg) {
#pragma unroll
                    for (int e = 0; e < 16; ++e) sq[gg] = fmaf(acc[gg][e], acc[gg][e], sq[gg]);
                    acc[gg] = v16f{};
                }
            }
        }
    }
}

// ---------------------------------------------------------------- matrix-core generation
// The exponents c2 - |qs - zs_j|^2 of a 32-point column tile for 32 samples come
// from two 32x32x16 BF16 products with the FP32 factors split into three BF16
// terms (the operand layout is described at pack_zop_kernel); exp2, the mean and
// the BF16 k operand on the VALU.  Lane l: sample 32 g + l % 32, points
// 8 (l / 32) + r (r < 8) and 16 + 8 (l / 32) + r - 8 of the tile.

// B operands (the samples' split factors) of the G groups for scaled queries qs.
template <int G>
__device__ __forceinline__ void gen_bop(const float qs[4], int hl, uint4 bop[G][2]) {
#pragma unroll
    for (int gg = 0; gg < G; ++gg) {
        float qv[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const float other = (G == 2) ? shfl_xor(qs[d], 32) : qs[d];
            qv[d] = (G == 1 || hl == gg) ? qs[d] : other;
        }
        // explicit fused multiply-adds: the same rounding wherever this is inlined
        const float qq = fmaf(qv[3], qv[3], fmaf(qv[2], qv[2], fmaf(qv[1], qv[1], qv[0] * qv[0])));
        uint32_t qh[4], qm[4], ql[4], nqq[3];
#pragma unroll
        for (int d = 0; d < 4; ++d) split3_bits(qv[d], qh[d], qm[d], ql[d]);
        split3_bits(-qq, nqq[0], nqq[1], nqq[2]);
        const uint32_t one = 0x3f80u;
        if (hl == 0) {   // slots 0-7 of both products: (qh, qm) and (qm, qh)
            bop[gg][0] = make_uint4(qh[0] | qh[1] << 16, qh[2] | qh[3] << 16, qm[0] | qm[1] << 16, qm[2] | qm[3] << 16);
            bop[gg][1] = make_uint4(qm[0] | qm[1] << 16, qm[2] | qm[3] << 16, qh[0] | qh[1] << 16, qh[2] | qh[3] << 16);
        } else {         // slots 8-15: (qh, ql) and (1, 1, 1, -qq h, -qq m, -qq l, 0, 0)
            bop[gg][0] = make_uint4(qh[0] | qh[1] << 16, qh[2] | qh[3] << 16, ql[0] | ql[1] << 16, ql[2] | ql[3] << 16);
            bop[gg][1] = make_uint4(one | one << 16, one | nqq[0] << 16, nqq[1] | nqq[2] << 16, 0u);
        }
    }
}

// A operands and alpha values of one column tile.
struct GenOps {
    uint4 a0, a1;
    v4f al[4];
};

// Fetches tile jt (clamped to the last tile, so a fetch past the end repeats it).
__device__ __forceinline__ void gen_fetch(GenOps &t, const uint4 *zop, const float *al, int NT, int jt, int lane,
                                          int hl) {
    const int jc = jt < NT ? jt : NT - 1;
    t.a0 = zop[(jc * 2) * 64 + lane];
    t.a1 = zop[(jc * 2 + 1) * 64 + lane];
    const v4f *ap = reinterpret_cast<const v4f *>(al + 32 * jc + 8 * hl);
    t.al[0] = ap[0];
    t.al[1] = ap[1];
    t.al[2] = ap[4];
    t.al[3] = ap[5];
}

// One tile for the G groups: k = exp2 of the exponents, the mean partials ms, and
// k packed to BF16 (hv) with, for the BF16x3 form, the BF16 remainders k - hi (lv).
template <int PREC, int G>
__device__ __forceinline__ void gen_tile(const GenOps &t, const uint4 bop[G][2], float ms[G], uint32_t hv[G][8],
                                         uint32_t lv[G][8]) {
#pragma unroll
    for (int gg = 0; gg < G; ++gg) {
        v16f e = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf(t.a0), as_bf(bop[gg][0]), v16f{}, 0, 0, 0);
        e = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf(t.a1), as_bf(bop[gg][1]), e, 0, 0, 0);
        float kv[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) kv[r] = __builtin_amdgcn_exp2f(e[r]);
#pragma unroll
        for (int r = 0; r < 16; ++r) ms[gg] = fmaf(kv[r], t.al[r >> 2][r & 3], ms[gg]);
#pragma unroll
        for (int i = 0; i < 8; ++i) hv[gg][i] = pack_bf16x2(kv[2 * i], kv[2 * i + 1]);
        if constexpr (PREC == GPMPPI_BF16X3) {
#pragma unroll
            for (int i = 0; i < 8; ++i)
                lv[gg][i] = pack_bf16x2(kv[2 * i] - bf16_to_f32((uint16_t)hv[gg][i]),
                                        kv[2 * i + 1] - bf16_to_f32((uint16_t)(hv[gg][i] >> 16)));
        }
    }
}

// Writes tile jt of the G groups' k operands to LDS.
template <int PREC, int G>
__device__ __forceinline__ void gen_store(unsigned char *lds, int Mpad, int jt, int lane, const uint32_t hv[G][8],
                                          const uint32_t lv[G][8]) {
#pragma unroll
    for (int gg = 0; gg < G; ++gg) {
        uint4 *K = reinterpret_cast<uint4 *>(lds + gg * kgroup_bytes<PREC>(Mpad)) + (size_t)jt * 128;
        K[lane] = make_uint4(hv[gg][0], hv[gg][1], hv[gg][2], hv[gg][3]);
        K[64 + lane] = make_uint4(hv[gg][4], hv[gg][5], hv[gg][6], hv[gg][7]);
        if constexpr (PREC == GPMPPI_BF16X3) {
            uint4 *L = reinterpret_cast<uint4 *>(lds + gg * kgroup_bytes<PREC>(Mpad) + (size_t)Mpad * 64) +
                       (size_t)jt * 128;
            L[lane] = make_uint4(lv[gg][0], lv[gg][1], lv[gg][2], lv[gg][3]);
            L[64 + lane] = make_uint4(lv[gg][4], lv[gg][5], lv[gg][6], lv[gg][7]);
        }
    }
}

// Kernel vectors of output o for the B samples of the block and their GP mean;
// called by all threads with the inputs of output o staged in LDS.  Ends with
// a workgroup barrier; returns the sample's GP mean.
template <int PREC, int G, int NW = kWaves>
__device__ __forceinline__ float gp_gen(const GpDev &g, int o, const float qs[4], int part, int sl,
                                        unsigned char *lds, float *pred) {
    using S = Shapes<PREC, G, NW>;
    constexpr bool kScalar = scalar_inputs<G>();
    const int Mpad = g.Mpad;
    const int nchunk = Mpad >> 3;
    const v4f *zs = reinterpret_cast<const v4f *>(lds + G * kgroup_bytes<PREC>(Mpad));   // staged inputs
    const int grp = sl >> 5, s32 = sl & 31;
    unsigned char *kg = lds + grp * kgroup_bytes<PREC>(Mpad);
    const int c0 = kScalar ? __builtin_amdgcn_readfirstlane(part) : part;
    float msum = 0.0f;
    if constexpr (PREC == GPMPPI_FP32) {
        // exact differences: k = exp2(c2 - sum_d (q_d - zs_d)^2)
        const const_v4p zsg = (const_v4p)g.zs + (size_t)o * Mpad;
        const const_v4p alg = (const_v4p)(g.alpha + (size_t)o * Mpad);
        const float c2 = g.c2[o];
        for (int c = c0; c < nchunk; c += S::parts) {
            float kv[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const v4f z = kScalar ? zsg[8 * c + e] : zs[8 * c + e];
                const float d0 = qs[0] - z.x, d1 = qs[1] - z.y, d2 = qs[2] - z.z, d3 = qs[3] - z.w;
                float acc = c2;
                acc = fmaf(-d0, d0, acc);
                acc = fmaf(-d1, d1, acc);
                acc = fmaf(-d2, d2, acc);
                acc = fmaf(-d3, d3, acc);
                kv[e] = __builtin_amdgcn_exp2f(acc);
            }
            const v4f a0 = kScalar ? alg[2 * c] : zs[Mpad + 2 * c];
            const v4f a1 = kScalar ? alg[2 * c + 1] : zs[Mpad + 2 * c + 1];
            msum = fmaf(kv[0], a0.x, msum);
            msum = fmaf(kv[1], a0.y, msum);
            msum = fmaf(kv[2], a0.z, msum);
            msum = fmaf(kv[3], a0.w, msum);
            msum = fmaf(kv[4], a1.x, msum);
            msum = fmaf(kv[5], a1.y, msum);
            msum = fmaf(kv[6], a1.z, msum);
            msum = fmaf(kv[7], a1.w, msum);
            float4 *K = reinterpret_cast<float4 *>(kg) + (size_t)c * 64;
            K[s32] = make_float4(kv[0], kv[2], kv[4], kv[6]);
            K[32 + s32] = make_float4(kv[1], kv[3], kv[5], kv[7]);
        }
    } else if constexpr (mfma_gen<PREC>()) {
        const int lane = threadIdx.x & 63, hl = lane >> 5;
        const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
        const float *al = reinterpret_cast<const float *>(lds + G * kgroup_bytes<PREC>(Mpad)) + (size_t)o * Mpad;
        const uint4 *zop = g.zop + o * g.zop_stride;
        uint4 bop[G][2];
        gen_bop<G>(qs, hl, bop);
        float ms[G];
#pragma unroll
        for (int gg = 0; gg < G; ++gg) ms[gg] = 0.0f;
        // this wave's tiles jt = wv, wv + NW, ..., each fetched one tile ahead into the
        // other of two register sets
        uint32_t hv[G][8], lv[G][8];
        GenOps ta, tb;
        gen_fetch(ta, zop, al, g.NT, wv, lane, hl);
        for (int jt = wv; jt < g.NT; jt += 2 * NW) {
            gen_fetch(tb, zop, al, g.NT, jt + NW, lane, hl);
            gen_tile<PREC, G>(ta, bop, ms, hv, lv);
            gen_store<PREC, G>(lds, Mpad, jt, lane, hv, lv);
            if (jt + NW >= g.NT) break;
            gen_fetch(ta, zop, al, g.NT, jt + 2 * NW, lane, hl);
            gen_tile<PREC, G>(tb, bop, ms, hv, lv);
            gen_store<PREC, G>(lds, Mpad, jt + NW, lane, hv, lv);
        }
        // partial means per (wave, half-wave) for each group's sample
#pragma unroll
        for (int gg = 0; gg < G; ++gg) pred[(wv * 2 + hl) * S::B + 32 * gg + (lane & 31)] = ms[gg];
    }
    // per-part partial means: the lanes of a part hold distinct samples
    if constexpr (!mfma_gen<PREC>()) pred[part * S::B + sl] = msum;
    __syncthreads();
    float m = 0.0f;
    constexpr int mparts = mfma_gen<PREC>() ? S::rparts : S::parts;
#pragma unroll
    for (int p = 0; p < mparts; ++p) m += pred[p * S::B + sl];
    return m;
}

// Variance of output o for the B samples of the block, after gp_gen: v = W k on
// the matrix cores, s2 = vscale (sn^2 + max(0, sf^2 - |v|^2)).  If next_o >= 0
// the staged inputs of output next_o replace those of o (forms that stage them;
// the caller synchronises before the next use).  side(w) is called by every
// wave w once its share of the contraction is done, before the workgroup
// synchronises: work that does not depend on this output can fill the time the
// waves wait for each other there.  Ends with a workgroup barrier.
template <int PREC, int G, int NW = kWaves, int WALK = kWalkAny, class Side = NoSideWork>
__device__ __forceinline__ float gp_walk(const GpDev &g, int o, int next_o, bool rev, int rotate, int blk,
                                         unsigned char *lds, float *vred, int sl, const Side &side = Side()) {
    using S = Shapes<PREC, G, NW>;
    constexpr bool kScalar = scalar_inputs<G>();
    const int Mpad = g.Mpad;
    StagedInputs st;
    if constexpr (!kScalar && !mfma_gen<PREC>()) {
        if (next_o >= 0) stage_load<PREC, NW>(st, g, next_o);
    }

    // ---- variance contraction on the matrix cores
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // units of work: row-tile pairs (wave_pair) or single row tiles (wave_row)
    const int NT = g.NT, NP = NT >> 1;
    const bool by_rows = WALK == kWalkAny ? walk_by_rows(NT, NW) : WALK == kWalkRows;
    const int nunit_all = by_rows ? NT : NP;
    const int rounds = (nunit_all + NW - 1) / NW;
    auto unit = [&](int i) { return by_rows ? wave_row<NW>(w, i) : wave_pair<NW>(w, i); };
    int nunits = rounds;
    if (rounds > 0 && unit(rounds - 1) >= nunit_all) nunits = rounds - 1;
    int nwork = 0;   // pair walk: iterations (even); row walk: blocks
    for (int i = 0; i < nunits; ++i) nwork += by_rows ? unit(i) + 1 : 2 * unit(i) + 2;
    const int r0 = (rotate && nunits > 0) ? (int)((unsigned)blk % (unsigned)nunits) : 0;
    uint64_t ulist = 0;   // this wave's units in visiting order (see Cursor, RowCursor)
    for (int n = 0; n < nunits; ++n) {
        int i = rev ? r0 - 1 - n : r0 + n;
        i %= nunits;
        if (i < 0) i += nunits;
        ulist |= (uint64_t)unit(i) << (8 * n);
    }
    const WRsrc<PREC> wrs = w_rsrc<PREC>(g, o);
    const int voff = 16 * lane;

    float sq[G];
    if (WALK != kWalkPairs && by_rows) {
        if constexpr (WALK != kWalkPairs) {
            if (rev)
                walk_rows<PREC, G, true>(wrs, voff, lds, lane, Mpad, ulist, nwork, sq);
            else
                walk_rows<PREC, G, false>(wrs, voff, lds, lane, Mpad, ulist, nwork, sq);
        }
    } else {
        if constexpr (WALK != kWalkRows) {
            if (rev)
                walk_pairs<PREC, G, true>(wrs, voff, lds, lane, Mpad, ulist, nwork, sq);
            else
                walk_pairs<PREC, G, false>(wrs, voff, lds, lane, Mpad, ulist, nwork, sq);
        }
    }
#pragma unroll
    for (int gg = 0; gg < G; ++gg) {
        sq[gg] += shfl_xor(sq[gg], 32);
        if (lane < 32) vred[w * S::B + gg * 32 + lane] = sq[gg];
    }
    side(w);
    __syncthreads();
    if constexpr (!kScalar && !mfma_gen<PREC>()) {
        if (next_o >= 0) stage_store<PREC, NW>(st, g, lds, G * kgroup_bytes<PREC>(Mpad));
    }
    float v2 = 0.0f;
#pragma unroll
    for (int ww = 0; ww < NW; ++ww) v2 += vred[ww * S::B + sl];
    return g.vscale[o] * (g.sn2[o] + fmaxf(0.0f, g.sf2[o] - v2));
}

// One GP output: gp_gen then gp_walk (see there).
template <int PREC, int G, int NW = kWaves, int WALK = kWalkAny, class Side = NoSideWork>
__device__ __forceinline__ void gp_output(const GpDev &g, int o, int next_o, const float qs[4], int part, int sl,
                                          bool rev, int rotate, int blk, unsigned char *lds, float *pred,
                                          float *vred, float &mean_out, float &var_out,
                                          const Side &side = Side()) {
    mean_out = gp_gen<PREC, G, NW>(g, o, qs, part, sl, lds, pred);
    var_out = gp_walk<PREC, G, NW, WALK>(g, o, next_o, rev, rotate, blk, lds, vred, sl, side);
}

}  // namespace gpmppi
