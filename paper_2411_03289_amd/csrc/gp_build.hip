// Once-per-GP-update build of each residual GP in FP64 on the GPU
// (Rasmussen & Williams Alg. 2.1 with the explicit inverse factor):
//   A = K(Z, Z) + sn^2 I         SE-ARD covariance (Sec. III-A, Sec. V-A)
//   L = chol(A)                  blocked left-looking Cholesky, 32x32 tiles
//   W = L^-1                     block-column forward substitution
//   alpha = W^T (W y) = A^-1 y
// and the packing of W, alpha and the scaled inputs into the FP32 / BF16
// layouts the rollout streams.  Padding rows/columns (M <= i < Mpad) carry
// the identity in A and are zeroed when packing.
#include "device_common.hpp"
#include "kernels.hpp"

namespace gpmppi {

constexpr int NB = 32;   // tile edge

__global__ void kmat_kernel(const double *Z, int M, int Mpad, double i0, double i1, double i2, double i3,
                            double sf2, double sn2, double *A) {
    const int j = blockIdx.x * 16 + threadIdx.x;
    const int i = blockIdx.y * 16 + threadIdx.y;
    if (i >= Mpad || j >= Mpad) return;
    double v;
    if (i < M && j < M) {
        const double d0 = Z[4 * i] - Z[4 * j], d1 = Z[4 * i + 1] - Z[4 * j + 1];
        const double d2 = Z[4 * i + 2] - Z[4 * j + 2], d3 = Z[4 * i + 3] - Z[4 * j + 3];
        const double r2 = d0 * d0 * i0 + d1 * d1 * i1 + d2 * d2 * i2 + d3 * d3 * i3;
        v = sf2 * exp(-0.5 * r2) + (i == j ? sn2 : 0.0);
    } else {
        v = (i == j) ? 1.0 : 0.0;
    }
    A[(size_t)i * Mpad + j] = v;
}

// Left-looking update of block column kb: A[ib][kb] -= sum_{pb<kb} L[ib][pb] L[kb][pb]^T
// for ib = kb + blockIdx.x; the diagonal block is then factored in place.
__global__ __launch_bounds__(256) void chol_column_kernel(double *A, int Mpad, int kb, uint32_t *flag) {
    __shared__ double Ta[NB][NB + 1], Tb[NB][NB + 1], C[NB][NB + 1];
    const int ib = kb + blockIdx.x;
    const int tid = threadIdx.x;
    const int row = tid >> 3, c0 = (tid & 7) * 4;   // each thread: 1 row x 4 columns
    double acc[4];
    for (int e = 0; e < 4; ++e) acc[e] = A[(size_t)(ib * NB + row) * Mpad + kb * NB + c0 + e];
    for (int pb = 0; pb < kb; ++pb) {
        for (int e = tid; e < NB * NB; e += 256) {
            const int rr = e / NB, cc = e % NB;
            Ta[rr][cc] = A[(size_t)(ib * NB + rr) * Mpad + pb * NB + cc];
            Tb[rr][cc] = A[(size_t)(kb * NB + rr) * Mpad + pb * NB + cc];
        }
        __syncthreads();
        for (int p = 0; p < NB; ++p) {
            const double a = Ta[row][p];
            for (int e = 0; e < 4; ++e) acc[e] -= a * Tb[c0 + e][p];
        }
        __syncthreads();
    }
    if (ib != kb) {
        for (int e = 0; e < 4; ++e) A[(size_t)(ib * NB + row) * Mpad + kb * NB + c0 + e] = acc[e];
        return;
    }
    for (int e = 0; e < 4; ++e) C[row][c0 + e] = acc[e];
    __syncthreads();
    for (int c = 0; c < NB; ++c) {
        if (tid == 0) {
            const double d = C[c][c];
            if (!(d > 0.0)) atomicOr(flag, 1u);
            C[c][c] = sqrt(d > 0.0 ? d : 1.0);
        }
        __syncthreads();
        if (tid > c && tid < NB) C[tid][c] /= C[c][c];
        __syncthreads();
        for (int e = tid; e < NB * NB; e += 256) {
            const int i = e / NB, j = e % NB;
            if (j > c && i >= j) C[i][j] -= C[i][c] * C[j][c];
        }
        __syncthreads();
    }
    for (int e = tid; e < NB * NB; e += 256) {
        const int i = e / NB, j = e % NB;
        A[(size_t)(kb * NB + i) * Mpad + kb * NB + j] = (j <= i) ? C[i][j] : 0.0;
    }
}

// L[ib][kb] = A[ib][kb] L[kb][kb]^-T for ib = kb + 1 + blockIdx.x.
__global__ __launch_bounds__(64) void chol_trsm_kernel(double *A, int Mpad, int kb) {
    __shared__ double Ld[NB][NB + 1], X[NB][NB + 1];
    const int ib = kb + 1 + blockIdx.x;
    const int tid = threadIdx.x;
    for (int e = tid; e < NB * NB; e += 64) {
        const int i = e / NB, j = e % NB;
        Ld[i][j] = A[(size_t)(kb * NB + i) * Mpad + kb * NB + j];
        X[i][j] = A[(size_t)(ib * NB + i) * Mpad + kb * NB + j];
    }
    __syncthreads();
    if (tid < NB) {
        const int rr = tid;   // row of X: X[r][c] = (A[r][c] - sum_{p<c} X[r][p] L[c][p]) / L[c][c]
        for (int c = 0; c < NB; ++c) {
            double v = X[rr][c];
            for (int p = 0; p < c; ++p) v -= X[rr][p] * Ld[c][p];
            X[rr][c] = v / Ld[c][c];
        }
    }
    __syncthreads();
    for (int e = tid; e < NB * NB; e += 64) {
        const int i = e / NB, j = e % NB;
        A[(size_t)(ib * NB + i) * Mpad + kb * NB + j] = X[i][j];
    }
}

// W[:, jb] = L^-1 e_jb by forward substitution over row blocks ib >= jb;
// block jb = blockIdx.x.  W is lower triangular; blocks above are zeroed.
__global__ __launch_bounds__(256) void trinv_kernel(const double *L, double *W, int Mpad) {
    __shared__ double Lt[NB][NB + 1], Xt[NB][NB + 1], R[NB][NB + 1];
    const int jb = blockIdx.x, nb = Mpad / NB;
    const int tid = threadIdx.x;
    const int row = tid >> 3, c0 = (tid & 7) * 4;
    for (int ib = 0; ib < jb; ++ib)
        for (int e = tid; e < NB * NB; e += 256)
            W[(size_t)(ib * NB + e / NB) * Mpad + jb * NB + e % NB] = 0.0;
    for (int ib = jb; ib < nb; ++ib) {
        double acc[4];
        for (int e = 0; e < 4; ++e) acc[e] = (ib == jb && row == c0 + e) ? 1.0 : 0.0;
        for (int kb = jb; kb < ib; ++kb) {
            for (int e = tid; e < NB * NB; e += 256) {
                const int i = e / NB, j = e % NB;
                Lt[i][j] = L[(size_t)(ib * NB + i) * Mpad + kb * NB + j];
                Xt[i][j] = W[(size_t)(kb * NB + i) * Mpad + jb * NB + j];
            }
            __syncthreads();
            for (int p = 0; p < NB; ++p) {
                const double a = Lt[row][p];
                for (int e = 0; e < 4; ++e) acc[e] -= a * Xt[p][c0 + e];
            }
            __syncthreads();
        }
        for (int e = 0; e < 4; ++e) R[row][c0 + e] = acc[e];
        for (int e = tid; e < NB * NB; e += 256) {
            const int i = e / NB, j = e % NB;
            Lt[i][j] = L[(size_t)(ib * NB + i) * Mpad + ib * NB + j];
        }
        __syncthreads();
        if (tid < NB) {   // column tid: solve Lt x = R[:, tid]
            const int c = tid;
            for (int i = 0; i < NB; ++i) {
                double v = R[i][c];
                for (int p = 0; p < i; ++p) v -= Lt[i][p] * R[p][c];
                R[i][c] = v / Lt[i][i];
            }
        }
        __syncthreads();
        for (int e = tid; e < NB * NB; e += 256) {
            const int i = e / NB, j = e % NB;
            W[(size_t)(ib * NB + i) * Mpad + jb * NB + j] = R[i][j];
        }
        __syncthreads();
    }
}

__global__ void matvec_lower_kernel(const double *W, const double *x, double *y, int Mpad, int transpose) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Mpad) return;
    double acc = 0.0;
    if (!transpose) {
        for (int j = 0; j <= i; ++j) acc += W[(size_t)i * Mpad + j] * x[j];
    } else {
        for (int j = i; j < Mpad; ++j) acc += W[(size_t)j * Mpad + i] * x[j];
    }
    y[i] = acc;
}

hipError_t build_gp_output(const GpBuildBuffers &b, int M, int Mpad, const double ell[4], double sf2,
                           double sn2, hipStream_t st) {
    const int nb = Mpad / NB;
    hipLaunchKernelGGL(kmat_kernel, dim3(Mpad / 16, Mpad / 16), dim3(16, 16), 0, st, b.Z, M, Mpad,
                       1.0 / (ell[0] * ell[0]), 1.0 / (ell[1] * ell[1]), 1.0 / (ell[2] * ell[2]),
                       1.0 / (ell[3] * ell[3]), sf2, sn2, b.A);
    for (int kb = 0; kb < nb; ++kb) {
        hipLaunchKernelGGL(chol_column_kernel, dim3(nb - kb), dim3(256), 0, st, b.A, Mpad, kb, b.flag);
        if (kb + 1 < nb) hipLaunchKernelGGL(chol_trsm_kernel, dim3(nb - kb - 1), dim3(64), 0, st, b.A, Mpad, kb);
    }
    hipLaunchKernelGGL(trinv_kernel, dim3(nb), dim3(256), 0, st, b.A, b.W, Mpad);
    hipLaunchKernelGGL(matvec_lower_kernel, dim3((Mpad + 255) / 256), dim3(256), 0, st, b.W, b.y, b.u, Mpad, 0);
    hipLaunchKernelGGL(matvec_lower_kernel, dim3((Mpad + 255) / 256), dim3(256), 0, st, b.W, b.u, b.alpha, Mpad, 1);
    return hipGetLastError();
}

// alpha = W^T (W y) for another target vector y on the same W (b.u is scratch).
hipError_t alpha_for_targets(const GpBuildBuffers &b, int Mpad, const double *y_d, double *alpha_d, hipStream_t st) {
    hipLaunchKernelGGL(matvec_lower_kernel, dim3((Mpad + 255) / 256), dim3(256), 0, st, b.W, y_d, b.u, Mpad, 0);
    hipLaunchKernelGGL(matvec_lower_kernel, dim3((Mpad + 255) / 256), dim3(256), 0, st, b.W, b.u, alpha_d, Mpad, 1);
    return hipGetLastError();
}

__global__ void combine_alpha_kernel(const double *alpha_terr, int n_terr, int Mpad, TerrainWeights w,
                                     double *out64, float *alpha32) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= Mpad) return;
    double a = 0.0;
    for (int i = 0; i < n_terr; ++i) a += w.w[i] * alpha_terr[(size_t)i * Mpad + j];
    if (out64) out64[j] = a;
    alpha32[j] = (float)a;
}

hipError_t combine_alpha(const double *alpha_terr, int n_terr, int Mpad, TerrainWeights w, double *out64,
                         float *alpha32, hipStream_t st) {
    hipLaunchKernelGGL(combine_alpha_kernel, dim3((Mpad + 255) / 256), dim3(256), 0, st, alpha_terr, n_terr, Mpad, w,
                       out64, alpha32);
    return hipGetLastError();
}

// Q = W^T W = A^-1 (FP64) into Qd, for the adjoint's r = Q k; one thread
// per entry, the sum running over the rows k >= max(i, j) where W is nonzero.
__global__ void qmat_kernel(const double *W, int Mpad, double *Qd) {
    const int j = blockIdx.x * 16 + threadIdx.x;
    const int i = blockIdx.y * 16 + threadIdx.y;
    if (i >= Mpad || j >= Mpad) return;
    double acc = 0.0;
    for (int k = (i > j ? i : j); k < Mpad; ++k) acc += W[(size_t)k * Mpad + i] * W[(size_t)k * Mpad + j];
    Qd[(size_t)i * Mpad + j] = acc;
}

// Dense FP32 packing of Q in the matrix-core operand order of the FP32 W
// blocks: block b = t NT + it, float4 [b][q][lane], component c holds
// Q[32t + l%32][32 it + 2(4q+c) + l/32].  Rows/columns beyond M are zero.
__global__ void pack_q_kernel(const double *Qd, int M, int Mpad, float4 *q32) {
    const int blk = blockIdx.x, lane = threadIdx.x;
    const int NT = Mpad / 32;
    const int t = blk / NT, it = blk % NT;
    const int i = 32 * t + (lane & 31);
    const int half = lane >> 5;
    auto qval = [&](int j) -> float { return (i < M && j < M) ? (float)Qd[(size_t)i * Mpad + j] : 0.0f; };
    for (int q = 0; q < 4; ++q) {
        float4 v;
        v.x = qval(32 * it + 2 * (4 * q + 0) + half);
        v.y = qval(32 * it + 2 * (4 * q + 1) + half);
        v.z = qval(32 * it + 2 * (4 * q + 2) + half);
        v.w = qval(32 * it + 2 * (4 * q + 3) + half);
        q32[(size_t)blk * 256 + q * 64 + lane] = v;
    }
}

hipError_t pack_q(const GpBuildBuffers &b, int M, int Mpad, float4 *q32, hipStream_t st) {
    // A (the Cholesky factor's storage) is free once W has been formed
    hipLaunchKernelGGL(qmat_kernel, dim3(Mpad / 16, Mpad / 16), dim3(16, 16), 0, st, b.W, Mpad, b.A);
    const int NT = Mpad / 32;
    hipLaunchKernelGGL(pack_q_kernel, dim3(NT * NT), dim3(64), 0, st, b.A, M, Mpad, q32);
    return hipGetLastError();
}

// Terrain means at n queries: out[q][i][o] = k_o(q)^T alpha_{o,i}; one
// workgroup per query, threads over training points, FP64 accumulation of the
// FP32 kernel values.  alpha_terr is [2][n_terr][Mpad] FP64.
__global__ __launch_bounds__(256) void terrain_means_kernel(const float *q, int n, const float *zs, const double *alpha_terr,
                                                            int n_terr, int Mpad, float s00, float s01, float s02,
                                                            float s03, float s10, float s11, float s12, float s13,
                                                            float c20, float c21, float *out) {
    __shared__ double red[8][4];
    const int qi = blockIdx.x, tid = threadIdx.x;
    const float4 qq = reinterpret_cast<const float4 *>(q)[qi];
    for (int o = 0; o < 2; ++o) {
        const float sc[4] = {o ? s10 : s00, o ? s11 : s01, o ? s12 : s02, o ? s13 : s03};
        const float qs[4] = {qq.x * sc[0], qq.y * sc[1], qq.z * sc[2], qq.w * sc[3]};
        const float c2 = o ? c21 : c20;
        double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int j = tid; j < Mpad; j += 256) {
            const float4 z = reinterpret_cast<const float4 *>(zs)[(size_t)o * Mpad + j];
            const float d0 = qs[0] - z.x, d1 = qs[1] - z.y, d2 = qs[2] - z.z, d3 = qs[3] - z.w;
            const double kv = (double)exp2f(c2 - (d0 * d0 + d1 * d1 + d2 * d2 + d3 * d3));
            for (int i = 0; i < n_terr; ++i) acc[i] += kv * alpha_terr[((size_t)o * n_terr + i) * Mpad + j];
        }
        for (int i = 0; i < n_terr; ++i) {
            double v = acc[i];
            for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
            if ((tid & 63) == 0) red[i][tid >> 6] = v;
        }
        __syncthreads();
        if (tid < n_terr) {
            const double v = red[tid][0] + red[tid][1] + red[tid][2] + red[tid][3];
            out[((size_t)qi * n_terr + tid) * 2 + o] = (float)v;
        }
        __syncthreads();
    }
}

hipError_t launch_terrain_means(const float *q, int n, const GpDev &g, const double *alpha_terr, int n_terr,
                                float *out, hipStream_t st) {
    hipLaunchKernelGGL(terrain_means_kernel, dim3(n), dim3(256), 0, st, q, n, g.zs, alpha_terr, n_terr, g.Mpad,
                       g.scale[0][0], g.scale[0][1], g.scale[0][2], g.scale[0][3], g.scale[1][0], g.scale[1][1],
                       g.scale[1][2], g.scale[1][3], g.c2[0], g.c2[1], out);
    return hipGetLastError();
}

// Packs the W blocks in the rollout's pair-major order: block index
// b = 2 (u (u + 1) + it) + side holds rows of tile t = 2u + side and columns of
// block column it (it <= 2u + 1); entries above the diagonal or beyond M are 0.
__global__ void pack_w_kernel(const double *W, int M, int Mpad, float4 *w32, uint4 *wbh, uint4 *wbl) {
    const int blk = blockIdx.x, lane = threadIdx.x;
    const int side = blk & 1, half_idx = blk >> 1;   // half_idx = u (u + 1) + it
    int u = 0;
    while ((u + 1) * (u + 2) <= half_idx) ++u;
    const int it = half_idx - u * (u + 1);
    const int t = 2 * u + side;
    const int i = 32 * t + (lane & 31);
    const int half = lane >> 5;
    auto wval = [&](int j) -> float {
        return (i < M && j < M && j <= i) ? (float)W[(size_t)i * Mpad + j] : 0.0f;
    };
    for (int q = 0; q < 4; ++q) {
        float4 v;
        v.x = wval(32 * it + 2 * (4 * q + 0) + half);
        v.y = wval(32 * it + 2 * (4 * q + 1) + half);
        v.z = wval(32 * it + 2 * (4 * q + 2) + half);
        v.w = wval(32 * it + 2 * (4 * q + 3) + half);
        w32[(size_t)blk * 256 + q * 64 + lane] = v;
    }
    for (int h = 0; h < 2; ++h) {
        uint16_t hi[8], lo[8];
        for (int e = 0; e < 8; ++e) {
            const float x = wval(32 * it + 16 * h + 8 * half + e);
            hi[e] = bf16_rne(x);
            lo[e] = bf16_rne(x - bf16_to_f32(hi[e]));
        }
        uint4 H, Lo;
        H.x = hi[0] | ((uint32_t)hi[1] << 16);
        H.y = hi[2] | ((uint32_t)hi[3] << 16);
        H.z = hi[4] | ((uint32_t)hi[5] << 16);
        H.w = hi[6] | ((uint32_t)hi[7] << 16);
        Lo.x = lo[0] | ((uint32_t)lo[1] << 16);
        Lo.y = lo[2] | ((uint32_t)lo[3] << 16);
        Lo.z = lo[4] | ((uint32_t)lo[5] << 16);
        Lo.w = lo[6] | ((uint32_t)lo[7] << 16);
        wbh[(size_t)blk * 128 + h * 64 + lane] = H;
        wbl[(size_t)blk * 128 + h * 64 + lane] = Lo;
    }
}

__global__ void pack_vec_kernel(const double *Z, const double *alpha, int M, int Mpad, double s0, double s1,
                                double s2, double s3, double c2, float *zs, float *al, float *zs2, float *cz) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= Mpad) return;
    double z[4] = {0.0, 0.0, 0.0, 0.0}, a = 0.0;
    if (j < M) {
        z[0] = Z[4 * j] * s0;
        z[1] = Z[4 * j + 1] * s1;
        z[2] = Z[4 * j + 2] * s2;
        z[3] = Z[4 * j + 3] * s3;
        a = alpha[j];
    }
    const float zf[4] = {(float)z[0], (float)z[1], (float)z[2], (float)z[3]};
    double zz = 0.0;
    for (int d = 0; d < 4; ++d) {
        zs[4 * j + d] = zf[d];
        zs2[4 * j + d] = 2.0f * zf[d];
        zz += (double)zf[d] * (double)zf[d];
    }
    al[j] = (float)a;
    cz[j] = (float)(c2 - zz);
}

// Three BF16 terms whose sum is the FP32 value x (round to nearest even at
// each stage; each remainder is exact in FP32).
__device__ __forceinline__ void split3_bf16(float x, uint16_t &h, uint16_t &m, uint16_t &l) {
    const __bf16 bh = (__bf16)x;
    const float r1 = x - (float)bh;
    const __bf16 bm = (__bf16)r1;
    const float r2 = r1 - (float)bm;
    const __bf16 bl = (__bf16)r2;
    __builtin_memcpy(&h, &bh, 2);
    __builtin_memcpy(&m, &bm, 2);
    __builtin_memcpy(&l, &bl, 2);
}

// A operands of the exponent products of the BF16 form.  For column tile jt
// the kernel-vector exponent of point j and sample s,
//   e_js = (c2 - |zs_j|^2) - |qs_s|^2 + sum_d (2 zs_jd) qs_sd,
// is the 32 x 32 product of two 32 x 32 x 16 matrix-core steps with the FP32
// factors split into three BF16 terms (h + m + l); the kept partial products
// hh, hm, mh, hl, mm, lh carry every bit down to 2^-24 of each factor:
//   step 0 slots:  0-3 zh   4-7 zh   8-11 zm   12-15 zh        (B: qh qm qh ql)
//   step 1 slots:  0-3 zm   4-7 zl   8-10 (c2 - |zs|^2) h m l, 11-13 one, 14-15 zero
//                                                              (B: qm qh 1 1 1 -qq h m l 0 0)
// Row rho of a tile holds point 32 jt + P(rho), P(8a + 4b + c) = 16 (a / 2) + 8 b + 4 (a % 2) + c,
// so that lane l of the product's accumulator (rows 8(r/4) + 4(l/32) + r%4) ends
// up with points 8 (l / 32) + r (r < 8) and 16 + 8 (l / 32) + r - 8: the k operand
// of the variance products in its lane order without any exchange.
// zop[(jt * 2 + step) * 64 + lane] = 8 BF16 slots 8 (lane / 32) .. + 7 of row lane % 32.
__global__ void pack_zop_kernel(const float *zs2, const float *cz, int Mpad, uint4 *zop) {
    const int NT = Mpad / 32;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NT * 128) return;
    const int lane = i & 63, step = (i >> 6) & 1, jt = i >> 7;
    const int rho = lane & 31, half = lane >> 5;
    const int a = rho >> 3, bb = (rho >> 2) & 1, c = rho & 3;
    const int j = 32 * jt + 16 * (a >> 1) + 8 * bb + 4 * (a & 1) + c;
    uint16_t zh[4], zm[4], zl[4], ch, cm, cl;
    for (int d = 0; d < 4; ++d) split3_bf16(zs2[4 * j + d], zh[d], zm[d], zl[d]);
    split3_bf16(cz[j], ch, cm, cl);
    const uint16_t one = 0x3f80;
    uint16_t slot[16];
    if (step == 0) {
        for (int d = 0; d < 4; ++d) {
            slot[d] = zh[d];
            slot[4 + d] = zh[d];
            slot[8 + d] = zm[d];
            slot[12 + d] = zh[d];
        }
    } else {
        for (int d = 0; d < 4; ++d) {
            slot[d] = zm[d];
            slot[4 + d] = zl[d];
        }
        slot[8] = ch;
        slot[9] = cm;
        slot[10] = cl;
        slot[11] = one;
        slot[12] = one;
        slot[13] = one;
        slot[14] = 0;
        slot[15] = 0;
    }
    const uint16_t *sv = slot + 8 * half;
    uint4 v;
    v.x = sv[0] | ((uint32_t)sv[1] << 16);
    v.y = sv[2] | ((uint32_t)sv[3] << 16);
    v.z = sv[4] | ((uint32_t)sv[5] << 16);
    v.w = sv[6] | ((uint32_t)sv[7] << 16);
    zop[i] = v;
}

hipError_t pack_gp_output(const GpBuildBuffers &b, int M, int Mpad, const double scale[4], double c2, uint4 *zop,
                          float *zs, float *alpha, float *zs2, float *cz, float4 *w32, uint4 *wbh, uint4 *wbl,
                          hipStream_t st) {
    const int NP = (Mpad / 32 + 1) / 2;
    hipLaunchKernelGGL(pack_w_kernel, dim3(2 * NP * (NP + 1)), dim3(64), 0, st, b.W, M, Mpad, w32, wbh, wbl);
    hipLaunchKernelGGL(pack_vec_kernel, dim3((Mpad + 255) / 256), dim3(256), 0, st, b.Z, b.alpha, M, Mpad,
                       scale[0], scale[1], scale[2], scale[3], c2, zs, alpha, zs2, cz);
    hipLaunchKernelGGL(pack_zop_kernel, dim3((Mpad / 32 * 128 + 255) / 256), dim3(256), 0, st, zs2, cz, Mpad, zop);
    return hipGetLastError();
}

}  // namespace gpmppi
