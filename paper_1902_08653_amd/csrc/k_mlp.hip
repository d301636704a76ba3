// k_mlp.hip -- the small per-coordinate MLP of the learned warm start.
//
// Three weight layers F -> H1 -> H2 -> 2 with ReLU between them; BF16 operands on
// gfx950's doubled-K MFMA (v_mfma_f32_16x16x32_bf16: 16 x 16 output, K = 32 per
// instruction, each lane holding 8 consecutive k of its row or column) with FP32
// accumulation; FP32 master weights and Adam state.  The GEMM is generic over strides so that one kernel serves the
// forward products, the weight gradients (A^T B) and the input gradients (A B^T).
#include <algorithm>

#include "common.hpp"
#include "launch.hpp"

namespace cdm {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// the MFMA fragment of 8 consecutive BF16 values at p (16-B aligned)
__device__ __forceinline__ bf16x8_t frag8(const unsigned short* p) { return *reinterpret_cast<const bf16x8_t*>(p); }
__device__ __forceinline__ f32x4_t mfma32(const bf16x8_t& a, const bf16x8_t& b, const f32x4_t& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}


// FP32 -> BF16 bits, round to nearest even, by gfx950's conversion instruction
// (v_cvt_pk_bf16_f32; a NaN stays a NaN)
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{lo, hi}, bf16x2_t));
}
__device__ __forceinline__ unsigned short f32_to_bf16(float f) {
    return __builtin_bit_cast(unsigned short, (__bf16)f);
}

// C[m][n] = sum_k A(m, k) B(k, n) (+ bias[n]); A(m, k) = A[m*sam + k*sak], B(k, n) = B[k*sbk + n*sbn];
// C row-major with leading dimension ldc.  64 x 64 tile per workgroup of 4 waves,
// each wave a 32 x 32 block of 2 x 2 MFMA 16 x 16 x 32 tiles.  beta: 0 overwrite, 1 accumulate.
constexpr int GT = 64;
constexpr int GK = 32;

__global__ __launch_bounds__(256) void k_gemm_bf16(const float* __restrict__ A, int64_t sam, int64_t sak,
                                                   const float* __restrict__ Bm, int64_t sbk, int64_t sbn,
                                                   float* __restrict__ C, int64_t ldc, int M, int N, int K,
                                                   const float* __restrict__ bias, int beta, int kc, int64_t zc,
                                                   int relu, const float* __restrict__ mask) {
    // split along K: workgroup z takes K range [z kc, z kc + kc) into C + z zc
    {
        const int z = blockIdx.z;
        A += (int64_t)z * kc * sak;
        Bm += (int64_t)z * kc * sbk;
        C += (int64_t)z * zc;
        K = min(kc, K - z * kc);
    }
    // both tiles k-fastest (a fragment is 8 consecutive k: one 16-B read); rows padded by
    // 8 values to keep the 16-B reads of a wave on distinct banks
    __shared__ __align__(16) unsigned short As[GT][GK + 8];
    __shared__ __align__(16) unsigned short Bs[GT][GK + 8];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    const int wm = (wid >> 1) * 32, wn = (wid & 1) * 32;
    f32x4_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += GK) {
        // stage A (64 x 32) and B (32 x 64) as BF16: 2048 elements each, 8 per thread
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int e = tid + 256 * q;
            const int am = e / GK, ak = e % GK;
            const int gm = m0 + am, gk = k0 + ak;
            As[am][ak] = (gm < M && gk < K) ? f32_to_bf16(A[(int64_t)gm * sam + (int64_t)gk * sak]) : (unsigned short)0;
            const int bk = e / GT, bn = e % GT;
            const int hk = k0 + bk, hn = n0 + bn;
            Bs[bn][bk] = (hk < K && hn < N) ? f32_to_bf16(Bm[(int64_t)hk * sbk + (int64_t)hn * sbn]) : (unsigned short)0;
        }
        __syncthreads();
        bf16x8_t a[2], b[2];
        const int kk = 8 * (lane >> 4);
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            a[i] = frag8(&As[wm + 16 * i + (lane & 15)][kk]);
            b[i] = frag8(&Bs[wn + 16 * i + (lane & 15)][kk]);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = mfma32(a[i], b[j], acc[i][j]);
        __syncthreads();
    }
    // D layout: lane -> column (lane & 15), rows 4 * (lane >> 4) + r
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
                const int gn = n0 + wn + 16 * j + (lane & 15);
                if (gm < M && gn < N) {
                    float v = acc[i][j][r];
                    if (bias) v += bias[gn];
                    if (relu) v = v > 0.f ? v : 0.f;
                    if (mask) v = mask[(int64_t)gm * ldc + gn] > 0.f ? v : 0.f;
                    float* cp = &C[(int64_t)gm * ldc + gn];
                    *cp = beta ? (*cp + v) : v;
                }
            }
}

// Large products (the training GEMMs): 128 x 128 tile per workgroup of 4 waves (each a
// 64 x 64 block of 4 x 4 MFMA tiles), K in chunks of 32 staged as BF16 in LDS with the next
// chunk's FP32 loads in flight during the current chunk's MFMAs.  Operands are read with
// 16-B loads along their contiguous dimension: AK = A contiguous in k (else in m), BN = B
// contiguous in n (else in k).  LDS keeps both tiles k-fastest, so an MFMA fragment (8
// consecutive k) is one 16-B read, and one 16 x 16 x 32 MFMA covers the chunk.
constexpr int G2T = 128, G2K = 32, G2P = G2K + 8;   // tile, K chunk, padded LDS row
template <bool AK, bool BN>
__global__ __launch_bounds__(256) void k_gemm2_bf16(const float* __restrict__ A, int64_t lda,
                                                    const float* __restrict__ Bm, int64_t ldb,
                                                    float* __restrict__ C, int64_t ldc, int M, int N, int K,
                                                    const float* __restrict__ bias, int beta, int kc, int64_t zc,
                                                    int relu, const float* __restrict__ mask) {
    // split along K: workgroup z takes K range [z kc, z kc + kc) into C + z zc
    {
        const int z = blockIdx.z;
        A += (int64_t)z * kc * (AK ? 1 : lda);
        Bm += (int64_t)z * kc * (BN ? ldb : 1);
        C += (int64_t)z * zc;
        K = min(kc, K - z * kc);
    }
    __shared__ __align__(16) unsigned short As[G2T][G2P];
    __shared__ __align__(16) unsigned short Bs[G2T][G2P];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int m0 = blockIdx.y * G2T, n0 = blockIdx.x * G2T;
    const int wm = (wid >> 1) * 64, wn = (wid & 1) * 64;
    // each thread moves 16 floats of A and 16 of B per chunk, as four 16-B loads along
    // the operand's contiguous dimension
    //   contiguous in k: row = tid / 2, k offset = (tid % 2) * 16
    //   contiguous in m or n: k = tid / 8, row offset = (tid % 8) * 16
    float4 ra[4], rb[4];
    auto load = [&](int k0) {
        if (AK) {
            const int r = tid >> 1, kk = k0 + (tid & 1) * 16;
            const int gm = m0 + r;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                ra[q] = (gm < M && kk + 4 * q < K) ? *reinterpret_cast<const float4*>(A + (int64_t)gm * lda + kk + 4 * q)
                                                   : make_float4(0.f, 0.f, 0.f, 0.f);
        } else {
            const int kk = k0 + (tid >> 3), mm = m0 + (tid & 7) * 16;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                ra[q] = (kk < K && mm + 4 * q < M) ? *reinterpret_cast<const float4*>(A + (int64_t)kk * lda + mm + 4 * q)
                                                   : make_float4(0.f, 0.f, 0.f, 0.f);
        }
        if (BN) {
            const int kk = k0 + (tid >> 3), nn = n0 + (tid & 7) * 16;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                rb[q] = (kk < K && nn + 4 * q < N) ? *reinterpret_cast<const float4*>(Bm + (int64_t)kk * ldb + nn + 4 * q)
                                                   : make_float4(0.f, 0.f, 0.f, 0.f);
        } else {
            const int r = tid >> 1, kk = k0 + (tid & 1) * 16;
            const int gn = n0 + r;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                rb[q] = (gn < N && kk + 4 * q < K) ? *reinterpret_cast<const float4*>(Bm + (int64_t)gn * ldb + kk + 4 * q)
                                                   : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    auto store = [&]() {
        if (AK) {   // 4 consecutive k per float4: two packed BF16 pairs, one 8-B store
            const int r = tid >> 1, kk = (tid & 1) * 16;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                *reinterpret_cast<uint2*>(&As[r][kk + 4 * q]) =
                    make_uint2(pack_bf16x2(ra[q].x, ra[q].y), pack_bf16x2(ra[q].z, ra[q].w));
        } else {
            const int kk = tid >> 3, mm = (tid & 7) * 16;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                As[mm + 4 * q + 0][kk] = f32_to_bf16(ra[q].x);
                As[mm + 4 * q + 1][kk] = f32_to_bf16(ra[q].y);
                As[mm + 4 * q + 2][kk] = f32_to_bf16(ra[q].z);
                As[mm + 4 * q + 3][kk] = f32_to_bf16(ra[q].w);
            }
        }
        if (BN) {
            const int kk = tid >> 3, nn = (tid & 7) * 16;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                Bs[nn + 4 * q + 0][kk] = f32_to_bf16(rb[q].x);
                Bs[nn + 4 * q + 1][kk] = f32_to_bf16(rb[q].y);
                Bs[nn + 4 * q + 2][kk] = f32_to_bf16(rb[q].z);
                Bs[nn + 4 * q + 3][kk] = f32_to_bf16(rb[q].w);
            }
        } else {    // B contiguous in k: packed like A
            const int r = tid >> 1, kk = (tid & 1) * 16;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                *reinterpret_cast<uint2*>(&Bs[r][kk + 4 * q]) =
                    make_uint2(pack_bf16x2(rb[q].x, rb[q].y), pack_bf16x2(rb[q].z, rb[q].w));
        }
    };
    f32x4_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    const int kq = 8 * (lane >> 4);
    load(0);
    for (int k0 = 0; k0 < K; k0 += G2K) {
        __syncthreads();   // the previous chunk's MFMAs are done with the tiles
        store();
        __syncthreads();
        if (k0 + G2K < K) load(k0 + G2K);
        bf16x8_t a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            a[i] = frag8(&As[wm + 16 * i + (lane & 15)][kq]);
            b[i] = frag8(&Bs[wn + 16 * i + (lane & 15)][kq]);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = mfma32(a[i], b[j], acc[i][j]);
    }
    // D layout: lane -> column (lane & 15), rows 4 * (lane >> 4) + r
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
                const int gn = n0 + wn + 16 * j + (lane & 15);
                if (gm < M && gn < N) {
                    float v = acc[i][j][r];
                    if (bias) v += bias[gn];
                    if (relu) v = v > 0.f ? v : 0.f;
                    if (mask) v = mask[(int64_t)gm * ldc + gn] > 0.f ? v : 0.f;
                    float* cp = &C[(int64_t)gm * ldc + gn];
                    *cp = beta ? (*cp + v) : v;
                }
            }
}

// S > 1: S splits of K (chunks of kc, a multiple of 32) side by side, split z writing C + z zc
static hipError_t gemm_bf16_one(const float* A, int64_t sam, int64_t sak, const float* B, int64_t sbk, int64_t sbn,
                                float* C, int64_t ldc, int M, int N, int K, const float* bias, int beta, hipStream_t st,
                                int S = 1, int kc = 0, int64_t zc = 0, int relu = 0, const float* mask = nullptr) {
    if (S == 1) kc = K;
    // the tiled kernel: large products whose operands are contiguous along one dimension,
    // with 16-B aligned rows (K, M, N multiples of 4 where they are contiguous)
    const bool big = M >= G2T && N >= G2T && kc >= G2K;
    const bool ak = sak == 1, am = sam == 1, bn = sbn == 1, bk = sbk == 1;
    auto al = [](const void* p, int64_t ld) { return ((uintptr_t)p % 16 == 0) && (ld % 4 == 0); };
    if (big && (ak || am) && (bn || bk) && (K % 4 == 0) && (M % 4 == 0) && (N % 4 == 0)) {
        const int64_t lda = ak ? sam : sak, ldb = bn ? sbk : sbn;
        if (al(A, lda) && al(B, ldb)) {
            const dim3 g((N + G2T - 1) / G2T, (M + G2T - 1) / G2T, S);
            if (ak && bn) hipLaunchKernelGGL((k_gemm2_bf16<true, true>), g, dim3(256), 0, st, A, lda, B, ldb, C, ldc, M, N, K, bias, beta, kc, zc, relu, mask);
            else if (ak) hipLaunchKernelGGL((k_gemm2_bf16<true, false>), g, dim3(256), 0, st, A, lda, B, ldb, C, ldc, M, N, K, bias, beta, kc, zc, relu, mask);
            else if (bn) hipLaunchKernelGGL((k_gemm2_bf16<false, true>), g, dim3(256), 0, st, A, lda, B, ldb, C, ldc, M, N, K, bias, beta, kc, zc, relu, mask);
            else hipLaunchKernelGGL((k_gemm2_bf16<false, false>), g, dim3(256), 0, st, A, lda, B, ldb, C, ldc, M, N, K, bias, beta, kc, zc, relu, mask);
            return hipGetLastError();
        }
    }
    dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT, S);
    hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, st, A, sam, sak, B, sbk, sbn, C, ldc, M, N, K, bias, beta, kc, zc,
                       relu, mask);
    return hipGetLastError();
}

// split-K finish: C = sum_s part[s] (fixed order) (+ bias), then relu or the mask
// [mask > 0] (leading dimension ldc) where given, (+ C if beta)
__global__ void k_splitk_sum(const float* __restrict__ part, int S, int M, int N, float* __restrict__ C, int64_t ldc,
                             const float* __restrict__ bias, int beta, int relu, const float* __restrict__ mask) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)M * N) return;
    const int m = (int)(e / N), n = (int)(e % N);
    float v = 0.f;
    for (int k = 0; k < S; ++k) v += part[(int64_t)k * M * N + e];
    if (bias) v += bias[n];
    if (relu) v = v > 0.f ? v : 0.f;
    if (mask) v = mask[(int64_t)m * ldc + n] > 0.f ? v : 0.f;
    float* cp = &C[(int64_t)m * ldc + n];
    *cp = beta ? (*cp + v) : v;
}

// C = A B (+ bias) (+ C): products with a long K and few output tiles (the weight
// gradients, K = rows) are split along K into S chunks computed side by side into
// `splitk` (S * M * N floats), then summed in chunk order.
hipError_t launch_gemm_bf16(const float* A, int64_t sam, int64_t sak, const float* B, int64_t sbk, int64_t sbn, float* C,
                            int64_t ldc, int M, int N, int K, const float* bias, int beta, hipStream_t st,
                            float* splitk, int64_t splitk_floats, int relu = 0, const float* mask = nullptr) {
    const int64_t tiles = (int64_t)((M + 63) / 64) * ((N + 63) / 64);
    int S = 1;
    if (splitk && K >= 4096 && tiles < 256) {
        S = (int)std::min<int64_t>(std::min<int64_t>(64, K / 256), splitk_floats / ((int64_t)M * N));
        S = std::max(S, 1);
    }
    if (S == 1) return gemm_bf16_one(A, sam, sak, B, sbk, sbn, C, ldc, M, N, K, bias, beta, st, 1, 0, 0, relu, mask);
    const int chunk = ((K + S - 1) / S + 31) / 32 * 32;   // multiple of the tiled kernel's K chunk
    const int s = (K + chunk - 1) / chunk;
    hipError_t e = gemm_bf16_one(A, sam, sak, B, sbk, sbn, splitk, N, M, N, K, nullptr, 0, st, s, chunk, (int64_t)M * N);
    if (e != hipSuccess) return e;
    const int64_t mn = (int64_t)M * N;
    hipLaunchKernelGGL(k_splitk_sum, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, st, (const float*)splitk, s, M,
                       N, C, ldc, bias, beta, relu, mask);
    return hipGetLastError();
}

// A = relu(Z)
__global__ void k_relu(const float* __restrict__ Z, float* __restrict__ A, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) A[i] = Z[i] > 0.f ? Z[i] : 0.f;
}
// dZ = dA * [Z > 0]
__global__ void k_relu_bwd(const float* __restrict__ Z, const float* __restrict__ dA, float* __restrict__ dZ, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dZ[i] = Z[i] > 0.f ? dA[i] : 0.f;
}
// dO = 2 (O - T) / (N * nout); per-block partial sums of (O - T)^2
__global__ void k_mse(const float* __restrict__ O, const float* __restrict__ Tg, float* __restrict__ dO, int64_t n,
                      float scale, float* __restrict__ part) {
    __shared__ float s[256];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float e = 0.f;
    if (i < n) {
        const float d = O[i] - Tg[i];
        dO[i] = 2.f * d * scale;
        e = d * d;
    }
    s[threadIdx.x] = e;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}
// Column sums of an M x N row-major matrix (bias gradients) in two fixed-order stages:
// workgroup (bx, by) sums rows [by R, (by + 1) R) of columns 64 bx .. 64 bx + 63 (four row
// lanes per column, combined in order) into part[by][n]; k_colsum_fin adds the CS_SPLIT
// partials of each column in order.
constexpr int CS_SPLIT = 64;
__global__ __launch_bounds__(256) void k_colsum(const float* __restrict__ X, int M, int N, float* __restrict__ part) {
    __shared__ float s[4][64];
    const int c = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int n = blockIdx.x * 64 + c;
    const int R = (M + CS_SPLIT - 1) / CS_SPLIT;
    const int m0 = blockIdx.y * R, m1 = min(M, m0 + R);
    float acc = 0.f;
    if (n < N)
        for (int m = m0 + q; m < m1; m += 4) acc += X[(int64_t)m * N + n];
    s[q][c] = acc;
    __syncthreads();
    if (q == 0 && n < N) part[(int64_t)blockIdx.y * N + n] = ((s[0][c] + s[1][c]) + s[2][c]) + s[3][c];
}
__global__ void k_colsum_fin(const float* __restrict__ part, int N, float* __restrict__ out) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float acc = 0.f;
    for (int k = 0; k < CS_SPLIT; ++k) acc += part[(int64_t)k * N + n];
    out[n] = acc;
}
// Adam (bias-corrected), FP32 master weights
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m1, float* __restrict__ m2,
                       int64_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.f - b1) * gi;
    const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = b;
    w[i] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

hipError_t launch_relu(const float* Z, float* A, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_relu, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, Z, A, n);
    return hipGetLastError();
}
hipError_t launch_relu_bwd(const float* Z, const float* dA, float* dZ, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_relu_bwd, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, Z, dA, dZ, n);
    return hipGetLastError();
}
hipError_t launch_mse(const float* O, const float* T, float* dO, int64_t n, float scale, float* part, hipStream_t st) {
    hipLaunchKernelGGL(k_mse, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, O, T, dO, n, scale, part);
    return hipGetLastError();
}
// part: CS_SPLIT * N floats of scratch
hipError_t launch_colsum(const float* X, int M, int N, float* out, float* part, hipStream_t st) {
    hipLaunchKernelGGL(k_colsum, dim3((N + 63) / 64, CS_SPLIT), dim3(256), 0, st, X, M, N, part);
    hipLaunchKernelGGL(k_colsum_fin, dim3((N + 255) / 256), dim3(256), 0, st, (const float*)part, N, out);
    return hipGetLastError();
}
hipError_t launch_adam(float* w, const float* g, float* m1, float* m2, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t st) {
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, w, g, m1, m2, n, lr, b1, b2, eps,
                       c1, c2);
    return hipGetLastError();
}

// ---- the narrow layers (nin <= 16 inputs, nout <= 4 outputs) on VALU -------------
// A GEMM of inner dimension 8 or output width 2 leaves the matrix cores idle and is
// bound by the activations it reads or writes, so these layers are plain loops with the
// tile GEMMs' arithmetic (BF16 operands, FP32 accumulation), fused with the ReLU, the
// ReLU mask of the backward pass and the bias gradients (FP32, as the column sums).
constexpr int NL_MAXIN = 16, NL_MAXOUT = 4, NL_RB = 32;
// the value of x rounded to BF16 (nearest even, the conversion the tile GEMMs use): every
// product operand is rounded as in the matrix-core layers, and the product of two BF16
// values is exact in FP32
__device__ __forceinline__ float bfr(float x) { return __uint_as_float((uint32_t)f32_to_bf16(x) << 16); }

// A1 = relu(X W1 + b1): workgroup -> 64 columns x NL_RB rows; thread -> column c0 + (tid
// & 63), rows q, q + 4, ... of the block (q = tid >> 6); the block's rows of X in LDS
__global__ __launch_bounds__(256) void k_nl_in_fwd(const float* __restrict__ X, const float* __restrict__ W1,
                                                   const float* __restrict__ b1, float* __restrict__ A1, int rows,
                                                   int nin, int h1) {
    __shared__ float xs[NL_RB][NL_MAXIN];
    const int c = blockIdx.x * 64 + (threadIdx.x & 63), q = threadIdx.x >> 6;
    const int rb = blockIdx.y * NL_RB;
    for (int e = threadIdx.x; e < NL_RB * NL_MAXIN; e += 256) {
        const int r = e / NL_MAXIN, k = e % NL_MAXIN;
        xs[r][k] = (rb + r < rows && k < nin) ? bfr(X[(int64_t)(rb + r) * nin + k]) : 0.f;
    }
    __syncthreads();
    if (c >= h1) return;
    float w[NL_MAXIN];
#pragma unroll
    for (int k = 0; k < NL_MAXIN; ++k) w[k] = k < nin ? bfr(W1[(int64_t)k * h1 + c]) : 0.f;
    const float b = b1[c];
    for (int r = q; r < NL_RB && rb + r < rows; r += 4) {
        float v = b;
#pragma unroll
        for (int k = 0; k < NL_MAXIN; ++k) v += xs[r][k] * w[k];
        A1[(int64_t)(rb + r) * h1 + c] = v > 0.f ? v : 0.f;
    }
}
// O = A2 W3 + b3: one wave per row, lanes striding the hidden units
__global__ __launch_bounds__(256) void k_nl_out_fwd(const float* __restrict__ A2, const float* __restrict__ W3,
                                                    const float* __restrict__ b3, float* __restrict__ O, int rows,
                                                    int h2, int nout) {
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (r >= rows) return;
    float acc[NL_MAXOUT] = {0.f, 0.f, 0.f, 0.f};
    for (int i = lane; i < h2; i += 64) {
        const float a = bfr(A2[(int64_t)r * h2 + i]);
#pragma unroll
        for (int j = 0; j < NL_MAXOUT; ++j)
            if (j < nout) acc[j] += a * bfr(W3[(int64_t)i * nout + j]);
    }
#pragma unroll
    for (int j = 0; j < NL_MAXOUT; ++j) {
        float v = acc[j];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (j < nout && lane == 0) O[(int64_t)r * nout + j] = v + b3[j];
    }
}
// Output layer backward: dZ2 = (dO W3^T) * [A2 > 0].  Workgroup (bx, by): hidden units
// 64 bx .. 64 bx + 63 over row split `by`; thread -> unit i = 64 bx + (tid & 63) and rows
// q, q + 4, ... of the split (q = tid >> 6).  The four row groups' sums of A2^T dO are
// combined in order in LDS into part[by][i][j]; the column sums of dO (bias gradient) of
// the split go to part[nsplit * h2 * nout + by * nout + j] from the workgroup bx = 0.
__global__ __launch_bounds__(256) void k_nl_out_bwd(const float* __restrict__ A2, const float* __restrict__ dO,
                                                    const float* __restrict__ W3, float* __restrict__ dZ2,
                                                    float* __restrict__ part, int rows, int h2, int nout, int rps) {
    __shared__ float red[4][64][NL_MAXOUT];
    __shared__ float redb[4][64][NL_MAXOUT];
    const int lc = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + lc, by = blockIdx.y, nsplit = gridDim.y;
    const bool on = i < h2;
    float w[NL_MAXOUT], aw[NL_MAXOUT] = {0.f, 0.f, 0.f, 0.f}, ab[NL_MAXOUT] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < NL_MAXOUT; ++j) w[j] = (on && j < nout) ? bfr(W3[(int64_t)i * nout + j]) : 0.f;
    const int r0 = by * rps, r1 = min(rows, r0 + rps);
    for (int r = r0 + q; r < r1; r += 4) {
        const float a = on ? A2[(int64_t)r * h2 + i] : 0.f, a16 = bfr(a);
        float d = 0.f;
#pragma unroll
        for (int j = 0; j < NL_MAXOUT; ++j)
            if (j < nout) {
                const float o = dO[(int64_t)r * nout + j], o16 = bfr(o);
                d += o16 * w[j];
                aw[j] += a16 * o16;
                ab[j] += o;
            }
        if (on) dZ2[(int64_t)r * h2 + i] = a > 0.f ? d : 0.f;
    }
#pragma unroll
    for (int j = 0; j < NL_MAXOUT; ++j) {
        red[q][lc][j] = aw[j];
        redb[q][lc][j] = ab[j];
    }
    __syncthreads();
    if (q == 0 && on) {
#pragma unroll
        for (int j = 0; j < NL_MAXOUT; ++j)
            if (j < nout) {
                part[((int64_t)by * h2 + i) * nout + j] = ((red[0][lc][j] + red[1][lc][j]) + red[2][lc][j]) + red[3][lc][j];
                if (i == 0)
                    part[(int64_t)nsplit * h2 * nout + by * nout + j] =
                        ((redb[0][lc][j] + redb[1][lc][j]) + redb[2][lc][j]) + redb[3][lc][j];
            }
    }
}
// Input layer backward: X^T dZ1 (nin x h1) and the column sums of dZ1, per row split, into
// part[by][k][c] (k = nin: the bias row).  Workgroup (bx, by): hidden units 64 bx .. + 63;
// thread -> unit c and rows q, q + 4, ... of the split, combined in order in LDS.
__global__ __launch_bounds__(256) void k_nl_in_bwd(const float* __restrict__ X, const float* __restrict__ dZ1,
                                                   float* __restrict__ part, int rows, int nin, int h1, int rps) {
    __shared__ float red[4][NL_MAXIN + 1][64];
    const int lc = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + lc, by = blockIdx.y;
    const bool on = c < h1;
    float acc[NL_MAXIN + 1];
#pragma unroll
    for (int k = 0; k <= NL_MAXIN; ++k) acc[k] = 0.f;
    const int r0 = by * rps, r1 = min(rows, r0 + rps);
    for (int r = r0 + q; r < r1; r += 4) {
        const float d = on ? dZ1[(int64_t)r * h1 + c] : 0.f, d16 = bfr(d);
#pragma unroll
        for (int k = 0; k < NL_MAXIN; ++k)
            if (k < nin) acc[k] += bfr(X[(int64_t)r * nin + k]) * d16;
        acc[NL_MAXIN] += d;
    }
#pragma unroll
    for (int k = 0; k <= NL_MAXIN; ++k) red[q][k][lc] = acc[k];
    __syncthreads();
    if (q != 0 || !on) return;
    float* pb = part + (int64_t)by * (nin + 1) * h1;
#pragma unroll
    for (int k = 0; k <= NL_MAXIN; ++k) {
        const int kk = k < nin ? k : (k == NL_MAXIN ? nin : -1);
        if (kk >= 0) pb[(int64_t)kk * h1 + c] = ((red[0][k][lc] + red[1][k][lc]) + red[2][k][lc]) + red[3][k][lc];
    }
}
// out[e] = sum over the nsplit partial copies (stride n) of part, in a fixed order: four
// thread groups take copies q, q + 4, ... (q = tid >> 6) of 64 consecutive elements,
// combined in order in LDS
__global__ __launch_bounds__(256) void k_nl_sum(const float* __restrict__ part, int nsplit, int64_t n,
                                                float* __restrict__ out) {
    __shared__ float red[4][64];
    const int lc = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int64_t e = (int64_t)blockIdx.x * 64 + lc;
    float v = 0.f;
    if (e < n) {
#pragma unroll 8
        for (int k = q; k < nsplit; k += 4) v += part[(int64_t)k * n + e];
    }
    red[q][lc] = v;
    __syncthreads();
    if (q == 0 && e < n) out[e] = ((red[0][lc] + red[1][lc]) + red[2][lc]) + red[3][lc];
}

// ---- per-coordinate features of a packed uneven batch --------------------------
// One wave per (instance, user): z = h_u^H y / (||h_u||^2 + lambda) (regularised
// matched filter), e = ||h_u||^2.  Row layout (NF = 8 floats):
//   [Re z, Im z, |z|, e, lambda, m/2048, n/m, 1]
template <typename V>
__global__ __launch_bounds__(256) void k_features(const V* __restrict__ H, const V* __restrict__ Y,
                                                  const WgJob* __restrict__ jobs, const int64_t* __restrict__ row_off,
                                                  int njobs, double lambda, float* __restrict__ F) {
    const int lane = threadIdx.x & 63;
    const int64_t gw = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    // locate (job, user) by a binary search over the row offsets
    int lo = 0, hi = njobs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (row_off[mid] <= gw) lo = mid;
        else hi = mid;
    }
    const WgJob jb = jobs[lo];
    const int64_t u = gw - row_off[lo];
    if (lo >= njobs || u >= jb.n || u < 0) return;
    const V* h = H + jb.h_off + u * jb.ld;
    const V* y = Y + jb.y_off;
    double gr = 0.0, gi = 0.0, e = 0.0;
    for (int i = lane; i < jb.m; i += 64) {
        const V hv = h[i], yv = y[i];
        gr += (double)hv.x * yv.x + (double)hv.y * yv.y;
        gi += (double)hv.x * yv.y - (double)hv.y * yv.x;
        e += (double)hv.x * hv.x + (double)hv.y * hv.y;
    }
    gr = wave_allsum(gr);
    gi = wave_allsum(gi);
    e = wave_allsum(e);
    if (lane == 0) {
        const double den = e + lambda;
        const double zr = den > 0.0 ? gr / den : 0.0, zi = den > 0.0 ? gi / den : 0.0;
        float* f = F + gw * 8;
        f[0] = (float)zr;
        f[1] = (float)zi;
        f[2] = (float)sqrt(zr * zr + zi * zi);
        f[3] = (float)e;
        f[4] = (float)lambda;
        f[5] = (float)jb.m / 2048.f;
        f[6] = (float)jb.n / (float)jb.m;
        f[7] = 1.f;
    }
}

hipError_t launch_features(bool c128, const void* H, const void* Y, const WgJob* jobs, const int64_t* row_off,
                           int njobs, int64_t nrows, double lambda, float* F, hipStream_t st) {
    if (c128)
        hipLaunchKernelGGL(k_features<double2>, dim3((unsigned)((nrows + 3) / 4)), dim3(256), 0, st,
                           (const double2*)H, (const double2*)Y, jobs, row_off, njobs, lambda, F);
    else
        hipLaunchKernelGGL(k_features<float2>, dim3((unsigned)((nrows + 3) / 4)), dim3(256), 0, st, (const float2*)H,
                           (const float2*)Y, jobs, row_off, njobs, lambda, F);
    return hipGetLastError();
}

// (rows x 2) FP32 network output -> interleaved complex warm start
template <typename V>
__global__ void k_out_complex(const float2* __restrict__ O, V* __restrict__ x, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const float2 o = O[i];
        V v;
        v.x = o.x;
        v.y = o.y;
        x[i] = v;
    }
}

hipError_t launch_out_complex(const float* O, void* x, int64_t n, bool c128, hipStream_t st) {
    const dim3 grid((unsigned)((n + 255) / 256));
    if (c128)
        hipLaunchKernelGGL(k_out_complex<double2>, grid, dim3(256), 0, st, (const float2*)O, (double2*)x, n);
    else
        hipLaunchKernelGGL(k_out_complex<float2>, grid, dim3(256), 0, st, (const float2*)O, (float2*)x, n);
    return hipGetLastError();
}

// ---- fused inference (warm-start prediction) -------------------------------------
// One launch evaluates the whole network for a tile of MI_R rows, with the same
// operand rounding as the layered forward pass (BF16 operands, FP32 accumulation):
//   layer 1 (nin <= 16, VALU): A1 = relu(bf16(X) bf16(W1) + b1), kept as BF16 in LDS;
//   layer 2 (MFMA 16x16x32): Z2 = A1 bf16(W2) + b2 by column blocks of 64 (one 16-column
//            slice per wave), B fragments straight from a transposed BF16 copy of W2;
//   layer 3 in the epilogue of each block: Y += bf16(relu(Z2)) bf16(W3), reduced over the
//            slice's 16 lanes and kept per wave in LDS; the waves' sums are added in a
//            fixed order at the end and written as the complex warm start.
// Only the activations of one tile ever exist, in LDS: nothing but X and x0 touches HBM.
constexpr int MI_R = 128;      // rows per workgroup
constexpr int MI_NT = 256;     // 4 waves

// packed inference weights: W1 and W3 as BF16-rounded FP32, W2 transposed as BF16 bits
__global__ void k_mlp_pack(const float* __restrict__ w, int nin, int hid, int64_t oW1, int64_t oW2, int64_t oW3,
                           float* __restrict__ w1r, unsigned short* __restrict__ w2t, float* __restrict__ w3r) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t hh = (int64_t)hid * hid;
    if (i < hh) {
        const int n = (int)(i / hid), k = (int)(i % hid);   // w2t[n][k] = W2[k][n]
        w2t[i] = f32_to_bf16(w[oW2 + (int64_t)k * hid + n]);
    }
    if (i < (int64_t)nin * hid) w1r[i] = __uint_as_float((uint32_t)f32_to_bf16(w[oW1 + i]) << 16);
    if (i < (int64_t)hid * 2) w3r[i] = __uint_as_float((uint32_t)f32_to_bf16(w[oW3 + i]) << 16);
}

template <int HID, typename V>
__global__ __launch_bounds__(MI_NT) void k_mlp_infer(const float* __restrict__ X, int64_t rows, int nin,
                                                     const float* __restrict__ w1r, const float* __restrict__ b1,
                                                     const unsigned short* __restrict__ w2t,
                                                     const float* __restrict__ b2, const float* __restrict__ w3r,
                                                     const float* __restrict__ b3, V* __restrict__ x0) {
    constexpr int LDA = HID + 8;                     // BF16 row stride of A1 (16 B pad: conflict-free b64 reads)
    extern __shared__ unsigned char smem_raw[];
    unsigned short* A1 = reinterpret_cast<unsigned short*>(smem_raw);           // [MI_R][LDA]
    float* xs = reinterpret_cast<float*>(A1 + MI_R * LDA);                      // [MI_R][16] BF16-rounded X
    float* yp = xs + MI_R * 16;                                                 // [4 waves][MI_R][2]
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * MI_R;
    // ---- stage X (rows past the end read as 0) and clear the layer-3 partials
    for (int e = tid; e < MI_R * 16; e += MI_NT) {
        const int r = e >> 4, k = e & 15;
        const float v = (k < nin && r0 + r < rows) ? X[(r0 + r) * nin + k] : 0.f;
        xs[e] = __uint_as_float((uint32_t)f32_to_bf16(v) << 16);
    }
    for (int e = tid; e < 4 * MI_R * 2; e += MI_NT) yp[e] = 0.f;
    __syncthreads();
    // ---- layer 1: thread t owns columns 2t', 2t'+1 (t' = t, t + 256, ... while < HID/2)
    for (int cp = tid; cp < HID / 2; cp += MI_NT) {
        const int c = 2 * cp;
        float wa[16], wb[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            wa[k] = k < nin ? w1r[(int64_t)k * HID + c] : 0.f;
            wb[k] = k < nin ? w1r[(int64_t)k * HID + c + 1] : 0.f;
        }
        const float ba = b1[c], bb = b1[c + 1];
        for (int r = 0; r < MI_R; ++r) {
            float za = 0.f, zb = 0.f;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const float xv = xs[r * 16 + k];
                za += xv * wa[k];
                zb += xv * wb[k];
            }
            za += ba;
            zb += bb;
            const uint32_t pa = f32_to_bf16(za > 0.f ? za : 0.f), pb = f32_to_bf16(zb > 0.f ? zb : 0.f);
            *reinterpret_cast<uint32_t*>(&A1[r * LDA + c]) = pa | (pb << 16);
        }
    }
    __syncthreads();
    // ---- layers 2 and 3
    const int kq = 8 * (lane >> 4);                  // this lane's k offset inside a 32-step
    float y0[MI_R / 16][4], y1[MI_R / 16][4];        // layer-3 partials of this lane's rows
#pragma unroll
    for (int i = 0; i < MI_R / 16; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) y0[i][r] = y1[i][r] = 0.f;
    for (int nb = 0; nb < HID; nb += 64) {
        const int col = nb + 16 * wid + (lane & 15);
        const unsigned short* bsrc = w2t + (int64_t)col * HID + kq;
        f32x4_t acc[MI_R / 16];
#pragma unroll
        for (int i = 0; i < MI_R / 16; ++i) acc[i] = f32x4_t{0.f, 0.f, 0.f, 0.f};
        // B fragments in groups of 4 thirty-two-steps of K: the next group's 4 loads are in
        // flight while the current group's MFMAs run (one L2 round trip per group)
        constexpr int GRP = 4;
        bf16x8_t cur[GRP], nxt[GRP];
#pragma unroll
        for (int k = 0; k < GRP; ++k) cur[k] = frag8(bsrc + 32 * k);
#pragma unroll 1
        for (int k0 = 0; k0 < HID; k0 += 32 * GRP) {
            if (k0 + 32 * GRP < HID) {
#pragma unroll
                for (int k = 0; k < GRP; ++k) nxt[k] = frag8(bsrc + k0 + 32 * GRP + 32 * k);
            }
#pragma unroll
            for (int k = 0; k < GRP; ++k) {
#pragma unroll
                for (int i = 0; i < MI_R / 16; ++i)
                    acc[i] = mfma32(frag8(&A1[(16 * i + (lane & 15)) * LDA + k0 + 32 * k + kq]), cur[k], acc[i]);
            }
#pragma unroll
            for (int k = 0; k < GRP; ++k) cur[k] = nxt[k];
        }
        // epilogue: lane holds Z2[16 i + 4 (lane >> 4) + r][col]
        const float bz = b2[col];
        const float wo0 = w3r[(int64_t)col * 2], wo1 = w3r[(int64_t)col * 2 + 1];
#pragma unroll
        for (int i = 0; i < MI_R / 16; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float z = acc[i][r] + bz;
                const float a2 = __uint_as_float((uint32_t)f32_to_bf16(z > 0.f ? z : 0.f) << 16);
                y0[i][r] += a2 * wo0;
                y1[i][r] += a2 * wo1;
            }
    }
    // sum over the 16 lanes of each row group (the wave's columns), then per wave into LDS
#pragma unroll
    for (int i = 0; i < MI_R / 16; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float a = y0[i][r], b = y1[i][r];
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) {
                a += __shfl_xor(a, o);
                b += __shfl_xor(b, o);
            }
            if ((lane & 15) == 0) {
                const int row = 16 * i + 4 * (lane >> 4) + r;
                yp[(wid * MI_R + row) * 2 + 0] = a;
                yp[(wid * MI_R + row) * 2 + 1] = b;
            }
        }
    __syncthreads();
    if (tid < MI_R && r0 + tid < rows) {
        float o0 = b3[0], o1 = b3[1];
        float s0 = 0.f, s1 = 0.f;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            s0 += yp[(w * MI_R + tid) * 2 + 0];
            s1 += yp[(w * MI_R + tid) * 2 + 1];
        }
        V v;
        v.x = s0 + o0;
        v.y = s1 + o1;
        x0[r0 + tid] = v;
    }
}

size_t mlp_infer_lds(int hid) { return (size_t)MI_R * (hid + 8) * 2 + (size_t)MI_R * 16 * 4 + 4 * MI_R * 2 * 4; }

// hid in {256, 512}; nin <= 16; nout = 2
hipError_t launch_mlp_infer(const float* w, int nin, int hid, int64_t oW1, int64_t ob1, int64_t oW2, int64_t ob2,
                            int64_t oW3, int64_t ob3, float* w1r, unsigned short* w2t, float* w3r, const float* X,
                            int64_t rows, void* x0, bool c128, hipStream_t st) {
    const int64_t pk = std::max<int64_t>((int64_t)hid * hid, (int64_t)nin * hid);
    hipLaunchKernelGGL(k_mlp_pack, dim3((unsigned)((pk + 255) / 256)), dim3(256), 0, st, w, nin, hid, oW1, oW2, oW3,
                       w1r, w2t, w3r);
    const size_t lds = mlp_infer_lds(hid);
    const dim3 grid((unsigned)((rows + MI_R - 1) / MI_R));
#define CDM_MI_LAUNCH(H_, V_)                                                                                     \
    do {                                                                                                         \
        hipError_t e_ = hipFuncSetAttribute((const void*)k_mlp_infer<H_, V_>,                                    \
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);               \
        if (e_ != hipSuccess) return e_;                                                                         \
        hipLaunchKernelGGL((k_mlp_infer<H_, V_>), grid, dim3(MI_NT), lds, st, X, rows, nin, w1r, w + ob1, w2t,   \
                           w + ob2, w3r, w + ob3, (V_*)x0);                                                      \
    } while (0)
    if (hid == 512) {
        if (c128) CDM_MI_LAUNCH(512, double2);
        else CDM_MI_LAUNCH(512, float2);
    } else if (hid == 256) {
        if (c128) CDM_MI_LAUNCH(256, double2);
        else CDM_MI_LAUNCH(256, float2);
    } else {
        return hipErrorInvalidValue;
    }
#undef CDM_MI_LAUNCH
    return hipGetLastError();
}

}  // namespace cdm

// ============================================================================
// C ABI of the warm-start MLP (host side)
// ============================================================================
namespace {
struct Mlp {
    int nin, h1, h2, nout, max_rows;
    int64_t nparam;
    float *w = nullptr, *g = nullptr, *m1 = nullptr, *m2 = nullptr;
    float *Z1, *A1, *Z2, *A2, *O, *dO, *dA2, *dZ2, *dA1, *dZ1, *part;
    float* cpart = nullptr;                   // column-sum partials (CS_SPLIT x widest layer)
    float* splitk = nullptr;                  // split-K partial products of the weight gradients
    int64_t splitk_floats = 0;
    float *w1r = nullptr, *w3r = nullptr;     // fused inference: BF16-rounded W1, W3
    unsigned short* w2t = nullptr;            // and W2 transposed as BF16
    bool fused = false;                       // shape served by k_mlp_infer
    void* ws = nullptr;
    int64_t step = 0;
    // parameter block offsets: W1 b1 W2 b2 W3 b3
    int64_t oW1, ob1, oW2, ob2, oW3, ob3;
};
thread_local char g_mlp_err[256] = "";
}  // namespace

struct cdm_mlp : Mlp {};

using namespace cdm;

#define MLP_TRY(call)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess) {                                                             \
            snprintf(g_mlp_err, sizeof(g_mlp_err), "%s: %s", #call, hipGetErrorString(e_)); \
            return CDM_EHIP;                                                                \
        }                                                                                   \
    } while (0)

// The narrow-layer path (nin <= 16, nout <= 4): the input and output layers on the
// kernels above, the hidden layer's ReLU in its GEMM's epilogue, and the ReLU masks of
// the backward pass taken from the activations (A > 0 exactly where Z > 0), so Z1 and Z2
// are not formed; their buffers hold the split partials of the weight gradients.
static bool mlp_narrow(const cdm_mlp* n) { return n->nin <= NL_MAXIN && n->nout <= NL_MAXOUT; }
static int mlp_splits(int rows, int64_t per_split, int64_t cap) {
    // row splits for the gradient partials (64 rows each, at most 256), within `cap`
    // floats of scratch
    int64_t s = std::min<int64_t>(256, std::max<int64_t>(1, rows / 64));
    s = std::min<int64_t>(s, std::max<int64_t>(1, cap / per_split));
    return (int)s;
}

static hipError_t mlp_forward(cdm_mlp* n, const float* X, int rows, hipStream_t st) {
    hipError_t e;
    float* w = n->w;
    if (mlp_narrow(n)) {
        hipLaunchKernelGGL(k_nl_in_fwd, dim3((n->h1 + 63) / 64, (rows + NL_RB - 1) / NL_RB), dim3(256), 0, st, X,
                           (const float*)(w + n->oW1), (const float*)(w + n->ob1), n->A1, rows, n->nin, n->h1);
        if ((e = hipGetLastError())) return e;
        if ((e = launch_gemm_bf16(n->A1, n->h1, 1, w + n->oW2, n->h2, 1, n->A2, n->h2, rows, n->h2, n->h1, w + n->ob2, 0, st,
                                  n->splitk, n->splitk_floats, 1, nullptr)))
            return e;
        hipLaunchKernelGGL(k_nl_out_fwd, dim3((rows + 3) / 4), dim3(256), 0, st, (const float*)n->A2,
                           (const float*)(w + n->oW3), (const float*)(w + n->ob3), n->O, rows, n->h2, n->nout);
        return hipGetLastError();
    }
    if ((e = launch_gemm_bf16(X, n->nin, 1, w + n->oW1, n->h1, 1, n->Z1, n->h1, rows, n->h1, n->nin, w + n->ob1, 0, st, n->splitk, n->splitk_floats)))
        return e;
    if ((e = launch_relu(n->Z1, n->A1, (int64_t)rows * n->h1, st))) return e;
    if ((e = launch_gemm_bf16(n->A1, n->h1, 1, w + n->oW2, n->h2, 1, n->Z2, n->h2, rows, n->h2, n->h1, w + n->ob2, 0, st, n->splitk, n->splitk_floats)))
        return e;
    if ((e = launch_relu(n->Z2, n->A2, (int64_t)rows * n->h2, st))) return e;
    return launch_gemm_bf16(n->A2, n->h2, 1, w + n->oW3, n->nout, 1, n->O, n->nout, rows, n->nout, n->h2, w + n->ob3,
                            0, st, n->splitk, n->splitk_floats);
}

// gradients of the mean squared error (1 / (rows * nout)) sum (O - T)^2 into n->g
static hipError_t mlp_backward(cdm_mlp* n, const float* X, const float* T, int rows, hipStream_t st) {
    hipError_t e;
    float* w = n->w;
    float* g = n->g;
    const int64_t no = (int64_t)rows * n->nout;
    if ((e = launch_mse(n->O, T, n->dO, no, 1.f / (float)no, n->part, st))) return e;
    if (mlp_narrow(n)) {
        const int64_t cap3 = (int64_t)n->max_rows * n->h2, cap1 = (int64_t)n->max_rows * n->h1;
        // layer 3: dZ2, the weight and bias gradient partials (scratch: Z2)
        const int s3 = mlp_splits(rows, (int64_t)n->h2 * n->nout + n->nout, cap3);
        const int rps3 = (rows + s3 - 1) / s3;
        hipLaunchKernelGGL(k_nl_out_bwd, dim3((n->h2 + 63) / 64, s3), dim3(256), 0, st, (const float*)n->A2,
                           (const float*)n->dO, (const float*)(w + n->oW3), n->dZ2, n->Z2, rows, n->h2, n->nout, rps3);
        if ((e = hipGetLastError())) return e;
        const int64_t n3 = (int64_t)n->h2 * n->nout;
        hipLaunchKernelGGL(k_nl_sum, dim3((unsigned)((n3 + 63) / 64)), dim3(256), 0, st, (const float*)n->Z2, s3, n3,
                           g + n->oW3);
        hipLaunchKernelGGL(k_nl_sum, dim3(1), dim3(256), 0, st, (const float*)(n->Z2 + (int64_t)s3 * n3), s3,
                           (int64_t)n->nout, g + n->ob3);
        if ((e = hipGetLastError())) return e;
        // layer 2 (matrix cores): weight gradient, bias gradient, dZ1 = (dZ2 W2^T) * [A1 > 0]
        if ((e = launch_gemm_bf16(n->A1, 1, n->h1, n->dZ2, n->h2, 1, g + n->oW2, n->h2, n->h1, n->h2, rows, nullptr, 0, st,
                                  n->splitk, n->splitk_floats)))
            return e;
        if ((e = launch_colsum(n->dZ2, rows, n->h2, g + n->ob2, n->cpart, st))) return e;
        if ((e = launch_gemm_bf16(n->dZ2, n->h2, 1, w + n->oW2, 1, n->h2, n->dZ1, n->h1, rows, n->h1, n->h2, nullptr, 0, st,
                                  n->splitk, n->splitk_floats, 0, n->A1)))
            return e;
        // layer 1: weight and bias gradient partials (scratch: Z1)
        const int s1 = mlp_splits(rows, (int64_t)(n->nin + 1) * n->h1, cap1);
        const int rps1 = (rows + s1 - 1) / s1;
        hipLaunchKernelGGL(k_nl_in_bwd, dim3((n->h1 + 63) / 64, s1), dim3(256), 0, st, X, (const float*)n->dZ1, n->Z1,
                           rows, n->nin, n->h1, rps1);
        if ((e = hipGetLastError())) return e;
        const int64_t n1 = (int64_t)(n->nin + 1) * n->h1;   // W1 (nin x h1) then b1 (h1): contiguous in g
        hipLaunchKernelGGL(k_nl_sum, dim3((unsigned)((n1 + 63) / 64)), dim3(256), 0, st, (const float*)n->Z1, s1, n1,
                           g + n->oW1);
        return hipGetLastError();
    }
    // layer 3
    if ((e = launch_gemm_bf16(n->A2, 1, n->h2, n->dO, n->nout, 1, g + n->oW3, n->nout, n->h2, n->nout, rows, nullptr, 0, st, n->splitk, n->splitk_floats)))
        return e;
    if ((e = launch_colsum(n->dO, rows, n->nout, g + n->ob3, n->cpart, st))) return e;
    if ((e = launch_gemm_bf16(n->dO, n->nout, 1, w + n->oW3, 1, n->nout, n->dA2, n->h2, rows, n->h2, n->nout, nullptr, 0, st, n->splitk, n->splitk_floats)))
        return e;
    if ((e = launch_relu_bwd(n->Z2, n->dA2, n->dZ2, (int64_t)rows * n->h2, st))) return e;
    // layer 2
    if ((e = launch_gemm_bf16(n->A1, 1, n->h1, n->dZ2, n->h2, 1, g + n->oW2, n->h2, n->h1, n->h2, rows, nullptr, 0, st, n->splitk, n->splitk_floats)))
        return e;
    if ((e = launch_colsum(n->dZ2, rows, n->h2, g + n->ob2, n->cpart, st))) return e;
    if ((e = launch_gemm_bf16(n->dZ2, n->h2, 1, w + n->oW2, 1, n->h2, n->dA1, n->h1, rows, n->h1, n->h2, nullptr, 0, st, n->splitk, n->splitk_floats)))
        return e;
    if ((e = launch_relu_bwd(n->Z1, n->dA1, n->dZ1, (int64_t)rows * n->h1, st))) return e;
    // layer 1
    if ((e = launch_gemm_bf16(X, 1, n->nin, n->dZ1, n->h1, 1, g + n->oW1, n->h1, n->nin, n->h1, rows, nullptr, 0, st, n->splitk, n->splitk_floats)))
        return e;
    return launch_colsum(n->dZ1, rows, n->h1, g + n->ob1, n->cpart, st);
}

extern "C" {

int32_t cdm_mlp_create(int32_t nin, int32_t h1, int32_t h2, int32_t nout, int32_t max_rows, cdm_mlp** out) {
    if (!out) return CDM_EINVAL;
    *out = nullptr;
    if (nin < 1 || h1 < 1 || h2 < 1 || nout < 1 || max_rows < 1) return CDM_ESHAPE;
    cdm_mlp* n = new cdm_mlp();
    n->nin = nin;
    n->h1 = h1;
    n->h2 = h2;
    n->nout = nout;
    n->max_rows = max_rows;
    n->oW1 = 0;
    n->ob1 = n->oW1 + (int64_t)nin * h1;
    n->oW2 = n->ob1 + h1;
    n->ob2 = n->oW2 + (int64_t)h1 * h2;
    n->oW3 = n->ob2 + h2;
    n->ob3 = n->oW3 + (int64_t)h2 * nout;
    n->nparam = n->ob3 + nout;
    const int64_t R = max_rows;
    n->fused = nin <= 16 && h1 == h2 && (h1 == 256 || h1 == 512) && nout == 2;
    // fused inference weights: nin*h1 + 2*h2 floats and h1*h2 BF16 (as floats: half of it)
    const int64_t fw = n->fused ? (int64_t)nin * h1 + 2 * (int64_t)h2 + ((int64_t)h1 * h2 + 1) / 2 + 64 : 0;
    const int64_t wmax = std::max<int64_t>(std::max(h1, h2), nout);
    // split-K scratch: up to 64 partial copies of the largest weight block
    const int64_t wblk = std::max<int64_t>(std::max<int64_t>((int64_t)nin * h1, (int64_t)h1 * h2), (int64_t)h2 * nout);
    const int64_t skf = (R >= 4096) ? std::min<int64_t>(64, R / 256) * wblk : 0;
    const int64_t fl = 4 * n->nparam + R * (4 * (int64_t)h1 + 4 * (int64_t)h2 + 2 * nout) + (R * nout + 255) / 256 + 64 + fw +
                       CS_SPLIT * wmax + skf + 64;
    if (hipMalloc(&n->ws, sizeof(float) * fl) != hipSuccess) {
        delete n;
        return CDM_ENOMEM;
    }
    float* p = (float*)n->ws;
    n->w = p; p += n->nparam;
    n->g = p; p += n->nparam;
    n->m1 = p; p += n->nparam;
    n->m2 = p; p += n->nparam;
    n->Z1 = p; p += R * h1;
    n->A1 = p; p += R * h1;
    n->dA1 = p; p += R * h1;
    n->dZ1 = p; p += R * h1;
    n->Z2 = p; p += R * h2;
    n->A2 = p; p += R * h2;
    n->dA2 = p; p += R * h2;
    n->dZ2 = p; p += R * h2;
    n->O = p; p += R * nout;
    n->dO = p; p += R * nout;
    n->part = p; p += (R * nout + 255) / 256 + 64;
    n->cpart = p; p += CS_SPLIT * wmax;
    n->splitk = skf ? p : nullptr;
    n->splitk_floats = skf;
    p += skf;
    if (n->fused) {
        n->w1r = p; p += (int64_t)nin * h1;
        n->w3r = p; p += 2 * (int64_t)h2 + 64;
        n->w2t = reinterpret_cast<unsigned short*>(p);
    }
    if (hipMemset(n->m1, 0, sizeof(float) * 2 * n->nparam) != hipSuccess) {
        (void)hipFree(n->ws);
        delete n;
        return CDM_EHIP;
    }
    *out = n;
    return CDM_OK;
}

int64_t cdm_mlp_param_count(const cdm_mlp* n) { return n ? n->nparam : -1; }

int32_t cdm_mlp_set_weights(cdm_mlp* n, const float* host, int64_t count) {
    if (!n || !host || count != n->nparam) return CDM_EINVAL;
    MLP_TRY(hipMemcpy(n->w, host, sizeof(float) * count, hipMemcpyHostToDevice));
    MLP_TRY(hipMemset(n->m1, 0, sizeof(float) * 2 * n->nparam));
    n->step = 0;
    return CDM_OK;
}

int32_t cdm_mlp_get_weights(const cdm_mlp* n, float* host, int64_t count) {
    if (!n || !host || count != n->nparam) return CDM_EINVAL;
    MLP_TRY(hipMemcpy(host, n->w, sizeof(float) * count, hipMemcpyDeviceToHost));
    return CDM_OK;
}

int32_t cdm_mlp_forward(cdm_mlp* n, const float* X, int32_t rows, float* Y, void* stream) {
    if (!n || !X || rows < 1 || rows > n->max_rows) return CDM_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    MLP_TRY(mlp_forward(n, X, rows, st));
    if (Y) MLP_TRY(hipMemcpyAsync(Y, n->O, sizeof(float) * (size_t)rows * n->nout, hipMemcpyDeviceToDevice, st));
    return CDM_OK;
}

int32_t cdm_mlp_gradients(cdm_mlp* n, const float* X, const float* T, int32_t rows, float* grads, float* loss_parts,
                          void* stream) {
    if (!n || !X || !T || rows < 1 || rows > n->max_rows) return CDM_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    MLP_TRY(mlp_forward(n, X, rows, st));
    MLP_TRY(mlp_backward(n, X, T, rows, st));
    if (grads) MLP_TRY(hipMemcpyAsync(grads, n->g, sizeof(float) * n->nparam, hipMemcpyDeviceToDevice, st));
    if (loss_parts)
        MLP_TRY(hipMemcpyAsync(loss_parts, n->part, sizeof(float) * (((size_t)rows * n->nout + 255) / 256),
                               hipMemcpyDeviceToDevice, st));
    return CDM_OK;
}

int32_t cdm_mlp_train_step(cdm_mlp* n, const float* X, const float* T, int32_t rows, float lr, void* stream) {
    if (!n || !X || !T || rows < 1 || rows > n->max_rows || !(lr > 0.f)) return CDM_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    MLP_TRY(mlp_forward(n, X, rows, st));
    MLP_TRY(mlp_backward(n, X, T, rows, st));
    n->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)n->step), c2 = 1.f - powf(b2, (float)n->step);
    MLP_TRY(launch_adam(n->w, n->g, n->m1, n->m2, n->nparam, lr, b1, b2, 1e-8f, c1, c2, st));
    return CDM_OK;
}

int32_t cdm_mlp_predict(cdm_mlp* n, const float* X, int64_t rows, void* x0, int32_t precision, void* stream) {
    if (!n || !X || !x0 || rows < 1 || n->nout != 2) return CDM_EINVAL;
    if (precision != CDM_C128 && precision != CDM_C64) return CDM_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const bool c128 = precision == CDM_C128;
    const size_t esz = c128 ? 16 : 8;
    if (n->fused) {   // one launch, activations in LDS only
        MLP_TRY(launch_mlp_infer(n->w, n->nin, n->h1, n->oW1, n->ob1, n->oW2, n->ob2, n->oW3, n->ob3, n->w1r, n->w2t,
                                 n->w3r, X, rows, x0, c128, st));
        return CDM_OK;
    }
    for (int64_t r0 = 0; r0 < rows; r0 += n->max_rows) {
        const int cnt = (int)std::min<int64_t>(n->max_rows, rows - r0);
        MLP_TRY(mlp_forward(n, X + r0 * n->nin, cnt, st));
        MLP_TRY(launch_out_complex(n->O, (char*)x0 + r0 * esz, cnt, c128, st));
    }
    return CDM_OK;
}

int32_t cdm_mlp_destroy(cdm_mlp* n) {
    if (!n) return CDM_OK;
    if (n->ws) (void)hipFree(n->ws);
    delete n;
    return CDM_OK;
}

}  // extern "C"
