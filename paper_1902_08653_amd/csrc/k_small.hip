// k_small.hip -- decentralized detection and precoding of many small clustered problems.
//
// The shape of the paper's throughput measurements (Sec. VI): S subcarriers, each with a
// channel H_s (B x U, B = C * B_c antennas in C clusters) shared by V received vectors.
// For every (s, v) each cluster c runs T sweeps of Algorithm 1 on its rows
// (H_{s,c}, y_{s,v,c}) from x = 0, and the C local estimates are fused (Sec. III):
//   x_hat = sum_c lambda_c x_c,  lambda_c = sigma_c^-2 / sum_c' sigma_c'^-2,
//   sigma_c^2 = (N0 / U) sum_u m_{u,c}  (N0/U cancels: lambda_c = s_c^-1 / sum s_c'^-1).
// Mapping: a quad of lanes per (subcarrier, cluster, vector) task.  A cluster is at most
// 32 x 16, so lane j of the quad keeps rows j, j + 4, ... (8 at most) of the residual and
// the task's U coordinates in registers; the coordinate dot is a quad reduction (two
// DPP quad swaps, equal bits in all four lanes).
// The channel of a workgroup's subcarriers is staged once in LDS and read there by
// every task of the same cluster (broadcast reads, padded so that neighbouring clusters
// fall in different banks).  Fusion of the C estimates of a vector goes through LDS.
// Precisions: complex64 (FP32), or complex FP16 (two halves per 32-bit word, the paper's
// format): the residual and channel in FP16, the dot products as packed FP16 products
// with FP32 accumulation (v_dot2_f32_f16), the residual update as packed FP16 fused
// multiply-adds; the per-coordinate scalar rule runs in FP32 in both.
#include <hip/hip_fp16.h>

#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "launch.hpp"

namespace cdm {

constexpr int SM_NT = 256;
constexpr int SM_LPT = 4;             // lanes per task
constexpr int SM_RPL = 8;             // rows per lane
constexpr int SM_BMAX = SM_LPT * SM_RPL;   // antennas per cluster at most
constexpr int SM_UMAX = 16;           // users per cluster at most
constexpr size_t SM_LDS = 64 * 1024;  // LDS budget of one workgroup
// Vectors per quad (VQ): with two, a lane runs two independent chains that share each
// channel read -- more work in flight per wave, half as many waves.  Chosen per launch.

template <bool F16> struct SmNum;
template <> struct SmNum<false> {
    using E = float2;       // stored complex value
    __device__ static E zero() { return make_float2(0.f, 0.f); }
    __device__ static float2 to_f(E e) { return e; }
    __device__ static E from_f(float2 f) { return f; }
    // acc += conj(h) r
    __device__ static void dot_acc(float2& acc, E h, E r) {
        acc.x += h.x * r.x + h.y * r.y;
        acc.y += h.x * r.y - h.y * r.x;
    }
    // r -= h d
    __device__ static void axpy(E& r, E h, float2 d) {
        r.x -= h.x * d.x - h.y * d.y;
        r.y -= h.x * d.y + h.y * d.x;
    }
};
template <> struct SmNum<true> {
    using E = __half2;      // (re, im)
    __device__ static E zero() { return __float2half2_rn(0.f); }
    __device__ static float2 to_f(E e) { return __half22float2(e); }
    __device__ static E from_f(float2 f) { return __floats2half2_rn(f.x, f.y); }
    __device__ static void dot_acc(float2& acc, E h, E r) {
        // Re += hr rr + hi ri;  Im += hr ri - hi rr = (-hi, hr) . (rr, ri)
        typedef _Float16 h2v __attribute__((ext_vector_type(2)));
        h2v hv, rv, sv;
        __builtin_memcpy(&hv, &h, 4);
        __builtin_memcpy(&rv, &r, 4);
        sv.x = -hv.y;
        sv.y = hv.x;
        acc.x = __builtin_amdgcn_fdot2(hv, rv, acc.x, false);
        acc.y = __builtin_amdgcn_fdot2(sv, rv, acc.y, false);
    }
    __device__ static void axpy(E& r, E h, float2 d) {
        // r.re -= hr dr - hi di,  r.im -= hi dr + hr di
        const __half2 a = __floats2half2_rn(-d.x, -d.x);
        const __half2 b = __floats2half2_rn(d.y, -d.y);
        r = __hfma2(h, a, r);
        r = __hfma2(__lowhigh2highlow(h), b, r);
    }
};

// Sum over the 4 lanes of a quad; every lane of the quad ends with the same bits.
__device__ __forceinline__ float quad_sum(float v) {
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xb1, 0xf, 0xf, false));  // [1,0,3,2]
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4e, 0xf, 0xf, false));  // [2,3,0,1]
    return v;
}

// LDS layout of one workgroup (NS subcarriers):
//   channel  [NS][C] blocks of UMAX x 32 complex (row i of user u at u * 32 + i), each
//            block padded by 16 B so that neighbouring blocks start in different banks
//   x_c      [NS][C][V][UMAX] FP32 complex
//   sum m    [NS][C] FP32
template <int UMAX> __host__ __device__ constexpr int sm_block(bool f16) {
    return UMAX * SM_BMAX + (f16 ? 4 : 2);   // elements
}
template <int UMAX> static size_t sm_lds_bytes(int NS, int C, int V, bool f16) {
    const size_t esz = f16 ? 4 : 8;
    return (size_t)NS * C * sm_block<UMAX>(f16) * esz + (size_t)NS * C * V * UMAX * 8 + (size_t)NS * C * 4;
}

template <bool F16, int UMAX, int VQ>
__global__ __launch_bounds__(SM_NT) void k_detect_small(const typename SmNum<F16>::E* __restrict__ H,
                                                        const typename SmNum<F16>::E* __restrict__ Y,
                                                        typename SmNum<F16>::E* __restrict__ X, int S, int V, int C,
                                                        int Bc, int U, int T, float lambda, int NS) {
    using N = SmNum<F16>;
    using E = typename N::E;
    constexpr int BLK = sm_block<UMAX>(F16);
    extern __shared__ __align__(16) unsigned char smem[];
    E* Hl = reinterpret_cast<E*>(smem);
    float2* xl = reinterpret_cast<float2*>(Hl + NS * C * BLK);
    float* wl = reinterpret_cast<float*>(xl + NS * C * V * UMAX);
    const int tid = threadIdx.x;
    const int s0 = blockIdx.x * NS;
    const int ns = min(NS, S - s0);
    const int B = C * Bc;
    // ---- stage the channel (zero rows past Bc and users past U)
    for (int e = tid; e < ns * C * UMAX * SM_BMAX; e += SM_NT) {
        const int i = e % SM_BMAX, u = (e / SM_BMAX) % UMAX, k = e / (SM_BMAX * UMAX);   // k = sub * C + c
        const int sub = k / C, c = k % C;
        E v = N::zero();
        if (i < Bc && u < U) v = H[(int64_t)(s0 + sub) * B * U + (int64_t)u * B + c * Bc + i];
        Hl[k * BLK + u * SM_BMAX + i] = v;
    }
    __syncthreads();
    // ---- one task per quad: T sweeps of Algorithm 1 on (H_{s,c}, y_{s,v,c}).  The loop
    // bound is the same for the four lanes of a quad, so a quad is always whole.
    const int VP = (V + VQ - 1) / VQ;
    const int tasks = ns * C * VP;
    const int j = tid % SM_LPT;
    for (int t = tid / SM_LPT; t < tasks; t += SM_NT / SM_LPT) {
        const int sub = t / (C * VP), rem = t % (C * VP);
        const int c = rem / VP, v0 = (rem % VP) * VQ;
        const E* hb = Hl + (sub * C + c) * BLK + j;     // this lane's rows: j + 4 k
        // the residuals of vectors v0, v0 + 1 (a vector past V is carried as zeros)
        E r[VQ][SM_RPL];
#pragma unroll
        for (int q = 0; q < VQ; ++q) {
            const int v = v0 + q;
            const E* yv = Y + ((int64_t)(s0 + sub) * V + min(v, V - 1)) * B + c * Bc;
#pragma unroll
            for (int k = 0; k < SM_RPL; ++k) {
                const int i = j + SM_LPT * k;
                r[q][k] = (i < Bc && v < V) ? yv[i] : N::zero();
            }
        }
        // Algorithm 1 preprocessing: m_u = 1/(||h_u||^2 + lambda), n_u = m_u ||h_u||^2 (FP32;
        // a column with ||h_u||^2 + lambda == 0 stays inactive: (0, 1))
        float mu[UMAX], nu[UMAX];
        float msum = 0.f;
#pragma unroll
        for (int u = 0; u < UMAX; ++u) {
            float e = 0.f;
#pragma unroll
            for (int k = 0; k < SM_RPL; ++k) {
                const float2 hf = N::to_f(hb[u * SM_BMAX + SM_LPT * k]);
                e += hf.x * hf.x + hf.y * hf.y;
            }
            e = quad_sum(e);
            const bool act = u < U && e + lambda > 0.f;
            mu[u] = act ? 1.f / (e + lambda) : 0.f;
            nu[u] = act ? mu[u] * e : 1.f;
            if (u < U) msum += mu[u];
        }
        float2 x[VQ][UMAX];
#pragma unroll
        for (int q = 0; q < VQ; ++q)
#pragma unroll
            for (int u = 0; u < UMAX; ++u) x[q][u] = make_float2(0.f, 0.f);
        for (int it = 0; it < T; ++it) {
#pragma unroll
            for (int u = 0; u < UMAX; ++u) {
                if (u < U) {
                    E h[SM_RPL];
#pragma unroll
                    for (int k = 0; k < SM_RPL; ++k) h[k] = hb[u * SM_BMAX + SM_LPT * k];
                    float2 g[VQ];
#pragma unroll
                    for (int q = 0; q < VQ; ++q) {
                        g[q] = make_float2(0.f, 0.f);
#pragma unroll
                        for (int k = 0; k < SM_RPL; ++k) N::dot_acc(g[q], h[k], r[q][k]);
                    }
#pragma unroll
                    for (int q = 0; q < VQ; ++q) {
                        g[q].x = quad_sum(g[q].x);
                        g[q].y = quad_sum(g[q].y);
                    }
#pragma unroll
                    for (int q = 0; q < VQ; ++q) {
                        const float2 xn = make_float2(mu[u] * g[q].x + nu[u] * x[q][u].x,
                                                      mu[u] * g[q].y + nu[u] * x[q][u].y);
                        const float2 d = make_float2(xn.x - x[q][u].x, xn.y - x[q][u].y);
                        x[q][u] = xn;
#pragma unroll
                        for (int k = 0; k < SM_RPL; ++k) N::axpy(r[q][k], h[k], d);
                    }
                }
            }
        }
        if (j == 0) {
#pragma unroll
            for (int q = 0; q < VQ; ++q) {
                const int v = v0 + q;
                if (v < V) {
                    float2* xo = xl + ((sub * C + c) * V + v) * UMAX;
#pragma unroll
                    for (int u = 0; u < UMAX; ++u) xo[u] = x[q][u];
                }
            }
            if (v0 == 0) wl[sub * C + c] = msum;
        }
    }
    __syncthreads();
    // ---- fusion: one thread per (subcarrier, vector, user), clusters in order
    for (int e = tid; e < ns * V * U; e += SM_NT) {
        const int u = e % U, v = (e / U) % V, sub = e / (U * V);
        // lambda_c = s_c^-1 / sum_c' s_c'^-1 with s_c = sum_u m_{u,c} (the factor N0/U of
        // sigma_c^2 cancels); a cluster without an active coordinate (s_c = 0) gets 0
        float tot = 0.f;
        for (int k = 0; k < C; ++k) {
            const float sk = wl[sub * C + k];
            tot += sk > 0.f ? 1.f / sk : 0.f;
        }
        float2 acc = make_float2(0.f, 0.f);
        for (int k = 0; k < C; ++k) {
            const float sk = wl[sub * C + k];
            const float w = (sk > 0.f && tot > 0.f) ? (1.f / sk) / tot : 0.f;
            const float2 xc = xl[((sub * C + k) * V + v) * UMAX + u];
            acc.x += w * xc.x;
            acc.y += w * xc.y;
        }
        X[((int64_t)(s0 + sub) * V + v) * U + u] = N::from_f(acc);
    }
}

// Two vectors per quad pay off for FP16 when they still leave at least four waves per SIMD
// of the whole chip (measured on the paper's shapes: FP16 with 8 clusters gains, every
// FP32 shape and FP16 with 4 clusters do not)
static int sm_vectors_per_quad(bool f16, int S, int C, int V) {
    const int64_t waves2 = (int64_t)S * C * ((V + 1) / 2) * SM_LPT / 64;
    return (f16 && waves2 >= 4 * 1024) ? 2 : 1;
}

template <bool F16, int UMAX, int VQ>
static hipError_t launch_small_vq(const void* H, const void* Y, void* X, int S, int V, int C, int Bc, int U, int T,
                                  float lam, hipStream_t st) {
    using E = typename SmNum<F16>::E;
    // subcarriers per workgroup: enough tasks to fill the 64 quads, within the LDS budget
    const int VP = (V + VQ - 1) / VQ;
    int NS = std::max(1, SM_NT / SM_LPT / (C * VP));
    while (NS > 1 && sm_lds_bytes<UMAX>(NS, C, V, F16) > SM_LDS) --NS;
    const size_t lds = sm_lds_bytes<UMAX>(NS, C, V, F16);
    if (lds > SM_LDS) return hipErrorInvalidValue;   // within the default dynamic LDS limit
    const int blocks = (S + NS - 1) / NS;
    hipLaunchKernelGGL((k_detect_small<F16, UMAX, VQ>), dim3(blocks), dim3(SM_NT), lds, st, (const E*)H,
                       (const E*)Y, (E*)X, S, V, C, Bc, U, T, lam, NS);
    return hipGetLastError();
}
template <bool F16, int UMAX>
static hipError_t launch_small(const void* H, const void* Y, void* X, int S, int V, int C, int Bc, int U, int T,
                               float lam, hipStream_t st) {
    return sm_vectors_per_quad(F16, S, C, V) == 2
               ? launch_small_vq<F16, UMAX, 2>(H, Y, X, S, V, C, Bc, U, T, lam, st)
               : launch_small_vq<F16, UMAX, 1>(H, Y, X, S, V, C, Bc, U, T, lam, st);
}

// ---- downlink: Algorithm 2 on the same shape ---------------------------------------
// For every (s, v) each cluster c runs T sweeps of eq. (4) on its rows from x_c = 0
// with the broadcast symbols s_{s,v}: with p_u = 1/||h_{u,c}|| and sbar_u = p_u s_u,
//   e = p_u h_{u,c}^H x_c - sbar_u,   x_c <- x_c - e p_u h_{u,c},
// then scales x_c to norm rho_c = rho / sqrt(C) (Sec. IV-B; rho <= 0: no scaling).
// The output of (s, v) is the stacked [x_1; ...; x_C] (B entries).  Same mapping as the
// detector (a quad per task, lane j holding rows j, j + 4, ... of x_c), no fusion step.
template <int UMAX> static size_t sm_pre_lds_bytes(int NS, int C, bool f16) {
    return (size_t)NS * C * sm_block<UMAX>(f16) * (f16 ? 4 : 8);
}

template <bool F16, int UMAX, int VQ>
__global__ __launch_bounds__(SM_NT) void k_precode_small(const typename SmNum<F16>::E* __restrict__ H,
                                                         const typename SmNum<F16>::E* __restrict__ Sym,
                                                         typename SmNum<F16>::E* __restrict__ X, int S, int V, int C,
                                                         int Bc, int U, int T, float rho_c, int NS) {
    using N = SmNum<F16>;
    using E = typename N::E;
    constexpr int BLK = sm_block<UMAX>(F16);
    extern __shared__ __align__(16) unsigned char smem[];
    E* Hl = reinterpret_cast<E*>(smem);
    const int tid = threadIdx.x;
    const int s0 = blockIdx.x * NS;
    const int ns = min(NS, S - s0);
    const int B = C * Bc;
    for (int e = tid; e < ns * C * UMAX * SM_BMAX; e += SM_NT) {
        const int i = e % SM_BMAX, u = (e / SM_BMAX) % UMAX, k = e / (SM_BMAX * UMAX);
        const int sub = k / C, c = k % C;
        E v = N::zero();
        if (i < Bc && u < U) v = H[(int64_t)(s0 + sub) * B * U + (int64_t)u * B + c * Bc + i];
        Hl[k * BLK + u * SM_BMAX + i] = v;
    }
    __syncthreads();
    const int VP = (V + VQ - 1) / VQ;
    const int tasks = ns * C * VP;
    const int j = tid % SM_LPT;
    for (int t = tid / SM_LPT; t < tasks; t += SM_NT / SM_LPT) {
        const int sub = t / (C * VP), rem = t % (C * VP);
        const int c = rem / VP, v0 = (rem % VP) * VQ;
        const E* hb = Hl + (sub * C + c) * BLK + j;
        // preprocessing (FP32): p_u = 1/||h_u|| (a zero column stays inactive), and sbar_u
        // of vectors v0, v0 + 1 (a vector past V is carried as zeros)
        float pu[UMAX];
        float2 sb[VQ][UMAX];
#pragma unroll
        for (int u = 0; u < UMAX; ++u) {
            float e = 0.f;
#pragma unroll
            for (int k = 0; k < SM_RPL; ++k) {
                const float2 hf = N::to_f(hb[u * SM_BMAX + SM_LPT * k]);
                e += hf.x * hf.x + hf.y * hf.y;
            }
            e = quad_sum(e);
            pu[u] = (u < U && e > 0.f) ? 1.f / sqrtf(e) : 0.f;
#pragma unroll
            for (int q = 0; q < VQ; ++q) {
                const int v = v0 + q;
                const E* sv = Sym + ((int64_t)(s0 + sub) * V + min(v, V - 1)) * U;
                const float2 su = (u < U && v < V) ? N::to_f(sv[u]) : make_float2(0.f, 0.f);
                sb[q][u] = make_float2(pu[u] * su.x, pu[u] * su.y);
            }
        }
        E x[VQ][SM_RPL];
#pragma unroll
        for (int q = 0; q < VQ; ++q)
#pragma unroll
            for (int k = 0; k < SM_RPL; ++k) x[q][k] = N::zero();
        for (int it = 0; it < T; ++it) {
#pragma unroll
            for (int u = 0; u < UMAX; ++u) {
                if (pu[u] != 0.f) {   // equal in the four lanes of the quad
                    E h[SM_RPL];
#pragma unroll
                    for (int k = 0; k < SM_RPL; ++k) h[k] = hb[u * SM_BMAX + SM_LPT * k];
                    float2 g[VQ];
#pragma unroll
                    for (int q = 0; q < VQ; ++q) {
                        g[q] = make_float2(0.f, 0.f);
#pragma unroll
                        for (int k = 0; k < SM_RPL; ++k) N::dot_acc(g[q], h[k], x[q][k]);
                    }
#pragma unroll
                    for (int q = 0; q < VQ; ++q) {
                        g[q].x = quad_sum(g[q].x);
                        g[q].y = quad_sum(g[q].y);
                    }
#pragma unroll
                    for (int q = 0; q < VQ; ++q) {
                        const float2 d = make_float2(pu[u] * (pu[u] * g[q].x - sb[q][u].x),
                                                     pu[u] * (pu[u] * g[q].y - sb[q][u].y));
#pragma unroll
                        for (int k = 0; k < SM_RPL; ++k) N::axpy(x[q][k], h[k], d);
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < VQ; ++q) {
            const int v = v0 + q;
            if (rho_c > 0.f) {
                float nn = 0.f;
#pragma unroll
                for (int k = 0; k < SM_RPL; ++k) {
                    const float2 xf = N::to_f(x[q][k]);
                    nn += xf.x * xf.x + xf.y * xf.y;
                }
                nn = quad_sum(nn);
                if (nn > 0.f) {
                    const float sc = rho_c / sqrtf(nn);
#pragma unroll
                    for (int k = 0; k < SM_RPL; ++k) {
                        const float2 xf = N::to_f(x[q][k]);
                        x[q][k] = N::from_f(make_float2(sc * xf.x, sc * xf.y));
                    }
                }
            }
            if (v < V) {
                E* xo = X + ((int64_t)(s0 + sub) * V + v) * B + c * Bc;
#pragma unroll
                for (int k = 0; k < SM_RPL; ++k) {
                    const int i = j + SM_LPT * k;
                    if (i < Bc) xo[i] = x[q][k];
                }
            }
        }
    }
}

template <bool F16, int UMAX, int VQ>
static hipError_t launch_precode_vq(const void* H, const void* Sym, void* X, int S, int V, int C, int Bc, int U,
                                   int T, float rho_c, hipStream_t st) {
    using E = typename SmNum<F16>::E;
    const int VP = (V + VQ - 1) / VQ;
    int NS = std::max(1, SM_NT / SM_LPT / (C * VP));
    while (NS > 1 && sm_pre_lds_bytes<UMAX>(NS, C, F16) > SM_LDS) --NS;
    const size_t lds = sm_pre_lds_bytes<UMAX>(NS, C, F16);
    if (lds > SM_LDS) return hipErrorInvalidValue;
    const int blocks = (S + NS - 1) / NS;
    hipLaunchKernelGGL((k_precode_small<F16, UMAX, VQ>), dim3(blocks), dim3(SM_NT), lds, st, (const E*)H,
                       (const E*)Sym, (E*)X, S, V, C, Bc, U, T, rho_c, NS);
    return hipGetLastError();
}
template <bool F16, int UMAX>
static hipError_t launch_precode(const void* H, const void* Sym, void* X, int S, int V, int C, int Bc, int U, int T,
                                 float rho_c, hipStream_t st) {
    return sm_vectors_per_quad(F16, S, C, V) == 2
               ? launch_precode_vq<F16, UMAX, 2>(H, Sym, X, S, V, C, Bc, U, T, rho_c, st)
               : launch_precode_vq<F16, UMAX, 1>(H, Sym, X, S, V, C, Bc, U, T, rho_c, st);
}

}  // namespace cdm

using namespace cdm;

extern "C" int32_t cdm_precode_batch(int32_t S, int32_t V, int32_t C, int32_t Bc, int32_t U, int32_t T_max,
                                     int32_t precision, const void* H, const void* Sym, double rho, void* X,
                                     void* stream) {
    if (!H || !Sym || !X) return CDM_EINVAL;
    if (!std::isfinite(rho)) return CDM_EINVAL;
    if (T_max < 1 || T_max > 100000) return CDM_EINVAL;
    if (precision != CDM_C64 && precision != CDM_C16) return CDM_EDTYPE;
    if (S < 1 || V < 1 || U < 1 || U > SM_UMAX || Bc < 1 || Bc > SM_BMAX) return CDM_ESHAPE;
    if (C != 1 && C != 2 && C != 4 && C != 8) return CDM_ESHAPE;
    if (Bc < U) return CDM_EINFEASIBLE;   // local zero-forcing needs Bc >= U
    const bool f16 = precision == CDM_C16;
    const float rho_c = rho > 0.0 ? (float)(rho / std::sqrt((double)C)) : 0.f;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    if (f16)
        e = U <= 8 ? launch_precode<true, 8>(H, Sym, X, S, V, C, Bc, U, T_max, rho_c, st)
                   : launch_precode<true, 16>(H, Sym, X, S, V, C, Bc, U, T_max, rho_c, st);
    else
        e = U <= 8 ? launch_precode<false, 8>(H, Sym, X, S, V, C, Bc, U, T_max, rho_c, st)
                   : launch_precode<false, 16>(H, Sym, X, S, V, C, Bc, U, T_max, rho_c, st);
    return e == hipSuccess ? CDM_OK : CDM_EHIP;
}

extern "C" int32_t cdm_detect_batch(int32_t S, int32_t V, int32_t C, int32_t Bc, int32_t U, int32_t T_max,
                                    int32_t precision, const void* H, const void* Y, double N0, double Ex, void* X,
                                    void* stream) {
    if (!H || !Y || !X) return CDM_EINVAL;
    if (!(Ex > 0.0) || !(N0 >= 0.0) || !std::isfinite(N0) || !std::isfinite(Ex)) return CDM_EINVAL;
    if (T_max < 1 || T_max > 100000) return CDM_EINVAL;
    if (precision != CDM_C64 && precision != CDM_C16) return CDM_EDTYPE;
    if (S < 1 || V < 1 || U < 1 || U > SM_UMAX || Bc < 1 || Bc > SM_BMAX) return CDM_ESHAPE;
    if (C != 1 && C != 2 && C != 4 && C != 8) return CDM_ESHAPE;
    if (N0 == 0.0 && Bc < U) return CDM_EINFEASIBLE;   // lambda = 0: eq. (1) needs Bc >= U
    const bool f16 = precision == CDM_C16;
    // one subcarrier's staging must fit the workgroup's LDS
    if ((U <= 8 ? sm_lds_bytes<8>(1, C, V, f16) : sm_lds_bytes<16>(1, C, V, f16)) > SM_LDS) return CDM_ESHAPE;
    const float lam = (float)(N0 / Ex);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    if (f16)
        e = U <= 8 ? launch_small<true, 8>(H, Y, X, S, V, C, Bc, U, T_max, lam, st)
                   : launch_small<true, 16>(H, Y, X, S, V, C, Bc, U, T_max, lam, st);
    else
        e = U <= 8 ? launch_small<false, 8>(H, Y, X, S, V, C, Bc, U, T_max, lam, st)
                   : launch_small<false, 16>(H, Y, X, S, V, C, Bc, U, T_max, lam, st);
    return e == hipSuccess ? CDM_OK : CDM_EHIP;
}
