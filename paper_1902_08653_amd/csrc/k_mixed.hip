// k_mixed.hip -- mixed-precision refinement around the panel engine.
//
// Low-precision copies of H (planar BF16, or planar FP8-e4m3 with one FP32 scale per
// block of 128 columns) carry the inner coordinate-descent sweeps; FP64 is used only
// for the outer residual and gradient.  One outer step:
//   r = y - H x                          (FP64, one pass over H)
//   g = H^H r - lambda x                 (FP64, one pass over H)
//   d ~ (H~^H H~ + lambda I)^-1 g        (inner CD sweeps from H~, FP32: the panel
//                                         engine with bias g, residual -H~ d)
//   x = x + d;  done once ||d|| <= tol ||x||.
// The fixed point has g = 0, i.e. exactly the stationarity of eq. (1) in FP64.
// Every kernel here takes the device `done` flag and does nothing once it is set,
// so a fixed number of outer launches can be enqueued without host round trips.
#include "common.hpp"
#include "launch.hpp"
#include "quant.hpp"

namespace cdm {

// ---- quantisers ---------------------------------------------------------------
// OCP E4M3 code of v: nearest representable value, ties to the even code, |v| >= 448
// saturating to 448 (the format has no infinities).
__device__ __forceinline__ uint8_t e4m3_code(float v) {
    if (isnan(v)) return 0x7f;
    const uint32_t sign = (v < 0.0f) ? 0x80u : 0u;
    const float a = fabsf(v);
    if (!(a < 448.0f)) return (uint8_t)(sign | 0x7eu);
    if (a < 0.015625f) {                       // below the smallest normal 2^-6: grid k * 2^-9
        const uint32_t k = (uint32_t)rintf(a * 512.0f);
        return (uint8_t)(sign | k);
    }
    int e2 = 0;
    (void)frexpf(a, &e2);                      // a = f * 2^e2, f in [0.5, 1)
    int E = e2 - 1;                            // a in [2^E, 2^(E+1))
    uint32_t k = (uint32_t)rintf((ldexpf(a, -E) - 1.0f) * 8.0f);
    if (k == 8u) {
        k = 0u;
        ++E;
    }
    uint32_t code = ((uint32_t)(E + 7) << 3) | k;
    if (code > 0x7eu) code = 0x7eu;
    return (uint8_t)(sign | code);
}

__global__ void k_quant_bf16(const double2* __restrict__ H, int64_t ld, int B, int U, uint16_t* __restrict__ re,
                             uint16_t* __restrict__ im) {
    const int64_t n = (int64_t)B * U;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        const int64_t u = k / B, i = k - u * B;
        const double2 h = H[u * ld + i];
        re[k] = bf16_code(h.x);
        im[k] = bf16_code(h.y);
    }
}

// one wave per column: largest |Re| or |Im|
__global__ __launch_bounds__(256) void k_col_amax(const double2* __restrict__ H, int64_t ld, int B, int U,
                                                  double* __restrict__ amax) {
    const int lane = threadIdx.x & 63;
    const int u = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (u >= U) return;
    double m = 0.0;
    for (int i = lane; i < B; i += 64) {
        const double2 h = H[(int64_t)u * ld + i];
        m = fmax(m, fmax(fabs(h.x), fabs(h.y)));
    }
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) m = fmax(m, __shfl_xor(m, s, 64));
    if (lane == 0) amax[u] = m;
}

// one FP32 scale per block of 128 columns: fl32(amax / 448), 1 for an all-zero block
__global__ void k_block_scale(const double* __restrict__ amax, int U, float* __restrict__ scale) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    const int nblk = (U + 127) / 128;
    if (b >= nblk) return;
    double m = 0.0;
    for (int u = b * 128; u < U && u < b * 128 + 128; ++u) m = fmax(m, amax[u]);
    scale[b] = (m > 0.0) ? (float)(m / 448.0) : 1.0f;
}

__global__ void k_quant_fp8(const double2* __restrict__ H, int64_t ld, int B, int U, const float* __restrict__ scale,
                            uint8_t* __restrict__ re, uint8_t* __restrict__ im) {
    const int64_t n = (int64_t)B * U;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        const int64_t u = k / B, i = k - u * B;
        const double2 h = H[u * ld + i];
        const double s = (double)scale[u >> 7];
        re[k] = e4m3_code((float)(h.x / s));
        im[k] = e4m3_code((float)(h.y / s));
    }
}

// ---- FP64 outer step ----------------------------------------------------------
// rpart[chunk][row] = sum_{u in chunk} H[row, u] x[u]
__global__ void k_mx_rows(const double2* __restrict__ H, int64_t ld, int B, int U, const double2* __restrict__ x,
                          int cols_per_chunk, double2* __restrict__ rpart, const uint32_t* __restrict__ done) {
    if (*done) return;
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    const int u0 = blockIdx.y * cols_per_chunk;
    const int u1 = min(U, u0 + cols_per_chunk);
    if (row >= B) return;
    // eight columns per round: their loads are in flight together
    double2 a0 = make_double2(0.0, 0.0), a1 = make_double2(0.0, 0.0);
    int u = u0;
    for (; u + 8 <= u1; u += 8) {
        double2 h[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) h[k] = H[(int64_t)(u + k) * ld + row];
#pragma unroll
        for (int k = 0; k < 8; k += 2) {
            cfma(a0, h[k], x[u + k]);
            cfma(a1, h[k + 1], x[u + k + 1]);
        }
    }
    for (; u < u1; ++u) cfma(a0, H[(int64_t)u * ld + row], x[u]);
    rpart[(int64_t)blockIdx.y * B + row] = make_double2(a0.x + a1.x, a0.y + a1.y);
}

// r = y - sum of the chunk partials (fixed order)
__global__ void k_mx_r(const double2* __restrict__ y, const double2* __restrict__ rpart, int nchunk, int B,
                       double2* __restrict__ r, const uint32_t* __restrict__ done) {
    if (*done) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B) return;
    double2 s = y[i];
    for (int c = 0; c < nchunk; ++c) {
        const double2 p = rpart[(int64_t)c * B + i];
        s.x -= p.x;
        s.y -= p.y;
    }
    r[i] = s;
}

// one wave per column: g_u = h_u^H r - lambda x_u (FP64), stored rounded to FP32 as the
// inner solve's bias; also zeroes the inner iterate d
__global__ __launch_bounds__(256) void k_mx_grad(const double2* __restrict__ H, int64_t ld, int B, int U,
                                                 const double2* __restrict__ r, const double2* __restrict__ x,
                                                 double lambda, float2* __restrict__ g32, float2* __restrict__ d32,
                                                 const uint32_t* __restrict__ done) {
    if (*done) return;
    const int lane = threadIdx.x & 63;
    const int u = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (u >= U) return;
    double ar = 0.0, ai = 0.0;
    for (int i = lane; i < B; i += 64) {
        const double2 h = H[(int64_t)u * ld + i];
        const double2 rv = r[i];
        ar += h.x * rv.x + h.y * rv.y;
        ai += h.x * rv.y - h.y * rv.x;
    }
    ar = wave_allsum(ar);
    ai = wave_allsum(ai);
    if (lane == 0) {
        const double2 xv = x[u];
        g32[u] = make_float2((float)(ar - lambda * xv.x), (float)(ai - lambda * xv.y));
        d32[u] = make_float2(0.0f, 0.0f);
    }
}

// zero the inner residual and the panel engine's control words
__global__ void k_mx_reset(float2* __restrict__ r32, int B, uint32_t* __restrict__ ctr, int nctr,
                           const uint32_t* __restrict__ done) {
    if (*done) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < B) r32[i] = make_float2(0.0f, 0.0f);
    // the abort/status words (ctr[2], ctr[3]) keep their values across outer steps
    if (i < nctr && i != 2 && i != 3) ctr[i] = 0u;
}

// x += d (FP64), stop test ||d|| <= tol ||x||, outer step count and statistics into info
__global__ __launch_bounds__(1024) void k_mx_update(double2* __restrict__ x, const float2* __restrict__ d32, int U,
                                                    double tol, int inner_sweeps, uint32_t* __restrict__ done,
                                                    cdm_info* __restrict__ info) {
    if (*done) return;
    __shared__ double sd[1024], sx[1024];
    double a = 0.0, b = 0.0;
    for (int u = threadIdx.x; u < U; u += 1024) {
        const float2 d = d32[u];
        double2 v = x[u];
        v.x += (double)d.x;
        v.y += (double)d.y;
        x[u] = v;
        a += (double)d.x * d.x + (double)d.y * d.y;
        b += v.x * v.x + v.y * v.y;
    }
    sd[threadIdx.x] = a;
    sx[threadIdx.x] = b;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sd[threadIdx.x] += sd[threadIdx.x + s];
            sx[threadIdx.x] += sx[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double S = sd[0], X = sx[0];
        cdm_info o = info[0];
        o.sweeps += 1;                               // outer steps
        o.reserved += (double)inner_sweeps;          // inner low-precision sweeps
        o.rel_step = (X > 0.0) ? sqrt(S / X) : (S > 0.0 ? INFINITY : 0.0);
        info[0] = o;
        if (sqrt(S) <= tol * sqrt(X)) *done = 1u;
    }
}

__global__ void k_mx_start(const double2* __restrict__ x0, double2* __restrict__ x, int U, cdm_info* __restrict__ info,
                           uint32_t* __restrict__ done) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u < U) x[u] = x0 ? x0[u] : make_double2(0.0, 0.0);
    if (u == 0) {
        cdm_info o;
        o.sweeps = 0;
        o.flags = 0;
        o.rel_step = 0.0;
        o.resid = -1.0;
        o.reserved = 0.0;
        info[0] = o;
        *done = 0u;
    }
}

// not converged within the outer cap -> flag
__global__ void k_mx_finish(const uint32_t* __restrict__ done, double tol, cdm_info* __restrict__ info) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && !*done && tol > 0.0) info[0].flags |= CDM_INFO_NOT_CONVERGED;
}

hipError_t launch_quantize(const MixedLaunch& L, hipStream_t st) {
    const int64_t n = (int64_t)L.B * L.U;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (L.src_kind == SRC_BF16) {
        hipLaunchKernelGGL(k_quant_bf16, dim3((unsigned)blocks), dim3(256), 0, st, (const double2*)L.H, L.ld, L.B, L.U,
                           L.q_re16, L.q_im16);
    } else {
        hipLaunchKernelGGL(k_col_amax, dim3((L.U + 3) / 4), dim3(256), 0, st, (const double2*)L.H, L.ld, L.B, L.U,
                           L.colamax);
        const int nblk = (L.U + 127) / 128;
        hipLaunchKernelGGL(k_block_scale, dim3((nblk + 255) / 256), dim3(256), 0, st, (const double*)L.colamax, L.U,
                           L.q_scale);
        hipLaunchKernelGGL(k_quant_fp8, dim3((unsigned)blocks), dim3(256), 0, st, (const double2*)L.H, L.ld, L.B,
                           L.U, (const float*)L.q_scale, L.q_re8, L.q_im8);
    }
    return hipGetLastError();
}

hipError_t launch_mixed_start(const MixedLaunch& L, hipStream_t st) {
    hipLaunchKernelGGL(k_mx_start, dim3((L.U + 255) / 256), dim3(256), 0, st, (const double2*)L.x0, (double2*)L.x,
                       L.U, L.info, L.done);
    return hipGetLastError();
}

hipError_t launch_mixed_outer_head(const MixedLaunch& L, hipStream_t st) {
    const int cpc = (L.U + L.nchunk - 1) / L.nchunk;
    hipLaunchKernelGGL(k_mx_rows, dim3((L.B + 255) / 256, L.nchunk), dim3(256), 0, st, (const double2*)L.H, L.ld, L.B,
                       L.U, (const double2*)L.x, cpc, (double2*)L.rpart, (const uint32_t*)L.done);
    hipLaunchKernelGGL(k_mx_r, dim3((L.B + 255) / 256), dim3(256), 0, st, (const double2*)L.y,
                       (const double2*)L.rpart, L.nchunk, L.B, (double2*)L.r64, (const uint32_t*)L.done);
    hipLaunchKernelGGL(k_mx_grad, dim3((L.U + 3) / 4), dim3(256), 0, st, (const double2*)L.H, L.ld, L.B, L.U,
                       (const double2*)L.r64, (const double2*)L.x, L.lambda, (float2*)L.g32, (float2*)L.d32,
                       (const uint32_t*)L.done);
    const int n = L.B > L.nctr ? L.B : L.nctr;
    hipLaunchKernelGGL(k_mx_reset, dim3((n + 255) / 256), dim3(256), 0, st, (float2*)L.r32, L.B, L.ctr, L.nctr,
                       (const uint32_t*)L.done);
    return hipGetLastError();
}

hipError_t launch_mixed_outer_tail(const MixedLaunch& L, hipStream_t st) {
    hipLaunchKernelGGL(k_mx_update, dim3(1), dim3(1024), 0, st, (double2*)L.x, (const float2*)L.d32, L.U, L.tol,
                       L.inner_sweeps, L.done, L.info);
    return hipGetLastError();
}

hipError_t launch_mixed_finish(const MixedLaunch& L, hipStream_t st) {
    hipLaunchKernelGGL(k_mx_finish, dim3(1), dim3(64), 0, st, (const uint32_t*)L.done, L.tol, L.info);
    return hipGetLastError();
}

}  // namespace cdm
