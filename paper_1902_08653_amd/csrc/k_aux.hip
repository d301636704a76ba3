// k_aux.hip -- initial residual, FP64 normal-equation residual, small helpers.
#include "common.hpp"
#include "launch.hpp"

namespace cdm {

// ---- init: r0 = y - H x0 (warm) or y (cold); x = x0 or 0 -------------------
template <typename T>
__global__ void k_init_cold(const cv<T>* __restrict__ y, cv<T>* __restrict__ r0, int B, cv<T>* __restrict__ x,
                            const cv<T>* __restrict__ x0, int U) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < B) r0[i] = y[i];
    if (i < U) x[i] = x0 ? x0[i] : czero<T>();
}

// rpart[chunk][row] = sum_{u in chunk} H[row, u] x0[u]  (rows across threads: coalesced)
template <typename T>
__global__ void k_matvec_chunk(const cv<T>* __restrict__ H, int64_t ld, int B, int U, const cv<T>* __restrict__ xv,
                               int cols_per_chunk, cv<T>* __restrict__ rpart) {
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    const int u0 = blockIdx.y * cols_per_chunk;
    const int u1 = min(U, u0 + cols_per_chunk);
    if (row >= B) return;
    cv<T> acc = czero<T>();
    for (int u = u0; u < u1; ++u) cfma(acc, H[(int64_t)u * ld + row], xv[u]);
    rpart[(int64_t)blockIdx.y * B + row] = acc;
}

template <typename T>
__global__ void k_init_warm_reduce(const cv<T>* __restrict__ y, const cv<T>* __restrict__ rpart, int nchunk, int B,
                                   cv<T>* __restrict__ r0) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B) return;
    cv<T> s = y[i];
    for (int c = 0; c < nchunk; ++c) {
        const cv<T> p = rpart[(int64_t)c * B + i];
        s.x -= p.x;
        s.y -= p.y;
    }
    r0[i] = s;
}

template <typename T> static hipError_t launch_init_t(const InitLaunch& L, hipStream_t st) {
    const int n = L.B > L.U ? L.B : L.U;
    hipLaunchKernelGGL(k_init_cold<T>, dim3((n + 255) / 256), dim3(256), 0, st, (const cv<T>*)L.y, (cv<T>*)L.r0,
                       L.B, (cv<T>*)L.x, (const cv<T>*)L.x0, L.U);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !L.x0) return e;
    const int cpc = (L.U + L.nchunk - 1) / L.nchunk;
    hipLaunchKernelGGL(k_matvec_chunk<T>, dim3((L.B + 255) / 256, L.nchunk), dim3(256), 0, st, (const cv<T>*)L.H,
                       L.ld, L.B, L.U, (const cv<T>*)L.x0, cpc, (cv<T>*)L.rpart);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_init_warm_reduce<T>, dim3((L.B + 255) / 256), dim3(256), 0, st, (const cv<T>*)L.y,
                       (const cv<T>*)L.rpart, L.nchunk, L.B, (cv<T>*)L.r0);
    return hipGetLastError();
}

hipError_t launch_init(const InitLaunch& L, hipStream_t st) {
    return L.c128 ? launch_init_t<double>(L, st) : launch_init_t<float>(L, st);
}

// ---- FP64 residual ||H^H (y - H x) - lambda x|| / ||H^H y|| -----------------
template <typename T>
__global__ void k_resid_rows(const cv<T>* __restrict__ H, int64_t ld, int B, int U, const cv<T>* __restrict__ x,
                             int cols_per_chunk, double2* __restrict__ rpart) {
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    const int u0 = blockIdx.y * cols_per_chunk;
    const int u1 = min(U, u0 + cols_per_chunk);
    if (row >= B) return;
    double2 acc = make_double2(0.0, 0.0);
    for (int u = u0; u < u1; ++u) {
        const cv<T> h = H[(int64_t)u * ld + row];
        const cv<T> xv = x[u];
        const double hr = h.x, hi = h.y, xr = xv.x, xi = xv.y;
        acc.x += hr * xr - hi * xi;
        acc.y += hr * xi + hi * xr;
    }
    rpart[(int64_t)blockIdx.y * B + row] = acc;
}

template <typename T>
__global__ void k_resid_r(const cv<T>* __restrict__ y, const double2* __restrict__ rpart, int nchunk, int B,
                          double2* __restrict__ r) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B) return;
    const cv<T> yv = y[i];
    double2 s = make_double2(yv.x, yv.y);
    for (int c = 0; c < nchunk; ++c) {
        const double2 p = rpart[(int64_t)c * B + i];
        s.x -= p.x;
        s.y -= p.y;
    }
    r[i] = s;
}

// one wave per column: a_u = h_u^H r - lambda x_u, b_u = h_u^H y; per-block sums of |a|^2, |b|^2
template <typename T>
__global__ __launch_bounds__(256) void k_resid_cols(const cv<T>* __restrict__ H, int64_t ld, int B, int U,
                                                    const double2* __restrict__ r, const cv<T>* __restrict__ y,
                                                    const cv<T>* __restrict__ x, double lambda,
                                                    double* __restrict__ colpart) {
    __shared__ double sa[4], sb[4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int u = blockIdx.x * 4 + wid;
    double na = 0.0, nb = 0.0;
    if (u < U) {
        double ar = 0, ai = 0, br = 0, bi = 0;
        for (int i = lane; i < B; i += 64) {
            const cv<T> h = H[(int64_t)u * ld + i];
            const double hr = h.x, hi = h.y;
            const double2 rv = r[i];
            const cv<T> yv = y[i];
            ar += hr * rv.x + hi * rv.y;
            ai += hr * rv.y - hi * rv.x;
            br += hr * (double)yv.x + hi * (double)yv.y;
            bi += hr * (double)yv.y - hi * (double)yv.x;
        }
        ar = wave_allsum(ar);
        ai = wave_allsum(ai);
        br = wave_allsum(br);
        bi = wave_allsum(bi);
        const cv<T> xv = x[u];
        ar -= lambda * (double)xv.x;
        ai -= lambda * (double)xv.y;
        na = ar * ar + ai * ai;
        nb = br * br + bi * bi;
    }
    if (lane == 0) {
        sa[wid] = na;
        sb[wid] = nb;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        colpart[2 * blockIdx.x + 0] = sa[0] + sa[1] + sa[2] + sa[3];
        colpart[2 * blockIdx.x + 1] = sb[0] + sb[1] + sb[2] + sb[3];
    }
}

__global__ void k_resid_final(const double* __restrict__ colpart, int nblk, double* __restrict__ out) {
    __shared__ double sa[256], sb[256];
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < nblk; k += 256) {
        a += colpart[2 * k];
        b += colpart[2 * k + 1];
    }
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sa[threadIdx.x] += sa[threadIdx.x + s];
            sb[threadIdx.x] += sb[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sb[0] > 0.0 ? sqrt(sa[0] / sb[0]) : sqrt(sa[0]);
}

template <typename T> static hipError_t launch_resid_t(const ResidLaunch& L, hipStream_t st) {
    const int cpc = (L.U + L.nchunk - 1) / L.nchunk;
    hipLaunchKernelGGL(k_resid_rows<T>, dim3((L.B + 255) / 256, L.nchunk), dim3(256), 0, st, (const cv<T>*)L.H, L.ld,
                       L.B, L.U, (const cv<T>*)L.x, cpc, (double2*)L.rpart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_resid_r<T>, dim3((L.B + 255) / 256), dim3(256), 0, st, (const cv<T>*)L.y,
                       (const double2*)L.rpart, L.nchunk, L.B, (double2*)L.r);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nblk = (L.U + 3) / 4;
    hipLaunchKernelGGL(k_resid_cols<T>, dim3(nblk), dim3(256), 0, st, (const cv<T>*)L.H, L.ld, L.B, L.U,
                       (const double2*)L.r, (const cv<T>*)L.y, (const cv<T>*)L.x, L.lambda, L.colpart);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_resid_final, dim3(1), dim3(256), 0, st, (const double*)L.colpart, nblk, L.out);
    return hipGetLastError();
}

hipError_t launch_resid(const ResidLaunch& L, hipStream_t st) {
    return L.c128 ? launch_resid_t<double>(L, st) : launch_resid_t<float>(L, st);
}

// ---- fusion of the local estimates (uplink, C > 1) --------------------------
// Sec. III: x_hat = sum_c lambda_c x_c with lambda_c = sigma_c^-2 / sum_c' sigma_c'^-2.
// With sigma_c^2 = (N0/U) s_c, s_c = sum_u m_{u,c}, the common factor N0/U cancels, so
// lambda_c = s_c^-1 / sum_c' s_c'^-1 (defined at N0 = 0 too).  A cluster with s_c = 0 (no
// active coordinate) gets weight 0.  Caller weights (lam_c, device, C values) are used
// as given.
template <typename T>
__global__ void k_fuse(const cv<T>* __restrict__ xloc, const double* __restrict__ msum,
                       const double* __restrict__ lam_c, int C, int U, cv<T>* __restrict__ x) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= U) return;
    double tot = 0.0;
    if (!lam_c)
        for (int c = 0; c < C; ++c) tot += msum[c] > 0.0 ? 1.0 / msum[c] : 0.0;
    double re = 0.0, im = 0.0;
    for (int c = 0; c < C; ++c) {
        const double wc = lam_c ? lam_c[c] : (msum[c] > 0.0 && tot > 0.0 ? (1.0 / msum[c]) / tot : 0.0);
        const cv<T> v = xloc[(int64_t)c * U + u];
        re += wc * (double)v.x;
        im += wc * (double)v.y;
    }
    x[u] = cmake<T>((T)re, (T)im);
}
hipError_t launch_fuse(bool c128, const void* xloc, const double* msum, const double* lam_c, int C, int U, void* x,
                       hipStream_t st) {
    if (c128)
        hipLaunchKernelGGL(k_fuse<double>, dim3((U + 255) / 256), dim3(256), 0, st, (const double2*)xloc, msum,
                           lam_c, C, U, (double2*)x);
    else
        hipLaunchKernelGGL(k_fuse<float>, dim3((U + 255) / 256), dim3(256), 0, st, (const float2*)xloc, msum,
                           lam_c, C, U, (float2*)x);
    return hipGetLastError();
}

// ---- helpers ---------------------------------------------------------------
__global__ void k_zero_u32(uint32_t* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}
hipError_t launch_zero_u32(uint32_t* p, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_u32, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

// Merge device-side status bits into info[0] and flag non-finite output.
template <typename T>
__global__ void k_finalize(const cv<T>* __restrict__ x, int U, const uint32_t* __restrict__ status,
                           cdm_info* __restrict__ info) {
    __shared__ int nf;
    if (threadIdx.x == 0) nf = 0;
    __syncthreads();
    int bad = 0;
    for (int u = threadIdx.x; u < U; u += blockDim.x) {
        const cv<T> v = x[u];
        if (!isfinite(v.x) || !isfinite(v.y)) bad = 1;
    }
    if (bad) atomicOr(&nf, 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        // status[0]: a cross-workgroup wait was abandoned; status[1]: CDM_INFO_* bits
        int fl = info[0].flags | (int)status[1];
        if (status[0]) fl |= CDM_INFO_TIMEOUT;
        if (nf) fl |= CDM_INFO_NONFINITE;
        info[0].flags = fl;
    }
}
hipError_t launch_finalize(const void* x, int U, bool c128, const uint32_t* status, cdm_info* info,
                           hipStream_t st) {
    if (c128)
        hipLaunchKernelGGL(k_finalize<double>, dim3(1), dim3(1024), 0, st, (const double2*)x, U, status, info);
    else
        hipLaunchKernelGGL(k_finalize<float>, dim3(1), dim3(1024), 0, st, (const float2*)x, U, status, info);
    return hipGetLastError();
}

__global__ void k_copy_resid(const double* __restrict__ src, cdm_info* __restrict__ info, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) info[i].resid = src[i];
}
hipError_t launch_copy_resid(const double* src, cdm_info* info, int count, hipStream_t st) {
    hipLaunchKernelGGL(k_copy_resid, dim3((count + 255) / 256), dim3(256), 0, st, src, info, count);
    return hipGetLastError();
}

// stand-in values for timing runs: an integer hash of (seed, i) mapped to [-scale/2, scale/2)
template <typename T>
__global__ void k_fill_hash(T* __restrict__ p, int64_t n, uint32_t seed, double scale) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint32_t h = (uint32_t)i * 0x9e3779b1u ^ (uint32_t)(i >> 32) * 0x85ebca77u ^ seed;
        h ^= h >> 16;
        h *= 0x7feb352du;
        h ^= h >> 15;
        h *= 0x846ca68bu;
        h ^= h >> 16;
        p[i] = (T)(scale * ((double)h * (1.0 / 4294967296.0) - 0.5));
    }
}
hipError_t launch_fill_hash(void* p, int64_t n, bool c128, uint32_t seed, double scale) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 256 * 64) blocks = 256 * 64;
    if (blocks < 1) return hipSuccess;
    if (c128)
        hipLaunchKernelGGL(k_fill_hash<double>, dim3((unsigned)blocks), dim3(256), 0, 0, (double*)p, n, seed, scale);
    else
        hipLaunchKernelGGL(k_fill_hash<float>, dim3((unsigned)blocks), dim3(256), 0, 0, (float*)p, n, seed, scale);
    return hipGetLastError();
}

// plain grid-stride 16-byte copy (counter calibration)
__global__ void k_stream_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}
// Read-only stream: every 16-byte word of src is loaded once, streaming (non-temporal),
// eight independent loads in flight per thread; workgroup b stores the XOR of the words it
// read in slot b of out, so that no load can be dropped and no two workgroups write the
// same place.
typedef uint32_t u4v_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 ld_stream(const uint4* p) {
    const u4v_t v = __builtin_nontemporal_load(reinterpret_cast<const u4v_t*>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
}
__global__ __launch_bounds__(256) void k_stream_read(const uint4* __restrict__ src, int64_t n, uint4* out) {
    constexpr int NL = 8;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    uint4 acc = make_uint4(0u, 0u, 0u, 0u);
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (NL - 1) * stride < n; i += NL * stride) {
        uint4 v[NL];
#pragma unroll
        for (int k = 0; k < NL; ++k) v[k] = ld_stream(src + i + k * stride);
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            acc.x ^= v[k].x;
            acc.y ^= v[k].y;
            acc.z ^= v[k].z;
            acc.w ^= v[k].w;
        }
    }
    for (; i < n; i += stride) {
        const uint4 v = ld_stream(src + i);
        acc.x ^= v.x;
        acc.y ^= v.y;
        acc.z ^= v.z;
        acc.w ^= v.w;
    }
    for (int o = 32; o > 0; o >>= 1) {
        acc.x ^= __shfl_xor(acc.x, o);
        acc.y ^= __shfl_xor(acc.y, o);
        acc.z ^= __shfl_xor(acc.z, o);
        acc.w ^= __shfl_xor(acc.w, o);
    }
    __shared__ uint4 wsum[4];
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint4 s = wsum[0];
        for (int k = 1; k < 4; ++k) {
            s.x ^= wsum[k].x;
            s.y ^= wsum[k].y;
            s.z ^= wsum[k].z;
            s.w ^= wsum[k].w;
        }
        out[blockIdx.x] = s;
    }
}
// a fixed grid of CDM_STREAM_READ_SLOTS workgroups: every slot is written, also where
// src is too short to give each workgroup a word (their slots get 0)
hipError_t launch_stream_read(const void* src, int64_t bytes, void* out, hipStream_t st) {
    const int64_t n = bytes / 16;
    hipLaunchKernelGGL(k_stream_read, dim3(CDM_STREAM_READ_SLOTS), dim3(256), 0, st, (const uint4*)src, n, (uint4*)out);
    return hipGetLastError();
}
hipError_t launch_stream_copy(const void* src, void* dst, int64_t bytes, hipStream_t st) {
    const int64_t n = bytes / 16;
    if (n == 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 256 * 64) blocks = 256 * 64;
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, st, (const uint4*)src, (uint4*)dst, n);
    return hipGetLastError();
}

}  // namespace cdm
