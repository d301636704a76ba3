// k_wg_mixed.hip -- mixed-precision refinement for an uneven batch of instances.
//
// Every instance (complex128 H, y, x) is refined in FP64 around FP32 coordinate
// descent on a low-precision copy H~ of its H.  One outer step s is three launches,
// each over the whole batch (instances already finished skip their work):
//   k_bm_resid   r = y - H x                 FP64, one pass over H (not while x = 0)
//   k_bm_grad    g = H^H r - lambda x        FP64, one pass over H; in the first step
//                                            also the copy H~ and m~_u, n~_u of Algorithm 1
//                                            from ||h~_u||^2 (same loads)
//   k_bm_inner   inner CD sweeps on (H~^H H~ + lambda I) d = g in FP32 from H~, with
//                the residual s = -H~ d in VGPRs and Algorithm 1's coordinate rule with
//                bias g:  d_u <- m~_u (g_u + h~_u^H s) + n~_u d_u,  s <- s - h~_u delta;
//                then x <- x + d
// The FP64 passes need no synchronisation inside an instance, so they run as plain
// streaming kernels; only the inner sweeps keep the workgroup-per-instance form
// (one barrier per coordinate), light enough for several workgroups per CU.
// Stop, checked after every inner sweep, with c_s = ||d|| / ||x + d|| the relative
// correction of the current step and c_{s-1} that of the previous one:
//   done   if c_s <= tol (the correction itself is below the tolerance), or if the
//          sweep step ||delta|| <= tol ||x + d|| and the geometric prediction of the
//          next correction, c_s^2 / c_{s-1}, is <= tol (outer steps contract by about
//          c_s / c_{s-1} each, so the next one would change x by less than tol);
//   next outer step  once ||delta|| <= max(tau ||d||, tol ||x + d||), or after
//          inner_max sweeps.
// The fixed point has g = 0 in FP64: the FP64 solution of eq. (1), not a rounded one.
#include <algorithm>

#include "common.hpp"
#include "launch.hpp"
#include "quant.hpp"
#include "wg.hpp"

namespace cdm {

// Low-precision copy of one complex128 element.
template <int Q> struct WgLow;
template <> struct WgLow<WG_LOW_C64> {        // complex64 rounding (8 B)
    using Raw = float2;
    __device__ static Raw enc(double2 h) { return make_float2((float)h.x, (float)h.y); }
    __device__ static float2 dec(Raw v) { return v; }
};
template <> struct WgLow<WG_LOW_BF16> {       // BF16 pair, Re in the low half (4 B)
    using Raw = uint32_t;
    __device__ static Raw enc(double2 h) {
        return (uint32_t)bf16_code(h.x) | ((uint32_t)bf16_code(h.y) << 16);
    }
    __device__ static float2 dec(Raw v) {
        return make_float2(__uint_as_float(v << 16), __uint_as_float(v & 0xffff0000u));
    }
};

// Element of a column-major block addressed as a wave-uniform column base plus a
// per-lane 32-bit byte offset, so that the base stays in scalar registers.
template <typename E> __device__ __forceinline__ E ld_col(const E* blk, int col, int64_t ld, uint32_t byte_off) {
    return *reinterpret_cast<const E*>(reinterpret_cast<const char*>(blk + (int64_t)col * ld) + byte_off);
}

// ---- per-instance state -----------------------------------------------------------
// x = x0 (or 0); info zeroed; done cleared.  Grid over max(sum n, batch).
__global__ void k_bm_init(const double2* __restrict__ X0, double2* __restrict__ X, int64_t total_n,
                          cdm_info* __restrict__ info, uint32_t* __restrict__ done, int batch) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < total_n) X[i] = X0 ? X0[i] : make_double2(0.0, 0.0);
    if (i < batch) {
        cdm_info o;
        o.sweeps = 0;
        o.flags = 0;
        o.rel_step = 0.0;
        o.resid = -1.0;
        o.reserved = 0.0;
        info[i] = o;
        done[i] = 0u;
    }
}

// ---- r = y - H x (FP64) -------------------------------------------------------------
// One workgroup per instance (blockIdx = job id); thread t owns rows t, t + 256, ...,
// in blocks of BM_RB rows per thread; columns stream in order with the next in flight.
constexpr int BM_NT = 256;
constexpr int BM_RB = 4;
__global__ __launch_bounds__(BM_NT) void k_bm_resid(const WgJob* __restrict__ jobs, const double2* __restrict__ H,
                                                    const double2* __restrict__ Y, const double2* __restrict__ X,
                                                    double2* __restrict__ R, const uint32_t* __restrict__ done) {
    const WgJob jb = jobs[blockIdx.x];
    if (done[jb.info_idx]) return;
    const int m = jb.m, n = jb.n;
    const int64_t ld = jb.ld;
    const double2* Hj = H + jb.h_off;
    const double2* xj = X + jb.x_off;
    for (int i0 = 0; i0 < m; i0 += BM_NT * BM_RB) {
        uint32_t rowc[BM_RB];
        bool live[BM_RB];
        double2 r[BM_RB], hc[BM_RB], hn[BM_RB];
#pragma unroll
        for (int q = 0; q < BM_RB; ++q) {
            const int i = i0 + (int)threadIdx.x + q * BM_NT;
            live[q] = i < m;
            rowc[q] = (uint32_t)(live[q] ? i : m - 1);
            r[q] = Y[jb.y_off + rowc[q]];
            hc[q] = ld_col(Hj, 0, ld, rowc[q] * 16u);
        }
        for (int u = 0; u < n; ++u) {
            if (u + 1 < n) {
#pragma unroll
                for (int q = 0; q < BM_RB; ++q) hn[q] = ld_col(Hj, u + 1, ld, rowc[q] * 16u);
            }
            const double2 xu = xj[u];
#pragma unroll
            for (int q = 0; q < BM_RB; ++q) {
                cfms(r[q], hc[q], xu);
                hc[q] = hn[q];
            }
        }
#pragma unroll
        for (int q = 0; q < BM_RB; ++q)
            if (live[q]) R[jb.y_off + rowc[q]] = r[q];
    }
}

// ---- g = H^H r - lambda x (FP64); first step: the copy H~ and (m~, n~) -----------
// One wave per (instance, user), found by a binary search over the packed x offsets.
template <int Q>
__global__ __launch_bounds__(256) void k_bm_grad(const WgJob* __restrict__ jobs, const int64_t* __restrict__ x_off,
                                                 int njobs, int64_t total_n, const double2* __restrict__ H,
                                                 const double2* __restrict__ R, const double2* __restrict__ Y,
                                                 const double2* __restrict__ X, double lambda, int first, int use_y,
                                                 typename WgLow<Q>::Raw* __restrict__ Hq, float2* __restrict__ G,
                                                 float2* __restrict__ CF, const uint32_t* __restrict__ done,
                                                 cdm_info* __restrict__ info) {
    using Raw = typename WgLow<Q>::Raw;
    const int lane = threadIdx.x & 63;
    const int64_t gw = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (gw >= total_n) return;
    int lo = 0, hi = njobs;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (x_off[mid] <= gw) lo = mid;
        else hi = mid;
    }
    const WgJob jb = jobs[lo];
    if (done[jb.info_idx]) return;
    const int u = (int)(gw - x_off[lo]);
    const double2* h = H + jb.h_off + (int64_t)u * jb.ld;
    // r = y while x = 0 (the cold first step needs no residual pass)
    const double2* r = (use_y ? Y : R) + jb.y_off;
    Raw* hq = Hq + jb.h_off + (int64_t)u * jb.ld;
    double gr = 0.0, gi = 0.0, e = 0.0;
    for (int i = lane; i < jb.m; i += 64) {
        const double2 hv = h[i], rv = r[i];
        gr += hv.x * rv.x + hv.y * rv.y;
        gi += hv.x * rv.y - hv.y * rv.x;
        if (first) {
            const Raw c = WgLow<Q>::enc(hv);
            hq[i] = c;
            const float2 hd = WgLow<Q>::dec(c);
            e += (double)(hd.x * hd.x + hd.y * hd.y);
        }
    }
    gr = wave_sum_last(gr);
    gi = wave_sum_last(gi);
    if (first) e = wave_sum_last(e);
    if (lane == 63) {
        const int64_t k = jb.x_off + u;
        const double2 xv = X[k];
        G[k] = make_float2((float)(gr - lambda * xv.x), (float)(gi - lambda * xv.y));
        if (first) {
            // Algorithm 1 preprocessing on H~: m~ = 1/(||h~_u||^2 + lambda), n~ = m~ ||h~_u||^2;
            // a column with ||h~_u||^2 + lambda == 0 stays inactive: (0, 1)
            const float ef = (float)e, lam = (float)lambda;
            if (ef + lam > 0.0f) {
                const float mu = 1.0f / (ef + lam);
                CF[k] = make_float2(mu, mu * ef);
            } else {
                CF[k] = make_float2(0.0f, 1.0f);
                atomicOr(&info[jb.info_idx].flags, CDM_INFO_ZERO_COLUMN);
            }
        }
    }
}

// ---- inner sweeps (FP32, from H~) and x += d -----------------------------------------
template <int Q, int NT, int RPT>
__device__ __forceinline__ void inner_instance(const WgJob& jb, const typename WgLow<Q>::Raw* __restrict__ Hq,
                                               const float2* __restrict__ G, const float2* __restrict__ CF,
                                               double2* __restrict__ X, cdm_info* __restrict__ info,
                                               uint32_t* __restrict__ done, double tol, int inner_max, double tau,
                                               int last, unsigned char* smem_raw, float (*red32)[NT / 64][2]) {
    using Raw = typename WgLow<Q>::Raw;
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    const int m = jb.m, n = jb.n;
    const int64_t ld = jb.ld;
    const Raw* Qj = Hq + jb.h_off;
    double2* x_s = reinterpret_cast<double2*>(smem_raw);  // x (FP64), for ||x + d||
    float2* g_s = reinterpret_cast<float2*>(x_s + n);     // bias g
    float2* d_s = g_s + n;                                // iterate d
    float2* cf_s = d_s + n;                               // (m~_u, n~_u)
    for (int u = tid; u < n; u += NT) {
        g_s[u] = G[jb.x_off + u];
        cf_s[u] = CF[jb.x_off + u];
        d_s[u] = make_float2(0.0f, 0.0f);
        x_s[u] = X[jb.x_off + u];
    }
    // rows past m load row m - 1 (in bounds) and are zeroed by a select
    uint32_t rowc[RPT];
    bool live[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int i = tid + q * NT;
        live[q] = i < m;
        rowc[q] = (uint32_t)(live[q] ? i : m - 1) * (uint32_t)sizeof(Raw);
    }
    float2 sr[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) sr[q] = make_float2(0.0f, 0.0f);
    // relative correction of the previous outer step (none before the first)
    const cdm_info prev = info[jb.info_idx];
    const bool have_prev = prev.sweeps > 0;
    const double c_prev = prev.rel_step;
    __syncthreads();
    bool conv = false;
    int j = 0;
    double S = 0.0, D = 0.0, XD = 0.0;
    while (j < inner_max) {
        ++j;
        S = 0.0;
        D = 0.0;
        XD = 0.0;
        float2 hc[RPT], hn[RPT];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const float2 v = WgLow<Q>::dec(ld_col<Raw>(Qj, 0, ld, rowc[q]));
            hc[q] = live[q] ? v : make_float2(0.0f, 0.0f);
        }
        for (int u = 0; u < n; ++u) {
            if (u + 1 < n) {
#pragma unroll
                for (int q = 0; q < RPT; ++q) {
                    const float2 v = WgLow<Q>::dec(ld_col<Raw>(Qj, u + 1, ld, rowc[q]));
                    hn[q] = live[q] ? v : make_float2(0.0f, 0.0f);
                }
            }
            float ar = 0.0f, ai = 0.0f;
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                ar += hc[q].x * sr[q].x + hc[q].y * sr[q].y;
                ai += hc[q].x * sr[q].y - hc[q].y * sr[q].x;
            }
            ar = wave_sum_last(ar);
            ai = wave_sum_last(ai);
            // read the coordinate's state before the barrier: thread 0 overwrites d_u after it
            const float2 du = d_s[u];
            const float2 gu = g_s[u];
            const float2 cf = cf_s[u];
            const double2 xu = x_s[u];
            const int par = u & 1;
            if (lane == 63) {
                red32[par][wid][0] = ar;
                red32[par][wid][1] = ai;
            }
            __syncthreads();
            float2 a = make_float2(0.0f, 0.0f);
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                a.x += red32[par][w][0];
                a.y += red32[par][w][1];
            }
            float2 dn;
            dn.x = cf.x * (gu.x + a.x) + cf.y * du.x;
            dn.y = cf.x * (gu.y + a.y) + cf.y * du.y;
            float2 dl;
            dl.x = dn.x - du.x;
            dl.y = dn.y - du.y;
            if (tid == 0) d_s[u] = dn;
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                cfms(sr[q], hc[q], dl);
                hc[q] = hn[q];
            }
            S += cabs2d(dl);
            D += cabs2d(dn);
            const double xr = xu.x + (double)dn.x, xi = xu.y + (double)dn.y;
            XD += xr * xr + xi * xi;
        }
        __syncthreads();   // the next sweep reuses the reduction slots and reads d_s
        const double c = XD > 0.0 ? sqrt(D / XD) : 0.0;       // relative correction
        const double st = XD > 0.0 ? sqrt(S / XD) : 0.0;      // relative sweep step
        if (c <= tol || (have_prev && st <= tol && c * c <= tol * c_prev)) {
            conv = true;
            break;
        }
        if (sqrt(S) <= tau * sqrt(D) || st <= tol) break;
    }
    int nf = 0;
    for (int u = tid; u < n; u += NT) {
        const float2 d = d_s[u];
        double2 v = x_s[u];
        v.x += (double)d.x;
        v.y += (double)d.y;
        if (!isfinite(v.x) || !isfinite(v.y)) nf = 1;
        X[jb.x_off + u] = v;
    }
    nf = __syncthreads_or(nf);
    if (tid == 0) {
        cdm_info o = prev;
        o.sweeps += 1;                         // outer steps
        o.reserved += (double)j;               // inner sweeps
        o.rel_step = (XD > 0.0) ? sqrt(D / XD) : (D > 0.0 ? INFINITY : 0.0);
        if (nf) o.flags |= CDM_INFO_NONFINITE;
        if (!conv && last) o.flags |= CDM_INFO_NOT_CONVERGED;
        info[jb.info_idx] = o;
        if (conv || nf) done[jb.info_idx] = 1u;
    }
}

template <int Q, int NT>
__global__ __launch_bounds__(NT) void k_bm_inner(const WgJob* __restrict__ jobs, int njobs,
                                                 const typename WgLow<Q>::Raw* __restrict__ Hq,
                                                 const float2* __restrict__ G, const float2* __restrict__ CF,
                                                 double2* __restrict__ X, cdm_info* __restrict__ info,
                                                 uint32_t* __restrict__ done, double tol, int inner_max, double tau,
                                                 int last, const int* __restrict__ order, uint32_t* __restrict__ queue) {
    constexpr int NW = NT / 64;
    extern __shared__ unsigned char smem_raw[];
    __shared__ float red32[2][NW][2];
    __shared__ int job_s;
    const int tid = threadIdx.x;
    for (;;) {
        // next job from the shared queue (slots in `order`: largest instances first)
        if (tid == 0) job_s = (int)atomicAdd(queue, 1u);
        __syncthreads();
        // the job index is wave-uniform: in a scalar register the job record and every
        // column base stay scalar too
        const int jslot = __builtin_amdgcn_readfirstlane(job_s);
        if (jslot >= njobs) return;
        const int jid = order ? __builtin_amdgcn_readfirstlane(order[jslot]) : jslot;
        const WgJob jb = jobs[jid];
        if (!done[jb.info_idx]) {
            switch (jb.rpt) {
                case 1: inner_instance<Q, NT, 1>(jb, Hq, G, CF, X, info, done, tol, inner_max, tau, last, smem_raw, red32); break;
                case 2: inner_instance<Q, NT, 2>(jb, Hq, G, CF, X, info, done, tol, inner_max, tau, last, smem_raw, red32); break;
                case 4: inner_instance<Q, NT, 4>(jb, Hq, G, CF, X, info, done, tol, inner_max, tau, last, smem_raw, red32); break;
                default: inner_instance<Q, NT, 8>(jb, Hq, G, CF, X, info, done, tol, inner_max, tau, last, smem_raw, red32); break;
            }
        }
        __syncthreads();
    }
}

// ---- optional FP64 residual of the result, one workgroup per instance ------------------
template <int RPT>
__device__ __forceinline__ void resid_one(const WgJob& jb, const double2* H, const double2* Y, const double2* x_s,
                                          double lambda, double (*red64)[4][4], cdm_info* info) {
    const double res = wg_fp64_resid<double, 256, RPT>(H + jb.h_off, jb.ld, Y + jb.y_off, x_s, jb.m, jb.n, lambda,
                                                      red64);
    if (threadIdx.x == 0) info[jb.info_idx].resid = res;
}
__global__ __launch_bounds__(256) void k_bm_resid_check(const WgJob* __restrict__ jobs, const double2* __restrict__ H,
                                                        const double2* __restrict__ Y, const double2* __restrict__ X,
                                                        double lambda, cdm_info* __restrict__ info) {
    extern __shared__ unsigned char smem_raw[];
    __shared__ double red64[2][4][4];
    const WgJob jb = jobs[blockIdx.x];
    double2* x_s = reinterpret_cast<double2*>(smem_raw);
    for (int u = threadIdx.x; u < jb.n; u += 256) x_s[u] = X[jb.x_off + u];
    __syncthreads();
    const int rpt = (jb.m + 255) / 256;
    if (rpt <= 1) resid_one<1>(jb, H, Y, x_s, lambda, red64, info);
    else if (rpt <= 2) resid_one<2>(jb, H, Y, x_s, lambda, red64, info);
    else if (rpt <= 4) resid_one<4>(jb, H, Y, x_s, lambda, red64, info);
    else resid_one<8>(jb, H, Y, x_s, lambda, red64, info);
}

// ---- host side ------------------------------------------------------------------------
template <int Q, int NT> static hipError_t launch_inner_t(const BmLaunch& L, int last, hipStream_t st) {
    using Raw = typename WgLow<Q>::Raw;
    hipLaunchKernelGGL((k_bm_inner<Q, NT>), dim3(L.grid), dim3(NT), bm_lds_bytes(L.n_max), st, L.jobs, L.njobs,
                       (const Raw*)L.Hq, (const float2*)L.G, (const float2*)L.CF, (double2*)L.X, L.info, L.done,
                       L.tol, L.inner_max, L.tau, last, L.order, L.queue);
    return hipGetLastError();
}
template <int Q, int NT> static hipError_t set_lds_t(size_t bytes) {
    return hipFuncSetAttribute((const void*)k_bm_inner<Q, NT>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}
template <int Q, int NT> static int occ_t(size_t bytes) {
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_bm_inner<Q, NT>, NT, bytes) != hipSuccess) return 0;
    return per;
}

#define CDM_BM_DISPATCH(FN, low, nt, ...)                                            \
    do {                                                                             \
        if (low == WG_LOW_C64) {                                                     \
            if (nt == 128) return FN<WG_LOW_C64, 128>(__VA_ARGS__);                  \
            if (nt == 256) return FN<WG_LOW_C64, 256>(__VA_ARGS__);                  \
            if (nt == 512) return FN<WG_LOW_C64, 512>(__VA_ARGS__);                  \
        } else if (low == WG_LOW_BF16) {                                             \
            if (nt == 128) return FN<WG_LOW_BF16, 128>(__VA_ARGS__);                 \
            if (nt == 256) return FN<WG_LOW_BF16, 256>(__VA_ARGS__);                 \
            if (nt == 512) return FN<WG_LOW_BF16, 512>(__VA_ARGS__);                 \
        }                                                                            \
    } while (0)

hipError_t bm_set_lds_limit(int low, int nt, size_t bytes) {
    CDM_BM_DISPATCH(set_lds_t, low, nt, bytes);
    return hipErrorInvalidValue;
}
int bm_occupancy(int low, int nt, size_t bytes) {
    CDM_BM_DISPATCH(occ_t, low, nt, bytes);
    return 0;
}
size_t bm_lds_bytes(int n_max) { return (size_t)n_max * (16 + 3 * 8); }

hipError_t launch_bm_init(const BmLaunch& L, hipStream_t st) {
    const int64_t cnt = std::max<int64_t>(L.total_n, L.njobs);
    hipLaunchKernelGGL(k_bm_init, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, (const double2*)L.X0,
                       (double2*)L.X, L.total_n, L.info, L.done, L.njobs);
    return hipGetLastError();
}

hipError_t launch_bm_step(const BmLaunch& L, int step, int last, hipStream_t st) {
    const bool first = step == 1;
    const bool need_r = !(first && L.X0 == nullptr);
    if (need_r)
        hipLaunchKernelGGL(k_bm_resid, dim3(L.njobs), dim3(BM_NT), 0, st, L.jobs, (const double2*)L.H,
                           (const double2*)L.Y, (const double2*)L.X, (double2*)L.R, (const uint32_t*)L.done);
    const dim3 gg((unsigned)((L.total_n + 3) / 4));
    if (L.low == WG_LOW_C64)
        hipLaunchKernelGGL(k_bm_grad<WG_LOW_C64>, gg, dim3(256), 0, st, L.jobs, L.x_off, L.njobs, L.total_n,
                           (const double2*)L.H, (const double2*)L.R, (const double2*)L.Y, (const double2*)L.X,
                           L.lambda, first ? 1 : 0, need_r ? 0 : 1, (float2*)L.Hq, (float2*)L.G, (float2*)L.CF,
                           (const uint32_t*)L.done, L.info);
    else
        hipLaunchKernelGGL(k_bm_grad<WG_LOW_BF16>, gg, dim3(256), 0, st, L.jobs, L.x_off, L.njobs, L.total_n,
                           (const double2*)L.H, (const double2*)L.R, (const double2*)L.Y, (const double2*)L.X,
                           L.lambda, first ? 1 : 0, need_r ? 0 : 1, (uint32_t*)L.Hq, (float2*)L.G, (float2*)L.CF,
                           (const uint32_t*)L.done, L.info);
    hipError_t e = launch_zero_u32(L.queue, 1, st);
    if (e != hipSuccess) return e;
    CDM_BM_DISPATCH(launch_inner_t, L.low, L.nt, L, last, st);
    return hipErrorInvalidValue;
}

hipError_t launch_bm_resid_check(const BmLaunch& L, hipStream_t st) {
    hipLaunchKernelGGL(k_bm_resid_check, dim3(L.njobs), dim3(256), (size_t)L.n_max * 16, st, L.jobs,
                       (const double2*)L.H, (const double2*)L.Y, (const double2*)L.X, L.lambda, L.info);
    return hipGetLastError();
}

}  // namespace cdm
