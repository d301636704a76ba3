// k_wg.hip -- "one workgroup per instance" engine for Algorithm 1 (uplink CD).
//
// Each workgroup owns one instance (an antenna cluster's local problem, or one
// entry of an uneven batch) and runs the whole local CD of Algorithm 1 on it:
// preprocessing (column energies, fused into the first sweep), init, T_max (or
// tolerance-bounded) cyclic sweeps, output.  The residual r stays in VGPRs for the
// whole solve (thread t owns rows t, t+NT, ...); each coordinate step is
//   partial h_u^H r over the thread's rows  ->  wave64 butterfly  ->  cross-wave
//   sum through LDS (one barrier)  ->  scalar rule, identical in every thread  ->
//   axpy r -= h_u delta on the thread's rows.
// Column u+1 is loaded while column u is reduced.  x and the per-column scalars
// (m_u, n_u) live in LDS.
#include "common.hpp"
#include "launch.hpp"
#include "wg.hpp"

namespace cdm {

// One uplink instance, RPT rows per thread (m <= NT * RPT).
template <typename T, int NT, int RPT>
__device__ __forceinline__ void cd_instance(const WgJob& jb, const cv<T>* __restrict__ H, const cv<T>* __restrict__ Y,
                                            const cv<T>* __restrict__ X0, cv<T>* __restrict__ X,
                                            cdm_info* __restrict__ info, T lambda, int T_max, double tol,
                                            double* __restrict__ msum, int64_t ld_arg, unsigned char* smem_raw,
                                            T (*red_s)[NT / 64][3], int& flag_s, int resid,
                                            double (*red64)[NT / 64][4], double lambda_d) {
    using V = cv<T>;
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
        // ---------------------------------------------------------------- one instance
        const int m = jb.m, n = jb.n;
        const int64_t ld = jb.ld > 0 ? jb.ld : ld_arg;   // ld <= 0: the solve's leading dimension
        const V* Hj = H + jb.h_off;
        V* x_s = reinterpret_cast<V*>(smem_raw);
        V* cf_s = x_s + n;   // (m_u, n_u) of Algorithm 1

        // rows past m load row m - 1 (in bounds) and are zeroed by a select, so that
        // no load sits behind a branch; column bases stay wave-uniform
        uint32_t rowc[RPT];
        bool live[RPT];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int i = tid + q * NT;
            live[q] = i < m;
            rowc[q] = (uint32_t)(live[q] ? i : m - 1) * (uint32_t)sizeof(V);
        }
        auto col = [&](int u, int q) -> V {
            const V v = *reinterpret_cast<const V*>(reinterpret_cast<const char*>(Hj + (int64_t)u * ld) + rowc[q]);
            return live[q] ? v : czero<T>();
        };
        V r[RPT];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const V v = *reinterpret_cast<const V*>(reinterpret_cast<const char*>(Y + jb.y_off) + rowc[q]);
            r[q] = live[q] ? v : czero<T>();
        }
        for (int u = tid; u < n; u += NT) x_s[u] = X0 ? X0[jb.x0_off + u] : czero<T>();
        __syncthreads();
        if (X0) {  // warm start: r = y - H x0
            for (int u = 0; u < n; ++u) {
                const V xu = x_s[u];
#pragma unroll
                for (int q = 0; q < RPT; ++q) cfms(r[q], col(u, q), xu);
            }
        }

        int sweeps = 0;
        double S = 0.0, Xn = 0.0;
        for (int t = 1; t <= T_max; ++t) {
            S = 0.0;
            Xn = 0.0;
            V hc[RPT], hn[RPT];
#pragma unroll
            for (int q = 0; q < RPT; ++q) hc[q] = col(0, q);
            for (int u = 0; u < n; ++u) {
                if (u + 1 < n) {
#pragma unroll
                    for (int q = 0; q < RPT; ++q) hn[q] = col(u + 1, q);
                }
                T gr = 0, gi = 0, ee = 0;
#pragma unroll
                for (int q = 0; q < RPT; ++q) {
                    gr += hc[q].x * r[q].x + hc[q].y * r[q].y;
                    gi += hc[q].x * r[q].y - hc[q].y * r[q].x;
                    if (t == 1) ee += hc[q].x * hc[q].x + hc[q].y * hc[q].y;
                }
                gr = wave_sum_last(gr);
                gi = wave_sum_last(gi);
                if (t == 1) ee = wave_sum_last(ee);
                // read x_u and the scalars before the barrier: thread 0 overwrites them after it
                const V xu = x_s[u];
                V cf = (t > 1) ? cf_s[u] : czero<T>();
                const int par = u & 1;
                if (lane == 63) {
                    red_s[par][wid][0] = gr;
                    red_s[par][wid][1] = gi;
                    red_s[par][wid][2] = ee;
                }
                __syncthreads();
                V g = czero<T>();
                T e = 0;
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    g.x += red_s[par][w][0];
                    g.y += red_s[par][w][1];
                    if (t == 1) e += red_s[par][w][2];
                }
                if (t == 1) {
                    // Algorithm 1 preprocessing: m_u = 1/(||h_u||^2 + lambda), n_u = m_u ||h_u||^2.
                    // A coordinate with ||h_u||^2 + lambda == 0 stays inactive: (m, n) = (0, 1).
                    if (e + lambda > T(0)) {
                        cf.x = T(1) / (e + lambda);
                        cf.y = cf.x * e;
                    } else {
                        cf.x = T(0);
                        cf.y = T(1);
                        if (tid == 0) flag_s |= CDM_INFO_ZERO_COLUMN;
                    }
                }
                // x_u <- m_u h_u^H r + n_u x_u ; delta = x_u(new) - x_u(old)
                V xn;
                xn.x = cf.x * g.x + cf.y * xu.x;
                xn.y = cf.x * g.y + cf.y * xu.y;
                V d;
                d.x = xn.x - xu.x;
                d.y = xn.y - xu.y;
                if (tid == 0) {
                    x_s[u] = xn;
                    if (t == 1) cf_s[u] = cf;
                }
                // r <- r - h_u delta
#pragma unroll
                for (int q = 0; q < RPT; ++q) cfms(r[q], hc[q], d);
                S += cabs2d(d);
                Xn += cabs2d(xn);
#pragma unroll
                for (int q = 0; q < RPT; ++q) hc[q] = hn[q];
            }
            __syncthreads();
            if (t == 1 && msum && tid == 0) {
                // sum_u m_u of this cluster, in index order (feeds the fusion weights)
                double ms = 0.0;
                for (int u = 0; u < n; ++u) ms += (double)cf_s[u].x;
                msum[jb.info_idx] = ms;
            }
            sweeps = t;
            if (tol > 0.0 && sqrt(S) <= tol * sqrt(Xn)) break;
        }
        // ---------------------------------------------------------------- output
        int nf = 0;
        for (int u = tid; u < n; u += NT) {
            const V v = x_s[u];
            if (!isfinite(v.x) || !isfinite(v.y)) nf = 1;
            X[jb.x_off + u] = v;
        }
        if (nf) atomicOr(&flag_s, CDM_INFO_NONFINITE);
        __syncthreads();
        // optional FP64 check of the stationarity of eq. (1)
        const double res = resid ? wg_fp64_resid<T, NT, RPT>(Hj, ld, Y + jb.y_off, x_s, m, n, lambda_d, red64) : -1.0;
        if (tid == 0) {
            const double rel = (Xn > 0.0) ? sqrt(S / Xn) : (S > 0.0 ? INFINITY : 0.0);
            int fl = flag_s;
            if (tol > 0.0 && !(rel <= tol)) fl |= CDM_INFO_NOT_CONVERGED;
            cdm_info o;
            o.sweeps = sweeps;
            o.flags = fl;
            o.rel_step = rel;
            o.resid = res;
            o.reserved = 0.0;
            info[jb.info_idx] = o;
        }
}

// RMAX: the largest rows-per-thread tile the launch needs (4 or 8).  Only tiles up to
// RMAX are compiled into the instance, so a launch whose instances fit 4 rows per
// thread is not held to the register footprint of the 8-row tile.
template <typename T, int NT, int RMAX>
__global__ __launch_bounds__(NT) void k_cd_wg(const WgJob* __restrict__ jobs, int njobs,
                                              const cv<T>* __restrict__ H, const cv<T>* __restrict__ Y,
                                              const cv<T>* __restrict__ X0, cv<T>* __restrict__ X,
                                              cdm_info* __restrict__ info, double lambda_d, int T_max,
                                              double tol, const int* __restrict__ order,
                                              uint32_t* __restrict__ queue, double* __restrict__ msum,
                                              int64_t ld_arg, int resid) {
    constexpr int NW = NT / 64;
    extern __shared__ unsigned char smem_raw[];
    __shared__ T red_s[2][NW][3];
    __shared__ double red64[2][NW][4];
    __shared__ int flag_s;
    __shared__ int job_s;
    const int tid = threadIdx.x;
    const T lambda = (T)lambda_d;
    for (;;) {
        // next job from the shared queue; the queue hands out slots in `order`
        // (largest instances first for uneven batches)
        if (tid == 0) {
            job_s = (int)atomicAdd(queue, 1u);
            flag_s = 0;
        }
        __syncthreads();
        // wave-uniform job index: the job record and the column bases stay scalar
        const int jslot = __builtin_amdgcn_readfirstlane(job_s);
        if (jslot >= njobs) return;
        const WgJob jb = jobs[order ? __builtin_amdgcn_readfirstlane(order[jslot]) : jslot];
        // row tile of this job, chosen on the host per size bucket
        if (jb.rpt == 1)
            cd_instance<T, NT, 1>(jb, H, Y, X0, X, info, lambda, T_max, tol, msum, ld_arg, smem_raw, red_s, flag_s, resid, red64, lambda_d);
        else if (jb.rpt == 2)
            cd_instance<T, NT, 2>(jb, H, Y, X0, X, info, lambda, T_max, tol, msum, ld_arg, smem_raw, red_s, flag_s, resid, red64, lambda_d);
        else if (RMAX == 4 || jb.rpt == 4)
            cd_instance<T, NT, 4>(jb, H, Y, X0, X, info, lambda, T_max, tol, msum, ld_arg, smem_raw, red_s, flag_s, resid, red64, lambda_d);
        else
            cd_instance<T, NT, RMAX>(jb, H, Y, X0, X, info, lambda, T_max, tol, msum, ld_arg, smem_raw, red_s, flag_s, resid, red64, lambda_d);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Algorithm 2 (decentralized ZF precoding by CD, eq. (4)), one workgroup per
// cluster.  The local precoded vector x_c (B_c entries) stays in VGPRs with the
// same row ownership as the uplink residual; per user u:
//   a = h_u^H x (partial, wave butterfly, LDS)      e = p_u a - p_u s_u
//   x <- x - e p_u h_u
// with p_u = 1/||h_u|| computed from the same column load in the first sweep
// (Algorithm 2 preprocessing: hbar_u = p_u h_u, sbar_u = p_u s_u).  After the
// sweeps: x_c <- rho_c x_c / ||x_c|| with rho_c = rho / sqrt(C) (Sec. IV-B).
template <typename T, int NT, int RPT>
__device__ __forceinline__ void zf_instance(const WgJob& jb, const cv<T>* __restrict__ H, const cv<T>* __restrict__ S,
                                            cv<T>* __restrict__ X, cdm_info* __restrict__ info, int T_max,
                                            double tol, double rho_c, int64_t ld_arg, unsigned char* smem_raw,
                                            T (*red_s)[NT / 64][3], double* nrm_s, int& flag_s) {
    using V = cv<T>;
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
        const int m = jb.m, n = jb.n;
        const int64_t ld = jb.ld > 0 ? jb.ld : ld_arg;
        const V* Hj = H + jb.h_off;
        T* p_s = reinterpret_cast<T*>(smem_raw);   // p_u (0 marks an inactive user)

        V x[RPT];
#pragma unroll
        for (int q = 0; q < RPT; ++q) x[q] = czero<T>();

        int sweeps = 0;
        double Ssum = 0.0, Xn = 0.0;
        for (int t = 1; t <= T_max; ++t) {
            Ssum = 0.0;
            V hc[RPT], hn[RPT];
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int i = tid + q * NT;
                hc[q] = (i < m) ? Hj[i] : czero<T>();
            }
            for (int u = 0; u < n; ++u) {
                if (u + 1 < n) {
#pragma unroll
                    for (int q = 0; q < RPT; ++q) {
                        const int i = tid + q * NT;
                        hn[q] = (i < m) ? Hj[(int64_t)(u + 1) * ld + i] : czero<T>();
                    }
                }
                T ar = 0, ai = 0, ee = 0;
#pragma unroll
                for (int q = 0; q < RPT; ++q) {
                    ar += hc[q].x * x[q].x + hc[q].y * x[q].y;
                    ai += hc[q].x * x[q].y - hc[q].y * x[q].x;
                    if (t == 1) ee += hc[q].x * hc[q].x + hc[q].y * hc[q].y;
                }
                ar = wave_allsum(ar);
                ai = wave_allsum(ai);
                if (t == 1) ee = wave_allsum(ee);
                const T pu_old = (t > 1) ? p_s[u] : T(0);
                const V su = S[jb.y_off + u];
                const int par = u & 1;
                if (lane == 0) {
                    red_s[par][wid][0] = ar;
                    red_s[par][wid][1] = ai;
                    red_s[par][wid][2] = ee;
                }
                __syncthreads();
                V a = czero<T>();
                T e = 0;
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    a.x += red_s[par][w][0];
                    a.y += red_s[par][w][1];
                    if (t == 1) e += red_s[par][w][2];
                }
                T pu = pu_old;
                if (t == 1) {
                    pu = (e > T(0)) ? T(1) / sqrt(e) : T(0);
                    if (!(e > T(0)) && tid == 0) flag_s |= CDM_INFO_ZERO_COLUMN;
                    if (tid == 0) p_s[u] = pu;
                }
                // err = hbar_u^H x - sbar_u ;  x <- x - err * hbar_u
                V err;
                err.x = pu * a.x - pu * su.x;
                err.y = pu * a.y - pu * su.y;
                V ep;
                ep.x = err.x * pu;
                ep.y = err.y * pu;
#pragma unroll
                for (int q = 0; q < RPT; ++q) cfms(x[q], hc[q], ep);
                if (pu != T(0)) Ssum += cabs2d(err);
#pragma unroll
                for (int q = 0; q < RPT; ++q) hc[q] = hn[q];
            }
            // ||x||^2 (fixed-order block reduction, identical in every thread)
            double xs = 0.0;
#pragma unroll
            for (int q = 0; q < RPT; ++q) xs += cabs2d(x[q]);
            xs = wave_allsum(xs);
            if (lane == 0) nrm_s[wid] = xs;
            __syncthreads();
            Xn = 0.0;
#pragma unroll
            for (int w = 0; w < NW; ++w) Xn += nrm_s[w];
            __syncthreads();
            sweeps = t;
            if (tol > 0.0 && sqrt(Ssum) <= tol * sqrt(Xn)) break;
        }
        // power scaling x_c <- rho_c x_c / ||x_c|| (rho_c <= 0: none; x_c = 0 stays 0)
        const double nrm = sqrt(Xn);
        const double sc = (rho_c > 0.0 && nrm > 0.0) ? rho_c / nrm : 1.0;
        int nf = 0;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int i = tid + q * NT;
            if (i < m) {
                V v;
                v.x = (T)((double)x[q].x * sc);
                v.y = (T)((double)x[q].y * sc);
                if (!isfinite(v.x) || !isfinite(v.y)) nf = 1;
                X[jb.x_off + i] = v;
            }
        }
        if (nf) atomicOr(&flag_s, CDM_INFO_NONFINITE);
        __syncthreads();
        if (tid == 0) {
            const double rel = (Xn > 0.0) ? sqrt(Ssum / Xn) : (Ssum > 0.0 ? INFINITY : 0.0);
            int fl = flag_s;
            if (tol > 0.0 && !(rel <= tol)) fl |= CDM_INFO_NOT_CONVERGED;
            cdm_info o;
            o.sweeps = sweeps;
            o.flags = fl;
            o.rel_step = rel;
            o.resid = -1.0;
            o.reserved = 0.0;
            info[jb.info_idx] = o;
        }
}

template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_zf_wg(const WgJob* __restrict__ jobs, int njobs,
                                              const cv<T>* __restrict__ H, const cv<T>* __restrict__ S,
                                              cv<T>* __restrict__ X, cdm_info* __restrict__ info, int T_max,
                                              double tol, double rho_c, uint32_t* __restrict__ queue,
                                              int64_t ld_arg) {
    constexpr int NW = NT / 64;
    extern __shared__ unsigned char smem_raw[];
    __shared__ T red_s[2][NW][3];
    __shared__ double nrm_s[NW];
    __shared__ int flag_s;
    __shared__ int job_s;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) {
            job_s = (int)atomicAdd(queue, 1u);
            flag_s = 0;
        }
        __syncthreads();
        const int jslot = job_s;
        if (jslot >= njobs) return;
        const WgJob jb = jobs[jslot];
        switch (jb.rpt) {
            case 1: zf_instance<T, NT, 1>(jb, H, S, X, info, T_max, tol, rho_c, ld_arg, smem_raw, red_s, nrm_s, flag_s); break;
            case 2: zf_instance<T, NT, 2>(jb, H, S, X, info, T_max, tol, rho_c, ld_arg, smem_raw, red_s, nrm_s, flag_s); break;
            case 4: zf_instance<T, NT, 4>(jb, H, S, X, info, T_max, tol, rho_c, ld_arg, smem_raw, red_s, nrm_s, flag_s); break;
            default: zf_instance<T, NT, 8>(jb, H, S, X, info, T_max, tol, rho_c, ld_arg, smem_raw, red_s, nrm_s, flag_s); break;
        }
        __syncthreads();
    }
}

template <typename T, int NT> static hipError_t launch_zf_t(const WgLaunch& L, hipStream_t st) {
    const size_t shm = (size_t)L.n_max * sizeof(T);
    hipLaunchKernelGGL((k_zf_wg<T, NT>), dim3(L.grid), dim3(NT), shm, st, L.jobs, L.njobs, (const cv<T>*)L.H,
                       (const cv<T>*)L.Y, (cv<T>*)L.X, L.info, L.T_max, L.tol, L.rho_c, L.queue, L.ld);
    return hipGetLastError();
}

template <typename T, int NT, int RMAX> static hipError_t launch_wg_t(const WgLaunch& L, hipStream_t st) {
    const size_t shm = (size_t)L.n_max * 2 * sizeof(cv<T>);
    hipLaunchKernelGGL((k_cd_wg<T, NT, RMAX>), dim3(L.grid), dim3(NT), shm, st, L.jobs, L.njobs, (const cv<T>*)L.H,
                       (const cv<T>*)L.Y, (const cv<T>*)L.X0, (cv<T>*)L.X, L.info, L.lambda, L.T_max, L.tol,
                       L.order, L.queue, L.msum, L.ld, L.resid);
    return hipGetLastError();
}

template <typename T, int NT, int RMAX> static hipError_t set_lds_t(size_t bytes) {
    hipError_t e = hipFuncSetAttribute((const void*)k_cd_wg<T, NT, RMAX>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_zf_wg<T, NT>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}
template <typename T, int NT, int RMAX> static int occ_t(size_t bytes) {
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_cd_wg<T, NT, RMAX>, NT, bytes) != hipSuccess) return 0;
    return per;
}

// complex128 runs on at most 512 threads (the planner's choice: its 8-rows-per-thread tile
// does not fit the register budget of a 1024-thread workgroup), so no such form is built
#define CDM_WG_DISPATCH_R(FN, c128, nt, rmax, ...)                                             \
    do {                                                                                       \
        if (rmax <= 4) {                                                                       \
            if (c128) {                                                                        \
                if (nt == 128) return FN<double, 128, 4>(__VA_ARGS__);                         \
                if (nt == 256) return FN<double, 256, 4>(__VA_ARGS__);                         \
                if (nt == 512) return FN<double, 512, 4>(__VA_ARGS__);                         \
            } else {                                                                           \
                if (nt == 128) return FN<float, 128, 4>(__VA_ARGS__);                          \
                if (nt == 256) return FN<float, 256, 4>(__VA_ARGS__);                          \
                if (nt == 512) return FN<float, 512, 4>(__VA_ARGS__);                          \
                if (nt == 1024) return FN<float, 1024, 4>(__VA_ARGS__);                        \
            }                                                                                  \
        } else {                                                                               \
            if (c128) {                                                                        \
                if (nt == 128) return FN<double, 128, 8>(__VA_ARGS__);                         \
                if (nt == 256) return FN<double, 256, 8>(__VA_ARGS__);                         \
                if (nt == 512) return FN<double, 512, 8>(__VA_ARGS__);                         \
            } else {                                                                           \
                if (nt == 128) return FN<float, 128, 8>(__VA_ARGS__);                          \
                if (nt == 256) return FN<float, 256, 8>(__VA_ARGS__);                          \
                if (nt == 512) return FN<float, 512, 8>(__VA_ARGS__);                          \
                if (nt == 1024) return FN<float, 1024, 8>(__VA_ARGS__);                        \
            }                                                                                  \
        }                                                                                      \
    } while (0)

#define CDM_WG_DISPATCH(FN, c128, nt, ...)                                   \
    do {                                                                     \
        if (c128) {                                                          \
            if (nt == 128) return FN<double, 128>(__VA_ARGS__);              \
            if (nt == 256) return FN<double, 256>(__VA_ARGS__);              \
            if (nt == 512) return FN<double, 512>(__VA_ARGS__);              \
        } else {                                                             \
            if (nt == 128) return FN<float, 128>(__VA_ARGS__);               \
            if (nt == 256) return FN<float, 256>(__VA_ARGS__);               \
            if (nt == 512) return FN<float, 512>(__VA_ARGS__);               \
            if (nt == 1024) return FN<float, 1024>(__VA_ARGS__);             \
        }                                                                    \
    } while (0)

hipError_t launch_wg(const WgLaunch& L, hipStream_t st) {
    CDM_WG_DISPATCH_R(launch_wg_t, L.c128, L.nt, L.rmax, L, st);
    return hipErrorInvalidValue;
}
hipError_t launch_zf(const WgLaunch& L, hipStream_t st) {
    CDM_WG_DISPATCH(launch_zf_t, L.c128, L.nt, L, st);
    return hipErrorInvalidValue;
}
hipError_t wg_set_lds_limit(bool c128, int nt, int rmax, size_t bytes) {
    CDM_WG_DISPATCH_R(set_lds_t, c128, nt, rmax, bytes);
    return hipErrorInvalidValue;
}
int wg_occupancy(bool c128, int nt, int rmax, size_t bytes) {
    CDM_WG_DISPATCH_R(occ_t, c128, nt, rmax, bytes);
    return 0;
}
size_t wg_lds_bytes(int n_max, bool c128) { return (size_t)n_max * 2 * (c128 ? 16 : 8); }

}  // namespace cdm
