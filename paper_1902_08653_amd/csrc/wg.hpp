// wg.hpp -- pieces shared by the one-workgroup-per-instance kernels.
#pragma once

#include "common.hpp"

namespace cdm {

// FP64 stationarity of eq. (1) for one instance held by one workgroup:
//   ||H^H (y - H x) - lambda x|| / ||H^H y||,
// with r = y - H x formed in FP64 on the thread's rows (thread t owns rows t, t+NT, ...)
// and one fixed-order cross-wave sum per column.  x_s is the instance's x in LDS.
// Every thread returns the same value.
template <typename T, int NT, int RPT>
__device__ double wg_fp64_resid(const cv<T>* __restrict__ Hj, int64_t ld, const cv<T>* __restrict__ Yj,
                                const cv<T>* x_s, int m, int n, double lam64, double (*red64)[NT / 64][4]) {
    using V = cv<T>;
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    double2 r64[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int i = tid + q * NT;
        const V yv = (i < m) ? Yj[i] : czero<T>();
        r64[q] = make_double2((double)yv.x, (double)yv.y);
    }
    for (int u = 0; u < n; ++u) {
        const V xv = x_s[u];
        const double xr = xv.x, xi = xv.y;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int i = tid + q * NT;
            if (i < m) {
                const V h = Hj[(int64_t)u * ld + i];
                r64[q].x -= (double)h.x * xr - (double)h.y * xi;
                r64[q].y -= (double)h.x * xi + (double)h.y * xr;
            }
        }
    }
    double A2 = 0.0, B2 = 0.0;
    for (int u = 0; u < n; ++u) {
        double ar = 0, ai = 0, br = 0, bi = 0;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int i = tid + q * NT;
            if (i < m) {
                const V h = Hj[(int64_t)u * ld + i];
                const V yv = Yj[i];
                const double hr = h.x, hi = h.y;
                ar += hr * r64[q].x + hi * r64[q].y;
                ai += hr * r64[q].y - hi * r64[q].x;
                br += hr * (double)yv.x + hi * (double)yv.y;
                bi += hr * (double)yv.y - hi * (double)yv.x;
            }
        }
        ar = wave_allsum(ar);
        ai = wave_allsum(ai);
        br = wave_allsum(br);
        bi = wave_allsum(bi);
        const int par = u & 1;
        if (lane == 0) {
            red64[par][wid][0] = ar;
            red64[par][wid][1] = ai;
            red64[par][wid][2] = br;
            red64[par][wid][3] = bi;
        }
        __syncthreads();
        double sa = 0, sb = 0, sc = 0, sd = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            sa += red64[par][w][0];
            sb += red64[par][w][1];
            sc += red64[par][w][2];
            sd += red64[par][w][3];
        }
        const V xv = x_s[u];
        sa -= lam64 * (double)xv.x;
        sb -= lam64 * (double)xv.y;
        A2 += sa * sa + sb * sb;
        B2 += sc * sc + sd * sd;
    }
    __syncthreads();
    return B2 > 0.0 ? sqrt(A2 / B2) : sqrt(A2);
}

}  // namespace cdm
