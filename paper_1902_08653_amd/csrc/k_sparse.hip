// k_sparse.hip -- sparse channel (CSR input) path of Algorithm 1.
//
// Coordinate descent walks columns, so the CSR matrix (rows = antennas) is first
// transposed to a column-compressed form with rows ascending inside each column
// (an integer step: counts, prefix sum, atomic fill, then a per-column sort by
// row, which makes the result unique and independent of the fill order).
//
// The sweep runs in ONE workgroup (the whole operator is a few tens of MB and the
// dependent chain is the bottleneck, not bandwidth).  Columns are taken in panels
// of 64 whose mutual coupling is resolved exactly with the panel Gram blocks of
// the sparse columns (row-list intersections) -- the same block form of the
// cyclic sweep as the dense panel engine: delta_K = (D + L)^-1 (g_K - lambda x_K).
// The residual r lives in global memory and is updated with atomic adds, since
// the columns of one panel may share rows.
#include "common.hpp"
#include "launch.hpp"

namespace cdm {

// ---- CSR -> CSC --------------------------------------------------------------
__global__ void k_csr_count(const int32_t* __restrict__ colidx, int64_t nnz, int32_t* __restrict__ cnt) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += stride)
        atomicAdd(&cnt[colidx[k] + 1], 1);
}

// exclusive prefix sum of cnt[0..n] in place (cnt[0] == 0 on entry), one workgroup
__global__ __launch_bounds__(1024) void k_scan_inplace(int32_t* __restrict__ a, int n1, int32_t* __restrict__ fill) {
    __shared__ int32_t part[1024];
    const int tid = threadIdx.x;
    const int per = (n1 + 1023) / 1024;
    const int lo = tid * per, hi = min(n1, lo + per);
    int32_t s = 0;
    for (int i = lo; i < hi; ++i) s += a[i];
    part[tid] = s;
    __syncthreads();
    if (tid == 0) {
        int32_t run = 0;
        for (int k = 0; k < 1024; ++k) {
            const int32_t v = part[k];
            part[k] = run;
            run += v;
        }
    }
    __syncthreads();
    int32_t run = part[tid];
    for (int i = lo; i < hi; ++i) {
        run += a[i];
        a[i] = run;            // inclusive scan of the shifted counts = column starts
    }
    __syncthreads();
    for (int i = lo; i < hi; ++i)
        if (i < n1 - 1) fill[i] = a[i];
}

template <typename T>
__global__ void k_csr_fill(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colidx,
                           const cv<T>* __restrict__ val, int B, int32_t* __restrict__ fill,
                           int32_t* __restrict__ rowidx, cv<T>* __restrict__ cval) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B) return;
    for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
        const int32_t pos = atomicAdd(&fill[colidx[k]], 1);
        rowidx[pos] = i;
        cval[pos] = val[k];
    }
}

// one wave per column: sort its (row, value) pairs by row (insertion sort in LDS)
template <typename T>
__global__ __launch_bounds__(256) void k_csc_sort(const int32_t* __restrict__ colptr, int U,
                                                  int32_t* __restrict__ rowidx, cv<T>* __restrict__ cval) {
    constexpr int CAP = 512;
    __shared__ int32_t rs[4][CAP];
    __shared__ cv<T> vs[4][CAP];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int u = blockIdx.x * 4 + wid;
    if (u >= U) return;
    const int32_t e0 = colptr[u], e1 = colptr[u + 1];
    const int len = e1 - e0;
    if (len <= CAP) {
        for (int k = lane; k < len; k += 64) {
            rs[wid][k] = rowidx[e0 + k];
            vs[wid][k] = cval[e0 + k];
        }
        // rank sort: each entry's position = number of smaller rows (rows are unique)
        __builtin_amdgcn_wave_barrier();
        int32_t myr[CAP / 64];
        cv<T> myv[CAP / 64];
        int myp[CAP / 64];
#pragma unroll
        for (int q = 0; q < CAP / 64; ++q) {
            const int k = lane + 64 * q;
            myp[q] = -1;
            if (k < len) {
                const int32_t rk = rs[wid][k];
                int p = 0;
                for (int j = 0; j < len; ++j) p += rs[wid][j] < rk ? 1 : 0;
                myr[q] = rk;
                myv[q] = vs[wid][k];
                myp[q] = p;
            }
        }
#pragma unroll
        for (int q = 0; q < CAP / 64; ++q)
            if (myp[q] >= 0) {
                rowidx[e0 + myp[q]] = myr[q];
                cval[e0 + myp[q]] = myv[q];
            }
    } else if (lane == 0) {
        // long column: in-place insertion sort by one lane
        for (int32_t a = e0 + 1; a < e1; ++a) {
            const int32_t rk = rowidx[a];
            const cv<T> vk = cval[a];
            int32_t b = a - 1;
            while (b >= e0 && rowidx[b] > rk) {
                rowidx[b + 1] = rowidx[b];
                cval[b + 1] = cval[b];
                --b;
            }
            rowidx[b + 1] = rk;
            cval[b + 1] = vk;
        }
    }
}

// ---- sparse panel Gram: G_uv = sum over common rows of conj(h_u) h_v ---------
// One workgroup per panel, one thread per (u >= v) pair, two-pointer merge of the
// two sorted row lists.  Output row-major [npanels][kp][kp] (lower part).
template <typename T>
__global__ __launch_bounds__(256) void k_sparse_gram(const int32_t* __restrict__ colptr, const int32_t* __restrict__ rowidx,
                                                     const cv<T>* __restrict__ cval, int U, int kp,
                                                     cv<T>* __restrict__ G) {
    const int K = blockIdx.x;
    const int npair = kp * (kp + 1) / 2;
    for (int pidx = threadIdx.x; pidx < npair; pidx += blockDim.x) {
        // pair index -> (a >= b) in row-major lower order
        int a = 0, rem = pidx;
        while (rem > a) {
            rem -= a + 1;
            ++a;
        }
        const int b = rem;
        const int u = K * kp + a, v = K * kp + b;
        double sr = 0.0, si = 0.0;
        if (u < U && v < U) {
            int32_t i = colptr[u], ie = colptr[u + 1];
            int32_t j = colptr[v], je = colptr[v + 1];
            while (i < ie && j < je) {
                const int32_t ri = rowidx[i], rj = rowidx[j];
                if (ri == rj) {
                    const cv<T> hu = cval[i], hv = cval[j];
                    sr += (double)hu.x * hv.x + (double)hu.y * hv.y;
                    si += (double)hu.x * hv.y - (double)hu.y * hv.x;
                    ++i;
                    ++j;
                } else if (ri < rj) {
                    ++i;
                } else {
                    ++j;
                }
            }
        }
        G[((int64_t)K * kp + a) * kp + b] = cmake<T>((T)sr, (T)si);
    }
}

// ---- the sweep ---------------------------------------------------------------
constexpr int SP_NT = 1024;
constexpr int SP_KP = 64;
constexpr int SP_NW = SP_NT / 64;            // 16 waves
constexpr int SP_CPW = SP_KP / SP_NW;        // 4 columns per wave

// The residual is changed only by this workgroup's device-scope atomic adds; it is
// read back with device-coherent loads (ld_dev), so no stale cached copy is used.
template <typename T>
__global__ __launch_bounds__(SP_NT) void k_cd_sparse(const int32_t* __restrict__ colptr,
                                                     const int32_t* __restrict__ rowidx,
                                                     const cv<T>* __restrict__ cval, cv<T>* __restrict__ r,
                                                     cv<T>* __restrict__ x, const cv<T>* __restrict__ M, int U,
                                                     int npanels, double lambda_d, int T_max, double tol,
                                                     cdm_info* __restrict__ info) {
    using V = cv<T>;
    constexpr int NE = SP_KP * (SP_KP + 1) / 2;
    constexpr int NS = SP_NT / SP_KP;       // matvec slices per row
    constexpr int SV = SP_KP / NS;
    __shared__ V Ms[NE];
    __shared__ V bsh[SP_KP], xsh[SP_KP], dsh[SP_KP];
    __shared__ V dpart[NS][SP_KP];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const T lambda = (T)lambda_d;
    int sweeps = 0;
    double S = 0.0, Xn = 0.0;
    for (int t = 1; t <= T_max; ++t) {
        S = 0.0;
        Xn = 0.0;
        for (int K = 0; K < npanels; ++K) {
            // stage the packed (D + L)^-1 of this panel
            const V* Mk = M + (int64_t)K * NE;
            for (int e = tid; e < NE; e += SP_NT) Ms[e] = Mk[e];
            // g_u = h_u^H r over the stored entries, one wave per column
#pragma unroll
            for (int c = 0; c < SP_CPW; ++c) {
                const int jl = wid * SP_CPW + c;
                const int u = K * SP_KP + jl;
                T gr = 0, gi = 0;
                if (u < U) {
                    const int32_t e0 = colptr[u], e1 = colptr[u + 1];
                    for (int32_t e = e0 + lane; e < e1; e += 64) {
                        const V h = cval[e];
                        const V rv = ld_dev(&r[rowidx[e]]);
                        gr += h.x * rv.x + h.y * rv.y;
                        gi += h.x * rv.y - h.y * rv.x;
                    }
                }
                gr = wave_allsum(gr);
                gi = wave_allsum(gi);
                if (lane == 0) {
                    const V xo = (u < U) ? ld_dev(&x[u]) : czero<T>();
                    bsh[jl] = cmake<T>(gr - lambda * xo.x, gi - lambda * xo.y);
                    xsh[jl] = xo;
                }
            }
            __syncthreads();
            {
                const int j = tid % SP_KP, sl = tid / SP_KP;
                const int v0 = sl * SV, v1 = min(v0 + SV - 1, j);
                V d = czero<T>();
                int off = v0 * SP_KP - (v0 * (v0 - 1)) / 2 + (j - v0);
                for (int v = v0; v <= v1; ++v) {
                    cfma(d, Ms[off], bsh[v]);
                    off += SP_KP - v - 1;
                }
                dpart[sl][j] = d;
            }
            __syncthreads();
            if (tid < SP_KP) {
                V s = dpart[0][tid];
#pragma unroll
                for (int k = 1; k < NS; ++k) {
                    s.x += dpart[k][tid].x;
                    s.y += dpart[k][tid].y;
                }
                dsh[tid] = s;
                const int u = K * SP_KP + tid;
                if (u < U) st_dev(&x[u], cmake<T>(xsh[tid].x + s.x, xsh[tid].y + s.y));
            }
            __syncthreads();
            {
                double s1 = 0.0, s2 = 0.0;
                for (int j = lane; j < SP_KP; j += 64) {
                    const V d = dsh[j];
                    s1 += cabs2d(d);
                    s2 += cabs2d(cmake<T>(xsh[j].x + d.x, xsh[j].y + d.y));
                }
                S += wave_allsum(s1);
                Xn += wave_allsum(s2);
            }
            // r -= h_u delta_u for every stored entry of the panel (rows may repeat
            // across the panel's columns: atomic adds)
#pragma unroll
            for (int c = 0; c < SP_CPW; ++c) {
                const int jl = wid * SP_CPW + c;
                const int u = K * SP_KP + jl;
                if (u < U) {
                    const V d = dsh[jl];
                    const int32_t e0 = colptr[u], e1 = colptr[u + 1];
                    for (int32_t e = e0 + lane; e < e1; e += 64) {
                        const V h = cval[e];
                        V* rp = &r[rowidx[e]];
                        atomicAdd(&rp->x, -(h.x * d.x - h.y * d.y));
                        atomicAdd(&rp->y, -(h.x * d.y + h.y * d.x));
                    }
                }
            }
            wave_drain_vmem();
            __syncthreads();
        }
        sweeps = t;
        if (tol > 0.0 && sqrt(S) <= tol * sqrt(Xn)) break;
    }
    if (tid == 0) {
        const double rel = (Xn > 0.0) ? sqrt(S / Xn) : (S > 0.0 ? INFINITY : 0.0);
        int fl = 0;
        if (tol > 0.0 && !(rel <= tol)) fl |= CDM_INFO_NOT_CONVERGED;
        cdm_info o;
        o.sweeps = sweeps;
        o.flags = fl;
        o.rel_step = rel;
        o.resid = -1.0;
        o.reserved = 0.0;
        info[0] = o;
    }
}

// r = y, x = x0 (or 0); warm start: r -= H x0 through the column-compressed form
template <typename T>
__global__ void k_sparse_init(const cv<T>* __restrict__ y, int B, const cv<T>* __restrict__ x0, int U,
                              cv<T>* __restrict__ r, cv<T>* __restrict__ x) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < B) r[i] = y[i];
    if (i < U) x[i] = x0 ? x0[i] : czero<T>();
}
template <typename T>
__global__ void k_sparse_warm(const int32_t* __restrict__ colptr, const int32_t* __restrict__ rowidx,
                              const cv<T>* __restrict__ cval, const cv<T>* __restrict__ x0, int U,
                              cv<T>* __restrict__ r) {
    const int u = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (u >= U) return;
    const cv<T> xv = x0[u];
    for (int32_t e = colptr[u] + lane; e < colptr[u + 1]; e += 64) {
        const cv<T> h = cval[e];
        cv<T>* rp = &r[rowidx[e]];
        atomicAdd(&rp->x, -(h.x * xv.x - h.y * xv.y));
        atomicAdd(&rp->y, -(h.x * xv.y + h.y * xv.x));
    }
}

template <typename T> static hipError_t launch_sparse_t(const SparseLaunch& L, hipStream_t st) {
    using V = cv<T>;
    // 1. CSR -> column-compressed, rows ascending per column
    hipError_t e = launch_zero_u32((uint32_t*)L.colptr, L.U + 1, st);
    if (e != hipSuccess) return e;
    if (L.nnz > 0) {
        int64_t blocks = (L.nnz + 255) / 256;
        if (blocks > 65536) blocks = 65536;
        hipLaunchKernelGGL(k_csr_count, dim3((unsigned)blocks), dim3(256), 0, st, L.colidx, L.nnz, L.colptr);
    }
    hipLaunchKernelGGL(k_scan_inplace, dim3(1), dim3(1024), 0, st, L.colptr, L.U + 1, L.fill);
    hipLaunchKernelGGL((k_csr_fill<T>), dim3((L.B + 255) / 256), dim3(256), 0, st, L.rowptr, L.colidx,
                       (const V*)L.val, L.B, L.fill, L.rowidx, (V*)L.cval);
    hipLaunchKernelGGL((k_csc_sort<T>), dim3((L.U + 3) / 4), dim3(256), 0, st, L.colptr, L.U, L.rowidx, (V*)L.cval);
    e = hipGetLastError();
    if (e != hipSuccess || L.transpose_only) return e;
    // 2. panel Gram blocks and (D + L)^-1
    hipLaunchKernelGGL((k_sparse_gram<T>), dim3(L.npanels), dim3(256), 0, st, L.colptr, L.rowidx, (const V*)L.cval,
                       L.U, SP_KP, (V*)L.gpart);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_gram_invert(L.c128, L.gpart, 1, L.npanels, SP_KP, L.U, L.lambda, L.M, L.e, L.status, st);
    if (e != hipSuccess) return e;
    // 3. init and sweeps
    const int n = L.B > L.U ? L.B : L.U;
    hipLaunchKernelGGL((k_sparse_init<T>), dim3((n + 255) / 256), dim3(256), 0, st, (const V*)L.y, L.B,
                       (const V*)L.x0, L.U, (V*)L.r, (V*)L.x);
    if (L.x0)
        hipLaunchKernelGGL((k_sparse_warm<T>), dim3((L.U + 3) / 4), dim3(256), 0, st, L.colptr, L.rowidx,
                           (const V*)L.cval, (const V*)L.x0, L.U, (V*)L.r);
    if (L.ev_sweep0) (void)hipEventRecord(L.ev_sweep0, st);
    hipLaunchKernelGGL((k_cd_sparse<T>), dim3(1), dim3(SP_NT), 0, st, L.colptr, L.rowidx, (const V*)L.cval, (V*)L.r,
                       (V*)L.x, (const V*)L.M, L.U, L.npanels, L.lambda, L.T_max, L.tol, L.info);
    if (L.ev_sweep1) (void)hipEventRecord(L.ev_sweep1, st);
    return hipGetLastError();
}

hipError_t launch_sparse(const SparseLaunch& L, hipStream_t st) {
    return L.c128 ? launch_sparse_t<double>(L, st) : launch_sparse_t<float>(L, st);
}

}  // namespace cdm
