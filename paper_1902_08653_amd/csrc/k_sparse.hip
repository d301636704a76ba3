// k_sparse.hip -- sparse channel (CSR input) path of Algorithm 1.
//
// Coordinate descent walks columns, so the CSR matrix (rows = antennas) is first
// transposed to a column-compressed form with rows ascending inside each column
// (an integer step: counts, prefix sum, atomic fill, then a per-column sort by
// row, which makes the result unique and independent of the fill order).
//
// Columns are taken in panels of 64 whose mutual coupling is resolved exactly with
// the panel Gram blocks of the sparse columns (row-list intersections) -- the same
// block form of the cyclic sweep as the dense panel engine:
// delta_K = (D + L)^-1 (g_K - lambda x_K).  The sweep is spread over row slices, one
// workgroup each, that hold their part of the residual in LDS; a panel costs each
// workgroup a few hundred stored entries and one exchange of 64 partial sums.
#include <algorithm>

#include "common.hpp"
#include "launch.hpp"

namespace cdm {

// ---- CSR -> CSC --------------------------------------------------------------
// Validation of the caller's CSR arrays before any indexed write: rowptr[0] == 0,
// rowptr non-decreasing, rowptr[B] == nnz, and in every row column indices in [0, U)
// and strictly increasing.  A violation sets CDM_INFO_BAD_INPUT in *status; the kernels
// that index with the caller's arrays then do nothing, so the column-compressed form
// stays empty (every column without entries) and every access stays in bounds.
__global__ void k_csr_check(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colidx, int B, int U,
                            int64_t nnz, uint32_t* __restrict__ status) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B) return;
    const int32_t a0 = rowptr[i], a1 = rowptr[i + 1];
    bool bad = a0 < 0 || a1 < a0 || (int64_t)a1 > nnz;
    if (i == 0 && a0 != 0) bad = true;
    if (i == B - 1 && (int64_t)a1 != nnz) bad = true;
    if (!bad) {
        int32_t prev = -1;
        for (int32_t k = a0; k < a1; ++k) {
            const int32_t c = colidx[k];
            if (c <= prev || c >= U) {   // c <= prev also catches c < 0 (prev >= -1)
                bad = true;
                break;
            }
            prev = c;
        }
    }
    if (bad) atomicOr(status, (uint32_t)CDM_INFO_BAD_INPUT);
}

__device__ __forceinline__ bool csr_bad(const uint32_t* status) {
    return (__atomic_load_n(status, __ATOMIC_RELAXED) & (uint32_t)CDM_INFO_BAD_INPUT) != 0u;
}

__global__ void k_csr_count(const int32_t* __restrict__ colidx, int64_t nnz, int32_t* __restrict__ cnt,
                            const uint32_t* status) {
    if (csr_bad(status)) return;
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
__global__ __launch_bounds__(256) void k_csr_fill(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colidx,
                                                  const cv<T>* __restrict__ val, int B, int32_t* __restrict__ fill,
                                                  int32_t* __restrict__ rowidx, cv<T>* __restrict__ cval,
                                                  const uint32_t* status) {
    // one wave per row: the row's entries take their slots in parallel, one returning atomic
    // each (the order within a column is arbitrary either way; k_csc_sort puts it in row order)
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= B || csr_bad(status)) return;
    for (int32_t k = rowptr[i] + lane; k < rowptr[i + 1]; k += 64) {
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
        // rank sort: each entry's position = number of smaller rows (rows are unique).
        // The column is in LDS, so each entry goes to its place in global memory at once.
        __builtin_amdgcn_wave_barrier();
        for (int k = lane; k < len; k += 64) {
            const int32_t rk = rs[wid][k];
            int p = 0;
            for (int j = 0; j < len; ++j) p += rs[wid][j] < rk ? 1 : 0;
            rowidx[e0 + p] = rk;
            cval[e0 + p] = vs[wid][k];
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
// SG_SPLIT workgroups per panel, one thread per (u >= v) pair, two-pointer merge of the
// two sorted row lists.  The merge is a chain of dependent loads, so the panel's row
// indices are staged in LDS first when they fit (SG_LDS entries, 64 KB); the values are
// read from global memory on matches only.  Output row-major [npanels][kp][kp] (lower part).
constexpr int SG_SPLIT = 4, SG_LDS = 16384;
template <typename T>
__global__ __launch_bounds__(256) void k_sparse_gram(const int32_t* __restrict__ colptr, const int32_t* __restrict__ rowidx,
                                                     const cv<T>* __restrict__ cval, int U, int kp,
                                                     cv<T>* __restrict__ G) {
    __shared__ int32_t rs[SG_LDS];
    const int K = blockIdx.x;
    const int npair = kp * (kp + 1) / 2;
    const int c0 = K * kp, c1 = min(U, c0 + kp);
    const int32_t base = colptr[c0];
    const int32_t cnt = colptr[c1] - base;
    const bool staged = cnt <= SG_LDS;
    if (staged)
        for (int k = threadIdx.x; k < cnt; k += blockDim.x) rs[k] = rowidx[base + k];
    __syncthreads();
    // the merge of columns u and v, with the row index of entry k from ld(k)
    auto merge = [&](int u, int v, auto ld, double& sr, double& si) {
        int32_t i = colptr[u], ie = colptr[u + 1];
        int32_t j = colptr[v], je = colptr[v + 1];
        while (i < ie && j < je) {
            const int32_t ri = ld(i), rj = ld(j);
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
    };
    for (int pidx = threadIdx.x + blockDim.x * blockIdx.y; pidx < npair; pidx += blockDim.x * SG_SPLIT) {
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
            if (staged)
                merge(u, v, [&](int32_t k) { return rs[k - base]; }, sr, si);
            else
                merge(u, v, [&](int32_t k) { return rowidx[k]; }, sr, si);
        }
        G[((int64_t)K * kp + a) * kp + b] = cmake<T>((T)sr, (T)si);
    }
}

// ---- row slices of the column-compressed form --------------------------------
// spt[s * U + u] = first entry of column u whose row is >= s * R (s = 0..P), so the
// entries of column u inside row slice s are [spt[s*U+u], spt[(s+1)*U+u]).
__global__ void k_sparse_slices(const int32_t* __restrict__ colptr, const int32_t* __restrict__ rowidx, int B,
                                int U, int P, int R, int32_t* __restrict__ spt) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)(P + 1) * U) return;
    const int s = (int)(k / U), u = (int)(k % U);
    const int64_t bound = min((int64_t)s * R, (int64_t)B);
    int32_t lo = colptr[u], hi = colptr[u + 1];
    while (lo < hi) {                       // lower bound of `bound` in the sorted rows
        const int32_t mid = lo + (hi - lo) / 2;
        if (rowidx[mid] < bound) lo = mid + 1; else hi = mid;
    }
    spt[k] = lo;
}

// ---- the sweep ---------------------------------------------------------------
// P workgroups, one per slice of R consecutive rows (antennas).  Each keeps its slice
// of r in LDS for the whole solve and walks the panels of 64 columns in order:
//   1. partial  p_s = H_{K,s}^H r_s  (its rows only; entries prefetched a panel ahead)
//   2. exchange: every workgroup publishes p_s and reads all P partials (tagged words,
//      one memory round trip), summing them in slice order, so every workgroup holds
//      the same b_K = sum_s p_s - lambda x_K bit for bit;
//   3. delta_K = (D + L)^-1 b_K and x_K += delta_K, computed redundantly everywhere;
//   4. r_s -= H_{K,s} delta_K through the row-ordered input (one thread per row: no
//      two threads touch one r entry, no atomics).
// The stopping sums are formed from the identical deltas, so all workgroups stop
// after the same sweep.  Each workgroup keeps a private copy of x (xp).
namespace {

// Tagged words: a 32-bit payload and a 32-bit tag (panel sequence + 1) in one 64-bit
// word, stored and loaded single-copy atomically at agent scope; a value whose words
// all carry the expected tag has arrived.  The buffer is cleared before each launch.
__device__ __forceinline__ void sp_st(uint64_t* p, uint32_t payload, uint32_t tag) {
    __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), ((unsigned long long)tag << 32) | payload,
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t sp_ld(const uint64_t* p) {
    return __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T> struct SpTag;
template <> struct SpTag<double> {
    // complex128: the 128 payload bits in three words of 48 bits, each with a 16-bit tag
    // (tag = sequence + 1 modulo 2^16; a slot is rewritten every second sequence, so the
    // value it held before carries a different tag)
    static constexpr int NW = 3;
    __device__ static void st48(uint64_t* p, uint64_t payload, uint32_t tag) {
        __hip_atomic_store(reinterpret_cast<unsigned long long*>(p),
                           (unsigned long long)((payload & 0xffffffffffffull) | ((uint64_t)(tag & 0xffffu) << 48)),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ static void put(uint64_t* p, double2 v, uint32_t tag) {
        const uint64_t a = (uint64_t)__double_as_longlong(v.x), b = (uint64_t)__double_as_longlong(v.y);
        st48(p + 0, a, tag);
        st48(p + 1, (a >> 48) | (b << 16), tag);
        st48(p + 2, b >> 32, tag);
    }
    __device__ static bool decode(const uint64_t (&wd)[3], uint32_t tag, double2& v) {
        const uint64_t t = (uint64_t)(tag & 0xffffu);
        const bool ok = ((wd[0] >> 48) == t) & ((wd[1] >> 48) == t) & ((wd[2] >> 48) == t);
        const uint64_t m = 0xffffffffffffull;
        const uint64_t a = (wd[0] & m) | ((wd[1] & 0xffffull) << 48);
        const uint64_t b = ((wd[1] & m) >> 16) | ((wd[2] & 0xffffffffull) << 32);
        v.x = __longlong_as_double((long long)a);
        v.y = __longlong_as_double((long long)b);
        return ok;
    }
};
template <> struct SpTag<float> {
    static constexpr int NW = 2;
    __device__ static void put(uint64_t* p, float2 v, uint32_t tag) {
        sp_st(p + 0, __float_as_uint(v.x), tag);
        sp_st(p + 1, __float_as_uint(v.y), tag);
    }
    __device__ static bool decode(const uint64_t (&wd)[2], uint32_t tag, float2& v) {
        const uint64_t w0 = wd[0], w1 = wd[1];
        const bool ok = ((uint32_t)(w0 >> 32) == tag) & ((uint32_t)(w1 >> 32) == tag);
        v.x = __uint_as_float((uint32_t)w0);
        v.y = __uint_as_float((uint32_t)w1);
        return ok;
    }
};

template <typename T> __device__ __forceinline__ T sp_quad_sum(T v) {
    v += dpp_take<0xb1, 0xf>(v);   // quad_perm [1,0,3,2]
    v += dpp_take<0x4e, 0xf>(v);   // quad_perm [2,3,0,1]
    return v;
}

}  // namespace

constexpr int SR_NT = 256;                // 4 waves
constexpr int SR_KP = 64;                 // panel width
constexpr int SR_G = SR_NT / SR_KP;       // threads per column in the partial (a quad)
#ifndef CDM_SPARSE_EG
#define CDM_SPARSE_EG 6
#endif
constexpr int SR_EG = CDM_SPARSE_EG;      // block entries per thread held in registers
constexpr int SR_SC = 4;                  // slices read per exchange attempt (per thread)
constexpr int SR_CAP = 1024;              // scatter staging (block entries per pass)
constexpr int SR_RMAX = SR_NT * 16;       // largest slice

// ---- row order inside each (slice, panel) block --------------------------------
// The entries of block (s, K) -- rows of slice s, columns of panel K -- are held by the
// sweep in column order.  pi[e] is entry e's position in the block's (row, column)
// order, so that the update r -= H delta can add each row's terms in a fixed order.
// Stored with the entry's row inside the slice: pk[e] = pi << 12 | (row - s * R)
// (R <= 4096, and a block holds at most 64 R entries).  bcnt[s * npanels + K] is the
// block's entry count, and roff[(s * npanels + K) * (R + 1) + i] the first position of
// the slice's row i in that order (i = R: the count).  One workgroup per block: count
// the entries per row, prefix-sum, then place the columns one after another (the rows
// of one column are distinct, so each row's next slot is taken at most once per step).
__global__ __launch_bounds__(256) void k_sparse_rank(const int32_t* __restrict__ rowidx,
                                                     const int32_t* __restrict__ spt, int U, int npanels,
                                                     int R, int32_t* __restrict__ pk, int32_t* __restrict__ bcnt,
                                                     int32_t* __restrict__ roff) {
    __shared__ int32_t cnt[SR_RMAX], fill[SR_RMAX];
    __shared__ int32_t wsum[256 / 64];
    const int s = blockIdx.x / npanels, K = blockIdx.x % npanels;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int row0 = s * R;
    for (int i = tid; i < R; i += 256) cnt[i] = 0;
    __syncthreads();
    const int ncol = min(SR_KP, U - K * SR_KP);
    for (int c = 0; c < ncol; ++c) {
        const int u = K * SR_KP + c;
        const int32_t lo = spt[(int64_t)s * U + u], hi = spt[(int64_t)(s + 1) * U + u];
        for (int32_t e = lo + tid; e < hi; e += 256) atomicAdd(&cnt[rowidx[e] - row0], 1);
    }
    __syncthreads();
    // exclusive prefix sum of cnt[0..R) into fill (each thread a contiguous run)
    const int per = (R + 255) / 256;
    const int i0 = min(R, tid * per), i1 = min(R, i0 + per);
    int32_t run = 0;
    for (int i = i0; i < i1; ++i) run += cnt[i];
    int32_t incl = run;
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        const int32_t o = __shfl_up(incl, m, 64);
        if (lane >= m) incl += o;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int32_t base = incl - run;
    for (int k = 0; k < w; ++k) base += wsum[k];
    int32_t* ro = roff + ((int64_t)s * npanels + K) * (R + 1);
    for (int i = i0; i < i1; ++i) {
        fill[i] = base;
        ro[i] = base;
        base += cnt[i];
    }
    if (tid == 255) {
        bcnt[(int64_t)s * npanels + K] = base;
        ro[R] = base;
    }
    __syncthreads();
    for (int c = 0; c < ncol; ++c) {
        const int u = K * SR_KP + c;
        const int32_t lo = spt[(int64_t)s * U + u], hi = spt[(int64_t)(s + 1) * U + u];
        for (int32_t e = lo + tid; e < hi; e += 256) {
            const int r = rowidx[e] - row0;
            pk[e] = (fill[r] << 12) | r;
            fill[r] += 1;
        }
        __syncthreads();
    }
}

struct SparseRsArgs {
    const void* cval;        // column-compressed values (rows ascending per column)
    const int32_t* pk;       // row-order position in the block << 12 | row in the slice
    const int32_t* spt;      // [P+1][U] slice pointers
    const int32_t* bcnt;     // [P][npanels] block entry counts
    const int32_t* roff;     // [P][npanels][R+1] row starts inside each block (row order)
    const void* M;           // [npanels] packed (D + L)^-1, column-major lower
    const void* r0;          // r = y - H x0 (B)
    void* x;                 // in: x0 (U); out: x
    void* xp;                // [P][U] private copies of x
    uint64_t* xbuf;          // [2][P][64][NW] tagged partials
    uint32_t* abort_flag;
    cdm_info* info;
    int64_t nnz;
    int B, U, npanels, R, T_max;
    double lambda, tol;
    uint64_t tmo;
};

// Every prefetch below is an unconditional load from a clamped (in-bounds) index whose
// validity is decided where the value is used, so no load waits for another.
template <typename T, int RPT>
__global__ __launch_bounds__(SR_NT) void k_cd_sparse(const SparseRsArgs a) {
    using V = cv<T>;
    using TG = SpTag<T>;
    constexpr int NT = SR_NT, KP = SR_KP, NE = KP * (KP + 1) / 2, NWV = NT / 64, NW = TG::NW;
    constexpr int MPT = (NE + NT - 1) / NT;
    constexpr int VPW = KP / NWV;          // matvec columns per wave
    __shared__ V rs[NT * RPT];
    __shared__ V Ms[NE];
    __shared__ V bsh[KP], dsh[KP];
    __shared__ V cbuf[SR_CAP];
    __shared__ double stop_s[NWV][2];
    __shared__ int fail_s;

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int s = blockIdx.x, P = gridDim.x;
    const int U = a.U, np = a.npanels;
    const int row0 = s * a.R;
    const int nrow = max(0, min(a.R, a.B - row0));
    const int32_t ncsc = (int32_t)max(a.nnz, (int64_t)1) - 1;   // last valid internal entry
    const int32_t* __restrict__ pkg = a.pk;
    const int32_t* __restrict__ spt = a.spt;
    const V* __restrict__ cval = (const V*)a.cval;
    const V* __restrict__ Mg = (const V*)a.M;
    V* xp = (V*)a.xp + (int64_t)s * U;
    const T lambda = (T)a.lambda;

    for (int i = tid; i < nrow; i += NT) rs[i] = ((const V*)a.r0)[row0 + i];
    for (int u = tid; u < U; u += NT) xp[u] = ((const V*)a.x)[u];
    if (tid == 0) fail_s = 0;

    // block mapping: column jl = tid / 4, quad member gq.  An empty range stands for a
    // padding column (u >= U).
    const int jl = tid >> 2, gq = tid & 3;
    auto ptrs = [&](int K, int32_t& lo, int32_t& hi) {
        const int u = min(K * KP + jl, U - 1);
        lo = spt[(int64_t)s * U + u];
        hi = spt[(int64_t)(s + 1) * U + u];
    };
    auto live = [&](int K, int32_t lo, int32_t hi) { return K * KP + jl < U ? hi : lo; };
    // entries of the current panel (ek, ev) and of the next one (nk, nv)
    int32_t ek[SR_EG], nk[SR_EG];
    V ev[SR_EG], nv[SR_EG];
    auto fetch_entries = [&](int32_t lo) {
#pragma unroll
        for (int k = 0; k < SR_EG; ++k) {
            const int32_t e = min(lo + gq + SR_G * k, ncsc);
            nk[k] = pkg[e];
            nv[k] = cval[e];
        }
    };
    // pointers run two panels ahead of the entries, the entries one panel ahead of use
    int32_t glo, ghi, nlo, nhi, lo1, hi1, lo2, hi2;
    ptrs(0, nlo, nhi);
    nhi = live(0, nlo, nhi);
    fetch_entries(nlo);
    ptrs(1 % np, lo1, hi1);
    ptrs(2 % np, lo2, hi2);
    int32_t nb_next = a.bcnt[(int64_t)s * np];
    // the owned rows' slot ranges in the current block (ro*) and the next one (rn*)
    int32_t ro0[RPT], ro1[RPT], rn0[RPT], rn1[RPT];
    auto fetch_roff = [&](int K) {
        const int32_t* ro = a.roff + ((int64_t)s * np + K) * (a.R + 1);
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int i = min(tid + q * NT, a.R);
            rn0[q] = ro[i];
            rn1[q] = ro[min(i + 1, a.R)];
        }
    };
    fetch_roff(0);
    // M_{K+1}, loaded during panel K into registers (scalar arrays: kept in registers)
    T mre[MPT], mim[MPT];
    auto fetch_M = [&](int K) {
        const V* Mk = Mg + (int64_t)K * NE;
#pragma unroll
        for (int k = 0; k < MPT; ++k) {
            const V m = Mk[min(tid + k * NT, NE - 1)];
            mre[k] = m.x;
            mim[k] = m.y;
        }
    };
    for (int e = tid; e < NE; e += NT) Ms[e] = Mg[e];
    const int cl = w * 16 + (lane & 15), grp = lane >> 4;
    __syncthreads();

    double S = 0.0, Xn = 0.0;     // stopping sums (group-0 lanes of each wave)
    int sweeps = 0;
    bool failed = false;
    uint32_t seq = 0;
    for (int t = 1; t <= a.T_max && !failed; ++t) {
        S = 0.0;
        Xn = 0.0;
        for (int K = 0; K < np; ++K, ++seq) {
            const int K1 = (K + 1) % np, K3 = (K + 3) % np;
            const uint32_t tag = seq + 1;
            const int par = (int)(seq & 1);
            // the prefetched block becomes the current one
            glo = nlo;
            ghi = nhi;
            const int32_t nb = nb_next;
#pragma unroll
            for (int k = 0; k < SR_EG; ++k) {
                ek[k] = nk[k];
                ev[k] = nv[k];
            }
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                ro0[q] = rn0[q];
                ro1[q] = rn1[q];
            }
            // 1. partial of this slice (reads from clamped indices, products masked: no
            //    branch between the LDS reads; entries past the register window: direct loads)
            {
                V p = czero<T>();
#pragma unroll
                for (int k = 0; k < SR_EG; ++k) {
                    const bool ok = glo + gq + SR_G * k < ghi;
                    const V rv = rs[ok ? (ek[k] & 4095) : 0];
                    V h = ev[k];
                    h.x = ok ? h.x : T(0);
                    h.y = ok ? h.y : T(0);
                    cfma_conj(p, h, rv);
                }
                for (int32_t e = glo + gq + SR_G * SR_EG; e < ghi; e += SR_G)
                    cfma_conj(p, cval[e], rs[pkg[e] & 4095]);
                p.x = sp_quad_sum(p.x);
                p.y = sp_quad_sum(p.y);
                if (gq == 0) TG::put(a.xbuf + (((int64_t)par * P + s) * KP + jl) * NW, p, tag);
            }
            // 2. prefetch: the next panel's block, the pointers after that, M_{K+1}
            fetch_entries(lo1);
            nlo = lo1;
            nhi = live(K1, lo1, hi1);
            lo1 = lo2;
            hi1 = hi2;
            ptrs(K3, lo2, hi2);
            nb_next = a.bcnt[(int64_t)s * np + K1];
            fetch_roff(K1);
            fetch_M(K1);
            // exchange and panel product: wave w owns columns [16 w, 16 w + 16); lane l
            // takes column cl = 16 w + (l & 15) and group l >> 4 of the slices (exchange)
            // or of the v range (panel product), the four groups meeting in a butterfly
            const int uK = K * KP + cl;
            V xK = xp[min(uK, U - 1)];   // used after the exchange
            // 3. exchange: group g sums slices g, g + 4, ... of column cl in order; each
            //    attempt issues all of its loads before testing any tag
            {
                V acc = czero<T>();
                for (int s0 = 0; s0 < P && !failed; s0 += NWV * SR_SC) {
                    V v[SR_SC];
                    bool have[SR_SC];
#pragma unroll
                    for (int k = 0; k < SR_SC; ++k) {
                        v[k] = czero<T>();
                        have[k] = s0 + NWV * k + grp >= P;
                    }
                    uint64_t t0 = 0;
                    bool started = false;
                    for (;;) {
                        // slices the whole wave already holds are not read again
                        uint64_t wd[SR_SC][NW];
#pragma unroll
                        for (int k = 0; k < SR_SC; ++k) {
                            const uint64_t* src =
                                a.xbuf + (((int64_t)par * P + min(s0 + NWV * k + grp, P - 1)) * KP + cl) * NW;
                            const bool want = __any(!have[k]);
#pragma unroll
                            for (int i = 0; i < NW; ++i) wd[k][i] = want ? sp_ld(src + i) : 0;
                        }
                        bool miss = false;
#pragma unroll
                        for (int k = 0; k < SR_SC; ++k) {
                            V got;
                            const bool ok = TG::decode(wd[k], tag, got);
                            if (!have[k] && ok) {
                                v[k] = got;
                                have[k] = true;
                            }
                            miss |= !have[k];
                        }
                        if (!__any(miss)) break;
                        if (!started) {
                            t0 = wall_clock64();
                            started = true;
                        }
                        if (ld_relaxed(a.abort_flag) || wall_clock64() - t0 > a.tmo) {
                            if (lane == 0) st_relaxed(a.abort_flag, 1u);
                            failed = true;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
#pragma unroll
                    for (int k = 0; k < SR_SC; ++k) {
                        acc.x += v[k].x;
                        acc.y += v[k].y;
                    }
                }
                acc.x += __shfl_xor(acc.x, 16, 64);
                acc.y += __shfl_xor(acc.y, 16, 64);
                acc.x += __shfl_xor(acc.x, 32, 64);
                acc.y += __shfl_xor(acc.y, 32, 64);
                if (uK >= U) xK = czero<T>();
                if (grp == 0) bsh[cl] = cmake<T>(acc.x - lambda * xK.x, acc.y - lambda * xK.y);
                if (failed && lane == 0) fail_s = 1;
            }
            __syncthreads();
            if (fail_s) {
                failed = true;
                break;
            }
            // 4. delta = (D + L)^-1 b: lane (j = cl, group g) sums v in [16 g, 16 g + 16),
            //    v <= j (every read index stays inside the packed triangle; v > j is masked)
            {
                const int j = cl, v0 = grp * VPW;
                V d = czero<T>();
#pragma unroll
                for (int k = 0; k < VPW; ++k) {
                    const int v = v0 + k;
                    V m = Ms[v * KP - (v * (v - 1)) / 2 + (j - v)];
                    const V bb = bsh[v];
                    m.x = v <= j ? m.x : T(0);
                    m.y = v <= j ? m.y : T(0);
                    cfma(d, m, bb);
                }
                d.x += __shfl_xor(d.x, 16, 64);
                d.y += __shfl_xor(d.y, 16, 64);
                d.x += __shfl_xor(d.x, 32, 64);
                d.y += __shfl_xor(d.y, 32, 64);
                xK = cmake<T>(xK.x + d.x, xK.y + d.y);
                if (grp == 0) {
                    dsh[cl] = d;
                    if (uK < U) {
                        S += cabs2d(d);
                        Xn += cabs2d(xK);
                        xp[uK] = xK;
                    }
                }
            }
            __syncthreads();
            // stage M_{K+1} (its loads were issued before the exchange; the panel product
            // that read M_K is done)
#pragma unroll
            for (int k = 0; k < MPT; ++k) {
                const int e = tid + k * NT;
                if (e < NE) Ms[e] = cmake<T>(mre[k], mim[k]);
            }
            // 5. r_s -= H_{K,s} delta: every entry's term goes to its row-order slot of the
            //    block, then each thread adds its own rows' slots in order (blocks larger
            //    than the staging area take several passes)
            {
                const V dj = dsh[jl];
                for (int c0 = 0; c0 < nb; c0 += SR_CAP) {
#pragma unroll
                    for (int k = 0; k < SR_EG; ++k) {
                        const int q = (ek[k] >> 12) - c0;
                        if (glo + gq + SR_G * k < ghi && q >= 0 && q < SR_CAP) cbuf[q] = cmul(ev[k], dj);
                    }
                    for (int32_t e = glo + gq + SR_G * SR_EG; e < ghi; e += SR_G) {
                        const int q = (pkg[e] >> 12) - c0;
                        if (q >= 0 && q < SR_CAP) cbuf[q] = cmul(cval[e], dj);
                    }
                    __syncthreads();
                    const int lim = min(SR_CAP, nb - c0);
                    int qa[RPT], qb[RPT];
                    V acc[RPT], rv[RPT];
#pragma unroll
                    for (int q = 0; q < RPT; ++q) {
                        const bool own = tid + q * NT < nrow;
                        qa[q] = max(ro0[q] - c0, 0);
                        qb[q] = own ? min(ro1[q] - c0, lim) : 0;
                        acc[q] = cbuf[qa[q] < qb[q] ? qa[q] : 0];
                        rv[q] = rs[own ? tid + q * NT : 0];
                    }
#pragma unroll
                    for (int q = 0; q < RPT; ++q) {
                        if (qa[q] >= qb[q]) continue;
                        for (int j = qa[q] + 1; j < qb[q]; ++j) {
                            acc[q].x += cbuf[j].x;
                            acc[q].y += cbuf[j].y;
                        }
                        rv[q].x -= acc[q].x;
                        rv[q].y -= acc[q].y;
                        rs[tid + q * NT] = rv[q];
                    }
                    __syncthreads();
                }
            }
        }
        if (failed) break;
        sweeps = t;
        {
            const double s1 = wave_allsum(S), s2 = wave_allsum(Xn);
            if (lane == 0) {
                stop_s[w][0] = s1;
                stop_s[w][1] = s2;
            }
        }
        __syncthreads();
        S = stop_s[0][0];
        Xn = stop_s[0][1];
#pragma unroll
        for (int k = 1; k < NWV; ++k) {
            S += stop_s[k][0];
            Xn += stop_s[k][1];
        }
        __syncthreads();
        if (a.tol > 0.0 && sqrt(S) <= a.tol * sqrt(Xn)) break;
    }
    if (s == 0) {
        for (int u = tid; u < U; u += NT) ((V*)a.x)[u] = xp[u];
        if (tid == 0) {
            const double rel = (Xn > 0.0) ? sqrt(S / Xn) : (S > 0.0 ? INFINITY : 0.0);
            int fl = 0;
            if (a.tol > 0.0 && !(rel <= a.tol)) fl |= CDM_INFO_NOT_CONVERGED;
            cdm_info o;
            o.sweeps = sweeps;
            o.flags = fl;
            o.rel_step = rel;
            o.resid = -1.0;
            o.reserved = 0.0;
            a.info[0] = o;
        }
    }
}

// r = y - H x0 (one thread per row, through the row-ordered input: fixed order, no
// atomics) and x = x0 (or 0)
template <typename T>
__global__ void k_sparse_init(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colidx,
                              const cv<T>* __restrict__ val, const cv<T>* __restrict__ y, int B,
                              const cv<T>* __restrict__ x0, int U, cv<T>* __restrict__ r, cv<T>* __restrict__ x,
                              const uint32_t* status) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < B) {
        cv<T> ri = y[i];
        if (x0 && !csr_bad(status))
            for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) cfms(ri, val[e], x0[colidx[e]]);
        r[i] = ri;
    }
    if (i < U) x[i] = x0 ? x0[i] : czero<T>();
}

template <typename T, int RPT> static hipError_t launch_sweep_t(const SparseRsArgs& A, int P, hipStream_t st) {
    void* args[] = {(void*)&A};
    return hipLaunchCooperativeKernel((const void*)k_cd_sparse<T, RPT>, dim3(P), dim3(SR_NT), args, 0, st);
}

template <typename T> static hipError_t launch_sparse_t(const SparseLaunch& L, hipStream_t st) {
    using V = cv<T>;
    // 1. CSR -> column-compressed, rows ascending per column
    hipError_t e = launch_zero_u32((uint32_t*)L.colptr, L.U + 1, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_csr_check, dim3((L.B + 255) / 256), dim3(256), 0, st, L.rowptr, L.colidx, L.B, L.U, L.nnz,
                       L.status);
    if (L.nnz > 0) {
        int64_t blocks = (L.nnz + 255) / 256;
        if (blocks > 65536) blocks = 65536;
        hipLaunchKernelGGL(k_csr_count, dim3((unsigned)blocks), dim3(256), 0, st, L.colidx, L.nnz, L.colptr,
                           L.status);
    }
    hipLaunchKernelGGL(k_scan_inplace, dim3(1), dim3(1024), 0, st, L.colptr, L.U + 1, L.fill);
    hipLaunchKernelGGL((k_csr_fill<T>), dim3((L.B + 3) / 4), dim3(256), 0, st, L.rowptr, L.colidx,
                       (const V*)L.val, L.B, L.fill, L.rowidx, (V*)L.cval, L.status);
    hipLaunchKernelGGL((k_csc_sort<T>), dim3((L.U + 3) / 4), dim3(256), 0, st, L.colptr, L.U, L.rowidx, (V*)L.cval);
    e = hipGetLastError();
    if (e != hipSuccess || L.transpose_only) return e;
    // 2. panel Gram blocks and (D + L)^-1
    hipLaunchKernelGGL((k_sparse_gram<T>), dim3(L.npanels, SG_SPLIT), dim3(256), 0, st, L.colptr, L.rowidx,
                       (const V*)L.cval, L.U, SR_KP, (V*)L.gpart);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_gram_invert(L.c128, L.gpart, 1, L.npanels, SR_KP, L.U, L.lambda, L.M, L.e, L.status, st);
    if (e != hipSuccess) return e;
    // 3. row slices, init, sweeps
    const int64_t nsp = (int64_t)(L.P + 1) * L.U;
    hipLaunchKernelGGL(k_sparse_slices, dim3((unsigned)((nsp + 255) / 256)), dim3(256), 0, st, L.colptr, L.rowidx,
                       L.B, L.U, L.P, L.R, L.spt);
    hipLaunchKernelGGL(k_sparse_rank, dim3((unsigned)(L.P * L.npanels)), dim3(256), 0, st, L.rowidx, L.spt, L.U,
                       L.npanels, L.R, L.pi, L.bcnt, L.roff);
    const int n = L.B > L.U ? L.B : L.U;
    hipLaunchKernelGGL((k_sparse_init<T>), dim3((n + 255) / 256), dim3(256), 0, st, L.rowptr, L.colidx,
                       (const V*)L.val, (const V*)L.y, L.B, (const V*)L.x0, L.U, (V*)L.r, (V*)L.x, L.status);
    e = launch_zero_u32((uint32_t*)L.xbuf, (int64_t)2 * L.P * SR_KP * SpTag<T>::NW * 2, st);
    if (e != hipSuccess) return e;
    SparseRsArgs A;
    A.cval = L.cval;
    A.pk = L.pi;
    A.spt = L.spt;
    A.bcnt = L.bcnt;
    A.roff = L.roff;
    A.M = L.M;
    A.r0 = L.r;
    A.x = L.x;
    A.xp = L.xp;
    A.xbuf = L.xbuf;
    A.abort_flag = L.abort_flag;
    A.info = L.info;
    A.nnz = L.nnz;
    A.B = L.B;
    A.U = L.U;
    A.npanels = L.npanels;
    A.R = L.R;
    A.T_max = L.T_max;
    A.lambda = L.lambda;
    A.tol = L.tol;
    A.tmo = L.timeout_ticks;
    if (L.ev_sweep0) (void)hipEventRecord(L.ev_sweep0, st);
    const int rpt = sparse_rows_per_thread(L.R);
    switch (rpt) {
        case 1: e = launch_sweep_t<T, 1>(A, L.P, st); break;
        case 2: e = launch_sweep_t<T, 2>(A, L.P, st); break;
        case 4: e = launch_sweep_t<T, 4>(A, L.P, st); break;
        case 8: e = launch_sweep_t<T, 8>(A, L.P, st); break;
        case 16: e = launch_sweep_t<T, 16>(A, L.P, st); break;
        default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    if (L.ev_sweep1) (void)hipEventRecord(L.ev_sweep1, st);
    return hipGetLastError();
}

// rows per thread of the sweep for slices of R rows: the power of two >= R / 256
int sparse_rows_per_thread(int R) {
    int rpt = 1;
    while (rpt * SR_NT < R) rpt *= 2;
    return rpt * SR_NT <= SR_RMAX ? rpt : 0;
}

void sparse_slices(int B, int ncu, int& P, int& R) {
    P = (B + CDM_SPARSE_SLICE_ROWS - 1) / CDM_SPARSE_SLICE_ROWS;
    P = std::max(1, std::min(P, std::min(64, ncu)));
    R = (B + P - 1) / P;
}

hipError_t launch_sparse(const SparseLaunch& L, hipStream_t st) {
    return L.c128 ? launch_sparse_t<double>(L, st) : launch_sparse_t<float>(L, st);
}

}  // namespace cdm
