// k_gram_mfma.hip -- panel Gram blocks on gfx950's matrix cores: the low-precision
// copies of H (BF16, FP8-e4m3) of the mixed-precision refinement, and complex128 H.
//
// The mixed-precision refinement runs its inner sweeps on a BF16 or FP8 copy of H, so
// the panel inverses M_K = (D + L)^-1 and the look-ahead cross blocks come from the
// Gram blocks of that copy (the inner problem's own matrix, Alg. 1 applied to the
// correction).  A Gram block is a dense contraction over the B rows:
//
//     G_uv = sum_rows conj(A_u) B_v
//          = (Ar^T Br + Ai^T Bi)_uv + i (Ar^T Bi - Ai^T Br)_uv,
//
// four real products of BF16 or FP8 operands with FP32 accumulation.  Products of two
// BF16 or two FP8 values are exact in FP32, so this is the arithmetic of the FP32
// vector form in another summation order; the MFMA instructions do it at matrix-core
// rate:
//   BF16: v_mfma_f32_16x16x32_bf16   (K = 32 rows per instruction),
//   FP8:  v_mfma_scale_f32_16x16x128_f8f6f4 with format 0 (OCP E4M3) and unit
//         scales (K = 128 rows); the per-128-column block scales s of the copy
//         factor out of the sum over rows, G_uv = s_u s_v (codes product sum).
//
// Workgroup: one 64x64 sub-block of one panel's block over one split of the rows
// (the grid and the partial layout of the FP32/FP64 vector kernel: gpart[split][K]
// [u][v], row-major, summed over splits downstream).  Four waves, each a 32x32
// quadrant (2x2 MFMA tiles, real and imaginary accumulators).  Per step of KS rows
// the workgroup stages the two 64-column tiles (Re and Im planes) in LDS, column by
// column with the rows contiguous, so that a lane's fragment (8 or 32 consecutive
// rows of one column) is one contiguous LDS read.  The k order inside a fragment is
// the same for both operands, so the sum over rows does not depend on how the
// hardware orders k within a fragment.
#include <type_traits>

#include "common.hpp"
#include "launch.hpp"

namespace cdm {

namespace {

typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
typedef int i32x8_t __attribute__((ext_vector_type(8)));

template <int FMT> struct LpFmt;
template <> struct LpFmt<SRC_BF16> {
    using E = uint16_t;
    static constexpr int KS = 32;    // rows per MFMA step
    static constexpr int VEC = 8;    // elements per 16-byte chunk
    static constexpr int PADK = 40;  // LDS elements per staged column (80 B: conflict-free fragment reads)
};
template <> struct LpFmt<SRC_FP8> {
    using E = uint8_t;
    static constexpr int KS = 128;
    static constexpr int VEC = 16;
    static constexpr int PADK = 144;  // 144 B per column
};

// one fragment: this lane's 8 (BF16) or 32 (FP8) consecutive rows of one staged column
struct FragBF16 {
    bf16x8_t v;
};
struct FragFP8 {
    i32x8_t v;
};
__device__ __forceinline__ FragBF16 load_frag(const uint16_t* p, FragBF16*) {
    FragBF16 f;
    f.v = *reinterpret_cast<const bf16x8_t*>(p);
    return f;
}
__device__ __forceinline__ FragFP8 load_frag(const uint8_t* p, FragFP8*) {
    FragFP8 f;
    f.v = *reinterpret_cast<const i32x8_t*>(p);
    return f;
}
// sign flip of every element (BF16: bit 15 of each half; E4M3: bit 7 of each byte)
__device__ __forceinline__ FragBF16 negate(FragBF16 f) {
    u32x4_t u = __builtin_bit_cast(u32x4_t, f.v);
    u ^= 0x80008000u;
    f.v = __builtin_bit_cast(bf16x8_t, u);
    return f;
}
__device__ __forceinline__ FragFP8 negate(FragFP8 f) {
    f.v ^= (int)0x80808080u;
    return f;
}
__device__ __forceinline__ f32x4_t mma(const FragBF16& a, const FragBF16& b, f32x4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, b.v, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4_t mma(const FragFP8& a, const FragFP8& b, f32x4_t c) {
    // A and B format 0 (FP8 E4M3), E8M0 scales 127 (2^0)
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a.v, b.v, c, 0, 0, 0, 127, 0, 127);
}

}  // namespace

template <int FMT, bool CROSS>
__global__ __launch_bounds__(256) void k_gram_lp(const typename LpFmt<FMT>::E* __restrict__ re,
                                                 const typename LpFmt<FMT>::E* __restrict__ im,
                                                 const float* __restrict__ scale, int64_t ld, int B, int U, int kp,
                                                 int nsub, int rows_per_split, float2* __restrict__ gpart,
                                                 int npanels, int dist, int vec_ok) {
    using F = LpFmt<FMT>;
    using E = typename F::E;
    using Frag = typename std::conditional<FMT == SRC_BF16, FragBF16, FragFP8>::type;
    constexpr int KS = F::KS, VEC = F::VEC, PADK = F::PADK;
    constexpr int CHUNKS = 64 * KS / VEC;                    // 16-byte chunks per staged tile
    __shared__ __attribute__((aligned(16))) E tile[4][64 * PADK];   // A re, A im, B re, B im

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;
    const int K = blockIdx.x / nsub;
    int sb = blockIdx.x % nsub;
    int bi = 0, bj = 0;
    if (CROSS) {
        bi = sb / (kp / 64);
        bj = sb % (kp / 64);
    } else {
        while (sb > bi) {   // sub-block (bi, bj), bi >= bj, row by row of the lower triangle
            sb -= bi + 1;
            ++bi;
        }
        bj = sb;
    }
    const int split = blockIdx.y;
    const int r_lo = split * rows_per_split;
    const int r_hi = min(B, r_lo + rows_per_split);
    const int colA0 = K * kp + bi * 64;
    const int colB0 = (CROSS ? (K + npanels - dist % npanels) % npanels : K) * kp + bj * 64;
    const bool same = colA0 == colB0;   // a diagonal sub-block: one tile serves as both operands

    // The KS rows from r0 of 64 columns from c0, as 16-byte chunks (CPT per thread, Re and
    // Im): fetched into registers a step ahead, then put into LDS (Re plane, Im plane).
    constexpr int CPT = CHUNKS / 256;
    union Chunk {
        uint4 q;
        E e[VEC];
    };
    auto fetch = [&](Chunk (&vr)[CPT], Chunk (&vi)[CPT], int c0, int r0) {
#pragma unroll
        for (int m = 0; m < CPT; ++m) {
            const int c = tid + 256 * m;
            const int cl = c / (KS / VEC);
            const int row = r0 + (c % (KS / VEC)) * VEC;
            const int col = c0 + cl;
            if (vec_ok && col < U && row + VEC <= r_hi) {
                const int64_t off = (int64_t)col * ld + row;
                vr[m].q = *reinterpret_cast<const uint4*>(re + off);
                vi[m].q = *reinterpret_cast<const uint4*>(im + off);
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const bool in = col < U && row + e < r_hi;
                    const int64_t off = (int64_t)min(col, U - 1) * ld + min(row + e, B - 1);
                    vr[m].e[e] = in ? re[off] : (E)0;
                    vi[m].e[e] = in ? im[off] : (E)0;
                }
            }
        }
    };
    auto put = [&](const Chunk (&vr)[CPT], const Chunk (&vi)[CPT], E* tr, E* ti) {
#pragma unroll
        for (int m = 0; m < CPT; ++m) {
            const int c = tid + 256 * m;
            const int o = (c / (KS / VEC)) * PADK + (c % (KS / VEC)) * VEC;
            *reinterpret_cast<uint4*>(tr + o) = vr[m].q;
            *reinterpret_cast<uint4*>(ti + o) = vi[m].q;
        }
    };

    const int qi = wv >> 1, qj = wv & 1;   // this wave's 32x32 quadrant
    f32x4_t accr[2][2], acci[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            accr[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
            acci[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
        }
    const int fk = (lane >> 4) * (KS / 4);   // first row of this lane's fragment
    const E* Bre = same ? tile[0] : tile[2];
    const E* Bim = same ? tile[1] : tile[3];
    // BF16: two register sets, the rows of step n + 2 fetched while step n computes, so each
    // step's loads have two steps' time to land before they are put into LDS.  FP8 (a
    // fragment is twice the registers) keeps one set: two would halve its occupancy.
    constexpr bool TWO = FMT == SRC_BF16;
    Chunk ar_[CPT], ai_[CPT], br_[CPT], bi_[CPT];
    Chunk ar2[TWO ? CPT : 1], ai2[TWO ? CPT : 1], br2[TWO ? CPT : 1], bi2[TWO ? CPT : 1];
    if (r_lo < r_hi) {
        fetch(ar_, ai_, colA0, r_lo);
        if (!same) fetch(br_, bi_, colB0, r_lo);
    }
    auto compute = [&]() {
        Frag ar[2], ai[2], an[2], br[2], bim[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int cu = 32 * qi + 16 * i + (lane & 15);
            ar[i] = load_frag(tile[0] + cu * PADK + fk, (Frag*)nullptr);
            ai[i] = load_frag(tile[1] + cu * PADK + fk, (Frag*)nullptr);
            an[i] = negate(ai[i]);
            const int cv_ = 32 * qj + 16 * i + (lane & 15);
            br[i] = load_frag(Bre + cv_ * PADK + fk, (Frag*)nullptr);
            bim[i] = load_frag(Bim + cv_ * PADK + fk, (Frag*)nullptr);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                accr[i][j] = mma(ar[i], br[j], accr[i][j]);
                accr[i][j] = mma(ai[i], bim[j], accr[i][j]);
                acci[i][j] = mma(ar[i], bim[j], acci[i][j]);
                acci[i][j] = mma(an[i], br[j], acci[i][j]);
            }
    };
    if constexpr (!TWO) {
        for (int r0 = r_lo; r0 < r_hi; r0 += KS) {
            put(ar_, ai_, tile[0], tile[1]);
            if (!same) put(br_, bi_, tile[2], tile[3]);
            __syncthreads();
            if (r0 + KS < r_hi) {   // in flight during this step's products
                fetch(ar_, ai_, colA0, r0 + KS);
                if (!same) fetch(br_, bi_, colB0, r0 + KS);
            }
            compute();
            __syncthreads();
        }
    } else {
    if (r_lo + KS < r_hi) {
        fetch(ar2, ai2, colA0, r_lo + KS);
        if (!same) fetch(br2, bi2, colB0, r_lo + KS);
    }
    for (int r0 = r_lo; r0 < r_hi; r0 += 2 * KS) {
        put(ar_, ai_, tile[0], tile[1]);
        if (!same) put(br_, bi_, tile[2], tile[3]);
        __syncthreads();
        if (r0 + 2 * KS < r_hi) {
            fetch(ar_, ai_, colA0, r0 + 2 * KS);
            if (!same) fetch(br_, bi_, colB0, r0 + 2 * KS);
        }
        compute();
        __syncthreads();
        if (r0 + KS >= r_hi) break;   // uniform across the workgroup
        put(ar2, ai2, tile[0], tile[1]);
        if (!same) put(br2, bi2, tile[2], tile[3]);
        __syncthreads();
        if (r0 + 3 * KS < r_hi) {
            fetch(ar2, ai2, colA0, r0 + 3 * KS);
            if (!same) fetch(br2, bi2, colB0, r0 + 3 * KS);
        }
        compute();
        __syncthreads();
    }
    }

    // D[16 x 16]: lane holds rows 4 (lane >> 4) .. + 3 of column lane & 15
    float2* out = gpart + ((int64_t)split * npanels + K) * kp * kp;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int v = 32 * qj + 16 * j + (lane & 15);
            float sv = 1.f;
            if (FMT == SRC_FP8) sv = scale[min(colB0 + v, U - 1) >> 7];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int u = 32 * qi + 16 * i + 4 * (lane >> 4) + e;
                float s = 1.f;
                if (FMT == SRC_FP8) s = scale[min(colA0 + u, U - 1) >> 7] * sv;
                out[(int64_t)(bi * 64 + u) * kp + bj * 64 + v] = make_float2(accr[i][j][e] * s, acci[i][j][e] * s);
            }
        }
}

// Partial Gram blocks of the BF16 or FP8 copy into L.gpart: the diagonal blocks
// (lower sub-blocks, cross = false) or the cross blocks H_K^H H_{K-dist}.
hipError_t launch_gram_lp(const GramLaunch& L, bool cross, int dist, hipStream_t st) {
    if (L.src_kind != SRC_BF16 && L.src_kind != SRC_FP8) return hipErrorInvalidValue;
    if (L.kp % 64 != 0 || L.nsplit < 1) return hipErrorInvalidValue;
    const int nb = L.kp / 64;
    const int nsub = cross ? nb * nb : nb * (nb + 1) / 2;
    const int ks = L.src_kind == SRC_BF16 ? LpFmt<SRC_BF16>::KS : LpFmt<SRC_FP8>::KS;
    const int vec = L.src_kind == SRC_BF16 ? LpFmt<SRC_BF16>::VEC : LpFmt<SRC_FP8>::VEC;
    int rps = (L.B + L.nsplit - 1) / L.nsplit;
    rps = (rps + ks - 1) / ks * ks;
    const int vec_ok = (L.ld % vec) == 0;
    const dim3 grid(L.npanels * nsub, L.nsplit);
    float2* gp = (float2*)L.gpart;
    if (L.src_kind == SRC_BF16) {
        if (cross)
            hipLaunchKernelGGL((k_gram_lp<SRC_BF16, true>), grid, dim3(256), 0, st, L.q_re16, L.q_im16, nullptr, L.ld,
                               L.B, L.U, L.kp, nsub, rps, gp, L.npanels, dist, vec_ok);
        else
            hipLaunchKernelGGL((k_gram_lp<SRC_BF16, false>), grid, dim3(256), 0, st, L.q_re16, L.q_im16, nullptr, L.ld,
                               L.B, L.U, L.kp, nsub, rps, gp, L.npanels, dist, vec_ok);
    } else {
        if (cross)
            hipLaunchKernelGGL((k_gram_lp<SRC_FP8, true>), grid, dim3(256), 0, st, L.q_re8, L.q_im8, L.q_scale, L.ld,
                               L.B, L.U, L.kp, nsub, rps, gp, L.npanels, dist, vec_ok);
        else
            hipLaunchKernelGGL((k_gram_lp<SRC_FP8, false>), grid, dim3(256), 0, st, L.q_re8, L.q_im8, L.q_scale, L.ld,
                               L.B, L.U, L.kp, nsub, rps, gp, L.npanels, dist, vec_ok);
    }
    return hipGetLastError();
}

// ---- complex128 and complex64 -------------------------------------------------------
// The same block partials for complex H on v_mfma_f64_16x16x4_f64 (complex128) or
// v_mfma_f32_16x16x4_f32 (complex64): four rows per instruction, FMA in the element's
// precision.  gfx950's FP64 and FP32 matrix rates equal their vector rates, so this gains
// by issue: one instruction does the work of sixteen wave-wide FMAs, from four operands
// per lane.  Staging: 32 rows of two 64-column tiles per step, split into Re and Im
// planes, column by column with a pitch of 34 elements: the staging writes (consecutive
// rows) and the fragment reads (16 columns x 2 rows per half-wave) are then
// conflict-free.  The two forms differ only in where the output rows sit: lane l holds
// rows (l >> 4) + 4 e of column l & 15 in the FP64 form, and rows 4 (l >> 4) + e in the
// FP32 one.
template <typename T> struct CxMfma;
template <> struct CxMfma<double> {
    typedef double acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int e) { return (lane >> 4) + 4 * e; }
};
template <> struct CxMfma<float> {
    typedef float acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int e) { return 4 * (lane >> 4) + e; }
};
constexpr int G64_KS = 32, G64_PITCH = 34;
// which 64x64 sub-blocks a launch covers: the cross blocks H_K^H H_{K-dist}; the diagonal
// blocks H_K^H H_K of 64-column panels (lower 16x16 tiles only); every sub-block on or below
// the diagonal of wider diagonal blocks (whole sub-blocks, one launch)
enum { GK_CROSS = 0, GK_DIAG = 1, GK_LOWER = 2 };

template <typename T, int KIND>
__device__ __forceinline__ void gram_cx(const cv<T>* __restrict__ H, int64_t ld, int B, int U, int kp, int nsub,
                                        int rows_per_split, cv<T>* __restrict__ gpart, int npanels, int dist) {
    using V = cv<T>;
    using MM = CxMfma<T>;
    using acc_t = typename MM::acc_t;
    // A re, A im, B re, B im; a diagonal sub-block has one tile for both operands
    constexpr int NTL = KIND == GK_DIAG ? 2 : 4;
    __shared__ T tile[NTL][64 * G64_PITCH];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;
    const int K = blockIdx.x / nsub;
    int sb = blockIdx.x % nsub;
    constexpr bool CROSS = KIND == GK_CROSS;
    int bi = 0, bj = 0;
    if (CROSS) {
        bi = sb / (kp / 64);
        bj = sb % (kp / 64);
    } else if (KIND == GK_LOWER) {
        while (sb > bi) {   // (bi, bj), bi >= bj, row by row of the lower triangle
            sb -= bi + 1;
            ++bi;
        }
        bj = sb;
    }
    const int split = blockIdx.y;
    const int r_lo = split * rows_per_split;
    const int r_hi = min(B, r_lo + rows_per_split);
    const int colA0 = K * kp + bi * 64;
    const int colB0 = (CROSS ? (K + npanels - dist % npanels) % npanels : K) * kp + bj * 64;
    const bool same = colA0 == colB0;

    // thread -> row r0 + (tid & 31), columns (tid >> 5) + 8 k of a tile; the next step's
    // values are loaded into registers while this step computes
    auto fetch = [&](V (&v)[8], int c0, int r0) {
        const int row = r0 + (tid & 31);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int col = c0 + (tid >> 5) + 8 * k;
            v[k] = (row < r_hi && col < U) ? ld_nt(H + (int64_t)col * ld + row) : czero<T>();
        }
    };
    auto put = [&](const V (&v)[8], T* tr, T* ti) {
        const int i = tid & 31;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int cl = (tid >> 5) + 8 * k;
            tr[cl * G64_PITCH + i] = v[k].x;
            ti[cl * G64_PITCH + i] = v[k].y;
        }
    };

    const int qi = wv >> 1, qj = wv & 1;
    acc_t accr[2][2], acci[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            accr[i][j] = acc_t{T(0), T(0), T(0), T(0)};
            acci[i][j] = acc_t{T(0), T(0), T(0), T(0)};
        }
    const T* Bre = same ? tile[0] : tile[NTL - 2];
    const T* Bim = same ? tile[1] : tile[NTL - 1];
    // The diagonal block of a 64-column panel is Hermitian, and only its lower triangle
    // (u >= v) is read downstream: its 10 lower 16x16 tiles go to the four waves as 3, 3, 2
    // and 2 tiles, instead of 4 each.  Neighbouring workgroups take the lists in reverse
    // wave order, so that the waves sharing a SIMD even out.
    constexpr bool tri = KIND == GK_DIAG;
    int tti[3] = {0, 0, 0}, ttj[3] = {0, 0, 0}, nt = 0;
    if (tri) {
        const int ws = ((blockIdx.x + blockIdx.y) & 1) ? 3 - wv : wv;
        // wave lists: (3,0)(3,1)(3,2) | (2,0)(2,1)(3,3) | (1,0)(2,2) | (0,0)(1,1)
        if (ws == 0) {
            tti[0] = 3; ttj[0] = 0; tti[1] = 3; ttj[1] = 1; tti[2] = 3; ttj[2] = 2; nt = 3;
        } else if (ws == 1) {
            tti[0] = 2; ttj[0] = 0; tti[1] = 2; ttj[1] = 1; tti[2] = 3; ttj[2] = 3; nt = 3;
        } else if (ws == 2) {
            tti[0] = 1; ttj[0] = 0; tti[1] = 2; ttj[1] = 2; nt = 2;
        } else {
            tti[0] = 0; ttj[0] = 0; tti[1] = 1; ttj[1] = 1; nt = 2;
        }
    }
    V va[8], vb[8];
    if (r_lo < r_hi) {
        fetch(va, colA0, r_lo);
        if (!same) fetch(vb, colB0, r_lo);
    }
    for (int r0 = r_lo; r0 < r_hi; r0 += G64_KS) {
        put(va, tile[0], tile[1]);
        if (!same) put(vb, tile[NTL - 2], tile[NTL - 1]);
        __syncthreads();
        if (r0 + G64_KS < r_hi) {   // in flight during this step's products
            fetch(va, colA0, r0 + G64_KS);
            if (!same) fetch(vb, colB0, r0 + G64_KS);
        }
        if constexpr (tri) {
#pragma unroll 2
            for (int k0 = 0; k0 < G64_KS; k0 += 4) {
                const int rk = k0 + (lane >> 4);
#pragma unroll
                for (int t = 0; t < 3; ++t) {
                    if (t < nt) {   // nt is uniform across the wave
                        const int cu = 16 * tti[t] + (lane & 15);
                        const int cv_ = 16 * ttj[t] + (lane & 15);
                        const T ar = tile[0][cu * G64_PITCH + rk], ai = tile[1][cu * G64_PITCH + rk];
                        const T br = tile[0][cv_ * G64_PITCH + rk], bm = tile[1][cv_ * G64_PITCH + rk];
                        auto& cr = accr[t >> 1][t & 1];
                        auto& ci = acci[t >> 1][t & 1];
                        cr = MM::mma(ar, br, cr);
                        cr = MM::mma(ai, bm, cr);
                        ci = MM::mma(ar, bm, ci);
                        ci = MM::mma(-ai, br, ci);
                    }
                }
            }
        } else {
#pragma unroll 2
            for (int k0 = 0; k0 < G64_KS; k0 += 4) {
                const int rk = k0 + (lane >> 4);   // this lane's row of the 4-row step
                T ar[2], ai[2], br[2], bm[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    const int cu = 32 * qi + 16 * i + (lane & 15);
                    const int cv_ = 32 * qj + 16 * i + (lane & 15);
                    ar[i] = tile[0][cu * G64_PITCH + rk];
                    ai[i] = tile[1][cu * G64_PITCH + rk];
                    br[i] = Bre[cv_ * G64_PITCH + rk];
                    bm[i] = Bim[cv_ * G64_PITCH + rk];
                }
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        accr[i][j] = MM::mma(ar[i], br[j], accr[i][j]);
                        accr[i][j] = MM::mma(ai[i], bm[j], accr[i][j]);
                        acci[i][j] = MM::mma(ar[i], bm[j], acci[i][j]);
                        acci[i][j] = MM::mma(-ai[i], br[j], acci[i][j]);
                    }
            }
        }
        __syncthreads();
    }
    V* out = gpart + ((int64_t)split * npanels + K) * kp * kp;
    if constexpr (tri) {   // the lower tiles only; the upper ones are left unwritten
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            if (t < nt) {
                const int v = 16 * ttj[t] + (lane & 15);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int u = 16 * tti[t] + MM::row(lane, e);
                    out[(int64_t)(bi * 64 + u) * kp + bj * 64 + v] =
                        cmake<T>(accr[t >> 1][t & 1][e], acci[t >> 1][t & 1][e]);
                }
            }
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int v = 32 * qj + 16 * j + (lane & 15);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int u = 32 * qi + 16 * i + MM::row(lane, e);
                out[(int64_t)(bi * 64 + u) * kp + bj * 64 + v] = cmake<T>(accr[i][j][e], acci[i][j][e]);
            }
        }
}

template <int KIND>
__global__ __launch_bounds__(256) void k_gram_f64(const double2* __restrict__ H, int64_t ld, int B, int U, int kp,
                                                  int nsub, int rows_per_split, double2* __restrict__ gpart,
                                                  int npanels, int dist) {
    gram_cx<double, KIND>(H, ld, B, U, kp, nsub, rows_per_split, gpart, npanels, dist);
}
template <int KIND>
__global__ __launch_bounds__(256) void k_gram_f32(const float2* __restrict__ H, int64_t ld, int B, int U, int kp,
                                                  int nsub, int rows_per_split, float2* __restrict__ gpart,
                                                  int npanels, int dist) {
    gram_cx<float, KIND>(H, ld, B, U, kp, nsub, rows_per_split, gpart, npanels, dist);
}

template <int KIND>
static void launch_gram_kind(const GramLaunch& L, int nsub, int rps, int dist, hipStream_t st) {
    const dim3 grid(L.npanels * nsub, L.nsplit);
    if (L.c128)
        hipLaunchKernelGGL((k_gram_f64<KIND>), grid, dim3(256), 0, st, (const double2*)L.H, L.ld, L.B, L.U, L.kp,
                           nsub, rps, (double2*)L.gpart, L.npanels, dist);
    else
        hipLaunchKernelGGL((k_gram_f32<KIND>), grid, dim3(256), 0, st, (const float2*)L.H, L.ld, L.B, L.U, L.kp,
                           nsub, rps, (float2*)L.gpart, L.npanels, dist);
}

hipError_t launch_gram_cx(const GramLaunch& L, bool cross, int dist, hipStream_t st) {
    if (L.src_kind != SRC_COMPLEX || L.kp % 64 != 0 || L.nsplit < 1) return hipErrorInvalidValue;
    const int nb = L.kp / 64;
    int rps = (L.B + L.nsplit - 1) / L.nsplit;
    rps = (rps + G64_KS - 1) / G64_KS * G64_KS;
    if (cross)
        launch_gram_kind<GK_CROSS>(L, nb * nb, rps, dist, st);
    else if (nb == 1)
        launch_gram_kind<GK_DIAG>(L, 1, rps, dist, st);
    else
        launch_gram_kind<GK_LOWER>(L, nb * (nb + 1) / 2, rps, dist, st);
    return hipGetLastError();
}

}  // namespace cdm
