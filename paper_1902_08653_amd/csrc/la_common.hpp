// la_common.hpp -- pieces shared by the look-ahead panel engines: the tagged words of
// the cross-workgroup exchange, the intra-workgroup LDS sequence words, and the row
// reduction of the partial products.
#pragma once
#include "panel.hpp"

namespace cdm {

constexpr int LA_NWT = 8;                 // tile waves
// b formed locally (X_K, 64 KB at most, fits the LDS next to M): complex128 panels
template <typename T, int KP> constexpr bool la_localb() { return (int)sizeof(cv<T>) * KP * KP <= 64 * 1024; }
// tile waves + one control wave (+ one X-staging wave where b is formed locally)
template <typename T, int KP> constexpr int la_threads() { return 64 * (LA_NWT + (la_localb<T, KP>() ? 2 : 1)); }

// Tagged words: a payload and a tag (panel sequence number + 1) in one 64-bit word
// (complex64: 32 + 32 bits; complex128: 48 + 16), stored and loaded single-copy
// atomically at agent scope.  A reader
// that sees the expected tag in every word of a value has that value, so the data is
// its own arrival signal: no store drain, no separate flag and no second read.  The
// exchange buffers are cleared before each launch.
__device__ __forceinline__ void st_tag(uint64_t* p, uint32_t payload, uint32_t tag) {
    __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), ((unsigned long long)tag << 32) | payload,
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_tag(const uint64_t* p) {
    return __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T> struct Tagged;
template <> struct Tagged<double> {
    // complex128: the 128 payload bits in three words of 48 bits, each with a 16-bit tag
    // (sequence + 1 modulo 2^16; a slot is rewritten every second sequence, so the value
    // it held before carries a different tag)
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
    // the words are loaded before any is tested (one memory round trip per attempt)
    __device__ static bool get(const uint64_t* p, uint32_t tag, double2& v) {
        const uint64_t w0 = ld_tag(p + 0), w1 = ld_tag(p + 1), w2 = ld_tag(p + 2);
        const uint64_t t = (uint64_t)(tag & 0xffffu);
        const bool ok = ((w0 >> 48) == t) & ((w1 >> 48) == t) & ((w2 >> 48) == t);
        const uint64_t m = 0xffffffffffffull;
        v.x = __longlong_as_double((long long)((w0 & m) | ((w1 & 0xffffull) << 48)));
        v.y = __longlong_as_double((long long)(((w1 & m) >> 16) | ((w2 & 0xffffffffull) << 32)));
        return ok;
    }
};
template <> struct Tagged<float> {              // complex64: two words
    static constexpr int NW = 2;
    __device__ static void put(uint64_t* p, float2 v, uint32_t tag) {
        st_tag(p + 0, __float_as_uint(v.x), tag);
        st_tag(p + 1, __float_as_uint(v.y), tag);
    }
    __device__ static bool get(const uint64_t* p, uint32_t tag, float2& v) {
        const uint64_t w0 = ld_tag(p + 0), w1 = ld_tag(p + 1);
        const bool ok = ((uint32_t)(w0 >> 32) == tag) & ((uint32_t)(w1 >> 32) == tag);
        v.x = __uint_as_float((uint32_t)w0);
        v.y = __uint_as_float((uint32_t)w1);
        return ok;
    }
};

// ---- intra-workgroup LDS words ------------------------------------------------------
// A writer completes its LDS data writes (lgkmcnt = 0) before it bumps a word; LDS
// operations of one wave are performed in order, so a reader that sees the word
// (and reads after it) sees the data.
__device__ __forceinline__ void lds_wait_writes() {
    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt = 0; vmcnt and expcnt left at their maxima
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}
__device__ __forceinline__ int lds_get(const int* p) {
    const int v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    return v;
}
__device__ __forceinline__ void lds_set(int* p, int v) {
    lds_wait_writes();
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_add(int* p, int v) {
    lds_wait_writes();
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// ---- row sums by DPP ---------------------------------------------------------------
// v of lane i + n within the lane's row of 16 (0 past the row's end): DPP row_shl,
// a register move with no LDS traffic
template <int N> __device__ __forceinline__ double row_shl(double x) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), 0x100 | N, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), 0x100 | N, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
template <int N> __device__ __forceinline__ float row_shl(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x100 | N, 0xF, 0xF, true));
}
// v of lane (i + N) mod 16 within the lane's row of 16: DPP row_ror
template <int N> __device__ __forceinline__ double row_ror(double x) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), 0x120 | N, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), 0x120 | N, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
template <int N> __device__ __forceinline__ float row_ror(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x120 | N, 0xF, 0xF, false));
}
// Rows of 16 (G = 16) or halves of the wave (G = 32) exchanged by gfx950's permlane
// swaps: with both operands v, the first result holds the even rows (lower half) in
// both places and the second the odd rows (upper half), so their sum is the same in
// every lane.
template <int G> __device__ __forceinline__ void swap_pair(uint32_t v, uint32_t& a, uint32_t& b) {
    if constexpr (G == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        a = r[0];
        b = r[1];
    } else {
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        a = r[0];
        b = r[1];
    }
}
template <int G> __device__ __forceinline__ double swap_add(double x) {
    uint32_t al, bl, ah, bh;
    swap_pair<G>((uint32_t)__double2loint(x), al, bl);
    swap_pair<G>((uint32_t)__double2hiint(x), ah, bh);
    return __hiloint2double((int)ah, (int)al) + __hiloint2double((int)bh, (int)bl);
}
template <int G> __device__ __forceinline__ float swap_add(float x) {
    uint32_t a, b;
    swap_pair<G>(__float_as_uint(x), a, b);
    return __uint_as_float(a) + __uint_as_float(b);
}
// Sum over the lanes that agree in their low log2(G) bits (G a power of two): rotations
// within rows of 16, then the row and half-wave swaps.  Every lane of a group ends with
// the same value (each step adds the same two operands in every lane of a pair).
template <int G, typename T> __device__ __forceinline__ T group_sum(T v) {
    if constexpr (G < 16) {
        v += row_ror<G>(v);
        return group_sum<2 * G>(v);
    } else if constexpr (G < 64) {
        return group_sum<2 * G>(swap_add<G>(v));
    } else {
        return v;
    }
}
// value of lane l (uniform l) in every lane
__device__ __forceinline__ double lane_value(double x, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), l),
                            __builtin_amdgcn_readlane(__double2loint(x), l));
}
__device__ __forceinline__ float lane_value(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

// Transpose-reduce of 4 values per lane (as wave_transpose_sum<T, 4>): the two exchange
// levels across half- and quarter-waves, then the sum over each row of 16 lanes by DPP
// shifts into the row's first lane (lanes 0, 16, 32, 48 hold the four sums)
template <typename T> __device__ __forceinline__ void transpose_sum4_rows(T (&v)[4], int lane) {
    int mask = 32;
#pragma unroll
    for (int lvl = 0; lvl < 2; ++lvl) {
        const int half = 2 >> lvl;
        const bool upper = (lane & mask) != 0;
#pragma unroll
        for (int i = 0; i < half; ++i) {
            T lo = v[i], hi = v[i + half];
            asm("" : "+v"(lo), "+v"(hi));
            const T send = upper ? lo : hi;
            const T keep = upper ? hi : lo;
            v[i] = keep + __shfl_xor(send, mask, 64);
        }
        mask >>= 1;
    }
    v[0] += row_shl<1>(v[0]);
    v[0] += row_shl<2>(v[0]);
    v[0] += row_shl<4>(v[0]);
    v[0] += row_shl<8>(v[0]);
}

}  // namespace cdm
