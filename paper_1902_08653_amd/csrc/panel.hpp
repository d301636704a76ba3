// panel.hpp -- types shared by the panel engines (tile sources, kernel arguments).
#pragma once
#include "common.hpp"
#include "launch.hpp"

namespace cdm {

constexpr int PANEL_NT = 512;   // 8 waves per workgroup, one workgroup per CU

// Tile sources: where the sweep reads H from.  `idx` is the element index
// col * ld + row of the column-major B x U matrix, `col` its column.
//
// load_rc(col, row, ld): the same element addressed as a wave-uniform column and a
// per-lane 32-bit row, so that the column base stays in scalar registers and only
// the row offset takes a vector register.
template <typename T> struct SrcC {            // interleaved complex (the caller's H)
    const cv<T>* H;
    __device__ __forceinline__ cv<T> load(int64_t idx, int) const { return ld_nt(H + idx); }
    __device__ __forceinline__ cv<T> load_rc(int col, uint32_t row, int64_t ld) const {
        const char* base = reinterpret_cast<const char*>(H + (int64_t)col * ld);
        return ld_nt(reinterpret_cast<const cv<T>*>(base + row * (uint32_t)sizeof(cv<T>)));
    }
    // raw form kept in registers between load and use (decoding at load time would
    // make the wave wait for the load there)
    using Raw = cv<T>;
    __device__ __forceinline__ Raw load_raw(int col, uint32_t row, int64_t ld) const { return load_rc(col, row, ld); }
    __device__ __forceinline__ cv<T> decode(const Raw& v, int) const { return v; }
};
struct SrcBF16 {                               // planar BF16 copy
    const uint16_t* re;
    const uint16_t* im;
    __device__ __forceinline__ float2 load(int64_t idx, int) const {
        return make_float2(__uint_as_float((uint32_t)re[idx] << 16), __uint_as_float((uint32_t)im[idx] << 16));
    }
    __device__ __forceinline__ float2 load_rc(int col, uint32_t row, int64_t ld) const {
        const int64_t c = (int64_t)col * ld;
        const uint16_t a = *reinterpret_cast<const uint16_t*>(reinterpret_cast<const char*>(re + c) + row * 2u);
        const uint16_t b = *reinterpret_cast<const uint16_t*>(reinterpret_cast<const char*>(im + c) + row * 2u);
        return make_float2(__uint_as_float((uint32_t)a << 16), __uint_as_float((uint32_t)b << 16));
    }
    struct Raw {
        uint32_t re, im;
    };
    __device__ __forceinline__ Raw load_raw(int col, uint32_t row, int64_t ld) const {
        const int64_t c = (int64_t)col * ld;
        Raw v;
        v.re = *reinterpret_cast<const uint16_t*>(reinterpret_cast<const char*>(re + c) + row * 2u);
        v.im = *reinterpret_cast<const uint16_t*>(reinterpret_cast<const char*>(im + c) + row * 2u);
        return v;
    }
    __device__ __forceinline__ float2 decode(const Raw& v, int) const {
        return make_float2(__uint_as_float(v.re << 16), __uint_as_float(v.im << 16));
    }
};
// E4M3 value of code c (bias 7; exponent field 0: subnormal m * 2^-9), times 2^-60.
// Placing the exponent and mantissa fields in the FP32 fields (bits 23.. and 20..)
// gives 2^(e-127) (1 + m/8) for e > 0 and m * 2^-129 (an FP32 subnormal, kept: the
// kernels run with FP32 denormals preserved) for e = 0: both the E4M3 value times
// 2^-120, exactly.  Times 2^60 is exact too.  The caller folds the other 2^60 into its
// scale, so value * scale is rounded once, as from the exact value.
__device__ __forceinline__ float e4m3_bits_scaled(uint32_t c) {
    return __uint_as_float(((c & 0x7fu) << 20) | ((c & 0x80u) << 24)) * 0x1p60f;
}
constexpr float E4M3_UNSCALE = 0x1p60f;
struct SrcFP8 {                                // planar FP8-e4m3 copy, one scale per 128 columns
    const uint8_t* re;
    const uint8_t* im;
    const float* scale;
    // s * 2^60 is exact (a power-of-two factor) for every block scale below 2^68
    __device__ __forceinline__ float2 load(int64_t idx, int col) const {
        const float s = scale[col >> 7] * E4M3_UNSCALE;
        return make_float2(e4m3_bits_scaled(re[idx]) * s, e4m3_bits_scaled(im[idx]) * s);
    }
    __device__ __forceinline__ float2 load_rc(int col, uint32_t row, int64_t ld) const {
        const int64_t c = (int64_t)col * ld;
        const float s = scale[col >> 7] * E4M3_UNSCALE;
        return make_float2(e4m3_bits_scaled(re[c + row]) * s, e4m3_bits_scaled(im[c + row]) * s);
    }
    struct Raw {
        uint32_t re, im;
    };
    __device__ __forceinline__ Raw load_raw(int col, uint32_t row, int64_t ld) const {
        const int64_t c = (int64_t)col * ld;
        Raw v;
        v.re = re[c + row];
        v.im = im[c + row];
        return v;
    }
    __device__ __forceinline__ float2 decode(const Raw& v, int col) const {
        const float s = scale[col >> 7] * E4M3_UNSCALE;
        return make_float2(e4m3_bits_scaled(v.re) * s, e4m3_bits_scaled(v.im) * s);
    }
};
constexpr int PANEL_NWV = PANEL_NT / 64;

template <typename T, class Src> struct PanelArgs {
    Src src;
    int64_t ld;
    const cv<T>* bias;      // optional: added to every b_u (inner correction solve)
    const uint32_t* done;   // optional: nonzero -> return at once (finished refinement)
    const cv<T>* r0;
    cv<T>* x;
    const cv<T>* M;
    const cv<T>* X;         // look-ahead schedule: cross blocks H_K^H H_{K-1}, row-major per panel
    const cv<T>* X2;        // deeper look-ahead: cross blocks H_K^H H_{K-2}, same layout
    cv<T>* part;
    cv<T>* gbuf;
    uint32_t* ctr;
    cdm_info* info;
    double lambda;
    double tol;
    uint64_t timeout_ticks;
    int B, U, npanels, T_max;
};


}  // namespace cdm
