// common.hpp -- device-side building blocks shared by the gfx950 kernels:
// interleaved complex arithmetic, wave64 reductions, cross-workgroup counters.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cdm.h"

namespace cdm {

template <typename T> struct cvec;
template <> struct cvec<double> { using type = double2; };
template <> struct cvec<float> { using type = float2; };
template <typename T> using cv = typename cvec<T>::type;

template <typename T> __device__ __forceinline__ cv<T> czero() { cv<T> z; z.x = T(0); z.y = T(0); return z; }
template <typename T> __device__ __forceinline__ cv<T> cmake(T re, T im) { cv<T> z; z.x = re; z.y = im; return z; }

// a * b
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
    V z; z.x = a.x * b.x - a.y * b.y; z.y = a.x * b.y + a.y * b.x; return z;
}
// acc += conj(a) * b
template <typename V> __device__ __forceinline__ void cfma_conj(V& acc, V a, V b) {
    acc.x += a.x * b.x + a.y * b.y;
    acc.y += a.x * b.y - a.y * b.x;
}
// acc -= a * b
template <typename V> __device__ __forceinline__ void cfms(V& acc, V a, V b) {
    acc.x -= a.x * b.x - a.y * b.y;
    acc.y -= a.x * b.y + a.y * b.x;
}
// acc += a * b
template <typename V> __device__ __forceinline__ void cfma(V& acc, V a, V b) {
    acc.x += a.x * b.x - a.y * b.y;
    acc.y += a.x * b.y + a.y * b.x;
}
template <typename V> __device__ __forceinline__ double cabs2d(V a) {
    return (double)a.x * (double)a.x + (double)a.y * (double)a.y;
}

// Butterfly all-reduce over the 64 lanes of a wave.  Every lane ends with the
// same bits: at each level a lane adds its partner's partial to its own, and the
// two partials of a pair are identical sets, so commutativity makes them equal.
template <typename T> __device__ __forceinline__ T wave_allsum(T v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// Sum over the 64 lanes of a wave into lane 63 only, with DPP moves (no LDS
// permute): quad swaps, row shifts by 4 and 8 (each row of 16 lanes then holds its
// sum in lane 15), then the row-15 and row-31 broadcasts fold the four rows into
// lane 63.  The other lanes end with partial sums.  Fixed order: deterministic.
template <int CTRL, int ROW_MASK> __device__ __forceinline__ float dpp_take(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, false));
}
template <int CTRL, int ROW_MASK> __device__ __forceinline__ double dpp_take(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <typename T> __device__ __forceinline__ T wave_sum_last(T v) {
    v += dpp_take<0xb1, 0xf>(v);    // quad_perm [1,0,3,2]
    v += dpp_take<0x4e, 0xf>(v);    // quad_perm [2,3,0,1]
    v += dpp_take<0x114, 0xf>(v);   // row_shr:4
    v += dpp_take<0x118, 0xf>(v);   // row_shr:8
    v += dpp_take<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
    v += dpp_take<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
    return v;
}

// Transpose-reduce of NV per-lane values (NV a power of two, 1 <= NV <= 64) over
// the 64 lanes.  On return v[0] of lane L holds the full 64-lane sum of value
// index  c = L >> (6 - log2(NV)); all lanes with that high part hold equal bits.
// Cost: NV - 1 + (6 - log2 NV) shuffles instead of 6 NV.
template <typename T, int NV> __device__ __forceinline__ void wave_transpose_sum(T (&v)[NV], int lane) {
    static_assert(NV >= 1 && NV <= 64 && (NV & (NV - 1)) == 0, "NV must be a power of two <= 64");
    int mask = 32;
#pragma unroll
    for (int lvl = 0; (1 << lvl) < NV; ++lvl) {
        const int half = NV >> (lvl + 1);
        const bool upper = (lane & mask) != 0;
#pragma unroll
        for (int i = 0; i < half; ++i) {
            // both values pinned in registers first: a select between two array
            // elements would otherwise become a dynamically indexed (scratch) load
            T lo = v[i], hi = v[i + half];
            asm("" : "+v"(lo), "+v"(hi));
            const T send = upper ? lo : hi;
            const T keep = upper ? hi : lo;
            v[i] = keep + __shfl_xor(send, mask, 64);
        }
        mask >>= 1;
    }
#pragma unroll
    for (; mask >= 1; mask >>= 1) v[0] += __shfl_xor(v[0], mask, 64);
}

// ---- cross-workgroup counters (device-wide, agent scope) --------------------
__device__ __forceinline__ uint32_t ld_relaxed(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void fence_release_agent() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ void fence_acquire_agent() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

// Streaming (non-temporal) load of one complex value: read once, keep it out of
// the way of data that is reused from L2.
typedef double d2v_t __attribute__((ext_vector_type(2)));
typedef float f2v_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld_nt(const double2* p) {
    const d2v_t v = __builtin_nontemporal_load(reinterpret_cast<const d2v_t*>(p));
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ float2 ld_nt(const float2* p) {
    const f2v_t v = __builtin_nontemporal_load(reinterpret_cast<const f2v_t*>(p));
    return make_float2(v.x, v.y);
}

// Device-coherent (agent-scope) relaxed loads and stores of one complex value.
// Used for the small cross-workgroup buffers so that neither side needs an L2
// write-back or invalidate: the stores write through to the device coherence
// point and the loads read from it.
__device__ __forceinline__ void st_dev(double2* p, double2 v) {
    unsigned long long* q = reinterpret_cast<unsigned long long*>(p);
    __hip_atomic_store(q + 0, __double_as_longlong(v.x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(q + 1, __double_as_longlong(v.y), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double2 ld_dev(const double2* p) {
    const unsigned long long* q = reinterpret_cast<const unsigned long long*>(p);
    double2 v;
    v.x = __longlong_as_double(__hip_atomic_load(q + 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    v.y = __longlong_as_double(__hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    return v;
}
__device__ __forceinline__ void st_dev(float2* p, float2 v) {
    unsigned long long* q = reinterpret_cast<unsigned long long*>(p);
    union { float2 f; unsigned long long u; } c;
    c.f = v;
    __hip_atomic_store(q, c.u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float2 ld_dev(const float2* p) {
    const unsigned long long* q = reinterpret_cast<const unsigned long long*>(p);
    union { float2 f; unsigned long long u; } c;
    c.u = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return c.f;
}

// Wait until every vector memory operation this wave issued has completed (for
// the device-coherent stores above: until they have reached the coherence point).
// Issued through the builtin (vmcnt = 0, expcnt and lgkmcnt left at their maxima) so
// that the compiler's own wait tracking knows it happened.
__device__ __forceinline__ void wave_drain_vmem() {
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// All threads of the workgroup: after this workgroup's st_dev stores, bump *ctr.
// Each wave drains its own stores, the barrier orders them before thread 0's
// increment.
__device__ __forceinline__ void wg_arrive(uint32_t* ctr) {
    wave_drain_vmem();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// All threads of the workgroup: wait until *ctr >= target.  Thread 0 polls with a
// wall-clock bound; on time-out it raises *abort_flag, and any waiter that sees
// the flag raised gives up too, so every wave of the grid reaches the kernel end.
// Returns false when the wait was abandoned.  Data published before the counter
// was bumped must be read with ld_dev after this returns.  `flag_s` is one LDS word.
__device__ __forceinline__ bool wg_wait_geq(const uint32_t* ctr, uint32_t target, uint32_t* abort_flag,
                                            uint64_t timeout_ticks, uint32_t* flag_s) {
    if (threadIdx.x == 0) {
        uint32_t ok = 1;
        if (ld_relaxed(ctr) < target) {
            const uint64_t t0 = wall_clock64();
            while (ld_relaxed(ctr) < target) {
                if (ld_relaxed(abort_flag)) { ok = 0; break; }
                if (wall_clock64() - t0 > timeout_ticks) {
                    st_relaxed(abort_flag, 1u);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        *flag_s = ok;
    }
    __syncthreads();
    return *flag_s != 0;
}

// Per-workgroup arrival flags: workgroup w publishes `value` in flags[w] with one
// device-coherent store (no read-modify-write, so arrivals never serialise on one
// address).  Call from all threads after this workgroup's st_dev stores.
__device__ __forceinline__ void wg_publish(uint32_t* flags, int w, uint32_t value) {
    wave_drain_vmem();
    __syncthreads();
    if (threadIdx.x == 0) st_relaxed(&flags[w], value);
}

// All threads: wait until flags[0..count) are all >= target.  Wave 0 polls every
// flag with one vector pass per round and a wave vote; time-out and abort as in
// wg_wait_geq.  `flag_s` is one LDS word.
__device__ __forceinline__ bool wg_wait_flags(const uint32_t* flags, int count, uint32_t target,
                                              uint32_t* abort_flag, uint64_t timeout_ticks, uint32_t* flag_s) {
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        uint32_t ok = 1;
        uint64_t t0 = 0;
        bool started = false;
        for (;;) {
            // all of a lane's flags are loaded before any is tested, so one polling
            // round costs one memory round trip, not one per flag
            bool mine = true;
            for (int base = 0; base < count; base += 256) {
                uint32_t v[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    // clamped, not guarded: a branch-free load sequence issues back to back
                    const int i = min(base + lane + 64 * k, count - 1);
                    v[k] = ld_relaxed(&flags[i]);
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) mine &= (v[k] >= target);
            }
            if (__all(mine)) break;
            if (!started) {
                t0 = wall_clock64();
                started = true;
            }
            if (ld_relaxed(abort_flag)) {
                ok = 0;
                break;
            }
            if (wall_clock64() - t0 > timeout_ticks) {
                if (lane == 0) st_relaxed(abort_flag, 1u);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        if (lane == 0) *flag_s = ok;
    }
    __syncthreads();
    return *flag_s != 0;
}

}  // namespace cdm
