// k_panel_la.hip -- look-ahead schedule of the panel engine.
//
// Same block form of the cyclic sweep as k_cd_panel (delta_K = M_K b_K with
// M_K = (D + L)^-1 of the panel Gram, b_K = H_K^H r - lambda x_K), but the partial
// products of panel K+1 are formed from the residual *before* panel K's update and
// corrected afterwards:
//     H_{K+1}^H (r - H_K delta_K) = H_{K+1}^H r - X_{K+1} delta_K,
//     X_{K+1} = H_{K+1}^H H_K  (formed once per solve, next to M).
// The exchange of panel K+1's partials therefore overlaps the wait for panel K's
// reduced b, and only one cross-workgroup hop per panel sits on the critical path.
// In exact arithmetic every delta is the same as in the sequential sweep.
//
// Workgroup: 8 tile waves and one control wave.  Tile waves own the rows (lane =
// row) and NC panel columns each; they keep three panels in registers (K for the
// update, K+1 for the look-ahead partial, K+2 in flight) and touch global memory
// only to stream H.  The control wave does every cross-workgroup exchange (partials
// out, flags, reducer sums, the reduced b in, the panel inverse into LDS).  Memory
// operations complete in issue order per wave, so a flag poll issued by a tile wave
// would wait for that wave's tile stream; keeping the two in different waves keeps
// the stream off the critical path.
#include "panel.hpp"

namespace cdm {

constexpr int LA_NWT = 8;                 // tile waves
constexpr int LA_NT = 64 * (LA_NWT + 1);  // + one control wave

// One wave: wait until flags[0..count) are all >= target.  Same time-out and abort
// protocol as wg_wait_flags, without a workgroup barrier.  Uniform result.
__device__ __forceinline__ bool wave_wait_flags(const uint32_t* flags, int count, uint32_t target,
                                                uint32_t* abort_flag, uint64_t timeout_ticks) {
    const int lane = threadIdx.x & 63;
    uint64_t t0 = 0;
    bool started = false;
    for (;;) {
        bool mine = true;
        for (int base = 0; base < count; base += 256) {
            uint32_t v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = ld_relaxed(&flags[min(base + lane + 64 * k, count - 1)]);
#pragma unroll
            for (int k = 0; k < 4; ++k) mine &= (v[k] >= target);
        }
        if (__all(mine)) return true;
        if (!started) {
            t0 = wall_clock64();
            started = true;
        }
        if (ld_relaxed(abort_flag)) return false;
        if (wall_clock64() - t0 > timeout_ticks) {
            if (lane == 0) st_relaxed(abort_flag, 1u);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// One wave: after this wave's st_dev stores, set flags[w] = value.
__device__ __forceinline__ void wave_publish(uint32_t* flags, int w, uint32_t value) {
    wave_drain_vmem();
    if ((threadIdx.x & 63) == 0) st_relaxed(&flags[w], value);
}

template <typename T, int KP, int RPL, class Src>
__global__ __launch_bounds__(LA_NT, 1) void k_cd_panel_la(PanelArgs<T, Src> a) {
    using V = cv<T>;
    constexpr int NC = KP / LA_NWT;             // panel columns per tile wave
    static_assert(NC >= 1 && NC <= 64 && (NC & (NC - 1)) == 0, "bad panel split");
    constexpr int NE = KP * (KP + 1) / 2;       // packed lower triangle of M_K
    constexpr int NS = 64 * LA_NWT / KP;        // matvec slices per row (tile threads)
    constexpr int KL = (KP + 63) / 64;          // panel entries per control lane

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    const bool ctl = wid == LA_NWT;
    const int w = blockIdx.x;
    const int P = gridDim.x;                    // the planner guarantees P >= KP
    const bool reducer = w < KP;                // reducer w owns panel column j = w
    const int B = a.B, U = a.U, np = a.npanels;
    const T lambda = (T)a.lambda;
    if (a.done && *a.done) return;              // uniform for the whole grid

    // packed M_K, staged by the control wave with LDS-direct loads in 1 KiB rows (the
    // array is padded to whole rows; M's buffer extends past its last panel)
    constexpr int MS_BYTES = (NE * (int)sizeof(V) + 1023) / 1024 * 1024;
    __shared__ __attribute__((aligned(16))) V Ms[MS_BYTES / sizeof(V)];
    __shared__ V psh[KP];                       // this workgroup's look-ahead partials
    __shared__ V bsh[KP];
    __shared__ V xsh[KP];
    __shared__ V dsh[KP];
    constexpr int SCR = (NS * KP > LA_NWT * RPL * 64) ? NS * KP : LA_NWT * RPL * 64;
    __shared__ V scr[SCR];
    V(*dpart)[KP] = reinterpret_cast<V(*)[KP]>(scr);
    V(*axs)[RPL][64] = reinterpret_cast<V(*)[RPL][64]>(scr);
    __shared__ int ctl_s;                       // 0 run, 1 stop after this sweep, 2 abandoned

    // ctr layout: [2] abort, [3] status, [16, 16+P) partial flags, [16+P, 16+P+KP)
    // reducer flags; a flag holds (panel sequence number of the published data) + 1
    uint32_t* abort_flag = a.ctr + 2;
    uint32_t* flagsA = a.ctr + 16;
    uint32_t* flagsB = a.ctr + 16 + P;

    const int row0 = w * 64 * RPL;
    V r[RPL];
    using Raw = typename Src::Raw;
    Raw t0[NC][RPL], t1[NC][RPL], t2[NC][RPL];
    if (!ctl) {
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            const int row = row0 + lane + 64 * q;
            r[q] = row < B ? a.r0[row] : czero<T>();
        }
    }

    // ---- tile waves ---------------------------------------------------------------
    // the wave index is uniform across the wave: keep column arithmetic scalar
    const int wu = __builtin_amdgcn_readfirstlane(wid);
    // Loads are unconditional (a branch around a load would make the wave wait for it
    // at the join): columns past U and rows past B read a clamped in-range element
    // instead.  Such columns are inactive (their M rows and columns and their X rows
    // are zero, so their delta is zero), and rows past B keep r = 0.
    auto load_tile = [&](Raw(&dst)[NC][RPL], int K) {
        const int col0 = K * KP + wu;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int col = min(col0 + LA_NWT * c, U - 1);
#pragma unroll
            for (int q = 0; q < RPL; ++q) {
                const uint32_t row = (uint32_t)min(row0 + lane + 64 * q, B - 1);
                dst[c][q] = a.src.load_raw(col, row, a.ld);
            }
        }
    };
    // partial products of one panel over this workgroup's rows, into psh
    auto tile_col = [&](int K, int c) { return min(K * KP + wu + LA_NWT * c, U - 1); };
    auto partial_to_lds = [&](const Raw(&t)[NC][RPL], int K) {
        constexpr int NH = (NC >= 2) ? NC / 2 : 1;
        constexpr int LOG_NH = (NH == 1) ? 0 : (NH == 2) ? 1 : (NH == 4) ? 2 : (NH == 8) ? 3 : (NH == 16) ? 4 : 5;
        constexpr int HSHIFT = 6 - LOG_NH;
#pragma unroll
        for (int h0 = 0; h0 < NC; h0 += NH) {
            T pr[NH], pi[NH];
#pragma unroll
            for (int c = 0; c < NH; ++c) {
                pr[c] = T(0);
                pi[c] = T(0);
#pragma unroll
                for (int q = 0; q < RPL; ++q) {
                    const V h = a.src.decode(t[h0 + c][q], tile_col(K, h0 + c));
                    pr[c] += h.x * r[q].x + h.y * r[q].y;
                    pi[c] += h.x * r[q].y - h.y * r[q].x;
                }
            }
            wave_transpose_sum<T, NH>(pr, lane);
            wave_transpose_sum<T, NH>(pi, lane);
            if ((lane & ((1 << HSHIFT) - 1)) == 0) psh[wid + LA_NWT * (h0 + (lane >> HSHIFT))] = cmake<T>(pr[0], pi[0]);
        }
    };

    // ---- control wave -------------------------------------------------------------
    auto publish_partials = [&](int slot, uint32_t val) {
#pragma unroll
        for (int i = 0; i < KL; ++i) {
            const int j = lane + 64 * i;
            if (j < KP) st_dev(&a.part[((int64_t)slot * KP + j) * P + w], psh[j]);
        }
        wave_publish(flagsA, w, val);
    };
    // reducer: sum over the P workgroups of column j = w (fixed order per lane, then a
    // fixed butterfly), uniform result
    auto presum = [&](int slot) -> V {
        const V* src = a.part + ((int64_t)slot * KP + w) * P;
        V acc = czero<T>();
        for (int base = 0; base < P; base += 256) {
            V v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = (base + lane + 64 * k < P) ? ld_dev(&src[base + lane + 64 * k]) : czero<T>();
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                acc.x += v[k].x;
                acc.y += v[k].y;
            }
        }
        acc.x = wave_allsum(acc.x);
        acc.y = wave_allsum(acc.y);
        return acc;
    };
    // reducer: publish b_j = g_j - lambda x_j (+ bias) of panel K for its column
    auto publish_b = [&](int K, int slot, V g, uint32_t val) {
        if (lane == 0) {
            const int u = K * KP + w;
            const V xo = (u < U) ? a.x[u] : czero<T>();
            if (a.bias && u < U) {
                const V bb = a.bias[u];
                g.x += bb.x;
                g.y += bb.y;
            }
            V b;
            b.x = g.x - lambda * xo.x;
            b.y = g.y - lambda * xo.y;
            st_dev(&a.gbuf[((int64_t)slot * KP + w) * 2 + 0], b);
            st_dev(&a.gbuf[((int64_t)slot * KP + w) * 2 + 1], xo);
        }
        wave_publish(flagsB, w, val);
    };
    auto stage_M = [&](int K) {
        // global -> LDS without passing through registers: lane l of each load moves
        // bytes [16 l, 16 l + 16) of a 1 KiB row
        const char* src = reinterpret_cast<const char*>(a.M + (int64_t)K * NE) + lane * 16;
        char* dst = reinterpret_cast<char*>(Ms);
#pragma unroll 4
        for (int off = 0; off < MS_BYTES; off += 1024)
            __builtin_amdgcn_global_load_lds(src + off, (__attribute__((address_space(3))) void*)(dst + off), 16, 0, 0);
    };

    // The tile waves and the control wave run separate loops that meet at the same
    // sequence of workgroup barriers (six per panel step: A partials ready, B reduced
    // b in LDS, C matvec partials, C' delta ready, D update and decisions, E end of
    // step).  Separate loops keep each wave class's memory-wait bookkeeping apart.
    // tile-wave pieces of a panel step
    auto tile_matvec = [&]() {
        // delta = M_K b; column v of the packed M holds rows v..KP-1 at offset
        // v*KP - v(v-1)/2; NS threads per row j over contiguous slices of v
        constexpr int SV = KP / NS;
        const int j = tid % KP;
        const int sl = tid / KP;
        const int v0 = sl * SV;
        const int v1 = min(v0 + SV - 1, j);
        V d0 = czero<T>(), d1 = czero<T>();
        int off = v0 * KP - (v0 * (v0 - 1)) / 2 + (j - v0);
        int v = v0;
        for (; v + 1 <= v1; v += 2) {
            cfma(d0, Ms[off], bsh[v]);
            off += KP - v - 1;
            cfma(d1, Ms[off], bsh[v + 1]);
            off += KP - v - 2;
        }
        if (v <= v1) cfma(d0, Ms[off], bsh[v]);
        V d;
        d.x = d0.x + d1.x;
        d.y = d0.y + d1.y;
        dpart[sl][j] = d;
    };
    auto tile_dsum = [&]() {
        if (tid < KP) {
            V s = dpart[0][tid];
#pragma unroll
            for (int k = 1; k < NS; ++k) {
                s.x += dpart[k][tid].x;
                s.y += dpart[k][tid].y;
            }
            dsh[tid] = s;
        }
    };
    auto tile_axs = [&](const Raw(&cur)[NC][RPL], int K) {
#pragma unroll
        for (int qq = 0; qq < RPL; ++qq) {
            V acc = czero<T>();
#pragma unroll
            for (int c = 0; c < NC; ++c) cfma(acc, a.src.decode(cur[c][qq], tile_col(K, c)), dsh[wid + LA_NWT * c]);
            axs[wid][qq][lane] = acc;
        }
    };
    auto tile_update = [&]() {
#pragma unroll
        for (int qq = 0; qq < RPL; ++qq) {
            V s = czero<T>();
#pragma unroll
            for (int v = 0; v < LA_NWT; ++v) {
                s.x += axs[v][qq][lane].x;
                s.y += axs[v][qq][lane].y;
            }
            if (row0 + lane + 64 * qq < B) {
                r[qq].x -= s.x;
                r[qq].y -= s.y;
            }
        }
    };

    if (!ctl) {
        // ================================ tile waves ================================
        if (a.T_max >= 1) {
            // issued set by set (no interleaving by the scheduler): the wait before the
            // first step's partial then only has to cover the second set
            load_tile(t0, 0);
            __builtin_amdgcn_sched_barrier(0);
            load_tile(t1, np > 1 ? 1 : 0);
            __builtin_amdgcn_sched_barrier(0);
            load_tile(t2, 2 % np);
            __builtin_amdgcn_sched_barrier(0);
            partial_to_lds(t0, 0);    // panel 0's partials from r0
        }
        __syncthreads();              // prologue A
        __syncthreads();              // prologue end (ctl_s = outcome)
        if (a.T_max < 1 || __builtin_amdgcn_readfirstlane(ctl_s) != 0) return;
        int K = 0;
        // One panel step with cur = panel K and nx = panel K+1 (the third register set
        // holds panel K+2, in flight).  A macro, not a function: the exits jump straight
        // out of the loop, so no control-flow join mixes a path without the step's
        // prefetch into the wait bookkeeping of the next step.
#define CDM_LA_TSTEP(cur, nx)                                                                        \
    {                                                                                                \
        const int K1 = (K + 1 < np) ? K + 1 : 0;                                                    \
        partial_to_lds(nx, K1); /* look-ahead partials of panel K+1, from r before K's update */    \
        __syncthreads();        /* A */                                                             \
        __syncthreads();        /* B */                                                             \
        tile_matvec();                                                                               \
        __syncthreads();        /* C */                                                             \
        tile_dsum();                                                                                 \
        __syncthreads();        /* C' */                                                            \
        tile_axs(cur, K);                                                                            \
        __syncthreads();        /* D */                                                             \
        tile_update();                                                                               \
        K = K1;                                                                                      \
        load_tile(cur, (K + 2) % np); /* cur is free: stream the new panel K+2 into it */           \
        __syncthreads();        /* E (axs and dpart share scratch) */                               \
    }
        // Steps run in groups of three (one per register-set rotation) and the loop has
        // a single exit at the end of a group: once the control wave has decided to stop
        // (converged, T_max, or abandoned), the remaining steps of the group are idle
        // steps (same barriers, nothing published), so every path into a step has
        // issued the same prefetches.
        for (;;) {
            CDM_LA_TSTEP(t0, t1)
            CDM_LA_TSTEP(t1, t2)
            CDM_LA_TSTEP(t2, t0)
            if (__builtin_amdgcn_readfirstlane(ctl_s) != 0) break;
        }
#undef CDM_LA_TSTEP
        return;
    }

    // ================================ control wave ================================
    uint32_t ok = 1;
    int sweeps = 0;
    double S = 0.0, Xn = 0.0, rel_last = 0.0;
    __syncthreads();                  // prologue A
    if (a.T_max >= 1) {
        publish_partials(0, 1u);
        if (reducer) {
            ok = wave_wait_flags(flagsA, P, 1u, abort_flag, a.timeout_ticks);
            if (ok) publish_b(0, 0, presum(0), 1u);   // no correction for the first panel
        }
    }
    if (lane == 0) ctl_s = ok ? 0 : 2;
    __syncthreads();                  // prologue end
    if (a.T_max >= 1 && ok) {
        int K = 0, t = 1;
        uint32_t q = 0;
        int state = 0;                // 0 running, 1 stopped, 2 abandoned (sticky)
        for (;;) {
            for (int g = 0; g < 3; ++g) {
                const bool live = state == 0;
                const int K1 = (K + 1 < np) ? K + 1 : 0;
                V presum_j = czero<T>();
                V xr[KL];
                __syncthreads();      // A
                if (live) {
                    publish_partials((q + 1) & 1, q + 2);
                    stage_M(K);
                    if (reducer) {
#pragma unroll
                        for (int i = 0; i < KL; ++i) {
                            const int v = lane + 64 * i;
                            xr[i] = (v < KP) ? a.X[((int64_t)K1 * KP + w) * KP + v] : czero<T>();
                        }
                        if (ok) ok = wave_wait_flags(flagsA, P, q + 2, abort_flag, a.timeout_ticks);
                        if (ok) presum_j = presum((q + 1) & 1);
                    }
                    if (ok) ok = wave_wait_flags(flagsB, KP, q + 1, abort_flag, a.timeout_ticks);
                    if (ok) {
#pragma unroll
                        for (int i = 0; i < KL; ++i) {
                            const int j = lane + 64 * i;
                            if (j < KP) {
                                bsh[j] = ld_dev(&a.gbuf[((int64_t)(q & 1) * KP + j) * 2 + 0]);
                                xsh[j] = ld_dev(&a.gbuf[((int64_t)(q & 1) * KP + j) * 2 + 1]);
                            }
                        }
                    }
                    wave_drain_vmem();    // includes the LDS-direct loads of M_K
                    if (!ok) state = 2;
                }
                __syncthreads();      // B
                __syncthreads();      // C
                __syncthreads();      // C'
                if (live && ok) {
                    // statistics, x of panel K, and b of panel K+1 (corrected by X_{K+1} delta_K)
                    double s1 = 0.0, s2 = 0.0;
#pragma unroll
                    for (int i = 0; i < KL; ++i) {
                        const int j = lane + 64 * i;
                        if (j < KP) {
                            const V d = dsh[j];
                            V xn;
                            xn.x = xsh[j].x + d.x;
                            xn.y = xsh[j].y + d.y;
                            s1 += cabs2d(d);
                            s2 += cabs2d(xn);
                        }
                    }
                    S += wave_allsum(s1);
                    Xn += wave_allsum(s2);
                    if (reducer) {
                        V c = czero<T>();
#pragma unroll
                        for (int i = 0; i < KL; ++i) {
                            const int v = lane + 64 * i;
                            if (v < KP) cfma(c, xr[i], dsh[v]);
                        }
                        c.x = wave_allsum(c.x);
                        c.y = wave_allsum(c.y);
                        if (lane == 0) {
                            const int u = K * KP + w;
                            if (u < U) {
                                V xn;
                                xn.x = xsh[w].x + dsh[w].x;
                                xn.y = xsh[w].y + dsh[w].y;
                                a.x[u] = xn;
                            }
                        }
                        V gg;
                        gg.x = presum_j.x - c.x;
                        gg.y = presum_j.y - c.y;
                        publish_b(K1, (q + 1) & 1, gg, q + 2);
                    }
                    if (K == np - 1) {
                        sweeps = t;
                        rel_last = (Xn > 0.0) ? sqrt(S / Xn) : (S > 0.0 ? INFINITY : 0.0);
                        if (t >= a.T_max || (a.tol > 0.0 && sqrt(S) <= a.tol * sqrt(Xn))) state = 1;
                        S = 0.0;
                        Xn = 0.0;
                        ++t;
                    }
                }
                if (lane == 0) ctl_s = state;
                __syncthreads();      // D
                K = K1;
                ++q;
                __syncthreads();      // E
            }
            if (state != 0) break;
        }
    }
    if (w == 0 && lane == 0) {
        int fl = 0;
        if (a.tol > 0.0 && !(rel_last <= a.tol)) fl |= CDM_INFO_NOT_CONVERGED;
        if (!ok) fl |= CDM_INFO_TIMEOUT;
        cdm_info o;
        o.sweeps = sweeps;
        o.flags = fl;
        o.rel_step = rel_last;
        o.resid = -1.0;
        o.reserved = 0.0;
        a.info[0] = o;
    }
}

template <typename T, int KP, int RPL, class Src>
static hipError_t launch_la_src(const PanelLaunch& L, const Src& src, hipStream_t st) {
    PanelArgs<T, Src> a;
    a.src = src;
    a.ld = L.ld;
    a.bias = (const cv<T>*)L.bias;
    a.done = L.done;
    a.r0 = (const cv<T>*)L.r0;
    a.x = (cv<T>*)L.x;
    a.M = (const cv<T>*)L.M;
    a.X = (const cv<T>*)L.X;
    a.part = (cv<T>*)L.part;
    a.gbuf = (cv<T>*)L.gbuf;
    a.ctr = L.ctr;
    a.info = L.info;
    a.lambda = L.lambda;
    a.tol = L.tol;
    a.timeout_ticks = L.timeout_ticks;
    a.B = L.B;
    a.U = L.U;
    a.npanels = L.npanels;
    a.T_max = L.T_max;
    void* args[] = {&a};
    return hipLaunchCooperativeKernel((const void*)k_cd_panel_la<T, KP, RPL, Src>, dim3(L.P), dim3(LA_NT), args, 0,
                                      st);
}

template <typename T, int KP, int RPL>
static hipError_t launch_la_t(const PanelLaunch& L, hipStream_t st) {
    if (L.src_kind == SRC_BF16) {
        if constexpr (sizeof(T) == 4) return launch_la_src<T, KP, RPL>(L, SrcBF16{L.q_re16, L.q_im16}, st);
        return hipErrorInvalidValue;
    }
    if (L.src_kind == SRC_FP8) {
        if constexpr (sizeof(T) == 4) return launch_la_src<T, KP, RPL>(L, SrcFP8{L.q_re8, L.q_im8, L.q_scale}, st);
        return hipErrorInvalidValue;
    }
    return launch_la_src<T, KP, RPL>(L, SrcC<T>{(const cv<T>*)L.H}, st);
}

template <typename T, int KP, int RPL>
static int la_coresident_t() {
    int dev = 0, ncu = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_cd_panel_la<T, KP, RPL, SrcC<T>>, LA_NT, 0) !=
        hipSuccess)
        return 0;
    return per * ncu;
}

// Look-ahead configurations: complex128 with 64-column panels, complex64 (and the
// FP32 inner solve of the mixed path) with 128-column panels; one 64-row block per
// workgroup.
hipError_t launch_panel_la(const PanelLaunch& L, hipStream_t st) {
    if (L.rpl != 1) return hipErrorInvalidValue;
    if (L.c128 && L.kp == 64) return launch_la_t<double, 64, 1>(L, st);
    if (!L.c128 && L.kp == 128) return launch_la_t<float, 128, 1>(L, st);
    return hipErrorInvalidValue;
}

int panel_la_max_coresident(bool c128, int kp) {
    if (c128 && kp == 64) return la_coresident_t<double, 64, 1>();
    if (!c128 && kp == 128) return la_coresident_t<float, 128, 1>();
    return 0;
}

}  // namespace cdm
