// k_panel_la.hip -- look-ahead schedule of the panel engine.
//
// Same block form of the cyclic sweep as k_cd_panel (delta_K = M_K b_K with
// M_K = (D + L)^-1 of the panel Gram, b_K = H_K^H r - lambda x_K), but the partial
// products of a panel are formed from the residual *before* the previous panel's
// update and corrected afterwards:
//     H_{K+1}^H (r - H_K delta_K) = H_{K+1}^H r - X_{K+1} delta_K,
//     X_{K+1} = H_{K+1}^H H_K  (formed once per solve, next to M).
// The exchange of panel K+1's partials thereby overlaps the wait for panel K's
// reduced b.  In exact arithmetic every delta equals the sequential sweep's.
// Where X_K fits the LDS next to M (64-column panels) the reducers publish
// q_K = H_K^H r - lambda x_K as soon as the partials are in, and every workgroup forms
// delta_K = M_K (q_K - X_K delta_{K-1}) = M_K q_K - Y_K delta_{K-1} itself, in one
// product, from -Y_K = -M_K X_K (formed once per solve in place of X_K) staged in LDS:
// the chain from one panel's delta to the next panel's then stays inside the
// workgroup, and the cross-workgroup exchange runs a panel ahead of it.  Otherwise
// (X_K would not fit: 128-column FP32 panels) the reducers apply the correction and
// publish b_K.
//
// Workgroup: 8 tile waves, one control wave and (local b) one X-staging wave,
// decoupled.
//  * Tile waves own the rows (lane = row) and NC panel columns each.  They keep
//    three panels in registers (K for the update, K+1 already reduced, K+2 for the
//    next look-ahead partials) and stream a fourth behind them; they touch global
//    memory only to stream H.  Per step: wait for b_K in LDS, delta_K = M_K b_K,
//    r -= H_K delta_K, prefetch panel K+3, partials of panel K+2 from the new r.
//    FP32 panels: each wave forms the delta of its own columns, summed across its
//    lanes; complex128: each wave forms a slice of every column's delta, the slices
//    summed through LDS.
//  * The control wave does every cross-workgroup exchange: it publishes the tile
//    waves' partials, gathers b_K into LDS (with M_K, staged by LDS-direct loads),
//    keeps the stop statistics, and in the reducer workgroups (w < KP; reducer w
//    owns panel column j = w) sums the P partials of its column and publishes b.
//    complex128: b_K and M_K at the top of step K, after the previous partials are
//    out; FP32 panels: during the step before, in one attempt once half of the tile
//    waves have their partials (the tile waves then go on without waiting for the
//    control wave to publish them).
//  * The X-staging wave moves -Y_K of the next step into LDS with LDS-direct loads
//    as soon as the tile waves have read the current one.  A wave that issues such
//    loads waits for them to land before its next LDS access, so they are kept out
//    of the control wave's loop.
//  * The waves meet only through LDS words (sequence counters), never at a
//    workgroup barrier, so a reducer's wait for partials does not hold back its own
//    tile waves.  The tile waves synchronise among themselves with an LDS arrival
//    counter.  Memory operations complete in issue order per wave, so keeping flag
//    polls out of the tile waves also keeps the tile stream off the critical path.
#include "la_common.hpp"

namespace cdm {

template <typename T, int KP, int RPL, class Src>
__global__ __launch_bounds__((la_threads<T, KP>()), 1) void k_cd_panel_la(PanelArgs<T, Src> a) {
    using V = cv<T>;
    constexpr int NC = KP / LA_NWT;             // panel columns per tile wave
    static_assert(NC >= 1 && NC <= 64 && (NC & (NC - 1)) == 0, "bad panel split");
    constexpr int NE = KP * (KP + 1) / 2;       // packed lower triangle of M_K
    constexpr int KL = (KP + 63) / 64;          // panel entries per control lane
    constexpr bool LOCALB = la_localb<T, KP>();   // X_K in LDS, b formed locally
    // FP32 panels: each tile wave forms the delta of its own (contiguous) columns and sums
    // the slices across its lanes; complex128: the tile waves form slices of every
    // column's delta, summed across waves through LDS (interleaved columns).  Each is the
    // faster of the two for its panels.
    constexpr bool OWN_DELTA = sizeof(T) == 4;
    constexpr int NS = 64 * LA_NWT / KP;        // matvec slices per row (tile threads)

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    const bool ctl = wid == LA_NWT;
    const bool xstg = LOCALB && wid == LA_NWT + 1;
    const int w = blockIdx.x;
    const int P = gridDim.x;                    // the planner keeps KP <= P <= 256
    const bool reducer = w < KP;
    const int B = a.B, U = a.U, np = a.npanels;
    const T lambda = (T)a.lambda;
    if (a.done && *a.done) return;              // uniform for the whole grid

    // packed M_K (two buffers, by step parity), staged by the control wave with
    // LDS-direct loads in 1 KiB rows (padded to whole rows; M's buffer extends past
    // its last panel)
    constexpr int MS_BYTES = (NE * (int)sizeof(V) + 1023) / 1024 * 1024;
    constexpr int MS_N = MS_BYTES / (int)sizeof(V);
    __shared__ __attribute__((aligned(16))) V Ms[2][MS_N];
    __shared__ V psh[2][KP];                    // look-ahead partials, by panel-sequence parity
    __shared__ V bsh[2][KP];                    // b of the step's panel, by step parity
    __shared__ V xsh[2][KP];                    // x of the step's panel before its update
    __shared__ V dsh[2][KP];                    // delta of the step's panel
    __shared__ V dpart[OWN_DELTA ? 1 : NS][KP];
    // -Y_K = -M_K X_K (column v at v * KP) for the local correction
    __shared__ __attribute__((aligned(16))) V Xs[LOCALB ? KP * KP : 1];
    __shared__ V axs[LA_NWT][RPL][64];
    // LDS words: b_ready = (last step whose b, x and M are in LDS) + 1; d_cnt = tile-wave
    // delta count (LA_NWT per step once the step's delta is in dsh: OWN_DELTA, each wave
    // adds one once it has read Xs and written its part, and no wave adds for step q + 1
    // before every wave has added for step q, since the waves meet at the step's barrier
    // in between; so d_cnt >= LA_NWT (q + 1) means step q's delta is complete); x_cnt:
    // the same count for the tile waves' reads of Xs (OWN_DELTA: d_cnt serves); p_done[k]
    // = partial panels written by tile wave k (per wave: the partials have no barrier
    // between steps, so a shared count could not tell a fast wave's second panel from a
    // slow wave's first); stop_w: 1 stopped (converged or T_max), 2 abandoned; t_bar:
    // tile-wave arrival counter; xs_ready = (last step whose -Y_K is in Xs) + 1.  One
    // array, so that every access is a fixed offset from one address.
    __shared__ int lw[8 + LA_NWT];
    int &b_ready = lw[0], &d_cnt = lw[1], &stop_w = lw[2], &t_bar = lw[3], &xs_ready = lw[4], &x_cnt = lw[5];
    int& x_read = OWN_DELTA ? d_cnt : x_cnt;
    int* p_done = lw + 8;
    if (tid < 8 + LA_NWT) lw[tid] = (tid == 4) ? 1 : 0;   // step 0 needs no X
    __syncthreads();   // the only workgroup barrier

    uint32_t* abort_flag = a.ctr + 2;
    const int row0 = w * 64 * RPL;
    const uint64_t tmo = a.timeout_ticks;

    if (xstg) {
        // ================================== X staging wave ==================================
        // -Y_K of step j into LDS once every tile wave has read that of step j - 1; its
        // own wave, so that waiting for these LDS-direct loads to land holds up no other
        // work
        if (!LOCALB || a.T_max < 1) return;
        for (int j = 1;; ++j) {
            const uint64_t t0 = wall_clock64();
            bool go = true;
            const int need = (j == 1) ? 0 : LA_NWT * j;   // step 0 reads no X
            while (__builtin_amdgcn_readfirstlane(lds_get(&x_read)) < need) {
                if (__builtin_amdgcn_readfirstlane(lds_get(&stop_w)) != 0 || wall_clock64() - t0 > 2 * tmo) {
                    go = false;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            if (!go) break;
            const char* src = reinterpret_cast<const char*>(a.X + (int64_t)(j % np) * KP * KP) + lane * 16;
            char* dst = reinterpret_cast<char*>(Xs);
#pragma unroll 4
            for (int off = 0; off < KP * KP * (int)sizeof(V); off += 1024)
                __builtin_amdgcn_global_load_lds(src + off, (__attribute__((address_space(3))) void*)(dst + off), 16, 0,
                                                 0);
            wave_drain_vmem();
            if (lane == 0) lds_set(&xs_ready, j + 1);
        }
        wave_drain_vmem();
        return;
    }

    if (!ctl) {
        // ===================================== tile waves =====================================
        if (a.T_max < 1) return;
        using Raw = typename Src::Raw;
        V r[RPL];
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            const int row = row0 + lane + 64 * q;
            r[q] = row < B ? a.r0[row] : czero<T>();
        }
        // the wave index is uniform across the wave: keep column arithmetic scalar
        const int wu = __builtin_amdgcn_readfirstlane(wid);
        // Loads are unconditional (a branch around a load would make the wave wait for
        // it at the join): columns past U and rows past B read a clamped in-range
        // element.  Such columns are inactive (their M rows and columns and their X rows
        // are zero, so their delta is zero), and rows past B keep r = 0.
        // panel column of this wave's c-th column
        auto pcol = [&](int c) { return OWN_DELTA ? wu * NC + c : wu + LA_NWT * c; };
        auto load_tile = [&](Raw(&dst)[NC][RPL], int K) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int col = min(K * KP + pcol(c), U - 1);
#pragma unroll
                for (int q = 0; q < RPL; ++q) {
                    const uint32_t row = (uint32_t)min(row0 + lane + 64 * q, B - 1);
                    dst[c][q] = a.src.load_raw(col, row, a.ld);
                }
            }
        };
        auto tile_col = [&](int K, int c) { return min(K * KP + pcol(c), U - 1); };
        // partial products of one panel over this workgroup's rows, into psh[s & 1]
        auto partial = [&](const Raw(&t)[NC][RPL], int K, int s) {
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
                if constexpr (NH == 4) {   // the row reduction by DPP fits exactly
                    transpose_sum4_rows<T>(pr, lane);
                    __builtin_amdgcn_sched_barrier(0);
                    transpose_sum4_rows<T>(pi, lane);
                } else {
                    wave_transpose_sum<T, NH>(pr, lane);
                    wave_transpose_sum<T, NH>(pi, lane);
                }
                if ((lane & ((1 << HSHIFT) - 1)) == 0)
                    psh[s & 1][pcol(h0 + (lane >> HSHIFT))] = cmake<T>(pr[0], pi[0]);
            }
            if (lane == 0) lds_set(&p_done[wu], s + 1);
        };
        // waits of the tile waves read LDS and the wall clock only (each bounded by the
        // same time-out as the cross-workgroup waits); `bad` ends the loop
        bool bad = false;
        int nbar = 0;
        auto tbar = [&]() {   // the 8 tile waves
            nbar += LA_NWT;
            if (lane == 0) lds_add(&t_bar, 1);
            const uint64_t t0 = wall_clock64();
            while (__builtin_amdgcn_readfirstlane(lds_get(&t_bar)) < nbar) {
                if (__builtin_amdgcn_readfirstlane(lds_get(&stop_w)) == 2 || wall_clock64() - t0 > tmo) {
                    bad = true;
                    return;
                }
            }
        };
        // wait until b of step q is in LDS; false: stop (converged, T_max or abandoned)
        auto wait_b = [&](int q) -> bool {
            const uint64_t t0 = wall_clock64();
            for (;;) {
                if (__builtin_amdgcn_readfirstlane(lds_get(&b_ready)) > q &&
                    (!LOCALB || __builtin_amdgcn_readfirstlane(lds_get(&xs_ready)) > q))
                    return true;
                if (__builtin_amdgcn_readfirstlane(lds_get(&stop_w)) != 0) return false;
                if (wall_clock64() - t0 > 2 * tmo) return false;
                __builtin_amdgcn_s_sleep(1);
            }
        };

        Raw t0[NC][RPL], t1[NC][RPL], t2[NC][RPL];
        // prologue: panels 0, 1, 2 in flight, set by set; partials of panels 0 and 1 from r0
        load_tile(t0, 0);
        __builtin_amdgcn_sched_barrier(0);
        load_tile(t1, np > 1 ? 1 : 0);
        __builtin_amdgcn_sched_barrier(0);
        load_tile(t2, 2 % np);
        __builtin_amdgcn_sched_barrier(0);
        partial(t0, 0, 0);
        partial(t1, np > 1 ? 1 : 0, 1);

        int K = 0;
        int q = 0;
        // One step: cur = panel K, nn = panel K+2 (its partials come at the end of this
        // step; the third set holds panel K+1).  A macro: its exits leave the loop directly.
#define CDM_LA_TSTEP(cur, nn)                                                                         \
    {                                                                                                 \
        if (!wait_b(q)) goto tdone;                                                                   \
        if constexpr (OWN_DELTA) {                                                                    \
            /* delta of this wave's columns j = wu NC + c; column v of the packed M holds rows        \
               v..KP-1 at offset v KP - v(v-1)/2.  LOCALB: b = q_K - X_K delta_{K-1}, so              \
               delta = M_K q_K + (-Y_K) delta_{K-1}, Y_K = M_K X_K (-Y_K in Xs); the first panel of  \
               the solve has no correction.  Lane (c, s) sums slice s of the terms; the slices are   \
               then summed across lanes, so no other wave takes part */                              \
            constexpr int NSL = 64 / NC, SV = KP / NSL;                                               \
            const V* Mq = Ms[q & 1];                                                                  \
            const V* bq = bsh[q & 1];                                                                 \
            int ln = lane;                                                                            \
            asm volatile("" : "+v"(ln)); /* lane-derived indices are formed here, not held */       \
            const int c_ = ln & (NC - 1), j = wu * NC + c_, v0 = (ln / NC) * SV;                      \
            const int v1 = min(v0 + SV - 1, j);                                                       \
            V d0 = czero<T>(), d1 = czero<T>();                                                       \
            if constexpr (LOCALB) {                                                                   \
                if (q > 0) { /* Xs holds -Y_K */                                                      \
                    __builtin_amdgcn_sched_barrier(0);                                                \
                    const V* dp = dsh[(q - 1) & 1];                                                   \
                    for (int u = v0; u < v0 + SV; u += 2) {                                           \
                        cfma(d0, Xs[u * KP + j], dp[u]);                                              \
                        cfma(d1, Xs[(u + 1) * KP + j], dp[u + 1]);                                    \
                    }                                                                                 \
                }                                                                                     \
            }                                                                                         \
            int off = v0 * KP - (v0 * (v0 - 1)) / 2 + (j - v0);                                       \
            int v = v0;                                                                               \
            for (; v + 1 <= v1; v += 2) {                                                             \
                cfma(d0, Mq[off], bq[v]);                                                             \
                off += KP - v - 1;                                                                    \
                cfma(d1, Mq[off], bq[v + 1]);                                                         \
                off += KP - v - 2;                                                                    \
            }                                                                                         \
            if (v <= v1) cfma(d0, Mq[off], bq[v]);                                                    \
            V dj = cmake<T>(group_sum<NC>(d0.x + d1.x), group_sum<NC>(d0.y + d1.y));                  \
            if (ln < NC) dsh[q & 1][j] = dj; /* for the next step and the control wave */             \
            if (ln == 0) lds_add(&d_cnt, 1); /* Xs read, delta written */                            \
            for (int qq = 0; qq < RPL; ++qq) {                                                        \
                V acc = czero<T>();                                                                   \
                for (int c = 0; c < NC; ++c)                                                          \
                    cfma(acc, a.src.decode(cur[c][qq], tile_col(K, c)),                               \
                         cmake<T>(lane_value(dj.x, c), lane_value(dj.y, c)));                         \
                axs[wu][qq][lane] = acc;                                                              \
            }                                                                                         \
        } else {                                                                                      \
            {   /* slice sl = wave of every column's delta (same sums as above, other split) */       \
                constexpr int SV = KP / NS;                                                           \
                const V* Mq = Ms[q & 1];                                                              \
                const V* bq = bsh[q & 1];                                                             \
                const int j = tid % KP, sl = tid / KP, v0 = sl * SV, v1 = min(v0 + SV - 1, j);        \
                V d0 = czero<T>(), d1 = czero<T>();                                                   \
                if constexpr (LOCALB) {                                                               \
                    if (q > 0) {                                                                      \
                        __builtin_amdgcn_sched_barrier(0);                                            \
                        const V* dp = dsh[(q - 1) & 1];                                               \
                        for (int u = v0; u < v0 + SV; u += 2) {                                       \
                            cfma(d0, Xs[u * KP + j], dp[u]);                                          \
                            cfma(d1, Xs[(u + 1) * KP + j], dp[u + 1]);                                \
                        }                                                                             \
                    }                                                                                 \
                }                                                                                     \
                int off = v0 * KP - (v0 * (v0 - 1)) / 2 + (j - v0);                                   \
                int v = v0;                                                                           \
                for (; v + 1 <= v1; v += 2) {                                                         \
                    cfma(d0, Mq[off], bq[v]);                                                         \
                    off += KP - v - 1;                                                                \
                    cfma(d1, Mq[off], bq[v + 1]);                                                     \
                    off += KP - v - 2;                                                                \
                }                                                                                     \
                if (v <= v1) cfma(d0, Mq[off], bq[v]);                                                \
                dpart[sl][j] = cmake<T>(d0.x + d1.x, d0.y + d1.y);                                    \
            }                                                                                         \
            tbar();                                                                                   \
            if (bad) goto tdone;                                                                      \
            if (tid == 0) lds_add(&x_cnt, LA_NWT); /* every wave is done reading Xs */                \
            if (tid < KP) {                                                                           \
                V s_ = dpart[0][tid];                                                                 \
                for (int k = 1; k < NS; ++k) {                                                        \
                    s_.x += dpart[k][tid].x;                                                          \
                    s_.y += dpart[k][tid].y;                                                          \
                }                                                                                     \
                dsh[q & 1][tid] = s_;                                                                 \
            }                                                                                         \
            tbar();                                                                                   \
            if (bad) goto tdone;                                                                      \
            if (tid == 0) lds_add(&d_cnt, LA_NWT);                                                    \
            for (int qq = 0; qq < RPL; ++qq) {                                                        \
                V acc = czero<T>();                                                                   \
                for (int c = 0; c < NC; ++c)                                                          \
                    cfma(acc, a.src.decode(cur[c][qq], tile_col(K, c)), dsh[q & 1][pcol(c)]);         \
                axs[wu][qq][lane] = acc;                                                              \
            }                                                                                         \
        }                                                                                             \
        tbar(); /* every wave's delta and residual contributions are in LDS */                        \
        if (bad) goto tdone;                                                                          \
        for (int qq = 0; qq < RPL; ++qq) {                                                            \
            V s_ = czero<T>();                                                                        \
            for (int v = 0; v < LA_NWT; ++v) {                                                        \
                s_.x += axs[v][qq][lane].x;                                                           \
                s_.y += axs[v][qq][lane].y;                                                           \
            }                                                                                         \
            if (row0 + lane + 64 * qq < B) {                                                          \
                r[qq].x -= s_.x;                                                                      \
                r[qq].y -= s_.y;                                                                      \
            }                                                                                         \
        }                                                                                             \
        load_tile(cur, (K + 3) % np); /* cur is free: stream panel K+3 into it */                    \
        partial(nn, (K + 2) % np, q + 2); /* look-ahead partials of panel K+2 from r after K */      \
        K = (K + 1 < np) ? K + 1 : 0;                                                                 \
        ++q;                                                                                          \
    }
        for (;;) {
            CDM_LA_TSTEP(t0, t2)
            CDM_LA_TSTEP(t1, t0)
            CDM_LA_TSTEP(t2, t1)
        }
#undef CDM_LA_TSTEP
    tdone:
        return;
    }

    // ==================================== control wave ====================================
    uint32_t ok = 1;
    int sweeps = 0;
    double S = 0.0, Xn = 0.0, rel_last = 0.0;
    // wait until every tile wave has written its columns of the first `n` partial panels
    auto wait_parts = [&](int n) -> bool {
        const uint64_t t0 = wall_clock64();
        for (;;) {
            const int v = lds_get(&p_done[lane & (LA_NWT - 1)]);
            if (__all(v >= n)) return true;
            if (wall_clock64() - t0 > tmo) return false;
            __builtin_amdgcn_s_sleep(1);
        }
    };
    auto wait_delta = [&](int q) -> bool {
        const uint64_t t0 = wall_clock64();
        while (__builtin_amdgcn_readfirstlane(lds_get(&d_cnt)) < LA_NWT * (q + 1)) {
            if (wall_clock64() - t0 > tmo) return false;
            __builtin_amdgcn_s_sleep(1);
        }
        return true;
    };
    // exchange buffers of tagged words: part [2][KP][P][NW] (slot, column, workgroup),
    // gbuf [2][KP][2][NW] (slot, column, {b, x})
    using TG = Tagged<T>;
    constexpr int NW = TG::NW;
    uint64_t* part64 = reinterpret_cast<uint64_t*>(a.part);
    uint64_t* gb64 = reinterpret_cast<uint64_t*>(a.gbuf);
    // common poll loop: `more()` re-reads what has not arrived yet and returns true
    // while something is still missing in this lane
    auto poll = [&](auto&& more) -> bool {
        uint64_t t0 = 0;
        bool started = false;
        for (;;) {
            if (!__any(more())) return true;
            if (!started) {
                t0 = wall_clock64();
                started = true;
            }
            if (ld_relaxed(abort_flag)) return false;
            if (wall_clock64() - t0 > tmo) {
                if (lane == 0) st_relaxed(abort_flag, 1u);
                return false;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    };
    // publish the partials of panel sequence s (psh[s & 1]); fire and forget
    auto publish_partials = [&](int s) {
#pragma unroll
        for (int i = 0; i < KL; ++i) {
            const int j = lane + 64 * i;
            if (j < KP) TG::put(part64 + (((int64_t)(s & 1) * KP + j) * P + w) * NW, psh[s & 1][j], (uint32_t)s + 1);
        }
    };
    // reducer: wait for the P partials of column j = w of sequence s and sum them (fixed
    // order per lane, then a fixed butterfly); uniform result
    auto gather_partials = [&](int s, V& out) -> bool {
        const uint64_t* src = part64 + ((int64_t)(s & 1) * KP + w) * P * NW;
        const uint32_t tag = (uint32_t)s + 1;
        V v[4];
        bool have[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = czero<T>();
            have[k] = lane + 64 * k >= P;   // lanes past P contribute zero
        }
        auto more = [&]() {
            // every attempt reloads all four (unconditional loads issue back to back)
            V nv[4];
            bool ok4[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) ok4[k] = TG::get(src + (int64_t)min(lane + 64 * k, P - 1) * NW, tag, nv[k]);
            bool miss = false;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (!have[k] && ok4[k]) {
                    v[k] = nv[k];
                    have[k] = true;
                }
                miss |= !have[k];
            }
            return miss;
        };
        if (!poll(more)) return false;
        V acc = czero<T>();
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            acc.x += v[k].x;
            acc.y += v[k].y;
        }
        acc.x = wave_allsum(acc.x);
        acc.y = wave_allsum(acc.y);
        out = acc;
        return true;
    };
    // everyone: b and x of sequence q (a step's panel) into LDS.  gb_more makes one
    // attempt (one memory round trip), keeps what has arrived and tells whether this
    // lane still misses something; gb_store puts the values in LDS.
    V gbv[KL], gxv[KL];
    bool ghb[KL], ghx[KL];
    auto gb_reset = [&]() {
#pragma unroll
        for (int i = 0; i < KL; ++i) ghb[i] = ghx[i] = lane + 64 * i >= KP;
    };
    auto gb_more = [&](int q) {
        const uint32_t tag = (uint32_t)q + 1;
        bool miss = false;
#pragma unroll
        for (int i = 0; i < KL; ++i) {
            const uint64_t* q0 = gb64 + (((int64_t)(q & 1) * KP + min(lane + 64 * i, KP - 1)) * 2) * NW;
            V nb, nx;
            const bool okb = TG::get(q0, tag, nb), okx = TG::get(q0 + NW, tag, nx);
            if (!ghb[i] && okb) {
                gbv[i] = nb;
                ghb[i] = true;
            }
            if (!ghx[i] && okx) {
                gxv[i] = nx;
                ghx[i] = true;
            }
            miss |= !(ghb[i] && ghx[i]);
        }
        return miss;
    };
    auto gb_store = [&](int q) {
#pragma unroll
        for (int i = 0; i < KL; ++i) {
            const int j = lane + 64 * i;
            if (j < KP) {
                bsh[q & 1][j] = gbv[i];
                xsh[q & 1][j] = gxv[i];
            }
        }
    };
    auto gather_b = [&](int q) -> bool {
        gb_reset();
        if (!poll([&]() { return gb_more(q); })) return false;
        gb_store(q);
        return true;
    };
    auto load_xb = [&](int K, V& xo, V& bb) {
        const int u = K * KP + w;
        xo = czero<T>();
        bb = czero<T>();
        if (lane == 0 && u < U) {
            xo = a.x[u];
            if (a.bias) bb = a.bias[u];
        }
    };
    auto publish_b = [&](int s, V g, V xo, V bb) {
        if (lane == 0) {
            g.x += bb.x;
            g.y += bb.y;
            V b;
            b.x = g.x - lambda * xo.x;
            b.y = g.y - lambda * xo.y;
            uint64_t* q0 = gb64 + (((int64_t)(s & 1) * KP + w) * 2) * NW;
            TG::put(q0, b, (uint32_t)s + 1);
            TG::put(q0 + NW, xo, (uint32_t)s + 1);
        }
    };
    // the same, loading x_j and bias_j of panel K itself (where they cannot be loaded
    // ahead: the reducer-side correction)
    auto publish_b_at = [&](int K, int s, V g) {
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
            uint64_t* q0 = gb64 + (((int64_t)(s & 1) * KP + w) * 2) * NW;
            TG::put(q0, b, (uint32_t)s + 1);
            TG::put(q0 + NW, xo, (uint32_t)s + 1);
        }
    };
    auto stage_M = [&](int K, int buf) {
        // global -> LDS without passing through registers: lane l of each load moves
        // bytes [16 l, 16 l + 16) of a 1 KiB row
        const char* src = reinterpret_cast<const char*>(a.M + (int64_t)K * NE) + lane * 16;
        char* dst = reinterpret_cast<char*>(Ms[buf]);
#pragma unroll 4
        for (int off = 0; off < MS_BYTES; off += 1024)
            __builtin_amdgcn_global_load_lds(src + off, (__attribute__((address_space(3))) void*)(dst + off), 16, 0, 0);
    };

    // LOCALB: the reducers publish q of the next panel before this step's delta unless the
    // next panel is this one (a single panel), whose x this step still changes
    const bool early = LOCALB && np > 1;
    // Where b of the next step is gathered.  FP32 panels: during this step, once half of
    // the tile waves have their partials, in one attempt (if it comes back complete, the
    // tile waves go on as soon as they finish, and the partials follow); complex128: at
    // the top of the next step, after the partials are out.  Each is the faster of the
    // two for its panels (measured on the 16384 x 8192 instance).
    constexpr bool GATHER_AHEAD = sizeof(T) == 4;

    int state = 0;   // 0 running, 1 stopped (converged or T_max), 2 abandoned
    if (a.T_max >= 1) {
        // prologue: partials of panels 0 and 1 (both from r0); b of panel 0 (no correction)
        ok = wait_parts(1);
        if (ok) publish_partials(0);
        if (ok) ok = wait_parts(2);
        if (ok) publish_partials(1);
        if (ok && reducer) {
            V g0;
            ok = gather_partials(0, g0);
            if (ok) publish_b_at(0, 0, g0);   // no correction for the first panel
        }
        // b, x and M of step 0; GATHER_AHEAD: those of every later step are gathered and
        // staged during the step before it
        if (GATHER_AHEAD && ok) {
            stage_M(0, 0);
            ok = gather_b(0);
            wave_drain_vmem();   // the LDS-direct loads of M_0 have landed
            if (ok && lane == 0) lds_set(&b_ready, 1);
        }
        int K = 0, t = 1;
        for (int q = 0; ok; ++q) {
            const int K1 = (K + 1 < np) ? K + 1 : 0;
            V xo1 = czero<T>(), bb1 = czero<T>();
            if (LOCALB && reducer && np > 1) load_xb(K1, xo1, bb1);
            if (!GATHER_AHEAD) {
                // b, x and M of this step's panel into LDS buffer q & 1 (free: the tile waves
                // finished step q - 2, whose delta this wave has already seen)
                stage_M(K, q & 1);
            }
            V xr[KL];
            if (!LOCALB && reducer) {   // row w of X_{K+1} (stored transposed)
#pragma unroll
                for (int i = 0; i < KL; ++i) {
                    const int v = lane + 64 * i;
                    xr[i] = (v < KP) ? a.X[((int64_t)K1 * KP + v) * KP + w] : czero<T>();
                }
            }
            if (!GATHER_AHEAD) {
                ok = gather_b(q);
                if (!ok) break;
                wave_drain_vmem();   // the LDS-direct loads of M_K have landed
                if (lane == 0) lds_set(&b_ready, q + 1);
            }
            // LOCALB reducer: q of panel K+1 from its look-ahead partials (published one
            // step ago), while this workgroup's tile waves work on panel K
            if (early && reducer) {
                V g;
                ok = gather_partials(q + 1, g);
                if (!ok) break;
                publish_b(q + 1, g, xo1, bb1);
            }
            // statistics and x of panel K once the tile waves have delta
            ok = wait_delta(q);
            if (!ok) break;
            double s1 = 0.0, s2 = 0.0;
#pragma unroll
            for (int i = 0; i < KL; ++i) {
                const int j = lane + 64 * i;
                if (j < KP) {
                    const V d = dsh[q & 1][j];
                    V xn;
                    xn.x = xsh[q & 1][j].x + d.x;
                    xn.y = xsh[q & 1][j].y + d.y;
                    s1 += cabs2d(d);
                    s2 += cabs2d(xn);
                }
            }
            S += wave_allsum(s1);
            Xn += wave_allsum(s2);
            if (reducer && lane == 0) {
                const int u = K * KP + w;
                if (u < U) {
                    V xn;
                    xn.x = xsh[q & 1][w].x + dsh[q & 1][w].x;
                    xn.y = xsh[q & 1][w].y + dsh[q & 1][w].y;
                    a.x[u] = xn;
                }
            }
            if (K == np - 1) {
                sweeps = t;
                rel_last = (Xn > 0.0) ? sqrt(S / Xn) : (S > 0.0 ? INFINITY : 0.0);
                const bool done = t >= a.T_max || (a.tol > 0.0 && sqrt(S) <= a.tol * sqrt(Xn));
                S = 0.0;
                Xn = 0.0;
                ++t;
                if (done) {
                    state = 1;
                    break;
                }
            }
            if (LOCALB && reducer && np == 1) load_xb(K1, xo1, bb1);
            // reducer: b of panel K+1 = (sum of its look-ahead partials) - X_{K+1} delta_K
            // - lambda x (the partials were published one step ago); with LOCALB and a
            // single panel, q of the next sweep's panel once this step's x is written
            if (!LOCALB && reducer) {
                V g;
                ok = gather_partials(q + 1, g);
                if (!ok) break;
                V c = czero<T>();
#pragma unroll
                for (int i = 0; i < KL; ++i) {
                    const int v = lane + 64 * i;
                    if (v < KP) cfma(c, xr[i], dsh[q & 1][v]);
                }
                c.x = wave_allsum(c.x);
                c.y = wave_allsum(c.y);
                publish_b_at(K1, q + 1, cmake<T>(g.x - c.x, g.y - c.y));
            } else if (LOCALB && !early && reducer) {
                V g;
                ok = gather_partials(q + 1, g);
                if (!ok) break;
                publish_b(q + 1, g, xo1, bb1);
            }
            if (!GATHER_AHEAD) {   // the tile waves' partials of panel K+2 (sequence q + 2)
                ok = wait_parts(q + 3);
                if (!ok) break;
                publish_partials(q + 2);
            } else {
                // M, b and x of the next step's panel into LDS buffers (q + 1) & 1 while the
                // tile waves still work on this step (the buffers are free: every tile wave is
                // past this step's delta, and so past the previous step's reads).  If the one
                // attempt at b comes back complete, the tile waves are released before the
                // partials of panel K+2 (sequence q + 2) are published; otherwise b is polled
                // for after.  Publishing the partials before b is in is safe: every reducer
                // has gathered the partials of sequence q, whose slot they take, before it
                // published b of this step.
                stage_M(K1, (q + 1) & 1);
                gb_reset();
                {   // one attempt once the first half of the tile waves have their partials
                    const uint64_t t0 = wall_clock64();
                    while (!__all(lds_get(&p_done[lane & (LA_NWT / 2 - 1)]) >= q + 3) && wall_clock64() - t0 <= tmo)
                        __builtin_amdgcn_s_sleep(1);
                }
                const bool have_b = !__any(gb_more(q + 1));
                if (have_b) {
                    gb_store(q + 1);
                    wave_drain_vmem();   // the LDS-direct loads of M_{K+1} have landed
                    if (lane == 0) lds_set(&b_ready, q + 2);
                }
                ok = wait_parts(q + 3);
                if (!ok) break;
                publish_partials(q + 2);
                if (!have_b) {
                    ok = poll([&]() { return gb_more(q + 1); });
                    if (!ok) break;
                    gb_store(q + 1);
                    wave_drain_vmem();
                    if (lane == 0) lds_set(&b_ready, q + 2);
                }
            }
            K = K1;
        }
    }
    if (!ok) state = 2;
    if (lane == 0) lds_set(&stop_w, state == 0 ? 1 : state);
    if (w == 0 && lane == 0) {
        int fl = 0;
        if (a.tol > 0.0 && !(rel_last <= a.tol)) fl |= CDM_INFO_NOT_CONVERGED;
        if (state == 2) fl |= CDM_INFO_TIMEOUT;
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
    a.X2 = nullptr;
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
    return hipLaunchCooperativeKernel((const void*)k_cd_panel_la<T, KP, RPL, Src>, dim3(L.P), dim3(la_threads<T, KP>()), args, 0,
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
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_cd_panel_la<T, KP, RPL, SrcC<T>>, la_threads<T, KP>(), 0) !=
        hipSuccess)
        return 0;
    return per * ncu;
}

// Look-ahead configurations, one 64-row block per workgroup: complex128 and complex64
// with 64-column panels (b formed locally), the FP32 inner solve of the mixed path with
// 128-column panels (correction at the reducers).
hipError_t launch_panel_la(const PanelLaunch& L, hipStream_t st) {
    if (L.rpl != 1) return hipErrorInvalidValue;
    if (L.c128 && L.kp == 64) return launch_la_t<double, 64, 1>(L, st);
    if (!L.c128 && L.kp == 128) return launch_la_t<float, 128, 1>(L, st);
    if (!L.c128 && L.kp == 64) return launch_la_t<float, 64, 1>(L, st);
    return hipErrorInvalidValue;
}

int panel_la_max_coresident(bool c128, int kp) {
    if (c128 && kp == 64) return la_coresident_t<double, 64, 1>();
    if (!c128 && kp == 128) return la_coresident_t<float, 128, 1>();
    if (!c128 && kp == 64) return la_coresident_t<float, 64, 1>();
    return 0;
}

}  // namespace cdm
