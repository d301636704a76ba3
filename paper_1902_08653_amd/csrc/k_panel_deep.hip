// k_panel_deep.hip -- the panel engine with a look-ahead of two panels (complex128,
// 64-column panels, at least three panels).
//
// The block form of the cyclic sweep is the same as in k_panel_la.hip: delta_K =
// M_K b_K, M_K = (D + L)^-1 of the panel Gram, b_K = H_K^H r - lambda x_K, with r the
// residual after panel K-1.  There, the partial products of panel K+2 are formed from
// the residual after panel K, so the two cross-workgroup hops of their exchange
// (partials to the reducers, q back to every workgroup) must fit into one panel step.
// Here the partials of panel K+3 are formed from the residual after panel K:
//     b_{K+3} = H_{K+3}^H r_{K+2} - lambda x_{K+3}
//             = p_{K+3} - X2_{K+3} delta_{K+1} - X_{K+3} delta_{K+2} - lambda x_{K+3},
//     p_{K+3} = H_{K+3}^H r_K,  X_K = H_K^H H_{K-1},  X2_K = H_K^H H_{K-2},
// so the exchange has two panel steps to arrive.  Reducer j (one workgroup per panel
// column) sums the partials of its column and subtracts row j of X2_{K+3} times
// delta_{K+1}, which its own tile waves have formed by then, and publishes
//     q_{K+3} = p_{K+3} - X2_{K+3} delta_{K+1} - lambda x_{K+3};
// every workgroup forms delta_{K+3} = M_{K+3} q_{K+3} + (-Y_{K+3}) delta_{K+2} itself
// (-Y = -M X in LDS), as in the one-panel schedule.  In exact arithmetic every delta
// equals the sequential sweep's.
//
// Opt-in (CDM_F_DEEP_LOOKAHEAD): each tile is read twice per sweep here (for its
// partials, and three steps later for its update), and the exchange's loads return
// behind that doubled stream, so on the devices measured the one-panel schedule is the
// faster one.
//
// Workgroup: 8 tile waves, one control wave, one X-staging wave (640 threads, one per
// CU, 64 rows each).
//  * Tile waves own the rows (lane = row) and 8 panel columns each.  They hold two
//    tiles: U (panel K, for the residual update) and Pb (panel K+3, for the partials).
//    After the update U is refilled with panel K+1 and after the partials Pb with panel
//    K+4, so a tile is read twice per sweep: for its partials, and three steps later
//    for its update, when it is still in the device's last-level cache.
//  * The control wave publishes the tile waves' partials, gathers b and x of step q + 1
//    (with M, staged by LDS-direct loads) while the tile waves work on step q, keeps the
//    stop statistics, and in the reducer workgroups forms and publishes q.
//  * The X-staging wave moves -Y_K into LDS once the tile waves have read the previous
//    one.
//  * The waves meet only through LDS sequence words.
#include "la_common.hpp"

namespace cdm {

constexpr int DP_KP = 64;
constexpr int DP_THREADS = 64 * (LA_NWT + 2);

template <typename T, class Src>
__global__ __launch_bounds__(DP_THREADS, 1) void k_cd_panel_deep(PanelArgs<T, Src> a) {
    using V = cv<T>;
    constexpr int KP = DP_KP;
    constexpr int NC = KP / LA_NWT;             // panel columns per tile wave
    constexpr int NE = KP * (KP + 1) / 2;       // packed lower triangle of M_K
    constexpr int NS = 64 * LA_NWT / KP;        // matvec slices per row (tile threads)
    static_assert(KP == 64, "one panel column per control lane");

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    const bool ctl = wid == LA_NWT;
    const bool xstg = wid == LA_NWT + 1;
    const int w = blockIdx.x;
    const int P = gridDim.x;                    // the planner keeps KP <= P <= 256
    const bool reducer = w < KP;
    const int B = a.B, U = a.U, np = a.npanels; // np >= 3
    const T lambda = (T)a.lambda;
    if (a.done && *a.done) return;              // uniform for the whole grid

    constexpr int MS_BYTES = (NE * (int)sizeof(V) + 1023) / 1024 * 1024;
    constexpr int MS_N = MS_BYTES / (int)sizeof(V);
    __shared__ __attribute__((aligned(16))) V Ms[2][MS_N];   // M of the step's panel, by step parity
    __shared__ __attribute__((aligned(16))) V Xs[KP * KP];   // -Y_K, column v at v * KP
    __shared__ V psh[4][KP];                    // partials, by panel sequence mod 4
    __shared__ V bsh[2][KP];                    // q of the step's panel, by step parity
    __shared__ V xsh[2][KP];                    // x of the step's panel before its update
    __shared__ V dsh[2][KP];                    // delta of the step's panel
    __shared__ V dpart[NS][KP];
    __shared__ V axs[LA_NWT][64];
    // b_ready = (last step whose q, x and M are in LDS) + 1; d_ready = (last step whose
    // delta is in dsh) + 1; p_done[k] = partial panels written by tile wave k; stop_w: 1
    // stopped, 2 abandoned; t_bar: tile-wave arrivals; xs_ready = (last step whose -Y is
    // in Xs) + 1; x_free = (last step whose product has read Xs) + 1
    __shared__ int b_ready, d_ready, stop_w, t_bar, xs_ready, x_free;
    __shared__ int p_done[LA_NWT];
    if (tid == 0) {
        b_ready = 0;
        d_ready = 0;
        stop_w = 0;
        t_bar = 0;
        xs_ready = 1;   // step 0 needs no -Y
        x_free = 1;     // nor reads it
    }
    if (tid < LA_NWT) p_done[tid] = 0;
    __syncthreads();   // the only workgroup barrier

    uint32_t* abort_flag = a.ctr + 2;
    const int row0 = w * 64;
    const uint64_t tmo = a.timeout_ticks;
    using TG = Tagged<T>;
    constexpr int NW = TG::NW;
    // exchange slots by sequence mod 4 (DP_SLOTS): partials [4][KP][P][NW], {q, x} [4][KP][2][NW]
    uint64_t* part64 = reinterpret_cast<uint64_t*>(a.part);
    uint64_t* gb64 = reinterpret_cast<uint64_t*>(a.gbuf);
    // publish the partials of sequence s (psh[s & 3]); fire and forget.  A slot is
    // rewritten with sequence s + 4 only after every reducer has read sequence s: the
    // X-staging wave publishes s + 4 once the tile waves are past the product of step
    // s + 1, which needs q_{s+1}, which every reducer publishes after it has gathered the
    // partials of s + 1, and so of s.  (Two slots would not do: the prologue publishes
    // sequences 0, 1 and 2 before any q is known.)  Likewise q_{s+4} follows q_s into
    // its slot only once every workgroup has gathered q_s (in step s - 1): a reducer
    // forms q_{s+4} from the partials of s + 4, published after the product of step
    // s + 1.  psh[s & 3] is rewritten by the partials of step s + 1 only once the tile
    // waves have entered that step, which needs -Y of it, which the X-staging wave
    // stages after it has published s.
    auto publish_partials = [&](int s) {
        TG::put(part64 + (((int64_t)(s & (DP_SLOTS - 1)) * KP + lane) * P + w) * NW, psh[s & 3][lane],
                (uint32_t)s + 1);
    };

    if (xstg) {
        // ================================== X staging wave ==================================
        // Iteration j: -Y of step j into Xs once the tile waves have read the previous one
        // (in step j - 1), then the partials of sequence j + 2 (formed at the end of step
        // j - 1) out to the reducers as soon as all tile waves have written them.
        if (a.T_max < 1) return;
        auto wait_lds = [&](auto&& ready) -> bool {
            const uint64_t t0 = wall_clock64();
            while (!ready()) {
                if (__builtin_amdgcn_readfirstlane(lds_get(&stop_w)) != 0 || wall_clock64() - t0 > 2 * tmo)
                    return false;
                __builtin_amdgcn_s_sleep(1);
            }
            return true;
        };
        for (int j = 1;; ++j) {
            if (!wait_lds([&]() { return __builtin_amdgcn_readfirstlane(lds_get(&x_free)) >= j; })) break;
            const char* src = reinterpret_cast<const char*>(a.X + (int64_t)(j % np) * KP * KP) + lane * 16;
            char* dst = reinterpret_cast<char*>(Xs);
#pragma unroll 4
            for (int off = 0; off < KP * KP * (int)sizeof(V); off += 1024)
                __builtin_amdgcn_global_load_lds(src + off, (__attribute__((address_space(3))) void*)(dst + off), 16, 0,
                                                 0);
            wave_drain_vmem();
            if (lane == 0) lds_set(&xs_ready, j + 1);
            if (!wait_lds([&]() { return (bool)__all(lds_get(&p_done[lane & (LA_NWT - 1)]) >= j + 3); })) break;
            publish_partials(j + 2);
        }
        wave_drain_vmem();
        return;
    }

    if (!ctl) {
        // ===================================== tile waves =====================================
        if (a.T_max < 1) return;
        using Raw = typename Src::Raw;
        const int row = row0 + lane;
        V r = row < B ? a.r0[row] : czero<T>();
        const int wu = __builtin_amdgcn_readfirstlane(wid);
        // unconditional loads of clamped in-range elements (columns past U are inactive:
        // their M rows and columns and their cross-block rows are zero; rows past B keep
        // r = 0)
        auto load_tile = [&](Raw(&dst)[NC], int K) {
            const int col0 = K * KP + wu;
            const uint32_t rr = (uint32_t)min(row, B - 1);
#pragma unroll
            for (int c = 0; c < NC; ++c) dst[c] = a.src.load_raw(min(col0 + LA_NWT * c, U - 1), rr, a.ld);
        };
        auto tile_col = [&](int K, int c) { return min(K * KP + wu + LA_NWT * c, U - 1); };
        // partial products of one panel over this workgroup's rows into psh[s & 3]
        auto partial = [&](const Raw(&t)[NC], int K, int s) {
            constexpr int NH = NC / 2;            // 4
#pragma unroll
            for (int h0 = 0; h0 < NC; h0 += NH) {
                T pr[NH], pi[NH];
#pragma unroll
                for (int c = 0; c < NH; ++c) {
                    const V h = a.src.decode(t[h0 + c], tile_col(K, h0 + c));
                    pr[c] = h.x * r.x + h.y * r.y;
                    pi[c] = h.x * r.y - h.y * r.x;
                }
                transpose_sum4_rows<T>(pr, lane);
                __builtin_amdgcn_sched_barrier(0);
                transpose_sum4_rows<T>(pi, lane);
                if ((lane & 15) == 0) psh[s & 3][wu + LA_NWT * (h0 + (lane >> 4))] = cmake<T>(pr[0], pi[0]);
            }
            if (lane == 0) lds_set(&p_done[wu], s + 1);
        };
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
        auto wait_b = [&](int q) -> bool {
            const uint64_t t0 = wall_clock64();
            for (;;) {
                if (__builtin_amdgcn_readfirstlane(lds_get(&b_ready)) > q &&
                    __builtin_amdgcn_readfirstlane(lds_get(&xs_ready)) > q)
                    return true;
                if (__builtin_amdgcn_readfirstlane(lds_get(&stop_w)) != 0) return false;
                if (wall_clock64() - t0 > 2 * tmo) return false;
                __builtin_amdgcn_s_sleep(1);
            }
        };

        Raw Ut[NC], Pt[NC];
        // prologue: partials of panels 0, 1, 2 from r0 (sequences 0, 1, 2), then U = panel
        // 0 and Pb = panel 3
        load_tile(Pt, 0);
        __builtin_amdgcn_sched_barrier(0);
        load_tile(Ut, 1 % np);
        __builtin_amdgcn_sched_barrier(0);
        partial(Pt, 0, 0);
        load_tile(Pt, 2 % np);
        __builtin_amdgcn_sched_barrier(0);
        partial(Ut, 1 % np, 1);
        load_tile(Ut, 0);
        __builtin_amdgcn_sched_barrier(0);
        partial(Pt, 2 % np, 2);
        load_tile(Pt, 3 % np);

        int K = 0;
        for (int q = 0;; ++q) {
            if (!wait_b(q)) break;
            {   // delta_K = M_K q_K + (-Y_K) delta_{K-1}; column v of the packed M holds rows
                // v..KP-1 at offset v*KP - v(v-1)/2; the first step has no correction
                constexpr int SV = KP / NS;
                const V* Mq = Ms[q & 1];
                const V* bq = bsh[q & 1];
                const int j = tid % KP, sl = tid / KP, v0 = sl * SV, v1 = min(v0 + SV - 1, j);
                V d0 = czero<T>(), d1 = czero<T>();
                if (q > 0) {
                    __builtin_amdgcn_sched_barrier(0);
                    const V* dp = dsh[(q - 1) & 1];
                    for (int u = v0; u < v0 + SV; u += 2) {
                        cfma(d0, Xs[u * KP + j], dp[u]);
                        cfma(d1, Xs[(u + 1) * KP + j], dp[u + 1]);
                    }
                }
                int off = v0 * KP - (v0 * (v0 - 1)) / 2 + (j - v0);
                int v = v0;
                for (; v + 1 <= v1; v += 2) {
                    cfma(d0, Mq[off], bq[v]);
                    off += KP - v - 1;
                    cfma(d1, Mq[off], bq[v + 1]);
                    off += KP - v - 2;
                }
                if (v <= v1) cfma(d0, Mq[off], bq[v]);
                dpart[sl][j] = cmake<T>(d0.x + d1.x, d0.y + d1.y);
            }
            tbar();
            if (bad) break;
            if (tid == 0) lds_set(&x_free, q + 1);   // every tile wave is done reading Xs
            if (tid < KP) {
                V s_ = dpart[0][tid];
                for (int k = 1; k < NS; ++k) {
                    s_.x += dpart[k][tid].x;
                    s_.y += dpart[k][tid].y;
                }
                dsh[q & 1][tid] = s_;
            }
            tbar();
            if (bad) break;
            if (tid == 0) lds_set(&d_ready, q + 1);
            {
                V acc = czero<T>();
#pragma unroll
                for (int c = 0; c < NC; ++c) cfma(acc, a.src.decode(Ut[c], tile_col(K, c)), dsh[q & 1][wu + LA_NWT * c]);
                axs[wu][lane] = acc;
            }
            tbar();
            if (bad) break;
            {
                V s_ = czero<T>();
#pragma unroll
                for (int k = 0; k < LA_NWT; ++k) {
                    s_.x += axs[k][lane].x;
                    s_.y += axs[k][lane].y;
                }
                if (row < B) {
                    r.x -= s_.x;
                    r.y -= s_.y;
                }
            }
            const int K1 = (K + 1 < np) ? K + 1 : 0;
            load_tile(Ut, K1);   // U is free: the next step's update tile (a cache hit)
            __builtin_amdgcn_sched_barrier(0);
            const int K3 = (K + 3) % np;
            partial(Pt, K3, q + 3);   // partials of panel K+3 from the residual after K
            load_tile(Pt, (K + 4) % np);
            K = K1;
        }
        return;
    }

    // ==================================== control wave ====================================
    uint32_t ok = 1;
    int sweeps = 0;
    double S = 0.0, Xn = 0.0, rel_last = 0.0;
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
        while (__builtin_amdgcn_readfirstlane(lds_get(&d_ready)) <= q) {
            if (wall_clock64() - t0 > tmo) return false;
            __builtin_amdgcn_s_sleep(1);
        }
        return true;
    };
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
    // reducer: the P partials of column j = w of sequence s, summed in a fixed order
    auto gather_partials = [&](int s, V& out) -> bool {
        const uint64_t* src = part64 + ((int64_t)(s & (DP_SLOTS - 1)) * KP + w) * P * NW;
        const uint32_t tag = (uint32_t)s + 1;
        V v[4];
        bool have[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = czero<T>();
            have[k] = lane + 64 * k >= P;
        }
        auto more = [&]() {
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
    // everyone: q and x of sequence s into LDS buffer s & 1
    auto gather_b = [&](int s) -> bool {
        const uint32_t tag = (uint32_t)s + 1;
        const uint64_t* q0 = gb64 + (((int64_t)(s & (DP_SLOTS - 1)) * KP + lane) * 2) * NW;
        V bv, xv;
        bool hb = false, hx = false;
        auto more = [&]() {
            V nb, nx;
            const bool okb = TG::get(q0, tag, nb), okx = TG::get(q0 + NW, tag, nx);
            if (!hb && okb) {
                bv = nb;
                hb = true;
            }
            if (!hx && okx) {
                xv = nx;
                hx = true;
            }
            return !(hb && hx);
        };
        if (!poll(more)) return false;
        bsh[s & 1][lane] = bv;
        xsh[s & 1][lane] = xv;
        return true;
    };
    // reducer: x and bias of its coordinate in panel K (x as this wave last wrote it)
    auto load_xb = [&](int K, V& xo, V& bb) {
        const int u = K * KP + w;
        xo = czero<T>();
        bb = czero<T>();
        if (u < U) {
            xo = a.x[u];
            if (a.bias) bb = a.bias[u];
        }
    };
    // reducer: publish q_s = g + bias - lambda x with x, for panel K of sequence s
    auto publish_q = [&](int s, V g, V xo, V bb) {
        if (lane == 0) {
            V b;
            b.x = g.x + bb.x - lambda * xo.x;
            b.y = g.y + bb.y - lambda * xo.y;
            uint64_t* q0 = gb64 + (((int64_t)(s & (DP_SLOTS - 1)) * KP + w) * 2) * NW;
            TG::put(q0, b, (uint32_t)s + 1);
            TG::put(q0 + NW, xo, (uint32_t)s + 1);
        }
    };
    auto stage_M = [&](int K, int buf) {
        const char* src = reinterpret_cast<const char*>(a.M + (int64_t)K * NE) + lane * 16;
        char* dst = reinterpret_cast<char*>(Ms[buf]);
#pragma unroll 4
        for (int off = 0; off < MS_BYTES; off += 1024)
            __builtin_amdgcn_global_load_lds(src + off, (__attribute__((address_space(3))) void*)(dst + off), 16, 0, 0);
    };

    int state = 0;   // 0 running, 1 stopped (converged or T_max), 2 abandoned
    if (a.T_max >= 1) {
        // prologue: the partials of sequences 0, 1, 2 (from r0; the X-staging wave
        // publishes the later ones); q_0 and q_1 need no distance-two correction (no delta
        // before step 0); q_0 and M_0 into LDS
        stage_M(0, 0);
        for (int s = 0; s < 3 && ok; ++s) {
            ok = wait_parts(s + 1);
            if (ok) publish_partials(s);
        }
        if (ok && reducer) {
            V g, xo, bb;
            ok = gather_partials(0, g);
            load_xb(0, xo, bb);
            if (ok) publish_q(0, g, xo, bb);
            if (ok) ok = gather_partials(1, g);
            load_xb(1 % np, xo, bb);
            if (ok) publish_q(1, g, xo, bb);
        }
        if (ok) ok = gather_b(0);
        wave_drain_vmem();   // the LDS-direct loads of M_0 have landed
        if (ok && lane == 0) lds_set(&b_ready, 1);
        int K = 0, t = 1;
        // statistics of step q and x of panel K; at the last panel of a sweep, the stop test
        auto stats = [&](int q, int K) -> bool {
            const V d = dsh[q & 1][lane];
            V xn;
            xn.x = xsh[q & 1][lane].x + d.x;
            xn.y = xsh[q & 1][lane].y + d.y;
            S += wave_allsum(cabs2d(d));
            Xn += wave_allsum(cabs2d(xn));
            if (reducer && lane == w) {
                const int u = K * KP + w;
                if (u < U) a.x[u] = xn;
            }
            if (K != np - 1) return false;
            sweeps = t;
            rel_last = (Xn > 0.0) ? sqrt(S / Xn) : (S > 0.0 ? INFINITY : 0.0);
            const bool done = t >= a.T_max || (a.tol > 0.0 && sqrt(S) <= a.tol * sqrt(Xn));
            S = 0.0;
            Xn = 0.0;
            ++t;
            return done;
        };
        // One step q (panel K) of the control wave.  The chain that paces the sweep runs
        // from the tile waves' delta_K through the reducers' q of sequence q + 2 to the tile
        // waves' next step; what lies on it is only the wait for delta, the gather of the
        // partials (published a step earlier), the correction, and the gather of b for step
        // q + 1 (published a step earlier).  The exchange hop of q itself has a step to
        // land.  Loads that do not depend on delta (M, and the reducer's row of X2 and x
        // and bias) are issued before the wait.
        for (int q = 0; ok; ++q) {
            const int K1 = (K + 1 < np) ? K + 1 : 0;
            const int K2 = (K + 2) % np;
            const bool last = K == np - 1;
            // M of step q + 1 into LDS buffer (q + 1) & 1, free since the tile waves passed
            // the product of step q - 1 (its only reader; they have delta of step q - 1)
            stage_M(K1, (q + 1) & 1);
            // reducer: row w of X2_{K+2} (element (w, lane)); x of its coordinate in panel
            // K+2, last written np - 2 >= 1 steps back by this wave, and the bias
            V xr = czero<T>(), xo, bb;
            if (reducer) {
                xr = a.X2[((int64_t)K2 * KP + lane) * KP + w];
                load_xb(K2, xo, bb);
            }
            ok = wait_delta(q);
            if (!ok) break;
            // at the last panel of a sweep the tile waves get step q + 1 only once the stop
            // test has passed: once set, b_ready lets every tile wave into the step, and all
            // of them must meet at its barriers
            if (last && stats(q, K)) {
                state = 1;
                break;
            }
            // reducer: q of sequence q + 2 from its partials (formed after step q - 1) less
            // row w of X2_{K+2} times delta_K (this step's, in dsh)
            if (reducer) {
                V g;
                ok = gather_partials(q + 2, g);
                if (!ok) break;
                V c = czero<T>();
                cfma(c, xr, dsh[q & 1][lane]);
                c.x = wave_allsum(c.x);
                c.y = wave_allsum(c.y);
                publish_q(q + 2, cmake<T>(g.x - c.x, g.y - c.y), xo, bb);
            }
            // q and x of step q + 1 (published by the reducers in step q - 1)
            ok = gather_b(q + 1);
            if (!ok) break;
            wave_drain_vmem();   // and the LDS-direct loads of M
            if (lane == 0) lds_set(&b_ready, q + 2);
            if (!last) stats(q, K);
            K = K1;
        }
    }
    if (!ok) state = 2;
    if (lane == 0) lds_set(&stop_w, state == 0 ? 1 : state);
    if (lane == 0) {
        int fl = 0;
        if (a.tol > 0.0 && !(rel_last <= a.tol)) fl |= CDM_INFO_NOT_CONVERGED;
        if (state == 2) fl |= CDM_INFO_TIMEOUT;
        if (w == 0) {
            cdm_info o;
            o.sweeps = sweeps;
            o.flags = fl;
            o.rel_step = rel_last;
            o.resid = -1.0;
            o.reserved = 0.0;
            a.info[0] = o;
        }
    }
}

hipError_t launch_panel_deep(const PanelLaunch& L, hipStream_t st) {
    if (!L.c128 || L.kp != DP_KP || L.rpl != 1 || L.npanels < 3 || L.src_kind != SRC_COMPLEX || !L.X || !L.X2)
        return hipErrorInvalidValue;
    using T = double;
    using Src = SrcC<T>;
    PanelArgs<T, Src> a;
    a.src = Src{(const cv<T>*)L.H};
    a.ld = L.ld;
    a.bias = (const cv<T>*)L.bias;
    a.done = L.done;
    a.r0 = (const cv<T>*)L.r0;
    a.x = (cv<T>*)L.x;
    a.M = (const cv<T>*)L.M;
    a.X = (const cv<T>*)L.X;
    a.X2 = (const cv<T>*)L.X2;
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
    return hipLaunchCooperativeKernel((const void*)k_cd_panel_deep<T, Src>, dim3(L.P), dim3(DP_THREADS), args, 0, st);
}

int panel_deep_max_coresident() {
    int dev = 0, ncu = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_cd_panel_deep<double, SrcC<double>>, DP_THREADS, 0) !=
        hipSuccess)
        return 0;
    return per * ncu;
}

}  // namespace cdm
