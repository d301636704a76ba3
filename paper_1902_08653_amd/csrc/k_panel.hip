// k_panel.hip -- cooperative "panel" engine for one large uplink instance.
//
// Block form of the cyclic sweep of Algorithm 1.  With r the residual at the start
// of a panel K of consecutive users, g_K = H_K^H r, b_u = g_u - lambda x_u, and
// G = H_K^H H_K split as D + L + L^H (D = diag(||h_u||^2 + lambda) after adding
// lambda), the U_K sequential coordinate updates of Algorithm 1 satisfy
//     delta_u = (b_u - sum_{v<u, v in K} G_uv delta_v) / (||h_u||^2 + lambda),
// i.e. (D + L) delta_K = b_K: exactly the same numbers, in exact arithmetic, as
// running the u-loop of Algorithm 1 one coordinate at a time.  Here
// M_K = (D + L)^-1 is formed once per solve (the panel Gram blocks on the matrix
// cores, k_gram_mfma.hip, then k_gram_invert), and every sweep applies
//     delta_K = M_K b_K,   x_K += delta_K,   r -= H_K delta_K.
//
// k_cd_panel runs all sweeps in one cooperative launch.  Workgroup w owns rows
// [64*RPL*w, 64*RPL*(w+1)) and keeps them of r in VGPRs; lane = row, and the
// NWV waves split each panel's columns.  Per panel:
//   1. partial g_K over the workgroup's rows (wave transpose-reduce), written to
//      a partial buffer, arrive on counter A;  the next panel's tile is loaded
//      into registers behind this;
//   2. reducer workgroup j (one per panel column) waits for A, sums the P
//      partials of column j in a fixed order, forms b_j = g_j - lambda x_j,
//      publishes (b_j, x_j), arrives on counter B; x_j is owned by reducer j;
//   3. every workgroup waits for B, computes delta_K = M_K b_K itself (identical
//      bits everywhere), applies r -= H_K delta_K from the tile still in
//      registers, and accumulates the stop statistics.
// H is read from HBM exactly once per sweep.
#include "panel.hpp"

namespace cdm {

template <typename T, int KP, int RPL, class Src>
__global__ __launch_bounds__(PANEL_NT, 1) void k_cd_panel(PanelArgs<T, Src> a) {
    using V = cv<T>;
    constexpr int NC = KP / PANEL_NWV;          // panel columns per wave
    static_assert(NC >= 1 && NC <= 64 && (NC & (NC - 1)) == 0, "bad panel split");

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    const int w = blockIdx.x;
    const int P = gridDim.x;
    const int R = P < KP ? P : KP;             // reducer workgroups
    const T lambda = (T)a.lambda;
    const int B = a.B, U = a.U;
    if (a.done && *a.done) return;   // uniform for the whole grid

    constexpr int NE = KP * (KP + 1) / 2;       // packed lower triangle of M_K
    constexpr int NS = PANEL_NT / KP;           // matvec slices per row
    __shared__ V Ms[NE];
    __shared__ V bsh[KP];
    __shared__ V xsh[KP];
    __shared__ V dsh[KP];
    // the matvec partials and the axpy partials are live in disjoint phases
    constexpr int SCR = (NS * KP > PANEL_NWV * RPL * 64) ? NS * KP : PANEL_NWV * RPL * 64;
    __shared__ V scr[SCR];
    V(*dpart)[KP] = reinterpret_cast<V(*)[KP]>(scr);
    V(*axs)[RPL][64] = reinterpret_cast<V(*)[RPL][64]>(scr);
    __shared__ uint32_t flag_s;

    // ctr layout: [2] abort, [3] status, [16, 16+P) partial-arrival flags,
    // [16+P, 16+P+KP) reducer flags; flag value = panel sequence number + 1
    uint32_t* abort_flag = a.ctr + 2;
    uint32_t* flagsA = a.ctr + 16;
    uint32_t* flagsB = a.ctr + 16 + P;

    const int row0 = w * 64 * RPL;
    V r[RPL];
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
        const int row = row0 + lane + 64 * q;
        r[q] = row < B ? a.r0[row] : czero<T>();
    }

    V tile[NC][RPL];
    V nxt[NC][RPL];
    auto load_panel = [&](int K) {
        // running per-lane element index: column K*KP + wid + NWV*c, row row0 + lane + 64q
        const int col0 = K * KP + wid;
        int64_t hi = (int64_t)col0 * a.ld + row0 + lane;
        const int64_t cstep = (int64_t)PANEL_NWV * a.ld;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int col = col0 + PANEL_NWV * c;
            const bool cok = col < U;
#pragma unroll
            for (int q = 0; q < RPL; ++q) {
                const bool rok = row0 + lane + 64 * q < B;
                nxt[c][q] = (cok && rok) ? a.src.load(hi + 64 * q, col) : czero<T>();
            }
            hi += cstep;
        }
    };
    load_panel(0);
    // stage the packed (D + L)^-1 of panel K into LDS, staged through registers
    auto stage_M = [&](int K) {
        constexpr int PER = (NE + PANEL_NT - 1) / PANEL_NT;
        // staged while the prefetch tile is not yet loaded, so its registers are free
        constexpr int CH = (sizeof(T) == 8) ? 8 : 16;
        const V* src = a.M + (int64_t)K * NE;
#pragma unroll
        for (int c0 = 0; c0 < PER; c0 += CH) {
            V buf[CH];
            // every load in range (clamped): a buffer filled under a per-thread condition
            // would be kept in scratch memory
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                const int e = (c0 + k) * PANEL_NT + tid;
                if (c0 + k < PER) buf[k] = src[min(e, NE - 1)];
            }
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                const int e = (c0 + k) * PANEL_NT + tid;
                if (c0 + k < PER && e < NE) Ms[e] = buf[k];
            }
        }
    };

    uint32_t seq = 0;
    int sweeps = 0;
    double S = 0.0, Xn = 0.0;
    bool ok = true;
    const bool reducer = w < R;

    for (int t = 1; t <= a.T_max && ok; ++t) {
        S = 0.0;
        Xn = 0.0;
        for (int K = 0; K < a.npanels; ++K) {
            const int par = seq & 1;
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int q = 0; q < RPL; ++q) tile[c][q] = nxt[c][q];

            // 1. partial g_K = H_K^H r over this workgroup's rows, in column halves to
            //    keep the per-lane partials small
            {
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
                            pr[c] += tile[h0 + c][q].x * r[q].x + tile[h0 + c][q].y * r[q].y;
                            pi[c] += tile[h0 + c][q].x * r[q].y - tile[h0 + c][q].y * r[q].x;
                        }
                    }
                    wave_transpose_sum<T, NH>(pr, lane);
                    wave_transpose_sum<T, NH>(pi, lane);
                    if ((lane & ((1 << HSHIFT) - 1)) == 0) {
                        const int j = wid + PANEL_NWV * (h0 + (lane >> HSHIFT));
                        st_dev(&a.part[((int64_t)par * KP + j) * P + w], cmake<T>(pr[0], pi[0]));
                    }
                }
            }
            wg_publish(flagsA, w, seq + 1);
            const int Kn = (K + 1 < a.npanels) ? K + 1 : 0;
            // with a single panel, M_0 and the tile stay in LDS and registers after the first step
            const bool one = a.npanels == 1;
            if (!reducer) {
                // M_K first: waiting for its loads must not wait for the tile stream
                // (vector loads complete in issue order)
                if (!one || seq == 0) stage_M(K);
                if (!one) load_panel(Kn);
            }

            // 2. reducers: g_j = sum of the P partials (fixed order: lane l adds p = l, l + 64,
            //    ..., then a fixed butterfly), b_j = g_j - lambda x_j.  One wave per column, so
            //    a reducer's columns are summed side by side with no workgroup barrier.
            if (reducer) {
                ok = wg_wait_flags(flagsA, P, seq + 1, abort_flag, a.timeout_ticks, &flag_s);
                if (ok) {
                    for (int j = w + P * wid; j < KP; j += P * PANEL_NWV) {
                        V g = czero<T>();
                        for (int p = lane; p < P; p += 64) {
                            const V v = ld_dev(&a.part[((int64_t)par * KP + j) * P + p]);
                            g.x += v.x;
                            g.y += v.y;
                        }
                        g.x = wave_allsum(g.x);
                        g.y = wave_allsum(g.y);
                        if (lane == 0) {
                            const int u = K * KP + j;
                            const V xo = (u < U) ? a.x[u] : czero<T>();
                            if (a.bias && u < U) {
                                const V bb = a.bias[u];
                                g.x += bb.x;
                                g.y += bb.y;
                            }
                            V b;
                            b.x = g.x - lambda * xo.x;
                            b.y = g.y - lambda * xo.y;
                            st_dev(&a.gbuf[((int64_t)par * KP + j) * 2 + 0], b);
                            st_dev(&a.gbuf[((int64_t)par * KP + j) * 2 + 1], xo);
                        }
                    }
                }
                wg_publish(flagsB, w, seq + 1);   // after every wave's stores (drain + barrier)
                if (!one || seq == 0) stage_M(K);
                if (!one) load_panel(Kn);
            }
            if (!ok) break;

            // 3. everyone: delta_K = M_K b_K, x_K += delta_K, r -= H_K delta_K
            ok = wg_wait_flags(flagsB, R, seq + 1, abort_flag, a.timeout_ticks, &flag_s);
            if (!ok) break;
            for (int j = tid; j < KP; j += PANEL_NT) {
                bsh[j] = ld_dev(&a.gbuf[((int64_t)par * KP + j) * 2 + 0]);
                xsh[j] = ld_dev(&a.gbuf[((int64_t)par * KP + j) * 2 + 1]);
            }
            __syncthreads();
            {
                // delta_j = sum_{v <= j} M_jv b_v from the packed M_K in LDS (column v holds
                // rows v..KP-1 at offset v*KP - v(v-1)/2); NS threads per row j, each over a
                // contiguous slice of v
                constexpr int SV = KP / NS;                // v per slice
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
                __syncthreads();
                if (tid < KP) {
                    V s = dpart[0][tid];
#pragma unroll
                    for (int k = 1; k < NS; ++k) {
                        s.x += dpart[k][tid].x;
                        s.y += dpart[k][tid].y;
                    }
                    dsh[tid] = s;
                }
            }
            __syncthreads();
            if (reducer && tid == 0) {
                for (int j = w; j < KP; j += P) {
                    const int u = K * KP + j;
                    if (u < U) {
                        V xn;
                        xn.x = xsh[j].x + dsh[j].x;
                        xn.y = xsh[j].y + dsh[j].y;
                        a.x[u] = xn;
                    }
                }
            }
            {
                double s1 = 0.0, s2 = 0.0;
                for (int j = lane; j < KP; j += 64) {
                    const V d = dsh[j];
                    V xn;
                    xn.x = xsh[j].x + d.x;
                    xn.y = xsh[j].y + d.y;
                    s1 += cabs2d(d);
                    s2 += cabs2d(xn);
                }
                S += wave_allsum(s1);
                Xn += wave_allsum(s2);
            }
#pragma unroll
            for (int q = 0; q < RPL; ++q) {
                V acc = czero<T>();
#pragma unroll
                for (int c = 0; c < NC; ++c) cfma(acc, tile[c][q], dsh[wid + PANEL_NWV * c]);
                axs[wid][q][lane] = acc;
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < RPL; ++q) {
                V s = czero<T>();
#pragma unroll
                for (int v = 0; v < PANEL_NWV; ++v) {
                    s.x += axs[v][q][lane].x;
                    s.y += axs[v][q][lane].y;
                }
                r[q].x -= s.x;
                r[q].y -= s.y;
            }
            ++seq;
        }
        if (!ok) break;
        sweeps = t;
        if (a.tol > 0.0 && sqrt(S) <= a.tol * sqrt(Xn)) break;
    }
    if (w == 0 && tid == 0) {
        const double rel = (Xn > 0.0) ? sqrt(S / Xn) : (S > 0.0 ? INFINITY : 0.0);
        int fl = 0;
        if (a.tol > 0.0 && !(rel <= a.tol)) fl |= CDM_INFO_NOT_CONVERGED;
        if (!ok) fl |= CDM_INFO_TIMEOUT;
        cdm_info o;
        o.sweeps = sweeps;
        o.flags = fl;
        o.rel_step = rel;
        o.resid = -1.0;
        o.reserved = 0.0;
        a.info[0] = o;
    }
}

template <typename T, int KP, int RPL, class Src>
static hipError_t launch_panel_src(const PanelLaunch& L, const Src& src, hipStream_t st) {
    PanelArgs<T, Src> a;
    a.src = src;
    a.ld = L.ld;
    a.bias = (const cv<T>*)L.bias;
    a.done = L.done;
    a.r0 = (const cv<T>*)L.r0;
    a.x = (cv<T>*)L.x;
    a.M = (const cv<T>*)L.M;
    a.X = nullptr;
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
    return hipLaunchCooperativeKernel((const void*)k_cd_panel<T, KP, RPL, Src>, dim3(L.P), dim3(PANEL_NT), args, 0,
                                      st);
}

template <typename T, int KP, int RPL>
static hipError_t launch_panel_t(const PanelLaunch& L, hipStream_t st) {
    if (L.src_kind == SRC_BF16) {
        if constexpr (sizeof(T) == 4) return launch_panel_src<T, KP, RPL>(L, SrcBF16{L.q_re16, L.q_im16}, st);
        return hipErrorInvalidValue;
    }
    if (L.src_kind == SRC_FP8) {
        if constexpr (sizeof(T) == 4) return launch_panel_src<T, KP, RPL>(L, SrcFP8{L.q_re8, L.q_im8, L.q_scale}, st);
        return hipErrorInvalidValue;
    }
    return launch_panel_src<T, KP, RPL>(L, SrcC<T>{(const cv<T>*)L.H}, st);
}

template <typename T, int KP, int RPL>
static int coresident_t() {
    int dev = 0, ncu = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_cd_panel<T, KP, RPL, SrcC<T>>, PANEL_NT, 0) != hipSuccess)
        return 0;
    return per * ncu;
}

hipError_t launch_panel(const PanelLaunch& L, hipStream_t st) {
    if (L.c128) {
        if (L.kp == 64 && L.rpl == 1) return launch_panel_t<double, 64, 1>(L, st);
        if (L.kp == 64 && L.rpl == 2) return launch_panel_t<double, 64, 2>(L, st);
        if (L.kp == 128 && L.rpl == 1) return launch_panel_t<double, 128, 1>(L, st);
    } else {
        if (L.kp == 128 && L.rpl == 1) return launch_panel_t<float, 128, 1>(L, st);
        if (L.kp == 128 && L.rpl == 2) return launch_panel_t<float, 128, 2>(L, st);
    }
    return hipErrorInvalidValue;
}

int panel_max_coresident(bool c128, int kp, int rpl) {
    if (c128) {
        if (kp == 64 && rpl == 1) return coresident_t<double, 64, 1>();
        if (kp == 64 && rpl == 2) return coresident_t<double, 64, 2>();
        if (kp == 128 && rpl == 1) return coresident_t<double, 128, 1>();
    } else {
        if (kp == 128 && rpl == 1) return coresident_t<float, 128, 1>();
        if (kp == 128 && rpl == 2) return coresident_t<float, 128, 2>();
    }
    return 0;
}

// Sum the split partials, form D + L (lambda on the diagonal; inactive coordinates
// with ||h_u||^2 + lambda == 0 decoupled), and invert it row by row:
//   M_uc = ([u == c] - sum_{c <= v < u} A_uv M_vc) / A_uu.
// One workgroup of kp threads per panel; thread c owns column c of M.  The rows of M
// the recurrence reads back live in LDS (dynamic, kp * kp values) where they fit, else in
// the global scratch Mrow.
// Sum of the Gram partials over the row splits, in place into split 0, for the elements
// with u >= v of every diagonal block (the only ones the inversion reads); the same fixed
// order as the inversion's own sum.  One thread per element: the whole chip works on it.
template <typename V>
__global__ __launch_bounds__(256) void k_sum_lower(V* __restrict__ part, int nsplit, int64_t n, int kp) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t rem = i % ((int64_t)kp * kp);
    if (rem / kp < rem % kp) return;
    V s = part[i];
    for (int k = 1; k < nsplit; ++k) {
        const V p = part[(int64_t)k * n + i];
        s.x += p.x;
        s.y += p.y;
    }
    part[i] = s;
}

// MLDS is a template argument so that the LDS form's accesses to Mr compile to LDS
// instructions: behind a run-time choice they are generic (flat) accesses, and each one then
// also waits for the thread's outstanding global loads and stores.
template <typename T, bool MLDS>
__global__ __launch_bounds__(256) void k_gram_invert(cv<T>* __restrict__ gpart, int nsplit, int npanels, int kp, int U,
                                                     double lambda, cv<T>* __restrict__ Mcm, cv<T>* __restrict__ Mrow,
                                                     double* __restrict__ e_out, uint32_t* __restrict__ status) {
    using V = cv<T>;
    extern __shared__ __attribute__((aligned(16))) char inv_dyn[];
    const int K = blockIdx.x;
    const int c = threadIdx.x;
    const int64_t pstride = (int64_t)npanels * kp * kp;
    V* A = gpart + (int64_t)K * kp * kp;          // split 0 slot receives the sum
    __shared__ V arow[256];
    __shared__ T dsh[256];
    __shared__ int act[256];
    // 1. sum over splits (elements with u >= v), fixed order.  Thread c (blockDim == kp) owns
    //    column v = c and is the only thread that reads these elements back below; four rows
    //    at a time, so that four loads per split are in flight.  (The panel pre-pass sums the
    //    splits beforehand with k_sum_lower and passes nsplit = 1.)
    for (int u0 = c; nsplit > 1 && u0 < kp; u0 += 4) {
        V s[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) s[i] = (u0 + i < kp) ? A[(int64_t)(u0 + i) * kp + c] : czero<T>();
        for (int sp = 1; sp < nsplit; ++sp) {
            const V* P = gpart + sp * pstride + (int64_t)K * kp * kp;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (u0 + i < kp) {
                    const V p = P[(int64_t)(u0 + i) * kp + c];
                    s[i].x += p.x;
                    s[i].y += p.y;
                }
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (u0 + i < kp) A[(int64_t)(u0 + i) * kp + c] = s[i];
    }
    __syncthreads();
    // 2. diagonal: energies, activity
    if (c < kp) {
        const int u = K * kp + c;
        const T e = A[(int64_t)c * kp + c].x;
        const bool valid = u < U;
        const bool live = valid && ((double)e + lambda > 0.0);
        act[c] = live ? 1 : 0;
        dsh[c] = live ? (T)((double)e + lambda) : T(1);
        if (valid) e_out[u] = (double)e;
        if (valid && !live) atomicOr(status, (uint32_t)CDM_INFO_ZERO_COLUMN);
    }
    __syncthreads();
    // 3. inverse of (D + L), row by row
    V* Mr = MLDS ? reinterpret_cast<V*>(inv_dyn) : Mrow + (int64_t)K * kp * kp;
    V* Mp = Mcm + (int64_t)K * (kp * (kp + 1) / 2);
    V an = czero<T>();   // this thread's element of the next row of A, loaded a row ahead
    for (int u = 0; u < kp; ++u) {
        const V acur = an;
        if (u + 1 < kp && c < u + 1) an = A[(int64_t)(u + 1) * kp + c];
        if (c < u) {
            const bool live = act[u] && act[c];
            arow[c] = live ? acur : czero<T>();
        }
        __syncthreads();
        if (c < kp) {
            V s = (u == c) ? cmake<T>(T(1), T(0)) : czero<T>();
            if (c < u) {
                // four accumulators over v = c, c+1, ... (the chain of dependent FMAs is the
                // kernel's critical path), added in a fixed order at the end
                // groups of four v; with M in LDS each group's operands are loaded one group
                // ahead, so that the loads overlap the FMAs (the same sums in the same order;
                // the compiler may contract the products differently).  With M in global
                // memory the plain loop measured faster.
                V s1 = czero<T>(), s2 = czero<T>(), s3 = czero<T>();
                int v = c;
                if (!MLDS) {
                    for (; v + 3 < u; v += 4) {
                        cfms(s, arow[v], Mr[(int64_t)v * kp + c]);
                        cfms(s1, arow[v + 1], Mr[(int64_t)(v + 1) * kp + c]);
                        cfms(s2, arow[v + 2], Mr[(int64_t)(v + 2) * kp + c]);
                        cfms(s3, arow[v + 3], Mr[(int64_t)(v + 3) * kp + c]);
                    }
                } else if (v + 3 < u) {
                    V a0 = arow[v], a1 = arow[v + 1], a2 = arow[v + 2], a3 = arow[v + 3];
                    V m0 = Mr[(int64_t)v * kp + c], m1 = Mr[(int64_t)(v + 1) * kp + c];
                    V m2 = Mr[(int64_t)(v + 2) * kp + c], m3 = Mr[(int64_t)(v + 3) * kp + c];
                    for (v += 4; v + 3 < u; v += 4) {
                        const V b0 = arow[v], b1 = arow[v + 1], b2 = arow[v + 2], b3 = arow[v + 3];
                        const V n0 = Mr[(int64_t)v * kp + c], n1 = Mr[(int64_t)(v + 1) * kp + c];
                        const V n2 = Mr[(int64_t)(v + 2) * kp + c], n3 = Mr[(int64_t)(v + 3) * kp + c];
                        cfms(s, a0, m0);
                        cfms(s1, a1, m1);
                        cfms(s2, a2, m2);
                        cfms(s3, a3, m3);
                        a0 = b0; a1 = b1; a2 = b2; a3 = b3;
                        m0 = n0; m1 = n1; m2 = n2; m3 = n3;
                    }
                    cfms(s, a0, m0);
                    cfms(s1, a1, m1);
                    cfms(s2, a2, m2);
                    cfms(s3, a3, m3);
                }
                for (; v < u; ++v) cfms(s, arow[v], Mr[(int64_t)v * kp + c]);
                s.x = (s.x + s1.x) + (s2.x + s3.x);
                s.y = (s.y + s1.y) + (s2.y + s3.y);
            }
            V m = czero<T>();
            if (c <= u && act[u]) {
                m.x = s.x / dsh[u];
                m.y = s.y / dsh[u];
            }
            Mr[(int64_t)u * kp + c] = m;
            if (c <= u) Mp[(int64_t)c * kp - ((int64_t)c * (c - 1)) / 2 + (u - c)] = m;
        }
        __syncthreads();
    }
}

// the row-major M of one panel in LDS where it fits (128 KB at most: complex64 k = 128,
// complex128 k = 64), else the global scratch
template <typename T>
static hipError_t launch_invert_t(cv<T>* gpart, int nsplit, int npanels, int kp, int U, double lambda, cv<T>* M,
                                  cv<T>* Mrow, double* e, uint32_t* status, hipStream_t st) {
    const size_t mb = (size_t)kp * kp * sizeof(cv<T>);
    int in_lds = mb <= (size_t)128 * 1024;
    if (in_lds && mb > 64 * 1024 &&
        hipFuncSetAttribute((const void*)k_gram_invert<T, true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)mb) !=
            hipSuccess) {
        (void)hipGetLastError();
        in_lds = 0;
    }
    if (in_lds)
        hipLaunchKernelGGL((k_gram_invert<T, true>), dim3(npanels), dim3(kp), mb, st, gpart, nsplit, npanels, kp, U,
                           lambda, M, Mrow, e, status);
    else
        hipLaunchKernelGGL((k_gram_invert<T, false>), dim3(npanels), dim3(kp), 0, st, gpart, nsplit, npanels, kp, U,
                           lambda, M, Mrow, e, status);
    return hipGetLastError();
}

template <typename T> static hipError_t launch_gram_t(const GramLaunch& L, hipStream_t st) {
    if (L.src_kind == SRC_BF16 || L.src_kind == SRC_FP8) {
        // the low-precision copies: matrix cores (FP32 partials, same layout)
        if constexpr (sizeof(T) == 4) {
            hipError_t e = launch_gram_lp(L, false, 1, st);
            if (e != hipSuccess) return e;
        } else {
            return hipErrorInvalidValue;
        }
    } else {   // complex H: FP64 (complex128) or FP32 (complex64) matrix cores
        hipError_t e = launch_gram_cx(L, false, 1, st);
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // M is written twice: column-major (used by the sweep) and row-major (the
    // recurrence reads its own earlier rows); the row-major copy lives in the
    // split-1 slot of gpart (at least two slots), free once the splits are summed.
    cv<T>* Mrow = (cv<T>*)L.gpart + (int64_t)L.npanels * L.kp * L.kp;
    if (L.nsplit > 1) {
        const int64_t n = (int64_t)L.npanels * L.kp * L.kp;
        hipLaunchKernelGGL(k_sum_lower<cv<T>>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (cv<T>*)L.gpart,
                           L.nsplit, n, L.kp);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return launch_invert_t<T>((cv<T>*)L.gpart, 1, L.npanels, L.kp, L.U, L.lambda, (cv<T>*)L.M, Mrow, L.e, L.status,
                              st);
}

hipError_t launch_gram_invert(bool c128, void* gpart, int nsplit, int npanels, int kp, int U, double lambda, void* M,
                              double* e, uint32_t* status, hipStream_t st) {
    if (c128) {
        using V = cv<double>;
        return launch_invert_t<double>((V*)gpart, nsplit, npanels, kp, U, lambda, (V*)M,
                                       (V*)gpart + (int64_t)npanels * kp * kp, e, status, st);
    }
    using V = cv<float>;
    return launch_invert_t<float>((V*)gpart, nsplit, npanels, kp, U, lambda, (V*)M,
                                  (V*)gpart + (int64_t)npanels * kp * kp, e, status, st);
}

hipError_t launch_gram(const GramLaunch& L, hipStream_t st) {
    return L.c128 ? launch_gram_t<double>(L, st) : launch_gram_t<float>(L, st);
}

// X[i] = sum over splits of part[s][i], fixed order
template <typename V>
// X (one kp x kp block per panel) = sum of the split partials, written transposed:
// element (j, v) of block K lands at (K, v, j), so that a product X_K delta reads
// consecutive j for consecutive lanes
__global__ void k_sum_splits(const V* __restrict__ part, int nsplit, int64_t n, int kp, V* __restrict__ X) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    V s = part[i];
    for (int k = 1; k < nsplit; ++k) {
        const V p = part[(int64_t)k * n + i];
        s.x += p.x;
        s.y += p.y;
    }
    const int64_t kk = (int64_t)kp * kp;
    const int64_t blk = i / kk, rem = i % kk;
    const int j = (int)(rem / kp), v = (int)(rem % kp);
    X[blk * kk + (int64_t)v * kp + j] = s;
}

// -Y_K = -M_K X_K for every panel, in place of X_K (complex128, 64-column panels: the
// look-ahead schedule then forms delta_K = M_K q_K + (-Y_K) delta_{K-1} in one product
// instead of correcting b first).  One workgroup per panel; M_K (packed lower, column
// by column) and X_K (column-major) are read into LDS before any result is written.
template <typename V, int KP>
__global__ __launch_bounds__(256) void k_fold_mx(const V* __restrict__ M, V* __restrict__ X) {
    constexpr int NE = KP * (KP + 1) / 2;
    __shared__ V Ms[NE];
    __shared__ V Xs[KP * KP];
    const int64_t K = blockIdx.x;
    const V* Mk = M + K * NE;
    V* Xk = X + K * KP * KP;
    for (int i = threadIdx.x; i < NE; i += 256) Ms[i] = Mk[i];
    for (int i = threadIdx.x; i < KP * KP; i += 256) Xs[i] = Xk[i];
    __syncthreads();
    for (int i = threadIdx.x; i < KP * KP; i += 256) {
        const int v = i / KP, j = i % KP;   // element (j, v), stored at v * KP + j
        V acc;
        acc.x = 0;
        acc.y = 0;
        for (int u = 0; u <= j; ++u) cfma(acc, Ms[u * KP - (u * (u - 1)) / 2 + (j - u)], Xs[v * KP + u]);
        acc.x = -acc.x;
        acc.y = -acc.y;
        Xk[i] = acc;
    }
}

template <typename T>
static hipError_t launch_gram_cross_t(const GramLaunch& L, void* X, hipStream_t st, int dist = 1, bool fold = true) {
    if (L.src_kind == SRC_BF16 || L.src_kind == SRC_FP8) {
        if constexpr (sizeof(T) == 4) {
            hipError_t e = launch_gram_lp(L, true, dist, st);
            if (e != hipSuccess) return e;
        } else {
            return hipErrorInvalidValue;
        }
    } else {
        hipError_t e = launch_gram_cx(L, true, dist, st);
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t n = (int64_t)L.npanels * L.kp * L.kp;
    hipLaunchKernelGGL(k_sum_splits<cv<T>>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       (const cv<T>*)L.gpart, L.nsplit, n, L.kp, (cv<T>*)X);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (fold && L.kp == 64) {   // the configurations whose look-ahead forms b locally
        hipLaunchKernelGGL((k_fold_mx<cv<T>, 64>), dim3(L.npanels), dim3(256), 0, st, (const cv<T>*)L.M, (cv<T>*)X);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_gram_cross(const GramLaunch& L, void* X, hipStream_t st) {
    return L.c128 ? launch_gram_cross_t<double>(L, X, st) : launch_gram_cross_t<float>(L, X, st);
}

hipError_t launch_gram_cross2(const GramLaunch& L, void* X2, hipStream_t st) {
    return L.c128 ? launch_gram_cross_t<double>(L, X2, st, 2, false) : launch_gram_cross_t<float>(L, X2, st, 2, false);
}

}  // namespace cdm
