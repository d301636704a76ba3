// runtime.hip -- the C ABI (include/cdm.h): plan creation, validation, workspace,
// engine choice and kernel dispatch.  Host code only; every numerical step runs
// in the kernels of k_wg.hip, k_panel.hip and k_aux.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "cdm.h"
#include "launch.hpp"

using namespace cdm;

namespace {

thread_local char g_last_error[512] = "";

void set_err(const char* where, hipError_t e) {
    snprintf(g_last_error, sizeof(g_last_error), "%s: %s", where, hipGetErrorString(e));
}

#define HIP_TRY(call)                               \
    do {                                            \
        hipError_t e_ = (call);                     \
        if (e_ != hipSuccess) {                     \
            set_err(#call, e_);                     \
            return CDM_EHIP;                        \
        }                                           \
    } while (0)

constexpr int kWgMaxRows = 8192;      // 1024 threads x 8 rows
constexpr size_t kLdsMax = 160 * 1024;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Arena {
    size_t off = 0;
    size_t take(size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    }
};

}  // namespace

struct cdm_plan {
    cdm_desc d{};
    bool batched = false;
    int device = 0;
    int ncu = 0;
    bool c128 = true;
    size_t esz = 16;          // bytes per complex element
    int engine = CDM_ENGINE_WG;
    // WG engine
    int wg_nt = 256, wg_rpt = 1, wg_grid = 1, n_max = 1;
    size_t wg_lds = 0;
    int njobs = 0;
    // PANEL engine
    int kp = 128, rpl = 1, P = 1, npanels = 1, nsplit = 1;
    uint64_t timeout_ticks = 0;
    // workspace
    char* ws = nullptr;
    size_t ws_bytes = 0;
    uint32_t* ctr = nullptr;  // [0] A, [1] B, [2] abort, [3] status, [4] queue
    WgJob* jobs = nullptr;
    int* order = nullptr;
    void* r0 = nullptr;
    void* M = nullptr;
    void* gpart = nullptr;
    void* part = nullptr;
    void* gbuf = nullptr;
    double* e = nullptr;
    void* xloc = nullptr;
    double* msum = nullptr;
    void* rpart = nullptr;    // warm-start product scratch
    int nchunk = 1;
    double* res_rpart = nullptr;
    double* res_r = nullptr;
    double* res_col = nullptr;
    double* res_out = nullptr;
    // batched layout
    std::vector<int64_t> H_off, y_off, x_off;
    std::string text;
};

static int32_t validate_common(const cdm_desc* d) {
    if (!d) return CDM_EINVAL;
    if (d->problem != CDM_UPLINK_LMMSE && d->problem != CDM_DOWNLINK_ZF) return CDM_EDTYPE;
    if (d->precision < CDM_C128 || d->precision > CDM_MIXED_FP8) return CDM_EDTYPE;
    if (d->layout != CDM_DENSE && d->layout != CDM_CSR) return CDM_EDTYPE;
    if (d->engine < CDM_ENGINE_AUTO || d->engine > CDM_ENGINE_PANEL) return CDM_EINVAL;
    if (d->T_max < 1 || d->T_max > 100000) return CDM_EINVAL;
    if (!(d->tol >= 0.0) || !std::isfinite(d->tol)) return CDM_EINVAL;
    return CDM_OK;
}

static int32_t device_setup(cdm_plan* p) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return CDM_ENODEV;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return CDM_ENODEV;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        snprintf(g_last_error, sizeof(g_last_error), "device %d is %s, this library is built for gfx950", dev,
                 prop.gcnArchName);
        return CDM_ENODEV;
    }
    p->device = dev;
    p->ncu = prop.multiProcessorCount;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) khz = 100000;
    p->timeout_ticks = (uint64_t)khz * 1000ull * 4ull;   // 4 s per cross-workgroup wait
    return CDM_OK;
}

static int32_t alloc_ws(cdm_plan* p, size_t bytes) {
    p->ws_bytes = bytes;
    if (hipMalloc((void**)&p->ws, bytes) != hipSuccess) {
        p->ws = nullptr;
        return CDM_ENOMEM;
    }
    return CDM_OK;
}

// choose the WG-engine tile for rows m_max
static bool wg_tile(int m_max, int* nt, int* rpt) {
    static const int nts[2] = {256, 1024};
    static const int rpts[4] = {1, 2, 4, 8};
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 4; ++b)
            if (nts[a] * rpts[b] >= m_max) {
                // prefer 256 threads up to 2048 rows, then 1024 threads
                if (nts[a] == 256 || m_max > 2048) {
                    *nt = nts[a];
                    *rpt = rpts[b];
                    return true;
                }
            }
    return false;
}

static int32_t setup_wg(cdm_plan* p, int m_max, int n_max, int njobs) {
    if (!wg_tile(m_max, &p->wg_nt, &p->wg_rpt)) return CDM_ESHAPE;
    p->n_max = std::max(1, n_max);
    p->wg_lds = wg_lds_bytes(p->n_max, p->c128);
    if (p->wg_lds + 2048 > kLdsMax) return CDM_ESHAPE;
    if (p->wg_lds > 64 * 1024) {
        if (wg_set_lds_limit(p->c128, p->wg_nt, p->wg_rpt, p->wg_lds) != hipSuccess) return CDM_ESHAPE;
    }
    const int occ = std::max(1, wg_occupancy(p->c128, p->wg_nt, p->wg_rpt, p->wg_lds));
    p->wg_grid = std::max(1, std::min(njobs, occ * p->ncu));
    p->njobs = njobs;
    return CDM_OK;
}

extern "C" {

int32_t cdm_version(void) { return CDM_ABI_VERSION; }

const char* cdm_status_string(int32_t s) {
    switch (s) {
        case CDM_OK: return "ok";
        case CDM_EINVAL: return "invalid argument";
        case CDM_ESHAPE: return "inconsistent or unsupported shape";
        case CDM_EDTYPE: return "unsupported precision/problem/layout";
        case CDM_ENOMEM: return "device allocation failed";
        case CDM_EHIP: return "HIP runtime error";
        case CDM_EINFEASIBLE: return "infeasible problem (B_c < U)";
        case CDM_ENOTIMPL: return "not implemented";
        case CDM_ENODEV: return "no gfx950 device";
        default: return "unknown status";
    }
}

const char* cdm_last_error(void) { return g_last_error; }

int32_t cdm_create(const cdm_desc* desc, cdm_plan** plan) {
    if (!plan) return CDM_EINVAL;
    *plan = nullptr;
    int32_t st = validate_common(desc);
    if (st) return st;
    const cdm_desc& d = *desc;
    if (d.B < 1 || d.U < 1 || d.C < 1 || d.B % d.C) return CDM_ESHAPE;
    const int Bc = d.B / d.C;
    if (d.problem == CDM_DOWNLINK_ZF && Bc < d.U) return CDM_EINFEASIBLE;
    if (d.problem != CDM_UPLINK_LMMSE || d.layout != CDM_DENSE ||
        (d.precision != CDM_C128 && d.precision != CDM_C64))
        return CDM_ENOTIMPL;

    cdm_plan* p = new cdm_plan();
    p->d = d;
    p->c128 = d.precision == CDM_C128;
    p->esz = p->c128 ? 16 : 8;
    st = device_setup(p);
    if (st) {
        delete p;
        return st;
    }

    // engine choice: one cooperative launch for a single large instance, else WG
    int engine = d.engine;
    const double elems = (double)d.B * d.U;
    if (engine == CDM_ENGINE_AUTO) engine = (d.C == 1 && d.B >= 2048 && elems >= 4.0e6) ? CDM_ENGINE_PANEL : CDM_ENGINE_WG;
    if (engine == CDM_ENGINE_PANEL && d.C != 1) engine = CDM_ENGINE_WG;
    if (engine == CDM_ENGINE_WG && Bc > kWgMaxRows) engine = CDM_ENGINE_PANEL;
    if (engine == CDM_ENGINE_PANEL && d.C != 1) {
        delete p;
        return CDM_ESHAPE;
    }
    p->engine = engine;

    Arena ar;
    const size_t o_ctr = ar.take(64);
    size_t o_jobs = 0, o_r0 = 0, o_M = 0, o_gpart = 0, o_part = 0, o_gbuf = 0, o_e = 0, o_xloc = 0,
           o_msum = 0, o_rpart = 0;
    p->nchunk = std::max(1, std::min(64, (d.U + 127) / 128));
    if (engine == CDM_ENGINE_WG) {
        st = setup_wg(p, Bc, d.U, d.C);
        if (st) {
            delete p;
            return st;
        }
        o_jobs = ar.take(sizeof(WgJob) * d.C);
        if (d.C > 1) {
            o_xloc = ar.take(p->esz * (size_t)d.C * d.U);
            o_msum = ar.take(sizeof(double) * d.C);
        }
    } else {
        // panel width and rows per lane: keep one 64*rpl-row block per co-resident workgroup
        const int kps_c128[2] = {128, 64};
        const int kps_c64[2] = {256, 128};
        const int* kps = p->c128 ? kps_c128 : kps_c64;
        bool found = false;
        for (int i = 0; i < 2 && !found; ++i) {
            const int kp = kps[i];
            if (d.panel && d.panel != kp) continue;
            const int rpl = (i == 0) ? 1 : 2;
            const int P = (d.B + 64 * rpl - 1) / (64 * rpl);
            const int maxc = panel_max_coresident(p->c128, kp, rpl);
            if (P <= maxc) {
                p->kp = kp;
                p->rpl = rpl;
                p->P = P;
                found = true;
            }
        }
        if (!found) {
            delete p;
            return CDM_ESHAPE;
        }
        p->npanels = (d.U + p->kp - 1) / p->kp;
        const int nb = p->kp / 64;
        const int nsub = nb * (nb + 1) / 2;
        p->nsplit = std::max(1, std::min(32, (1024 + p->npanels * nsub - 1) / (p->npanels * nsub)));
        p->nsplit = std::min(p->nsplit, std::max(1, d.B / 256));
        const size_t kk = (size_t)p->kp * p->kp * p->npanels;
        o_r0 = ar.take(p->esz * d.B);
        o_M = ar.take(p->esz * kk);
        o_gpart = ar.take(p->esz * kk * std::max(2, p->nsplit));
        o_part = ar.take(p->esz * 2 * (size_t)p->kp * p->P);
        o_gbuf = ar.take(p->esz * 2 * (size_t)p->kp * 2);
        o_e = ar.take(sizeof(double) * d.U);
        o_rpart = ar.take(p->esz * (size_t)p->nchunk * d.B);
    }
    const size_t o_res_rpart = ar.take(16 * (size_t)p->nchunk * d.B);
    const size_t o_res_r = ar.take(16 * (size_t)d.B);
    const size_t o_res_col = ar.take(16 * (size_t)((d.U + 3) / 4 + 1));
    const size_t o_res_out = ar.take(8 * (size_t)d.C);

    st = alloc_ws(p, ar.off);
    if (st) {
        delete p;
        return st;
    }
    char* b = p->ws;
    p->ctr = (uint32_t*)(b + o_ctr);
    if (engine == CDM_ENGINE_WG) {
        p->jobs = (WgJob*)(b + o_jobs);
        if (d.C > 1) {
            p->xloc = b + o_xloc;
            p->msum = (double*)(b + o_msum);
        }
        std::vector<WgJob> jobs(d.C);
        for (int c = 0; c < d.C; ++c) {
            WgJob& j = jobs[c];
            j.h_off = (int64_t)c * Bc;
            j.ld = 0;   // the solve's ldh
            j.y_off = (int64_t)c * Bc;
            j.x0_off = 0;
            j.x_off = (int64_t)c * d.U;
            j.m = Bc;
            j.n = d.U;
            j.info_idx = c;
            j.pad = 0;
        }
        if (hipMemcpy(p->jobs, jobs.data(), sizeof(WgJob) * d.C, hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(p->ws);
            delete p;
            return CDM_EHIP;
        }
    } else {
        p->r0 = b + o_r0;
        p->M = b + o_M;
        p->gpart = b + o_gpart;
        p->part = b + o_part;
        p->gbuf = b + o_gbuf;
        p->e = (double*)(b + o_e);
        p->rpart = b + o_rpart;
    }
    p->res_rpart = (double*)(b + o_res_rpart);
    p->res_r = (double*)(b + o_res_r);
    p->res_col = (double*)(b + o_res_col);
    p->res_out = (double*)(b + o_res_out);

    char buf[512];
    if (engine == CDM_ENGINE_WG)
        snprintf(buf, sizeof(buf),
                 "{\"engine\": \"wg\", \"precision\": \"%s\", \"B\": %d, \"U\": %d, \"C\": %d, \"nt\": %d, "
                 "\"rpt\": %d, \"grid\": %d, \"lds\": %zu, \"workspace\": %zu}",
                 p->c128 ? "c128" : "c64", d.B, d.U, d.C, p->wg_nt, p->wg_rpt, p->wg_grid, p->wg_lds, p->ws_bytes);
    else
        snprintf(buf, sizeof(buf),
                 "{\"engine\": \"panel\", \"precision\": \"%s\", \"B\": %d, \"U\": %d, \"panel\": %d, \"rpl\": %d, "
                 "\"workgroups\": %d, \"npanels\": %d, \"gram_splits\": %d, \"workspace\": %zu}",
                 p->c128 ? "c128" : "c64", d.B, d.U, p->kp, p->rpl, p->P, p->npanels, p->nsplit, p->ws_bytes);
    p->text = buf;
    *plan = p;
    return CDM_OK;
}

static int32_t run_resid(cdm_plan* p, const void* H, int64_t ldh, const void* y, double lambda, const void* x,
                         double* out, hipStream_t st) {
    ResidLaunch R;
    R.c128 = p->c128;
    R.B = p->d.B;
    R.U = p->d.U;
    R.H = H;
    R.ld = ldh;
    R.y = y;
    R.x = x;
    R.rpart = p->res_rpart;
    R.nchunk = p->nchunk;
    R.r = p->res_r;
    R.colpart = p->res_col;
    R.lambda = lambda;
    R.out = out;
    HIP_TRY(launch_resid(R, st));
    return CDM_OK;
}

int32_t cdm_solve(cdm_plan* p, const void* H, int64_t ldh, const int32_t* rowptr, const int32_t* colidx,
                  const void* rhs, double N0, double Ex, double rho, const void* x0, void* x, void* info,
                  void* stream) {
    (void)rowptr;
    (void)colidx;
    (void)rho;
    if (!p || p->batched || !H || !rhs || !x || !info) return CDM_EINVAL;
    if (!(Ex > 0.0) || !(N0 >= 0.0) || !std::isfinite(N0) || !std::isfinite(Ex)) return CDM_EINVAL;
    const cdm_desc& d = p->d;
    if (ldh < d.B) return CDM_ESHAPE;
    const double lambda = N0 / Ex;
    const int Bc = d.B / d.C;
    if (lambda == 0.0 && Bc < d.U) return CDM_EINFEASIBLE;
    hipStream_t st = (hipStream_t)stream;
    cdm_info* inf = (cdm_info*)info;

    HIP_TRY(launch_zero_u32(p->ctr, 16, st));
    if (p->engine == CDM_ENGINE_WG) {
        WgLaunch L;
        L.c128 = p->c128;
        L.nt = p->wg_nt;
        L.rpt = p->wg_rpt;
        L.grid = p->wg_grid;
        L.n_max = p->n_max;
        L.jobs = p->jobs;
        L.njobs = d.C;
        L.order = nullptr;
        L.queue = p->ctr + 4;
        L.H = H;
        L.Y = rhs;
        L.X0 = x0;
        L.X = d.C > 1 ? p->xloc : x;
        L.info = inf;
        L.lambda = lambda;
        L.T_max = d.T_max;
        L.tol = d.tol;
        L.msum = d.C > 1 ? p->msum : nullptr;
        L.ld = ldh;
        HIP_TRY(launch_wg(L, st));
        if (d.C > 1) HIP_TRY(launch_fuse(p->c128, p->xloc, p->msum, d.C, d.U, N0, x, st));
    } else {
        GramLaunch G;
        G.c128 = p->c128;
        G.kp = p->kp;
        G.B = d.B;
        G.U = d.U;
        G.npanels = p->npanels;
        G.nsplit = p->nsplit;
        G.H = H;
        G.ld = ldh;
        G.gpart = p->gpart;
        G.M = p->M;
        G.e = p->e;
        G.status = p->ctr + 3;
        G.lambda = lambda;
        HIP_TRY(launch_gram(G, st));
        InitLaunch I;
        I.c128 = p->c128;
        I.B = d.B;
        I.U = d.U;
        I.H = H;
        I.ld = ldh;
        I.y = rhs;
        I.x0 = x0;
        I.r0 = p->r0;
        I.x = x;
        I.rpart = p->rpart;
        I.nchunk = p->nchunk;
        HIP_TRY(launch_init(I, st));
        PanelLaunch L;
        L.c128 = p->c128;
        L.kp = p->kp;
        L.rpl = p->rpl;
        L.P = p->P;
        L.B = d.B;
        L.U = d.U;
        L.npanels = p->npanels;
        L.H = H;
        L.ld = ldh;
        L.r0 = p->r0;
        L.x = x;
        L.M = p->M;
        L.part = p->part;
        L.gbuf = p->gbuf;
        L.ctr = p->ctr;
        L.info = inf;
        L.lambda = lambda;
        L.T_max = d.T_max;
        L.tol = d.tol;
        L.timeout_ticks = p->timeout_ticks;
        HIP_TRY(launch_panel(L, st));
        HIP_TRY(launch_finalize(x, d.U, p->c128, p->ctr + 2, inf, st));
    }
    if (d.flags & CDM_F_RESIDUAL) {
        int32_t s2 = run_resid(p, H, ldh, rhs, lambda, x, p->res_out, st);
        if (s2) return s2;
        HIP_TRY(launch_copy_resid(p->res_out, inf, 1, st));
    }
    return CDM_OK;
}

int32_t cdm_residual(cdm_plan* p, const void* H, int64_t ldh, const void* y, double N0, double Ex, const void* x,
                     double* out, void* stream) {
    if (!p || p->batched || !H || !y || !x || !out) return CDM_EINVAL;
    if (!(Ex > 0.0) || !(N0 >= 0.0)) return CDM_EINVAL;
    if (ldh < p->d.B) return CDM_ESHAPE;
    return run_resid(p, H, ldh, y, N0 / Ex, x, out, (hipStream_t)stream);
}

int32_t cdm_create_batched(const cdm_desc* desc, int32_t batch, const int32_t* m, const int32_t* n,
                           cdm_plan** plan) {
    if (!plan) return CDM_EINVAL;
    *plan = nullptr;
    int32_t st = validate_common(desc);
    if (st) return st;
    if (batch < 1 || !m || !n) return CDM_EINVAL;
    const cdm_desc& d = *desc;
    if (d.problem != CDM_UPLINK_LMMSE || d.layout != CDM_DENSE ||
        (d.precision != CDM_C128 && d.precision != CDM_C64))
        return CDM_ENOTIMPL;
    int m_max = 0, n_max = 0;
    for (int i = 0; i < batch; ++i) {
        if (m[i] < 1 || n[i] < 1 || m[i] > kWgMaxRows) return CDM_ESHAPE;
        m_max = std::max(m_max, m[i]);
        n_max = std::max(n_max, n[i]);
    }
    cdm_plan* p = new cdm_plan();
    p->d = d;
    p->batched = true;
    p->c128 = d.precision == CDM_C128;
    p->esz = p->c128 ? 16 : 8;
    st = device_setup(p);
    if (st) {
        delete p;
        return st;
    }
    p->engine = CDM_ENGINE_WG;
    st = setup_wg(p, m_max, n_max, batch);
    if (st) {
        delete p;
        return st;
    }
    p->H_off.resize(batch);
    p->y_off.resize(batch);
    p->x_off.resize(batch);
    std::vector<WgJob> jobs(batch);
    int64_t ho = 0, yo = 0, xo = 0;
    for (int i = 0; i < batch; ++i) {
        p->H_off[i] = ho;
        p->y_off[i] = yo;
        p->x_off[i] = xo;
        WgJob& j = jobs[i];
        j.h_off = ho;
        j.ld = m[i];
        j.y_off = yo;
        j.x0_off = xo;
        j.x_off = xo;
        j.m = m[i];
        j.n = n[i];
        j.info_idx = i;
        j.pad = 0;
        ho += (int64_t)m[i] * n[i];
        yo += m[i];
        xo += n[i];
    }
    // largest work first (longest-processing-time order), ties by index
    std::vector<int> order(batch);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return (int64_t)m[a] * n[a] > (int64_t)m[b] * n[b];
    });
    Arena ar;
    const size_t o_ctr = ar.take(64);
    const size_t o_jobs = ar.take(sizeof(WgJob) * batch);
    const size_t o_order = ar.take(sizeof(int) * batch);
    st = alloc_ws(p, ar.off);
    if (st) {
        delete p;
        return st;
    }
    p->ctr = (uint32_t*)(p->ws + o_ctr);
    p->jobs = (WgJob*)(p->ws + o_jobs);
    p->order = (int*)(p->ws + o_order);
    if (hipMemcpy(p->jobs, jobs.data(), sizeof(WgJob) * batch, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->order, order.data(), sizeof(int) * batch, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(p->ws);
        delete p;
        return CDM_EHIP;
    }
    char buf[512];
    snprintf(buf, sizeof(buf),
             "{\"engine\": \"wg-batched\", \"precision\": \"%s\", \"batch\": %d, \"m_max\": %d, \"n_max\": %d, "
             "\"nt\": %d, \"rpt\": %d, \"grid\": %d, \"lds\": %zu, \"workspace\": %zu}",
             p->c128 ? "c128" : "c64", batch, m_max, n_max, p->wg_nt, p->wg_rpt, p->wg_grid, p->wg_lds,
             p->ws_bytes);
    p->text = buf;
    *plan = p;
    return CDM_OK;
}

int32_t cdm_batched_offsets(const cdm_plan* p, int64_t* H_off, int64_t* y_off, int64_t* x_off) {
    if (!p || !p->batched) return CDM_EINVAL;
    const size_t n = p->H_off.size();
    if (H_off) std::memcpy(H_off, p->H_off.data(), n * sizeof(int64_t));
    if (y_off) std::memcpy(y_off, p->y_off.data(), n * sizeof(int64_t));
    if (x_off) std::memcpy(x_off, p->x_off.data(), n * sizeof(int64_t));
    return CDM_OK;
}

int32_t cdm_solve_batched(cdm_plan* p, const void* H, const void* y, double N0, double Ex, const void* x0, void* x,
                          void* info, void* stream) {
    if (!p || !p->batched || !H || !y || !x || !info) return CDM_EINVAL;
    if (!(Ex > 0.0) || !(N0 >= 0.0) || !std::isfinite(N0) || !std::isfinite(Ex)) return CDM_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(launch_zero_u32(p->ctr, 16, st));
    WgLaunch L;
    L.c128 = p->c128;
    L.nt = p->wg_nt;
    L.rpt = p->wg_rpt;
    L.grid = p->wg_grid;
    L.n_max = p->n_max;
    L.jobs = p->jobs;
    L.njobs = p->njobs;
    L.order = p->order;
    L.queue = p->ctr + 4;
    L.H = H;
    L.Y = y;
    L.X0 = x0;
    L.X = x;
    L.info = (cdm_info*)info;
    L.lambda = N0 / Ex;
    L.T_max = p->d.T_max;
    L.tol = p->d.tol;
    L.msum = nullptr;
    L.ld = 1;
    HIP_TRY(launch_wg(L, st));
    return CDM_OK;
}

int32_t cdm_plan_describe(const cdm_plan* p, char* buf, int32_t len) {
    if (!p || !buf || len < 1) return CDM_EINVAL;
    std::snprintf(buf, (size_t)len, "%s", p->text.c_str());
    return CDM_OK;
}

int32_t cdm_destroy(cdm_plan* p) {
    if (!p) return CDM_OK;
    if (p->ws) (void)hipFree(p->ws);
    delete p;
    return CDM_OK;
}

}  // extern "C"
