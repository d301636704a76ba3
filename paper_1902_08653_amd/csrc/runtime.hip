// runtime.hip -- the C ABI (include/cdm.h): plan creation, validation, workspace,
// engine choice and kernel dispatch.  Host code only; every numerical step runs
// in the kernels of k_wg.hip, k_panel.hip and k_aux.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
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
constexpr int kWgMixedMaxRows = 2048; // mixed-precision batched path: 256 threads x 8 rows
constexpr int kWgMixedInnerMax = 64;  // inner sweeps per outer step at most
constexpr double kWgMixedTauC64 = 1e-5;   // inner stop ||delta|| <= tau ||d||: complex64 copy
constexpr double kWgMixedTauBf16 = 3e-2;  // BF16 copy (its rounding bounds the outer gain per step)
constexpr int kCtrWords = 2048;       // control words: counters, abort/status, arrival flags
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
    int wg_nt = 256, wg_rpt = 1, wg_grid = 1, n_max = 1;   // wg_rpt: rows per thread of the largest job
    size_t wg_lds = 0;
    int wg_low = WG_LOW_NONE; // batched mixed precision: format of the inner copy
    void* wg_hq = nullptr;    // the inner copy (packed like H)
    int wg_inner_max = 0;
    double wg_tau = 0.0;
    void* bm_R = nullptr;     // FP64 residuals (packed like y)
    void* bm_G = nullptr;     // inner biases (packed like x)
    void* bm_CF = nullptr;    // inner scalars (packed like x)
    uint32_t* bm_done = nullptr;
    int njobs = 0;
    // PANEL engine
    int kp = 128, rpl = 1, P = 1, npanels = 1, nsplit = 1;
    bool la = false;          // look-ahead schedule (k_cd_panel_la)
    bool deep = false;        // its two-panel form (k_cd_panel_deep)
    void* X2 = nullptr;       // the latter's cross blocks H_K^H H_{K-2}
    size_t part_bytes = 0, gbuf_bytes = 0;
    void* X = nullptr;        // its cross blocks H_K^H H_{K-1}
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
    std::vector<int> bc;      // cluster sizes B_c (rows of each cluster, in order)
    int bc_min = 0, bc_max = 0;
    void* rpart = nullptr;    // warm-start product scratch
    int nchunk = 1;
    double* res_rpart = nullptr;
    double* res_r = nullptr;
    double* res_col = nullptr;
    double* res_out = nullptr;
    // mixed precision
    bool mixed = false;
    int src_kind = SRC_COMPLEX;
    uint16_t* q_re16 = nullptr;
    uint16_t* q_im16 = nullptr;
    uint8_t* q_re8 = nullptr;
    uint8_t* q_im8 = nullptr;
    float* q_scale = nullptr;
    double* colamax = nullptr;
    void* mx_r64 = nullptr;
    void* mx_g32 = nullptr;
    void* mx_d32 = nullptr;
    void* mx_r32 = nullptr;
    uint32_t* mx_done = nullptr;
    // sparse (CSR input)
    int32_t* sp_colptr = nullptr;
    int32_t* sp_fill = nullptr;
    int32_t* sp_rowidx = nullptr;
    void* sp_cval = nullptr;
    void* sp_r = nullptr;
    int32_t* sp_spt = nullptr;
    int32_t* sp_pi = nullptr;
    int32_t* sp_bcnt = nullptr;
    int32_t* sp_roff = nullptr;
    void* sp_xp = nullptr;
    uint64_t* sp_xbuf = nullptr;
    int sp_P = 1, sp_R = 1;
    // batched layout
    std::vector<int64_t> H_off, y_off, x_off;
    int64_t* xoff_dev = nullptr;
    int64_t total_n = 0;
    std::string text;
    // stage timing (CDM_F_TIMING)
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    bool timed = false;
};

static void ev_record(cdm_plan* p, int i, hipStream_t st) {
    if (p->timed) (void)hipEventRecord(p->ev[i], st);
}

static int32_t setup_timing(cdm_plan* p) {
    if (!(p->d.flags & CDM_F_TIMING)) return CDM_OK;
    for (int i = 0; i < 5; ++i)
        if (hipEventCreate(&p->ev[i]) != hipSuccess) return CDM_EHIP;
    p->timed = true;
    return CDM_OK;
}

static int32_t validate_common(const cdm_desc* d) {
    if (!d) return CDM_EINVAL;
    if (d->problem != CDM_UPLINK_LMMSE && d->problem != CDM_DOWNLINK_ZF) return CDM_EDTYPE;
    if (d->precision < CDM_C128 || d->precision > CDM_MIXED_C64) return CDM_EDTYPE;
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

// rows per thread for an instance of m rows on nt threads (0: too large); the
// mixed-precision kernel takes at most 4
static int rpt_for(int m, int nt, int cap = 8) {
    for (int r = 1; r <= cap; r *= 2)
        if ((int64_t)nt * r >= m) return r;
    return 0;
}

// threads per workgroup for single-instance (cluster) plans; the FP64 kernel is kept
// at <= 512 threads (its 8-rows-per-thread tile does not fit 1024-thread register budgets)
static int wg_nt_single(int m, bool c128) { return m <= 2048 ? 256 : (c128 ? 512 : 1024); }

static int32_t setup_wg(cdm_plan* p, int m_max, int n_max, int njobs, int nt) {
    const int cap = 8;
    if (rpt_for(m_max, nt, cap) == 0) return CDM_ESHAPE;
    p->wg_nt = nt;
    p->wg_rpt = rpt_for(m_max, nt, cap);
    p->n_max = std::max(1, n_max);
    p->wg_lds = p->wg_low ? bm_lds_bytes(p->n_max) : wg_lds_bytes(p->n_max, p->c128);
    if (p->wg_lds + 2048 > kLdsMax) return CDM_ESHAPE;
    if (p->wg_lds > 64 * 1024) {
        const hipError_t e = p->wg_low ? bm_set_lds_limit(p->wg_low, nt, p->wg_lds)
                                       : wg_set_lds_limit(p->c128, nt, p->wg_rpt, p->wg_lds);
        if (e != hipSuccess) return CDM_ESHAPE;
    }
    const int occ = std::max(1, p->wg_low ? bm_occupancy(p->wg_low, nt, p->wg_lds)
                                          : wg_occupancy(p->c128, nt, p->wg_rpt, p->wg_lds));
    p->wg_grid = std::max(1, std::min(njobs, occ * p->ncu));
    p->njobs = njobs;
    return CDM_OK;
}

extern "C" int32_t cdm_destroy(cdm_plan* p);

static constexpr int kSpKp = 64;

// Sparse plans: column-compressed copy, panel inverses and residual, all in one
// workspace sized from desc->nnz.
static int32_t create_sparse(cdm_plan* p, cdm_plan** plan) {
    const cdm_desc& d = p->d;
    p->engine = 3;
    p->kp = kSpKp;
    p->npanels = (d.U + kSpKp - 1) / kSpKp;
    const size_t nnz = (size_t)std::max<int64_t>(d.nnz, 1);
    const size_t ne = (size_t)kSpKp * (kSpKp + 1) / 2;
    Arena ar;
    const size_t o_ctr = ar.take(64);
    const size_t o_colptr = ar.take(4 * ((size_t)d.U + 1));
    const size_t o_fill = ar.take(4 * (size_t)d.U);
    const size_t o_rowidx = ar.take(4 * nnz);
    const size_t o_cval = ar.take(p->esz * nnz);
    const size_t o_r = ar.take(p->esz * (size_t)d.B);
    const size_t o_M = ar.take(p->esz * ne * p->npanels);
    const size_t o_gpart = ar.take(p->esz * 2 * (size_t)kSpKp * kSpKp * p->npanels);
    const size_t o_e = ar.take(8 * (size_t)d.U);
    sparse_slices(d.B, p->ncu, p->sp_P, p->sp_R);
    if (sparse_rows_per_thread(p->sp_R) == 0) {
        delete p;
        return CDM_ESHAPE;
    }
    const size_t o_spt = ar.take(4 * (size_t)(p->sp_P + 1) * d.U);
    const size_t o_pi = ar.take(4 * nnz);
    const size_t o_bcnt = ar.take(4 * (size_t)p->sp_P * p->npanels);
    const size_t o_roff = ar.take(4 * (size_t)p->sp_P * p->npanels * (p->sp_R + 1));
    const size_t o_xp = ar.take(p->esz * (size_t)p->sp_P * d.U);
    const size_t o_xbuf = ar.take(8 * (size_t)2 * p->sp_P * kSpKp * 4);
    int32_t st = alloc_ws(p, ar.off);
    if (st) {
        delete p;
        return st;
    }
    char* b = p->ws;
    p->ctr = (uint32_t*)(b + o_ctr);
    p->sp_colptr = (int32_t*)(b + o_colptr);
    p->sp_fill = (int32_t*)(b + o_fill);
    p->sp_rowidx = (int32_t*)(b + o_rowidx);
    p->sp_cval = b + o_cval;
    p->sp_r = b + o_r;
    p->M = b + o_M;
    p->gpart = b + o_gpart;
    p->e = (double*)(b + o_e);
    p->sp_spt = (int32_t*)(b + o_spt);
    p->sp_pi = (int32_t*)(b + o_pi);
    p->sp_bcnt = (int32_t*)(b + o_bcnt);
    p->sp_roff = (int32_t*)(b + o_roff);
    p->sp_xp = b + o_xp;
    p->sp_xbuf = (uint64_t*)(b + o_xbuf);
    char buf[512];
    snprintf(buf, sizeof(buf),
             "{\"engine\": \"sparse\", \"precision\": \"%s\", \"B\": %d, \"U\": %d, \"nnz\": %lld, \"panel\": %d, "
             "\"npanels\": %d, \"workgroups\": %d, \"slice_rows\": %d, \"workspace\": %zu}",
             p->c128 ? "c128" : "c64", d.B, d.U, (long long)d.nnz, kSpKp, p->npanels, p->sp_P, p->sp_R, p->ws_bytes);
    p->text = buf;
    st = setup_timing(p);
    if (st) {
        cdm_destroy(p);
        return st;
    }
    *plan = p;
    return CDM_OK;
}

static int32_t run_sparse(cdm_plan* p, const void* val, const int32_t* rowptr, const int32_t* colidx, const void* y,
                          double lambda, const void* x0, void* x, cdm_info* info, bool transpose_only,
                          hipStream_t st) {
    const cdm_desc& d = p->d;
    SparseLaunch L;
    L.c128 = p->c128;
    L.B = d.B;
    L.U = d.U;
    L.npanels = p->npanels;
    L.nnz = d.nnz;
    L.rowptr = rowptr;
    L.colidx = colidx;
    L.val = val;
    L.colptr = p->sp_colptr;
    L.fill = p->sp_fill;
    L.rowidx = p->sp_rowidx;
    L.cval = p->sp_cval;
    L.gpart = p->gpart;
    L.M = p->M;
    L.e = p->e;
    L.status = p->ctr + 3;
    L.y = y;
    L.x0 = x0;
    L.r = p->sp_r;
    L.x = x;
    L.info = info;
    L.lambda = lambda;
    L.T_max = d.T_max;
    L.tol = d.tol;
    L.transpose_only = transpose_only;
    L.P = p->sp_P;
    L.R = p->sp_R;
    L.spt = p->sp_spt;
    L.pi = p->sp_pi;
    L.bcnt = p->sp_bcnt;
    L.roff = p->sp_roff;
    L.xp = p->sp_xp;
    L.xbuf = p->sp_xbuf;
    L.abort_flag = p->ctr + 2;
    L.timeout_ticks = p->timeout_ticks;
    L.ev_sweep0 = p->timed ? p->ev[2] : nullptr;
    L.ev_sweep1 = p->timed ? p->ev[3] : nullptr;
    HIP_TRY(launch_zero_u32(p->ctr, 16, st));
    HIP_TRY(launch_sparse(L, st));
    return CDM_OK;
}

// low-precision CD sweeps per outer refinement step of a single mixed solve
static int inner_sweeps_for(int src_kind) {
    return src_kind == SRC_FP8 ? CDM_MIXED_INNER_SWEEPS_FP8 : CDM_MIXED_INNER_SWEEPS_BF16;
}

// The panel sweep launch.  The look-ahead schedule's exchange buffers carry sequence
// tags and start each launch cleared (a fill kernel, so the solve stays capturable).
static hipError_t launch_sweep(cdm_plan* p, const PanelLaunch& L, hipStream_t st) {
    if (!p->la) return launch_panel(L, st);
    hipError_t e = launch_zero_u32((uint32_t*)p->part, (int)(p->part_bytes / 4), st);
    if (e == hipSuccess) e = launch_zero_u32((uint32_t*)p->gbuf, (int)(p->gbuf_bytes / 4), st);
    if (e == hipSuccess) {
        if (p->deep) {
            PanelLaunch D = L;
            D.X2 = p->X2;
            e = launch_panel_deep(D, st);
        } else {
            e = launch_panel_la(L, st);
        }
    }
    return e;
}

static int32_t run_resid(cdm_plan* p, const void* H, int64_t ldh, const void* y, double lambda, const void* x,
                         double* out, hipStream_t st);

// Mixed precision: quantise H, Gram blocks of the quantised copy, then T_max outer
// FP64 steps (each a no-op once converged) around the FP32 panel engine.
static int32_t solve_mixed(cdm_plan* p, const void* H, int64_t ldh, const void* y, double lambda, const void* x0,
                           void* x, cdm_info* inf, hipStream_t st) {
    const cdm_desc& d = p->d;
    MixedLaunch M;
    M.src_kind = p->src_kind;
    M.B = d.B;
    M.U = d.U;
    M.H = H;
    M.ld = ldh;
    M.y = y;
    M.x0 = x0;
    M.x = x;
    M.q_re16 = p->q_re16;
    M.q_im16 = p->q_im16;
    M.q_re8 = p->q_re8;
    M.q_im8 = p->q_im8;
    M.q_scale = p->q_scale;
    M.colamax = p->colamax;
    M.rpart = p->rpart;
    M.nchunk = p->nchunk;
    M.r64 = p->mx_r64;
    M.g32 = p->mx_g32;
    M.d32 = p->mx_d32;
    M.r32 = p->mx_r32;
    M.ctr = p->ctr;
    M.nctr = kCtrWords;
    M.done = p->mx_done;
    M.info = inf;
    M.lambda = lambda;
    M.tol = d.tol;
    M.inner_sweeps = inner_sweeps_for(p->src_kind);
    ev_record(p, 0, st);
    HIP_TRY(launch_zero_u32(p->ctr, kCtrWords, st));
    HIP_TRY(launch_quantize(M, st));
    GramLaunch G;
    G.c128 = false;
    G.src_kind = p->src_kind;
    G.q_re16 = p->q_re16;
    G.q_im16 = p->q_im16;
    G.q_re8 = p->q_re8;
    G.q_im8 = p->q_im8;
    G.q_scale = p->q_scale;
    G.kp = p->kp;
    G.B = d.B;
    G.U = d.U;
    G.npanels = p->npanels;
    G.nsplit = p->nsplit;
    G.H = nullptr;
    G.ld = d.B;
    G.gpart = p->gpart;
    G.M = p->M;
    G.e = p->e;
    G.status = p->ctr + 3;
    G.lambda = lambda;
    HIP_TRY(launch_gram(G, st));
    if (p->la) HIP_TRY(launch_gram_cross(G, p->X, st));
    HIP_TRY(launch_mixed_start(M, st));
    ev_record(p, 1, st);
    ev_record(p, 2, st);
    PanelLaunch L;
    L.c128 = false;
    L.src_kind = p->src_kind;
    L.q_re16 = p->q_re16;
    L.q_im16 = p->q_im16;
    L.q_re8 = p->q_re8;
    L.q_im8 = p->q_im8;
    L.q_scale = p->q_scale;
    L.bias = p->mx_g32;
    L.done = p->mx_done;
    L.kp = p->kp;
    L.rpl = p->rpl;
    L.P = p->P;
    L.B = d.B;
    L.U = d.U;
    L.npanels = p->npanels;
    L.H = nullptr;
    L.ld = d.B;
    L.r0 = p->mx_r32;
    L.x = p->mx_d32;
    L.M = p->M;
    L.X = p->X;
    L.part = p->part;
    L.gbuf = p->gbuf;
    L.ctr = p->ctr;
    L.lambda = lambda;
    L.T_max = inner_sweeps_for(p->src_kind);
    L.tol = 0.0;
    L.timeout_ticks = p->timeout_ticks;
    L.info = (cdm_info*)((char*)p->mx_done + 32);   // the inner launches' own record (unused)
    for (int k = 0; k < d.T_max; ++k) {
        HIP_TRY(launch_mixed_outer_head(M, st));
        HIP_TRY(launch_sweep(p, L, st));
        HIP_TRY(launch_mixed_outer_tail(M, st));
    }
    HIP_TRY(launch_mixed_finish(M, st));
    ev_record(p, 3, st);
    if (d.flags & CDM_F_RESIDUAL) {   // as for the plain precisions: only when asked
        int32_t s2 = run_resid(p, H, ldh, y, lambda, x, p->res_out, st);
        if (s2) return s2;
        HIP_TRY(launch_copy_resid(p->res_out, inf, 1, st));
    }
    ev_record(p, 4, st);
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
    if (d.B < 1 || d.U < 1 || d.C < 1 || d.C > d.B) return CDM_ESHAPE;
    if (!d.Bc && d.B % d.C) return CDM_ESHAPE;
    // cluster sizes: C contiguous row blocks, B/C rows each or the caller's Bc[] (Sec. II-A)
    std::vector<int> bc(d.C, d.B / std::max(1, d.C));
    if (d.Bc) {
        int64_t sum = 0;
        for (int c = 0; c < d.C; ++c) {
            if (d.Bc[c] < 1) return CDM_ESHAPE;
            bc[c] = d.Bc[c];
            sum += d.Bc[c];
        }
        if (sum != d.B) return CDM_ESHAPE;
    }
    const int Bc = *std::max_element(bc.begin(), bc.end());      // the largest cluster
    const int Bc_min = *std::min_element(bc.begin(), bc.end());
    if (d.problem == CDM_DOWNLINK_ZF && Bc_min < d.U) return CDM_EINFEASIBLE;
    if (d.precision == CDM_MIXED_C64) return CDM_ENOTIMPL;   // batched plans only
    const bool mixed = d.precision == CDM_MIXED_BF16 || d.precision == CDM_MIXED_FP8;
    if (mixed && (d.problem != CDM_UPLINK_LMMSE || d.layout != CDM_DENSE || d.C != 1)) return CDM_ENOTIMPL;
    if (mixed && !(d.tol > 0.0)) return CDM_EINVAL;
    if (d.layout == CDM_CSR && (d.problem != CDM_UPLINK_LMMSE || d.C != 1)) return CDM_ENOTIMPL;
    if (d.layout == CDM_CSR && (d.nnz < 0 || d.nnz > 0x7fffffffLL)) return CDM_ESHAPE;
    if (d.problem == CDM_DOWNLINK_ZF &&
        (d.engine == CDM_ENGINE_PANEL || Bc > (d.precision == CDM_C128 ? kWgMaxRows / 2 : kWgMaxRows)))
        return CDM_ENOTIMPL;

    cdm_plan* p = new cdm_plan();
    p->d = d;
    p->d.Bc = nullptr;   // the sizes are kept in the plan, not the caller's array
    p->bc = bc;
    p->bc_min = Bc_min;
    p->bc_max = Bc;
    p->mixed = mixed;
    p->src_kind = d.precision == CDM_MIXED_BF16 ? SRC_BF16 : (d.precision == CDM_MIXED_FP8 ? SRC_FP8 : SRC_COMPLEX);
    p->c128 = d.precision == CDM_C128;      // mixed: the inner engine runs in FP32
    p->esz = p->c128 ? 16 : 8;
    st = device_setup(p);
    if (st) {
        delete p;
        return st;
    }

    if (d.layout == CDM_CSR) return create_sparse(p, plan);
    if (mixed && d.engine == CDM_ENGINE_WG) {
        delete p;
        return CDM_ENOTIMPL;
    }

    // engine choice: the panel engine (one cooperative launch, a workgroup per 64-row block)
    // for a single instance, unless it is narrow; the per-instance engine (one workgroup per
    // instance or cluster) otherwise.  Measured single-instance solves: the panel engine is
    // ahead from U = 128 at every B >= 256 (256 x 128 complex128: 3.4 against 5.7 ms; 2048 x
    // 512: 3.1 against 18.9 ms), behind at U = 64 up to B = 2048 (complex64 0.83 against 0.47
    // ms), and even or ahead from B * U = 2^18 at U = 64
    int engine = d.engine;
    const double elems = (double)d.B * d.U;
    if (engine == CDM_ENGINE_AUTO)
        engine = (d.C == 1 && d.B >= 256 && (d.U >= 128 || elems >= 262144.0)) ? CDM_ENGINE_PANEL : CDM_ENGINE_WG;
    if (mixed) engine = CDM_ENGINE_PANEL;
    if (d.problem == CDM_DOWNLINK_ZF) engine = CDM_ENGINE_WG;
    if (engine == CDM_ENGINE_PANEL && d.C != 1) engine = CDM_ENGINE_WG;
    if (engine == CDM_ENGINE_WG && Bc > (p->c128 ? kWgMaxRows / 2 : kWgMaxRows)) engine = CDM_ENGINE_PANEL;
    if (engine == CDM_ENGINE_PANEL && d.C != 1) {
        delete p;
        return CDM_ESHAPE;
    }
    p->engine = engine;

    Arena ar;
    const size_t o_ctr = ar.take(kCtrWords * 4);
    size_t o_jobs = 0, o_r0 = 0, o_M = 0, o_gpart = 0, o_part = 0, o_gbuf = 0, o_e = 0, o_xloc = 0,
           o_msum = 0, o_rpart = 0, o_X = 0, o_X2 = 0;
    p->nchunk = std::max(1, std::min(64, (d.U + 127) / 128));
    if (engine == CDM_ENGINE_WG) {
        st = setup_wg(p, Bc, d.U, d.C, wg_nt_single(Bc, p->c128));
        if (st) {
            delete p;
            return st;
        }
        o_jobs = ar.take(sizeof(WgJob) * d.C);
        if (d.C > 1 && d.problem == CDM_UPLINK_LMMSE) {
            o_xloc = ar.take(p->esz * (size_t)d.C * d.U);
            o_msum = ar.take(sizeof(double) * d.C);
        }
    } else {
        // panel width and rows per lane: one 64*rpl-row block per co-resident workgroup
        // (the packed panel inverse must fit in LDS next to the sweep's own buffers)
        static const int cand_c128[2][2] = {{128, 1}, {64, 2}};
        static const int cand_c64[2][2] = {{128, 1}, {128, 2}};
        const int(*cand)[2] = p->c128 ? cand_c128 : cand_c64;
        bool found = false;
        if (!(d.flags & CDM_F_NO_LOOKAHEAD)) {
            // look-ahead schedule: 64-row blocks, one reducer workgroup per panel column
            // 64-column panels with b formed locally (complex128, complex64); the mixed
            // path's FP32 inner solve over a 2- or 1-byte copy takes 128-column panels,
            // whose chain steps are as fast and half as many
            const int kp = mixed ? 128 : 64;
            const int P = (d.B + 63) / 64;
            if ((!d.panel || d.panel == kp) && P >= kp && P <= 256 && P <= panel_la_max_coresident(p->c128, kp) &&
                16 + P + kp <= kCtrWords) {
                p->kp = kp;
                p->rpl = 1;
                p->P = P;
                p->la = true;
                found = true;
            }
        }
        for (int i = 0; i < 2 && !found; ++i) {
            const int kp = cand[i][0], rpl = cand[i][1];
            if (d.panel && d.panel != kp) continue;
            const int P = (d.B + 64 * rpl - 1) / (64 * rpl);
            const int maxc = panel_max_coresident(p->c128, kp, rpl);
            if (P <= maxc && 16 + P + kp <= kCtrWords) {
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
        // complex128 64-column panels, at least three of them: the look-ahead of two panels
        p->deep = p->la && p->c128 && p->kp == 64 && p->npanels >= 3 && (d.flags & CDM_F_DEEP_LOOKAHEAD) &&
                  p->P <= panel_deep_max_coresident();
        const int nb = p->kp / 64;
        const int nsub = nb * (nb + 1) / 2;
        p->nsplit = std::max(1, std::min(32, (1024 + p->npanels * nsub - 1) / (p->npanels * nsub)));
        p->nsplit = std::min(p->nsplit, std::max(1, d.B / 256));
        const size_t kk = (size_t)p->kp * p->kp * p->npanels;
        o_r0 = ar.take(p->esz * d.B);
        o_M = ar.take(p->esz * kk);
        o_gpart = ar.take(p->esz * kk * std::max(2, p->nsplit));
        // the look-ahead schedule exchanges tagged words: twice the bytes per value (two
        // sequence slots); its two-panel form keeps DP_SLOTS slots
        const size_t slots = p->deep ? DP_SLOTS : 2;
        p->part_bytes = (p->la ? 2 : 1) * p->esz * slots * (size_t)p->kp * p->P;
        p->gbuf_bytes = (p->la ? 2 : 1) * p->esz * slots * (size_t)p->kp * 2;
        o_part = ar.take(p->part_bytes);
        o_gbuf = ar.take(p->gbuf_bytes);
        o_e = ar.take(sizeof(double) * d.U);
        o_rpart = ar.take(16 * (size_t)p->nchunk * d.B);
        if (p->la) o_X = ar.take(p->esz * kk);
        if (p->deep) o_X2 = ar.take(p->esz * kk);
    }
    size_t o_q1 = 0, o_q2 = 0, o_qs = 0, o_ca = 0, o_r64 = 0, o_g32 = 0, o_d32 = 0, o_r32 = 0, o_done = 0;
    if (mixed) {
        const size_t bu = (size_t)d.B * d.U;
        const size_t qb = p->src_kind == SRC_BF16 ? 2 : 1;
        o_q1 = ar.take(qb * bu);
        o_q2 = ar.take(qb * bu);
        o_qs = ar.take(4 * (size_t)((d.U + 127) / 128));
        o_ca = ar.take(8 * (size_t)d.U);
        o_r64 = ar.take(16 * (size_t)d.B);
        o_g32 = ar.take(8 * (size_t)d.U);
        o_d32 = ar.take(8 * (size_t)d.U);
        o_r32 = ar.take(8 * (size_t)d.B);
        o_done = ar.take(64);
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
        if (d.C > 1 && d.problem == CDM_UPLINK_LMMSE) {
            p->xloc = b + o_xloc;
            p->msum = (double*)(b + o_msum);
        }
        std::vector<WgJob> jobs(d.C);
        int64_t row0 = 0;
        for (int c = 0; c < d.C; ++c) {
            WgJob& j = jobs[c];
            j.h_off = row0;
            j.ld = 0;   // the solve's ldh
            const bool dl = d.problem == CDM_DOWNLINK_ZF;
            j.y_off = dl ? 0 : row0;        // downlink: s is broadcast to every cluster
            j.x0_off = 0;
            j.x_off = dl ? row0 : (int64_t)c * d.U;
            j.m = bc[c];
            j.n = d.U;
            j.info_idx = c;
            j.rpt = rpt_for(bc[c], p->wg_nt);
            row0 += bc[c];
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
        if (p->la) p->X = b + o_X;
        if (p->deep) p->X2 = b + o_X2;
    }
    if (mixed) {
        if (p->src_kind == SRC_BF16) {
            p->q_re16 = (uint16_t*)(b + o_q1);
            p->q_im16 = (uint16_t*)(b + o_q2);
        } else {
            p->q_re8 = (uint8_t*)(b + o_q1);
            p->q_im8 = (uint8_t*)(b + o_q2);
        }
        p->q_scale = (float*)(b + o_qs);
        p->colamax = (double*)(b + o_ca);
        p->mx_r64 = b + o_r64;
        p->mx_g32 = b + o_g32;
        p->mx_d32 = b + o_d32;
        p->mx_r32 = b + o_r32;
        p->mx_done = (uint32_t*)(b + o_done);
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
                 "{\"engine\": \"panel\", \"schedule\": \"%s\", \"lookahead_panels\": %d, \"precision\": \"%s\", "
                 "\"B\": %d, \"U\": %d, \"panel\": %d, \"rpl\": %d, \"workgroups\": %d, \"npanels\": %d, "
                 "\"gram_splits\": %d, \"inner_sweeps\": %d, \"workspace\": %zu}",
                 p->la ? "lookahead" : "two-hop", p->deep ? 2 : (p->la ? 1 : 0),
                 mixed ? (p->src_kind == SRC_BF16 ? "mixed-bf16" : "mixed-fp8") : (p->c128 ? "c128" : "c64"), d.B, d.U,
                 p->kp, p->rpl, p->P, p->npanels, p->nsplit, mixed ? inner_sweeps_for(p->src_kind) : 0, p->ws_bytes);
    p->text = buf;
    st = setup_timing(p);
    if (st) {
        cdm_destroy(p);
        return st;
    }
    *plan = p;
    return CDM_OK;
}

static int32_t run_resid(cdm_plan* p, const void* H, int64_t ldh, const void* y, double lambda, const void* x,
                         double* out, hipStream_t st) {
    ResidLaunch R;
    R.c128 = p->c128 || p->mixed;   // mixed plans take complex128 H, y, x
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
                  const void* rhs, double N0, double Ex, double rho, const void* x0, const double* lambda_c,
                  void* x, void* info, void* stream) {
    (void)rowptr;
    (void)colidx;
    (void)rho;
    if (!p || p->batched || !H || !rhs || !x || !info) return CDM_EINVAL;
    const cdm_desc& d = p->d;
    if (d.problem == CDM_UPLINK_LMMSE && (!(Ex > 0.0) || !(N0 >= 0.0) || !std::isfinite(N0) || !std::isfinite(Ex)))
        return CDM_EINVAL;
    if (d.layout == CDM_DENSE && ldh < d.B) return CDM_ESHAPE;
    const double lambda = N0 / Ex;
    if (lambda_c && (d.problem != CDM_UPLINK_LMMSE || d.C == 1)) return CDM_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    cdm_info* inf = (cdm_info*)info;
    if (d.problem == CDM_DOWNLINK_ZF) {
        if (x0) return CDM_EINVAL;
        ev_record(p, 0, st);
        HIP_TRY(launch_zero_u32(p->ctr, 16, st));
        ev_record(p, 1, st);
        ev_record(p, 2, st);
        WgLaunch L;
        L.c128 = p->c128;
        L.nt = p->wg_nt;
        L.rmax = p->wg_rpt;
        L.grid = p->wg_grid;
        L.n_max = p->n_max;
        L.jobs = p->jobs;
        L.njobs = d.C;
        L.order = nullptr;
        L.queue = p->ctr + 4;
        L.H = H;
        L.Y = rhs;
        L.X0 = nullptr;
        L.X = x;
        L.info = inf;
        L.lambda = 0.0;
        L.T_max = d.T_max;
        L.tol = d.tol;
        L.msum = nullptr;
        L.ld = ldh;
        L.rho_c = rho > 0.0 ? rho / std::sqrt((double)d.C) : 0.0;
        L.resid = 0;
        HIP_TRY(launch_zf(L, st));
        ev_record(p, 3, st);
        ev_record(p, 4, st);
        return CDM_OK;
    }
    if (lambda == 0.0 && p->bc_min < d.U) return CDM_EINFEASIBLE;
    if (d.layout == CDM_CSR) {
        if (!rowptr || !colidx) return CDM_EINVAL;
        ev_record(p, 0, st);
        ev_record(p, 1, st);
        int32_t s2 = run_sparse(p, H, rowptr, colidx, rhs, lambda, x0, x, inf, false, st);
        if (s2) return s2;
        HIP_TRY(launch_finalize(x, d.U, p->c128, p->ctr + 2, inf, st));
        ev_record(p, 4, st);
        return CDM_OK;
    }

    if (p->mixed) return solve_mixed(p, H, ldh, rhs, lambda, x0, x, inf, st);
    ev_record(p, 0, st);
    HIP_TRY(launch_zero_u32(p->ctr, p->engine == CDM_ENGINE_PANEL ? kCtrWords : 16, st));
    if (p->engine == CDM_ENGINE_WG) {
        ev_record(p, 1, st);
        ev_record(p, 2, st);
        WgLaunch L;
        L.c128 = p->c128;
        L.nt = p->wg_nt;
        L.rmax = p->wg_rpt;
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
        L.rho_c = 0.0;
        L.resid = 0;
        HIP_TRY(launch_wg(L, st));
        ev_record(p, 3, st);
        if (d.C > 1) HIP_TRY(launch_fuse(p->c128, p->xloc, p->msum, lambda_c, d.C, d.U, x, st));
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
        if (p->la) HIP_TRY(launch_gram_cross(G, p->X, st));
        if (p->deep) HIP_TRY(launch_gram_cross2(G, p->X2, st));
        ev_record(p, 1, st);
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
        ev_record(p, 2, st);
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
        L.X = p->X;
        L.part = p->part;
        L.gbuf = p->gbuf;
        L.ctr = p->ctr;
        L.info = inf;
        L.lambda = lambda;
        L.T_max = d.T_max;
        L.tol = d.tol;
        L.timeout_ticks = p->timeout_ticks;
        HIP_TRY(launch_sweep(p, L, st));
        ev_record(p, 3, st);
        HIP_TRY(launch_finalize(x, d.U, p->c128, p->ctr + 2, inf, st));
    }
    if (d.flags & CDM_F_RESIDUAL) {
        int32_t s2 = run_resid(p, H, ldh, rhs, lambda, x, p->res_out, st);
        if (s2) return s2;
        HIP_TRY(launch_copy_resid(p->res_out, inf, 1, st));
    }
    ev_record(p, 4, st);
    return CDM_OK;
}

int32_t cdm_csr_transpose(cdm_plan* p, const void* val, const int32_t* rowptr, const int32_t* colidx,
                          int32_t* colptr_out, int32_t* rowidx_out, void* cval_out, void* stream) {
    if (!p || p->d.layout != CDM_CSR || !val || !rowptr || !colidx) return CDM_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    int32_t s2 = run_sparse(p, val, rowptr, colidx, nullptr, 0.0, nullptr, nullptr, nullptr, true, st);
    if (s2) return s2;
    const size_t nnz = (size_t)p->d.nnz;
    if (colptr_out)
        HIP_TRY(hipMemcpyAsync(colptr_out, p->sp_colptr, 4 * ((size_t)p->d.U + 1), hipMemcpyDeviceToDevice, st));
    if (rowidx_out && nnz) HIP_TRY(hipMemcpyAsync(rowidx_out, p->sp_rowidx, 4 * nnz, hipMemcpyDeviceToDevice, st));
    if (cval_out && nnz) HIP_TRY(hipMemcpyAsync(cval_out, p->sp_cval, p->esz * nnz, hipMemcpyDeviceToDevice, st));
    uint32_t status = 0;
    HIP_TRY(hipMemcpyAsync(&status, p->ctr + 3, 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return (status & CDM_INFO_BAD_INPUT) ? CDM_EINVAL : CDM_OK;
}

int32_t cdm_quantized_copy(cdm_plan* p, const void* H, int64_t ldh, void* re_out, void* im_out, float* scale_out,
                           void* stream) {
    if (!p || !p->mixed || !H) return CDM_EINVAL;
    if (ldh < p->d.B) return CDM_ESHAPE;
    hipStream_t st = (hipStream_t)stream;
    MixedLaunch M{};
    M.src_kind = p->src_kind;
    M.B = p->d.B;
    M.U = p->d.U;
    M.H = H;
    M.ld = ldh;
    M.q_re16 = p->q_re16;
    M.q_im16 = p->q_im16;
    M.q_re8 = p->q_re8;
    M.q_im8 = p->q_im8;
    M.q_scale = p->q_scale;
    M.colamax = p->colamax;
    HIP_TRY(launch_quantize(M, st));
    const size_t n = (size_t)p->d.B * p->d.U * (p->src_kind == SRC_BF16 ? 2 : 1);
    const void* qr = p->src_kind == SRC_BF16 ? (const void*)p->q_re16 : (const void*)p->q_re8;
    const void* qi = p->src_kind == SRC_BF16 ? (const void*)p->q_im16 : (const void*)p->q_im8;
    if (re_out) HIP_TRY(hipMemcpyAsync(re_out, qr, n, hipMemcpyDeviceToDevice, st));
    if (im_out) HIP_TRY(hipMemcpyAsync(im_out, qi, n, hipMemcpyDeviceToDevice, st));
    if (scale_out && p->src_kind == SRC_FP8)
        HIP_TRY(hipMemcpyAsync(scale_out, p->q_scale, 4 * (size_t)((p->d.U + 127) / 128), hipMemcpyDeviceToDevice, st));
    return CDM_OK;
}

int32_t cdm_residual(cdm_plan* p, const void* H, int64_t ldh, const void* y, double N0, double Ex, const void* x,
                     double* out, void* stream) {
    if (!p || p->batched || !H || !y || !x || !out) return CDM_EINVAL;
    if (!(Ex > 0.0) || !(N0 >= 0.0)) return CDM_EINVAL;
    if (ldh < p->d.B) return CDM_ESHAPE;
    return run_resid(p, H, ldh, y, N0 / Ex, x, out, (hipStream_t)stream);
}

// Time one persistent launch of the batched engine with nt threads per workgroup
// on `jobs` (device), 2 fixed sweeps; returns milliseconds (< 0 on failure).
static double time_batched(cdm_plan* p, int nt, int m_max, int n_max, WgJob* jobs_d, const std::vector<WgJob>& jobs,
                           int* order_d, void* H, void* Y, void* X, cdm_info* info, uint32_t* ctr, void* Hq,
                           void* mscratch) {
    const int njobs = (int)jobs.size();
    std::vector<WgJob> jj = jobs;
    for (auto& j : jj) j.rpt = rpt_for(j.m, nt);
    if (hipMemcpy(jobs_d, jj.data(), sizeof(WgJob) * njobs, hipMemcpyHostToDevice) != hipSuccess) return -1.0;
    const bool mx = p->wg_low != WG_LOW_NONE;
    const size_t lds = mx ? bm_lds_bytes(std::max(1, n_max)) : wg_lds_bytes(std::max(1, n_max), p->c128);
    const int rmax = rpt_for(m_max, nt);
    if (lds > 64 * 1024 &&
        (mx ? bm_set_lds_limit(p->wg_low, nt, lds) : wg_set_lds_limit(p->c128, nt, rmax, lds)) != hipSuccess)
        return -1.0;
    const int occ = std::max(1, mx ? bm_occupancy(p->wg_low, nt, lds) : wg_occupancy(p->c128, nt, rmax, lds));
    WgLaunch L;
    L.c128 = p->c128;
    L.nt = nt;
    L.rmax = rmax;
    L.grid = std::max(1, std::min(njobs, occ * p->ncu));
    L.n_max = std::max(1, n_max);
    L.jobs = jobs_d;
    L.njobs = njobs;
    L.order = order_d;
    L.queue = ctr + 4;
    L.H = H;
    L.Y = Y;
    L.X0 = nullptr;
    L.X = X;
    L.info = info;
    L.lambda = 0.1;
    L.T_max = 2;
    L.tol = 0.0;
    L.msum = nullptr;
    L.ld = 1;
    L.rho_c = 0.0;
    L.resid = 0;
    // mixed: one cold outer step with a fixed count of inner sweeps (tol = tau = 0);
    // its buffers follow the sample's own packing (scratch holds R, G, CF, done)
    BmLaunch M{};
    if (mx) {
        const int64_t sy = jobs.back().y_off + jobs.back().m, sx = jobs.back().x_off + jobs.back().n;
        char* sc = (char*)mscratch;
        M.low = p->wg_low;
        M.nt = nt;
        M.grid = L.grid;
        M.n_max = L.n_max;
        M.jobs = jobs_d;
        M.njobs = njobs;
        M.order = order_d;
        M.queue = ctr + 4;
        M.x_off = (const int64_t*)sc;
        M.total_n = sx;
        M.H = H;
        M.Y = Y;
        M.X0 = nullptr;
        M.X = X;
        M.Hq = Hq;
        M.R = sc + align256(8 * (size_t)njobs);
        M.G = (char*)M.R + align256(16 * (size_t)sy);
        M.CF = (char*)M.G + align256(8 * (size_t)sx);
        M.done = (uint32_t*)((char*)M.CF + align256(8 * (size_t)sx));
        M.info = info;
        M.lambda = 0.1;
        M.tol = 0.0;
        M.inner_max = 8;
        M.tau = 0.0;
    }
    (void)m_max;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1.0;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1.0;
    }
    double best = -1.0;
    for (int rep = 0; rep < 3; ++rep) {
        if (launch_zero_u32(ctr, 16, nullptr) != hipSuccess) break;
        (void)hipEventRecord(e0, nullptr);
        const hipError_t le = mx ? (launch_bm_init(M, nullptr) == hipSuccess ? launch_bm_step(M, 1, 0, nullptr)
                                                                              : hipErrorUnknown)
                                 : launch_wg(L, nullptr);
        if (le != hipSuccess) break;
        (void)hipEventRecord(e1, nullptr);
        if (hipEventSynchronize(e1) != hipSuccess) break;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0 && (best < 0 || ms < best)) best = ms;   // first run warms up
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

int32_t cdm_create_batched(const cdm_desc* desc, int32_t batch, const int32_t* m, const int32_t* n,
                           cdm_plan** plan) {
    if (!plan) return CDM_EINVAL;
    *plan = nullptr;
    int32_t st = validate_common(desc);
    if (st) return st;
    if (batch < 1 || !m || !n) return CDM_EINVAL;
    if (desc->Bc || desc->C != 1) return CDM_ENOTIMPL;   // one cluster per batch entry
    const cdm_desc& d = *desc;
    const int low = d.precision == CDM_MIXED_C64 ? WG_LOW_C64 : (d.precision == CDM_MIXED_BF16 ? WG_LOW_BF16 : 0);
    if (d.problem != CDM_UPLINK_LMMSE || d.layout != CDM_DENSE ||
        (d.precision != CDM_C128 && d.precision != CDM_C64 && !low))
        return CDM_ENOTIMPL;
    if (low && !(d.tol > 0.0)) return CDM_EINVAL;
    const int rows_cap = low ? kWgMixedMaxRows : kWgMaxRows;
    int m_max = 0, n_max = 0;
    int64_t total_mn = 0;
    for (int i = 0; i < batch; ++i) {
        if (m[i] < 1 || n[i] < 1 || m[i] > rows_cap) return CDM_ESHAPE;
        m_max = std::max(m_max, m[i]);
        n_max = std::max(n_max, n[i]);
        total_mn += (int64_t)m[i] * n[i];
    }
    cdm_plan* p = new cdm_plan();
    p->d = d;
    p->batched = true;
    p->c128 = d.precision != CDM_C64;   // mixed plans keep H, y and x in complex128
    p->esz = p->c128 ? 16 : 8;
    p->wg_low = low;
    p->wg_inner_max = kWgMixedInnerMax;
    p->wg_tau = low == WG_LOW_BF16 ? kWgMixedTauBf16 : kWgMixedTauC64;
    st = device_setup(p);
    if (st) {
        delete p;
        return st;
    }
    p->engine = CDM_ENGINE_WG;
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
        j.rpt = 0;
        ho += (int64_t)m[i] * n[i];
        yo += m[i];
        xo += n[i];
    }
    p->total_n = xo;
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
    const size_t o_xoff = ar.take(sizeof(int64_t) * batch);
    const size_t lowsz = low == WG_LOW_C64 ? 8 : 4;
    const size_t o_hq = low ? ar.take(lowsz * (size_t)total_mn) : 0;
    int64_t total_m = 0;
    for (int i = 0; i < batch; ++i) total_m += m[i];
    const size_t o_R = low ? ar.take(16 * (size_t)total_m) : 0;
    const size_t o_G = low ? ar.take(8 * (size_t)xo) : 0;
    const size_t o_CF = low ? ar.take(8 * (size_t)xo) : 0;
    const size_t o_done = low ? ar.take(4 * (size_t)batch) : 0;
    st = alloc_ws(p, ar.off);
    if (st) {
        delete p;
        return st;
    }
    p->ctr = (uint32_t*)(p->ws + o_ctr);
    p->jobs = (WgJob*)(p->ws + o_jobs);
    p->order = (int*)(p->ws + o_order);
    p->xoff_dev = (int64_t*)(p->ws + o_xoff);
    if (low) {
        p->wg_hq = p->ws + o_hq;
        p->bm_R = p->ws + o_R;
        p->bm_G = p->ws + o_G;
        p->bm_CF = p->ws + o_CF;
        p->bm_done = (uint32_t*)(p->ws + o_done);
    }
    if (hipMemcpy(p->xoff_dev, p->x_off.data(), sizeof(int64_t) * batch, hipMemcpyHostToDevice) != hipSuccess) {
        cdm_destroy(p);
        return CDM_EHIP;
    }

    // ---- tile choice: threads per workgroup for the whole launch; rows per
    // thread then follow per job.  With CDM_F_AUTOTUNE each candidate is timed
    // on a spread sample of this batch's shapes (synthetic values).
    static const int cands[3] = {128, 256, 512};   // the mixed kernel is built for these three
    int nt = 0;
    std::string tune = "null";
    if (d.flags & CDM_F_AUTOTUNE) {
        const int S = std::min(batch, 1024);
        std::vector<WgJob> sj(S);
        std::vector<int> sorder(S);
        int64_t sh = 0, sy = 0, sx = 0;
        int sm_max = 0, sn_max = 0;
        for (int k = 0; k < S; ++k) {
            const int i = order[(int64_t)k * batch / S];   // spread over the LPT order
            WgJob j = jobs[i];
            j.h_off = sh;
            j.ld = j.m;
            j.y_off = sy;
            j.x0_off = sx;
            j.x_off = sx;
            j.info_idx = k;
            sj[k] = j;
            sorder[k] = k;
            sh += (int64_t)j.m * j.n;
            sy += j.m;
            sx += j.n;
            sm_max = std::max(sm_max, j.m);
            sn_max = std::max(sn_max, j.n);
        }
        void *Hs = nullptr, *Ys = nullptr, *Xs = nullptr, *aux = nullptr, *Hqs = nullptr, *Ms = nullptr;
        // mixed: packed x offsets, then R, G, CF and done flags of the sample
        const size_t ms_bytes = align256(8 * (size_t)S) + align256(16 * (size_t)sy) + 2 * align256(8 * (size_t)sx) +
                                align256(4 * (size_t)S);
        bool ok = hipMalloc(&Hs, p->esz * (size_t)sh) == hipSuccess && hipMalloc(&Ys, p->esz * (size_t)sy) == hipSuccess &&
                  hipMalloc(&Xs, p->esz * (size_t)sx) == hipSuccess &&
                  (!low || (hipMalloc(&Hqs, lowsz * (size_t)sh) == hipSuccess &&
                            hipMalloc(&Ms, ms_bytes) == hipSuccess)) &&
                  hipMalloc(&aux, 64 + sizeof(cdm_info) * S + sizeof(WgJob) * S + sizeof(int) * S) == hipSuccess;
        if (ok) {
            uint32_t* tctr = (uint32_t*)aux;
            cdm_info* tinfo = (cdm_info*)((char*)aux + 64);
            WgJob* tjobs = (WgJob*)((char*)tinfo + sizeof(cdm_info) * S);
            int* tord = (int*)((char*)tjobs + sizeof(WgJob) * S);
            ok = hipMemcpy(tord, sorder.data(), sizeof(int) * S, hipMemcpyHostToDevice) == hipSuccess &&
                 launch_fill_hash(Hs, (int64_t)sh * 2, p->c128, 0x9e3779b9u, 1.0 / std::sqrt((double)sm_max)) == hipSuccess &&
                 launch_fill_hash(Ys, (int64_t)sy * 2, p->c128, 0x7f4a7c15u, 1.0) == hipSuccess;
            if (ok && Ms) {
                std::vector<int64_t> sxo(S);
                for (int k = 0; k < S; ++k) sxo[k] = sj[k].x_off;
                ok = hipMemcpy(Ms, sxo.data(), sizeof(int64_t) * S, hipMemcpyHostToDevice) == hipSuccess;
            }
            double best = -1.0;
            char tb[256];
            int tl = snprintf(tb, sizeof(tb), "{");
            for (int c = 0; ok && c < 3; ++c) {
                if (rpt_for(m_max, cands[c]) == 0) continue;
                const double ms = time_batched(p, cands[c], sm_max, sn_max, tjobs, sj, tord, Hs, Ys, Xs, tinfo, tctr, Hqs,
                                               Ms);
                tl += snprintf(tb + tl, sizeof(tb) - tl, "%s\"%d\": %.3f", tl > 1 ? ", " : "", cands[c], ms);
                if (ms > 0 && (best < 0 || ms < best)) {
                    best = ms;
                    nt = cands[c];
                }
            }
            snprintf(tb + tl, sizeof(tb) - tl, "}");
            tune = tb;
        }
        if (Hs) (void)hipFree(Hs);
        if (Ys) (void)hipFree(Ys);
        if (Xs) (void)hipFree(Xs);
        if (aux) (void)hipFree(aux);
        if (Hqs) (void)hipFree(Hqs);
        if (Ms) (void)hipFree(Ms);
        (void)hipGetLastError();
    }
    if (nt == 0) nt = rpt_for(m_max, 256) ? 256 : (rpt_for(m_max, 512) ? 512 : 1024);
    st = setup_wg(p, m_max, n_max, batch, nt);
    if (st) {
        cdm_destroy(p);
        return st;
    }
    for (auto& j : jobs) j.rpt = rpt_for(j.m, nt);
    if (hipMemcpy(p->jobs, jobs.data(), sizeof(WgJob) * batch, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->order, order.data(), sizeof(int) * batch, hipMemcpyHostToDevice) != hipSuccess) {
        cdm_destroy(p);
        return CDM_EHIP;
    }
    char buf[768];
    const char* pname = low == WG_LOW_C64 ? "mixed-c64" : (low == WG_LOW_BF16 ? "mixed-bf16" : (p->c128 ? "c128" : "c64"));
    char mx[160] = "";
    if (low)
        snprintf(mx, sizeof(mx), ", \"inner_max\": %d, \"inner_tau\": %g, \"inner_copy_bytes\": %zu",
                 p->wg_inner_max, p->wg_tau, lowsz * (size_t)total_mn);
    snprintf(buf, sizeof(buf),
             "{\"engine\": \"%s\", \"precision\": \"%s\", \"batch\": %d, \"m_max\": %d, \"n_max\": %d, "
             "\"nt\": %d, \"grid\": %d, \"lds\": %zu, \"workspace\": %zu, \"autotune_ms\": %s%s}",
             low ? "wg-batched-mixed" : "wg-batched", pname, batch, m_max, n_max, p->wg_nt, p->wg_grid, p->wg_lds,
             p->ws_bytes, tune.c_str(), mx);
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
    L.rmax = p->wg_rpt;
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
    L.rho_c = 0.0;
    L.resid = (p->d.flags & CDM_F_RESIDUAL) ? 1 : 0;
    if (p->wg_low) {
        BmLaunch M{};
        M.low = p->wg_low;
        M.nt = p->wg_nt;
        M.grid = p->wg_grid;
        M.n_max = p->n_max;
        M.jobs = p->jobs;
        M.njobs = p->njobs;
        M.order = p->order;
        M.queue = p->ctr + 4;
        M.x_off = p->xoff_dev;
        M.total_n = p->total_n;
        M.H = H;
        M.Y = y;
        M.X0 = x0;
        M.X = x;
        M.Hq = p->wg_hq;
        M.R = p->bm_R;
        M.G = p->bm_G;
        M.CF = p->bm_CF;
        M.done = p->bm_done;
        M.info = (cdm_info*)info;
        M.lambda = N0 / Ex;
        M.tol = p->d.tol;
        M.inner_max = p->wg_inner_max;
        M.tau = p->wg_tau;
        HIP_TRY(launch_bm_init(M, st));
        for (int s = 1; s <= p->d.T_max; ++s) HIP_TRY(launch_bm_step(M, s, s == p->d.T_max, st));
        if (L.resid) HIP_TRY(launch_bm_resid_check(M, st));
    } else {
        HIP_TRY(launch_wg(L, st));
    }
    return CDM_OK;
}

int32_t cdm_batched_features(cdm_plan* p, const void* H, const void* y, double N0, double Ex, float* F, void* stream) {
    if (!p || !p->batched || !H || !y || !F) return CDM_EINVAL;
    if (!(Ex > 0.0) || !(N0 >= 0.0)) return CDM_EINVAL;
    const int64_t rows = p->total_n;
    HIP_TRY(launch_features(p->c128, H, y, p->jobs, p->xoff_dev, p->njobs, rows, N0 / Ex, F, (hipStream_t)stream));
    return CDM_OK;
}

int32_t cdm_plan_describe(const cdm_plan* p, char* buf, int32_t len) {
    if (!p || !buf || len < 1) return CDM_EINVAL;
    std::snprintf(buf, (size_t)len, "%s", p->text.c_str());
    return CDM_OK;
}

int32_t cdm_plan_timings(const cdm_plan* p, double* out_ms, int32_t n, int32_t* count) {
    if (!p || !out_ms || !count || !p->timed) return CDM_EINVAL;
    int k = 0;
    for (int i = 0; i < 4 && k < n; ++i, ++k) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, p->ev[i], p->ev[i + 1]));
        out_ms[k] = ms;
    }
    *count = k;
    return CDM_OK;
}

int32_t cdm_stream_copy(const void* src, void* dst, int64_t bytes, void* stream) {
    if (!src || !dst || bytes < 0 || (bytes & 15)) return CDM_EINVAL;
    HIP_TRY(launch_stream_copy(src, dst, bytes, (hipStream_t)stream));
    return CDM_OK;
}

int32_t cdm_stream_read(const void* src, int64_t bytes, void* out, void* stream) {
    if (!src || !out || bytes < 0 || (bytes & 15)) return CDM_EINVAL;
    HIP_TRY(launch_stream_read(src, bytes, out, (hipStream_t)stream));
    return CDM_OK;
}

int32_t cdm_destroy(cdm_plan* p) {
    if (!p) return CDM_OK;
    for (int i = 0; i < 5; ++i)
        if (p->ev[i]) (void)hipEventDestroy(p->ev[i]);
    if (p->ws) (void)hipFree(p->ws);
    delete p;
    return CDM_OK;
}

}  // extern "C"

// ---- the entry point that allocates nothing ------------------------------------------
// cdm_solve_noalloc runs the per-cluster (one workgroup per cluster) solve with every
// buffer beyond the caller's inputs and outputs in `scratch`, a file-scope device array
// of fixed size: the queue and status words, the job records, and (uplink, C > 1) the
// local estimates and the sums of m_u,c that the fusion reads.  Each device holds its
// own copy of the array until the process ends; host code uses the address that
// hipGetSymbolAddress returns for the current device, never the array's name.
namespace {

constexpr size_t kNaBytes = CDM_NOALLOC_SCRATCH_BYTES;
constexpr size_t kNaCtr = 0;          // 64 control words (queue counter, status)
constexpr size_t kNaJobs = 256;       // CDM_NOALLOC_MAX_CLUSTERS job records
constexpr size_t kNaMsum = 4096;      // one double per cluster
constexpr size_t kNaXloc = 8192;      // C x U local estimates
static_assert(kNaJobs + sizeof(WgJob) * CDM_NOALLOC_MAX_CLUSTERS <= kNaMsum, "job records overlap");
static_assert(kNaMsum + 8 * CDM_NOALLOC_MAX_CLUSTERS <= kNaXloc, "cluster sums overlap");

__device__ __align__(256) unsigned char scratch[kNaBytes];

constexpr int kNaMaxDev = 64;
void* g_na_ptr[kNaMaxDev] = {};
int g_na_ncu[kNaMaxDev] = {};
std::mutex g_na_mu;

// The device's scratch address and CU count, set up once per device with it current.
int32_t na_device(int dev, char** ptr, int* ncu) {
    if (dev < 0 || dev >= kNaMaxDev) return CDM_ENODEV;
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (!g_na_ptr[dev]) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return CDM_ENODEV;
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
            snprintf(g_last_error, sizeof(g_last_error), "device %d is %s, this library is built for gfx950", dev,
                     prop.gcnArchName);
            return CDM_ENODEV;
        }
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_err("hipGetSymbolAddress(scratch)", e);
            return CDM_EHIP;
        }
        g_na_ncu[dev] = prop.multiProcessorCount;
        g_na_ptr[dev] = p;
    }
    *ptr = (char*)g_na_ptr[dev];
    *ncu = g_na_ncu[dev];
    return CDM_OK;
}

// Job records of the C clusters (contiguous row blocks), written on the device so that
// the solve issues no host-to-device copy.
struct NaJobsArg {
    int C, U, downlink;
    int32_t m[CDM_NOALLOC_MAX_CLUSTERS];
    int32_t rpt[CDM_NOALLOC_MAX_CLUSTERS];
    int64_t row0[CDM_NOALLOC_MAX_CLUSTERS];
};
__global__ void k_na_jobs(NaJobsArg a, WgJob* jobs) {
    const int c = threadIdx.x;
    if (c >= a.C) return;
    WgJob j;
    j.h_off = a.row0[c];
    j.ld = 0;
    j.y_off = a.downlink ? 0 : a.row0[c];
    j.x0_off = 0;
    j.x_off = a.downlink ? a.row0[c] : (int64_t)c * a.U;
    j.m = a.m[c];
    j.n = a.U;
    j.info_idx = c;
    j.rpt = a.rpt[c];
    jobs[c] = j;
}

}  // namespace

extern "C" int32_t cdm_solve_noalloc(const cdm_desc* desc, const void* H, int64_t ldh, const void* rhs, double N0,
                                     double Ex, double rho, const void* x0, const double* lambda_c, void* x,
                                     void* info, void* stream) {
    int32_t st0 = validate_common(desc);
    if (st0) return st0;
    const cdm_desc& d = *desc;
    if (!H || !rhs || !x || !info) return CDM_EINVAL;
    if (d.layout != CDM_DENSE || (d.precision != CDM_C128 && d.precision != CDM_C64)) return CDM_EDTYPE;
    if (d.engine == CDM_ENGINE_PANEL) return CDM_ENOTIMPL;
    const bool dl = d.problem == CDM_DOWNLINK_ZF;
    if (d.B < 1 || d.U < 1 || d.C < 1 || d.C > d.B) return CDM_ESHAPE;
    if (!d.Bc && d.B % d.C) return CDM_ESHAPE;
    if (ldh < d.B) return CDM_ESHAPE;
    if (dl && (x0 || lambda_c)) return CDM_EINVAL;
    if (lambda_c && d.C == 1) return CDM_EINVAL;
    if (!dl && (!(Ex > 0.0) || !(N0 >= 0.0) || !std::isfinite(N0) || !std::isfinite(Ex))) return CDM_EINVAL;
    const bool c128 = d.precision == CDM_C128;
    const size_t esz = c128 ? 16 : 8;
    if (d.C > CDM_NOALLOC_MAX_CLUSTERS ||
        (!dl && d.C > 1 && kNaXloc + esz * (size_t)d.C * d.U > kNaBytes)) {
        snprintf(g_last_error, sizeof(g_last_error),
                 "cdm_solve_noalloc: C = %d clusters x U = %d users exceed the static scratch (%d clusters, %zu bytes)",
                 d.C, d.U, CDM_NOALLOC_MAX_CLUSTERS, kNaBytes);
        return CDM_ESHAPE;
    }
    NaJobsArg ja;
    ja.C = d.C;
    ja.U = d.U;
    ja.downlink = dl ? 1 : 0;
    int bc_min = d.B, bc_max = 0;
    int64_t row0 = 0;
    for (int c = 0; c < d.C; ++c) {
        const int m = d.Bc ? d.Bc[c] : d.B / d.C;
        if (m < 1) return CDM_ESHAPE;
        ja.m[c] = m;
        ja.row0[c] = row0;
        row0 += m;
        bc_min = std::min(bc_min, m);
        bc_max = std::max(bc_max, m);
    }
    if (row0 != d.B) return CDM_ESHAPE;
    if (dl && bc_min < d.U) return CDM_EINFEASIBLE;
    const double lambda = dl ? 0.0 : N0 / Ex;
    if (!dl && lambda == 0.0 && bc_min < d.U) return CDM_EINFEASIBLE;
    if (bc_max > (c128 ? kWgMaxRows / 2 : kWgMaxRows)) return CDM_ESHAPE;   // one workgroup per cluster
    const int nt = wg_nt_single(bc_max, c128);
    const int rmax = rpt_for(bc_max, nt);
    if (rmax == 0) return CDM_ESHAPE;
    for (int c = 0; c < d.C; ++c) ja.rpt[c] = rpt_for(ja.m[c], nt);
    const size_t lds = wg_lds_bytes(d.U, c128);
    if (lds + 2048 > kLdsMax) return CDM_ESHAPE;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return CDM_ENODEV;
    char* sp = nullptr;
    int ncu = 0;
    int32_t st1 = na_device(dev, &sp, &ncu);
    if (st1) return st1;
    if (lds > 64 * 1024 && wg_set_lds_limit(c128, nt, rmax, lds) != hipSuccess) return CDM_ESHAPE;
    const int occ = std::max(1, wg_occupancy(c128, nt, rmax, lds));

    hipStream_t st = (hipStream_t)stream;
    uint32_t* ctr = (uint32_t*)(sp + kNaCtr);
    WgJob* jobs = (WgJob*)(sp + kNaJobs);
    double* msum = (double*)(sp + kNaMsum);
    void* xloc = sp + kNaXloc;
    HIP_TRY(launch_zero_u32(ctr, 16, st));
    hipLaunchKernelGGL(k_na_jobs, dim3(1), dim3(CDM_NOALLOC_MAX_CLUSTERS), 0, st, ja, jobs);
    HIP_TRY(hipGetLastError());
    WgLaunch L;
    L.c128 = c128;
    L.nt = nt;
    L.rmax = rmax;
    L.grid = std::max(1, std::min(d.C, occ * ncu));
    L.n_max = d.U;
    L.jobs = jobs;
    L.njobs = d.C;
    L.order = nullptr;
    L.queue = ctr + 4;
    L.H = H;
    L.Y = rhs;
    L.info = (cdm_info*)info;
    L.T_max = d.T_max;
    L.tol = d.tol;
    L.ld = ldh;
    L.resid = 0;
    if (dl) {
        L.X0 = nullptr;
        L.X = x;
        L.lambda = 0.0;
        L.msum = nullptr;
        L.rho_c = rho > 0.0 ? rho / std::sqrt((double)d.C) : 0.0;
        HIP_TRY(launch_zf(L, st));
        return CDM_OK;
    }
    const bool fuse = d.C > 1;
    L.X0 = x0;
    L.X = fuse ? xloc : x;
    L.lambda = lambda;
    L.msum = fuse ? msum : nullptr;
    L.rho_c = 0.0;
    HIP_TRY(launch_wg(L, st));
    if (fuse) HIP_TRY(launch_fuse(c128, xloc, msum, lambda_c, d.C, d.U, x, st));
    return CDM_OK;
}
