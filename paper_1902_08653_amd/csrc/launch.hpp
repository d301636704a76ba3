// launch.hpp -- host-side launch descriptors shared by the runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cdm.h"

namespace cdm {

// One instance handled by one workgroup (uplink Algorithm 1, one cluster or one
// entry of an uneven batch).  Offsets are in complex elements.
struct WgJob {
    int64_t h_off;    // first element of the instance's H block
    int64_t ld;       // leading dimension of that block
    int64_t y_off;    // first element of its y
    int64_t x0_off;   // first element of its warm start (if any)
    int64_t x_off;    // first element of its output x
    int32_t m;        // rows (antennas)
    int32_t n;        // columns (users)
    int32_t info_idx; // cdm_info record to write
    int32_t rpt;      // rows per thread for this job (1, 2, 4, 8): m <= nt * rpt
};

struct WgLaunch {
    bool c128;
    int nt;           // threads per workgroup (128, 256, 512, 1024)
    int grid;         // workgroups (persistent; they pull jobs from `queue`)
    int n_max;        // largest n of any job (sizes the LDS)
    const WgJob* jobs;
    int njobs;
    const int* order; // queue slot -> job id (device), NULL = identity
    uint32_t* queue;  // device counter, zero before the launch
    const void* H;
    const void* Y;
    const void* X0;
    void* X;
    cdm_info* info;
    double lambda;
    int T_max;
    double tol;
    double* msum;     // optional: sum_u m_u per job (cluster fusion weights)
    int64_t ld;       // leading dimension for jobs whose own ld is <= 0
    double rho_c;     // downlink: per-cluster power rho/sqrt(C) (<= 0: no scaling)
    int resid;        // uplink: also write the FP64 normal-equation residual per job
    int rmax = 8;     // largest rows-per-thread tile among the jobs (<= 4 or 8)
};
hipError_t launch_wg(const WgLaunch& L, hipStream_t st);
// Algorithm 2 (downlink ZF precoding), same job and tile conventions; Y is s (U).
hipError_t launch_zf(const WgLaunch& L, hipStream_t st);
size_t wg_lds_bytes(int n_max, bool c128);
// Mixed-precision refinement of an uneven batch (complex128 H, y, x): per outer step
// an FP64 residual pass, an FP64 gradient pass (first step: also the low-precision
// copy Hq and the inner scalars) and the persistent inner-sweep launch.
enum WgLowKind { WG_LOW_NONE = 0, WG_LOW_C64 = 1, WG_LOW_BF16 = 2 };
struct BmLaunch {
    int low;              // WG_LOW_C64 or WG_LOW_BF16: format of Hq
    int nt;               // threads per workgroup of the inner launch (128, 256, 512)
    int grid;             // its persistent workgroups
    int n_max;            // largest n (sizes its LDS)
    const WgJob* jobs;    // by job id (rpt set for nt)
    int njobs;
    const int* order;     // queue slot -> job id
    uint32_t* queue;      // queue counter (cleared per step)
    const int64_t* x_off; // device packed x offsets by job id
    int64_t total_n;
    const void* H;
    const void* Y;
    const void* X0;       // optional warm start
    void* X;              // iterate / output
    void* Hq;             // low-precision copy, packed like H
    void* R;              // FP64 residual, packed like y
    void* G;              // FP32 inner bias, packed like x
    void* CF;             // FP32 (m~, n~), packed like x
    uint32_t* done;       // per job
    cdm_info* info;
    double lambda;
    double tol;
    int inner_max;
    double tau;
};
hipError_t launch_bm_init(const BmLaunch& L, hipStream_t st);
hipError_t launch_bm_step(const BmLaunch& L, int step, int last, hipStream_t st);
hipError_t launch_bm_resid_check(const BmLaunch& L, hipStream_t st);
size_t bm_lds_bytes(int n_max);
hipError_t bm_set_lds_limit(int low, int nt, size_t bytes);
int bm_occupancy(int low, int nt, size_t bytes);
// rmax: the largest rows-per-thread tile of the launch (<= 4 or 8)
hipError_t wg_set_lds_limit(bool c128, int nt, int rmax, size_t bytes);
int wg_occupancy(bool c128, int nt, int rmax, size_t bytes);

// Fusion of C local estimates (Sec. III): x = sum_c lambda_c x_c with
// lambda_c = sigma_c^-2 / sum_c' sigma_c'^-2 and sigma_c^2 = (N0/U) sum_u m_{u,c}.
hipError_t launch_fuse(bool c128, const void* xloc, const double* msum, const double* lam_c, int C, int U, void* x,
                       hipStream_t st);

// Where the panel engine reads H from.
enum SrcKind { SRC_COMPLEX = 0, SRC_BF16 = 1, SRC_FP8 = 2 };

// Cooperative panel engine for one large instance.
struct PanelLaunch {
    bool c128;
    int src_kind = SRC_COMPLEX;      // SRC_BF16 / SRC_FP8 (FP32 arithmetic only): q_* below
    const uint16_t* q_re16 = nullptr;
    const uint16_t* q_im16 = nullptr;
    const uint8_t* q_re8 = nullptr;
    const uint8_t* q_im8 = nullptr;
    const float* q_scale = nullptr;
    const void* bias = nullptr;      // optional per-column addend of b_u (inner correction solve)
    const uint32_t* done = nullptr;  // optional device flag: nonzero -> the launch does nothing
    int kp;              // panel width (columns per panel)
    int rpl;             // rows per lane (each workgroup owns 64*rpl rows)
    int P;               // workgroups (one per row block), all co-resident
    int B, U, npanels;
    const void* H;
    int64_t ld;
    const void* r0;      // initial residual (B)
    void* x;             // in: x^(0) (U), out: x^(T)
    const void* M;       // [npanels][kp*(kp+1)/2] packed lower (D + L)^-1 per panel, column by column
    const void* X = nullptr;  // look-ahead: [npanels][kp][kp] X_K = H_K^H H_{K-1 mod npanels}, transposed
                              // (element (j, v) of X_K at (K, v, j))
    const void* X2 = nullptr; // deeper look-ahead: H_K^H H_{K-2 mod npanels}, same layout
    void* part;          // [2][kp][P] partial dot products
    void* gbuf;          // [2][kp][2] reduced right-hand sides and old x
    uint32_t* ctr;       // [2] abort, [3] status word, [16..) arrival flags
    cdm_info* info;
    double lambda;
    int T_max;
    double tol;
    uint64_t timeout_ticks;
};
hipError_t launch_panel(const PanelLaunch& L, hipStream_t st);
int panel_max_coresident(bool c128, int kp, int rpl);
// Look-ahead schedule (one cross-workgroup hop per panel on the critical path):
// complex128 with kp = 64, complex64 / FP32 inner solves with kp = 128; rpl = 1 and
// P >= kp; needs PanelLaunch::X.
hipError_t launch_panel_la(const PanelLaunch& L, hipStream_t st);
int panel_la_max_coresident(bool c128, int kp);
// Deeper look-ahead (complex128, kp = 64, npanels >= 3): the partials of panel K+3 are
// formed after panel K's update, so that their exchange has two panel steps to arrive;
// needs PanelLaunch::X (as -M_K X_K) and X2.
hipError_t launch_panel_deep(const PanelLaunch& L, hipStream_t st);
// its exchange buffers hold DP_SLOTS sequences: part DP_SLOTS x kp x P and gbuf DP_SLOTS x
// kp x 2 values of 24 B (three tagged 64-bit words per complex128 value)
constexpr int DP_SLOTS = 4;
int panel_deep_max_coresident();

// Panel Gram blocks and the inverses of the Gauss-Seidel splitting matrices.
struct GramLaunch {
    bool c128;
    int src_kind = SRC_COMPLEX;
    const uint16_t* q_re16 = nullptr;
    const uint16_t* q_im16 = nullptr;
    const uint8_t* q_re8 = nullptr;
    const uint8_t* q_im8 = nullptr;
    const float* q_scale = nullptr;
    int kp;
    int B, U, npanels, nsplit;
    const void* H;
    int64_t ld;
    void* gpart;         // [nsplit][npanels][kp][kp] partial Gram blocks (row-major, lower part)
    void* M;             // out: [npanels][kp*(kp+1)/2] packed lower (D + L)^-1, column by column
    double* e;           // out: column energies ||h_u||^2 (U), FP64
    uint32_t* status;    // ORed CDM_INFO_ZERO_COLUMN
    double lambda;
};
hipError_t launch_gram(const GramLaunch& L, hipStream_t st);
// Partial Gram blocks of the BF16 or FP8 copy on the matrix cores, into L.gpart (the
// layout of the vector kernel's partials): diagonal blocks (lower sub-blocks) or, with
// cross, the blocks H_K^H H_{K-dist mod npanels}.
hipError_t launch_gram_lp(const GramLaunch& L, bool cross, int dist, hipStream_t st);
// The same for complex H (complex128 on the FP64, complex64 on the FP32 matrix cores).
hipError_t launch_gram_cx(const GramLaunch& L, bool cross, int dist, hipStream_t st);
// Cross blocks X_K = H_K^H H_{K-1 mod npanels} (full kp x kp, transposed) into X,
// using gpart as split scratch (call after launch_gram: its contents are consumed,
// and M is read).  For complex128 with 64-column panels X receives -M_K X_K
// instead, the form the look-ahead schedule uses there.
hipError_t launch_gram_cross(const GramLaunch& L, void* X, hipStream_t st);
// Cross blocks at distance two, H_K^H H_{K-2 mod npanels} (transposed, never folded),
// for the deeper look-ahead's reducer-side correction.
hipError_t launch_gram_cross2(const GramLaunch& L, void* X2, hipStream_t st);

// (D + L)^-1 from summed Gram blocks already in gpart (row-major, lower part).
hipError_t launch_gram_invert(bool c128, void* gpart, int nsplit, int npanels, int kp, int U, double lambda, void* M,
                              double* e, uint32_t* status, hipStream_t st);

// Sparse (CSR input) single-instance path.
struct SparseLaunch {
    bool c128;
    int B, U, npanels;
    int64_t nnz;
    const int32_t* rowptr;   // CSR input (device)
    const int32_t* colidx;
    const void* val;
    int32_t* colptr;         // workspace: column-compressed copy
    int32_t* fill;
    int32_t* rowidx;
    void* cval;
    void* gpart;             // [2][npanels][64][64]
    void* M;                 // [npanels][64*65/2]
    double* e;
    uint32_t* status;
    const void* y;
    const void* x0;
    void* r;
    void* x;
    cdm_info* info;
    double lambda;
    int T_max;
    double tol;
    bool transpose_only;
    int P, R;                // row slices (one workgroup each) of R rows
    int32_t* spt;            // [P+1][U] slice pointers into the column-compressed form
    int32_t* pi;             // [nnz] row-order position of each entry inside its block
    int32_t* bcnt;           // [P][npanels] block entry counts
    int32_t* roff;           // [P][npanels][R+1] row starts inside each block
    void* xp;                // [P][U] per-workgroup copies of x
    uint64_t* xbuf;          // [2][P][64][4] tagged partials
    uint32_t* abort_flag;
    uint64_t timeout_ticks;
    hipEvent_t ev_sweep0, ev_sweep1;   // optional events around the sweep kernel
};
hipError_t launch_sparse(const SparseLaunch& L, hipStream_t st);
// Rows per slice the sparse sweep aims for (slices = ceil(B / rows), 1..64).
#ifndef CDM_SPARSE_SLICE_ROWS
#define CDM_SPARSE_SLICE_ROWS 1024
#endif
void sparse_slices(int B, int ncu, int& P, int& R);
int sparse_rows_per_thread(int R);   // 0: R too large for the sweep's LDS slice

// Mixed-precision refinement (outer FP64 steps around the FP32 panel engine).
struct MixedLaunch {
    int src_kind;            // SRC_BF16 or SRC_FP8
    int B, U;
    const void* H;           // complex128 caller data
    int64_t ld;
    const void* y;
    const void* x0;
    void* x;                 // complex128 iterate / output
    uint16_t* q_re16;
    uint16_t* q_im16;
    uint8_t* q_re8;
    uint8_t* q_im8;
    float* q_scale;
    double* colamax;         // [U]
    void* rpart;             // [nchunk][B] double2
    int nchunk;
    void* r64;               // [B] double2
    void* g32;               // [U] float2 (inner bias)
    void* d32;               // [U] float2 (inner iterate)
    void* r32;               // [B] float2 (inner residual, starts at 0)
    uint32_t* ctr;           // panel engine control words to reset per outer step
    int nctr;
    uint32_t* done;          // device flag
    cdm_info* info;
    double lambda;
    double tol;
    int inner_sweeps;
};
hipError_t launch_quantize(const MixedLaunch& L, hipStream_t st);
hipError_t launch_mixed_start(const MixedLaunch& L, hipStream_t st);
hipError_t launch_mixed_outer_head(const MixedLaunch& L, hipStream_t st);
hipError_t launch_mixed_outer_tail(const MixedLaunch& L, hipStream_t st);
hipError_t launch_mixed_finish(const MixedLaunch& L, hipStream_t st);

// Warm-start MLP and its features.
hipError_t launch_features(bool c128, const void* H, const void* Y, const WgJob* jobs, const int64_t* row_off,
                           int njobs, int64_t nrows, double lambda, float* F, hipStream_t st);

// r0 = y (cold) or y - H x0 (warm); x = x0 or 0.
struct InitLaunch {
    bool c128;
    int B, U;
    const void* H;
    int64_t ld;
    const void* y;
    const void* x0;
    void* r0;
    void* x;
    void* rpart;         // [nchunk][B] scratch for the warm-start product
    int nchunk;
};
hipError_t launch_init(const InitLaunch& L, hipStream_t st);

// FP64 normal-equation residual ||H^H (y - H x) - lambda x|| / ||H^H y||.
struct ResidLaunch {
    bool c128;
    int B, U;
    const void* H;
    int64_t ld;
    const void* y;
    const void* x;
    double* rpart;       // [nchunk][2B] scratch
    int nchunk;
    double* r;           // [2B] scratch
    double* colpart;     // [2 * ceil(U/4)] scratch
    double lambda;
    double* out;         // device scalar
};
hipError_t launch_resid(const ResidLaunch& L, hipStream_t st);

// Small helpers.
hipError_t launch_zero_u32(uint32_t* p, int n, hipStream_t st);
hipError_t launch_finalize(const void* x, int U, bool c128, const uint32_t* status, cdm_info* info,
                           hipStream_t st);
hipError_t launch_copy_resid(const double* src, cdm_info* info, int count, hipStream_t st);
hipError_t launch_stream_read(const void* src, int64_t bytes, void* out, hipStream_t st);
hipError_t launch_stream_copy(const void* src, void* dst, int64_t bytes, hipStream_t st);
// Fill n reals (double if c128 else float) with scale * (u - 1/2), u a hash of (seed, i) in
// [0, 1): stand-in values for timing runs.
hipError_t launch_fill_hash(void* p, int64_t n, bool c128, uint32_t seed, double scale);

}  // namespace cdm
