/*
 * cd_oracle.c -- plain, slow FP64 CPU oracle for decentralized coordinate-descent
 * (CD) data detection and precoding in massive MU-MIMO
 * (K. Li, O. Castaneda, C. Jeon, J. R. Cavallaro, C. Studer, arXiv 1902.08653).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or load
 * this file; only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header, table or helper with the GPU library.
 *
 * Conventions
 *   - Complex numbers are C99 `double complex` (interleaved re, im in memory).
 *   - The uplink channel H is B x U, column-major with leading dimension ldh >= B,
 *     so the u-th user column h_u is contiguous (Sec. II-A, uplink model).
 *   - The downlink channel is the conjugate transpose of the same stored matrix
 *     (Sec. II-B, reciprocity), so H is passed in uplink orientation there too.
 *   - lambda := N0 / Ex is the regulariser of eq. (1).
 *
 * Stop rule (the paper runs a fixed number of sweeps T_max, Alg. 1 and Alg. 2, and
 * says "until convergence" in Sec. IV-A without a criterion):
 *   tol == 0 : exactly T_max sweeps.
 *   tol  > 0 : after sweep t stop when sqrt(sum_u |delta_u|^2) <= tol * ||x^(t)||_2,
 *              or when t == T_max.
 *
 * Every function follows the paper's steps in the paper's order with no blocking,
 * fusion or reordering.  Floating point sums run sequentially in index order.
 *
 * Pins (checked by tests/test_oracle_pins.py, none of which re-types this code):
 *   closed form of eq. (1) / eq. (2) via LAPACK, Gauss-Seidel equivalence on the
 *   explicitly formed normal equations, per-step invariants (residual identity,
 *   coordinate optimality, monotone objective), special cases (U = 1, orthogonal
 *   columns, y = 0), the asymptotic rate of the Gauss-Seidel splitting, exact
 *   rational brute force on tiny Gaussian-integer inputs, and scipy's CSR->CSC.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define CDO_FLAG_ZERO_COLUMN   1   /* some coordinate had ||h_u||^2 + lambda == 0; it stays inactive */
#define CDO_FLAG_NONFINITE     2   /* the output holds NaN or Inf */
#define CDO_FLAG_NOT_CONVERGED 4   /* tol > 0 and the cap T_max was reached first */

typedef double complex cplx;

static double abs2(cplx z) { return creal(z) * creal(z) + cimag(z) * cimag(z); }

/* ------------------------------------------------------------------------- */
/* Alg. 1 preprocessing: e_u = ||h_u||^2, m_u = (e_u + N0/Ex)^-1, n_u = m_u e_u.  */
/* ------------------------------------------------------------------------- */
void cdo_column_scalars(int Bc, int U, const cplx* H, long ldh, double lambda,
                        double* e, double* m, double* n)
{
    for (int u = 0; u < U; ++u) {
        double s = 0.0;
        for (int i = 0; i < Bc; ++i) s += abs2(H[(long)u * ldh + i]);
        e[u] = s;
        m[u] = 1.0 / (s + lambda);
        n[u] = m[u] * s;
    }
}

/* ------------------------------------------------------------------------- */
/* Alg. 1, local CD at one antenna cluster (rows Bc of H_c, ld ldh).           */
/*   Init: r = y, x = 0 (or the warm start x0 with r = y - H x0).              */
/*   for t = 1..T_max, for u = 1..U:                                           */
/*      x_u^(t) = m_u h_u^H r + n_u x_u^(t-1);  delta = x_u^(t) - x_u^(t-1);   */
/*      r = r - h_u delta.                                                     */
/* Optional traces (NULL to skip):                                             */
/*   sweep_x [T_max*U]      x after each sweep,                                */
/*   step_x  [T_max*U*U]    x after each coordinate step,                      */
/*   step_r  [T_max*U*Bc]   r after each coordinate step,                      */
/*   sweep_s [T_max]        sum_u |delta_u|^2 of each sweep.                   */
/* Returns the number of sweeps performed.                                     */
/* ------------------------------------------------------------------------- */
int cdo_local_cd(int Bc, int U, const cplx* H, long ldh, const cplx* y, double lambda,
                 const cplx* x0, int T_max, double tol,
                 cplx* x, double* rel_step, int* flags,
                 cplx* sweep_x, cplx* step_x, cplx* step_r, double* sweep_s)
{
    double* e = (double*)malloc(sizeof(double) * (size_t)(U > 0 ? U : 1));
    double* m = (double*)malloc(sizeof(double) * (size_t)(U > 0 ? U : 1));
    double* n = (double*)malloc(sizeof(double) * (size_t)(U > 0 ? U : 1));
    cplx* r = (cplx*)malloc(sizeof(cplx) * (size_t)(Bc > 0 ? Bc : 1));
    int fl = 0;

    /* Preprocessing (Alg. 1). */
    cdo_column_scalars(Bc, U, H, ldh, lambda, e, m, n);
    for (int u = 0; u < U; ++u)
        if (!(e[u] + lambda > 0.0)) fl |= CDO_FLAG_ZERO_COLUMN;

    /* Init (Alg. 1): r = y, x = 0; a warm start x0 gives r = y - H x0. */
    for (int i = 0; i < Bc; ++i) r[i] = y[i];
    for (int u = 0; u < U; ++u) x[u] = x0 ? x0[u] : 0.0;
    if (x0) {
        for (int u = 0; u < U; ++u)
            for (int i = 0; i < Bc; ++i) r[i] -= H[(long)u * ldh + i] * x[u];
    }

    int t_done = 0;
    double last_rel = 0.0;
    for (int t = 1; t <= T_max; ++t) {
        double S = 0.0;
        for (int u = 0; u < U; ++u) {
            const cplx* h = H + (long)u * ldh;
            cplx delta = 0.0;
            if (e[u] + lambda > 0.0) {
                cplx g = 0.0;                                  /* h_u^H r */
                for (int i = 0; i < Bc; ++i) g += conj(h[i]) * r[i];
                cplx xnew = m[u] * g + n[u] * x[u];            /* scalar rule */
                delta = xnew - x[u];
                x[u] = xnew;
                for (int i = 0; i < Bc; ++i) r[i] -= h[i] * delta;   /* residual update */
            }
            S += abs2(delta);
            if (step_x) memcpy(step_x + ((long)(t - 1) * U + u) * U, x, sizeof(cplx) * (size_t)U);
            if (step_r) memcpy(step_r + ((long)(t - 1) * U + u) * Bc, r, sizeof(cplx) * (size_t)Bc);
        }
        double X = 0.0;
        for (int u = 0; u < U; ++u) X += abs2(x[u]);
        if (sweep_x) memcpy(sweep_x + (long)(t - 1) * U, x, sizeof(cplx) * (size_t)U);
        if (sweep_s) sweep_s[t - 1] = S;
        t_done = t;
        last_rel = (X > 0.0) ? sqrt(S / X) : (S > 0.0 ? INFINITY : 0.0);
        if (tol > 0.0 && sqrt(S) <= tol * sqrt(X)) break;
    }
    if (tol > 0.0 && !(last_rel <= tol)) fl |= CDO_FLAG_NOT_CONVERGED;
    for (int u = 0; u < U; ++u)
        if (!isfinite(creal(x[u])) || !isfinite(cimag(x[u]))) fl |= CDO_FLAG_NONFINITE;

    if (rel_step) *rel_step = last_rel;
    if (flags) *flags = fl;
    free(e); free(m); free(n); free(r);
    return t_done;
}

/* ------------------------------------------------------------------------- */
/* Alg. 1 end to end: C clusters of Bc[c] consecutive rows (B = sum_c Bc[c]),  */
/* local CD at each, then the fusion x_hat = sum_c lambda_c x_hat_c.           */
/* The fusion weight is lambda_c = sigma_c^-2 / sum_c' sigma_c'^-2 (Sec. III); */
/* the paper leaves sigma_c^2 undefined.  Reading used here: the diagonal      */
/* approximation of the local L-MMSE error, sigma_c^2 = (N0/U) sum_u m_{u,c}.  */
/* The factor N0/U is common to every cluster and cancels from the ratio, so   */
/* the weights are formed as lambda_c = s_c^-1 / sum_c' s_c'^-1 with           */
/* s_c = sum_u m_{u,c}: equal to the definition for N0 > 0, and defined at     */
/* N0 = 0 as its limit.  A cluster with s_c = 0 (possible only at N0 = 0 when  */
/* every column of it is zero, so every coordinate is inactive) carries no     */
/* estimate and gets weight 0; if every cluster does, x_hat = 0.               */
/* lam_c (C weights) overrides the weights, used as given, when not NULL.      */
/* Bc == NULL means C equal blocks (B % C == 0).                               */
/* Per-cluster outputs: x_local [C*U] (may be NULL), sweeps/rel_step/flags [C].*/
/* ------------------------------------------------------------------------- */
int cdo_uplink_cd(int B, int U, int C, const int* Bc, const cplx* H, long ldh,
                  const cplx* y, double N0, double Ex, const cplx* x0, const double* lam_c,
                  int T_max, double tol, cplx* x_hat, cplx* x_local,
                  int* sweeps, double* rel_step, int* flags, double* weights_out)
{
    double lambda = N0 / Ex;
    cplx* xl = (cplx*)malloc(sizeof(cplx) * (size_t)C * (size_t)(U > 0 ? U : 1));
    double* w = (double*)malloc(sizeof(double) * (size_t)C);
    double* m = (double*)malloc(sizeof(double) * (size_t)(U > 0 ? U : 1));
    double* e = (double*)malloc(sizeof(double) * (size_t)(U > 0 ? U : 1));
    double* n = (double*)malloc(sizeof(double) * (size_t)(U > 0 ? U : 1));
    int row0 = 0;
    for (int c = 0; c < C; ++c) {
        int bc = Bc ? Bc[c] : B / C;
        const cplx* Hc = H + row0;
        sweeps[c] = cdo_local_cd(bc, U, Hc, ldh, y + row0, lambda, x0, T_max, tol,
                                 xl + (long)c * U, &rel_step[c], &flags[c],
                                 NULL, NULL, NULL, NULL);
        /* sigma_c^2 reading (see header comment): s_c = sum_u m_{u,c}, where an  */
        /* inactive coordinate (||h_u||^2 + lambda == 0) has m_u = 0.             */
        cdo_column_scalars(bc, U, Hc, ldh, lambda, e, m, n);
        double sm = 0.0;
        for (int u = 0; u < U; ++u) sm += (e[u] + lambda > 0.0) ? m[u] : 0.0;
        w[c] = (sm > 0.0) ? 1.0 / sm : 0.0;
        row0 += bc;
    }
    if (lam_c) {
        for (int c = 0; c < C; ++c) w[c] = lam_c[c];
    } else {
        double tot = 0.0;
        for (int c = 0; c < C; ++c) tot += w[c];
        for (int c = 0; c < C; ++c) w[c] = (tot > 0.0) ? w[c] / tot : 0.0;
    }
    for (int u = 0; u < U; ++u) {
        cplx s = 0.0;
        for (int c = 0; c < C; ++c) s += w[c] * xl[(long)c * U + u];
        x_hat[u] = s;
    }
    if (x_local) memcpy(x_local, xl, sizeof(cplx) * (size_t)C * (size_t)U);
    if (weights_out) memcpy(weights_out, w, sizeof(double) * (size_t)C);
    free(xl); free(w); free(m); free(e); free(n);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Alg. 2 / eq. (4), local ZF precoding by CD at one cluster.                  */
/* The local downlink channel is H_c^dl = (H_c^ul)^H (U x Bc); its u-th row    */
/* is h_u^H with h_u the u-th column of the stored uplink block.               */
/* Preprocessing: p_u = ||h_u||^-1, hbar_u = p_u h_u, sbar_u = p_u s_u.        */
/* Init x = 0 (Bc).  Cyclic over t and u:                                      */
/*     x <- x - (hbar_u^H x - sbar_u) hbar_u                 (eq. (4))          */
/* The step size per coordinate is |hbar_u^H x - sbar_u| (hbar_u has unit norm)*/
/* and feeds the same relative-step stop rule as the uplink.                   */
/* The power scaling x <- rho_c x / ||x|| is applied by the caller.            */
/* ------------------------------------------------------------------------- */
int cdo_local_zf_cd(int Bc, int U, const cplx* H, long ldh, const cplx* s,
                    int T_max, double tol, cplx* x, double* rel_step, int* flags,
                    cplx* sweep_x, cplx* step_x)
{
    double* p = (double*)malloc(sizeof(double) * (size_t)(U > 0 ? U : 1));
    cplx* sbar = (cplx*)malloc(sizeof(cplx) * (size_t)(U > 0 ? U : 1));
    int fl = 0;
    for (int u = 0; u < U; ++u) {
        double nn = 0.0;
        for (int i = 0; i < Bc; ++i) nn += abs2(H[(long)u * ldh + i]);
        if (nn > 0.0) {
            p[u] = 1.0 / sqrt(nn);
        } else {
            p[u] = 0.0;                 /* zero row of H^dl: coordinate inactive */
            fl |= CDO_FLAG_ZERO_COLUMN;
        }
        sbar[u] = p[u] * s[u];
    }
    for (int i = 0; i < Bc; ++i) x[i] = 0.0;
    int t_done = 0;
    double last_rel = 0.0;
    for (int t = 1; t <= T_max; ++t) {
        double S = 0.0;
        for (int u = 0; u < U; ++u) {
            if (p[u] == 0.0) {
                if (step_x) memcpy(step_x + ((long)(t - 1) * U + u) * Bc, x, sizeof(cplx) * (size_t)Bc);
                continue;
            }
            const cplx* h = H + (long)u * ldh;
            cplx a = 0.0;                                   /* hbar_u^H x */
            for (int i = 0; i < Bc; ++i) a += conj(p[u] * h[i]) * x[i];
            cplx err = a - sbar[u];
            for (int i = 0; i < Bc; ++i) x[i] -= err * (p[u] * h[i]);
            S += abs2(err);
            if (step_x) memcpy(step_x + ((long)(t - 1) * U + u) * Bc, x, sizeof(cplx) * (size_t)Bc);
        }
        double X = 0.0;
        for (int i = 0; i < Bc; ++i) X += abs2(x[i]);
        if (sweep_x) memcpy(sweep_x + (long)(t - 1) * Bc, x, sizeof(cplx) * (size_t)Bc);
        t_done = t;
        last_rel = (X > 0.0) ? sqrt(S / X) : (S > 0.0 ? INFINITY : 0.0);
        if (tol > 0.0 && sqrt(S) <= tol * sqrt(X)) break;
    }
    if (tol > 0.0 && !(last_rel <= tol)) fl |= CDO_FLAG_NOT_CONVERGED;
    for (int i = 0; i < Bc; ++i)
        if (!isfinite(creal(x[i])) || !isfinite(cimag(x[i]))) fl |= CDO_FLAG_NONFINITE;
    if (rel_step) *rel_step = last_rel;
    if (flags) *flags = fl;
    free(p); free(sbar);
    return t_done;
}

/* ------------------------------------------------------------------------- */
/* Alg. 2 end to end: broadcast s, local CD at each cluster, then the local    */
/* power scaling x_c <- rho_c x_c / ||x_c|| with rho_c^2 = rho^2 / C           */
/* (Sec. IV-B); output is the stacked [x_1; ...; x_C] (B entries).             */
/* rho <= 0 skips the scaling (returns the unscaled local ZF iterates).        */
/* x_c == 0 stays 0.                                                           */
/* ------------------------------------------------------------------------- */
int cdo_downlink_cd(int B, int U, int C, const int* Bc, const cplx* H, long ldh,
                    const cplx* s, double rho, int T_max, double tol, cplx* x,
                    int* sweeps, double* rel_step, int* flags)
{
    int row0 = 0;
    double rho_c = rho / sqrt((double)C);
    for (int c = 0; c < C; ++c) {
        int bc = Bc ? Bc[c] : B / C;
        cplx* xc = x + row0;
        sweeps[c] = cdo_local_zf_cd(bc, U, H + row0, ldh, s, T_max, tol, xc,
                                    &rel_step[c], &flags[c], NULL, NULL);
        if (rho > 0.0) {
            double nn = 0.0;
            for (int i = 0; i < bc; ++i) nn += abs2(xc[i]);
            double nrm = sqrt(nn);
            if (nrm > 0.0)
                for (int i = 0; i < bc; ++i) xc[i] = rho_c * xc[i] / nrm;
        }
        row0 += bc;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Sparse H: CSR (rows = antennas) -> column-compressed form, because CD walks */
/* columns.  Definition: entry k of row i with column j lands in column j;     */
/* within a column, entries are ordered by increasing row (rows are visited in */
/* increasing order and each row's entries are appended in turn).  Column      */
/* indices of the input are assumed to be strictly increasing within a row.    */
/* ------------------------------------------------------------------------- */
void cdo_csr_to_csc(int B, int U, const int32_t* rowptr, const int32_t* colidx,
                    const cplx* val, int32_t* colptr, int32_t* rowidx, cplx* cval)
{
    for (int j = 0; j <= U; ++j) colptr[j] = 0;
    for (int i = 0; i < B; ++i)
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k) colptr[colidx[k] + 1] += 1;
    for (int j = 0; j < U; ++j) colptr[j + 1] += colptr[j];
    int32_t* fill = (int32_t*)malloc(sizeof(int32_t) * (size_t)(U > 0 ? U : 1));
    for (int j = 0; j < U; ++j) fill[j] = colptr[j];
    for (int i = 0; i < B; ++i)
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            int32_t j = colidx[k];
            rowidx[fill[j]] = i;
            cval[fill[j]] = val[k];
            fill[j] += 1;
        }
    free(fill);
}

/* ------------------------------------------------------------------------- */
/* Alg. 1 (one cluster, C = 1) on a column-compressed sparse H.  Identical     */
/* steps to cdo_local_cd; sums run over the stored entries of each column in   */
/* increasing row order.                                                       */
/* ------------------------------------------------------------------------- */
int cdo_local_cd_csc(int B, int U, const int32_t* colptr, const int32_t* rowidx,
                     const cplx* cval, const cplx* y, double lambda, const cplx* x0,
                     int T_max, double tol, cplx* x, double* rel_step, int* flags)
{
    double* e = (double*)malloc(sizeof(double) * (size_t)(U > 0 ? U : 1));
    cplx* r = (cplx*)malloc(sizeof(cplx) * (size_t)(B > 0 ? B : 1));
    int fl = 0;
    for (int u = 0; u < U; ++u) {
        double s = 0.0;
        for (int32_t k = colptr[u]; k < colptr[u + 1]; ++k) s += abs2(cval[k]);
        e[u] = s;
        if (!(s + lambda > 0.0)) fl |= CDO_FLAG_ZERO_COLUMN;
    }
    for (int i = 0; i < B; ++i) r[i] = y[i];
    for (int u = 0; u < U; ++u) x[u] = x0 ? x0[u] : 0.0;
    if (x0)
        for (int u = 0; u < U; ++u)
            for (int32_t k = colptr[u]; k < colptr[u + 1]; ++k) r[rowidx[k]] -= cval[k] * x[u];
    int t_done = 0;
    double last_rel = 0.0;
    for (int t = 1; t <= T_max; ++t) {
        double S = 0.0;
        for (int u = 0; u < U; ++u) {
            cplx delta = 0.0;
            if (e[u] + lambda > 0.0) {
                double mu = 1.0 / (e[u] + lambda);
                double nu = mu * e[u];
                cplx g = 0.0;
                for (int32_t k = colptr[u]; k < colptr[u + 1]; ++k) g += conj(cval[k]) * r[rowidx[k]];
                cplx xnew = mu * g + nu * x[u];
                delta = xnew - x[u];
                x[u] = xnew;
                for (int32_t k = colptr[u]; k < colptr[u + 1]; ++k) r[rowidx[k]] -= cval[k] * delta;
            }
            S += abs2(delta);
        }
        double X = 0.0;
        for (int u = 0; u < U; ++u) X += abs2(x[u]);
        t_done = t;
        last_rel = (X > 0.0) ? sqrt(S / X) : (S > 0.0 ? INFINITY : 0.0);
        if (tol > 0.0 && sqrt(S) <= tol * sqrt(X)) break;
    }
    if (tol > 0.0 && !(last_rel <= tol)) fl |= CDO_FLAG_NOT_CONVERGED;
    for (int u = 0; u < U; ++u)
        if (!isfinite(creal(x[u])) || !isfinite(cimag(x[u]))) fl |= CDO_FLAG_NONFINITE;
    if (rel_step) *rel_step = last_rel;
    if (flags) *flags = fl;
    free(e); free(r);
    return t_done;
}

/* ------------------------------------------------------------------------- */
/* Stationarity of eq. (1): the relative normal-equation residual              */
/*     || H^H (y - H x) - lambda x || / || H^H y ||                            */
/* (0 exactly at the unique minimiser when lambda > 0).                        */
/* ------------------------------------------------------------------------- */
double cdo_normal_residual(int B, int U, const cplx* H, long ldh, const cplx* y,
                           double lambda, const cplx* x)
{
    cplx* r = (cplx*)malloc(sizeof(cplx) * (size_t)(B > 0 ? B : 1));
    for (int i = 0; i < B; ++i) r[i] = y[i];
    for (int u = 0; u < U; ++u)
        for (int i = 0; i < B; ++i) r[i] -= H[(long)u * ldh + i] * x[u];
    double num = 0.0, den = 0.0;
    for (int u = 0; u < U; ++u) {
        cplx a = 0.0, b = 0.0;
        for (int i = 0; i < B; ++i) {
            a += conj(H[(long)u * ldh + i]) * r[i];
            b += conj(H[(long)u * ldh + i]) * y[i];
        }
        num += abs2(a - lambda * x[u]);
        den += abs2(b);
    }
    free(r);
    return den > 0.0 ? sqrt(num / den) : sqrt(num);
}

/* ------------------------------------------------------------------------- */
/* Low-precision copies of H for the mixed-precision refinement (not part of   */
/* the paper; definitions of this project, written out plainly):               */
/*   BF16: each real component is rounded to FP32 (nearest, ties to even),     */
/*         then to BF16 (the top 16 bits of FP32; nearest, ties to even).      */
/*   FP8 : OCP E4M3 (1 sign, 4 exponent bits with bias 7, 3 mantissa bits; no  */
/*         infinities; largest finite 448).  One FP32 scale per block of 128   */
/*         consecutive columns, s = fl32(amax / 448) with amax the largest     */
/*         |Re| or |Im| in the block (s = 1 for an all-zero block); each        */
/*         component v = fl32(h / s) is coded to the nearest E4M3 value, ties   */
/*         to the even code, magnitudes above 448 saturating to 448.            */
/* ------------------------------------------------------------------------- */
uint16_t cdo_bf16_code(double v)
{
    float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
    /* nearest of the two BF16 neighbours of f, ties to the even one */
    uint32_t lo = u & 0xffff0000u;
    uint32_t rem = u & 0x0000ffffu;
    uint32_t q = lo >> 16;
    if (rem > 0x8000u || (rem == 0x8000u && (q & 1u))) q += 1u;
    return (uint16_t)q;
}

double cdo_bf16_value(uint16_t c)
{
    uint32_t u = (uint32_t)c << 16;
    float f;
    memcpy(&f, &u, 4);
    return (double)f;
}

double cdo_e4m3_value(uint8_t c)
{
    int s = (c >> 7) & 1, e = (c >> 3) & 15, m = c & 7;
    double v;
    if (e == 15 && m == 7) return NAN;
    if (e == 0) v = ldexp((double)m, -9);
    else v = ldexp(1.0 + m / 8.0, e - 7);
    return s ? -v : v;
}

/* nearest code by exhaustive comparison with every finite non-negative code */
uint8_t cdo_e4m3_code(float v)
{
    if (isnan(v)) return 0x7f;
    uint8_t sign = (v < 0.0f) ? 0x80 : 0x00;
    double a = fabs((double)v);
    if (a >= 448.0) return sign | 0x7e;
    int best = 0;
    double bd = INFINITY;
    for (int c = 0; c <= 0x7e; ++c) {
        double d = fabs(cdo_e4m3_value((uint8_t)c) - a);
        if (d < bd || (d == bd && (c & 1) == 0 && (best & 1) == 1)) {
            bd = d;
            best = c;
        }
    }
    return sign | (uint8_t)best;
}

/* Quantise a B x U column-major complex H (ld) into planar codes (column-major,
 * ld = B).  kind 0: BF16 into re16/im16; kind 1: FP8 into re8/im8 with scales
 * (ceil(U/128) floats). */
void cdo_quantize(int kind, int B, int U, const cplx* H, long ldh, uint16_t* re16, uint16_t* im16,
                  uint8_t* re8, uint8_t* im8, float* scales)
{
    if (kind == 0) {
        for (int u = 0; u < U; ++u)
            for (int i = 0; i < B; ++i) {
                cplx h = H[(long)u * ldh + i];
                re16[(long)u * B + i] = cdo_bf16_code(creal(h));
                im16[(long)u * B + i] = cdo_bf16_code(cimag(h));
            }
        return;
    }
    int nblk = (U + 127) / 128;
    for (int b = 0; b < nblk; ++b) {
        double amax = 0.0;
        for (int u = b * 128; u < U && u < b * 128 + 128; ++u)
            for (int i = 0; i < B; ++i) {
                cplx h = H[(long)u * ldh + i];
                if (fabs(creal(h)) > amax) amax = fabs(creal(h));
                if (fabs(cimag(h)) > amax) amax = fabs(cimag(h));
            }
        float s = (amax > 0.0) ? (float)(amax / 448.0) : 1.0f;
        scales[b] = s;
        for (int u = b * 128; u < U && u < b * 128 + 128; ++u)
            for (int i = 0; i < B; ++i) {
                cplx h = H[(long)u * ldh + i];
                re8[(long)u * B + i] = cdo_e4m3_code((float)(creal(h) / (double)s));
                im8[(long)u * B + i] = cdo_e4m3_code((float)(cimag(h) / (double)s));
            }
    }
}
