// Device-side types and kernel launchers (kernels.hip).
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

#include "sweep_limits.hpp"

namespace rsilu {

// Device scalars of Algorithm 1 and the stop/breakdown flags.
struct alignas(256) DevState {
    double rho, alpha, beta, delta;
    double nb;    // ||D^{-1} z0|| = ||A^T b||
    double zn;    // latest ||D^{-1} z|| = ||A^T r||
    double tol;
    double atr;   // exit: true ||A^T (b - A x)||
    int32_t iter;    // completed iterations
    int32_t maxit;
    int32_t done;    // nonzero: every later kernel of the solve returns at once
    int32_t status;  // 0 converged / running, 1 not converged, 2 breakdown
    int32_t err;     // a sync-free wait exceeded its bound
    int32_t pad0;
    uint32_t ticket[4];  // chunk dispensers of the sync-free solves
    // LSQR: alpha, beta, the Givens rotation's state and step coefficients, ||D^{-1} s||,
    // and a stop requested by the scalar step, committed after the x update
    double la, lb, rhobar, phibar, phi_rho, theta_rho, snorm;
    int32_t lstop, lstop_status;
};

// CSR operator in device memory (values in FP64, or FP32 for the factors of
// the FP32 preconditioner).
template <class T>
struct DCsrT {
    const int32_t *ptr;
    const int32_t *col;
    const T *val;
    int32_t nrows;
};
using DCsr = DCsrT<double>;

// Split of long rows into fixed segments (reduced in a fixed order).
struct DPlan {
    const int32_t *long_rows;
    const int32_t *seg_ptr;
    const int32_t *seg_beg;
    const int32_t *seg_end;
    int32_t nlong, nseg, lanes, long_thresh;
    int32_t unroll;  // entries per lane loaded at once by the paired-row kernel (2, 3 or 4)
};

// Triangular operator: strictly triangular CSR, optional diagonal, level-ordered rows,
// chunks of one level each.
template <class T>
struct DTriT {
    DCsrT<T> a;
    const T *diag;        // nullptr: unit diagonal
    const int32_t *rows;  // rows in level order
    const int32_t *chunk; // nchunks + 1 positions into rows
    int32_t nchunks;
    int32_t lanes;        // lanes per row (64 / chunk capacity)
};
using DTri = DTriT<double>;

enum Epi : int32_t {
    EPI_PLAIN = 0,  // y = A x
    EPI_SQ = 1,     // y = A x, partial sums of y^2
    EPI_SUB = 2,    // y = aux - A x
    EPI_WSQ = 3,    // y = A x, partial sums of (aux * y)^2
    EPI_NEG = 4,    // y = -A x
    EPI_ADD = 5     // y = aux + A x
};
// (the FP32 products use EPI_PLAIN, EPI_SUB and EPI_NEG only)

enum Fin : int32_t {
    FIN_NONE = 0,   // long rows only
    FIN_INIT = 1,   // nb = sqrt(sum); nb == 0 -> done, converged, 0 iterations
    FIN_ALPHA = 2,  // delta = sum; alpha = rho / delta
    FIN_STOP = 3,   // zn = sqrt(sum); ++iter; stop test
    FIN_RHO0 = 4,   // rho = sum
    FIN_BETA = 5,   // beta = sum / rho; rho = sum
    FIN_ATR = 6,    // atr = sqrt(sum)
    // (7 to 9: unused; the CG steps on S~ form their scalars in their own kernels)
    FIN_L_BETA1 = 10,  // LSQR init: lb = phibar = sqrt(sum) (= ||P b||); 0 -> done, converged
    FIN_L_S1 = 11,     // LSQR init: snorm = sqrt(sum); nb = zn = lb snorm (= ||A^T b||)
    FIN_L_ALPHA0 = 12, // LSQR init: la = rhobar = sqrt(sum); <= 0 or not finite -> breakdown
    FIN_L_BETA = 13,   // LSQR: lb = sqrt(sum)
    FIN_L_SNORM = 14,  // LSQR: snorm = sqrt(sum)
    FIN_L_ALPHA = 15   // LSQR: la = sqrt(sum), Givens step, ++iter, stop test (requested in lstop)
};

constexpr int kBlock = 256;


// ---- launchers (all asynchronous on `s`); `done` may be nullptr
void launch_gather(hipStream_t s, int32_t m, int32_t n, const int32_t *perm, const double *b, double *r,
                   double *xh, const int32_t *done);
// y = op(A) x with epilogue; long rows through segments; partial sums of the
// epilogue norm, then the single-block finish (reduction + scalar step).
template <class T>
void launch_spmv(hipStream_t s, const DCsrT<T> &a, const DPlan &pl, const T *x, T *y, const T *aux, Epi epi,
                 Fin fin, double *partials, T *segpart, DevState *st, const int32_t *done);
// a . b and the scalar step `fin` (per-block partials, then one block)
void launch_dot(hipStream_t s, int32_t n, const double *a, const double *b, Fin fin, double *partials,
                DevState *st, const int32_t *done);
// x_hat += alpha p; r -= alpha q; sentinel-fill the sync-free outputs; reset tickets
void launch_update(hipStream_t s, int32_t n, int32_t m, const double *p, double *xh, const double *q, double *r,
                   double *f0, double *f1, double *f2, double *f3, DevState *st, const int32_t *done);
void launch_fill(hipStream_t s, int32_t n, double *f0, double *f1, double *f2, double *f3, DevState *st);
// sentinel-fill f0, f1 and clear tickets 0 and 1 (honours `done`)
void launch_refill(hipStream_t s, int32_t n, double *f0, double *f1, DevState *st, const int32_t *done);
void launch_pupdate(hipStream_t s, int32_t n, const double *h, double *p, const DevState *st, bool first,
                    const int32_t *done);
void launch_scale_out(hipStream_t s, int32_t n, const double *xh, const double *colnorm, double *x);
void launch_residual(hipStream_t s, int32_t m, const int32_t *perm, const double *b, const double *ax, double *r);
// Triangular solve T x = rhs (unit diagonal if T.diag is null). Optionally y2 = add + x.
// Sync-free: x must be sentinel-filled and the ticket zero (launch_fill / launch_update).
void launch_trsv_syncfree(hipStream_t s, const DTri &t, const double *rhs, double *x, const double *add,
                          double *y2, DevState *st, int ticket, const int32_t *done);
template <class T>
void launch_trsv_level(hipStream_t s, const DTriT<T> &t, int32_t beg, int32_t end, const T *rhs, T *x, const T *add,
                       T *y2, const int32_t *done);
// nb consecutive batches of a hybrid sweep by one workgroup, starting with the
// batch at byte `off` of `blob` (its size and row count given); rhs_lo and
// add_lo are the right-hand side and addend in level order. scheme: the level
// scheme the blob was built for (kSchemeTwoPhase, kSchemeSegmented,
// kSchemeSegmentedWide or kSchemeRows; other values: two phases).
template <class T>
void launch_trsv_sweep(hipStream_t s, const unsigned char *blob, int64_t off, int32_t size, int32_t npos_first,
                       int32_t p0, int32_t nb, int32_t scheme, const T *rhs_lo, T *x, const T *add_lo, T *y2,
                       const int32_t *done);
// dst[p] = src[rows[p]] (and dst2 from src2 when given)
template <class T>
void launch_gather_lo(hipStream_t s, int32_t n, const int32_t *rows, const T *src, T *dst, const T *src2, T *dst2,
                      const int32_t *done);
// out = in converted (FP64 <-> FP32, round to nearest)
void launch_cvt(hipStream_t s, int32_t n, const double *in, float *out, const int32_t *done);
// LSQR steps (device scalars in st):
// t -= la u with the partial sums of t^2, then the single-block finish (fin)
void launch_lsqr_t(hipStream_t s, int32_t m, const double *u, double *t, Fin fin, double *partials, DevState *st,
                   const int32_t *done);
// out = in / lb (in when lb = 0)
void launch_lsqr_scale(hipStream_t s, int32_t m, const double *in, double *out, const DevState *st,
                       const int32_t *done);
// sv -= lb Mv with the partial sums of (colnorm s)^2, then the finish (fin)
void launch_lsqr_s(hipStream_t s, int32_t n, double *sv, const double *Mv, const double *colnorm, Fin fin,
                   double *partials, DevState *st, const int32_t *done);
// x_hat += phi_rho w; when la > 0: v = h / la, Mv = s / la, w = v - theta_rho w (init: w = v)
void launch_lsqr_v(hipStream_t s, int32_t n, const double *h, const double *sv, double *xh, double *v, double *Mv,
                   double *w, bool init, const DevState *st, const int32_t *done);
// a stop requested by FIN_L_ALPHA takes effect
void launch_lsqr_commit(hipStream_t s, DevState *st);
void launch_cvt(hipStream_t s, int32_t n, const float *in, double *out, const int32_t *done);
// w = (L L^T)^{-1} u with L packed lower (k x k), in place on w (w = u on entry)
void launch_dense_chol_solve(hipStream_t s, int32_t k, const double *lfac, double *w, const int32_t *done);
void launch_copy(hipStream_t s, int32_t n, const double *src, double *dst, const int32_t *done);
// dst += src
void launch_add(hipStream_t s, int32_t n, const double *src, double *dst, const int32_t *done);
// CG on S~: res = p = u, w = 0; then w += alpha p, res -= alpha q; p = res + beta p. The
// scalars come from per-block partials (cg_nparts(k) of each, in arrays of kCgParts):
// pq_parts of (p, q), rr_old / rr_new of (res, res) or (res, z) of the previous / this step,
// each kernel forming alpha or beta itself.
int cg_nparts(int32_t k);
// per-block partials of a . b over k entries (cg_nparts(k) blocks)
void launch_cg_dot(hipStream_t s, int32_t k, const double *a, const double *b, double *parts, const int32_t *done);
void launch_cg_init(hipStream_t s, int32_t k, const double *u, double *w, double *res, double *p, const int32_t *done);
void launch_cg_update(hipStream_t s, int32_t k, const double *p, const double *q, double *w, double *res,
                      const double *pq_parts, const double *rr_parts, const int32_t *done);
void launch_cg_dir(hipStream_t s, int32_t k, const double *res, double *p, const double *rr_old, const double *rr_new,
                   const int32_t *done);
// Jacobi-preconditioned CG on S~: res = u, z = u / d, p = z, w = 0; the update with
// z = res / d and the partials of res . z (into rr_new)
void launch_pcg_init(hipStream_t s, int32_t k, const double *u, const double *d, double *w, double *res, double *z,
                     double *p, const int32_t *done);
void launch_pcg_update_dot(hipStream_t s, int32_t k, const double *p, const double *q, const double *d, double *w,
                           double *res, double *z, const double *pq_parts, const double *rr_old, double *rr_new,
                           const int32_t *done);
// the update with the partials of res . res (into rr_new)
void launch_cg_update_dot(hipStream_t s, int32_t k, const double *p, const double *q, double *w, double *res,
                          const double *pq_parts, const double *rr_old, double *rr_new, const int32_t *done);
// Chebyshev steps on S~: r = omega u, d = r / theta, w = 0; then per step, with
// q = Y~ (Y~^T d): w += d, r -= d + q, d = c1 d + c2 r, and out = w when out is given (the
// last step)
template <class T>
void launch_cheb_init(hipStream_t s, int32_t k, const T *u, T *r, T *d, T *w, double theta, double omega,
                      const int32_t *done);
template <class T>
void launch_cheb_update(hipStream_t s, int32_t k, const T *q, T *r, T *d, T *w, T *out, double c1, double c2,
                        const int32_t *done);

}  // namespace rsilu
