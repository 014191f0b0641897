// HIP kernels for CDNA4 (gfx950) of the preconditioned CGLS solve.
//
// Everything on this path is sparse FP64 streaming (about 0.15 flop per byte),
// so the kernels are written for HBM bandwidth and latency, not for MFMA:
//  - CSR products give each row a group of G lanes of a 64-wide wavefront
//    (G chosen from the mean row length) so consecutive rows' entries are read
//    contiguously; rows far longer than the mean are cut into fixed segments
//    reduced in a fixed order, so results never depend on scheduling.
//  - Norms and dot products are reduced per block in a fixed tree and then by
//    one block in index order (bit-reproducible), and the same single block
//    advances the scalar recurrence of Algorithm 1 on the device.
//  - Triangular solves run "sync-free": one launch; wavefronts take chunks of
//    rows (one level each) from an atomic ticket in level order and wait on
//    their inputs, which are published with a single 64-bit store over a
//    signalling-NaN sentinel (no flag array, no fences). Taking chunks in level
//    order guarantees that every awaited row belongs to a wave already running.
#include <cmath>
#include <cstdint>

#include <type_traits>

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace rsilu {

namespace {

// Signalling NaN: arithmetic only ever produces quiet NaNs, so no computed
// value can equal it.
constexpr unsigned long long kSentinel = 0x7FF4DEADBEEF0001ull;
constexpr unsigned long long kQuietNaN = 0x7FF8000000000000ull;
constexpr int kSpinLimit = 1 << 20;
constexpr int kSpmvRows = 2;  // rows per lane group of k_spmv_mr

__device__ __forceinline__ bool stop_now(const int32_t *done) { return done != nullptr && *done != 0; }

template <int G, class T>
__device__ __forceinline__ T group_sum(T v)
{
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Sum over aligned groups of G lanes (G a power of two up to 64) left in the LAST lane of
// each group, by DPP moves (register to register, no LDS): row shifts right by 1, 2, 4
// and 8 within the 16-lane rows (a lane's sum of itself and the lanes below it in the
// row), then for G >= 32 lane 15 of each row added into rows 1 and 3 and for G = 64
// lane 31 into rows 2 and 3. Lanes shifted in from outside a row read 0. Every lane
// must be active. Only the group's last lane holds the group's sum.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_f32(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xf, false));
}
template <int CTRL, int ROWS, class T>
__device__ __forceinline__ T dpp_add(T v)
{
    if constexpr (std::is_same<T, double>::value)
        return v + dpp_f64<CTRL, ROWS>(v);
    else
        return v + dpp_f32<CTRL, ROWS>(v);
}
template <int G, class T>
__device__ __forceinline__ T group_sum_last(T v)
{
    static_assert(G >= 2 && G <= 64 && (G & (G - 1)) == 0, "group of 2..64 lanes");
    v = dpp_add<0x111, 0xf>(v);                       // row_shr:1
    if constexpr (G >= 4) v = dpp_add<0x112, 0xf>(v);  // row_shr:2
    if constexpr (G >= 8) v = dpp_add<0x114, 0xf>(v);  // row_shr:4
    if constexpr (G >= 16) v = dpp_add<0x118, 0xf>(v); // row_shr:8
    if constexpr (G >= 32) v = dpp_add<0x142, 0xa>(v); // row_bcast:15 into rows 1, 3
    if constexpr (G >= 64) v = dpp_add<0x143, 0xc>(v); // row_bcast:31 into rows 2, 3
    return v;
}

// The chip deals a launch's blocks to its 8 XCDs round robin (block b to XCD b % 8),
// and each XCD has its own L2. Renumbering the blocks so that each XCD takes one
// contiguous range of them keeps the rows an XCD processes, and the input entries
// they gather, together in its L2. A bijection of [0, nb).
__device__ __forceinline__ int xcd_block(int b, int nb)
{
    constexpr int kXcd = 8;
    const int q = nb / kXcd, r = nb % kXcd;
    const int x = b % kXcd, i = b / kXcd;
    return x * q + min(x, r) + i;
}

// Fixed-order sum of one value per thread of a 256-thread block; thread 0 gets it.
__device__ __forceinline__ double block_sum256(double v, double *lds4)
{
    v = group_sum<64>(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) lds4[wv] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) s = ((lds4[0] + lds4[1]) + lds4[2]) + lds4[3];
    return s;
}

// The sum of nparts per-block partials, formed exactly as k_reduce_fin forms it, returned
// to every thread of the block (lds5: 5 doubles).
__device__ __forceinline__ double block_total_of(const double *__restrict__ parts, int nparts, double *lds5)
{
    double s = 0.0;
    for (int k = threadIdx.x; k < nparts; k += kBlock) s += parts[k];
    const double t = block_sum256(s, lds5);
    if (threadIdx.x == 0) lds5[4] = t;
    __syncthreads();
    return lds5[4];
}

// The CG scalars on S~ from the inner products: alpha = rr / (p, q), 0 when either is not
// positive or not finite; beta = rr_new / rr_old, 0 when rr_old is not positive or rr_new
// not finite.
__device__ __forceinline__ double cg_alpha_of(double rr, double pq)
{
    return (rr > 0.0 && pq > 0.0 && isfinite(pq) && isfinite(rr)) ? rr / pq : 0.0;
}
__device__ __forceinline__ double cg_beta_of(double rr_old, double rr_new)
{
    return (rr_old > 0.0 && isfinite(rr_new)) ? rr_new / rr_old : 0.0;
}

__device__ void apply_fin(Fin fin, double total, DevState *st)
{
    switch (fin) {
    case FIN_INIT: {
        const double nb = sqrt(total);
        st->nb = nb;
        st->zn = nb;
        if (nb == 0.0) {
            st->done = 1;
            st->status = 0;
        } else if (!isfinite(nb)) {
            st->done = 1;
            st->status = 2;
        }
        break;
    }
    case FIN_ALPHA:
        st->delta = total;
        if (!(total > 0.0) || !isfinite(total)) {
            st->done = 1;
            st->status = 2;
        } else {
            st->alpha = st->rho / total;
        }
        break;
    case FIN_STOP: {
        const double zn = sqrt(total);
        st->zn = zn;
        st->iter += 1;
        if (zn <= st->tol * st->nb) {
            st->done = 1;
            st->status = 0;
        } else if (!isfinite(zn)) {
            st->done = 1;
            st->status = 2;
        } else if (st->iter >= st->maxit) {
            st->done = 1;
            st->status = 1;
        }
        break;
    }
    case FIN_RHO0:
        st->rho = total;
        if (total == 0.0 || !isfinite(total)) {
            st->done = 1;
            st->status = 2;
        }
        break;
    case FIN_BETA:
        if (total == 0.0 || !isfinite(total)) {
            st->done = 1;
            st->status = 2;
        } else {
            st->beta = total / st->rho;
            st->rho = total;
        }
        break;
    case FIN_ATR:
        st->atr = sqrt(total);
        break;
    case FIN_L_BETA1: {
        const double b1 = sqrt(total);
        st->lb = b1;
        st->phibar = b1;
        st->nb = 0.0;
        if (b1 == 0.0) {
            st->done = 1;
            st->status = 0;
        } else if (!isfinite(b1)) {
            st->done = 1;
            st->status = 2;
        }
        break;
    }
    case FIN_L_S1:
        st->snorm = sqrt(total);
        st->nb = st->lb * st->snorm;
        st->zn = st->nb;
        if (st->nb == 0.0) {
            st->done = 1;
            st->status = 0;
        } else if (!isfinite(st->nb)) {
            st->done = 1;
            st->status = 2;
        }
        break;
    case FIN_L_ALPHA0:
        if (!(total > 0.0) || !isfinite(total)) {
            st->done = 1;
            st->status = 2;
        } else {
            st->la = sqrt(total);
            st->rhobar = st->la;
        }
        if (st->maxit == 0 && !st->done) {
            st->done = 1;
            st->status = 1;
        }
        break;
    case FIN_L_BETA:
        st->lb = sqrt(total);
        if (!isfinite(st->lb)) {
            st->done = 1;
            st->status = 2;
        }
        break;
    case FIN_L_SNORM:
        st->snorm = sqrt(total);
        break;
    case FIN_L_ALPHA: {
        const double la = total > 0.0 ? sqrt(total) : 0.0;
        const double rho = sqrt(st->rhobar * st->rhobar + st->lb * st->lb);
        const double c = st->rhobar / rho, sn = st->lb / rho;
        const double theta = sn * la;
        st->rhobar = -c * la;
        const double phi = c * st->phibar;
        st->phibar = sn * st->phibar;
        st->phi_rho = phi / rho;
        st->theta_rho = theta / rho;
        st->la = la;
        st->iter += 1;
        const double est = fabs(st->phibar * c) * st->snorm;
        st->zn = est;
        st->lstop = 0;
        if (!isfinite(est) || !isfinite(total) || !isfinite(rho)) {
            st->lstop = 1;
            st->lstop_status = 2;
        } else if (est <= st->tol * st->nb) {
            st->lstop = 1;
            st->lstop_status = 0;
        } else if (la == 0.0) {
            st->lstop = 1;
            st->lstop_status = total < 0.0 ? 2 : 0;
        } else if (st->iter >= st->maxit) {
            st->lstop = 1;
            st->lstop_status = 1;
        }
        break;
    }
    default:
        break;
    }
}

// ------------------------------------------------------------------ products

template <int G, int EPI, class T>
__global__ __launch_bounds__(kBlock) void k_spmv(DCsrT<T> a, int32_t long_thresh, const T *__restrict__ x,
                                                  T *__restrict__ y, const T *__restrict__ aux,
                                                  double *__restrict__ partials, const int32_t *done)
{
    __shared__ double lds4[4];
    if (stop_now(done)) return;
    constexpr int RPB = kBlock / G;
    const int row = xcd_block(blockIdx.x, gridDim.x) * RPB + threadIdx.x / G;
    const int gl = threadIdx.x % G;
    T sum = 0;
    bool own = false;
    if (row < a.nrows) {
        const int b = a.ptr[row], e = a.ptr[row + 1];
        if (e - b <= long_thresh) {
            own = true;
            for (int k = b + gl; k < e; k += G) sum += a.val[k] * x[a.col[k]];
        }
    }
    sum = group_sum<G>(sum);
    double contrib = 0.0;
    if (own && gl == 0) {
        T out = sum;
        if (EPI == EPI_SUB) out = aux[row] - sum;
        if (EPI == EPI_NEG) out = -sum;
        if (EPI == EPI_ADD) out = aux[row] + sum;
        y[row] = out;
        if (EPI == EPI_SQ) contrib = out * out;
        if (EPI == EPI_WSQ) {
            const double t = aux[row] * out;
            contrib = t * t;
        }
    }
    if constexpr (EPI == EPI_SQ || EPI == EPI_WSQ) {
        const double s = block_sum256(contrib, lds4);
        if (threadIdx.x == 0) partials[xcd_block(blockIdx.x, gridDim.x)] = s;
    }
}

// Two or more rows per lane group (RPT) for rows of up to U*G entries: the
// row pointers of all of a thread's rows, then their first U entries per
// lane (at clamped in-bounds positions, masked values), then the gathers are
// all in flight before any is used, so a block spends one memory latency per
// dependent step for RPT rows instead of one. Rows are interleaved across the
// block so one load instruction covers consecutive rows; entries past U*G go
// through a loop. A row's sum is formed by DPP moves in its group's last lane,
// which stores it. The stop flag is read beside the first loads and masks the
// stores (every load is in bounds either way). Rows longer than long_thresh
// are left to the segment kernel, as in k_spmv. Needs nnz >= 1.
template <int G, int RPT, int U, int EPI, class T>
__global__ __launch_bounds__(kBlock) void k_spmv_mr(DCsrT<T> a, int32_t long_thresh, const T *__restrict__ x,
                                                     T *__restrict__ y, const T *__restrict__ aux,
                                                     double *__restrict__ partials, const int32_t *done)
{
    __shared__ double lds4[4];
    const bool live = !stop_now(done);
    constexpr int RPB = kBlock / G;
    const int gl = threadIdx.x % G;
    const int bid = xcd_block(blockIdx.x, gridDim.x);
    const int base = bid * RPB * RPT + threadIdx.x / G;
    int b[RPT], e[RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int rc = min(base + j * RPB, a.nrows - 1);
        b[j] = a.ptr[rc];
        e[j] = a.ptr[rc + 1];
    }
    int c[RPT][U];
    T v[RPT][U];
#pragma unroll
    for (int j = 0; j < RPT; ++j)
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = b[j] + gl + u * G;
            const int kc = max(min(k, e[j] - 1), 0);
            c[j][u] = a.col[kc];
            const T vv = a.val[kc];
            v[j][u] = k < e[j] ? vv : (T)0;
        }
    T xv[RPT][U];
#pragma unroll
    for (int j = 0; j < RPT; ++j)
#pragma unroll
        for (int u = 0; u < U; ++u) xv[j][u] = x[c[j][u]];
    double contrib = 0.0;
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        T sum = v[j][0] * xv[j][0];
#pragma unroll
        for (int u = 1; u < U; ++u) sum += v[j][u] * xv[j][u];
        for (int k = b[j] + gl + U * G; k < e[j]; k += G) sum += a.val[k] * x[a.col[k]];
        sum = group_sum_last<G>(sum);
        const int row = base + j * RPB;
        if (live && row < a.nrows && e[j] - b[j] <= long_thresh && gl == G - 1) {
            T out = sum;
            if (EPI == EPI_SUB) out = aux[row] - sum;
            if (EPI == EPI_NEG) out = -sum;
            if (EPI == EPI_ADD) out = aux[row] + sum;
            y[row] = out;
            if (EPI == EPI_SQ) contrib += out * out;
            if (EPI == EPI_WSQ) {
                const double t = aux[row] * out;
                contrib += t * t;
            }
        }
    }
    if constexpr (EPI == EPI_SQ || EPI == EPI_WSQ) {
        const double s = block_sum256(contrib, lds4);
        if (threadIdx.x == 0 && live) partials[bid] = s;
    }
}

// One block per segment of a long row.
template <class T>
__global__ __launch_bounds__(kBlock) void k_spmv_seg(DCsrT<T> a, DPlan pl, const T *__restrict__ x,
                                                      T *__restrict__ segpart, const int32_t *done)
{
    __shared__ double lds4[4];
    if (stop_now(done)) return;
    const int s = blockIdx.x;
    const int b = pl.seg_beg[s], e = pl.seg_end[s];
    T sum = 0;
    for (int k = b + threadIdx.x; k < e; k += kBlock) sum += a.val[k] * x[a.col[k]];
    const double t = block_sum256((double)sum, lds4);
    if (threadIdx.x == 0) segpart[s] = (T)t;
}

// Single block: finish the long rows, reduce the partials in index order and
// take the scalar step of Algorithm 1 selected by `fin`.
template <int EPI, class T>
__global__ __launch_bounds__(kBlock) void k_finish(DPlan pl, int32_t nparts, T *__restrict__ y,
                                                    const T *__restrict__ aux, const T *__restrict__ segpart,
                                                    double *__restrict__ partials, Fin fin, DevState *st,
                                                    const int32_t *done)
{
    __shared__ double lds4[4];
    if (stop_now(done)) return;
    for (int i = threadIdx.x; i < pl.nlong; i += kBlock) {
        const int row = pl.long_rows[i];
        T s = 0;
        for (int q = pl.seg_ptr[i]; q < pl.seg_ptr[i + 1]; ++q) s += segpart[q];
        T out = (EPI == EPI_SUB) ? aux[row] - s : (EPI == EPI_NEG ? -s : (EPI == EPI_ADD ? aux[row] + s : s));
        y[row] = out;
        double c = 0.0;
        if (EPI == EPI_SQ) c = out * out;
        if (EPI == EPI_WSQ) {
            const double t = aux[row] * out;
            c = t * t;
        }
        partials[nparts + i] = c;
    }
    if (fin == FIN_NONE) return;
    __syncthreads();
    const int total_n = nparts + pl.nlong;
    double s = 0.0;
    for (int k = threadIdx.x; k < total_n; k += kBlock) s += partials[k];
    const double total = block_sum256(s, lds4);
    if (threadIdx.x == 0) apply_fin(fin, total, st);
}

// Two-stage reductions: per-block partials in a fixed tree, then one block adds them
// in index order and takes the scalar step. (Finishing in the last block of the same
// launch, counted on a device ticket, needs a device-scope release per block, which on
// this chip writes back the block's XCD L2: measured 19.6 us per dot product against
// 9.2 us for the two launches.)
__global__ __launch_bounds__(kBlock) void k_dot(int32_t n, const double *__restrict__ a,
                                                 const double *__restrict__ b, double *__restrict__ partials,
                                                 const int32_t *done)
{
    __shared__ double lds4[4];
    if (stop_now(done)) return;
    double s = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) s += a[i] * b[i];
    const double t = block_sum256(s, lds4);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ __launch_bounds__(kBlock) void k_reduce_fin(int32_t nparts, const double *__restrict__ partials,
                                                        Fin fin, DevState *st, const int32_t *done)
{
    __shared__ double lds4[4];
    if (stop_now(done)) return;
    double s = 0.0;
    for (int k = threadIdx.x; k < nparts; k += kBlock) s += partials[k];
    const double total = block_sum256(s, lds4);
    if (threadIdx.x == 0) apply_fin(fin, total, st);
}

// ------------------------------------------------------------------ vectors

__global__ __launch_bounds__(kBlock) void k_gather(int32_t m, int32_t n, const int32_t *__restrict__ perm,
                                                    const double *__restrict__ b, double *__restrict__ r,
                                                    double *__restrict__ xh, const int32_t *done)
{
    if (stop_now(done)) return;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < m; i += gridDim.x * kBlock) {
        r[i] = b[perm[i]];
        if (i < n) xh[i] = 0.0;
    }
}

__global__ __launch_bounds__(kBlock) void k_update(int32_t n, int32_t m, const double *__restrict__ p,
                                                    double *__restrict__ xh, const double *__restrict__ q,
                                                    double *__restrict__ r, double *f0, double *f1, double *f2,
                                                    double *f3, DevState *st, const int32_t *done)
{
    if (stop_now(done)) return;
    const double alpha = st->alpha;
    const double sent = __longlong_as_double((long long)kSentinel);
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < m; i += gridDim.x * kBlock) {
        r[i] = r[i] - alpha * q[i];
        if (i < n) {
            xh[i] = xh[i] + alpha * p[i];
            if (f0) {
                f0[i] = sent;
                f1[i] = sent;
                f2[i] = sent;
                f3[i] = sent;
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x < 4) st->ticket[threadIdx.x] = 0u;
}

__global__ __launch_bounds__(kBlock) void k_fill(int32_t n, double *f0, double *f1, double *f2, double *f3,
                                                  DevState *st)
{
    const double sent = __longlong_as_double((long long)kSentinel);
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        if (f0) f0[i] = sent;
        if (f1) f1[i] = sent;
        if (f2) f2[i] = sent;
        if (f3) f3[i] = sent;
    }
    if (blockIdx.x == 0 && threadIdx.x < 4) st->ticket[threadIdx.x] = 0u;
    if (blockIdx.x == 0 && threadIdx.x == 0) st->err = 0;
}

// Sentinel-fill two more sync-free outputs and clear tickets 0 and 1 (between
// the sweeps of one preconditioner application that needs more than four).
__global__ __launch_bounds__(kBlock) void k_refill(int32_t n, double *f0, double *f1, DevState *st,
                                                    const int32_t *done)
{
    if (stop_now(done)) return;
    const double sent = __longlong_as_double((long long)kSentinel);
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        f0[i] = sent;
        f1[i] = sent;
    }
    if (blockIdx.x == 0 && threadIdx.x < 2) st->ticket[threadIdx.x] = 0u;
}

__global__ __launch_bounds__(kBlock) void k_pupdate(int32_t n, const double *__restrict__ h, double *__restrict__ p,
                                                     const DevState *st, int32_t first, const int32_t *done)
{
    if (stop_now(done)) return;
    const double beta = first ? 0.0 : st->beta;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
        p[i] = first ? h[i] : h[i] + beta * p[i];
}

__global__ __launch_bounds__(kBlock) void k_scale_out(int32_t n, const double *__restrict__ xh,
                                                       const double *__restrict__ colnorm, double *__restrict__ x)
{
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) x[i] = xh[i] / colnorm[i];
}

__global__ __launch_bounds__(kBlock) void k_residual(int32_t m, const int32_t *__restrict__ perm,
                                                      const double *__restrict__ b, const double *__restrict__ ax,
                                                      double *__restrict__ r)
{
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < m; i += gridDim.x * kBlock) r[i] = b[perm[i]] - ax[i];
}

__global__ __launch_bounds__(kBlock) void k_copy(int32_t n, const double *__restrict__ src, double *__restrict__ dst,
                                                  const int32_t *done)
{
    if (stop_now(done)) return;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) dst[i] = src[i];
}

__global__ __launch_bounds__(kBlock) void k_add(int32_t n, const double *__restrict__ src, double *__restrict__ dst,
                                                 const int32_t *done)
{
    if (stop_now(done)) return;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) dst[i] = dst[i] + src[i];
}

__global__ __launch_bounds__(kBlock) void k_lsqr_t(int32_t m, const double *__restrict__ u, double *__restrict__ t,
                                                   double *__restrict__ partials, const DevState *st,
                                                   const int32_t *done)
{
    __shared__ double lds4[4];
    if (stop_now(done)) return;
    const double a = st->la;
    double sq = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < m; i += gridDim.x * kBlock) {
        const double v = t[i] - a * u[i];
        t[i] = v;
        sq += v * v;
    }
    const double tot = block_sum256(sq, lds4);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlock) void k_lsqr_scale(int32_t m, const double *__restrict__ in,
                                                       double *__restrict__ out, const DevState *st,
                                                       const int32_t *done)
{
    if (stop_now(done)) return;
    const double d = st->lb;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < m; i += gridDim.x * kBlock) out[i] = d > 0.0 ? in[i] / d : in[i];
}

__global__ __launch_bounds__(kBlock) void k_lsqr_s(int32_t n, double *__restrict__ sv, const double *__restrict__ Mv,
                                                   const double *__restrict__ colnorm, double *__restrict__ partials,
                                                   const DevState *st, const int32_t *done)
{
    __shared__ double lds4[4];
    if (stop_now(done)) return;
    const double b = st->lb;
    double sq = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const double v = Mv ? sv[i] - b * Mv[i] : sv[i];
        sv[i] = v;
        const double w = colnorm[i] * v;
        sq += w * w;
    }
    const double tot = block_sum256(sq, lds4);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlock) void k_lsqr_v(int32_t n, const double *__restrict__ h, const double *__restrict__ sv,
                                                   double *__restrict__ xh, double *__restrict__ v,
                                                   double *__restrict__ Mv, double *__restrict__ w, int32_t init,
                                                   const DevState *st, const int32_t *done)
{
    if (stop_now(done)) return;
    const double la = st->la, pr = st->phi_rho, tr = st->theta_rho;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        if (init) {
            const double vi = h[i] / la;
            v[i] = vi;
            Mv[i] = sv[i] / la;
            w[i] = vi;
            continue;
        }
        const double wo = w[i];
        xh[i] = xh[i] + pr * wo;
        if (la > 0.0) {
            const double vi = h[i] / la;
            v[i] = vi;
            Mv[i] = sv[i] / la;
            w[i] = vi - tr * wo;
        }
    }
}

__global__ void k_lsqr_commit(DevState *st)
{
    if (threadIdx.x == 0 && st->done == 0 && st->lstop) {
        st->status = st->lstop_status;
        st->done = 1;
    }
}

__global__ __launch_bounds__(kBlock) void k_cg_init(int32_t k, const double *__restrict__ u, double *__restrict__ w,
                                                    double *__restrict__ res, double *__restrict__ p,
                                                    const int32_t *done)
{
    if (stop_now(done)) return;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < k; i += gridDim.x * kBlock) {
        w[i] = 0.0;
        res[i] = u[i];
        p[i] = u[i];
    }
}

// The CG steps' scalars are formed by every block from the per-block partials of the
// previous launches (pq: (p, q); rr_old / rr_new: (res, z) of the previous / this step), in
// the order of k_reduce_fin, so no single-block launch sits between the steps' kernels.
__global__ __launch_bounds__(kBlock) void k_cg_update(int32_t k, const double *__restrict__ p,
                                                      const double *__restrict__ q, double *__restrict__ w,
                                                      double *__restrict__ res, int32_t nparts,
                                                      const double *__restrict__ pq_parts,
                                                      const double *__restrict__ rr_parts, const int32_t *done)
{
    __shared__ double lds_a[5], lds_b[5];
    if (stop_now(done)) return;
    const double a = cg_alpha_of(block_total_of(rr_parts, nparts, lds_b), block_total_of(pq_parts, nparts, lds_a));
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < k; i += gridDim.x * kBlock) {
        w[i] = w[i] + a * p[i];
        res[i] = res[i] - a * q[i];
    }
}

// w += alpha p, res -= alpha q, and the per-block partials of res . res (the grid of
// k_dot, so the sums are those of a separate dot product)
__global__ __launch_bounds__(kBlock) void k_cg_update_dot(int32_t k, const double *__restrict__ p,
                                                          const double *__restrict__ q, double *__restrict__ w,
                                                          double *__restrict__ res, int32_t nparts,
                                                          const double *__restrict__ pq_parts,
                                                          const double *__restrict__ rr_old, double *__restrict__ partials,
                                                          const int32_t *done)
{
    __shared__ double lds4[4];
    __shared__ double lds_a[5], lds_b[5];
    if (stop_now(done)) return;
    const double a = cg_alpha_of(block_total_of(rr_old, nparts, lds_b), block_total_of(pq_parts, nparts, lds_a));
    double s = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < k; i += gridDim.x * kBlock) {
        w[i] = w[i] + a * p[i];
        const double r = res[i] - a * q[i];
        res[i] = r;
        s += r * r;
    }
    const double t = block_sum256(s, lds4);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// Jacobi-preconditioned CG on S~ (d = diag(S~)): set-up, and the update with z = res / d and
// the per-block partials of res . z (the grid of k_dot)
__global__ __launch_bounds__(kBlock) void k_pcg_init(int32_t k, const double *__restrict__ u,
                                                     const double *__restrict__ d, double *__restrict__ w,
                                                     double *__restrict__ res, double *__restrict__ z,
                                                     double *__restrict__ p, const int32_t *done)
{
    if (stop_now(done)) return;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < k; i += gridDim.x * kBlock) {
        const double ui = u[i];
        const double zi = ui / d[i];
        w[i] = 0.0;
        res[i] = ui;
        z[i] = zi;
        p[i] = zi;
    }
}

__global__ __launch_bounds__(kBlock) void k_pcg_update_dot(int32_t k, const double *__restrict__ p,
                                                           const double *__restrict__ q, const double *__restrict__ d,
                                                           double *__restrict__ w, double *__restrict__ res,
                                                           double *__restrict__ z, int32_t nparts,
                                                           const double *__restrict__ pq_parts,
                                                           const double *__restrict__ rr_old, double *__restrict__ partials,
                                                           const int32_t *done)
{
    __shared__ double lds4[4];
    __shared__ double lds_a[5], lds_b[5];
    if (stop_now(done)) return;
    const double a = cg_alpha_of(block_total_of(rr_old, nparts, lds_b), block_total_of(pq_parts, nparts, lds_a));
    double s = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < k; i += gridDim.x * kBlock) {
        w[i] = w[i] + a * p[i];
        const double r = res[i] - a * q[i];
        res[i] = r;
        const double zi = r / d[i];
        z[i] = zi;
        s += r * zi;
    }
    const double t = block_sum256(s, lds4);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ __launch_bounds__(kBlock) void k_cg_dir(int32_t k, const double *__restrict__ res, double *__restrict__ p,
                                                   int32_t nparts, const double *__restrict__ rr_old,
                                                   const double *__restrict__ rr_new, const int32_t *done)
{
    __shared__ double lds_a[5], lds_b[5];
    if (stop_now(done)) return;
    const double bt = cg_beta_of(block_total_of(rr_old, nparts, lds_a), block_total_of(rr_new, nparts, lds_b));
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < k; i += gridDim.x * kBlock) p[i] = res[i] + bt * p[i];
}

// Chebyshev steps on S~ w = u (RSILU_S_CHEB): the set-up r = omega u, d = r / theta, w = 0
// (omega = 1 unless the degree is too low for the interval), and one step's update once
// q = Y~ (Y~^T d) is formed: w += d, r -= d + q, d = c1 d + c2 r; the last step also
// writes w to out.
template <class T>
__global__ __launch_bounds__(kBlock) void k_cheb_init(int32_t k, const T *__restrict__ u, T *__restrict__ r,
                                                      T *__restrict__ d, T *__restrict__ w, T theta, T omega,
                                                      const int32_t *done)
{
    if (stop_now(done)) return;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < k; i += gridDim.x * kBlock) {
        const T ri = omega * u[i];
        r[i] = ri;
        d[i] = ri / theta;
        w[i] = (T)0;
    }
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_cheb_update(int32_t k, const T *__restrict__ q, T *__restrict__ r,
                                                        T *__restrict__ d, T *__restrict__ w, T *__restrict__ out,
                                                        T c1, T c2, const int32_t *done)
{
    if (stop_now(done)) return;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < k; i += gridDim.x * kBlock) {
        const T di = d[i];
        const T wi = w[i] + di;
        const T ri = r[i] - (di + q[i]);
        w[i] = wi;
        r[i] = ri;
        d[i] = c1 * di + c2 * ri;
        if (out) out[i] = wi;
    }
}

template <class A, class B>
__global__ __launch_bounds__(kBlock) void k_cvt(int32_t n, const A *__restrict__ in, B *__restrict__ out,
                                                 const int32_t *done)
{
    if (stop_now(done)) return;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) out[i] = (B)in[i];
}

// ------------------------------------------------------------------ triangular solves

template <int G>
__global__ __launch_bounds__(kBlock) void k_trsv_syncfree(DTri t, const double *__restrict__ rhs, double *x,
                                                           const double *__restrict__ add, double *__restrict__ y2,
                                                           DevState *st, int32_t tk, const int32_t *done)
{
    if (stop_now(done)) return;
    const int lane = threadIdx.x & 63;
    const int grp = lane / G, gl = lane % G;
    unsigned long long *xb = reinterpret_cast<unsigned long long *>(x);
    for (;;) {
        unsigned int c = 0;
        if (lane == 0) c = atomicAdd(&st->ticket[tk], 1u);
        c = __shfl(c, 0);
        if (c >= (unsigned int)t.nchunks) break;
        const int beg = t.chunk[c], end = t.chunk[c + 1];
        const int idx = beg + grp;
        const bool act = idx < end;
        const int row = act ? t.rows[idx] : 0;
        double sum = 0.0;
        if (act) {
            const int b = t.a.ptr[row], e = t.a.ptr[row + 1];
            for (int k = b + gl; k < e; k += G) {
                const int cc = t.a.col[k];
                const double v = t.a.val[k];
                unsigned long long bits;
                int spins = 0;
                for (;;) {
                    bits = __hip_atomic_load(xb + cc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (bits != kSentinel) break;
                    ++spins;
                    // bounded wait: past the limit, or once any wave has given up,
                    // publish NaN and stop the solve (every later kernel sees done)
                    if (spins > kSpinLimit ||
                        ((spins & 255) == 0 &&
                         __hip_atomic_load(&st->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) {
                        __hip_atomic_store(&st->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        __hip_atomic_store(&st->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        bits = kQuietNaN;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                sum += v * __longlong_as_double((long long)bits);
            }
        }
        sum = group_sum<G>(sum);
        if (act && gl == 0) {
            double r = rhs[row] - sum;
            if (t.diag) r = r / t.diag[row];
            __hip_atomic_store(xb + row, (unsigned long long)__double_as_longlong(r), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            if (y2) y2[row] = add[row] + r;
        }
    }
}

template <int G, class T>
__global__ __launch_bounds__(kBlock) void k_trsv_level(DTriT<T> t, int32_t beg, int32_t end, const T *__restrict__ rhs,
                                                        T *x, const T *__restrict__ add, T *__restrict__ y2,
                                                        const int32_t *done)
{
    if (stop_now(done)) return;
    constexpr int RPB = kBlock / G;
    const int idx = beg + blockIdx.x * RPB + threadIdx.x / G;
    const int gl = threadIdx.x % G;
    const bool act = idx < end;
    const int row = act ? t.rows[idx] : 0;
    T sum = 0;
    if (act) {
        const int b = t.a.ptr[row], e = t.a.ptr[row + 1];
        for (int k = b + gl; k < e; k += G) sum += t.a.val[k] * x[t.a.col[k]];
    }
    sum = group_sum<G>(sum);
    if (act && gl == 0) {
        T r = rhs[row] - sum;
        if (t.diag) r = r / t.diag[row];
        x[row] = r;
        if (y2) y2[row] = add[row] + r;
    }
}

// Single-workgroup sweep over nb consecutive batches of narrow levels (the
// hybrid schedule's runs). Every row reads its inputs from LDS: results of its
// own batch, of the previous batch, or the batch's older inputs gathered from
// x. While a batch's levels are solved (LDS reads, global stores only), the
// next batch's blob, its slice of the level-ordered right-hand side (and
// addend) and its older inputs are already in flight into registers; they are
// written to LDS after the batch's last level. The older inputs of batch b+1
// lie in batches <= b-1 or earlier launches, so they are final when batch b
// starts; the list of them travels in batch b's blob.
// Blob layout: int32 hdr[kSweepHdr] = {nlev, npos, nent, next, has_diag,
// cur_base, p0, size, next_size, next_npos, next_next, nchunk},
// lev_off[nlev+1], lev_chunk[nlev+1], rowid[npos], ext_idx[next],
// next_ext[kSweepExt], uint16 rchunk[npos+1], cstart[nchunk+1], eslot[nent],
// then (16-aligned) T eval[nent], rdiag[npos] (reciprocal diagonal; T = double, or float for the
// FP32 preconditioner), and for the segmented scheme uint16 crow[nchunk] (the
// position of the chunk's row in the batch, bit 15 set on the row's last chunk;
// 0x7fff on padding chunks). A row's entries are cut into chunks of at most
// kSweepChunk; eslot indexes the LDS window xw = [even batches' results | odd
// batches' results | older inputs].
template <class T>
__device__ __forceinline__ void load_chunk(const unsigned char *vb, int c, T &a, T &b, T &cc, T &d);
template <>
__device__ __forceinline__ void load_chunk<double>(const unsigned char *vb, int c, double &a, double &b, double &cc,
                                                   double &d)
{
    const double2 *v = reinterpret_cast<const double2 *>(vb);
    const double2 p = v[2 * c], q = v[2 * c + 1];
    a = p.x;
    b = p.y;
    cc = q.x;
    d = q.y;
}
template <>
__device__ __forceinline__ void load_chunk<float>(const unsigned char *vb, int c, float &a, float &b, float &cc,
                                                  float &d)
{
    const float4 p = reinterpret_cast<const float4 *>(vb)[c];
    a = p.x;
    b = p.y;
    cc = p.z;
    d = p.w;
}

// Segmented inclusive sum over the 16-lane groups of a wavefront: lanes with
// equal key form contiguous segments inside one group; after shifts of 1, 2, 4
// and 8 lanes each lane holds the sum of its segment up to itself, so a
// segment's last lane holds the segment's sum. Every lane must be active.
template <int D>
__device__ __forceinline__ double shr_f64(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x110 + D, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x110 + D, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int D>
__device__ __forceinline__ float shr_f32(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x110 + D, 0xf, 0xf, false));
}
template <int D>
__device__ __forceinline__ int shr_key(int k)
{
    return __builtin_amdgcn_update_dpp(-1, k, 0x110 + D, 0xf, 0xf, false);
}
template <class T, int D>
__device__ __forceinline__ T seg_step(T v, int key)
{
    T o;
    if constexpr (std::is_same<T, double>::value)
        o = shr_f64<D>(v);
    else
        o = shr_f32<D>(v);
    return shr_key<D>(key) == key ? v + o : v;
}
// Segments longer than 16 lanes (they never cross the wavefront) continue over
// the 16-lane groups with the broadcast of lane 15 of each group to the next
// (groups 1 and 3) and of lane 31 to groups 2 and 3.
template <int CTRL, int ROWS>
__device__ __forceinline__ double bcast_f64(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ float bcast_f32(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xf, false));
}
template <class T, int CTRL, int ROWS>
__device__ __forceinline__ T seg_bcast(T v, int key)
{
    T o;
    if constexpr (std::is_same<T, double>::value)
        o = bcast_f64<CTRL, ROWS>(v);
    else
        o = bcast_f32<CTRL, ROWS>(v);
    return __builtin_amdgcn_update_dpp(-1, key, CTRL, ROWS, 0xf, false) == key ? v + o : v;
}

// span: the longest segment in lanes (uniform); shifts at or beyond it add nothing.
// WIDE: segments may span the wavefront's four 16-lane groups.
template <class T, bool WIDE>
__device__ __forceinline__ T seg_scan(T v, int key, int span)
{
    if (span > 1) v = seg_step<T, 1>(v, key);
    if (span > 2) v = seg_step<T, 2>(v, key);
    if (span > 4) v = seg_step<T, 4>(v, key);
    if (span > 8) v = seg_step<T, 8>(v, key);
    if constexpr (WIDE) {
        if (span > 16) {
            v = seg_bcast<T, 0x142, 0xa>(v, key);  // row_bcast:15 into groups 1 and 3
            v = seg_bcast<T, 0x143, 0xc>(v, key);  // row_bcast:31 into groups 2 and 3
        }
    }
    return v;
}

template <class T, int SCHEME>
__global__ __launch_bounds__(kSweepThreads) void k_trsv_sweep(const unsigned char *__restrict__ blob, int64_t off,
                                                               int32_t size, int32_t npos_first, int32_t p0,
                                                               int32_t nb, const T *__restrict__ rhs_lo, T *x,
                                                               const T *__restrict__ add_lo, T *y2,
                                                               const int32_t *done)
{
    constexpr int VB = (kSweepBlob / 16 + kSweepThreads - 1) / kSweepThreads;
    constexpr int VP = (kSweepPos + kSweepThreads - 1) / kSweepThreads;
    constexpr int VE = (kSweepExt + kSweepThreads - 1) / kSweepThreads;
    __shared__ __attribute__((aligned(16))) unsigned char sb[kSweepBlob];
    __shared__ T xw[2 * kSweepPos + kSweepExt + 8];
    __shared__ T rl[kSweepPos];
    __shared__ T al[kSweepPos];
    __shared__ T prod[kSweepLevEnt];
    if (stop_now(done)) return;
    const int tid = threadIdx.x;
    if (tid == 0) xw[kSweepZeroSlot] = 0;
    static_assert(VB <= 5 && VP == 2 && VE == 2, "staging registers are written out for these limits");
    // Staging registers for the next batch. Loads are unconditional with
    // clamped indices (always in bounds: a batch has at least one row and one
    // blob vector) so the values stay in registers; only LDS writes are
    // predicated.
    uint4 rb0, rb1, rb2, rb3, rb4;
    T rr0, rr1, ra0, ra1, re0, re1;
    uint4 *sb4 = reinterpret_cast<uint4 *>(sb);
    const int t0 = tid, t1 = tid + kSweepThreads, t2 = tid + 2 * kSweepThreads, t3 = tid + 3 * kSweepThreads,
              t4 = tid + 4 * kSweepThreads;
#define RSILU_LOAD_BATCH(BOFF, NVEC, BP0, BNPOS)                                        \
    {                                                                                   \
        const uint4 *src_ = reinterpret_cast<const uint4 *>(blob + (BOFF));             \
        const int lastv_ = (NVEC) - 1, lastp_ = (BNPOS) - 1;                            \
        rb0 = src_[min(t0, lastv_)];                                                    \
        rb1 = src_[min(t1, lastv_)];                                                    \
        rb2 = src_[min(t2, lastv_)];                                                    \
        rb3 = src_[min(t3, lastv_)];                                                    \
        if (VB > 4) rb4 = src_[min(t4, lastv_)];                                        \
        rr0 = rhs_lo[(BP0) + min(t0, lastp_)];                                          \
        rr1 = rhs_lo[(BP0) + min(t1, lastp_)];                                          \
        ra0 = y2 ? add_lo[(BP0) + min(t0, lastp_)] : (T)0;                              \
        ra1 = y2 ? add_lo[(BP0) + min(t1, lastp_)] : (T)0;                              \
    }
#define RSILU_LOAD_EXT(LIST, CNT)                                                       \
    {                                                                                   \
        const int lastj_ = (CNT) - 1;                                                   \
        re0 = (CNT) > 0 ? x[(LIST)[min(t0, lastj_)]] : (T)0;                            \
        re1 = (CNT) > 0 ? x[(LIST)[min(t1, lastj_)]] : (T)0;                            \
    }
#define RSILU_STORE_BATCH(NVEC, BNPOS)                                                  \
    {                                                                                   \
        if (t0 < (NVEC)) sb4[t0] = rb0;                                                 \
        if (t1 < (NVEC)) sb4[t1] = rb1;                                                 \
        if (t2 < (NVEC)) sb4[t2] = rb2;                                                 \
        if (t3 < (NVEC)) sb4[t3] = rb3;                                                 \
        if (VB > 4 && t4 < (NVEC)) sb4[t4] = rb4;                                       \
        if (t0 < (BNPOS)) {                                                             \
            rl[t0] = rr0;                                                               \
            al[t0] = ra0;                                                               \
        }                                                                               \
        if (t1 < (BNPOS)) {                                                             \
            rl[t1] = rr1;                                                               \
            al[t1] = ra1;                                                               \
        }                                                                               \
    }
#define RSILU_STORE_EXT(CNT)                                                            \
    {                                                                                   \
        if (t0 < (CNT)) xw[2 * kSweepPos + t0] = re0;                                   \
        if (t1 < (CNT)) xw[2 * kSweepPos + t1] = re1;                                   \
    }

    // prologue: the first batch, then its own older inputs
    RSILU_LOAD_BATCH(off, size >> 4, p0, npos_first)
    RSILU_STORE_BATCH(size >> 4, npos_first)
    __syncthreads();
    {
        const int32_t *hdr = reinterpret_cast<const int32_t *>(sb);
        const int32_t *own_ext = hdr + kSweepHdr + 2 * (hdr[0] + 1) + hdr[1];
        RSILU_LOAD_EXT(own_ext, hdr[3])
        RSILU_STORE_EXT(hdr[3])
    }
    __syncthreads();

    for (int b = 0; b < nb; ++b) {
        const int32_t *hdr = reinterpret_cast<const int32_t *>(sb);
        const int nlev = hdr[0], npos = hdr[1], nent = hdr[2], next = hdr[3], hd = hdr[4], cur = hdr[5];
        const int size_next = hdr[8], npos_next = hdr[9], nnext = hdr[10], nchunk = hdr[11];
        const int32_t *lev_off = hdr + kSweepHdr;
        const int32_t *lev_chunk = lev_off + nlev + 1;
        const int32_t *rowid = lev_chunk + nlev + 1;
        const int32_t *ext_idx = rowid + npos;
        const int32_t *next_ext = ext_idx + next;
        const uint16_t *rchunk = reinterpret_cast<const uint16_t *>(next_ext + kSweepExt);
        const int o_slot = ((int)(reinterpret_cast<const unsigned char *>(rchunk + npos + 1) - sb) + 7) & ~7;
        const int o_val = (o_slot + 8 * nchunk + 15) & ~15;
        const uint2 *eslot4 = reinterpret_cast<const uint2 *>(sb + o_slot);  // 4 uint16 slots per chunk
        const unsigned char *evals = sb + o_val;                             // 4 values per chunk
        const T *dg = reinterpret_cast<const T *>(sb + o_val + 4 * (int)sizeof(T) * nchunk);
        (void)nent;
        // level offsets live in the lanes of every wavefront (nlev <= 63)
        const int lane = tid & 63;
        const int lo_v = lane <= nlev ? lev_off[lane] : 0;
        const int lc_v = lane <= nlev ? lev_chunk[lane] : 0;
        const bool more = b + 1 < nb;
        const int64_t noff = off + size;
        const int np0 = p0 + npos;
        if (more) {
            RSILU_LOAD_BATCH(noff, size_next >> 4, np0, npos_next)
            RSILU_LOAD_EXT(next_ext, nnext)
        }
        if constexpr (SCHEME == kSchemeSegmented || SCHEME == kSchemeSegmentedWide) {
            // One phase per level, one chunk per thread: a row's chunks sit on
            // consecutive lanes of one 16-lane group (the setup pads the level so;
            // in the wide variant a row of 17 to 64 chunks stays inside the
            // wavefront instead), the chunk sums are combined by a segmented
            // inclusive scan over DPP row shifts (1, 2, 4, 8; then the lane 15 and
            // lane 31 broadcasts in the wide variant), and the row's last lane
            // solves the row.
            (void)nent;
            const uint32_t zzs = (uint32_t)kSweepZeroSlot | ((uint32_t)kSweepZeroSlot << 16);
            const uint16_t *crow = reinterpret_cast<const uint16_t *>(sb + o_val + 4 * (int)sizeof(T) * nchunk +
                                                                      (hd ? (int)sizeof(T) * npos : 0));
            const int wbase = __builtin_amdgcn_readfirstlane(tid & ~63);
            for (int L = 0; L < nlev; ++L) {
                const int lc = __builtin_amdgcn_readlane(lc_v, L);
                const int ca = lc & 0xffff, cb = __builtin_amdgcn_readlane(lc_v, L + 1) & 0xffff;
                const int span = lc >> 16;  // the level's longest row in chunks (lanes)
                if (ca + wbase < cb) {  // the wavefront holds chunks of this level
                    const int c = ca + tid;
                    const bool has = c < cb;
                    const int cc = min(c, cb - 1);
                    // LDS returns in issue order: the slot words first, then the
                    // gathers they address, and only then the row data that the
                    // row's last lane needs after the scan.
                    const uint2 sl0 = eslot4[cc];
                    const int cr = crow[cc];
                    T v0, v1, v2, v3;
                    load_chunk<T>(evals, cc, v0, v1, v2, v3);
                    const uint2 sl = has ? sl0 : make_uint2(zzs, zzs);
                    const T g0 = xw[sl.x & 0xffffu], g1 = xw[sl.x >> 16];
                    const T g2 = xw[sl.y & 0xffffu], g3 = xw[sl.y >> 16];
                    __builtin_amdgcn_sched_barrier(0);
                    const int key = has ? (cr & 0x7fff) : 0xffff;
                    const bool last = has && (cr & 0x8000) != 0;
                    const int pp = min(cr & 0x7fff, npos - 1);
                    const T rhs = rl[pp];
                    const T dgv = hd ? dg[pp] : (T)1;
                    const T add = al[pp];
                    const int row = rowid[pp];
                    T t = v0 * g0;
                    t += v1 * g1;
                    t += v2 * g2;
                    t += v3 * g3;
                    T v = has ? t : (T)0;
                    v = seg_scan<T, SCHEME == kSchemeSegmentedWide>(v, key, span);
                    if (last) {
                        const int p = cr & 0x7fff;
                        T r = rhs - v;
                        if (hd) r = r * dgv;  // reciprocal of the diagonal, stored by the setup
                        xw[cur + p] = r;
                        x[row] = r;
                        if (y2) y2[row] = add + r;
                    }
                }
                __syncthreads();
            }
        } else if constexpr (SCHEME == kSchemeRows) {
            constexpr int NR = kRowsRound;
            // One phase per level: one row per thread. A thread loads its row's
            // chunks NR at a time (all slot words, then all values, then all
            // gathers, so each gather waits only for its own slot word), forms
            // the chunk sums and adds them to the row sum in chunk order (the
            // order of the two-phase scheme); one barrier per level publishes
            // the results.
            (void)lc_v;
            (void)nent;
            const uint32_t zz = (uint32_t)kSweepZeroSlot | ((uint32_t)kSweepZeroSlot << 16);
            const int wbase = __builtin_amdgcn_readfirstlane(tid & ~63);
            for (int L = 0; L < nlev; ++L) {
                const int pa = __builtin_amdgcn_readlane(lo_v, L), pb = __builtin_amdgcn_readlane(lo_v, L + 1);
                if (pa + wbase < pb) {  // the wavefront holds rows of this level
                    const int p = pa + tid;
                    const int pp = min(p, pb - 1);  // lanes past the level repeat its last row
                    const int r0 = rchunk[pp], r1 = rchunk[pp + 1];
                    const T rhs = rl[pp];
                    const T dgv = hd ? dg[pp] : (T)1;
                    const T add = al[pp];
                    const int row = rowid[pp];
                    T s = 0;
                    for (int q = r0; q < r1; q += NR) {
                        uint2 sl[NR];
                        T v[NR][4];
                        bool ok[NR];
#pragma unroll
                        for (int j = 0; j < NR; ++j) {
                            ok[j] = q + j < r1;
                            sl[j] = eslot4[min(q + j, r1 - 1)];
                        }
                        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                        for (int j = 0; j < NR; ++j)
                            load_chunk<T>(evals, min(q + j, r1 - 1), v[j][0], v[j][1], v[j][2], v[j][3]);
                        __builtin_amdgcn_sched_barrier(0);
                        T g[NR][4];
#pragma unroll
                        for (int j = 0; j < NR; ++j) {
                            const uint2 t = ok[j] ? sl[j] : make_uint2(zz, zz);
                            g[j][0] = xw[t.x & 0xffffu];
                            g[j][1] = xw[t.x >> 16];
                            g[j][2] = xw[t.y & 0xffffu];
                            g[j][3] = xw[t.y >> 16];
                        }
                        T cs[NR];
#pragma unroll
                        for (int j = 0; j < NR; ++j) {
                            T t = v[j][0] * g[j][0];
                            t += v[j][1] * g[j][1];
                            t += v[j][2] * g[j][2];
                            t += v[j][3] * g[j][3];
                            cs[j] = ok[j] ? t : (T)0;
                        }
#pragma unroll
                        for (int j = 0; j < NR; ++j) s += cs[j];
                    }
                    T r = rhs - s;
                    if (hd) r = r * dgv;  // reciprocal of the diagonal, stored by the setup
                    if (p < pb) {
                        xw[cur + p] = r;
                        x[row] = r;
                        if (y2) y2[row] = add + r;
                    }
                }
                __syncthreads();
            }
        } else {
        // Level loop: one chunk and one row per thread. Phase 1 forms the
        // chunk sums (four entries each, padded with the zero slot so the
        // loads are branch-free); phase 2 adds each row's chunk sums, solves
        // the row and publishes it in LDS for later levels.
        struct Meta {
            int cidx;      // chunk index in the level (-1: none)
            uint2 sl;      // four LDS slots
            T v0, v1, v2, v3;
            int pidx;      // row position in the batch (-1: none)
            int c0, nch;   // the row's chunks, relative to the level
            T rhs, dg, add;
            int row;
        };
        auto fetch = [&](int L) {
            Meta m;
            const int pa = __builtin_amdgcn_readlane(lo_v, L), pb = __builtin_amdgcn_readlane(lo_v, L + 1);
            const int ca = __builtin_amdgcn_readlane(lc_v, L), cb = __builtin_amdgcn_readlane(lc_v, L + 1);
            const int c = ca + tid;
            m.cidx = -1;
            if (c < cb) {
                m.cidx = tid;
                m.sl = eslot4[c];
                load_chunk<T>(evals, c, m.v0, m.v1, m.v2, m.v3);
            }
            const int p = pa + tid;
            m.pidx = -1;
            if (p < pb) {
                m.pidx = p;
                m.c0 = rchunk[p] - ca;
                m.nch = rchunk[p + 1] - rchunk[p];
                m.rhs = rl[p];
                m.dg = hd ? dg[p] : (T)1;
                m.add = y2 ? al[p] : (T)0;
                m.row = rowid[p];
            }
            return m;
        };
        for (int L = 0; L < nlev; ++L) {
            const Meta m = fetch(L);
            // chunk sums: kSweepChunk entries of one row (padded with the zero slot)
            if (m.cidx >= 0) {
                T s = m.v0 * xw[m.sl.x & 0xffffu];
                s += m.v1 * xw[m.sl.x >> 16];
                s += m.v2 * xw[m.sl.y & 0xffffu];
                s += m.v3 * xw[m.sl.y >> 16];
                prod[m.cidx] = s;
            }
            __syncthreads();
            // row sums over the row's chunk sums (up to four read at once)
            if (m.pidx >= 0) {
                T s = 0;
                if (m.nch > 0) {
                    const int c0 = m.c0, last = m.c0 + m.nch - 1;
                    const T a0 = prod[c0], a1 = prod[min(c0 + 1, last)], a2 = prod[min(c0 + 2, last)],
                            a3 = prod[min(c0 + 3, last)];
                    s = a0;
                    s = m.nch > 1 ? s + a1 : s;
                    s = m.nch > 2 ? s + a2 : s;
                    s = m.nch > 3 ? s + a3 : s;
                    for (int c = c0 + 4; c <= last; ++c) s += prod[c];
                }
                T r = m.rhs - s;
                if (hd) r = r * m.dg;  // reciprocal of the diagonal, stored by the setup
                xw[cur + m.pidx] = r;
                x[m.row] = r;
                if (y2) y2[m.row] = m.add + r;
            }
            __syncthreads();
        }
        }
        if (more) {
            RSILU_STORE_BATCH(size_next >> 4, npos_next)
            RSILU_STORE_EXT(nnext)
            off = noff;
            size = size_next;
            p0 = np0;
            __syncthreads();
        }
    }
#undef RSILU_LOAD_BATCH
#undef RSILU_LOAD_EXT
#undef RSILU_STORE_BATCH
#undef RSILU_STORE_EXT
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_gather_lo(int32_t n, const int32_t *__restrict__ rows,
                                                       const T *__restrict__ src, T *__restrict__ dst,
                                                       const T *__restrict__ src2, T *__restrict__ dst2,
                                                       const int32_t *done)
{
    if (stop_now(done)) return;
    for (int p = blockIdx.x * kBlock + threadIdx.x; p < n; p += gridDim.x * kBlock) {
        const int r = rows[p];
        dst[p] = src[r];
        if (src2) dst2[p] = src2[r];
    }
}

// ------------------------------------------------------------------ dense S~ (Section 3.2)

__device__ __forceinline__ long long pk(long long i, long long j) { return i * (i + 1) / 2 + j; }

// Solve L L^T w = u in place (w holds u on entry), L packed lower by rows.
// 64-row panels: the diagonal block is solved by one wavefront from LDS, the
// rest of the vector is updated by the whole block.
__global__ __launch_bounds__(1024) void k_dense_chol(int32_t k, const double *__restrict__ L, double *w,
                                                      const int32_t *done)
{
    __shared__ double D[64][65];
    __shared__ double yp[64];
    if (stop_now(done)) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int p0 = 0; p0 < k; p0 += 64) {
        const int pb = min(64, k - p0);
        for (int e = tid; e < 64 * 64; e += 1024) {
            const int i = e >> 6, j = e & 63;
            if (i < pb && j <= i) D[i][j] = L[pk(p0 + i, p0 + j)];
        }
        if (tid < pb) yp[tid] = w[p0 + tid];
        __syncthreads();
        if (wv == 0) {
            double yi = lane < pb ? yp[lane] : 0.0;
            for (int j = 0; j < pb; ++j) {
                const double yj = __shfl(yi, j) / D[j][j];
                if (lane == j)
                    yi = yj;
                else if (lane > j && lane < pb)
                    yi -= D[lane][j] * yj;
            }
            if (lane < pb) {
                yp[lane] = yi;
                w[p0 + lane] = yi;
            }
        }
        __syncthreads();
        for (int i = p0 + pb + tid; i < k; i += 1024) {
            const double *Li = L + pk(i, p0);
            double s = 0.0;
            for (int jj = 0; jj < pb; ++jj) s += Li[jj] * yp[jj];
            w[i] -= s;
        }
        __syncthreads();
    }
    for (int p0 = ((k - 1) / 64) * 64; p0 >= 0; p0 -= 64) {
        const int pb = min(64, k - p0);
        for (int e = tid; e < 64 * 64; e += 1024) {
            const int i = e >> 6, j = e & 63;
            if (i < pb && j <= i) D[i][j] = L[pk(p0 + i, p0 + j)];
        }
        if (tid < pb) yp[tid] = w[p0 + tid];
        __syncthreads();
        if (wv == 0) {
            double yi = lane < pb ? yp[lane] : 0.0;
            for (int s = pb - 1; s >= 0; --s) {
                const double ws = __shfl(yi, s) / D[s][s];
                if (lane == s)
                    yi = ws;
                else if (lane < s)
                    yi -= D[s][lane] * ws;
            }
            if (lane < pb) {
                yp[lane] = yi;
                w[p0 + lane] = yi;
            }
        }
        __syncthreads();
        for (int c = tid; c < p0; c += 1024) {
            double s = 0.0;
            for (int r = 0; r < pb; ++r) s += L[pk(p0 + r, c)] * yp[r];
            w[c] -= s;
        }
        __syncthreads();
    }
}

int grid_for(long long n, int cap = 8192)
{
    long long g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

// Kernel of a product: the paired-row kernel with U entries per lane in flight for
// G = lanes <= 32 (U from the plan), one row per group of 64 lanes beyond.
template <int EPI, class T>
void spmv_dispatch(hipStream_t s, int lanes, int unroll, int blocks, const DCsrT<T> &a, int32_t lt, const T *x, T *y,
                   const T *aux, double *partials, const int32_t *done)
{
#define RSILU_SPMV_MR(G, U)                                                                                    \
    hipLaunchKernelGGL((k_spmv_mr<G, kSpmvRows, U, EPI, T>), dim3(blocks), dim3(kBlock), 0, s, a, lt, x, y, aux, \
                       partials, done)
    if (lanes == 4 && unroll == 2) RSILU_SPMV_MR(4, 2);
    else if (lanes == 8 && unroll == 2) RSILU_SPMV_MR(8, 2);
    else if (lanes == 8) RSILU_SPMV_MR(8, 4);
    else if (lanes == 16 && unroll == 3) RSILU_SPMV_MR(16, 3);
    else if (lanes == 16) RSILU_SPMV_MR(16, 4);
    else if (lanes == 32 && unroll == 3) RSILU_SPMV_MR(32, 3);
    else if (lanes == 32) RSILU_SPMV_MR(32, 4);
    else if (lanes == 2)
        hipLaunchKernelGGL((k_spmv<2, EPI, T>), dim3(blocks), dim3(kBlock), 0, s, a, lt, x, y, aux, partials, done);
    else
        hipLaunchKernelGGL((k_spmv<64, EPI, T>), dim3(blocks), dim3(kBlock), 0, s, a, lt, x, y, aux, partials, done);
#undef RSILU_SPMV_MR
}

// Rows per block of the kernel spmv_dispatch picks.
int spmv_rows_per_block(int lanes)
{
    if (lanes >= 4 && lanes <= 32) return (kBlock / lanes) * kSpmvRows;
    return kBlock / (lanes == 2 ? 2 : 64);
}

}  // namespace

// ------------------------------------------------------------------ launchers

void launch_gather(hipStream_t s, int32_t m, int32_t n, const int32_t *perm, const double *b, double *r,
                   double *xh, const int32_t *done)
{
    hipLaunchKernelGGL(k_gather, dim3(grid_for(m)), dim3(kBlock), 0, s, m, n, perm, b, r, xh, done);
}

template <class T>
void launch_spmv(hipStream_t s, const DCsrT<T> &a, const DPlan &pl, const T *x, T *y, const T *aux, Epi epi,
                 Fin fin, double *partials, T *segpart, DevState *st, const int32_t *done)
{
    if (a.nrows <= 0) return;
    const int lanes = pl.lanes, unroll = pl.unroll;
    const int rpb = spmv_rows_per_block(lanes);
    const int blocks = (int)((a.nrows + rpb - 1) / rpb);
    constexpr bool fp64 = std::is_same<T, double>::value;
    switch (epi) {
    case EPI_PLAIN: spmv_dispatch<EPI_PLAIN, T>(s, lanes, unroll, blocks, a, pl.long_thresh, x, y, aux, partials, done); break;
    case EPI_SUB: spmv_dispatch<EPI_SUB, T>(s, lanes, unroll, blocks, a, pl.long_thresh, x, y, aux, partials, done); break;
    case EPI_NEG: spmv_dispatch<EPI_NEG, T>(s, lanes, unroll, blocks, a, pl.long_thresh, x, y, aux, partials, done); break;
    case EPI_ADD: spmv_dispatch<EPI_ADD, T>(s, lanes, unroll, blocks, a, pl.long_thresh, x, y, aux, partials, done); break;
    case EPI_SQ:
        if constexpr (fp64) spmv_dispatch<EPI_SQ, T>(s, lanes, unroll, blocks, a, pl.long_thresh, x, y, aux, partials, done);
        break;
    case EPI_WSQ:
        if constexpr (fp64) spmv_dispatch<EPI_WSQ, T>(s, lanes, unroll, blocks, a, pl.long_thresh, x, y, aux, partials, done);
        break;
    }
    if (pl.nseg > 0)
        hipLaunchKernelGGL(k_spmv_seg<T>, dim3(pl.nseg), dim3(kBlock), 0, s, a, pl, x, segpart, done);
    const bool norm = (epi == EPI_SQ || epi == EPI_WSQ);
    if (pl.nlong > 0 || (norm && fin != FIN_NONE)) {
        const int nparts = norm ? blocks : 0;
        switch (epi) {
        case EPI_PLAIN:
            hipLaunchKernelGGL((k_finish<EPI_PLAIN, T>), dim3(1), dim3(kBlock), 0, s, pl, nparts, y, aux, segpart,
                               partials, fin, st, done);
            break;
        case EPI_SUB:
            hipLaunchKernelGGL((k_finish<EPI_SUB, T>), dim3(1), dim3(kBlock), 0, s, pl, nparts, y, aux, segpart,
                               partials, fin, st, done);
            break;
        case EPI_NEG:
            hipLaunchKernelGGL((k_finish<EPI_NEG, T>), dim3(1), dim3(kBlock), 0, s, pl, nparts, y, aux, segpart,
                               partials, fin, st, done);
            break;
        case EPI_ADD:
            hipLaunchKernelGGL((k_finish<EPI_ADD, T>), dim3(1), dim3(kBlock), 0, s, pl, nparts, y, aux, segpart,
                               partials, fin, st, done);
            break;
        case EPI_SQ:
            if constexpr (fp64)
                hipLaunchKernelGGL((k_finish<EPI_SQ, T>), dim3(1), dim3(kBlock), 0, s, pl, nparts, y, aux, segpart,
                                   partials, fin, st, done);
            break;
        case EPI_WSQ:
            if constexpr (fp64)
                hipLaunchKernelGGL((k_finish<EPI_WSQ, T>), dim3(1), dim3(kBlock), 0, s, pl, nparts, y, aux, segpart,
                                   partials, fin, st, done);
            break;
        }
    }
}
template void launch_spmv<double>(hipStream_t, const DCsrT<double> &, const DPlan &, const double *, double *,
                                  const double *, Epi, Fin, double *, double *, DevState *, const int32_t *);
template void launch_spmv<float>(hipStream_t, const DCsrT<float> &, const DPlan &, const float *, float *,
                                 const float *, Epi, Fin, double *, float *, DevState *, const int32_t *);

void launch_dot(hipStream_t s, int32_t n, const double *a, const double *b, Fin fin, double *partials,
                DevState *st, const int32_t *done)
{
    const int g = grid_for(n, 2048);
    hipLaunchKernelGGL(k_dot, dim3(g), dim3(kBlock), 0, s, n, a, b, partials, done);
    hipLaunchKernelGGL(k_reduce_fin, dim3(1), dim3(kBlock), 0, s, g, partials, fin, st, done);
}

void launch_pcg_init(hipStream_t s, int32_t k, const double *u, const double *d, double *w, double *res, double *z,
                     double *p, const int32_t *done)
{
    hipLaunchKernelGGL(k_pcg_init, dim3(grid_for(k)), dim3(kBlock), 0, s, k, u, d, w, res, z, p, done);
}

int cg_nparts(int32_t k) { return grid_for(k, kCgParts); }

void launch_cg_dot(hipStream_t s, int32_t k, const double *a, const double *b, double *parts, const int32_t *done)
{
    hipLaunchKernelGGL(k_dot, dim3(cg_nparts(k)), dim3(kBlock), 0, s, k, a, b, parts, done);
}

void launch_pcg_update_dot(hipStream_t s, int32_t k, const double *p, const double *q, const double *d, double *w,
                           double *res, double *z, const double *pq_parts, const double *rr_old, double *rr_new,
                           const int32_t *done)
{
    const int g = cg_nparts(k);
    hipLaunchKernelGGL(k_pcg_update_dot, dim3(g), dim3(kBlock), 0, s, k, p, q, d, w, res, z, g, pq_parts, rr_old,
                       rr_new, done);
}

void launch_cg_update_dot(hipStream_t s, int32_t k, const double *p, const double *q, double *w, double *res,
                          const double *pq_parts, const double *rr_old, double *rr_new, const int32_t *done)
{
    const int g = cg_nparts(k);
    hipLaunchKernelGGL(k_cg_update_dot, dim3(g), dim3(kBlock), 0, s, k, p, q, w, res, g, pq_parts, rr_old, rr_new,
                       done);
}

void launch_update(hipStream_t s, int32_t n, int32_t m, const double *p, double *xh, const double *q, double *r,
                   double *f0, double *f1, double *f2, double *f3, DevState *st, const int32_t *done)
{
    hipLaunchKernelGGL(k_update, dim3(grid_for(m)), dim3(kBlock), 0, s, n, m, p, xh, q, r, f0, f1, f2, f3, st,
                       done);
}

void launch_fill(hipStream_t s, int32_t n, double *f0, double *f1, double *f2, double *f3, DevState *st)
{
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(kBlock), 0, s, n, f0, f1, f2, f3, st);
}

void launch_refill(hipStream_t s, int32_t n, double *f0, double *f1, DevState *st, const int32_t *done)
{
    hipLaunchKernelGGL(k_refill, dim3(grid_for(n)), dim3(kBlock), 0, s, n, f0, f1, st, done);
}

void launch_pupdate(hipStream_t s, int32_t n, const double *h, double *p, const DevState *st, bool first,
                    const int32_t *done)
{
    hipLaunchKernelGGL(k_pupdate, dim3(grid_for(n)), dim3(kBlock), 0, s, n, h, p, st, first ? 1 : 0, done);
}

void launch_scale_out(hipStream_t s, int32_t n, const double *xh, const double *colnorm, double *x)
{
    hipLaunchKernelGGL(k_scale_out, dim3(grid_for(n)), dim3(kBlock), 0, s, n, xh, colnorm, x);
}

void launch_residual(hipStream_t s, int32_t m, const int32_t *perm, const double *b, const double *ax, double *r)
{
    hipLaunchKernelGGL(k_residual, dim3(grid_for(m)), dim3(kBlock), 0, s, m, perm, b, ax, r);
}

void launch_copy(hipStream_t s, int32_t n, const double *src, double *dst, const int32_t *done)
{
    hipLaunchKernelGGL(k_copy, dim3(grid_for(n)), dim3(kBlock), 0, s, n, src, dst, done);
}

void launch_add(hipStream_t s, int32_t n, const double *src, double *dst, const int32_t *done)
{
    hipLaunchKernelGGL(k_add, dim3(grid_for(n)), dim3(kBlock), 0, s, n, src, dst, done);
}

void launch_trsv_syncfree(hipStream_t s, const DTri &t, const double *rhs, double *x, const double *add,
                          double *y2, DevState *st, int ticket, const int32_t *done)
{
    if (t.nchunks <= 0) return;
    // enough waves to cover the widest levels; each wave keeps taking chunks
    int blocks = (t.nchunks + 3) / 4;
    if (blocks > 2048) blocks = 2048;
#define RSILU_TRSV_CASE(G)                                                                                      \
    case G:                                                                                                     \
        hipLaunchKernelGGL(k_trsv_syncfree<G>, dim3(blocks), dim3(kBlock), 0, s, t, rhs, x, add, y2, st, ticket, \
                           done);                                                                               \
        break;
    switch (t.lanes) {
        RSILU_TRSV_CASE(1)
        RSILU_TRSV_CASE(2)
        RSILU_TRSV_CASE(4)
        RSILU_TRSV_CASE(8)
        RSILU_TRSV_CASE(16)
        RSILU_TRSV_CASE(32)
        RSILU_TRSV_CASE(64)
    default:
        break;
    }
#undef RSILU_TRSV_CASE
}

template <class T>
void launch_trsv_level(hipStream_t s, const DTriT<T> &t, int32_t beg, int32_t end, const T *rhs, T *x, const T *add,
                       T *y2, const int32_t *done)
{
    const int rpb = kBlock / t.lanes;
    const int blocks = (end - beg + rpb - 1) / rpb;
    if (blocks <= 0) return;
#define RSILU_TRSVL_CASE(G)                                                                                      \
    case G:                                                                                                      \
        hipLaunchKernelGGL((k_trsv_level<G, T>), dim3(blocks), dim3(kBlock), 0, s, t, beg, end, rhs, x, add, y2, done); \
        break;
    switch (t.lanes) {
        RSILU_TRSVL_CASE(1)
        RSILU_TRSVL_CASE(2)
        RSILU_TRSVL_CASE(4)
        RSILU_TRSVL_CASE(8)
        RSILU_TRSVL_CASE(16)
        RSILU_TRSVL_CASE(32)
        RSILU_TRSVL_CASE(64)
    default:
        break;
    }
#undef RSILU_TRSVL_CASE
}
template void launch_trsv_level<double>(hipStream_t, const DTriT<double> &, int32_t, int32_t, const double *, double *,
                                        const double *, double *, const int32_t *);
template void launch_trsv_level<float>(hipStream_t, const DTriT<float> &, int32_t, int32_t, const float *, float *,
                                       const float *, float *, const int32_t *);

template <class T>
void launch_trsv_sweep(hipStream_t s, const unsigned char *blob, int64_t off, int32_t size, int32_t npos_first,
                       int32_t p0, int32_t nb, int32_t scheme, const T *rhs_lo, T *x, const T *add_lo, T *y2,
                       const int32_t *done)
{
    if (nb <= 0) return;
    switch (scheme) {
    case kSchemeSegmentedWide:
        hipLaunchKernelGGL((k_trsv_sweep<T, kSchemeSegmentedWide>), dim3(1), dim3(kSweepThreads), 0, s, blob, off,
                           size, npos_first, p0, nb, rhs_lo, x, add_lo, y2, done);
        break;
    case kSchemeSegmented:
        hipLaunchKernelGGL((k_trsv_sweep<T, kSchemeSegmented>), dim3(1), dim3(kSweepThreads), 0, s, blob, off, size,
                           npos_first, p0, nb, rhs_lo, x, add_lo, y2, done);
        break;
    case kSchemeRows:
        hipLaunchKernelGGL((k_trsv_sweep<T, kSchemeRows>), dim3(1), dim3(kSweepThreads), 0, s, blob, off, size, npos_first, p0,
                           nb, rhs_lo, x, add_lo, y2, done);
        break;
    default:
        hipLaunchKernelGGL((k_trsv_sweep<T, kSchemeTwoPhase>), dim3(1), dim3(kSweepThreads), 0, s, blob, off, size, npos_first, p0,
                           nb, rhs_lo, x, add_lo, y2, done);
    }
}
template void launch_trsv_sweep<double>(hipStream_t, const unsigned char *, int64_t, int32_t, int32_t, int32_t, int32_t,
                                        int32_t, const double *, double *, const double *, double *, const int32_t *);
template void launch_trsv_sweep<float>(hipStream_t, const unsigned char *, int64_t, int32_t, int32_t, int32_t, int32_t,
                                       int32_t, const float *, float *, const float *, float *, const int32_t *);

template <class T>
void launch_gather_lo(hipStream_t s, int32_t n, const int32_t *rows, const T *src, T *dst, const T *src2, T *dst2,
                      const int32_t *done)
{
    hipLaunchKernelGGL(k_gather_lo<T>, dim3(grid_for(n)), dim3(kBlock), 0, s, n, rows, src, dst, src2, dst2, done);
}
template void launch_gather_lo<double>(hipStream_t, int32_t, const int32_t *, const double *, double *, const double *,
                                       double *, const int32_t *);
template void launch_gather_lo<float>(hipStream_t, int32_t, const int32_t *, const float *, float *, const float *,
                                      float *, const int32_t *);

void launch_lsqr_t(hipStream_t s, int32_t m, const double *u, double *t, Fin fin, double *partials, DevState *st,
                   const int32_t *done)
{
    const int g = grid_for(m, 2048);
    hipLaunchKernelGGL(k_lsqr_t, dim3(g), dim3(kBlock), 0, s, m, u, t, partials, st, done);
    hipLaunchKernelGGL(k_reduce_fin, dim3(1), dim3(kBlock), 0, s, g, partials, fin, st, done);
}

void launch_lsqr_scale(hipStream_t s, int32_t m, const double *in, double *out, const DevState *st,
                       const int32_t *done)
{
    hipLaunchKernelGGL(k_lsqr_scale, dim3(grid_for(m)), dim3(kBlock), 0, s, m, in, out, st, done);
}

void launch_lsqr_s(hipStream_t s, int32_t n, double *sv, const double *Mv, const double *colnorm, Fin fin,
                   double *partials, DevState *st, const int32_t *done)
{
    const int g = grid_for(n, 2048);
    hipLaunchKernelGGL(k_lsqr_s, dim3(g), dim3(kBlock), 0, s, n, sv, Mv, colnorm, partials, st, done);
    hipLaunchKernelGGL(k_reduce_fin, dim3(1), dim3(kBlock), 0, s, g, partials, fin, st, done);
}

void launch_lsqr_v(hipStream_t s, int32_t n, const double *h, const double *sv, double *xh, double *v, double *Mv,
                   double *w, bool init, const DevState *st, const int32_t *done)
{
    hipLaunchKernelGGL(k_lsqr_v, dim3(grid_for(n)), dim3(kBlock), 0, s, n, h, sv, xh, v, Mv, w, init ? 1 : 0, st,
                       done);
}

void launch_lsqr_commit(hipStream_t s, DevState *st)
{
    hipLaunchKernelGGL(k_lsqr_commit, dim3(1), dim3(64), 0, s, st);
}

void launch_cg_init(hipStream_t s, int32_t k, const double *u, double *w, double *res, double *p, const int32_t *done)
{
    hipLaunchKernelGGL(k_cg_init, dim3(grid_for(k)), dim3(kBlock), 0, s, k, u, w, res, p, done);
}

void launch_cg_update(hipStream_t s, int32_t k, const double *p, const double *q, double *w, double *res,
                      const double *pq_parts, const double *rr_parts, const int32_t *done)
{
    hipLaunchKernelGGL(k_cg_update, dim3(grid_for(k)), dim3(kBlock), 0, s, k, p, q, w, res, cg_nparts(k), pq_parts,
                       rr_parts, done);
}

void launch_cg_dir(hipStream_t s, int32_t k, const double *res, double *p, const double *rr_old, const double *rr_new,
                   const int32_t *done)
{
    hipLaunchKernelGGL(k_cg_dir, dim3(grid_for(k)), dim3(kBlock), 0, s, k, res, p, cg_nparts(k), rr_old, rr_new, done);
}

template <class T>
void launch_cheb_init(hipStream_t s, int32_t k, const T *u, T *r, T *d, T *w, double theta, double omega,
                      const int32_t *done)
{
    hipLaunchKernelGGL(k_cheb_init<T>, dim3(grid_for(k)), dim3(kBlock), 0, s, k, u, r, d, w, (T)theta, (T)omega,
                       done);
}
template void launch_cheb_init<double>(hipStream_t, int32_t, const double *, double *, double *, double *, double,
                                       double, const int32_t *);
template void launch_cheb_init<float>(hipStream_t, int32_t, const float *, float *, float *, float *, double, double,
                                      const int32_t *);

template <class T>
void launch_cheb_update(hipStream_t s, int32_t k, const T *q, T *r, T *d, T *w, T *out, double c1, double c2,
                        const int32_t *done)
{
    hipLaunchKernelGGL(k_cheb_update<T>, dim3(grid_for(k)), dim3(kBlock), 0, s, k, q, r, d, w, out, (T)c1, (T)c2,
                       done);
}
template void launch_cheb_update<double>(hipStream_t, int32_t, const double *, double *, double *, double *, double *,
                                         double, double, const int32_t *);
template void launch_cheb_update<float>(hipStream_t, int32_t, const float *, float *, float *, float *, float *,
                                        double, double, const int32_t *);

void launch_cvt(hipStream_t s, int32_t n, const double *in, float *out, const int32_t *done)
{
    hipLaunchKernelGGL((k_cvt<double, float>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, in, out, done);
}

void launch_cvt(hipStream_t s, int32_t n, const float *in, double *out, const int32_t *done)
{
    hipLaunchKernelGGL((k_cvt<float, double>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, in, out, done);
}

void launch_dense_chol_solve(hipStream_t s, int32_t k, const double *lfac, double *w, const int32_t *done)
{
    if (k <= 0) return;
    hipLaunchKernelGGL(k_dense_chol, dim3(1), dim3(1024), 0, s, k, lfac, w, done);
}

}  // namespace rsilu
